// FP32 element internal-force kernel f = -K u (VALU contractions through LDS).
//
// One workgroup owns one element at a time, one lane per GLL point (the n^3
// points padded to whole 64-lane wavefronts).  Per element, in one fused
// traversal (the paper's Sec. IV-D single grid-point traversal with scalar
// intermediates):
//   gather u[ibool] -> LDS,
//   three forward contractions with D along xi/eta/zeta (Sec. II-B),
//   inverse-Jacobian map, isotropic stress, weighted fluxes in registers,
//   fluxes -> LDS, three transpose contractions with D^T (Sec. II-B, weak form),
//   scatter-add to f (plain read-modify-write inside a colour, or atomics).
// Coloured assembly may come with first-touch flags: the point that reaches
// its node first in launch order stores its force without reading f, so the
// force vector needs no clearing before the pass.
//
// Geometry paths (the paper's Sec. IV-D regular/irregular specialisation,
// chosen per launch, never per point):
//   kRegular   affine element: one Gamma per element (scalar loads);
//   kStored    per-point Gamma = J^{-1} streamed from memory (9 floats/point);
//   kTrilinear J rebuilt at each point from the 8x3 coefficients of the
//              element's trilinear map (scalar loads), no per-point geometry
//              traffic.  With C the cofactor matrix of J (J^{-1} = C^T/det J)
//              and lambda' = lambda w det J, mu' = mu w det J as stored:
//              g' = du C^T, sigma'' = lambda' tr(g') I + mu' (g' + g'^T),
//              Phi = sigma'' C / det^2  (equal to w det J sigma J^{-T}).
//
// The streaming inputs (node numbers, Gamma, lambda', mu') use non-temporal
// loads so they do not evict u and f from the caches.
#include "elem_common.hpp"

namespace semx {
namespace {

// Per-lane inputs of one element.
struct PointIn {
  int g;
  bool first;  // the lane's point is the first to reach its node (store, no read)
  float G[9];  // Gamma (kStored); unused otherwise
  float lw, mw;
  float u[3];
  float f[3];
};

template <int NG, int GEO, bool ATOMIC>
__device__ __forceinline__ void load_point(const ForceArgs& a, const float* __restrict__ mat,
                                           const float* __restrict__ u, const float* f, int pos, int pp,
                                           int g, PointIn& P) {
  constexpr int N3 = Shape<NG>::N3;
  P.g = g;
  if constexpr (GEO == kStored) {
    const float* gp = a.gam_pt + (size_t)pos * 9 * N3 + pp;
#pragma unroll
    for (int d = 0; d < 9; ++d) P.G[d] = ldnt(gp + d * N3);
  }
  P.lw = ldnt(mat + (size_t)pos * 2 * N3 + pp);
  P.mw = ldnt(mat + (size_t)pos * 2 * N3 + N3 + pp);
  P.u[0] = u[3 * (size_t)g + 0];
  P.u[1] = u[3 * (size_t)g + 1];
  P.u[2] = u[3 * (size_t)g + 2];
  P.first = false;
  if constexpr (!ATOMIC) {
    if (a.first) P.first = (a.first[(size_t)pos * a.first_words + (pp >> 5)] >> (pp & 31)) & 1u;
    P.f[0] = P.f[1] = P.f[2] = 0.0f;
    if (!P.first) {
      P.f[0] = f[3 * (size_t)g + 0];
      P.f[1] = f[3 * (size_t)g + 1];
      P.f[2] = f[3 * (size_t)g + 2];
    }
  }
}

// One workgroup handles R consecutive launch positions (elements) in
// straight-line code: the inputs of element m+1 are loaded while element m
// computes.  Straight-line code (no loop) lets the compiler count outstanding
// memory operations exactly, so waits for prefetched data never wait for the
// scatter stores issued after them.
// Node number of local point (i, j, k) of the element at launch position
// `pos`: from the ibool stream, or (AFF) from the element's affine numbering
// g0 + i sx + j sy + k sz (four scalar loads per element, no per-point stream
// and no dependent round trip before the gather).
template <int NG, bool AFF>
__device__ __forceinline__ int node_of(const ForceArgs& a, int pos, int pp, int i, int j, int k) {
  if constexpr (AFF) {
    const int* r = a.aff + (size_t)pos * 4;
    return r[0] + i * r[1] + j * r[2] + k * r[3];
  } else {
    return ldnt(a.ibool + (size_t)pos * Shape<NG>::N3 + pp);
  }
}

template <int NG, int GEO, bool ATOMIC, int R, bool AFF>
__global__ __launch_bounds__(Shape<NG>::BLK) void force_f32_kernel(ForceArgs a) {
  constexpr int N3 = Shape<NG>::N3;
  __shared__ float s_u[3 * N3];
  __shared__ float s_q[9 * N3];
  __shared__ float s_D[NG * NG];

  const int ngrp = (int)((a.count + R - 1) / R);
  const int grp = xcd_group(ngrp);
  if (grp >= ngrp) return;  // uniform over the block
  const int r0 = grp * R;
  const int nr = min(R, (int)a.count - r0);
  const int P0 = (int)a.pos0 + r0;

  const int p = threadIdx.x;
  const bool act = p < N3;
  const int pp = act ? p : 0;
  const int i = pp % NG, j = (pp / NG) % NG, k = pp / (NG * NG);

  const int model = blockIdx.y;
  const float* __restrict__ u = a.u + (size_t)model * a.nglob * 3;
  float* f = a.f + (size_t)model * a.nglob * 3;
  const float* __restrict__ mat = a.mat + (size_t)model * a.nspec * 2 * N3;

  PointIn P[2];
  int g_next = (nr > 1) ? node_of<NG, AFF>(a, P0 + 1, pp, i, j, k) : 0;
  load_point<NG, GEO, ATOMIC>(a, mat, u, f, P0, pp, node_of<NG, AFF>(a, P0, pp, i, j, k), P[0]);

  // D in LDS: the lane's rows and columns are read per contraction step,
  // which keeps the register count low enough for 8 waves per SIMD.
  if (p < NG * NG) s_D[p] = a.D[p];
  float rx = 0.f, ry = 0.f, rz = 0.f;  // reference coordinates (trilinear path)
  if constexpr (GEO == kTrilinear) {
    rx = a.xi[i];
    ry = a.xi[j];
    rz = a.xi[k];
  }

#pragma unroll
  for (int m = 0; m < R; ++m) {
    if (m >= nr) break;  // uniform over the block
    PointIn& cur = P[m & 1];
    PointIn& nxt = P[(m + 1) & 1];
    if (m > 0) __syncthreads();  // the previous element has finished reading s_q / s_u
    if (act) {
      s_u[pp] = cur.u[0];
      s_u[N3 + pp] = cur.u[1];
      s_u[2 * N3 + pp] = cur.u[2];
    }
    if (m + 1 < nr) {
      load_point<NG, GEO, ATOMIC>(a, mat, u, f, P0 + m + 1, pp, g_next, nxt);
      if (m + 2 < nr) g_next = node_of<NG, AFF>(a, P0 + m + 2, pp, i, j, k);
    }
    __syncthreads();

    float du[3][3];
    ref_grad<NG>(s_u, s_D, i, j, k, du);
    float Mg[9], scale, det;
    geom_map<GEO>(a, P0 + m, cur.G, rx, ry, rz, Mg, scale, det);
    float gr[3][3];
    apply_map(du, Mg, gr);
    stress_flux(gr, cur.lw, cur.mw, scale, Mg, s_q, N3, pp, act);
    __syncthreads();

    float F[3];
    ref_div<NG>(s_q, s_D, i, j, k, F);
    if (act) {
      float* fg = f + 3 * (size_t)cur.g;
      if constexpr (ATOMIC) {
        unsafeAtomicAdd(fg + 0, F[0]);
        unsafeAtomicAdd(fg + 1, F[1]);
        unsafeAtomicAdd(fg + 2, F[2]);
      } else {
        fg[0] = cur.f[0] + F[0];
        fg[1] = cur.f[1] + F[1];
        fg[2] = cur.f[2] + F[2];
      }
    }
  }
}

#ifndef SEMX_F32_ELEMS_PER_BLOCK
#define SEMX_F32_ELEMS_PER_BLOCK 1
#endif

template <int NG, int GEO, bool ATOMIC, bool AFF>
hipError_t launch_one(const ForceArgs& a, hipStream_t s) {
  constexpr int R = SEMX_F32_ELEMS_PER_BLOCK;
  const int64_t ngrp = (a.count + R - 1) / R;
  const int64_t nb = ((ngrp + kNumXcd - 1) / kNumXcd) * kNumXcd;
  dim3 grid((unsigned)nb, (unsigned)a.nmodels), block(Shape<NG>::BLK);
  force_f32_kernel<NG, GEO, ATOMIC, R, AFF><<<grid, block, 0, s>>>(a);
  return hipGetLastError();
}

template <int NG, bool AFF>
hipError_t launch_n(int geo, bool atomic, const ForceArgs& a, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  switch (geo) {
    case kRegular:
      return atomic ? launch_one<NG, kRegular, true, AFF>(a, s) : launch_one<NG, kRegular, false, AFF>(a, s);
    case kStored:
      return atomic ? launch_one<NG, kStored, true, AFF>(a, s) : launch_one<NG, kStored, false, AFF>(a, s);
    case kTrilinear:
      return atomic ? launch_one<NG, kTrilinear, true, AFF>(a, s) : launch_one<NG, kTrilinear, false, AFF>(a, s);
    default:
      return hipErrorInvalidValue;
  }
}

// Memory skeleton of force_f32_kernel (coloured assembly, one element per
// workgroup): the same grid, block mapping and per-lane loads and stores
// (node number, geometry, material, u, first-touch bit, f read unless first,
// f store), without the contractions and the pointwise arithmetic.  Its
// duration is the floor that the kernel's access pattern alone sets on the
// memory system.  f receives meaningless values.
template <int NG, int GEO, bool AFF>
__global__ __launch_bounds__(Shape<NG>::BLK) void force_skeleton_kernel(ForceArgs a) {
  constexpr int N3 = Shape<NG>::N3;
  const int ngrp = (int)a.count;
  const int grp = xcd_group(ngrp);
  if (grp >= ngrp) return;  // uniform over the block
  const int p = threadIdx.x;
  if (p >= N3) return;
  const int pos = (int)a.pos0 + grp;
  const int model = blockIdx.y;
  const float* __restrict__ u = a.u + (size_t)model * a.nglob * 3;
  float* f = a.f + (size_t)model * a.nglob * 3;
  const float* __restrict__ mat = a.mat + (size_t)model * a.nspec * 2 * N3;
  PointIn P;
  load_point<NG, GEO, false>(a, mat, u, f, pos, p, node_of<NG, AFF>(a, pos, p, p % NG, (p / NG) % NG, p / (NG * NG)),
                             P);
  float s = P.lw + P.mw;
  if constexpr (GEO == kStored) {
#pragma unroll
    for (int d = 0; d < 9; ++d) s += P.G[d];
  } else {
    constexpr int NS = GEO == kRegular ? 9 : 24;
    const float* src = GEO == kRegular ? a.gam_el + (size_t)pos * 9 : a.tri + (size_t)pos * 24;
#pragma unroll
    for (int d = 0; d < NS; ++d) s += src[d];
  }
  float* fg = f + 3 * (size_t)P.g;
  fg[0] = P.f[0] + s * P.u[0];
  fg[1] = P.f[1] + s * P.u[1];
  fg[2] = P.f[2] + s * P.u[2];
}

template <int NG, bool AFF>
hipError_t launch_skeleton_n(int geo, const ForceArgs& a, hipStream_t s) {
  static_assert(SEMX_F32_ELEMS_PER_BLOCK == 1, "the skeleton mirrors one element per workgroup");
  if (a.count <= 0) return hipSuccess;
  const int64_t nb = ((a.count + kNumXcd - 1) / kNumXcd) * kNumXcd;
  dim3 grid((unsigned)nb, (unsigned)a.nmodels), block(Shape<NG>::BLK);
  switch (geo) {
    case kRegular: force_skeleton_kernel<NG, kRegular, AFF><<<grid, block, 0, s>>>(a); break;
    case kStored: force_skeleton_kernel<NG, kStored, AFF><<<grid, block, 0, s>>>(a); break;
    case kTrilinear: force_skeleton_kernel<NG, kTrilinear, AFF><<<grid, block, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// A launch range whose first `naff` elements are affine-numbered: two launches.
template <class F>
hipError_t split_affine(int64_t naff, const ForceArgs& a, F launch) {
  naff = naff < 0 ? 0 : (naff > a.count ? a.count : naff);
  ForceArgs b = a;
  b.count = naff;
  hipError_t e = naff > 0 ? launch(b, true) : hipSuccess;
  if (e != hipSuccess || naff == a.count) return e;
  b.pos0 = a.pos0 + naff;
  b.count = a.count - naff;
  return launch(b, false);
}

template <int NG>
hipError_t launch_f32_any(int geo, bool atomic, bool aff, const ForceArgs& a, hipStream_t s) {
  return aff ? launch_n<NG, true>(geo, atomic, a, s) : launch_n<NG, false>(geo, atomic, a, s);
}

template <int NG>
hipError_t launch_skeleton_any(int geo, bool aff, const ForceArgs& a, hipStream_t s) {
  return aff ? launch_skeleton_n<NG, true>(geo, a, s) : launch_skeleton_n<NG, false>(geo, a, s);
}

hipError_t launch_f32_n(int n, int geo, bool atomic, bool aff, const ForceArgs& a, hipStream_t s) {
  switch (n) {
    case 2: return launch_f32_any<2>(geo, atomic, aff, a, s);
    case 3: return launch_f32_any<3>(geo, atomic, aff, a, s);
    case 4: return launch_f32_any<4>(geo, atomic, aff, a, s);
    case 5: return launch_f32_any<5>(geo, atomic, aff, a, s);
    case 6: return launch_f32_any<6>(geo, atomic, aff, a, s);
    case 7: return launch_f32_any<7>(geo, atomic, aff, a, s);
    case 8: return launch_f32_any<8>(geo, atomic, aff, a, s);
    case 9: return launch_f32_any<9>(geo, atomic, aff, a, s);
    case 10: return launch_f32_any<10>(geo, atomic, aff, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_force_skeleton(int n, int geo, int64_t naff, const ForceArgs& a, hipStream_t s) {
  return split_affine(naff, a, [&](const ForceArgs& b, bool aff) -> hipError_t {
    switch (n) {
      case 2: return launch_skeleton_any<2>(geo, aff, b, s);
      case 3: return launch_skeleton_any<3>(geo, aff, b, s);
      case 4: return launch_skeleton_any<4>(geo, aff, b, s);
      case 5: return launch_skeleton_any<5>(geo, aff, b, s);
      case 6: return launch_skeleton_any<6>(geo, aff, b, s);
      case 7: return launch_skeleton_any<7>(geo, aff, b, s);
      case 8: return launch_skeleton_any<8>(geo, aff, b, s);
      case 9: return launch_skeleton_any<9>(geo, aff, b, s);
      case 10: return launch_skeleton_any<10>(geo, aff, b, s);
      default: return hipErrorInvalidValue;
    }
  });
}

hipError_t launch_force_f32(int n, int geo, bool atomic, const ForceArgs& a, hipStream_t s) {
  return launch_f32_n(n, geo, atomic, false, a, s);
}

hipError_t launch_force_f32_split(int n, int geo, bool atomic, int64_t naff, const ForceArgs& a, hipStream_t s) {
  return split_affine(naff, a, [&](const ForceArgs& b, bool aff) { return launch_f32_n(n, geo, atomic, aff, b, s); });
}

}  // namespace semx
