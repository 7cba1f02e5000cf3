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

// First-touch bit of local point pp of the element at launch position pos
// (coloured assembly): the element's NW = ceil(n^3/32) words are uniform over
// the workgroup, so for NW <= 8 they come through the scalar cache and each
// lane picks its word with a select chain; the f read that depends on the
// bit then waits for a scalar load, not for a vector-memory round trip.
template <int N3>
__device__ __forceinline__ bool first_touch(const ForceArgs& a, int pos, int pp) {
  constexpr int NW = (N3 + 31) / 32;
  if (!a.first) return false;
  const uint32_t* w = a.first + (size_t)pos * a.first_words;
  if constexpr (NW <= 8) {
    uint32_t word = w[0];
#pragma unroll
    for (int c = 1; c < NW; ++c) {
      const uint32_t wc = w[c];
      word = (pp >> 5) == c ? wc : word;
    }
    return (word >> (pp & 31)) & 1u;
  } else {
    return (w[pp >> 5] >> (pp & 31)) & 1u;
  }
}

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

// Read of the prior force at node g for a coloured, affine-numbered element
// (coloured assembly with first-touch bits): a raw buffer load over the
// element's node span, with the offset pushed out of range at first-touch
// points, so the hardware returns zeros there and fetches nothing, and the
// load is a plain unconditional instruction the compiler can count exactly
// (no branch, so later waits for u do not also wait for f).  The host
// classifies an element as affine only when its span fits a 31-bit byte
// offset.
template <int NG>
__device__ __forceinline__ void prior_force_affine(const float* f, const int* r, int g, bool first, float fo[3]) {
  const int sx = r[1], sy = r[2], sz = r[3];
  const int gmin = r[0] + (NG - 1) * (min(sx, 0) + min(sy, 0) + min(sz, 0));
  const int span = (NG - 1) * (abs(sx) + abs(sy) + abs(sz)) + 1;
  __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)(f + 3 * (size_t)gmin), (short)0, span * 12, kBufferWord3);
  typedef unsigned v3u __attribute__((ext_vector_type(3)));
  // out of range: 2^31 lies past any num_records <= 2^31 - 1, and adding the
  // 8 bytes of the last dword cannot wrap a 32-bit offset
  const v3u v = __builtin_amdgcn_raw_buffer_load_b96(rs, first ? INT32_MIN : (g - gmin) * 12, 0, 0);
  fo[0] = __uint_as_float(v.x);
  fo[1] = __uint_as_float(v.y);
  fo[2] = __uint_as_float(v.z);
}

// Per-element geometry that is uniform over the workgroup: Gamma (kRegular,
// 9 floats) or the trilinear coefficients (kTrilinear, 24 floats).
template <int GEO>
struct ElemGeom {
  static constexpr int NS = GEO == kRegular ? 9 : (GEO == kTrilinear ? 24 : 1);
  float v[NS];
};

// One workgroup owns one element (one lane per GLL point).  Every load an
// element needs is issued before its first wait: the constant tables (D and
// the GLL nodes, L2-resident), the per-element scalars (node-numbering
// coefficients, geometry, first-touch words), the material and the u gather.
// The f read depends only on the first-touch bit (a scalar load) and is
// consumed at the very end, so its latency runs under the contractions.
template <int NG, int GEO, bool ATOMIC, bool AFF>
__global__ __launch_bounds__(Shape<NG>::BLK) void force_f32_kernel(ForceArgs a) {
  constexpr int N3 = Shape<NG>::N3;
  constexpr int ND = NG * NG;
  __shared__ float s_u[3 * N3];
  __shared__ float s_q[9 * N3];
  __shared__ float s_D[ND + NG];  // D (row-major), then the GLL nodes

  const int ngrp = (int)a.count;
  const int grp = xcd_group(ngrp);
  if (grp >= ngrp) return;  // uniform over the block
  const int pos = (int)a.pos0 + grp;

  const int p = threadIdx.x;
  const bool act = p < N3;
  const int pp = act ? p : 0;
  const int i = pp % NG, j = (pp / NG) % NG, k = pp / (NG * NG);

  const int model = blockIdx.y;
  const float* __restrict__ u = a.u + (size_t)model * a.nglob * 3;
  float* f = a.f + (size_t)model * a.nglob * 3;
  const float* __restrict__ mat = a.mat + (size_t)model * a.nspec * 2 * N3;

  float tab = 0.0f;
  if (p < ND) tab = a.D[p];
  else if (GEO == kTrilinear && p < ND + NG) tab = a.xi[p - ND];

  ElemGeom<GEO> eg;
  if constexpr (GEO != kStored) {
    const float* src = GEO == kRegular ? a.gam_el + (size_t)pos * 9 : a.tri + (size_t)pos * 24;
#pragma unroll
    for (int d = 0; d < ElemGeom<GEO>::NS; ++d) eg.v[d] = src[d];
  }
  float G[9];
  if constexpr (GEO == kStored) {
    const float* gp = a.gam_pt + (size_t)pos * 9 * N3 + pp;
#pragma unroll
    for (int d = 0; d < 9; ++d) G[d] = ldnt(gp + d * N3);
  }

  const int g = node_of<NG, AFF>(a, pos, pp, i, j, k);
  const float lw = ldnt(mat + (size_t)pos * 2 * N3 + pp);
  const float mw = ldnt(mat + (size_t)pos * 2 * N3 + N3 + pp);
  const float u0 = u[3 * (size_t)g + 0];
  const float u1 = u[3 * (size_t)g + 1];
  const float u2 = u[3 * (size_t)g + 2];
  float fo[3] = {0.0f, 0.0f, 0.0f};
  if constexpr (!ATOMIC && AFF) {
    prior_force_affine<NG>(f, a.aff + (size_t)pos * 4, g, first_touch<N3>(a, pos, pp), fo);
  } else if constexpr (!ATOMIC) {
    if (!first_touch<N3>(a, pos, pp)) {
      fo[0] = f[3 * (size_t)g + 0];
      fo[1] = f[3 * (size_t)g + 1];
      fo[2] = f[3 * (size_t)g + 2];
    }
  }

  if constexpr (GEO != kStored) {
    // keep the element's geometry loads ahead of the first barrier (they
    // would otherwise be sunk past it, onto the element's critical path);
    // placed after every load, so no load is seen as clobbered by it
#pragma unroll
    for (int d = 0; d < ElemGeom<GEO>::NS; ++d) asm volatile("" ::"s"(eg.v[d]));
  }
  if (p < ND + NG) s_D[p] = tab;
  if (act) {
    s_u[pp] = u0;
    s_u[N3 + pp] = u1;
    s_u[2 * N3 + pp] = u2;
  }
  __syncthreads();

  float rx = 0.f, ry = 0.f, rz = 0.f;  // reference coordinates (trilinear path)
  if constexpr (GEO == kTrilinear) {
    rx = s_D[ND + i];
    ry = s_D[ND + j];
    rz = s_D[ND + k];
  }
  float du[3][3];
  ref_grad<NG>(s_u, s_D, i, j, k, du);
  float Mg[9], scale, det;
  geom_map_from<GEO>(eg.v, G, rx, ry, rz, Mg, scale, det);
  float gr[3][3];
  apply_map(du, Mg, gr);
  stress_flux(gr, lw, mw, scale, Mg, s_q, N3, pp, act);
  __syncthreads();

  float F[3];
  ref_div<NG>(s_q, s_D, i, j, k, F);
  if (act) {
    float* fg = f + 3 * (size_t)g;
    if constexpr (ATOMIC) {
      unsafeAtomicAdd(fg + 0, F[0]);
      unsafeAtomicAdd(fg + 1, F[1]);
      unsafeAtomicAdd(fg + 2, F[2]);
    } else {
      fg[0] = fo[0] + F[0];
      fg[1] = fo[1] + F[1];
      fg[2] = fo[2] + F[2];
    }
  }
}

template <int NG, int GEO, bool ATOMIC, bool AFF>
hipError_t launch_one(const ForceArgs& a, hipStream_t s) {
  const int64_t nb = ((a.count + kNumXcd - 1) / kNumXcd) * kNumXcd;
  dim3 grid((unsigned)nb, (unsigned)a.nmodels), block(Shape<NG>::BLK);
  force_f32_kernel<NG, GEO, ATOMIC, AFF><<<grid, block, 0, s>>>(a);
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

// Memory skeleton of force_f32_kernel (coloured assembly): the same grid,
// block mapping and per-lane loads and stores (node number, geometry,
// material, u, first-touch bit, f read unless first, f store), without the
// contractions and the pointwise arithmetic.  Its duration is the floor that
// the kernel's access pattern alone sets on the memory system.  f receives
// meaningless values.
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
  float s = 0.0f;
  if constexpr (GEO == kStored) {
    const float* gp = a.gam_pt + (size_t)pos * 9 * N3 + p;
#pragma unroll
    for (int d = 0; d < 9; ++d) s += ldnt(gp + d * N3);
  } else {
    constexpr int NS = GEO == kRegular ? 9 : 24;
    const float* src = GEO == kRegular ? a.gam_el + (size_t)pos * 9 : a.tri + (size_t)pos * 24;
#pragma unroll
    for (int d = 0; d < NS; ++d) s += src[d];
  }
  const int g = node_of<NG, AFF>(a, pos, p, p % NG, (p / NG) % NG, p / (NG * NG));
  s += ldnt(mat + (size_t)pos * 2 * N3 + p) + ldnt(mat + (size_t)pos * 2 * N3 + N3 + p);
  const float u0 = u[3 * (size_t)g + 0], u1 = u[3 * (size_t)g + 1], u2 = u[3 * (size_t)g + 2];
  float fo[3] = {0.0f, 0.0f, 0.0f};
  if constexpr (AFF) {
    prior_force_affine<NG>(f, a.aff + (size_t)pos * 4, g, first_touch<N3>(a, pos, p), fo);
  } else if (!first_touch<N3>(a, pos, p)) {
    fo[0] = f[3 * (size_t)g + 0];
    fo[1] = f[3 * (size_t)g + 1];
    fo[2] = f[3 * (size_t)g + 2];
  }
  float* fg = f + 3 * (size_t)g;
  fg[0] = fo[0] + s * u0;
  fg[1] = fo[1] + s * u1;
  fg[2] = fo[2] + s * u2;
}

template <int NG, bool AFF>
hipError_t launch_skeleton_n(int geo, const ForceArgs& a, hipStream_t s) {
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
