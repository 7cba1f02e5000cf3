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

// First-touch bit of the lane's point (coloured assembly).  Point p's bit is
// bit p & 31 of word p >> 5 of the element's bitmask, so the 64 lanes of wave
// w read words 2w and 2w + 1: the pair is uniform over the wave, comes
// through the scalar cache, and turns into the lane's bit with one select on
// the 64-bit mask.  The f read that depends on the bit then waits for a
// scalar load, not for a vector-memory round trip.  Lanes past the element's
// points (p >= n^3) see bits of a zero word or of no point; they store nothing.
template <int N3>
__device__ __forceinline__ bool first_touch(const ForceArgs& a, int pos) {
  constexpr int NW = (N3 + 31) / 32;
  if (!a.first) return false;
  const uint32_t* w = a.first + (size_t)pos * a.first_words;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const uint64_t lo = wave * 2 < NW ? w[wave * 2] : 0u;
  const uint64_t hi = wave * 2 + 1 < NW ? w[wave * 2 + 1] : 0u;
  return __builtin_amdgcn_inverse_ballot_w64(lo | (hi << 32));
}

// Node number of local point (i, j, k) of the element at launch position
// `pos` from the ibool stream (elements without an affine numbering).
template <int NG>
__device__ __forceinline__ int node_of(const ForceArgs& a, int pos, int pp) {
  return ldnt(a.ibool + (size_t)pos * Shape<NG>::N3 + pp);
}

// The node span of an affine-numbered element (node g = g0 + i sx + j sy +
// k sz; four scalar loads per element, no per-point stream and no dependent
// round trip before the gather): raw buffer resources over the element's
// nodes in u and f, and the lane's byte offset into them.  With 32-bit
// offsets from a per-element base, the gather, the prior-force read and the
// store need no 64-bit address arithmetic.  The host classifies an element
// as affine only when its span fits a 31-bit byte offset.
struct AffSpan {
  __amdgpu_buffer_rsrc_t ru, rf;
  int off;
};

template <int NG>
__device__ __forceinline__ AffSpan aff_span(const ForceArgs& a, int pos, const float* u, float* f, int i, int j,
                                            int k) {
  const int* r = a.aff + (size_t)pos * 4;
  const int sx = r[1], sy = r[2], sz = r[3];
  const int lo = (NG - 1) * (min(sx, 0) + min(sy, 0) + min(sz, 0));
  const int gmin = r[0] + lo;
  const int bytes = ((NG - 1) * (abs(sx) + abs(sy) + abs(sz)) + 1) * 12;
  AffSpan s;
  s.ru = __builtin_amdgcn_make_buffer_rsrc((void*)(u + 3 * (size_t)gmin), (short)0, bytes, kBufferWord3);
  s.rf = __builtin_amdgcn_make_buffer_rsrc((void*)(f + 3 * (size_t)gmin), (short)0, bytes, kBufferWord3);
  s.off = (i * sx + j * sy + k * sz - lo) * 12;
  return s;
}

typedef unsigned semx_v3u __attribute__((ext_vector_type(3)));

__device__ __forceinline__ void unpack3(semx_v3u v, float x[3]) {
  x[0] = __uint_as_float(v.x);
  x[1] = __uint_as_float(v.y);
  x[2] = __uint_as_float(v.z);
}

// u at the lane's node of an affine element.
__device__ __forceinline__ void gather_affine(const AffSpan& s, float x[3]) {
  unpack3(__builtin_amdgcn_raw_buffer_load_b96(s.ru, s.off, 0, 0), x);
}

// Prior force at the lane's node of an affine element: at first-touch points
// the offset is pushed out of range, so the hardware returns zeros and
// fetches nothing, and the read stays one unconditional instruction that the
// compiler counts exactly (no branch, so the wait for u does not also wait
// for f).  2^31 lies past any num_records <= 2^31 - 1, and adding the 8 bytes
// of the last dword cannot wrap a 32-bit offset.
__device__ __forceinline__ void prior_force_affine(const AffSpan& s, bool first, float x[3]) {
  unpack3(__builtin_amdgcn_raw_buffer_load_b96(s.rf, first ? INT32_MIN : s.off, 0, 0), x);
}

__device__ __forceinline__ void store_affine(const AffSpan& s, const float x[3]) {
  semx_v3u v;
  v.x = __float_as_uint(x[0]);
  v.y = __float_as_uint(x[1]);
  v.z = __float_as_uint(x[2]);
  __builtin_amdgcn_raw_buffer_store_b96(v, s.rf, s.off, 0, 0);
}

// Per-element geometry that is uniform over the workgroup: Gamma (kRegular,
// 9 floats) or the trilinear coefficients (kTrilinear, 24 floats).
template <int GEO>
struct ElemGeom {
  static constexpr int NS = GEO == kRegular ? 9 : (GEO == kTrilinear ? 24 : 1);
  float v[NS];
};

// One workgroup owns one element (one lane per GLL point).  Every load the
// element's first half needs is issued before its first wait: the constant
// tables (D and the GLL nodes, L2-resident), the per-element scalars
// (node-numbering coefficients, geometry, first-touch words), the material
// and the u gather.  The prior-force read depends only on the first-touch bit
// (a scalar load) and is consumed at the very end, so its latency runs under
// the transpose contractions.
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

  const float lw = ldnt(mat + (size_t)pos * 2 * N3 + pp);
  const float mw = ldnt(mat + (size_t)pos * 2 * N3 + N3 + pp);
  float uo[3], fo[3] = {0.0f, 0.0f, 0.0f};
  AffSpan sp;
  int g = 0;
  bool first = false;
  if constexpr (AFF) {
    sp = aff_span<NG>(a, pos, u, f, i, j, k);
    gather_affine(sp, uo);
    if constexpr (ATOMIC) {
      const int* r = a.aff + (size_t)pos * 4;
      g = r[0] + i * r[1] + j * r[2] + k * r[3];
    } else {
      first = first_touch<N3>(a, pos);
    }
  } else {
    g = node_of<NG>(a, pos, pp);
    uo[0] = u[3 * (size_t)g + 0];
    uo[1] = u[3 * (size_t)g + 1];
    uo[2] = u[3 * (size_t)g + 2];
    if constexpr (!ATOMIC) {
      if (!first_touch<N3>(a, pos)) {
        fo[0] = f[3 * (size_t)g + 0];
        fo[1] = f[3 * (size_t)g + 1];
        fo[2] = f[3 * (size_t)g + 2];
      }
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
    s_u[pp] = uo[0];
    s_u[N3 + pp] = uo[1];
    s_u[2 * N3 + pp] = uo[2];
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
  // the prior force of an affine element is read here: it is needed only
  // after the transpose contractions, and issuing it earlier keeps three
  // more registers live through the stress (65 instead of 63, 7 waves per
  // SIMD instead of 8)
  if constexpr (AFF && !ATOMIC) prior_force_affine(sp, first, fo);
  __syncthreads();

  float F[3];
  ref_div<NG>(s_q, s_D, i, j, k, F);
  if (act) {
    if constexpr (ATOMIC) {
      float* fg = f + 3 * (size_t)g;
      // an element-interior point is its node's only reference (checked at
      // upload): its force is the node's whole force, stored without an atomic
      const bool own = a.excl_interior && i > 0 && i < NG - 1 && j > 0 && j < NG - 1 && k > 0 && k < NG - 1;
      if (own) {
        fg[0] = F[0];
        fg[1] = F[1];
        fg[2] = F[2];
      } else {
        unsafeAtomicAdd(fg + 0, F[0]);
        unsafeAtomicAdd(fg + 1, F[1]);
        unsafeAtomicAdd(fg + 2, F[2]);
      }
    } else {
      const float out[3] = {fo[0] + F[0], fo[1] + F[1], fo[2] + F[2]};
      if constexpr (AFF) {
        store_affine(sp, out);
      } else {
        float* fg = f + 3 * (size_t)g;
        fg[0] = out[0];
        fg[1] = out[1];
        fg[2] = out[2];
      }
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
  s += ldnt(mat + (size_t)pos * 2 * N3 + p) + ldnt(mat + (size_t)pos * 2 * N3 + N3 + p);
  float uo[3], fo[3] = {0.0f, 0.0f, 0.0f};
  if constexpr (AFF) {
    const AffSpan sp = aff_span<NG>(a, pos, u, f, p % NG, (p / NG) % NG, p / (NG * NG));
    gather_affine(sp, uo);
    prior_force_affine(sp, first_touch<N3>(a, pos), fo);
    const float out[3] = {fo[0] + s * uo[0], fo[1] + s * uo[1], fo[2] + s * uo[2]};
    store_affine(sp, out);
  } else {
    const int g = node_of<NG>(a, pos, p);
    uo[0] = u[3 * (size_t)g + 0];
    uo[1] = u[3 * (size_t)g + 1];
    uo[2] = u[3 * (size_t)g + 2];
    if (!first_touch<N3>(a, pos)) {
      fo[0] = f[3 * (size_t)g + 0];
      fo[1] = f[3 * (size_t)g + 1];
      fo[2] = f[3 * (size_t)g + 2];
    }
    float* fg = f + 3 * (size_t)g;
    fg[0] = fo[0] + s * uo[0];
    fg[1] = fo[1] + s * uo[1];
    fg[2] = fo[2] + s * uo[2];
  }
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
