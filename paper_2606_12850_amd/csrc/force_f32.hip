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
  load_elem_geom<GEO>(a, pos, eg);
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
    sp = aff_span<NG, 3>(a, pos, u, f, i, j, k);
    gather_affine<3>(sp, uo);
    if constexpr (ATOMIC) {
      g = aff_node(a, pos, i, j, k);
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

  pin_elem_geom<GEO>(eg);
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
  if constexpr (AFF && !ATOMIC) prior_force_affine<3>(sp, first, fo);
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
        store_affine<3>(sp, out);
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
    const AffSpan sp = aff_span<NG, 3>(a, pos, u, f, p % NG, (p / NG) % NG, p / (NG * NG));
    gather_affine<3>(sp, uo);
    prior_force_affine<3>(sp, first_touch<N3>(a, pos), fo);
    const float out[3] = {fo[0] + s * uo[0], fo[1] + s * uo[1], fo[2] + s * uo[2]};
    store_affine<3>(sp, out);
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
