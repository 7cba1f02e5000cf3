// FP32 element force kernels of the scalar (acoustic) operator f = -K p.
//
// The acoustic weak form (the paper's equal-accuracy experiment runs an
// acoustic solver, Sec. V-C) with GLL quadrature (Sec. II-B) has the
// elastic operator's structure with one field component: three forward
// contractions with D give the reference gradient of p, the geometry map
// gives the physical gradient, the flux is Phi_d = (W / rho) sum_b g_b
// Gamma_db, and three transpose contractions with D^T give the force.  The
// per-point weight W / rho (W = w_i w_j w_k det J) sits in the first half of
// the material table; the mass carries W / kappa.
//
// Two layouts, as for the elastic operator:
//   force_ac_kernel      NGLL <= 10: one workgroup per element, one lane per
//                        point, p and the three flux cubes in LDS;
//   force_ac_col_kernel  NGLL 11..16: one lane per (i, j) column, the
//                        column of p and its force accumulators in registers,
//                        the element walked slice by slice in k (at NGLL 16
//                        the xi contractions on DPP row rotations).
// Geometry paths, first-touch coloured stores and atomic assembly follow
// the elastic kernels.
#include "dpp_rows.hpp"
#include "elem_common.hpp"

namespace semx {
namespace {

// physical gradient times det' (geometry map Mg), then the weighted flux
// phi_d = scale * r * sum_b g_b Mg[d][b]
__device__ __forceinline__ void scalar_flux(const float d[3], const float Mg[9], float r, float scale,
                                            float phi[3]) {
  float g[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) g[b] = d[0] * Mg[0 * 3 + b] + d[1] * Mg[1 * 3 + b] + d[2] * Mg[2 * 3 + b];
  const float s = r * scale;
#pragma unroll
  for (int dd = 0; dd < 3; ++dd) phi[dd] = s * (g[0] * Mg[dd * 3 + 0] + g[1] * Mg[dd * 3 + 1] + g[2] * Mg[dd * 3 + 2]);
}

__device__ __forceinline__ bool first_bit(const ForceArgs& a, int pos, int q) {
  return a.first && ((a.first[(size_t)pos * a.first_words + (q >> 5)] >> (q & 31)) & 1u);
}

// One workgroup per element, one lane per point.  As in the elastic FP32
// kernel, every load of the element's first half is issued before its first
// wait (D and the GLL nodes, the element's geometry scalars, the first-touch
// words through the scalar cache, the material and the p gather), and an
// affine-numbered element (AFF) gathers, reads its prior force and stores
// through buffers over its node span, the prior force as one unconditional
// request issued after the flux.
template <int NG, int GEO, bool ATOMIC, bool AFF>
__global__ __launch_bounds__(Shape<NG>::BLK) void force_ac_kernel(ForceArgs a) {
  constexpr int N3 = Shape<NG>::N3;
  constexpr int ND = NG * NG;
  __shared__ float s_p[N3];
  __shared__ float s_q[3 * N3];
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
  const float* __restrict__ u = a.u + (size_t)model * a.nglob;
  float* f = a.f + (size_t)model * a.nglob;
  const float* __restrict__ mat = a.mat + ((size_t)model * a.nspec + pos) * 2 * N3;

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
  const float r = ldnt(mat + pp);
  float pv, fo = 0.0f;
  AffSpan sp;
  int g = 0;
  bool first = false;
  if constexpr (AFF) {
    sp = aff_span<NG, 1>(a, pos, u, f, i, j, k);
    gather_affine<1>(sp, &pv);
    if constexpr (ATOMIC) g = aff_node(a, pos, i, j, k);
    else first = first_touch<N3>(a, pos);
  } else {
    g = node_of<NG>(a, pos, pp);
    pv = u[g];
    if constexpr (!ATOMIC)
      if (!first_touch<N3>(a, pos)) fo = f[g];
  }
  pin_elem_geom<GEO>(eg);
  if (p < ND + NG) s_D[p] = tab;
  if (act) s_p[pp] = pv;
  __syncthreads();

  float rx = 0.f, ry = 0.f, rz = 0.f;
  if constexpr (GEO == kTrilinear) {
    rx = s_D[ND + i];
    ry = s_D[ND + j];
    rz = s_D[ND + k];
  }
  float d[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    d[0] += s_D[i * NG + q] * s_p[q + NG * (j + NG * k)];
    d[1] += s_D[j * NG + q] * s_p[i + NG * (q + NG * k)];
    d[2] += s_D[k * NG + q] * s_p[i + NG * (j + NG * q)];
  }
  float Mg[9], scale, det;
  geom_map_from<GEO>(eg.v, G, rx, ry, rz, Mg, scale, det);
  float phi[3];
  scalar_flux(d, Mg, r, scale, phi);
  if (act) {
    s_q[pp] = phi[0];
    s_q[N3 + pp] = phi[1];
    s_q[2 * N3 + pp] = phi[2];
  }
  if constexpr (AFF && !ATOMIC) prior_force_affine<1>(sp, first, &fo);
  __syncthreads();

  float sum = 0.0f;
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    sum += s_D[q * NG + i] * s_q[q + NG * (j + NG * k)];
    sum += s_D[q * NG + j] * s_q[N3 + i + NG * (q + NG * k)];
    sum += s_D[q * NG + k] * s_q[2 * N3 + i + NG * (j + NG * q)];
  }
  if (act) {
    if constexpr (ATOMIC) {
      // element-interior points own their node (checked at upload, f zero on entry)
      const bool own = a.excl_interior && i > 0 && i < NG - 1 && j > 0 && j < NG - 1 && k > 0 && k < NG - 1;
      if (own) f[g] = -sum;
      else unsafeAtomicAdd(f + g, -sum);
    } else {
      const float out = fo - sum;
      if constexpr (AFF) store_affine<1>(sp, &out);
      else f[g] = out;
    }
  }
}

template <int NG>
struct AcColShape {
  static constexpr int N2 = NG * NG;
  static constexpr int N3 = NG * NG * NG;
  static constexpr int BLK = ((N2 + 63) / 64) * 64;
};

template <int NG, int GEO, bool ATOMIC>
__global__ __launch_bounds__(AcColShape<NG>::BLK) void force_ac_col_kernel(ForceArgs a) {
  constexpr int N2 = AcColShape<NG>::N2;
  constexpr int N3 = AcColShape<NG>::N3;
  __shared__ int s_g[N3];
  __shared__ float s_p[N2];
  __shared__ float s_q[2 * N2];
  __shared__ float s_D[N2];
  constexpr bool TD = (NG % 4) == 0;  // D transposed for row strides 12, 16 (see force_col_kernel)
  __shared__ float s_Dt[TD ? N2 : 1];
  // NGLL 16: xi contractions on DPP row rotations, coefficients of rotation
  // R in s_Cf[R][i] = D[i][src], s_Cb[R][i] = D[src][i] (see force_col_kernel)
  constexpr bool XDPP = NG == 16;
  __shared__ float s_Cf[XDPP ? 256 : 1];
  __shared__ float s_Cb[XDPP ? 256 : 1];

  const int ngrp = (int)a.count;
  const int grp = xcd_group(ngrp);
  if (grp >= ngrp) return;  // uniform over the block
  const int pos = (int)a.pos0 + grp;

  const int l = threadIdx.x;
  const bool act = l < N2;
  const int ll = act ? l : 0;
  const int i = ll % NG, j = ll / NG;

  const int model = blockIdx.y;
  const float* __restrict__ u = a.u + (size_t)model * a.nglob;
  float* f = a.f + (size_t)model * a.nglob;
  const float* __restrict__ mat = a.mat + ((size_t)model * a.nspec + pos) * 2 * N3;

  for (int t = l; t < N2; t += blockDim.x) {
    s_D[t] = a.D[t];
    if constexpr (TD) s_Dt[(t % NG) * NG + t / NG] = a.D[t];
  }
  if constexpr (XDPP) {
    float src[16];
    row_sources<0>((float)(l & 15), src);  // every lane active (n^2 = 256 = block)
    if (l < 16) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int sl = (int)src[r];
        s_Cf[r * 16 + l] = a.D[l * 16 + sl];
        s_Cb[r * 16 + l] = a.D[sl * 16 + l];
      }
    }
  }
  for (int t = l; t < N3; t += blockDim.x) s_g[t] = ldnt(a.ibool + (size_t)pos * N3 + t);
  __syncthreads();

  float pc[NG];  // the lane's column of p
#pragma unroll
  for (int k = 0; k < NG; ++k) pc[k] = u[s_g[ll + N2 * k]];
  float acc[NG];  // sum_d sum_a D_{a, l_d} Phi_d(...) at the column's points
#pragma unroll
  for (int k = 0; k < NG; ++k) acc[k] = 0.0f;

  float rx = 0.f, ry = 0.f;
  const float* src = nullptr;
  if constexpr (GEO == kTrilinear) {
    rx = a.xi[i];
    ry = a.xi[j];
    src = a.tri + (size_t)pos * 24;
  }
  if constexpr (GEO == kRegular) src = a.gam_el + (size_t)pos * 9;

  // rolled slice loop, column entries picked by selects (stay in registers)
#pragma unroll 1
  for (int k = 0; k < NG; ++k) {
    const int q = ll + N2 * k;
    if (k > 0) __syncthreads();  // the previous slice's readers are done
    float pk = 0.0f;
#pragma unroll
    for (int b = 0; b < NG; ++b)
      if (b == k) pk = pc[b];
    if (act) s_p[ll] = pk;
    __syncthreads();
    float d[3] = {0.f, 0.f, 0.f};
    if constexpr (XDPP) row_contract1<0>(s_Cf + i, pk, d[0]);
#pragma unroll
    for (int b = 0; b < NG; ++b) {
      if constexpr (!XDPP) d[0] += (TD ? s_Dt[b * NG + i] : s_D[i * NG + b]) * s_p[b + NG * j];
      d[1] += (TD ? s_Dt[b * NG + j] : s_D[j * NG + b]) * s_p[i + NG * b];
      d[2] += s_D[k * NG + b] * pc[b];
    }
    float G[9];
    if constexpr (GEO == kStored) {
      const float* gp = a.gam_pt + (size_t)pos * 9 * N3 + q;
#pragma unroll
      for (int dd = 0; dd < 9; ++dd) G[dd] = ldnt(gp + dd * N3);
    }
    float Mg[9], scale, det;
    geom_map_from<GEO>(src, G, rx, ry, (GEO == kTrilinear) ? a.xi[k] : 0.f, Mg, scale, det);
    float phi[3];
    scalar_flux(d, Mg, ldnt(mat + q), scale, phi);
    // zeta part: point k feeds every point k' of the column with D[k][k']
#pragma unroll
    for (int b = 0; b < NG; ++b) acc[b] += s_D[k * NG + b] * phi[2];
    if (act) {
      if constexpr (!XDPP) s_q[ll] = phi[0];
      s_q[N2 + ll] = phi[1];
    }
    float sxy = 0.0f;
    if constexpr (XDPP) row_contract1<0>(s_Cb + i, phi[0], sxy);
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NG; ++b) {
      if constexpr (!XDPP) sxy += s_D[b * NG + i] * s_q[b + NG * j];
      sxy += s_D[b * NG + j] * s_q[N2 + i + NG * b];
    }
#pragma unroll
    for (int b = 0; b < NG; ++b)
      if (b == k) acc[b] += sxy;
  }

  if (act) {
#pragma unroll
    for (int k = 0; k < NG; ++k) {
      const int q = ll + N2 * k;
      float* fg = f + s_g[q];
      if constexpr (ATOMIC) {
        unsafeAtomicAdd(fg, -acc[k]);
      } else {
        if (first_bit(a, pos, q)) *fg = -acc[k];
        else *fg = *fg - acc[k];
      }
    }
  }
}

template <int NG, int GEO, bool ATOMIC, bool AFF>
hipError_t launch_ac(const ForceArgs& a, hipStream_t s) {
  const int64_t nb = ((a.count + kNumXcd - 1) / kNumXcd) * kNumXcd;
  if constexpr (NG <= kMaxNLow) {
    dim3 grid((unsigned)nb, (unsigned)a.nmodels), block(Shape<NG>::BLK);
    force_ac_kernel<NG, GEO, ATOMIC, AFF><<<grid, block, 0, s>>>(a);
  } else {
    dim3 grid((unsigned)nb, (unsigned)a.nmodels), block(AcColShape<NG>::BLK);
    force_ac_col_kernel<NG, GEO, ATOMIC><<<grid, block, 0, s>>>(a);
  }
  return hipGetLastError();
}

template <int NG, bool AFF>
hipError_t launch_ac_g(int geo, bool atomic, const ForceArgs& a, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  switch (geo) {
    case kRegular:
      return atomic ? launch_ac<NG, kRegular, true, AFF>(a, s) : launch_ac<NG, kRegular, false, AFF>(a, s);
    case kStored:
      return atomic ? launch_ac<NG, kStored, true, AFF>(a, s) : launch_ac<NG, kStored, false, AFF>(a, s);
    case kTrilinear:
      return atomic ? launch_ac<NG, kTrilinear, true, AFF>(a, s) : launch_ac<NG, kTrilinear, false, AFF>(a, s);
    default:
      return hipErrorInvalidValue;
  }
}

// the column kernel (NGLL 11..16) reads node numbers only
template <int NG>
hipError_t launch_ac_n(int geo, bool atomic, bool aff, const ForceArgs& a, hipStream_t s) {
  if constexpr (NG <= kMaxNLow) {
    if (aff) return launch_ac_g<NG, true>(geo, atomic, a, s);
  }
  return launch_ac_g<NG, false>(geo, atomic, a, s);
}

hipError_t launch_ac_any(int n, int geo, bool atomic, bool aff, const ForceArgs& a, hipStream_t s) {
  switch (n) {
    case 2: return launch_ac_n<2>(geo, atomic, aff, a, s);
    case 3: return launch_ac_n<3>(geo, atomic, aff, a, s);
    case 4: return launch_ac_n<4>(geo, atomic, aff, a, s);
    case 5: return launch_ac_n<5>(geo, atomic, aff, a, s);
    case 6: return launch_ac_n<6>(geo, atomic, aff, a, s);
    case 7: return launch_ac_n<7>(geo, atomic, aff, a, s);
    case 8: return launch_ac_n<8>(geo, atomic, aff, a, s);
    case 9: return launch_ac_n<9>(geo, atomic, aff, a, s);
    case 10: return launch_ac_n<10>(geo, atomic, aff, a, s);
    case 11: return launch_ac_n<11>(geo, atomic, aff, a, s);
    case 12: return launch_ac_n<12>(geo, atomic, aff, a, s);
    case 13: return launch_ac_n<13>(geo, atomic, aff, a, s);
    case 14: return launch_ac_n<14>(geo, atomic, aff, a, s);
    case 15: return launch_ac_n<15>(geo, atomic, aff, a, s);
    case 16: return launch_ac_n<16>(geo, atomic, aff, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_force_acoustic(int n, int geo, bool atomic, int64_t naff, const ForceArgs& a, hipStream_t s) {
  return split_affine(naff, a, [&](const ForceArgs& b, bool aff) { return launch_ac_any(n, geo, atomic, aff, b, s); });
}

}  // namespace semx
