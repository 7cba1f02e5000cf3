// FP32 element internal-force kernel for high orders (NGLL 11..16).  The
// force pass takes it at NGLL 11 and for irregular elements at 12; the
// matrix-core tile kernel (force_tile16.hip) is faster elsewhere.
//
// Same operator as force_f32.hip (Sec. II-B weak form: three forward and
// three transpose sum-factorised contractions around the pointwise
// Gamma map, isotropic stress and weighted flux; Sec. IV-D fused traversal
// and regular/irregular geometry paths), laid out for elements whose n^3
// points (up to 4096) do not fit one lane each:
//   one workgroup per element, one lane per (i, j) column (n^2 lanes, at most
//   256), the lane keeping u and the force accumulators of its n points
//   along zeta in registers;
//   the element is walked slice by slice in k: the xi and eta derivatives
//   read the slice of u from LDS, the zeta derivative the lane's own column;
//   the zeta part of the transpose contraction goes straight into the
//   column accumulators (point k feeds every k' with D[k][k']), the xi and
//   eta parts through one LDS slice of fluxes.
// LDS holds the element's node numbers, one slice of u (3 n^2), one slice of
// fluxes (6 n^2), D and (NGLL 12, 16) its transpose: 27 KB at NGLL 16, instead of the
// 12 n^3 floats (192 KB) a point-per-lane layout would need.
// At NGLL 16 a slice row is exactly one 16-lane DPP row of a wavefront, and
// the xi contractions (forward derivative and transpose flux) rotate the
// row's values across lanes (row_ror) instead of reading them from LDS.
// Assembly: plain read-modify-write inside a colour (with first-touch stores)
// or FP32 atomics, as in the lower-order kernel.
#include "dpp_rows.hpp"
#include "elem_common.hpp"

namespace semx {
namespace {

template <int NG>
struct ColShape {
  static constexpr int N2 = NG * NG;
  static constexpr int N3 = NG * NG * NG;
  static constexpr int BLK = ((N2 + 63) / 64) * 64;
};

// Three waves per SIMD: at NGLL 15-16 this costs a few spilled registers
// (64 bytes of scratch per lane at NGLL 16) and measured 11 % faster there
// (the kernel is latency-bound: more waves hide the slice barriers).
template <int NG, int GEO, bool ATOMIC>
__global__ __launch_bounds__(ColShape<NG>::BLK) __attribute__((amdgpu_waves_per_eu(3))) void force_col_kernel(
    ForceArgs a) {
  constexpr int N2 = ColShape<NG>::N2;
  constexpr int N3 = ColShape<NG>::N3;
  __shared__ int s_g[N3];
  __shared__ float s_u[3 * N2];
  __shared__ float s_q[6 * N2];
  __shared__ float s_D[N2];
  // D transposed (NGLL a multiple of 4): the xi and eta derivatives read row
  // i (j) of D, which differs per lane; at a row stride of 12 or 16 words
  // those reads share few LDS banks, down a column of s_Dt they are
  // consecutive across lanes.  Odd strides are conflict-free row-wise and
  // keep the vector reads of s_D (measured: transposing them is slower).
  constexpr bool TD = (NG % 4) == 0;
  __shared__ float s_Dt[TD ? N2 : 1];
  // NGLL 16: a slice row is one 16-lane DPP row, so the xi contractions
  // rotate values across the row instead of reading it from LDS; the
  // coefficients of rotation R are s_Cf[R][i] = D[i][src] (forward) and
  // s_Cb[R][i] = D[src][i] (transpose), src the lane it brings in.
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
  const float* __restrict__ u = a.u + (size_t)model * a.nglob * 3;
  float* f = a.f + (size_t)model * a.nglob * 3;
  const float* __restrict__ mat = a.mat + (size_t)model * a.nspec * 2 * N3 + (size_t)pos * 2 * N3;

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

  // the lane's column of u
  float uc[3][NG];
#pragma unroll
  for (int k = 0; k < NG; ++k) {
    const int g = s_g[ll + N2 * k];
    uc[0][k] = u[3 * (size_t)g + 0];
    uc[1][k] = u[3 * (size_t)g + 1];
    uc[2][k] = u[3 * (size_t)g + 2];
  }
  float acc[3][NG];  // sum_d sum_a D_{a, l_d} Phi_cd(...) at the column's points
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int k = 0; k < NG; ++k) acc[c][k] = 0.0f;

  float rx = 0.f, ry = 0.f;
  const float* src = nullptr;
  if constexpr (GEO == kTrilinear) {
    rx = a.xi[i];
    ry = a.xi[j];
    src = a.tri + (size_t)pos * 24;
  }
  if constexpr (GEO == kRegular) src = a.gam_el + (size_t)pos * 9;

  // The slice loop stays rolled (unrolled, the compiler hoists work across
  // slices and spills); the column arrays are indexed by the slice through
  // selects over the static column index, so they stay in registers.
#pragma unroll 1
  for (int k = 0; k < NG; ++k) {
    const int q = ll + N2 * k;
    if (k > 0) __syncthreads();  // the previous slice's readers are done
    float uk[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < NG; ++b)
      if (b == k) {
        uk[0] = uc[0][b];
        uk[1] = uc[1][b];
        uk[2] = uc[2][b];
      }
    if (act) {
      s_u[ll] = uk[0];
      s_u[N2 + ll] = uk[1];
      s_u[2 * N2 + ll] = uk[2];
    }
    __syncthreads();
    // reference derivatives du[c][d] at (i, j, k)
    float du[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) du[c][0] = du[c][1] = du[c][2] = 0.0f;
    if constexpr (XDPP) {
      float x0[3] = {0.f, 0.f, 0.f};
      row_contract3<0>(s_Cf + i, uk, x0);
#pragma unroll
      for (int c = 0; c < 3; ++c) du[c][0] = x0[c];
    }
#pragma unroll
    for (int b = 0; b < NG; ++b) {
      const float dj = TD ? s_Dt[b * NG + j] : s_D[j * NG + b];
      const float dk = s_D[k * NG + b];
      if constexpr (!XDPP) {
        const float di = TD ? s_Dt[b * NG + i] : s_D[i * NG + b];
#pragma unroll
        for (int c = 0; c < 3; ++c) du[c][0] += di * s_u[c * N2 + b + NG * j];
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        du[c][1] += dj * s_u[c * N2 + i + NG * b];
        du[c][2] += dk * uc[c][b];
      }
    }
    float G[9];
    if constexpr (GEO == kStored) {
      const float* gp = a.gam_pt + (size_t)pos * 9 * N3 + q;
#pragma unroll
      for (int d = 0; d < 9; ++d) G[d] = ldnt(gp + d * N3);
    }
    float Mg[9], scale, det;
    geom_map_from<GEO>(src, G, rx, ry, (GEO == kTrilinear) ? a.xi[k] : 0.f, Mg, scale, det);
    float gr[3][3];
    apply_map(du, Mg, gr);
    const float lw = ldnt(mat + q), mw = ldnt(mat + N3 + q);
    const float ltr = lw * (gr[0][0] + gr[1][1] + gr[2][2]);
    float sg[3][3];
    sg[0][0] = ltr + 2.0f * mw * gr[0][0];
    sg[1][1] = ltr + 2.0f * mw * gr[1][1];
    sg[2][2] = ltr + 2.0f * mw * gr[2][2];
    sg[0][1] = sg[1][0] = mw * (gr[0][1] + gr[1][0]);
    sg[0][2] = sg[2][0] = mw * (gr[0][2] + gr[2][0]);
    sg[1][2] = sg[2][1] = mw * (gr[1][2] + gr[2][1]);
    float phi[3][3];  // phi[c][d] = scale sum_b sg[c][b] Mg[d][b]
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d)
        phi[c][d] = scale * (sg[c][0] * Mg[d * 3 + 0] + sg[c][1] * Mg[d * 3 + 1] + sg[c][2] * Mg[d * 3 + 2]);
    // zeta part: point k feeds every point k' of the column with D[k][k']
#pragma unroll
    for (int b = 0; b < NG; ++b) {
      const float dkb = s_D[k * NG + b];
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c][b] += dkb * phi[c][2];
    }
    // xi and eta parts through the slice of fluxes
    if (act) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if constexpr (!XDPP) s_q[(2 * c + 0) * N2 + ll] = phi[c][0];
        s_q[(2 * c + 1) * N2 + ll] = phi[c][1];
      }
    }
    float sxy[3] = {0.f, 0.f, 0.f};
    if constexpr (XDPP) {
      const float p0[3] = {phi[0][0], phi[1][0], phi[2][0]};
      row_contract3<0>(s_Cb + i, p0, sxy);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float s = 0.0f;
#pragma unroll
      for (int b = 0; b < NG; ++b) {
        if constexpr (!XDPP) s += s_D[b * NG + i] * s_q[(2 * c + 0) * N2 + b + NG * j];
        s += s_D[b * NG + j] * s_q[(2 * c + 1) * N2 + i + NG * b];
      }
      sxy[c] += s;
    }
#pragma unroll
    for (int b = 0; b < NG; ++b)
      if (b == k) {
        acc[0][b] += sxy[0];
        acc[1][b] += sxy[1];
        acc[2][b] += sxy[2];
      }
  }

  if (act) {
#pragma unroll
    for (int k = 0; k < NG; ++k) {
      const int q = ll + N2 * k;
      float* fg = f + 3 * (size_t)s_g[q];
      if constexpr (ATOMIC) {
        unsafeAtomicAdd(fg + 0, -acc[0][k]);
        unsafeAtomicAdd(fg + 1, -acc[1][k]);
        unsafeAtomicAdd(fg + 2, -acc[2][k]);
      } else {
        const bool first = a.first && ((a.first[(size_t)pos * a.first_words + (q >> 5)] >> (q & 31)) & 1u);
        if (first) {
          fg[0] = -acc[0][k];
          fg[1] = -acc[1][k];
          fg[2] = -acc[2][k];
        } else {
          fg[0] = fg[0] - acc[0][k];
          fg[1] = fg[1] - acc[1][k];
          fg[2] = fg[2] - acc[2][k];
        }
      }
    }
  }
}

template <int NG, int GEO, bool ATOMIC>
hipError_t launch_col(const ForceArgs& a, hipStream_t s) {
  const int64_t nb = ((a.count + kNumXcd - 1) / kNumXcd) * kNumXcd;
  dim3 grid((unsigned)nb, (unsigned)a.nmodels), block(ColShape<NG>::BLK);
  force_col_kernel<NG, GEO, ATOMIC><<<grid, block, 0, s>>>(a);
  return hipGetLastError();
}

template <int NG>
hipError_t launch_col_n(int geo, bool atomic, const ForceArgs& a, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  switch (geo) {
    case kRegular:
      return atomic ? launch_col<NG, kRegular, true>(a, s) : launch_col<NG, kRegular, false>(a, s);
    case kStored:
      return atomic ? launch_col<NG, kStored, true>(a, s) : launch_col<NG, kStored, false>(a, s);
    case kTrilinear:
      return atomic ? launch_col<NG, kTrilinear, true>(a, s) : launch_col<NG, kTrilinear, false>(a, s);
    default:
      return hipErrorInvalidValue;
  }
}

// Memory skeleton of force_col_kernel (coloured assembly): the same grid,
// block mapping, node numbers staged in LDS, column gather of u, per-point
// material and (kStored) Gamma, first-touch bits and column scatter of f,
// without the slice contractions, the pointwise arithmetic and the slice
// barriers.  f receives meaningless values.
template <int NG, int GEO>
__global__ __launch_bounds__(ColShape<NG>::BLK) void force_col_skeleton_kernel(ForceArgs a) {
  constexpr int N2 = ColShape<NG>::N2;
  constexpr int N3 = ColShape<NG>::N3;
  __shared__ int s_g[N3];
  const int ngrp = (int)a.count;
  const int grp = xcd_group(ngrp);
  if (grp >= ngrp) return;  // uniform over the block
  const int pos = (int)a.pos0 + grp;
  const int l = threadIdx.x;
  const int model = blockIdx.y;
  const float* __restrict__ u = a.u + (size_t)model * a.nglob * 3;
  float* f = a.f + (size_t)model * a.nglob * 3;
  const float* __restrict__ mat = a.mat + (size_t)model * a.nspec * 2 * N3 + (size_t)pos * 2 * N3;
  for (int t = l; t < N3; t += blockDim.x) s_g[t] = ldnt(a.ibool + (size_t)pos * N3 + t);
  __syncthreads();
  if (l >= N2) return;  // no barrier follows
  float sg = 0.0f;
  if constexpr (GEO != kStored) {
    constexpr int NS = GEO == kRegular ? 9 : 24;
    const float* src = GEO == kRegular ? a.gam_el + (size_t)pos * 9 : a.tri + (size_t)pos * 24;
#pragma unroll
    for (int d = 0; d < NS; ++d) sg += src[d];
  }
#pragma unroll 4
  for (int k = 0; k < NG; ++k) {
    const int q = l + N2 * k;
    const int g = s_g[q];
    float m = sg + ldnt(mat + q) + ldnt(mat + N3 + q);
    if constexpr (GEO == kStored) {
      const float* gp = a.gam_pt + (size_t)pos * 9 * N3 + q;
#pragma unroll
      for (int d = 0; d < 9; ++d) m += ldnt(gp + d * N3);
    }
    const float x0 = u[3 * (size_t)g + 0], x1 = u[3 * (size_t)g + 1], x2 = u[3 * (size_t)g + 2];
    float* fg = f + 3 * (size_t)g;
    const bool first = a.first && ((a.first[(size_t)pos * a.first_words + (q >> 5)] >> (q & 31)) & 1u);
    if (first) {
      fg[0] = m * x0;
      fg[1] = m * x1;
      fg[2] = m * x2;
    } else {
      fg[0] = fg[0] + m * x0;
      fg[1] = fg[1] + m * x1;
      fg[2] = fg[2] + m * x2;
    }
  }
}

template <int NG>
hipError_t launch_col_skeleton_n(int geo, const ForceArgs& a, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  const int64_t nb = ((a.count + kNumXcd - 1) / kNumXcd) * kNumXcd;
  dim3 grid((unsigned)nb, (unsigned)a.nmodels), block(ColShape<NG>::BLK);
  switch (geo) {
    case kRegular: force_col_skeleton_kernel<NG, kRegular><<<grid, block, 0, s>>>(a); break;
    case kStored: force_col_skeleton_kernel<NG, kStored><<<grid, block, 0, s>>>(a); break;
    case kTrilinear: force_col_skeleton_kernel<NG, kTrilinear><<<grid, block, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_force_high_skeleton(int n, int geo, const ForceArgs& a, hipStream_t s) {
  switch (n) {
    case 11: return launch_col_skeleton_n<11>(geo, a, s);
    case 12: return launch_col_skeleton_n<12>(geo, a, s);
    case 13: return launch_col_skeleton_n<13>(geo, a, s);
    case 14: return launch_col_skeleton_n<14>(geo, a, s);
    case 15: return launch_col_skeleton_n<15>(geo, a, s);
    case 16: return launch_col_skeleton_n<16>(geo, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_force_high(int n, int geo, bool atomic, const ForceArgs& a, hipStream_t s) {
  switch (n) {
    case 11: return launch_col_n<11>(geo, atomic, a, s);
    case 12: return launch_col_n<12>(geo, atomic, a, s);
    case 13: return launch_col_n<13>(geo, atomic, a, s);
    case 14: return launch_col_n<14>(geo, atomic, a, s);
    case 15: return launch_col_n<15>(geo, atomic, a, s);
    case 16: return launch_col_n<16>(geo, atomic, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace semx
