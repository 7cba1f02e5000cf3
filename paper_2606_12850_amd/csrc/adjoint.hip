// Discrete adjoint of the explicit Newmark run and the sensitivity kernels
// K_lambda, K_mu, K_rho (gradients of a seismogram misfit with respect to
// lambda, mu and rho at every element-local point).
//
// The forward run is, for n >= 1, the central-difference recursion
//   M (u^{n+1} - 2u^n + u^{n-1}) = dt^2 (f_src^n - K u^n),  M u^1 = dt^2/2 f_src^0,
// with seismograms s^n = R u^n.  For chi(s) with g^m = R^T dchi/ds^m the
// adjoint fields run backwards, psi^{nt+1} = psi^{nt+2} = 0,
//   psi^m = 2 psi^{m+1} - psi^{m+2} + M^{-1} (dt^2 (-K psi^{m+1}) + g^m),
// reusing the force operator (K is symmetric), and, with W = w_i w_j w_k det J,
//   dchi/dlambda = -dt^2 sum_{m=1}^{nt-1} W div psi^{m+1} div u^m,
//   dchi/dmu     = -dt^2 sum_{m=1}^{nt-1} 2 W eps(psi^{m+1}) : eps(u^m),
//   dchi/drho    = -dt^2 sum_{m=1}^{nt-1} W psi^{m+1} . a^m  -  W psi^1 . u^1,
// (the last from u^{m+1} - 2u^m + u^{m-1} = dt^2 a^m, which avoids the FP32
// cancellation of the displacement second difference).  The elastic operator
// is the one of the paper's Sec. II-B weak form; K linear in (lambda, mu) and
// the lumped mass linear in rho give the parameter derivatives above.
//
// Forward states are checkpointed every `every` steps; the backward pass
// recomputes each segment from its checkpoint (bitwise equal to the first
// pass with coloured assembly) and keeps u^m, a^m of the segment in memory.
#include <cmath>
#include <cstring>

#include <algorithm>
#include <string>

#include "elem_common.hpp"

namespace semx {
namespace {

struct AdjArgs {
  ForceArgs fa;             // fa.u = psi^{m+1}, fa.f = force accumulator
  const float* um;          // u^m  [nmodels][nglob][3]
  const float* am;          // a^m
  const double* wdet;       // [nspec][n3] launch order
  double* kl;               // [nmodels][nspec][n3] launch order, FP64 accumulators
  double* km;
  double* kr;
  float coef;               // -dt^2
  float uscale;             // power-of-two scale applied to u^m, a^m of this segment
  double inv_uscale;        // 1 / uscale, applied before accumulating
};

// Fused adjoint force + sensitivity accumulation, one element per block.
template <int NG, int GEO, bool ATOMIC>
__global__ __launch_bounds__(Shape<NG>::BLK) void adjoint_force_kernel(AdjArgs A) {
  constexpr int N3 = Shape<NG>::N3;
  __shared__ float s_u[3 * N3];  // psi^{m+1}
  __shared__ float s_v[3 * N3];  // u^m
  __shared__ float s_q[9 * N3];
  __shared__ float s_D[NG * NG];
  const ForceArgs& a = A.fa;
  const int grp = xcd_group((int)a.count);
  if (grp >= a.count) return;
  const int pos = (int)a.pos0 + grp;
  const int p = threadIdx.x;
  const bool act = p < N3;
  const int pp = act ? p : 0;
  const int i = pp % NG, j = (pp / NG) % NG, k = pp / (NG * NG);
  const int model = blockIdx.y;
  const size_t vofs = (size_t)model * a.nglob * 3;
  const float* psi = a.u + vofs;
  float* f = a.f + vofs;
  const float* mat = a.mat + (size_t)model * a.nspec * 2 * N3;

  const int g = a.ibool[(size_t)pos * N3 + pp];
  float G[9];
  if constexpr (GEO == kStored) {
#pragma unroll
    for (int d = 0; d < 9; ++d) G[d] = a.gam_pt[((size_t)pos * 9 + d) * N3 + pp];
  }
  const float lw = mat[(size_t)pos * 2 * N3 + pp], mw = mat[(size_t)pos * 2 * N3 + N3 + pp];
  const float W = (float)A.wdet[(size_t)pos * N3 + pp];
  float ps[3], uu[3], aa[3], f0[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    ps[c] = psi[3 * (size_t)g + c];
    uu[c] = A.uscale * A.um[vofs + 3 * (size_t)g + c];
    aa[c] = A.uscale * A.am[vofs + 3 * (size_t)g + c];
    if constexpr (!ATOMIC) f0[c] = f[3 * (size_t)g + c];
  }
  if (p < NG * NG) s_D[p] = a.D[p];
  if (act) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      s_u[c * N3 + pp] = ps[c];
      s_v[c * N3 + pp] = uu[c];
    }
  }
  float rx = 0.f, ry = 0.f, rz = 0.f;
  if constexpr (GEO == kTrilinear) {
    rx = a.xi[i];
    ry = a.xi[j];
    rz = a.xi[k];
  }
  __syncthreads();

  float dp[3][3], du[3][3];
  ref_grad<NG>(s_u, s_D, i, j, k, dp);
  ref_grad<NG>(s_v, s_D, i, j, k, du);
  float Mg[9], scale, det;
  geom_map<GEO>(a, pos, G, rx, ry, rz, Mg, scale, det);
  float gp[3][3], gu[3][3];
  apply_map(dp, Mg, gp);
  apply_map(du, Mg, gu);
  // sensitivity densities (gp, gu are det' times the physical gradients)
  if (act) {
    const float divp = gp[0][0] + gp[1][1] + gp[2][2];
    const float divu = gu[0][0] + gu[1][1] + gu[2][2];
    float ee = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int b = 0; b < 3; ++b) ee += 0.25f * (gp[c][b] + gp[b][c]) * (gu[c][b] + gu[b][c]);
    const size_t kq = ((size_t)model * a.nspec + pos) * N3 + pp;
    const float ws = A.coef * W * scale;
    A.kl[kq] += (double)(ws * divp * divu) * A.inv_uscale;
    A.km[kq] += (double)(2.0f * ws * ee) * A.inv_uscale;
    A.kr[kq] += (double)(A.coef * W * (ps[0] * aa[0] + ps[1] * aa[1] + ps[2] * aa[2])) * A.inv_uscale;
  }
  stress_flux(gp, lw, mw, scale, Mg, s_q, N3, pp, act);
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
      fg[0] = f0[0] + F[0];
      fg[1] = f0[1] + F[1];
      fg[2] = f0[2] + F[2];
    }
  }
}

template <int NG>
hipError_t launch_adj_n(int geo, bool atomic, const AdjArgs& A, hipStream_t s) {
  if (A.fa.count <= 0) return hipSuccess;
  const int64_t nb = ((A.fa.count + kNumXcd - 1) / kNumXcd) * kNumXcd;
  dim3 grid((unsigned)nb, (unsigned)A.fa.nmodels), block(Shape<NG>::BLK);
#define SEMX_ADJ_LAUNCH(GEO)                                                      \
  if (atomic) adjoint_force_kernel<NG, GEO, true><<<grid, block, 0, s>>>(A);      \
  else adjoint_force_kernel<NG, GEO, false><<<grid, block, 0, s>>>(A);
  switch (geo) {
    case kRegular: SEMX_ADJ_LAUNCH(kRegular) break;
    case kStored: SEMX_ADJ_LAUNCH(kStored) break;
    case kTrilinear: SEMX_ADJ_LAUNCH(kTrilinear) break;
    default: return hipErrorInvalidValue;
  }
#undef SEMX_ADJ_LAUNCH
  return hipGetLastError();
}

// NGLL 11..16: the same fused adjoint force and sensitivity accumulation
// on the column layout of the high-order force kernel (one lane per (i, j)
// column, psi and u^m of the column in registers, slices of both and of
// the fluxes through LDS; the zeta part of the transpose contraction goes
// into the column accumulators).
template <int NG>
struct AdjCol {
  static constexpr int N2 = NG * NG;
  static constexpr int N3 = NG * NG * NG;
  static constexpr int BLK = ((N2 + 63) / 64) * 64;
};

// Two waves per SIMD: left to itself the compiler takes up to 306 VGPRs and
// AGPRs at NGLL 14-16 (one wave per SIMD); capped at 256 it spills 8
// registers at NGLL 16 (trilinear) and none elsewhere, and the adjoint pass
// measured 7-26 % faster.  The DPP row contractions of force_col_kernel
// raise the pressure here (two column fields) and measured slower, with or
// without the cap.
template <int NG, int GEO, bool ATOMIC>
__global__ __launch_bounds__(AdjCol<NG>::BLK) __attribute__((amdgpu_waves_per_eu(2))) void adjoint_col_kernel(
    AdjArgs A) {
  constexpr int N2 = AdjCol<NG>::N2;
  constexpr int N3 = AdjCol<NG>::N3;
  __shared__ int s_g[N3];
  __shared__ float s_w[6 * N2];  // slice of psi (components 0..2) and u^m (3..5)
  __shared__ float s_q[6 * N2];  // slice of xi and eta fluxes
  __shared__ float s_D[N2];
  constexpr bool TD = (NG % 4) == 0;  // D transposed for row strides 12, 16 (see force_col_kernel)
  __shared__ float s_Dt[TD ? N2 : 1];
  const ForceArgs& a = A.fa;
  const int grp = xcd_group((int)a.count);
  if (grp >= a.count) return;
  const int pos = (int)a.pos0 + grp;
  const int l = threadIdx.x;
  const bool act = l < N2;
  const int ll = act ? l : 0;
  const int i = ll % NG, j = ll / NG;
  const int model = blockIdx.y;
  const size_t vofs = (size_t)model * a.nglob * 3;
  const float* psi = a.u + vofs;
  float* f = a.f + vofs;
  const float* mat = a.mat + (size_t)model * a.nspec * 2 * N3 + (size_t)pos * 2 * N3;

  for (int t = l; t < N2; t += blockDim.x) {
    s_D[t] = a.D[t];
    if constexpr (TD) s_Dt[(t % NG) * NG + t / NG] = a.D[t];
  }
  for (int t = l; t < N3; t += blockDim.x) s_g[t] = a.ibool[(size_t)pos * N3 + t];
  __syncthreads();

  float pc[3][NG], uc[3][NG], acc[3][NG];
#pragma unroll
  for (int k = 0; k < NG; ++k) {
    const size_t g3 = 3 * (size_t)s_g[ll + N2 * k];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      pc[c][k] = psi[g3 + c];
      uc[c][k] = A.uscale * A.um[vofs + g3 + c];
      acc[c][k] = 0.0f;
    }
  }
  float rx = 0.f, ry = 0.f;
  const float* src = nullptr;
  if constexpr (GEO == kTrilinear) {
    rx = a.xi[i];
    ry = a.xi[j];
    src = a.tri + (size_t)pos * 24;
  }
  if constexpr (GEO == kRegular) src = a.gam_el + (size_t)pos * 9;

#pragma unroll 1
  for (int k = 0; k < NG; ++k) {
    const int q = ll + N2 * k;
    if (k > 0) __syncthreads();  // the previous slice's readers are done
    float pk[3] = {0.f, 0.f, 0.f}, uk[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < NG; ++b)
      if (b == k) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          pk[c] = pc[c][b];
          uk[c] = uc[c][b];
        }
      }
    if (act) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        s_w[c * N2 + ll] = pk[c];
        s_w[(3 + c) * N2 + ll] = uk[c];
      }
    }
    __syncthreads();
    float dp[3][3], du[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d) dp[c][d] = du[c][d] = 0.0f;
#pragma unroll
    for (int b = 0; b < NG; ++b) {
      const float di = TD ? s_Dt[b * NG + i] : s_D[i * NG + b];
      const float dj = TD ? s_Dt[b * NG + j] : s_D[j * NG + b];
      const float dk = s_D[k * NG + b];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        dp[c][0] += di * s_w[c * N2 + b + NG * j];
        dp[c][1] += dj * s_w[c * N2 + i + NG * b];
        dp[c][2] += dk * pc[c][b];
        du[c][0] += di * s_w[(3 + c) * N2 + b + NG * j];
        du[c][1] += dj * s_w[(3 + c) * N2 + i + NG * b];
        du[c][2] += dk * uc[c][b];
      }
    }
    float G[9];
    if constexpr (GEO == kStored) {
#pragma unroll
      for (int d = 0; d < 9; ++d) G[d] = a.gam_pt[((size_t)pos * 9 + d) * N3 + q];
    }
    float Mg[9], scale, det;
    geom_map_from<GEO>(src, G, rx, ry, (GEO == kTrilinear) ? a.xi[k] : 0.f, Mg, scale, det);
    float gp[3][3], gu[3][3];
    apply_map(dp, Mg, gp);
    apply_map(du, Mg, gu);
    if (act) {
      const float W = (float)A.wdet[(size_t)pos * N3 + q];
      const size_t g3 = 3 * (size_t)s_g[q];
      float aa[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) aa[c] = A.uscale * A.am[vofs + g3 + c];
      const float divp = gp[0][0] + gp[1][1] + gp[2][2];
      const float divu = gu[0][0] + gu[1][1] + gu[2][2];
      float ee = 0.0f;
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b) ee += 0.25f * (gp[c][b] + gp[b][c]) * (gu[c][b] + gu[b][c]);
      const size_t kq = ((size_t)model * a.nspec + pos) * N3 + q;
      const float ws = A.coef * W * scale;
      A.kl[kq] += (double)(ws * divp * divu) * A.inv_uscale;
      A.km[kq] += (double)(2.0f * ws * ee) * A.inv_uscale;
      A.kr[kq] += (double)(A.coef * W * (pk[0] * aa[0] + pk[1] * aa[1] + pk[2] * aa[2])) * A.inv_uscale;
    }
    const float lw = mat[q], mw = mat[N3 + q];
    const float ltr = lw * (gp[0][0] + gp[1][1] + gp[2][2]);
    float sg[3][3];
    sg[0][0] = ltr + 2.0f * mw * gp[0][0];
    sg[1][1] = ltr + 2.0f * mw * gp[1][1];
    sg[2][2] = ltr + 2.0f * mw * gp[2][2];
    sg[0][1] = sg[1][0] = mw * (gp[0][1] + gp[1][0]);
    sg[0][2] = sg[2][0] = mw * (gp[0][2] + gp[2][0]);
    sg[1][2] = sg[2][1] = mw * (gp[1][2] + gp[2][1]);
    float phi[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d)
        phi[c][d] = scale * (sg[c][0] * Mg[d * 3 + 0] + sg[c][1] * Mg[d * 3 + 1] + sg[c][2] * Mg[d * 3 + 2]);
#pragma unroll
    for (int b = 0; b < NG; ++b) {
      const float dkb = s_D[k * NG + b];
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c][b] += dkb * phi[c][2];
    }
    if (act) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        s_q[(2 * c + 0) * N2 + ll] = phi[c][0];
        s_q[(2 * c + 1) * N2 + ll] = phi[c][1];
      }
    }
    __syncthreads();
    float sxy[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float sacc = 0.0f;
#pragma unroll
      for (int b = 0; b < NG; ++b) {
        sacc += s_D[b * NG + i] * s_q[(2 * c + 0) * N2 + b + NG * j];
        sacc += s_D[b * NG + j] * s_q[(2 * c + 1) * N2 + i + NG * b];
      }
      sxy[c] = sacc;
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
      float* fg = f + 3 * (size_t)s_g[ll + N2 * k];
      if constexpr (ATOMIC) {
        unsafeAtomicAdd(fg + 0, -acc[0][k]);
        unsafeAtomicAdd(fg + 1, -acc[1][k]);
        unsafeAtomicAdd(fg + 2, -acc[2][k]);
      } else {
        fg[0] = fg[0] - acc[0][k];
        fg[1] = fg[1] - acc[1][k];
        fg[2] = fg[2] - acc[2][k];
      }
    }
  }
}

template <int NG>
hipError_t launch_adj_col(int geo, bool atomic, const AdjArgs& A, hipStream_t s) {
  if (A.fa.count <= 0) return hipSuccess;
  const int64_t nb = ((A.fa.count + kNumXcd - 1) / kNumXcd) * kNumXcd;
  dim3 grid((unsigned)nb, (unsigned)A.fa.nmodels), block(AdjCol<NG>::BLK);
#define SEMX_ADJC_LAUNCH(GEO)                                                   \
  if (atomic) adjoint_col_kernel<NG, GEO, true><<<grid, block, 0, s>>>(A);     \
  else adjoint_col_kernel<NG, GEO, false><<<grid, block, 0, s>>>(A);
  switch (geo) {
    case kRegular: SEMX_ADJC_LAUNCH(kRegular) break;
    case kStored: SEMX_ADJC_LAUNCH(kStored) break;
    case kTrilinear: SEMX_ADJC_LAUNCH(kTrilinear) break;
    default: return hipErrorInvalidValue;
  }
#undef SEMX_ADJC_LAUNCH
  return hipGetLastError();
}

hipError_t launch_adjoint_force(int n, int geo, bool atomic, const AdjArgs& A, hipStream_t s) {
  switch (n) {
    case 2: return launch_adj_n<2>(geo, atomic, A, s);
    case 3: return launch_adj_n<3>(geo, atomic, A, s);
    case 4: return launch_adj_n<4>(geo, atomic, A, s);
    case 5: return launch_adj_n<5>(geo, atomic, A, s);
    case 6: return launch_adj_n<6>(geo, atomic, A, s);
    case 7: return launch_adj_n<7>(geo, atomic, A, s);
    case 8: return launch_adj_n<8>(geo, atomic, A, s);
    case 9: return launch_adj_n<9>(geo, atomic, A, s);
    case 10: return launch_adj_n<10>(geo, atomic, A, s);
    case 11: return launch_adj_col<11>(geo, atomic, A, s);
    case 12: return launch_adj_col<12>(geo, atomic, A, s);
    case 13: return launch_adj_col<13>(geo, atomic, A, s);
    case 14: return launch_adj_col<14>(geo, atomic, A, s);
    case 15: return launch_adj_col<15>(geo, atomic, A, s);
    case 16: return launch_adj_col<16>(geo, atomic, A, s);
    default: return hipErrorInvalidValue;
  }
}

// Adjoint source: fb[node] += inv_dt2 * l_q(x_r) * gseis[model][r][c][m]  (R^T g)
__global__ void adj_source_kernel(int nrec, int n3, int64_t nt_max, int64_t m, int nmodels, int64_t nglob,
                                  float inv_dt2, const int32_t* __restrict__ nodes, const float* __restrict__ wts,
                                  const float* __restrict__ gseis, float* __restrict__ fb) {
  const int64_t total = (int64_t)nmodels * nrec * n3;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t rq = t % ((int64_t)nrec * n3);
    const int model = (int)(t / ((int64_t)nrec * n3));
    const int r = (int)(rq / n3);
    const float w = wts[rq] * inv_dt2;
    float* fg = fb + ((int64_t)model * nglob + nodes[rq]) * 3;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float gv = gseis[(((int64_t)model * nrec + r) * 3 + c) * nt_max + m];
      if (gv != 0.0f) unsafeAtomicAdd(fg + c, w * gv);
    }
  }
}

// psi^m = 2 psi^{m+1} - psi^{m+2} + dt^2 M^{-1} fb;  fb = 0
__device__ __forceinline__ float adj_entry(float p1, float p0, float dt2, float m, float f) {
  return 2.0f * p1 - p0 + dt2 * m * f;
}

__global__ void adj_update_kernel(int64_t nnodes, float dt2, const float* __restrict__ minv,
                                  const float* __restrict__ p1, const float* __restrict__ p0,
                                  float* __restrict__ p2, float* __restrict__ fb) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < 3 * nnodes;
       t += (int64_t)gridDim.x * blockDim.x) {
    p2[t] = adj_entry(p1[t], p0[t], dt2, minv[t / 3], fb[t]);
    fb[t] = 0.0f;
  }
}

// The same with four consecutive entries per lane (16-byte accesses; every
// array 16-byte aligned).  The last (3 nnodes) % 4 entries go to the first
// lanes.
typedef float adj_f4 __attribute__((ext_vector_type(4)));
__global__ void adj_update4_kernel(int64_t nnodes, float dt2, const float* __restrict__ minv,
                                   const float* __restrict__ p1, const float* __restrict__ p0,
                                   float* __restrict__ p2, float* __restrict__ fb) {
  const int64_t len = 3 * nnodes, len4 = len / 4;
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int64_t q = gid; q < len4; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t0 = 4 * q;
    const adj_f4 a = *reinterpret_cast<const adj_f4*>(p1 + t0);
    const adj_f4 b = *reinterpret_cast<const adj_f4*>(p0 + t0);
    const adj_f4 f = *reinterpret_cast<const adj_f4*>(fb + t0);
    adj_f4 r;
#pragma unroll
    for (int e = 0; e < 4; ++e) r[e] = adj_entry(a[e], b[e], dt2, minv[(t0 + e) / 3], f[e]);
    *reinterpret_cast<adj_f4*>(p2 + t0) = r;
    *reinterpret_cast<adj_f4*>(fb + t0) = (adj_f4){0.0f, 0.0f, 0.0f, 0.0f};
  }
  const int64_t t = 4 * len4 + gid;
  if (t < len) {
    p2[t] = adj_entry(p1[t], p0[t], dt2, minv[t / 3], fb[t]);
    fb[t] = 0.0f;
  }
}

// kr += -W psi^1 . (uscale u^1) at every element-local point (start-up term)
__global__ void adj_rho_start_kernel(int n3, int64_t nspec, int nmodels, int64_t nglob,
                                     const int32_t* __restrict__ ibool, const double* __restrict__ wdet,
                                     const float* __restrict__ psi1, const float* __restrict__ u1, float uscale,
                                     double inv_uscale, double* __restrict__ kr) {
  const int64_t total = (int64_t)nmodels * nspec * n3;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pt = t % (nspec * n3);
    const int model = (int)(t / (nspec * n3));
    const int64_t g = ((int64_t)model * nglob + ibool[pt]) * 3;
    const float v = -(float)wdet[pt] * (psi1[g] * (uscale * u1[g]) + psi1[g + 1] * (uscale * u1[g + 1]) +
                                        psi1[g + 2] * (uscale * u1[g + 2]));
    kr[t] += (double)v * inv_uscale;
  }
}

// max |x| into *out (bit pattern of a non-negative float orders like an int)
__global__ void maxabs_kernel(int64_t n, const float* __restrict__ x, unsigned int* __restrict__ out) {
  float mx = 0.0f;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    mx = fmaxf(mx, fabsf(x[t]));
  if (mx > 0.0f) atomicMax(out, __float_as_uint(mx));
}

// out[model][order[pos]][q] = scale * acc[model][pos][q]   (FP64 output: the
// physical gradients may lie below the FP32 range)
__global__ void unpermute_kernel(int n3, int64_t nspec, int nmodels, const int32_t* __restrict__ order,
                                 const double* __restrict__ acc, double scale, double* __restrict__ out) {
  const int64_t total = (int64_t)nmodels * nspec * n3;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t mp = t / n3;
    const int q = (int)(t - mp * n3);
    const int64_t model = mp / nspec, pos = mp - model * nspec;
    out[(model * nspec + order[pos]) * n3 + q] = scale * acc[t];
  }
}

int64_t state_len(const semx_ctx* c) { return (int64_t)c->nmodels * c->nglob * 3; }

int d2d(semx_ctx* c, void* dst, const void* src, size_t bytes) {
  SEMX_HIP(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream));
  return SEMX_OK;
}

// Largest |x| over n floats (device), via a one-word device buffer.
int max_abs(semx_ctx* c, const float* x, int64_t n, unsigned int* dword, float* out) {
  SEMX_HIP(c, hipMemsetAsync(dword, 0, sizeof(unsigned int), c->stream));
  maxabs_kernel<<<grid_1d(n, 4096), 256, 0, c->stream>>>(n, x, dword);
  SEMX_HIP(c, hipGetLastError());
  unsigned int h = 0;
  SEMX_HIP(c, hipMemcpyAsync(&h, dword, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  SEMX_HIP(c, hipStreamSynchronize(c->stream));
  std::memcpy(out, &h, sizeof(float));
  return SEMX_OK;
}

// power of two p with p * x in [1, 2) (1 for x = 0)
float pow2_normaliser(float x) {
  if (!(x > 0.0f) || !std::isfinite(x)) return 1.0f;
  return std::ldexp(1.0f, -std::ilogb(x));
}

}  // namespace

int save_checkpoint(semx_ctx* c) {
  if (c->ckpt_every <= 0 || c->it % c->ckpt_every != 0) return SEMX_OK;
  const int64_t k = c->it / c->ckpt_every;
  int rc = complete_step(c);
  if (rc) return rc;
  const int64_t len = state_len(c);
  const size_t vb = sizeof(float) * len;
  if ((int64_t)c->ckpts.size() <= k) {
    c->ckpts.resize(k + 1);
    c->ckpt_gen.resize(k + 1, -1);
  }
  if (c->ckpts[k].bytes != 3 * vb) {
    rc = dev_alloc(c, c->ckpts[k], 3 * vb);
    if (rc) return rc;
  }
  char* base = c->ckpts[k].as<char>();
  rc = d2d(c, base, c->d_u.p, vb);
  if (!rc) rc = d2d(c, base + vb, c->d_v.p, vb);
  if (!rc) rc = d2d(c, base + 2 * vb, c->d_a.p, vb);
  if (rc) return rc;
  c->ckpt_gen[k] = c->run_gen;
  c->ckpt_count = k + 1;
  return SEMX_OK;
}

}  // namespace semx

using namespace semx;

extern "C" {

int semx_set_checkpointing(semx_ctx* c, int64_t every) {
  if (!c) return SEMX_EINVAL;
  if (every < 0) return fail(c, SEMX_EINVAL, "set_checkpointing: negative interval");
  if (every > 0 && c->storage != SEMX_F32) return fail(c, SEMX_ESTATE, "set_checkpointing: the adjoint needs FP32 storage");
  if (every > 0 && c->physics != SEMX_ELASTIC)
    return fail(c, SEMX_EINVAL, "set_checkpointing: the adjoint covers the elastic operator only");
  c->ckpt_every = every;
  c->ckpt_count = 0;
  std::fill(c->ckpt_gen.begin(), c->ckpt_gen.end(), -1);
  if (every == 0) {
    for (DevBuf& b : c->ckpts) dev_free(b);
    c->ckpts.clear();
    c->ckpt_gen.clear();
  }
  return SEMX_OK;
}

int semx_adjoint(semx_ctx* c, const float* gseis_dev, int64_t nt, double* g_lambda_dev, double* g_mu_dev,
                 double* g_rho_dev) {
  if (!c) return SEMX_EINVAL;
  c->err.clear();
  if (!c->have_mesh || !c->have_model || !c->have_dt) return fail(c, SEMX_ESTATE, "adjoint: mesh, model and dt required");
  if (c->storage != SEMX_F32) return fail(c, SEMX_ESTATE, "adjoint: needs FP32 storage");
  if (c->physics != SEMX_ELASTIC) return fail(c, SEMX_EINVAL, "adjoint: the elastic operator only");
  if (!gseis_dev || !g_lambda_dev || !g_mu_dev || !g_rho_dev) return fail(c, SEMX_EINVAL, "adjoint: null pointer");
  if (c->rec.nrec == 0) return fail(c, SEMX_ESTATE, "adjoint: no receivers");
  if (c->ckpt_every <= 0 || c->ckpt_count == 0)
    return fail(c, SEMX_ESTATE, "adjoint: enable checkpointing before the forward run (semx_set_checkpointing + semx_reset)");
  if (nt < 1 || nt > c->it || nt > c->rec.nt_max)
    return fail(c, SEMX_EINVAL, "adjoint: nt must lie in [1, min(steps taken, nt_max)]");
  const int64_t K = c->ckpt_every;
  const int64_t nseg = (nt + K - 1) / K;
  if (c->ckpt_count < nseg) return fail(c, SEMX_ESTATE, "adjoint: missing forward checkpoints");
  const int64_t len = state_len(c);
  const size_t vb = sizeof(float) * len;
  // every checkpoint the backward pass restores must come from this run (the
  // same model, sources, batch size and start) and hold the current state size
  for (int64_t seg = 0; seg < nseg; ++seg)
    if (seg >= (int64_t)c->ckpts.size() || c->ckpts[seg].bytes != 3 * vb || c->ckpt_gen[seg] != c->run_gen)
      return fail(c, SEMX_ESTATE, "adjoint: forward checkpoint " + std::to_string(seg) +
                                      " is not from the current run (reset and step again after changing the "
                                      "model, sources or state)");
  const int64_t npt = (int64_t)c->nmodels * c->nspec * c->n3;
  const int64_t nn = (int64_t)c->nmodels * c->nglob;
  // slots of the segment and psi buffers start on 16-byte boundaries (the
  // update kernels' four-entry form); the padding stays zero
  const int64_t lenp = (len + 3) / 4 * 4;
  const size_t vbp = sizeof(float) * lenp;

  // buffers
  DevBuf saved, segu, sega, psi, fb, acc;
  auto cleanup = [&]() {
    for (DevBuf* b : {&saved, &segu, &sega, &psi, &fb, &acc}) dev_free(*b);
  };
  int rc = dev_alloc(c, saved, 4 * vb);
  if (!rc) rc = dev_alloc(c, segu, (K + 1) * vbp);
  if (!rc) rc = dev_alloc(c, sega, (K + 1) * vbp);
  if (!rc) rc = dev_alloc(c, psi, 3 * vbp);
  if (!rc) rc = dev_alloc(c, fb, vb);
  if (!rc) rc = dev_alloc(c, acc, 3 * sizeof(double) * npt);
  if (rc) { cleanup(); return rc; }
  // keep the caller's forward state
  const int64_t it_saved = c->it;
  const bool pend_saved = c->pending_correct;
  char* sv = saved.as<char>();
  rc = d2d(c, sv, c->d_u.p, vb);
  if (!rc) rc = d2d(c, sv + vb, c->d_v.p, vb);
  if (!rc) rc = d2d(c, sv + 2 * vb, c->d_a.p, vb);
  if (!rc) rc = d2d(c, sv + 3 * vb, c->d_f.p, vb);
  float* p[3] = {psi.as<float>(), psi.as<float>() + lenp, psi.as<float>() + 2 * lenp};
  double* kl = acc.as<double>();
  double* km = kl + npt;
  double* kr = km + npt;
  if (!rc) rc = fill_zero(c, psi.as<float>(), 3 * lenp);
  if (!rc) rc = fill_zero(c, segu.as<float>(), (K + 1) * lenp);
  if (!rc) rc = fill_zero(c, fb.as<float>(), len);
  if (!rc) rc = fill_zero(c, acc.as<float>(), 6 * npt);  // 3 * npt doubles of zero bits
  if (rc) { cleanup(); return rc; }
  // FP32 range: the adjoint is linear in gseis and the sensitivities bilinear
  // in (psi, u), so gseis is normalised once and the forward field of each
  // segment by its own power of two (exact); contributions are rescaled into
  // FP64 accumulators and the result is scaled back at the end.
  unsigned int* dword = reinterpret_cast<unsigned int*>(fb.as<float>());
  float gmax = 0.0f;
  rc = max_abs(c, gseis_dev, (int64_t)c->nmodels * c->rec.nrec * 3 * c->rec.nt_max, dword, &gmax);
  if (!rc) rc = fill_zero(c, fb.as<float>(), len);
  if (rc) { cleanup(); return rc; }
  const float sg = pow2_normaliser(gmax);
  float su = 1.0f;

  AdjArgs A{};
  A.fa.ibool = c->d_ibool.as<int32_t>();
  A.fa.gam_pt = c->d_gam_pt.as<float>();
  A.fa.gam_el = c->d_gam_el.as<float>();
  A.fa.tri = c->d_tri.as<float>();
  A.fa.xi = c->d_xi32.as<float>();
  A.fa.mat = c->d_mat.as<float>();
  A.fa.f = fb.as<float>();
  A.fa.D = c->d_D.as<float>();
  A.fa.nspec = c->nspec;
  A.fa.nglob = c->nglob;
  A.fa.nmodels = c->nmodels;
  A.wdet = c->d_wdet.as<double>();
  A.kl = kl;
  A.km = km;
  A.kr = kr;
  const float dt = (float)c->dt;
  A.coef = -dt * dt;
  const bool atomic = c->ncolors == 0;
  const auto& launches = atomic ? c->atomic_launches : c->colored_launches;
  int i0 = 0, i1 = 1, i2 = 2;  // p[i0] = psi^{m+2}, p[i1] = psi^{m+1}, p[i2] = psi^m

  for (int64_t seg = nseg - 1; seg >= 0 && !rc; --seg) {
    const int64_t n0 = seg * K, n1 = std::min(n0 + K, nt);
    // restore checkpoint seg and recompute u^n, a^n for n in [n0, n1]
    const char* ck = c->ckpts[seg].as<char>();
    rc = d2d(c, c->d_u.p, ck, vb);
    if (!rc) rc = d2d(c, c->d_v.p, ck + vb, vb);
    if (!rc) rc = d2d(c, c->d_a.p, ck + 2 * vb, vb);
    if (!rc) rc = fill_zero(c, c->d_f.as<float>(), len);
    c->it = n0;
    c->pending_correct = false;
    if (!rc) rc = d2d(c, segu.as<char>(), c->d_u.p, vb);
    if (!rc) rc = d2d(c, sega.as<char>(), c->d_a.p, vb);
    // the forward run's own fused Newmark pass stores u^s and a^{s-1} into the
    // segment buffers (bitwise the forward states); the last a after the loop
    float* su0 = segu.as<float>();
    float* sa0 = sega.as<float>();
    for (int64_t s = 1; s <= n1 - n0 && !rc; ++s)
      rc = step_once(c, false, su0 + s * lenp, s >= 2 ? sa0 + (s - 1) * lenp : nullptr);
    if (!rc) rc = complete_step(c, sa0 + (n1 - n0) * lenp);
    // normaliser of this segment's forward field
    if (!rc) {
      float umax = 0.0f;
      rc = max_abs(c, segu.as<float>(), (n1 - n0 + 1) * lenp, dword, &umax);
      if (!rc) rc = fill_zero(c, fb.as<float>(), len);
      su = pow2_normaliser(umax);
      A.uscale = su;
      A.inv_uscale = 1.0 / (double)su;
    }
    // backward over m = n1 .. n0+1
    for (int64_t m = n1; m >= n0 + 1 && !rc; --m) {
      if (m <= nt - 1) {
        A.fa.u = p[i1];
        A.um = segu.as<float>() + (m - n0) * lenp;
        A.am = sega.as<float>() + (m - n0) * lenp;
        for (const auto& L : launches) {
          A.fa.pos0 = L.pos0;
          A.fa.count = L.count;
          const int geo = L.irregular ? c->irregular_geo : kRegular;
          hipError_t e = launch_adjoint_force(c->n, geo, atomic, A, c->stream);
          if (e != hipSuccess) { rc = hip_fail(c, e, "adjoint force kernel"); break; }
        }
        if (rc) break;
      }
      const int64_t total = (int64_t)c->nmodels * c->rec.nrec * c->n3;
      adj_source_kernel<<<grid_1d(total), 256, 0, c->stream>>>(
          c->rec.nrec, c->n3, c->rec.nt_max, m - 1, c->nmodels, c->nglob, sg / (dt * dt),
          c->rec.nodes.as<int32_t>(), c->rec.wts.as<float>(), gseis_dev, fb.as<float>());
      adj_update4_kernel<<<grid_1d((3 * nn + 3) / 4), 256, 0, c->stream>>>(nn, dt * dt, c->d_minv.as<float>(),
                                                                           p[i1], p[i0], p[i2], fb.as<float>());
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) { rc = hip_fail(c, e, "adjoint update"); break; }
      const int t = i0;
      i0 = i1;
      i1 = i2;
      i2 = t;
    }
  }
  if (!rc) {
    // start-up term with psi^1 (p[i1]) and u^1 (segment 0, slot 1)
    adj_rho_start_kernel<<<grid_1d(npt), 256, 0, c->stream>>>(c->n3, c->nspec, c->nmodels, c->nglob,
                                                              c->d_ibool.as<int32_t>(), c->d_wdet.as<double>(),
                                                              p[i1], segu.as<float>() + lenp, su, 1.0 / (double)su, kr);
    unpermute_kernel<<<grid_1d(npt), 256, 0, c->stream>>>(c->n3, c->nspec, c->nmodels, c->d_order.as<int32_t>(), kl,
                                                          1.0 / (double)sg, g_lambda_dev);
    unpermute_kernel<<<grid_1d(npt), 256, 0, c->stream>>>(c->n3, c->nspec, c->nmodels, c->d_order.as<int32_t>(), km,
                                                          1.0 / (double)sg, g_mu_dev);
    unpermute_kernel<<<grid_1d(npt), 256, 0, c->stream>>>(c->n3, c->nspec, c->nmodels, c->d_order.as<int32_t>(), kr,
                                                          1.0 / (double)sg, g_rho_dev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) rc = hip_fail(c, e, "adjoint finish");
  }
  // restore the caller's state
  int rc2 = d2d(c, c->d_u.p, sv, vb);
  if (!rc2) rc2 = d2d(c, c->d_v.p, sv + vb, vb);
  if (!rc2) rc2 = d2d(c, c->d_a.p, sv + 2 * vb, vb);
  if (!rc2) rc2 = d2d(c, c->d_f.p, sv + 3 * vb, vb);
  c->it = it_saved;
  c->pending_correct = pend_saved;
  if (!rc && !rc2) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) rc = hip_fail(c, e, "adjoint sync");
  }
  cleanup();
  return rc ? rc : rc2;
}

}  // extern "C"
