// FP32 element internal-force kernel f = -K u (VALU contractions through LDS).
//
// One workgroup owns one element at a time (one lane per GLL point, the
// n^3 points padded to whole 64-lane wavefronts) and walks a contiguous slice
// of the launch's element list.  Per element, in one fused traversal
// (the paper's Sec. IV-D "single grid-point traversal" with scalar
// intermediates):
//   gather u[ibool] -> LDS,
//   three forward contractions with D along xi/eta/zeta (Sec. II-B),
//   inverse-Jacobian map, isotropic stress, weighted fluxes in registers,
//   fluxes -> LDS, three transpose contractions with D^T (Sec. II-B, weak form),
//   scatter-add to f (plain read-modify-write inside a colour, or atomics).
// The per-lane rows and columns of D stay in registers for the whole kernel.
#include "semx_internal.hpp"

namespace semx {
namespace {

template <int NG>
struct Shape {
  static constexpr int N3 = NG * NG * NG;
  static constexpr int BLK = ((N3 + 63) / 64) * 64;
};

template <int NG, bool IRREG, bool ATOMIC>
__global__ __launch_bounds__(Shape<NG>::BLK) void force_f32_kernel(ForceArgs a) {
  constexpr int N3 = Shape<NG>::N3;
  __shared__ float s_u[3 * N3];
  __shared__ float s_q[9 * N3];

  const int p = threadIdx.x;
  const bool act = p < N3;
  const int pp = act ? p : 0;
  const int i = pp % NG, j = (pp / NG) % NG, k = pp / (NG * NG);

  // D rows (forward) and columns (transpose) needed by this lane.
  float Di[NG], Dj[NG], Dk[NG], Ti[NG], Tj[NG], Tk[NG];
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    Di[q] = a.D[i * NG + q];
    Dj[q] = a.D[j * NG + q];
    Dk[q] = a.D[k * NG + q];
    Ti[q] = a.D[q * NG + i];
    Tj[q] = a.D[q * NG + j];
    Tk[q] = a.D[q * NG + k];
  }

  const int model = blockIdx.y;
  const float* __restrict__ u = a.u + (size_t)model * a.nglob * 3;
  float* __restrict__ f = a.f + (size_t)model * a.nglob * 3;
  const float* __restrict__ mat = a.mat + (size_t)model * a.nspec * 2 * N3;

  // XCD-aware slicing: blocks are dispatched round-robin over the XCDs, so
  // block b runs on XCD b % 8; each XCD walks one contiguous eighth of the
  // list, keeping elements that share nodes within one L2.
  const int bpx = gridDim.x / kNumXcd;
  const int xcd = blockIdx.x % kNumXcd;
  const int lb = blockIdx.x / kNumXcd;
  const int64_t chunk = (a.count + kNumXcd - 1) / kNumXcd;
  const int64_t beg = xcd * chunk;
  const int64_t end = (beg + chunk < a.count) ? beg + chunk : a.count;

  for (int64_t pos = beg + lb; pos < end; pos += bpx) {
    const int e = a.elems[pos];
    const size_t eb = (size_t)e * N3;
    const int g = a.ibool[eb + pp];
    float G[9];
    if constexpr (IRREG) {
      const float* gp = a.gam_pt + (size_t)e * 9 * N3 + pp;
#pragma unroll
      for (int d = 0; d < 9; ++d) G[d] = gp[d * N3];
    } else {
#pragma unroll
      for (int d = 0; d < 9; ++d) G[d] = a.gam_el[(size_t)e * 9 + d];
    }
    const float lamw = mat[(size_t)e * 2 * N3 + pp];
    const float muw = mat[(size_t)e * 2 * N3 + N3 + pp];
    const float ux = u[3 * (size_t)g + 0];
    const float uy = u[3 * (size_t)g + 1];
    const float uz = u[3 * (size_t)g + 2];
    if (act) {
      s_u[pp] = ux;
      s_u[N3 + pp] = uy;
      s_u[2 * N3 + pp] = uz;
    }
    __syncthreads();

    // reference derivatives du[c][d] = d u_c / d xi_d
    float du[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) du[c][0] = du[c][1] = du[c][2] = 0.0f;
#pragma unroll
    for (int q = 0; q < NG; ++q) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        du[c][0] += Di[q] * s_u[c * N3 + q + NG * (j + NG * k)];
        du[c][1] += Dj[q] * s_u[c * N3 + i + NG * (q + NG * k)];
        du[c][2] += Dk[q] * s_u[c * N3 + i + NG * (j + NG * q)];
      }
    }
    // physical gradient gr[c][b] = sum_d du[c][d] Gamma[d][b]
    float gr[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int b = 0; b < 3; ++b)
        gr[c][b] = du[c][0] * G[0 * 3 + b] + du[c][1] * G[1 * 3 + b] + du[c][2] * G[2 * 3 + b];
    // isotropic stress (already weighted by w_i w_j w_k det J)
    const float ltr = lamw * (gr[0][0] + gr[1][1] + gr[2][2]);
    float sg[3][3];
    sg[0][0] = ltr + 2.0f * muw * gr[0][0];
    sg[1][1] = ltr + 2.0f * muw * gr[1][1];
    sg[2][2] = ltr + 2.0f * muw * gr[2][2];
    sg[0][1] = sg[1][0] = muw * (gr[0][1] + gr[1][0]);
    sg[0][2] = sg[2][0] = muw * (gr[0][2] + gr[2][0]);
    sg[1][2] = sg[2][1] = muw * (gr[1][2] + gr[2][1]);
    // fluxes Phi[c][d] = sum_b sigma[c][b] Gamma[d][b]
    if (act) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d)
          s_q[(c * 3 + d) * N3 + pp] =
              sg[c][0] * G[d * 3 + 0] + sg[c][1] * G[d * 3 + 1] + sg[c][2] * G[d * 3 + 2];
    }
    __syncthreads();

    float F[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float s = 0.0f;
#pragma unroll
      for (int q = 0; q < NG; ++q) {
        s += Ti[q] * s_q[(c * 3 + 0) * N3 + q + NG * (j + NG * k)];
        s += Tj[q] * s_q[(c * 3 + 1) * N3 + i + NG * (q + NG * k)];
        s += Tk[q] * s_q[(c * 3 + 2) * N3 + i + NG * (j + NG * q)];
      }
      F[c] = -s;
    }
    if (act) {
      float* fg = f + 3 * (size_t)g;
      if constexpr (ATOMIC) {
        unsafeAtomicAdd(fg + 0, F[0]);
        unsafeAtomicAdd(fg + 1, F[1]);
        unsafeAtomicAdd(fg + 2, F[2]);
      } else {
        fg[0] += F[0];
        fg[1] += F[1];
        fg[2] += F[2];
      }
    }
  }
}

template <int NG>
hipError_t launch_n(bool irregular, bool atomic, const ForceArgs& a, int grid_cap, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  int64_t nb = a.count < grid_cap ? a.count : grid_cap;
  nb = ((nb + kNumXcd - 1) / kNumXcd) * kNumXcd;
  dim3 grid((unsigned)nb, (unsigned)a.nmodels), block(Shape<NG>::BLK);
  if (irregular) {
    if (atomic) force_f32_kernel<NG, true, true><<<grid, block, 0, s>>>(a);
    else force_f32_kernel<NG, true, false><<<grid, block, 0, s>>>(a);
  } else {
    if (atomic) force_f32_kernel<NG, false, true><<<grid, block, 0, s>>>(a);
    else force_f32_kernel<NG, false, false><<<grid, block, 0, s>>>(a);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_force_f32(int n, bool irregular, bool atomic, const ForceArgs& a, int grid_cap,
                            hipStream_t s) {
  switch (n) {
    case 2: return launch_n<2>(irregular, atomic, a, grid_cap, s);
    case 3: return launch_n<3>(irregular, atomic, a, grid_cap, s);
    case 4: return launch_n<4>(irregular, atomic, a, grid_cap, s);
    case 5: return launch_n<5>(irregular, atomic, a, grid_cap, s);
    case 6: return launch_n<6>(irregular, atomic, a, grid_cap, s);
    case 7: return launch_n<7>(irregular, atomic, a, grid_cap, s);
    case 8: return launch_n<8>(irregular, atomic, a, grid_cap, s);
    case 9: return launch_n<9>(irregular, atomic, a, grid_cap, s);
    case 10: return launch_n<10>(irregular, atomic, a, grid_cap, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace semx
