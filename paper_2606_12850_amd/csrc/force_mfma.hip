// Mixed-precision force kernel: the six small contractions of the operator
// (three forward, three transpose; Sec. II-B) run on gfx950 matrix cores as
// v_mfma_f32_16x16x32_{bf16,f16} with FP32 accumulation; the geometry map,
// stress and assembly stay FP32.
//
// MFMA mapping.  For direction d the contraction of component c along the
// element's "lines" (the n^2 index pairs orthogonal to d) is
//   C[line][(c,i)] = sum_{(c',a)} A[line][(c',a)] B[(c',a)][(c,i)],
//   A[line][(c,a)] = field_c(a along d, line),
//   B = block-diagonal copies of D^T (forward) or D (transpose),
// with G = min(3, 16/n) components packed along K and N (K uses 16 of the 32
// slots of the 16x16x32 tile).  Lines fill the M dimension in tiles of 16.
// This is the matrix-core counterpart of the paper's packing of several
// small products into one outer-product tile (Sec. IV-A); the useful fraction
// of each MFMA is (G n / 32)(G n / 16)(1/G) of its multiply-adds.
//
// Precision treatment (low-precision operands only):
//   * the forward operand is u - u(local node 0) per component, so a rigid
//     translation gives exactly zero derivatives (D 1 = 0 no longer holds
//     after rounding D);
//   * operands are scaled per element by a power of two so that the largest
//     magnitude is in [0.5, 1) (FP16 range); results are unscaled in FP32.
#include "elem_common.hpp"

namespace semx {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int P>
struct Op;
template <>
struct Op<SEMX_C_BF16> {
  using vec = bf16x8;
  using elt = __bf16;
  __device__ static f32x4 mma(vec a, vec b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};
template <>
struct Op<SEMX_C_F16> {
  using vec = f16x8;
  using elt = _Float16;
  __device__ static f32x4 mma(vec a, vec b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};

// element-local point of (index a along direction dir, line)
template <int NG>
__device__ __forceinline__ int line_point(int dir, int a, int line) {
  if (dir == 0) return a + NG * line;                      // line = j + NG k
  if (dir == 1) return (line % NG) + NG * (a + NG * (line / NG));  // line = i + NG k
  return line + NG * NG * a;                               // line = i + NG j
}

// Block-wide maximum (all lanes of the block call it; uses s_red[16]).
__device__ __forceinline__ float block_max(float v, float* s_red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) s_red[w] = v;
  __syncthreads();
  float m = 0.0f;
  for (int t = 0; t < (int)(blockDim.x / 64); ++t) m = fmaxf(m, s_red[t]);
  __syncthreads();
  return m;
}

// power of two p with p * x in [0.5, 1) (1 for x = 0)
__device__ __forceinline__ float pow2_scale(float x) {
  if (!(x > 0.0f)) return 1.0f;
  int e;
  frexpf(x, &e);  // x = f 2^e, f in [0.5, 1)
  return ldexpf(1.0f, -e);
}

template <int NG, int GEO, bool ATOMIC, int PREC>
__global__ __launch_bounds__(Shape<NG>::BLK) void force_mfma_kernel(ForceArgs a) {
  using O = Op<PREC>;
  using vec = typename O::vec;
  using elt = typename O::elt;
  constexpr int N3 = Shape<NG>::N3;
  constexpr int NW = Shape<NG>::BLK / 64;          // waves per block
  constexpr int G = (3 < 16 / NG) ? 3 : 16 / NG;   // components per MFMA
  constexpr int NGRP = (3 + G - 1) / G;            // component groups
  constexpr int NL = NG * NG;                       // lines per direction
  constexpr int NT = (NL + 15) / 16;                // M tiles
  constexpr int NJOB = 3 * NGRP * NT;               // MFMAs per contraction pass
  __shared__ float s_u[3 * N3];
  __shared__ float s_d[9 * N3];  // derivatives, then transpose partial sums
  __shared__ float s_q[9 * N3];
  __shared__ float s_D[NG * NG];
  __shared__ float s_red[16];

  const int grp = xcd_group((int)a.count);
  if (grp >= a.count) return;
  const int pos = (int)a.pos0 + grp;
  const int p = threadIdx.x;
  const bool act = p < N3;
  const int pp = act ? p : 0;
  const int i = pp % NG, j = (pp / NG) % NG, k = pp / (NG * NG);
  const int lane = p & 63, wave = p >> 6;
  const int model = blockIdx.y;
  const float* __restrict__ u = a.u + (size_t)model * a.nglob * 3;
  float* f = a.f + (size_t)model * a.nglob * 3;
  const float* __restrict__ mat = a.mat + (size_t)model * a.nspec * 2 * N3;

  const int g = ldnt(a.ibool + (size_t)pos * N3 + pp);
  float G9[9];
  if constexpr (GEO == kStored) {
#pragma unroll
    for (int d = 0; d < 9; ++d) G9[d] = ldnt(a.gam_pt + ((size_t)pos * 9 + d) * N3 + pp);
  }
  const float lw = ldnt(mat + (size_t)pos * 2 * N3 + pp), mw = ldnt(mat + (size_t)pos * 2 * N3 + N3 + pp);
  float uu[3], f0[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    uu[c] = u[3 * (size_t)g + c];
    if constexpr (!ATOMIC) f0[c] = f[3 * (size_t)g + c];
  }
  if (p < NG * NG) s_D[p] = a.D[p];
  if (act)
#pragma unroll
    for (int c = 0; c < 3; ++c) s_u[c * N3 + pp] = uu[c];
  float rx = 0.f, ry = 0.f, rz = 0.f;
  if constexpr (GEO == kTrilinear) {
    rx = a.xi[i];
    ry = a.xi[j];
    rz = a.xi[k];
  }
  __syncthreads();

  // per-lane B operands: block-diagonal D^T (forward) and D (transpose)
  const int col = lane & 15, kg = lane >> 4;
  vec Bf, Bt;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int kk = 8 * kg + t;
    float vf = 0.0f, vt = 0.0f;
    if (kk < G * NG && col < G * NG && kk / NG == col / NG) {
      const int aa = kk % NG, ii = col % NG;
      vf = s_D[ii * NG + aa];  // D[i][a]
      vt = s_D[aa * NG + ii];  // D[a][i]
    }
    Bf[t] = (elt)vf;
    Bt[t] = (elt)vt;
  }

  // forward operand: u - u(node 0), scaled per element
  float ub[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) ub[c] = s_u[c * N3];
  float um = 0.0f;
  if (act)
#pragma unroll
    for (int c = 0; c < 3; ++c) um = fmaxf(um, fabsf(uu[c] - ub[c]));
  const float su = pow2_scale(block_max(um, s_red));
  const float isu = 1.0f / su;

  for (int job = wave; job < NJOB; job += NW) {
    const int dir = job / (NGRP * NT);
    const int cg = (job / NT) % NGRP;
    const int tile = job % NT;
    vec A;
    const int line = tile * 16 + (lane & 15);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int kk = 8 * kg + t;
      const int c = cg * G + kk / NG;
      float v = 0.0f;
      if (kk < G * NG && c < 3 && line < NL) v = (s_u[c * N3 + line_point<NG>(dir, kk % NG, line)] - ub[c]) * su;
      A[t] = (elt)v;
    }
    f32x4 C = {0.f, 0.f, 0.f, 0.f};
    C = O::mma(A, Bf, C);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int ln = tile * 16 + 4 * kg + t;
      const int c = cg * G + col / NG;
      if (col < G * NG && c < 3 && ln < NL) s_d[(c * 3 + dir) * N3 + line_point<NG>(dir, col % NG, ln)] = C[t] * isu;
    }
  }
  __syncthreads();

  // pointwise: geometry map, stress, fluxes (FP32)
  float du[3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = 0; d < 3; ++d) du[c][d] = s_d[(c * 3 + d) * N3 + pp];
  float Mg[9], scale, det;
  geom_map<GEO>(a, pos, G9, rx, ry, rz, Mg, scale, det);
  float gr[3][3];
  apply_map(du, Mg, gr);
  stress_flux(gr, lw, mw, scale, Mg, s_q, N3, pp, act);
  float qm = 0.0f;
  if (act)
#pragma unroll
    for (int t = 0; t < 9; ++t) qm = fmaxf(qm, fabsf(s_q[t * N3 + pp]));
  const float sq = pow2_scale(block_max(qm, s_red));  // block_max synchronises: s_q complete
  const float isq = 1.0f / sq;

  for (int job = wave; job < NJOB; job += NW) {
    const int dir = job / (NGRP * NT);
    const int cg = (job / NT) % NGRP;
    const int tile = job % NT;
    vec A;
    const int line = tile * 16 + (lane & 15);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int kk = 8 * kg + t;
      const int c = cg * G + kk / NG;
      float v = 0.0f;
      if (kk < G * NG && c < 3 && line < NL) v = s_q[(c * 3 + dir) * N3 + line_point<NG>(dir, kk % NG, line)] * sq;
      A[t] = (elt)v;
    }
    f32x4 C = {0.f, 0.f, 0.f, 0.f};
    C = O::mma(A, Bt, C);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int ln = tile * 16 + 4 * kg + t;
      const int c = cg * G + col / NG;
      if (col < G * NG && c < 3 && ln < NL) s_d[(dir * 3 + c) * N3 + line_point<NG>(dir, col % NG, ln)] = C[t] * isq;
    }
  }
  __syncthreads();

  if (act) {
    float F[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) F[c] = -(s_d[(0 * 3 + c) * N3 + pp] + s_d[(1 * 3 + c) * N3 + pp] + s_d[(2 * 3 + c) * N3 + pp]);
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

template <int NG, int PREC>
hipError_t launch_mfma_n(int geo, bool atomic, const ForceArgs& a, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  const int64_t nb = ((a.count + kNumXcd - 1) / kNumXcd) * kNumXcd;
  dim3 grid((unsigned)nb, (unsigned)a.nmodels), block(Shape<NG>::BLK);
#define SEMX_MFMA_LAUNCH(GEO)                                                            \
  if (atomic) force_mfma_kernel<NG, GEO, true, PREC><<<grid, block, 0, s>>>(a);          \
  else force_mfma_kernel<NG, GEO, false, PREC><<<grid, block, 0, s>>>(a);
  switch (geo) {
    case kRegular: SEMX_MFMA_LAUNCH(kRegular) break;
    case kStored: SEMX_MFMA_LAUNCH(kStored) break;
    case kTrilinear: SEMX_MFMA_LAUNCH(kTrilinear) break;
    default: return hipErrorInvalidValue;
  }
#undef SEMX_MFMA_LAUNCH
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_mfma_p(int n, int geo, bool atomic, const ForceArgs& a, hipStream_t s) {
  switch (n) {
    case 4: return launch_mfma_n<4, PREC>(geo, atomic, a, s);
    case 5: return launch_mfma_n<5, PREC>(geo, atomic, a, s);
    case 6: return launch_mfma_n<6, PREC>(geo, atomic, a, s);
    case 7: return launch_mfma_n<7, PREC>(geo, atomic, a, s);
    case 8: return launch_mfma_n<8, PREC>(geo, atomic, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool mfma_supported(int n) { return n >= 4 && n <= 8; }

hipError_t launch_force_mfma(int n, int prec, int geo, bool atomic, const ForceArgs& a, hipStream_t s) {
  if (prec == SEMX_C_BF16) return launch_mfma_p<SEMX_C_BF16>(n, geo, atomic, a, s);
  if (prec == SEMX_C_F16) return launch_mfma_p<SEMX_C_F16>(n, geo, atomic, a, s);
  return hipErrorInvalidValue;
}

}  // namespace semx
