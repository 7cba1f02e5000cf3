// Matrix-core force kernel: the six small contractions of the operator
// (three forward, three transpose; Sec. II-B) run on gfx950 matrix cores as
// v_mfma_f32_16x16x32_{bf16,f16} (mixed precision) or v_mfma_f32_16x16x4f32
// (FP32 operands, n instructions of K = 4 per tile) with FP32 accumulation;
// the geometry map, stress and assembly stay FP32.
//
// MFMA mapping.  For direction d the contraction of component c along the
// element's "lines" (the n^2 index pairs orthogonal to d) is
//   C[line][(c,i)] = sum_{(c',a)} A[line][(c',a)] B[(c',a)][(c,i)],
//   A[line][(c,a)] = field_c(a along d, line),
//   B = block-diagonal copies of D^T (forward) or D (transpose),
// with G = min(3, 16/n) components per tile: component c of the group takes
// the K slots 8c .. 8c+n-1 (the eight slots one 16-lane group supplies, so
// every operand address is base + a * stride) and the N columns
// c n .. c n + n-1.  Lines fill the M dimension in tiles of 16.
// This is the matrix-core counterpart of the paper's packing of several
// small products into one outer-product tile (Sec. IV-A); the useful fraction
// of each MFMA is (G n / 32)(G n / 16)(1/G) of its multiply-adds.
//
// Assembly as in the FP32 kernel: read-modify-write inside a colour (with
// first-touch stores when the launch carries them) or atomics.
//
// Precision treatment (low-precision operands only):
//   * the forward operand is u - u(local node 0) per component, so a rigid
//     translation gives exactly zero derivatives (D 1 = 0 no longer holds
//     after rounding D);
//   * FP16 operands are scaled per element by a power of two so that the
//     largest magnitude is in [0.5, 1) (FP16 range); results are unscaled in
//     FP32.  BF16 shares FP32's exponent range and is not scaled (a power of
//     two would not change its rounding).
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
struct Op<SEMX_C_MFMA_F32> {  // FP32 operands: K = 4 per instruction, one value per lane
  using vec = float __attribute__((ext_vector_type(8)));
  using elt = float;
  __device__ static f32x4 mma1(float a, float b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
template <>
struct Op<SEMX_C_F16> {
  using vec = f16x8;
  using elt = _Float16;
  __device__ static f32x4 mma(vec a, vec b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};

// First element-local point of `line` for contractions along `dir`, and the
// step between consecutive points of the line: the points of the line are
// line_base + a * line_stride, a = 0..NG-1.
template <int NG>
__device__ __forceinline__ int line_base(int dir, int line) {
  if (dir == 0) return NG * line;                              // line = j + NG k
  if (dir == 1) return (line % NG) + NG * NG * (line / NG);    // line = i + NG k
  return line;                                                 // line = i + NG j
}
template <int NG>
__device__ __forceinline__ int line_stride(int dir) {
  return dir == 0 ? 1 : (dir == 1 ? NG : NG * NG);
}

// Wave maximum of v, written to s_red[wave] (read after the next barrier).
__device__ __forceinline__ void wave_max_to(float v, float* s_red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x / 64] = v;
}

// power of two p with p * x in [0.5, 1) (1 for x = 0)
__device__ __forceinline__ float pow2_scale(float x) {
  if (!(x > 0.0f)) return 1.0f;
  int e;
  frexpf(x, &e);  // x = f 2^e, f in [0.5, 1)
  return ldexpf(1.0f, -e);
}

// One contraction pass on the matrix cores.  Job = (direction, component
// group, tile of 16 lines).  A[line][8 c + a] = src_c(point a of line) for
// the G components of the group (lane group kg = lane / 16 holds component
// kg, K slots 8 kg .. 8 kg + 7, of which the first NG are used); B is the
// block-diagonal matrix of the pass; C[line][c NG + i] lands at point i of
// the line in dst[(c, dir)].  `dst_cd` selects the index of the
// (component, direction) slice: (c * 3 + dir) forward, (dir * 3 + c) transpose.
template <int NG, int PREC, bool TRANSPOSE>
__device__ __forceinline__ void contract_pass(const float* src, int src_stride_c, int src_stride_d, float* dst,
                                              typename Op<PREC>::vec B, const float* ub, float sc, float isc,
                                              int wave, int lane) {
  using O = Op<PREC>;
  using vec = typename O::vec;
  using elt = typename O::elt;
  constexpr int N3 = NG * NG * NG;
  constexpr int NW = Shape<NG>::BLK / 64;
  constexpr int G = (3 < 16 / NG) ? 3 : 16 / NG;
  constexpr int NGRP = (3 + G - 1) / G;
  constexpr int NL = NG * NG;
  constexpr int NT = (NL + 15) / 16;
  constexpr int NJOB = 3 * NGRP * NT;
  const int col = lane & 15, kg = lane >> 4;
#pragma unroll
  for (int jj = 0; jj < (NJOB + NW - 1) / NW; ++jj) {
    const int job = wave + jj * NW;
    if (job >= NJOB) break;  // uniform over the wave
    const int dir = job / (NGRP * NT);
    const int cg = (job / NT) % NGRP;
    const int tile = job % NT;
    const int stride = line_stride<NG>(dir);
    // A operand
    const int ca = cg * G + kg;
    const int line = tile * 16 + col;
    const bool va = kg < G && ca < 3 && line < NL;
    const float* sp = src + (va ? ca * src_stride_c + dir * src_stride_d + line_base<NG>(dir, line) : 0);
    const float off = !va ? 0.0f : (ca == 0 ? ub[0] : (ca == 1 ? ub[1] : ub[2]));
    f32x4 C = {0.f, 0.f, 0.f, 0.f};
    if constexpr (PREC == SEMX_C_MFMA_F32) {
      // one K = 4 step per point a of the line: lane group kg supplies its
      // component's value at point a and the matching row of the block of D
#pragma unroll
      for (int t = 0; t < NG; ++t) C = O::mma1(va ? sp[t * stride] : 0.0f, B[t], C);
    } else {
      vec A;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        float v = 0.0f;
        if (t < NG && va) v = (sp[t * stride] - off) * sc;
        A[t] = (elt)v;
      }
      C = O::mma(A, B, C);
    }
    // C rows 4 kg + r of the tile, column col = c_local * NG + i
    const int cc = cg * G + col / NG, i = col % NG;
    if (col < G * NG && cc < 3) {
      float* dp = dst + (TRANSPOSE ? (dir * 3 + cc) : (cc * 3 + dir)) * N3 + i * stride;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ln = tile * 16 + 4 * kg + r;
        if (ln < NL) dp[line_base<NG>(dir, ln)] = C[r] * isc;
      }
    }
  }
}

template <int NG, int GEO, bool ATOMIC, int PREC>
__global__ __launch_bounds__(Shape<NG>::BLK) void force_mfma_kernel(ForceArgs a) {
  using O = Op<PREC>;
  using vec = typename O::vec;
  using elt = typename O::elt;
  constexpr int N3 = Shape<NG>::N3;
  constexpr int NW = Shape<NG>::BLK / 64;
  constexpr int G = (3 < 16 / NG) ? 3 : 16 / NG;
  constexpr bool SCALE = PREC == SEMX_C_F16;  // BF16 has the FP32 exponent range
  __shared__ float s_u[3 * N3];
  __shared__ float s_d[9 * N3];  // derivatives, then transpose partial sums
  __shared__ float s_q[9 * N3];
  __shared__ float s_D[NG * NG];
  __shared__ float s_red[2][16];

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
  bool first = false;  // first point to reach its node in launch order: store, no read
  if constexpr (!ATOMIC)
    if (a.first) first = (a.first[(size_t)pos * a.first_words + (pp >> 5)] >> (pp & 31)) & 1u;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    uu[c] = u[3 * (size_t)g + c];
    if constexpr (!ATOMIC)
      if (!first) f0[c] = f[3 * (size_t)g + c];
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

  // B operands: block-diagonal D^T (forward: B[8c + a][c NG + i] = D[i][a])
  // and D (transpose: B[8c + a][c NG + i] = D[a][i]), c < G
  const int col = lane & 15, kg = lane >> 4;
  vec Bf, Bt;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    float vf = 0.0f, vt = 0.0f;
    if (t < NG && kg < G && col < G * NG && col / NG == kg) {
      const int ii = col % NG;
      vf = s_D[ii * NG + t];  // D[i][a]
      vt = s_D[t * NG + ii];  // D[a][i]
    }
    Bf[t] = (elt)vf;
    Bt[t] = (elt)vt;
  }

  // forward operand: u - u(node 0) (exact zero for a rigid translation);
  // FP16 also scales it per element by a power of two
  float ub[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) ub[c] = PREC == SEMX_C_MFMA_F32 ? 0.0f : s_u[c * N3];
  float su = 1.0f, isu = 1.0f;
  if constexpr (SCALE) {
    float um = 0.0f;
    if (act)
#pragma unroll
      for (int c = 0; c < 3; ++c) um = fmaxf(um, fabsf(uu[c] - ub[c]));
    wave_max_to(um, s_red[0]);
    __syncthreads();
    float m = 0.0f;
#pragma unroll
    for (int w = 0; w < NW; ++w) m = fmaxf(m, s_red[0][w]);
    su = pow2_scale(m);
    isu = 1.0f / su;
  }
  contract_pass<NG, PREC, false>(s_u, N3, 0, s_d, Bf, ub, su, isu, wave, lane);
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
  float sq = 1.0f, isq = 1.0f;
  if constexpr (SCALE) {
    float qm = 0.0f;
    if (act)
#pragma unroll
      for (int t = 0; t < 9; ++t) qm = fmaxf(qm, fabsf(s_q[t * N3 + pp]));
    wave_max_to(qm, s_red[1]);
  }
  __syncthreads();  // s_q complete
  if constexpr (SCALE) {
    float m = 0.0f;
#pragma unroll
    for (int w = 0; w < NW; ++w) m = fmaxf(m, s_red[1][w]);
    sq = pow2_scale(m);
    isq = 1.0f / sq;
  }
  const float zero3[3] = {0.f, 0.f, 0.f};
  // flux slice (c, d) sits at s_q[(c * 3 + d) * N3]: component stride 3 N3, direction stride N3
  contract_pass<NG, PREC, true>(s_q, 3 * N3, N3, s_d, Bt, zero3, sq, isq, wave, lane);
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

bool mfma_supported(int n, int) { return (n >= 4 && n <= 8) || (n >= kTileMinNMixed && n <= 16); }

hipError_t launch_force_mfma(int n, int prec, int geo, bool atomic, const ForceArgs& a, hipStream_t s) {
  if (prec == SEMX_C_BF16) return launch_mfma_p<SEMX_C_BF16>(n, geo, atomic, a, s);
  if (prec == SEMX_C_F16) return launch_mfma_p<SEMX_C_F16>(n, geo, atomic, a, s);
  if (prec == SEMX_C_MFMA_F32) return launch_mfma_p<SEMX_C_MFMA_F32>(n, geo, atomic, a, s);
  return hipErrorInvalidValue;
}

}  // namespace semx
