// Element internal-force kernel for NGLL 11..16 on the matrix cores (FP32
// operands from NGLL 13, 16-bit operands from NGLL 11).
//
// The operator is that of force_f32.hip and force_high.hip (Sec. II-B weak
// form: three forward and three transpose sum-factorised contractions with
// the 16 x 16 derivative matrix D around the pointwise Gamma map, isotropic
// stress and weighted flux; Sec. IV-D fused traversal).  At NGLL 16 every
// contraction is an exact 16 x 16 x 16 matrix product, so all six run as
// v_mfma_f32_16x16x4f32 (FP32 operands, FP32 accumulation, four K = 4 steps
// per product) and the vector units keep only the pointwise work.  NGLL 11
// to 15 use the same 16-point tile with padding: D is extended by zero rows
// and columns and u, lambda, mu are zero at the padding points, so every
// padded product term is zero and the padding points carry zero flux; only
// the real points are loaded and stored.
//
// Layout.  One workgroup per element, 16 waves.  The matrix-core result tile
// gives lane l of a wave the rows 4 g + t (t = 0..3) of column c, with
// g = l / 16, c = l % 16; the kernel uses that as its point layout:
//   S layout (wave w = slice k):        lane holds (i = 4g+t, j = c, k = w)
//   Z layout (wave w = plane j):        lane holds (i = c, j = w, k = 4g+t)
// Summing the contraction index in the order b = 4 g + m (step m = 0..3,
// lane group g) makes the B operand of step m the lane's own point t = m,
// so the xi contractions (forward and transpose) read registers only, and
// the D operands are eight constant registers per lane:
//   Dr[m] = D[c][4g+m],  Dt[m] = D[4g+m][c].
// The eta contractions take their other operand transposed from LDS and land
// in S layout too; the zeta contractions need the contraction index k in the
// tile, so they run in Z layout and exchange operands and results with the S
// layout through LDS.  Per element: 36 + 36 matrix instructions per wave.
//
// LDS: three regions of 3 x 4096 floats (144 KB, so one workgroup per
// compute unit): R0 = u, later the eta fluxes; R1 = zeta derivatives, later
// the zeta transpose result; R2 = the zeta fluxes.  Four barriers per element.
//
// Assembly as in the other element kernels: read-modify-write inside a
// colour (first-touch stores when the launch carries them) or FP32 atomics.
//
// NC = 1 runs the scalar (acoustic) operator on the same tiles: one field
// component (three forward and three transpose products per element), the
// flux Phi_d = (W / rho) sum_b g_b Gamma_db from the first half of the
// material table, and a third of the LDS.
#include <algorithm>

#include "elem_common.hpp"

namespace semx {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kN = 16;
constexpr int kN3 = kN * kN * kN;
constexpr int kWaves = 16;
constexpr int kBlk = 64 * kWaves;

// LDS word of element-local point (i, j, k) in one 4096-float field: rows of
// 16 along i with two XOR swizzles, a bijection of the field.  The 4 low-row
// bits of j pick one of four 16-word windows and the row's 4-word groups are
// permuted by j, so that
//   * the S-layout row reads and writes (16 bytes per lane: i = 4g .. 4g+3,
//     j = c) give the 16 lanes of each group distinct 16-byte bank groups,
//   * the transposed S reads (i = c, j = 4g+m) and the Z-layout accesses
//     (i = c, k = 4g+m) give the 64 lanes 64 distinct banks.
__device__ __forceinline__ int lds_at(int i, int j, int k) {
  return (i ^ (j & 12)) + 16 * (j ^ (((j >> 2) ^ (k >> 2)) & 3)) + 256 * k;
}

__device__ __forceinline__ f32x4 mma(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// 16-bit operands: one v_mfma_f32_16x16x32_{bf16,f16} per 16 x 16 x 16
// product.  Lane group g supplies the K slots 8 g .. 8 g + 7 (A row / B
// column l % 16); slot 8 g + t (t < 4) carries contraction index 4 g + t and
// the upper four slots are zero, so the operands are the same values the
// FP32 path feeds to its four K = 4 steps.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
template <int PREC>
struct Low;
template <>
struct Low<SEMX_C_BF16> {
  using vec = bf16x8;
  using elt = __bf16;
  __device__ static f32x4 mma(vec a, vec b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};
template <>
struct Low<SEMX_C_F16> {
  using vec = f16x8;
  using elt = _Float16;
  __device__ static f32x4 mma(vec a, vec b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};
template <>
struct Low<SEMX_C_F32> {  // unused placeholder so that the FP32 instantiation compiles
  using vec = f16x8;
  using elt = _Float16;
  __device__ static f32x4 mma(vec a, vec b, f32x4 c) { return c; }
};

// x0..x3 (times s) in the low four slots of a 16-bit operand
template <int PREC>
__device__ __forceinline__ typename Low<PREC>::vec pack4(float x0, float x1, float x2, float x3) {
  using elt = typename Low<PREC>::elt;
  typename Low<PREC>::vec v;
  v[0] = (elt)x0;
  v[1] = (elt)x1;
  v[2] = (elt)x2;
  v[3] = (elt)x3;
  v[4] = v[5] = v[6] = v[7] = (elt)0.0f;
  return v;
}

// power of two p with p * x in [0.5, 1) (1 for x = 0)
__device__ __forceinline__ float pow2_scale(float x) {
  if (!(x > 0.0f)) return 1.0f;
  int e;
  frexpf(x, &e);
  return ldexpf(1.0f, -e);
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  return v;
}

// a value that is the same on every lane, moved to a scalar register
__device__ __forceinline__ float uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ f32x4 ld4(const float* s) { return *reinterpret_cast<const f32x4*>(s); }
__device__ __forceinline__ void st4(float* s, f32x4 v) { *reinterpret_cast<f32x4*>(s) = v; }

// The lane's own points (S layout) in the element's arrays: element-local
// index q[t] = i + NG j + NG^2 k of point t, and which of the four are real
// points (i, j, k < NG; always all four at NGLL 16).
template <int NG>
struct OwnPts {
  int q0;       // q of point t is q0 + t (consecutive along i)
  uint32_t ok;  // bit t
  __device__ OwnPts(int g, int c, int w) {
    q0 = 4 * g + NG * c + NG * NG * w;
    ok = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (4 * g + t < NG && c < NG && w < NG) ok |= 1u << t;
  }
  __device__ int q(int t) const { return q0 + t; }
  __device__ bool real(int t) const { return (ok >> t) & 1u; }
};

// What the element loop requests ahead of an element's arithmetic: its node
// numbers (computed on the affine path), first-touch bits, u and material.
struct Ahead {
  int node[4];
  uint32_t fw;  // bit t: own point t is the first to reach its node
  float uo[3][4];
  f32x4 lam4, mu4;
};

// At NGLL 16 the four points are contiguous and 16-byte aligned (vector
// loads); below it they are loaded one by one, zero at padding points.
template <int NG>
__device__ __forceinline__ void load_mat(const ForceArgs& a, int model, int pos, const OwnPts<NG>& P, Ahead& h) {
  constexpr int E3 = NG * NG * NG;
  const float* __restrict__ mat = a.mat + (size_t)model * a.nspec * 2 * E3 + (size_t)pos * 2 * E3;
  if constexpr (NG == kN) {
    h.lam4 = ld4(mat + P.q0);
    h.mu4 = ld4(mat + E3 + P.q0);
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      h.lam4[t] = P.real(t) ? mat[P.q(t)] : 0.0f;
      h.mu4[t] = P.real(t) ? mat[E3 + P.q(t)] : 0.0f;
    }
  }
}

template <int NG, bool ATOMIC, bool AFF, bool MAT, int NC = 3>
__device__ __forceinline__ void load_ahead(const ForceArgs& a, const float* __restrict__ u, int model, int pos,
                                           const OwnPts<NG>& P, int g, int c, int w, Ahead& h) {
  constexpr int E3 = NG * NG * NG;
  if constexpr (AFF) {
    const int32_t* r = a.aff + (size_t)pos * 4;
    const int base = r[0] + c * r[2] + w * r[3];
#pragma unroll
    for (int t = 0; t < 4; ++t) h.node[t] = base + (4 * g + t) * r[1];
  } else if constexpr (NG == kN) {
    const int4 nd = *reinterpret_cast<const int4*>(a.ibool + (size_t)pos * E3 + P.q0);
    h.node[0] = nd.x;
    h.node[1] = nd.y;
    h.node[2] = nd.z;
    h.node[3] = nd.w;
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) h.node[t] = P.real(t) ? a.ibool[(size_t)pos * E3 + P.q(t)] : 0;
  }
  h.fw = 0;
  if constexpr (!ATOMIC) {
    if (a.first) {
      const uint32_t* fb = a.first + (size_t)pos * a.first_words;
      if constexpr (NG == kN) {
        h.fw = fb[P.q0 >> 5] >> (P.q0 & 31);
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (P.real(t)) h.fw |= ((fb[P.q(t) >> 5] >> (P.q(t) & 31)) & 1u) << t;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    h.uo[0][t] = h.uo[1][t] = h.uo[2][t] = 0.0f;
    if (P.real(t)) {
#pragma unroll
      for (int e = 0; e < NC; ++e) h.uo[e][t] = u[NC * (size_t)h.node[t] + e];
    }
  }
  if constexpr (MAT) load_mat<NG>(a, model, pos, P, h);
}

// Element loop.  Regular path (tile_persistent): the grid holds one
// workgroup per compute unit (one fills its LDS or its registers) and each
// walks its share of the launch, dealt XCD by XCD as in xcd_group (the
// workgroups on XCD x take the x-th eighth of the range, in steps of the
// number of workgroups there); the next element's node numbers and u (and
// at NGLL 16 with FP32 operands its material) are requested before the
// current one's last two barriers, so that their latency hides behind its
// transpose contractions and assembly.  With per-point geometry (and FP16
// operands on padded tiles) one element per workgroup, its loads requested
// at its start.  Inside a colour no other workgroup of the launch touches
// the element's nodes, so the prior f there may be read at any time before
// the assembly: at the start of the arithmetic in general, and in the
// persistent elastic form after the pointwise stage, just before the next
// element's loads, so that the 12 values are not held through the stress
// computation (this removed the 8-40 bytes per lane that the padded orders
// spilled there with FP32 and BF16 operands, and took 4-21 % off an apply
// at NGLL 11-15).
// The persistent form (the next element requested ahead).  Elastic: on the
// regular path only, and with FP16 operands only at NGLL 16; on padded
// tiles FP16 needs more registers (36-60 bytes per lane spilled) and,
// measured per apply at 2e7 nodes, loses 20-35 %, so it keeps one element
// per workgroup there; with per-point or trilinear geometry the persistent
// form spills 84-176 bytes and loses up to 50 %.  The scalar operator
// (NC = 1) has the room: it gains 5-14 % on every geometry path.  The launch
// sizes the grid by the same rule.
template <int NG, int GEO, int PREC, int NC>
constexpr bool tile_persistent() {
  return NC == 1 || (GEO == kRegular && (NG == kN || PREC != SEMX_C_F16));
}

template <int NG, int GEO, bool ATOMIC, bool AFF, int PREC, int NC>
__global__ __launch_bounds__(kBlk) void force_tile16_kernel(ForceArgs a) {
  static_assert(NC == 3 || PREC == SEMX_C_F32, "the scalar (acoustic) operator runs in FP32");
  constexpr int E3 = NG * NG * NG;
  // persistent, next element requested ahead
  constexpr bool AHEAD = tile_persistent<NG, GEO, PREC, NC>();
  constexpr bool LOW = PREC == SEMX_C_BF16 || PREC == SEMX_C_F16;
  // 16-bit operands and padded tiles need the registers: material at the start
  constexpr bool MAT_AHEAD = AHEAD && !LOW && NG == kN;
  constexpr bool SCALE = PREC == SEMX_C_F16;  // BF16 has the FP32 exponent range
  using L = Low<PREC>;
  using lvec = typename L::vec;
  __shared__ __attribute__((aligned(16))) float r0[NC * kN3];
  __shared__ __attribute__((aligned(16))) float r1[NC * kN3];
  __shared__ __attribute__((aligned(16))) float r2[NC * kN3];
  __shared__ float s_red[2][kWaves];  // FP16: per-wave maxima of the operands

  const int ngrp = (int)a.count;
  const int gpx = (ngrp + kNumXcd - 1) / kNumXcd;
  const int per_xcd = (int)gridDim.x / kNumXcd;
  const int xbeg = ((int)blockIdx.x % kNumXcd) * gpx;
  const int xend = min(xbeg + gpx, ngrp);
  int grp = xbeg + (int)blockIdx.x / kNumXcd;
  if (grp >= xend) return;  // uniform over the block

  const int w = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int g = l >> 4, c = l & 15;
  const int model = blockIdx.y;
  const float* __restrict__ u = a.u + (size_t)model * a.nglob * NC;
  float* f = a.f + (size_t)model * a.nglob * NC;
  const OwnPts<NG> P(g, c, w);          // own points (S layout)
  const int sS = lds_at(4 * g, c, w);  // first of the 4 contiguous LDS words of the own points

  // D (NG x NG) padded to 16 x 16 with zeros
  float Dr[4], Dt[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const bool in = c < NG && 4 * g + m < NG;
    Dr[m] = in ? a.D[c * NG + 4 * g + m] : 0.0f;
    Dt[m] = in ? a.D[(4 * g + m) * NG + c] : 0.0f;
  }
  lvec Dr16{}, Dt16{};
  if constexpr (LOW) {
    Dr16 = pack4<PREC>(Dr[0], Dr[1], Dr[2], Dr[3]);
    Dt16 = pack4<PREC>(Dt[0], Dt[1], Dt[2], Dt[3]);
  }
  float ry = 0.f, rz = 0.f;  // padding points take the nearest node's coordinates (finite, zero flux)
  if constexpr (GEO == kTrilinear) {
    ry = a.xi[min(c, NG - 1)];
    rz = a.xi[min(w, NG - 1)];
  }

  Ahead cur;
  if constexpr (AHEAD) load_ahead<NG, ATOMIC, AFF, MAT_AHEAD, NC>(a, u, model, (int)a.pos0 + grp, P, g, c, w, cur);
  for (;;) {
    const int pos = (int)a.pos0 + grp;
    if constexpr (!AHEAD) load_ahead<NG, ATOMIC, AFF, true, NC>(a, u, model, pos, P, g, c, w, cur);
    if constexpr (AHEAD && !MAT_AHEAD) load_mat<NG>(a, model, pos, P, cur);
    float fo[3][4];
    auto read_prior = [&]() {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        fo[0][t] = fo[1][t] = fo[2][t] = 0.0f;
        if (!ATOMIC && P.real(t) && !((cur.fw >> t) & 1u)) {  // the point's values in one request
          const float* fp = f + NC * (size_t)cur.node[t];
#pragma unroll
          for (int e = 0; e < NC; ++e) fo[e][t] = fp[e];
        }
      }
    };
    if constexpr (!(AHEAD && NC == 3)) read_prior();
    float u0[3] = {0.f, 0.f, 0.f};  // 16-bit operands: u at local point (0,0,0), their offset
    if constexpr (LOW) {
      const int n0 = AFF ? a.aff[(size_t)pos * 4] : a.ibool[(size_t)pos * E3];
#pragma unroll
      for (int e = 0; e < 3; ++e) u0[e] = uniform(u[3 * (size_t)n0 + e]);
    }
    // LDS holds u (FP32 operands) or u - u0 (16-bit operands), zero at
    // padding points either way
    if constexpr (LOW) {
#pragma unroll
      for (int e = 0; e < 3; ++e)
#pragma unroll
        for (int t = 0; t < 4; ++t) cur.uo[e][t] = P.real(t) ? cur.uo[e][t] - u0[e] : 0.0f;
    }
#pragma unroll
    for (int e = 0; e < NC; ++e)
      st4(r0 + e * kN3 + sS, f32x4{cur.uo[e][0], cur.uo[e][1], cur.uo[e][2], cur.uo[e][3]});
    if constexpr (SCALE) {  // largest |u - u0| of the element, per wave
      float um = 0.0f;
#pragma unroll
      for (int e = 0; e < 3; ++e)
#pragma unroll
        for (int t = 0; t < 4; ++t) um = fmaxf(um, fabsf(cur.uo[e][t]));
      um = wave_max(um);
      if (l == 0) s_red[0][w] = um;
    }
    __syncthreads();  // B1: u in R0

    // ---- forward contractions ----
    f32x4 dx[NC], dy[NC];
    float su = 1.0f, isu = 1.0f;
    if constexpr (SCALE) {
      float m = 0.0f;
#pragma unroll
      for (int v = 0; v < kWaves; ++v) m = fmaxf(m, s_red[0][v]);
      su = uniform(pow2_scale(m));
      isu = uniform(1.0f / su);
    }
#pragma unroll
    for (int e = 0; e < NC; ++e) {
      f32x4 x = {0.f, 0.f, 0.f, 0.f}, y = {0.f, 0.f, 0.f, 0.f}, z = {0.f, 0.f, 0.f, 0.f};
      if constexpr (LOW) {
        // operands (u - u0) su: a rigid translation gives exactly zero
        float ya[4], zb[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          ya[m] = r0[e * kN3 + lds_at(c, 4 * g + m, w)] * su;
          zb[m] = r0[e * kN3 + lds_at(c, w, 4 * g + m)] * su;
        }
        x = L::mma(Dr16, pack4<PREC>(cur.uo[e][0] * su, cur.uo[e][1] * su, cur.uo[e][2] * su, cur.uo[e][3] * su), x);
        y = L::mma(pack4<PREC>(ya[0], ya[1], ya[2], ya[3]), Dr16, y);
        z = L::mma(Dr16, pack4<PREC>(zb[0], zb[1], zb[2], zb[3]), z);
        x *= isu;
        y *= isu;
        z *= isu;
      } else {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          x = mma(Dr[m], cur.uo[e][m], x);                               // sum_b D[i][b] u(b, j, k)
          y = mma(r0[e * kN3 + lds_at(c, 4 * g + m, w)], Dr[m], y);      // sum_b u(i, b, k) D[j][b]
          z = mma(Dr[m], r0[e * kN3 + lds_at(c, w, 4 * g + m)], z);      // sum_b D[k][b] u(i, j, b)  (Z)
        }
      }
      dx[e] = x;
      dy[e] = y;
#pragma unroll
      for (int t = 0; t < 4; ++t) r1[e * kN3 + lds_at(c, w, 4 * g + t)] = z[t];
    }
    __syncthreads();  // B2: zeta derivatives in R1; R0 free
    f32x4 dz[NC];
#pragma unroll
    for (int e = 0; e < NC; ++e) dz[e] = ld4(r1 + e * kN3 + sS);

    // ---- pointwise: geometry map, stress, weighted fluxes ----
    const float* src = nullptr;
    if constexpr (GEO == kTrilinear) src = a.tri + (size_t)pos * 24;
    if constexpr (GEO == kRegular) src = a.gam_el + (size_t)pos * 9;
    f32x4 gam4[9];
    if constexpr (GEO == kStored) {
      const float* gp = a.gam_pt + (size_t)pos * 9 * E3;
#pragma unroll
      for (int d = 0; d < 9; ++d) {
        if constexpr (NG == kN) {
          gam4[d] = ld4(gp + d * E3 + P.q0);
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t) gam4[d][t] = P.real(t) ? gp[d * E3 + P.q(t)] : 0.0f;
        }
      }
    }
    f32x4 p0[NC], p1[NC], p2[NC];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      float G[9];
      if constexpr (GEO == kStored) {
#pragma unroll
        for (int d = 0; d < 9; ++d) G[d] = gam4[d][t];
      }
      const float rx = (GEO == kTrilinear) ? a.xi[min(4 * g + t, NG - 1)] : 0.f;
      float Mg[9], scale, det;
      geom_map_from<GEO>(src, G, rx, ry, rz, Mg, scale, det);
      if constexpr (NC == 1) {
        // scalar operator: physical gradient times det' (Mg), then the
        // weighted flux phi_d = (W / rho) scale sum_b g_b Mg[d][b]
        const float dr[3] = {dx[0][t], dy[0][t], dz[0][t]};
        float gs[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) gs[b] = dr[0] * Mg[0 * 3 + b] + dr[1] * Mg[1 * 3 + b] + dr[2] * Mg[2 * 3 + b];
        const float sw = cur.lam4[t] * scale;
        p0[0][t] = sw * (gs[0] * Mg[0] + gs[1] * Mg[1] + gs[2] * Mg[2]);
        p1[0][t] = sw * (gs[0] * Mg[3] + gs[1] * Mg[4] + gs[2] * Mg[5]);
        p2[0][t] = sw * (gs[0] * Mg[6] + gs[1] * Mg[7] + gs[2] * Mg[8]);
      } else {
        float du[3][3];
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          du[e][0] = dx[e][t];
          du[e][1] = dy[e][t];
          du[e][2] = dz[e][t];
        }
        float gr[3][3];
        apply_map(du, Mg, gr);
        const float lw = cur.lam4[t], mw = cur.mu4[t];
        const float ltr = lw * (gr[0][0] + gr[1][1] + gr[2][2]);
        float sg[3][3];
        sg[0][0] = ltr + 2.0f * mw * gr[0][0];
        sg[1][1] = ltr + 2.0f * mw * gr[1][1];
        sg[2][2] = ltr + 2.0f * mw * gr[2][2];
        sg[0][1] = sg[1][0] = mw * (gr[0][1] + gr[1][0]);
        sg[0][2] = sg[2][0] = mw * (gr[0][2] + gr[2][0]);
        sg[1][2] = sg[2][1] = mw * (gr[1][2] + gr[2][1]);
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          float ph[3];
#pragma unroll
          for (int d = 0; d < 3; ++d)
            ph[d] = scale * (sg[e][0] * Mg[d * 3 + 0] + sg[e][1] * Mg[d * 3 + 1] + sg[e][2] * Mg[d * 3 + 2]);
          p0[e][t] = ph[0];
          p1[e][t] = ph[1];
          p2[e][t] = ph[2];
        }
      }
    }
#pragma unroll
    for (int e = 0; e < NC; ++e) {
      st4(r0 + e * kN3 + sS, p1[e]);
      st4(r2 + e * kN3 + sS, p2[e]);
    }
    // ---- transpose contractions ----
    // The xi and eta contractions stay inside the wave's own slice k = w
    // (the eta operand read back from LDS was written by this wave), so
    // 16-bit operands take a per-wave scale there; the zeta operand crosses
    // waves and takes the element's.
    f32x4 F[NC];
    float sqw = 1.0f, isqw = 1.0f;
    if constexpr (SCALE) {
      float qm = 0.0f, zm = 0.0f;
#pragma unroll
      for (int e = 0; e < 3; ++e)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          qm = fmaxf(qm, fmaxf(fabsf(p0[e][t]), fabsf(p1[e][t])));
          zm = fmaxf(zm, fabsf(p2[e][t]));
        }
      sqw = uniform(pow2_scale(wave_max(qm)));
      isqw = uniform(1.0f / sqw);
      zm = wave_max(zm);
      if (l == 0) s_red[1][w] = zm;
    }
#pragma unroll
    for (int e = 0; e < NC; ++e) {
      f32x4 x = {0.f, 0.f, 0.f, 0.f};
      if constexpr (LOW) {
        x = L::mma(Dt16, pack4<PREC>(p0[e][0] * sqw, p0[e][1] * sqw, p0[e][2] * sqw, p0[e][3] * sqw), x);
      } else {
#pragma unroll
        for (int m = 0; m < 4; ++m) x = mma(Dt[m], p0[e][m], x);  // sum_a D[a][i] phi0(a, j, k)
      }
      F[e] = x;
    }
    if constexpr (AHEAD && NC == 3) read_prior();
    const int nxt = grp + per_xcd;
    const bool more = AHEAD && nxt < xend;  // uniform over the block
    Ahead ahead;
    if constexpr (AHEAD) {
      if (more) load_ahead<NG, ATOMIC, AFF, MAT_AHEAD, NC>(a, u, model, (int)a.pos0 + nxt, P, g, c, w, ahead);
    }
    __syncthreads();  // B3: eta fluxes in R0, zeta fluxes in R2; R1 free
    if constexpr (LOW) {
      float sq = 1.0f, isq = 1.0f;
      if constexpr (SCALE) {
        float m = 0.0f;
#pragma unroll
        for (int v = 0; v < kWaves; ++v) m = fmaxf(m, s_red[1][v]);
        sq = uniform(pow2_scale(m));
        isq = uniform(1.0f / sq);
      }
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        float xa[4], zb[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          xa[m] = r0[e * kN3 + lds_at(c, 4 * g + m, w)] * sqw;
          zb[m] = r2[e * kN3 + lds_at(c, w, 4 * g + m)] * sq;
        }
        f32x4 z = {0.f, 0.f, 0.f, 0.f};
        const f32x4 x = L::mma(pack4<PREC>(xa[0], xa[1], xa[2], xa[3]), Dt16, F[e]);
        z = L::mma(Dt16, pack4<PREC>(zb[0], zb[1], zb[2], zb[3]), z);
        F[e] = x * isqw;
        z *= isq;
#pragma unroll
        for (int t = 0; t < 4; ++t) r1[e * kN3 + lds_at(c, w, 4 * g + t)] = z[t];
      }
    } else {
#pragma unroll
      for (int e = 0; e < NC; ++e) {
        f32x4 x = F[e], z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          x = mma(r0[e * kN3 + lds_at(c, 4 * g + m, w)], Dt[m], x);  // sum_a phi1(i, a, k) D[a][j]
          z = mma(Dt[m], r2[e * kN3 + lds_at(c, w, 4 * g + m)], z);  // sum_a D[a][k] phi2(i, j, a)  (Z)
        }
        F[e] = x;
#pragma unroll
        for (int t = 0; t < 4; ++t) r1[e * kN3 + lds_at(c, w, 4 * g + t)] = z[t];
      }
    }
    __syncthreads();  // B4: zeta transpose result in R1 (R0, R2 free for the next element)
#pragma unroll
    for (int e = 0; e < NC; ++e) F[e] += ld4(r1 + e * kN3 + sS);

    // ---- assembly ----
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (!P.real(t)) continue;
      float* fg = f + NC * (size_t)cur.node[t];
#pragma unroll
      for (int e = 0; e < NC; ++e) {
        if constexpr (ATOMIC) unsafeAtomicAdd(fg + e, -F[e][t]);
        else fg[e] = fo[e][t] - F[e][t];
      }
    }
    if (!AHEAD || !more) break;
    grp = nxt;
    if constexpr (AHEAD) cur = ahead;
  }
}

// Workgroups of the persistent grid: one per compute unit of the current
// device, rounded up to a multiple of the XCD count.
int64_t resident_groups() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (cache[dev] == 0) {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0) ncu = 256;
    cache[dev] = ((ncu + kNumXcd - 1) / kNumXcd) * kNumXcd;
  }
  return cache[dev];
}

template <int NG, int GEO, bool ATOMIC, bool AFF, int PREC, int NC>
hipError_t launch_t16(const ForceArgs& a, hipStream_t s) {
  int64_t nb = ((a.count + kNumXcd - 1) / kNumXcd) * kNumXcd;
  if (tile_persistent<NG, GEO, PREC, NC>()) nb = std::min<int64_t>(nb, resident_groups());
  dim3 grid((unsigned)nb, (unsigned)a.nmodels), block(kBlk);
  force_tile16_kernel<NG, GEO, ATOMIC, AFF, PREC, NC><<<grid, block, 0, s>>>(a);
  return hipGetLastError();
}

template <int NG, bool AFF, int PREC, int NC>
hipError_t launch_t16_geo(int geo, bool atomic, const ForceArgs& a, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  switch (geo) {
    case kRegular:
      return atomic ? launch_t16<NG, kRegular, true, AFF, PREC, NC>(a, s)
                    : launch_t16<NG, kRegular, false, AFF, PREC, NC>(a, s);
    case kStored:
      return atomic ? launch_t16<NG, kStored, true, AFF, PREC, NC>(a, s)
                    : launch_t16<NG, kStored, false, AFF, PREC, NC>(a, s);
    case kTrilinear:
      return atomic ? launch_t16<NG, kTrilinear, true, AFF, PREC, NC>(a, s)
                    : launch_t16<NG, kTrilinear, false, AFF, PREC, NC>(a, s);
    default:
      return hipErrorInvalidValue;
  }
}

template <int NG, int PREC, int NC>
hipError_t launch_t16_split(int geo, bool atomic, int64_t naff, const ForceArgs& a, hipStream_t s) {
  // the launch's first naff elements have an affine numbering
  naff = naff < 0 ? 0 : (naff > a.count ? a.count : naff);
  ForceArgs b = a;
  b.count = naff;
  hipError_t e = launch_t16_geo<NG, true, PREC, NC>(geo, atomic, b, s);
  if (e != hipSuccess || naff == a.count) return e;
  b.pos0 = a.pos0 + naff;
  b.count = a.count - naff;
  return launch_t16_geo<NG, false, PREC, NC>(geo, atomic, b, s);
}

template <int PREC, int NC>
hipError_t launch_t16_n(int n, int geo, bool atomic, int64_t naff, const ForceArgs& a, hipStream_t s) {
  switch (n) {
    case 11: return launch_t16_split<11, PREC, NC>(geo, atomic, naff, a, s);
    case 12: return launch_t16_split<12, PREC, NC>(geo, atomic, naff, a, s);
    case 13: return launch_t16_split<13, PREC, NC>(geo, atomic, naff, a, s);
    case 14: return launch_t16_split<14, PREC, NC>(geo, atomic, naff, a, s);
    case 15: return launch_t16_split<15, PREC, NC>(geo, atomic, naff, a, s);
    case 16: return launch_t16_split<16, PREC, NC>(geo, atomic, naff, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_force_tile16_acoustic(int n, int geo, bool atomic, int64_t naff, const ForceArgs& a,
                                        hipStream_t s) {
  if (n < kTileMinNAcoustic) return hipErrorInvalidValue;
  return launch_t16_n<SEMX_C_F32, 1>(n, geo, atomic, naff, a, s);
}

hipError_t launch_force_tile16(int n, int prec, int geo, bool atomic, int64_t naff, const ForceArgs& a,
                               hipStream_t s) {
  switch (prec) {
    case SEMX_C_F32:
    case SEMX_C_MFMA_F32: return launch_t16_n<SEMX_C_F32, 3>(n, geo, atomic, naff, a, s);
    case SEMX_C_BF16: return launch_t16_n<SEMX_C_BF16, 3>(n, geo, atomic, naff, a, s);
    case SEMX_C_F16: return launch_t16_n<SEMX_C_F16, 3>(n, geo, atomic, naff, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace semx
