// Device building blocks shared by the element kernels (force, adjoint,
// mixed precision): lane layout, sum-factorised contractions through LDS,
// the per-point geometry map and the weighted isotropic stress/flux.
#pragma once
#include "semx_internal.hpp"

namespace semx {

template <int NG>
struct Shape {
  static constexpr int N3 = NG * NG * NG;
  static constexpr int BLK = ((N3 + 63) / 64) * 64;
};

template <class T>
__device__ __forceinline__ T ldnt(const T* p) {
  return __builtin_nontemporal_load(p);
}

// Reference derivatives du[c][d] = d u_c / d xi_d of the element field in
// s_u ([3][N3], i fastest) at lane point (i,j,k): the three forward
// contractions with D (Sec. II-B, xi-derivative as a small matrix product).
template <int NG>
__device__ __forceinline__ void ref_grad(const float* s_u, const float* s_D, int i, int j, int k,
                                         float du[3][3]) {
  constexpr int N3 = NG * NG * NG;
#pragma unroll
  for (int c = 0; c < 3; ++c) du[c][0] = du[c][1] = du[c][2] = 0.0f;
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    const float di = s_D[i * NG + q], dj = s_D[j * NG + q], dk = s_D[k * NG + q];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      du[c][0] += di * s_u[c * N3 + q + NG * (j + NG * k)];
      du[c][1] += dj * s_u[c * N3 + i + NG * (q + NG * k)];
      du[c][2] += dk * s_u[c * N3 + i + NG * (j + NG * q)];
    }
  }
}

// Transpose contractions of the fluxes in s_q ([9][N3], component c,
// direction d at (c*3+d)): F_c = -sum_d sum_a D_{a,l_d} Phi_cd(...).
template <int NG>
__device__ __forceinline__ void ref_div(const float* s_q, const float* s_D, int i, int j, int k, float F[3]) {
  constexpr int N3 = NG * NG * NG;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float s = 0.0f;
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      s += s_D[q * NG + i] * s_q[(c * 3 + 0) * N3 + q + NG * (j + NG * k)];
      s += s_D[q * NG + j] * s_q[(c * 3 + 1) * N3 + i + NG * (q + NG * k)];
      s += s_D[q * NG + k] * s_q[(c * 3 + 2) * N3 + i + NG * (j + NG * q)];
    }
    F[c] = -s;
  }
}

// Geometry map of one point.  Mg is Gamma (kStored, kRegular) or the
// transposed cofactor matrix of J (kTrilinear, J^{-1} = C^T / det J); the
// physical gradient is g = du Mg / det' with det' = 1 (Gamma) or det J, and
// `scale` = 1/det'^2 restores the flux weighting on the trilinear path.
// `det` returns det J on the trilinear path (else 0).  `src` holds the
// element's Gamma (kRegular, 9 floats) or trilinear coefficients
// (kTrilinear, 24 floats: c0..c7 of x, y, z); `G` the point's Gamma (kStored).
template <int GEO>
__device__ __forceinline__ void geom_map_from(const float* src, const float* G, float rx, float ry, float rz,
                                              float Mg[9], float& scale, float& det) {
  scale = 1.0f;
  det = 0.0f;
  if constexpr (GEO == kStored) {
#pragma unroll
    for (int d = 0; d < 9; ++d) Mg[d] = G[d];
  } else if constexpr (GEO == kRegular) {
#pragma unroll
    for (int d = 0; d < 9; ++d) Mg[d] = src[d];
  } else {
    // x_a(r) = c0 + c1 rx + c2 ry + c3 rz + c4 rx ry + c5 rx rz + c6 ry rz + c7 rx ry rz
    float J[3][3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const float* c = src + 8 * ax;
      J[ax][0] = c[1] + c[4] * ry + c[5] * rz + c[7] * (ry * rz);
      J[ax][1] = c[2] + c[4] * rx + c[6] * rz + c[7] * (rx * rz);
      J[ax][2] = c[3] + c[5] * rx + c[6] * ry + c[7] * (rx * ry);
    }
    const float C00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const float C01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const float C02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const float C10 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    const float C11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    const float C12 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    const float C20 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    const float C21 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    const float C22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    det = J[0][0] * C00 + J[0][1] * C01 + J[0][2] * C02;
    Mg[0] = C00; Mg[1] = C10; Mg[2] = C20;
    Mg[3] = C01; Mg[4] = C11; Mg[5] = C21;
    Mg[6] = C02; Mg[7] = C12; Mg[8] = C22;
    // hardware reciprocal (1 ulp): the weighting needs no correctly rounded
    // quotient, and the IEEE division sequence costs ten instructions a point
    const float id = __builtin_amdgcn_rcpf(det);
    scale = id * id;
  }
}

// geom_map_from with the element's data read from the per-position arrays.
template <int GEO>
__device__ __forceinline__ void geom_map(const ForceArgs& a, int pos, const float* G, float rx, float ry,
                                         float rz, float Mg[9], float& scale, float& det) {
  const float* src = nullptr;
  if constexpr (GEO == kRegular) src = a.gam_el + (size_t)pos * 9;
  if constexpr (GEO == kTrilinear) src = a.tri + (size_t)pos * 24;
  geom_map_from<GEO>(src, G, rx, ry, rz, Mg, scale, det);
}

// gr[c][b] = sum_d du[c][d] Mg[d][b]
__device__ __forceinline__ void apply_map(const float du[3][3], const float Mg[9], float gr[3][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      gr[c][b] = du[c][0] * Mg[0 * 3 + b] + du[c][1] * Mg[1 * 3 + b] + du[c][2] * Mg[2 * 3 + b];
}

// Weighted isotropic stress sigma = lambda' tr(g) I + mu' (g + g^T) times
// `scale`, and fluxes Phi[c][d] = sum_b sigma[c][b] Mg[d][b] written to s_q.
__device__ __forceinline__ void stress_flux(const float gr[3][3], float lamw, float muw, float scale,
                                            const float Mg[9], float* s_q, int N3, int pp, bool act) {
  // the weight `scale` is folded into the two moduli before the stress
  const float ls = lamw * scale, ms = muw * scale, ms2 = 2.0f * ms;
  const float ltr = ls * (gr[0][0] + gr[1][1] + gr[2][2]);
  float sg[3][3];
  sg[0][0] = ltr + ms2 * gr[0][0];
  sg[1][1] = ltr + ms2 * gr[1][1];
  sg[2][2] = ltr + ms2 * gr[2][2];
  sg[0][1] = sg[1][0] = ms * (gr[0][1] + gr[1][0]);
  sg[0][2] = sg[2][0] = ms * (gr[0][2] + gr[2][0]);
  sg[1][2] = sg[2][1] = ms * (gr[1][2] + gr[2][1]);
  if (act) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d)
        s_q[(c * 3 + d) * N3 + pp] = sg[c][0] * Mg[d * 3 + 0] + sg[c][1] * Mg[d * 3 + 1] + sg[c][2] * Mg[d * 3 + 2];
  }
}

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

// Node number of local point pp of the element at launch position `pos`
// from the ibool stream (elements without an affine numbering).
template <int NG>
__device__ __forceinline__ int node_of(const ForceArgs& a, int pos, int pp) {
  return ldnt(a.ibool + (size_t)pos * Shape<NG>::N3 + pp);
}

// The node span of an affine-numbered element (node g = g0 + i sx + j sy +
// k sz; four scalar loads per element, no per-point stream and no dependent
// round trip before the gather): raw buffer resources over the element's
// nodes in u and f (NC floats per node), and the lane's byte offset into
// them.  With 32-bit offsets from a per-element base, the gather, the
// prior-force read and the store need no 64-bit address arithmetic.  The
// host classifies an element as affine only when its span fits a 31-bit
// byte offset at three components per node.
struct AffSpan {
  __amdgpu_buffer_rsrc_t ru, rf;
  int off;
};

template <int NG, int NC>
__device__ __forceinline__ AffSpan aff_span(const ForceArgs& a, int pos, const float* u, float* f, int i, int j,
                                            int k) {
  const int* r = a.aff + (size_t)pos * 4;
  const int sx = r[1], sy = r[2], sz = r[3];
  const int lo = (NG - 1) * (min(sx, 0) + min(sy, 0) + min(sz, 0));
  const int gmin = r[0] + lo;
  const int bytes = ((NG - 1) * (abs(sx) + abs(sy) + abs(sz)) + 1) * 4 * NC;
  AffSpan s;
  s.ru = __builtin_amdgcn_make_buffer_rsrc((void*)(u + NC * (size_t)gmin), (short)0, bytes, kBufferWord3);
  s.rf = __builtin_amdgcn_make_buffer_rsrc((void*)(f + NC * (size_t)gmin), (short)0, bytes, kBufferWord3);
  s.off = (i * sx + j * sy + k * sz - lo) * 4 * NC;
  return s;
}

// Node number of local point (i, j, k) of an affine-numbered element.
__device__ __forceinline__ int aff_node(const ForceArgs& a, int pos, int i, int j, int k) {
  const int* r = a.aff + (size_t)pos * 4;
  return r[0] + i * r[1] + j * r[2] + k * r[3];
}

typedef unsigned semx_v3u __attribute__((ext_vector_type(3)));

// The NC values at the lane's node of an affine element, from buffer `r` at
// byte offset `off` (one request per point).
template <int NC>
__device__ __forceinline__ void buf_load(__amdgpu_buffer_rsrc_t r, int off, float x[NC]) {
  if constexpr (NC == 3) {
    const semx_v3u v = __builtin_amdgcn_raw_buffer_load_b96(r, off, 0, 0);
    x[0] = __uint_as_float(v.x);
    x[1] = __uint_as_float(v.y);
    x[2] = __uint_as_float(v.z);
  } else {
    static_assert(NC == 1, "one or three components per node");
    x[0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  }
}

// u at the lane's node of an affine element.
template <int NC>
__device__ __forceinline__ void gather_affine(const AffSpan& s, float x[NC]) {
  buf_load<NC>(s.ru, s.off, x);
}

// Prior force at the lane's node of an affine element: at first-touch points
// the offset is pushed out of range, so the hardware returns zeros and
// fetches nothing, and the read stays one unconditional instruction that the
// compiler counts exactly (no branch, so the wait for u does not also wait
// for f).  2^31 lies past any num_records <= 2^31 - 1, and adding the 8 bytes
// of the last dword cannot wrap a 32-bit offset.
template <int NC>
__device__ __forceinline__ void prior_force_affine(const AffSpan& s, bool first, float x[NC]) {
  buf_load<NC>(s.rf, first ? INT32_MIN : s.off, x);
}

template <int NC>
__device__ __forceinline__ void store_affine(const AffSpan& s, const float x[NC]) {
  if constexpr (NC == 3) {
    semx_v3u v;
    v.x = __float_as_uint(x[0]);
    v.y = __float_as_uint(x[1]);
    v.z = __float_as_uint(x[2]);
    __builtin_amdgcn_raw_buffer_store_b96(v, s.rf, s.off, 0, 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x[0]), s.rf, s.off, 0, 0);
  }
}

// Per-element geometry that is uniform over the workgroup: Gamma (kRegular,
// 9 floats) or the trilinear coefficients (kTrilinear, 24 floats).
template <int GEO>
struct ElemGeom {
  static constexpr int NS = GEO == kRegular ? 9 : (GEO == kTrilinear ? 24 : 1);
  float v[NS];
};

// Loads of the element's uniform geometry (scalar loads), issued where the
// caller puts them.
template <int GEO>
__device__ __forceinline__ void load_elem_geom(const ForceArgs& a, int pos, ElemGeom<GEO>& eg) {
  if constexpr (GEO != kStored) {
    const float* src = GEO == kRegular ? a.gam_el + (size_t)pos * 9 : a.tri + (size_t)pos * 24;
#pragma unroll
    for (int d = 0; d < ElemGeom<GEO>::NS; ++d) eg.v[d] = src[d];
  }
}

// Keeps the element's geometry loads ahead of the caller's first barrier
// (they would otherwise be sunk past it, onto the element's critical path).
// Call after every other load of the element: the compiler treats the empty
// asm statements as possible writers, so loads after them would no longer
// come through the scalar cache.
template <int GEO>
__device__ __forceinline__ void pin_elem_geom(const ElemGeom<GEO>& eg) {
  if constexpr (GEO != kStored) {
#pragma unroll
    for (int d = 0; d < ElemGeom<GEO>::NS; ++d) asm volatile("" ::"s"(eg.v[d]));
  }
}

// A launch range whose first `naff` elements are affine-numbered: two launches.
template <class F>
inline hipError_t split_affine(int64_t naff, const ForceArgs& a, F launch) {
  naff = naff < 0 ? 0 : (naff > a.count ? a.count : naff);
  ForceArgs b = a;
  b.count = naff;
  hipError_t e = naff > 0 ? launch(b, true) : hipSuccess;
  if (e != hipSuccess || naff == a.count) return e;
  b.pos0 = a.pos0 + naff;
  b.count = a.count - naff;
  return launch(b, false);
}

// XCD-aware group index: blocks are dispatched round-robin over the XCDs, so
// block b runs on XCD b % 8; groups are dealt so that each XCD walks one
// contiguous eighth of the launch range (elements sharing nodes meet in one L2).
__device__ __forceinline__ int xcd_group(int ngrp) {
  const int gpx = (ngrp + kNumXcd - 1) / kNumXcd;
  return (blockIdx.x % kNumXcd) * gpx + blockIdx.x / kNumXcd;
}

}  // namespace semx
