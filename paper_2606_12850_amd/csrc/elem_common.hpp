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

// XCD-aware group index: blocks are dispatched round-robin over the XCDs, so
// block b runs on XCD b % 8; groups are dealt so that each XCD walks one
// contiguous eighth of the launch range (elements sharing nodes meet in one L2).
__device__ __forceinline__ int xcd_group(int ngrp) {
  const int gpx = (ngrp + kNumXcd - 1) / kNumXcd;
  return (blockIdx.x % kNumXcd) * gpx + blockIdx.x / kNumXcd;
}

}  // namespace semx
