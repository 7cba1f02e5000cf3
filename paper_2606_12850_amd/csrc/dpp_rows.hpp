// Contractions along a 16-point row held one value per lane in a 16-lane
// DPP row of a wavefront (the NGLL 16 column kernels: a slice row of the
// element is exactly one DPP row).  Rotations move values between the lanes
// of a row without going through LDS.
#pragma once
#include <hip/hip_runtime.h>

namespace semx {
namespace {

// Rotation of a value within each 16-lane DPP row: lane i receives the
// value of another lane of its row (R = 0: its own).  Every lane of the row
// must be active.
template <int R>
__device__ __forceinline__ float row_ror(float x) {
  if constexpr (R == 0) return x;
  else return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x120 + R, 0xF, 0xF, true));
}

// out[c] += sum_R w[R * 16] * row_ror<R>(x[c]), R = 0..15
template <int R>
__device__ __forceinline__ void row_contract3(const float* w, const float x[3], float out[3]) {
  if constexpr (R < 16) {
    const float wr = w[R * 16];
    out[0] += wr * row_ror<R>(x[0]);
    out[1] += wr * row_ror<R>(x[1]);
    out[2] += wr * row_ror<R>(x[2]);
    row_contract3<R + 1>(w, x, out);
  }
}

// Source lane (within its row) of row_ror<R> for lane i, R = 0..15.
template <int R>
__device__ __forceinline__ void row_sources(float i, float src[16]) {
  if constexpr (R < 16) {
    src[R] = row_ror<R>(i);
    row_sources<R + 1>(i, src);
  }
}

// out += sum_R w[R * 16] * row_ror<R>(x), R = 0..15 (one component)
template <int R>
__device__ __forceinline__ void row_contract1(const float* w, float x, float& out) {
  if constexpr (R < 16) {
    out += w[R * 16] * row_ror<R>(x);
    row_contract1<R + 1>(w, x, out);
  }
}

}  // namespace
}  // namespace semx
