// Streaming reference for roofline fractions: the device's achievable HBM
// bandwidth measured with the library's own copy kernel (one 16-byte
// element per lane, non-temporal loads and stores), next to the published
// peak.  One pass per lane measured faster on MI355X than grid-stride loops
// (6.5 against 4.3-5.9 TB/s at 1-4 GiB).
#include <hip/hip_runtime.h>

#include "semx_internal.hpp"

namespace semx {
namespace {

typedef float vec4 __attribute__((ext_vector_type(4)));

__global__ void stream_copy_kernel(const vec4* __restrict__ src, vec4* __restrict__ dst, int64_t n) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) {
    const vec4 v = __builtin_nontemporal_load(src + t);
    __builtin_nontemporal_store(v, dst + t);
  }
}

}  // namespace
}  // namespace semx

using namespace semx;

extern "C" int semx_stream_bandwidth(semx_ctx* c, int64_t nbytes, int reps, double* gbps) {
  if (!c || !gbps) return SEMX_EINVAL;
  if (nbytes <= 0 || nbytes % 16 != 0 || reps <= 0)
    return fail(c, SEMX_EINVAL, "stream_bandwidth: nbytes must be a positive multiple of 16 and reps positive");
  const int64_t n = nbytes / 16;
  if ((n + 255) / 256 > 0x7fffffffLL) return fail(c, SEMX_EINVAL, "stream_bandwidth: nbytes too large");
  DevBuf a, b;
  int rc = dev_alloc(c, a, (size_t)nbytes);
  if (!rc) rc = dev_alloc(c, b, (size_t)nbytes);
  if (rc) {
    dev_free(a);
    dev_free(b);
    return rc;
  }
  const unsigned grid = (unsigned)((n + 255) / 256);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMemsetAsync(a.p, 0, (size_t)nbytes, c->stream);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {  // warm
    stream_copy_kernel<<<grid, 256, 0, c->stream>>>(a.as<vec4>(), b.as<vec4>(), n);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
  for (int k = 0; k < reps && e == hipSuccess; ++k) {
    stream_copy_kernel<<<grid, 256, 0, c->stream>>>(a.as<vec4>(), b.as<vec4>(), n);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  dev_free(a);
  dev_free(b);
  if (e != hipSuccess) return hip_fail(c, e, "stream_bandwidth");
  *gbps = 2.0 * (double)nbytes * reps / (ms * 1e-3) / 1e9;
  return SEMX_OK;
}
