// Surrogate network kernels: a multilayer perceptron with BF16 matrix-core
// GEMMs (v_mfma_f32_16x16x32_bf16, FP32 accumulation), fused bias + SiLU
// epilogue, SiLU backward, column sums, mean-squared-error loss and Adam with
// FP32 master weights and a BF16 working copy.
//
// Layer l: Z_l = H_l W_l^T + b_l (W_l stored [out][in]), H_{l+1} = SiLU(Z_l)
// for hidden layers, the last layer linear.  Backward with G = dL/dZ_l:
//   dW_l = G^T H_l,  db_l = sum over the batch of G,  dH_l = G W_l,
//   dL/dZ_{l-1} = dH_l * SiLU'(Z_{l-1}).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "semx_internal.hpp"

struct semx_mlp {
  int nl = 0;
  std::vector<int> w;
  int max_batch = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int64_t nparam = 0;
  std::vector<int64_t> woff, boff;
  semx::DevBuf theta, theta_bf, grad, m, v;
  std::vector<semx::DevBuf> Z, H;  // Z[l] [B][w[l+1]], H[l] (l >= 1) [B][w[l]]
  semx::DevBuf g0, g1;             // backward work [B][max width]
  semx::DevBuf scratch;
  semx::DevBuf splitk;             // split-K partial sums
  const float* x_saved = nullptr;
  int batch_saved = 0;
  int device = 0;                  // device current at creation (allocation-free forward)
};

namespace semx {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 32, PADK = 8;
constexpr int64_t kSplitWs = 2 << 20;  // floats of split-K partial sums per network (8 MB)

// Workspace of semx_mlp_forward_noalloc: two activation buffers of
// kNoAllocFloats / 2 floats each, in the code object's own device memory (each
// GPU the library runs on holds one copy until the process ends).  Host code
// never passes `scratch` itself to a kernel: its name is a host-side handle;
// the device address comes from hipGetSymbolAddress, once per device.
constexpr int64_t kNoAllocFloats = 4 << 20;  // 16 MB
__device__ __align__(256) float scratch[kNoAllocFloats];
constexpr int kMaxDevices = 64;
float* g_scratch_dev[kMaxDevices] = {};  // device address of `scratch`, per device
hipError_t g_scratch_err[kMaxDevices] = {};
std::once_flag g_scratch_once[kMaxDevices];

// Resolve `scratch` on the current device (once per device).
hipError_t noalloc_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::call_once(g_scratch_once[dev], [dev]() {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_err[dev] = e;
    g_scratch_dev[dev] = e == hipSuccess ? static_cast<float*>(ptr) : nullptr;
  });
  return g_scratch_err[dev];
}

__device__ __forceinline__ float to_f(float x) { return x; }
__device__ __forceinline__ float to_f(__bf16 x) { return (float)x; }

// Eight consecutive elements starting at p (16-byte aligned when `vec`).
template <class T>
__device__ __forceinline__ void load8(const T* p, float v[8]);
template <>
__device__ __forceinline__ void load8<float>(const float* p, float v[8]) {
  const float4 a = *reinterpret_cast<const float4*>(p), b = *reinterpret_cast<const float4*>(p + 4);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}
template <>
__device__ __forceinline__ void load8<__bf16>(const __bf16* p, float v[8]) {
  const bf16x8 a = *reinterpret_cast<const bf16x8*>(p);
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = (float)a[e];
}

// One operand tile T[r][k] (64 rows x BK) of X(r, k) = X[r * sr + k * sk],
// rows r0 .. r0+63, k in [k0, kend).  KC: X is contiguous along k (sk = 1),
// a thread loads 8 consecutive k of one row; otherwise it is contiguous
// along r (sr = 1) and a thread loads 8 consecutive rows of one k.  `vec`
// allows 16-byte vector loads (checked alignment); ragged edges use scalar
// loads with bounds.
template <class T, bool KC>
__device__ __forceinline__ void load_tile(__bf16 (*Ts)[BK + PADK], const T* __restrict__ X, int64_t sr, int64_t sk,
                                          int R, int r0, int k0, int kend, bool vec, int t) {
  float v[8];
  if constexpr (KC) {
    const int rr = t >> 2, kk = (t & 3) * 8;
    const int r = r0 + rr, k = k0 + kk;
    if (vec && r < R && k + 8 <= kend) {
      load8<T>(X + (int64_t)r * sr + k, v);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (r < R && k + e < kend) ? to_f(X[(int64_t)r * sr + (int64_t)(k + e) * sk]) : 0.0f;
    }
    bf16x8 w;
#pragma unroll
    for (int e = 0; e < 8; ++e) w[e] = (__bf16)v[e];
    *reinterpret_cast<bf16x8*>(&Ts[rr][kk]) = w;
  } else {
    const int kk = t >> 3, rr = (t & 7) * 8;
    const int r = r0 + rr, k = k0 + kk;
    if (vec && k < kend && r + 8 <= R) {
      load8<T>(X + r + (int64_t)k * sk, v);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (r + e < R && k < kend) ? to_f(X[(int64_t)(r + e) * sr + (int64_t)k * sk]) : 0.0f;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) Ts[rr + e][kk] = (__bf16)v[e];
  }
}

// C[m][n] (+)= sum_k A(m,k) B(k,n), A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn].
// EPI 1: + bias[n]; EPI 2: + bias[n] and H[m][n] = SiLU(C[m][n]); EPI 3:
// C[m][n] = SiLU(sum + bias[n]) (inference: the pre-activation is not kept).
// Split-K (gridDim.z > 1, EPI 0 only): slice z covers k in [z kchunk,
// (z+1) kchunk) and stores its partial sums to C + z M N (row stride N).
template <class TA, class TB, int EPI, bool AKC, bool BKC>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K, int kchunk, const TA* __restrict__ A,
                                                   int64_t sam, int64_t sak, int veca, const TB* __restrict__ B,
                                                   int64_t sbk, int64_t sbn, int vecb, float* __restrict__ C,
                                                   int64_t ldc, const float* __restrict__ bias, float* __restrict__ H,
                                                   int accumulate) {
  __shared__ __attribute__((aligned(16))) __bf16 As[BM][BK + PADK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[BN][BK + PADK];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int bm = blockIdx.y * BM, bn = blockIdx.x * BN;
  const int wm = wv >> 1, wn = wv & 1;
  const bool split = gridDim.z > 1;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    load_tile<TA, AKC>(As, A, sam, sak, M, bm, k0, kend, veca != 0, t);
    load_tile<TB, BKC>(Bs, B, sbn, sbk, N, bn, k0, kend, vecb != 0, t);
    __syncthreads();
    bf16x8 av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) av[a] = *reinterpret_cast<const bf16x8*>(&As[wm * 32 + a * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int b = 0; b < 2; ++b) bv[b] = *reinterpret_cast<const bf16x8*>(&Bs[wn * 32 + b * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
    __syncthreads();
  }
  float* Cz = split ? C + (int64_t)blockIdx.z * M * N : C;
  const int64_t ldz = split ? N : ldc;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = bm + wm * 32 + a * 16 + 4 * (lane >> 4) + r;
        const int n = bn + wn * 32 + b * 16 + (lane & 15);
        if (m < M && n < N) {
          float v = acc[a][b][r];
          const int64_t o = (int64_t)m * ldz + n;
          if (!split) {
            if (accumulate) v += Cz[o];
            if (EPI >= 1) v += bias[n];
          }
          if (EPI == 3) {
            Cz[o] = v / (1.0f + expf(-v));
          } else {
            Cz[o] = v;
            if (EPI == 2) H[o] = v / (1.0f + expf(-v));
          }
        }
      }
}

// C[m][n] = sum over the nz slices of P (fixed order: deterministic).
__global__ void splitk_reduce_kernel(int M, int N, int nz, const float* __restrict__ P, float* __restrict__ C,
                                     int64_t ldc) {
  const int64_t MN = (int64_t)M * N;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < MN; t += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int z = 0; z < nz; ++z) s += P[z * MN + t];
    C[(t / N) * ldc + t % N] = s;
  }
}

template <class T>
bool aligned16(const T* p, int64_t stride) {
  return (reinterpret_cast<uintptr_t>(p) % 16 == 0) && ((stride * (int64_t)sizeof(T)) % 16 == 0);
}

template <class TA, class TB, int EPI, bool AKC, bool BKC>
hipError_t gemm_launch(hipStream_t s, int M, int N, int K, const TA* A, int64_t sam, int64_t sak, const TB* B,
                       int64_t sbk, int64_t sbn, float* C, int64_t ldc, const float* bias, float* H, int accumulate,
                       float* ws) {
  // vector loads need unit stride along the loaded direction and 16-byte alignment
  const int veca = (AKC ? sak == 1 : sam == 1) && aligned16(A, AKC ? sam : sak);
  const int vecb = (BKC ? sbk == 1 : sbn == 1) && aligned16(B, BKC ? sbn : sbk);
  const int tiles = ((N + BN - 1) / BN) * ((M + BM - 1) / BM);
  int nz = 1, kchunk = K;
  if (EPI == 0 && !accumulate && ws && tiles < 128 && K >= 1024) {
    nz = std::min<int>(32, (512 + tiles - 1) / tiles);
    kchunk = (((K + nz - 1) / nz + BK - 1) / BK) * BK;
    nz = (K + kchunk - 1) / kchunk;
    while (nz > 1 && (int64_t)nz * M * N > kSplitWs) {
      kchunk *= 2;
      nz = (K + kchunk - 1) / kchunk;
    }
  }
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, nz), block(256);
  gemm_kernel<TA, TB, EPI, AKC, BKC><<<grid, block, 0, s>>>(M, N, K, kchunk, A, sam, sak, veca, B, sbk, sbn, vecb,
                                                            nz > 1 ? ws : C, ldc, bias, H, accumulate);
  if (nz > 1) {
    const int64_t MN = (int64_t)M * N;
    const unsigned nb = (unsigned)std::min<int64_t>((MN + 255) / 256, 4096);
    splitk_reduce_kernel<<<nb, 256, 0, s>>>(M, N, nz, ws, C, ldc);
  }
  return hipGetLastError();
}

// Dispatch on operand layout: contiguous along k (stride 1) or along m / n.
template <class TA, class TB, int EPI>
hipError_t gemm(hipStream_t s, int M, int N, int K, const TA* A, int64_t sam, int64_t sak, const TB* B, int64_t sbk,
                int64_t sbn, float* C, int64_t ldc, const float* bias, float* H, int accumulate, float* ws = nullptr) {
  const bool akc = sak == 1 || sam != 1;
  const bool bkc = sbk == 1 || sbn != 1;
  if (akc && bkc)
    return gemm_launch<TA, TB, EPI, true, true>(s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, H, accumulate, ws);
  if (akc)
    return gemm_launch<TA, TB, EPI, true, false>(s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, H, accumulate, ws);
  if (bkc)
    return gemm_launch<TA, TB, EPI, false, true>(s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, H, accumulate, ws);
  return gemm_launch<TA, TB, EPI, false, false>(s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, H, accumulate, ws);
}

// g *= SiLU'(z)
__global__ void silu_bwd_kernel(int64_t n, const float* __restrict__ z, float* __restrict__ g) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const float s = 1.0f / (1.0f + expf(-z[t]));
    g[t] *= s * (1.0f + z[t] * (1.0f - s));
  }
}

// db[n] = sum_m g[m][n]
__global__ void colsum_kernel(int M, int N, const float* __restrict__ g, float* __restrict__ db) {
  for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int m = 0; m < M; ++m) s += g[(int64_t)m * N + n];
    db[n] = s;
  }
}

// loss += sum (y - t)^2 / n (FP64), dy = 2 (y - t) / n
__global__ void mse_kernel(int64_t n, const float* __restrict__ y, const float* __restrict__ t, float* __restrict__ dy,
                           double* __restrict__ loss) {
  __shared__ double red[256];
  double s = 0.0;
  const float inv = 1.0f / (float)n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float d = y[i] - t[i];
    if (dy) dy[i] = 2.0f * d * inv;
    s += (double)d * (double)d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, red[0] / (double)n);
}

// y[r][c] = a[c] x[r][c] + b[c] (column-wise affine map; x and y may alias)
__global__ void affine_cols_kernel(int64_t n, int cols, const float* x, const float* __restrict__ a,
                                   const float* __restrict__ b, float* y) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(t % cols);
    y[t] = a[c] * x[t] + b[c];
  }
}

// Ensemble statistics of one row per block: members' predictions P[k][r][c]
// (normalised units), mean over members mapped back through a[c] m + b[c],
// and the spread indicator || a * std || / || mean (physical) || with the
// unbiased standard deviation over the members (zero for one member); the
// two norms are FP64 block reductions in a fixed order.
__global__ void ensemble_kernel(int members, int64_t rows, int cols, const float* __restrict__ P,
                                const float* __restrict__ a, const float* __restrict__ b, float* __restrict__ mean,
                                float* __restrict__ ind) {
  __shared__ double red[2][256];
  const int64_t r = blockIdx.x;
  if (r >= rows) return;
  double s_sp = 0.0, s_mn = 0.0;
  const float inv_m = 1.0f / (float)members;
  const float inv_m1 = members > 1 ? 1.0f / (float)(members - 1) : 0.0f;
  for (int c = threadIdx.x; c < cols; c += blockDim.x) {
    float sum = 0.0f;
    for (int k = 0; k < members; ++k) sum += P[((int64_t)k * rows + r) * cols + c];
    const float mu = sum * inv_m;
    float ss = 0.0f;
    for (int k = 0; k < members; ++k) {
      const float d = P[((int64_t)k * rows + r) * cols + c] - mu;
      ss += d * d;
    }
    const float sd = a[c] * sqrtf(ss * inv_m1);
    const float mp = a[c] * mu + b[c];
    mean[r * cols + c] = mp;
    s_sp += (double)sd * sd;
    s_mn += (double)mp * mp;
  }
  red[0][threadIdx.x] = s_sp;
  red[1][threadIdx.x] = s_mn;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      red[0][threadIdx.x] += red[0][threadIdx.x + st];
      red[1][threadIdx.x] += red[1][threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) ind[r] = (float)(sqrt(red[0][0]) / fmax(sqrt(red[1][0]), 1e-30));
}

__global__ void adam_kernel(int64_t n, float lr, float b1, float b2, float eps, float c1, float c2,
                            const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                            float* __restrict__ th, __bf16* __restrict__ thb) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float t = th[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    th[i] = t;
    thb[i] = (__bf16)t;
  }
}

__global__ void to_bf16_kernel(int64_t n, const float* __restrict__ x, __bf16* __restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (__bf16)x[i];
}

unsigned g1(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

int mfail(semx_mlp* p, int code, const std::string& m) {
  if (p) p->err = m;
  return code;
}

int mhip(semx_mlp* p, hipError_t e, const char* what) {
  return mfail(p, SEMX_EHIP, std::string("HIP error ") + hipGetErrorName(e) + " in " + what);
}

int malloc_buf(semx_mlp* p, DevBuf& b, size_t bytes) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
  if (!bytes) return SEMX_OK;
  if (hipMalloc(&b.p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return mfail(p, SEMX_ENOMEM, "hipMalloc failed");
  }
  b.bytes = bytes;
  return SEMX_OK;
}

}  // namespace
}  // namespace semx

using namespace semx;

#define MLP_HIP(p, call)                          \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return mhip(p, e_, #call); \
  } while (0)

extern "C" {

int semx_mlp_create(semx_mlp** out, int nlayers, const int* widths, int max_batch, void* hip_stream) {
  if (!out) return SEMX_EINVAL;
  *out = nullptr;
  if (nlayers < 1 || nlayers > 16 || !widths || max_batch < 1) return SEMX_EINVAL;
  for (int l = 0; l <= nlayers; ++l)
    if (widths[l] < 1 || widths[l] > (1 << 20)) return SEMX_EINVAL;
  semx_mlp* p = new semx_mlp();
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return SEMX_EHIP;
  }
  // the allocation-free forward's workspace on this device (resolved once per device)
  if (noalloc_setup(p->device) != hipSuccess) {
    delete p;
    return SEMX_EHIP;
  }
  p->nl = nlayers;
  p->w.assign(widths, widths + nlayers + 1);
  p->max_batch = max_batch;
  p->stream = static_cast<hipStream_t>(hip_stream);
  int64_t off = 0, maxw = 0;
  for (int l = 0; l < nlayers; ++l) {
    p->woff.push_back(off);
    off += (int64_t)p->w[l + 1] * p->w[l];
    p->boff.push_back(off);
    off += p->w[l + 1];
  }
  for (int x : p->w) maxw = std::max<int64_t>(maxw, x);
  p->nparam = off;
  int rc = malloc_buf(p, p->theta, sizeof(float) * off);
  if (!rc) rc = malloc_buf(p, p->theta_bf, sizeof(__bf16) * off);
  if (!rc) rc = malloc_buf(p, p->grad, sizeof(float) * off);
  if (!rc) rc = malloc_buf(p, p->m, sizeof(float) * off);
  if (!rc) rc = malloc_buf(p, p->v, sizeof(float) * off);
  if (!rc) rc = malloc_buf(p, p->g0, sizeof(float) * max_batch * maxw);
  if (!rc) rc = malloc_buf(p, p->g1, sizeof(float) * max_batch * maxw);
  if (!rc) rc = malloc_buf(p, p->scratch, 64);
  if (!rc) rc = malloc_buf(p, p->splitk, sizeof(float) * semx::kSplitWs);
  p->Z.resize(nlayers);
  p->H.resize(nlayers + 1);
  for (int l = 0; l < nlayers && !rc; ++l) {
    rc = malloc_buf(p, p->Z[l], sizeof(float) * max_batch * p->w[l + 1]);
    if (!rc && l + 1 < nlayers) rc = malloc_buf(p, p->H[l + 1], sizeof(float) * max_batch * p->w[l + 1]);
  }
  if (rc) {
    semx_mlp_destroy(p);
    return rc;
  }
  *out = p;
  return SEMX_OK;
}

int semx_mlp_destroy(semx_mlp* p) {
  if (!p) return SEMX_OK;
  (void)hipStreamSynchronize(p->stream);
  for (DevBuf* b : {&p->theta, &p->theta_bf, &p->grad, &p->m, &p->v, &p->g0, &p->g1, &p->scratch, &p->splitk})
    dev_free(*b);
  for (auto& b : p->Z) dev_free(b);
  for (auto& b : p->H) dev_free(b);
  delete p;
  return SEMX_OK;
}

const char* semx_mlp_last_error(const semx_mlp* p) { return p ? p->err.c_str() : "null network"; }

int semx_mlp_num_params(semx_mlp* p, int64_t* n) {
  if (!p || !n) return SEMX_EINVAL;
  *n = p->nparam;
  return SEMX_OK;
}

int semx_mlp_set_params(semx_mlp* p, const float* params) {
  if (!p || !params) return SEMX_EINVAL;
  MLP_HIP(p, hipMemcpyAsync(p->theta.p, params, sizeof(float) * p->nparam, hipMemcpyHostToDevice, p->stream));
  to_bf16_kernel<<<g1(p->nparam), 256, 0, p->stream>>>(p->nparam, p->theta.as<float>(), p->theta_bf.as<__bf16>());
  MLP_HIP(p, hipMemsetAsync(p->m.p, 0, sizeof(float) * p->nparam, p->stream));
  MLP_HIP(p, hipMemsetAsync(p->v.p, 0, sizeof(float) * p->nparam, p->stream));
  MLP_HIP(p, hipStreamSynchronize(p->stream));
  return SEMX_OK;
}

int semx_mlp_get_params(semx_mlp* p, float* params) {
  if (!p || !params) return SEMX_EINVAL;
  MLP_HIP(p, hipMemcpyAsync(params, p->theta.p, sizeof(float) * p->nparam, hipMemcpyDeviceToHost, p->stream));
  MLP_HIP(p, hipStreamSynchronize(p->stream));
  return SEMX_OK;
}

int semx_mlp_get_grads(semx_mlp* p, float* grads) {
  if (!p || !grads) return SEMX_EINVAL;
  MLP_HIP(p, hipMemcpyAsync(grads, p->grad.p, sizeof(float) * p->nparam, hipMemcpyDeviceToHost, p->stream));
  MLP_HIP(p, hipStreamSynchronize(p->stream));
  return SEMX_OK;
}

int semx_mlp_forward(semx_mlp* p, const float* x_dev, int batch, float* y_dev) {
  if (!p || !x_dev || !y_dev) return SEMX_EINVAL;
  if (batch < 1 || batch > p->max_batch) return mfail(p, SEMX_EINVAL, "forward: batch outside [1, max_batch]");
  const __bf16* W = p->theta_bf.as<__bf16>();
  const float* th = p->theta.as<float>();
  const float* h = x_dev;
  for (int l = 0; l < p->nl; ++l) {
    const int in = p->w[l], out = p->w[l + 1];
    const bool last = l + 1 == p->nl;
    float* z = last ? y_dev : p->Z[l].as<float>();
    hipError_t e;
    // A(m,k) = h[m*in + k], B(k,n) = W[n*in + k]
    if (last)
      e = gemm<float, __bf16, 1>(p->stream, batch, out, in, h, in, 1, W + p->woff[l], 1, in, z, out, th + p->boff[l],
                                 nullptr, 0);
    else
      e = gemm<float, __bf16, 2>(p->stream, batch, out, in, h, in, 1, W + p->woff[l], 1, in, z, out, th + p->boff[l],
                                 p->H[l + 1].as<float>(), 0);
    if (e != hipSuccess) return mhip(p, e, "mlp forward gemm");
    if (!last) h = p->H[l + 1].as<float>();
  }
  // the output layer's pre-activation is y itself; keep a copy for backward bookkeeping
  p->x_saved = x_dev;
  p->batch_saved = batch;
  return SEMX_OK;
}

int semx_mlp_forward_noalloc(semx_mlp* p, const float* x_dev, int batch, float* y_dev) {
  if (!p || !x_dev || !y_dev) return SEMX_EINVAL;
  if (batch < 1) return mfail(p, SEMX_EINVAL, "forward_noalloc: batch must be >= 1");
  int hmax = 0;
  for (int l = 1; l < p->nl; ++l) hmax = std::max(hmax, p->w[l]);
  if ((int64_t)batch * hmax > kNoAllocFloats / 2)
    return mfail(p, SEMX_EINVAL, "forward_noalloc: batch x widest hidden layer above " +
                                     std::to_string(kNoAllocFloats / 2) + " floats");
  float* ws = (p->device >= 0 && p->device < kMaxDevices) ? g_scratch_dev[p->device] : nullptr;
  if (!ws) return mfail(p, SEMX_ESTATE, "forward_noalloc: workspace address not resolved on this device");
  float* buf[2] = {ws, ws + kNoAllocFloats / 2};
  const __bf16* W = p->theta_bf.as<__bf16>();
  const float* th = p->theta.as<float>();
  const float* h = x_dev;
  for (int l = 0; l < p->nl; ++l) {
    const int in = p->w[l], out = p->w[l + 1];
    const bool last = l + 1 == p->nl;
    float* z = last ? y_dev : buf[l & 1];
    hipError_t e;
    if (last)
      e = gemm<float, __bf16, 1>(p->stream, batch, out, in, h, in, 1, W + p->woff[l], 1, in, z, out, th + p->boff[l],
                                 nullptr, 0);
    else
      e = gemm<float, __bf16, 3>(p->stream, batch, out, in, h, in, 1, W + p->woff[l], 1, in, z, out, th + p->boff[l],
                                 nullptr, 0);
    if (e != hipSuccess) return mhip(p, e, "mlp forward_noalloc gemm");
    h = z;
  }
  return SEMX_OK;
}

int semx_mlp_backward(semx_mlp* p, const float* dy_dev, int batch) {
  if (!p || !dy_dev) return SEMX_EINVAL;
  if (!p->x_saved || batch != p->batch_saved)
    return mfail(p, SEMX_ESTATE, "backward: call forward with the same batch first (its input must stay alive)");
  const __bf16* W = p->theta_bf.as<__bf16>();
  float* gr = p->grad.as<float>();
  const float* g = dy_dev;
  float* bufs[2] = {p->g0.as<float>(), p->g1.as<float>()};
  int cur = 0;
  for (int l = p->nl - 1; l >= 0; --l) {
    const int in = p->w[l], out = p->w[l + 1];
    const float* h = (l == 0) ? p->x_saved : p->H[l].as<float>();
    // dW = G^T H : C[n_out][k_in] = sum_b G[b][n_out] H[b][k_in]
    hipError_t e = gemm<float, float, 0>(p->stream, out, in, batch, g, 1, out, h, in, 1, gr + p->woff[l], in, nullptr,
                                          nullptr, 0, p->splitk.as<float>());
    if (e != hipSuccess) return mhip(p, e, "mlp wgrad gemm");
    colsum_kernel<<<g1(out), 256, 0, p->stream>>>(batch, out, g, gr + p->boff[l]);
    if (l == 0) break;
    // dH = G W : C[b][k_in] = sum_o G[b][o] W[o][k_in]
    float* dh = bufs[cur];
    e = gemm<float, __bf16, 0>(p->stream, batch, in, out, g, out, 1, W + p->woff[l], in, 1, dh, in, nullptr, nullptr, 0,
                               p->splitk.as<float>());
    if (e != hipSuccess) return mhip(p, e, "mlp dgrad gemm");
    silu_bwd_kernel<<<g1((int64_t)batch * in), 256, 0, p->stream>>>((int64_t)batch * in, p->Z[l - 1].as<float>(), dh);
    g = dh;
    cur ^= 1;
  }
  MLP_HIP(p, hipGetLastError());
  return SEMX_OK;
}

int semx_mlp_mse(semx_mlp* p, const float* y_dev, const float* t_dev, int64_t n, float* dy_dev, double* loss) {
  if (!p || !y_dev || !t_dev || n < 1) return SEMX_EINVAL;
  double* d = p->scratch.as<double>();
  MLP_HIP(p, hipMemsetAsync(d, 0, sizeof(double), p->stream));
  mse_kernel<<<g1(n) > 1024 ? 1024 : g1(n), 256, 0, p->stream>>>(n, y_dev, t_dev, dy_dev, d);
  MLP_HIP(p, hipGetLastError());
  if (loss) {
    MLP_HIP(p, hipMemcpyAsync(loss, d, sizeof(double), hipMemcpyDeviceToHost, p->stream));
    MLP_HIP(p, hipStreamSynchronize(p->stream));
  }
  return SEMX_OK;
}

int semx_mlp_adam(semx_mlp* p, float lr, float beta1, float beta2, float eps, int64_t step) {
  if (!p || step < 1 || !(lr >= 0.0f)) return SEMX_EINVAL;
  const float c1 = 1.0f - std::pow(beta1, (float)step), c2 = 1.0f - std::pow(beta2, (float)step);
  adam_kernel<<<g1(p->nparam), 256, 0, p->stream>>>(p->nparam, lr, beta1, beta2, eps, c1, c2, p->grad.as<float>(),
                                                    p->m.as<float>(), p->v.as<float>(), p->theta.as<float>(),
                                                    p->theta_bf.as<__bf16>());
  MLP_HIP(p, hipGetLastError());
  return SEMX_OK;
}

int semx_mlp_affine(semx_mlp* p, const float* x_dev, int64_t rows, int cols, const float* scale_dev,
                    const float* shift_dev, float* y_dev) {
  if (!p || !x_dev || !y_dev || !scale_dev || !shift_dev || rows < 0 || cols < 1) return SEMX_EINVAL;
  if (rows == 0) return SEMX_OK;
  const int64_t n = rows * (int64_t)cols;
  affine_cols_kernel<<<g1(n) > 8192 ? 8192 : g1(n), 256, 0, p->stream>>>(n, cols, x_dev, scale_dev, shift_dev, y_dev);
  MLP_HIP(p, hipGetLastError());
  return SEMX_OK;
}

int semx_mlp_ensemble(semx_mlp* p, const float* preds_dev, int members, int64_t rows, int cols,
                      const float* scale_dev, const float* shift_dev, float* mean_dev, float* indicator_dev) {
  if (!p || !preds_dev || !scale_dev || !shift_dev || !mean_dev || !indicator_dev || members < 1 || rows < 0 ||
      cols < 1)
    return SEMX_EINVAL;
  if (rows == 0) return SEMX_OK;
  if (rows > INT32_MAX) return mfail(p, SEMX_EINVAL, "ensemble: too many rows");
  ensemble_kernel<<<(unsigned)rows, 256, 0, p->stream>>>(members, rows, cols, preds_dev, scale_dev, shift_dev,
                                                         mean_dev, indicator_dev);
  MLP_HIP(p, hipGetLastError());
  return SEMX_OK;
}

}  // extern "C"
