// libsemx C interface: context, mesh/model upload, force apply, explicit
// Newmark time loop, sources, receivers, checkpoints, energy.
//
// Everything here is either host bookkeeping (validation, colouring, launch
// lists) or a small HIP kernel; the hot operator lives in force_*.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "semx_internal.hpp"

namespace semx {

int fail(semx_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(semx_ctx* c, hipError_t e, const char* what) {
  std::string m = std::string("HIP error ") + hipGetErrorName(e) + " (" + hipGetErrorString(e) +
                  ") in " + what;
  return fail(c, SEMX_EHIP, m);
}

int dev_alloc(semx_ctx* c, DevBuf& b, size_t bytes) {
  dev_free(b);
  if (bytes == 0) return SEMX_OK;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return fail(c, SEMX_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  b.bytes = bytes;
  return SEMX_OK;
}

void dev_free(DevBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t n, int cap = 1 << 16) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

// ---------------------------------------------------------------------------
// Geometry (FP64): J = dx/dxi of the trilinear map at every GLL point,
// det J, Gamma = J^{-1} (rows: gradients of the reference coordinates), and
// W = w_i w_j w_k det J.  Gamma goes out in FP32 and/or FP64 when requested.
// Outputs are stored at the element's launch position (order[pos] = element).
// ---------------------------------------------------------------------------
__global__ void geom_kernel(int n, int64_t nspec, const double* __restrict__ vert,
                            const int32_t* __restrict__ ev, const int32_t* __restrict__ order,
                            const double* __restrict__ xi, const double* __restrict__ w,
                            float* __restrict__ gam_pt, double* __restrict__ wdet, int* __restrict__ bad,
                            double* __restrict__ gam64) {
  const int n3 = n * n * n;
  const int64_t total = nspec * n3;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pos = t / n3;
    const int q = (int)(t - pos * n3);
    const int64_t e = order[pos];
    const int i = q % n, j = (q / n) % n, k = q / (n * n);
    const double r0 = xi[i], r1 = xi[j], r2 = xi[k];
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const double sa = (v & 1) ? 1.0 : -1.0, sb = (v & 2) ? 1.0 : -1.0, sc = (v & 4) ? 1.0 : -1.0;
      const double fa = 1.0 + sa * r0, fb = 1.0 + sb * r1, fc = 1.0 + sc * r2;
      const double d0 = 0.125 * sa * fb * fc, d1 = 0.125 * fa * sb * fc, d2 = 0.125 * fa * fb * sc;
      const double* x = vert + 3 * (int64_t)ev[8 * e + v];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        J[c][0] += x[c] * d0;
        J[c][1] += x[c] * d1;
        J[c][2] += x[c] * d2;
      }
    }
    // cofactor matrix C[a][b]; det = sum_b J[0][b] C[0][b]; J^{-1} = C^T / det
    double C[3][3];
    C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
    if (!(det > 0.0)) atomicOr(bad, 1);
    const double inv = 1.0 / det;
    wdet[t] = w[i] * w[j] * w[k] * det;
    if (gam_pt) {
      float* gp = gam_pt + pos * 9 * n3 + q;
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int b = 0; b < 3; ++b) gp[(d * 3 + b) * n3] = (float)(C[b][d] * inv);
    }
    if (gam64) {
      double* gp = gam64 + pos * 9 * n3 + q;
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int b = 0; b < 3; ++b) gp[(d * 3 + b) * n3] = C[b][d] * inv;
    }
  }
}

// Smallest distance between GLL points adjacent along xi, eta or zeta (FP64),
// reduced with an integer atomicMin on the bit pattern (positive doubles
// order like their bits).
__global__ void spacing_kernel(int n, int64_t nspec, const double* __restrict__ vert,
                               const int32_t* __restrict__ ev, const double* __restrict__ xi,
                               unsigned long long* __restrict__ out) {
  const int n3 = n * n * n;
  const int64_t total = nspec * n3;
  double best = 1e300;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = t / n3;
    const int q = (int)(t - e * n3);
    const int ijk[3] = {q % n, (q / n) % n, q / (n * n)};
    double x0[3];
    auto map = [&](int a, int b, int c, double* x) {
      const double r[3] = {xi[a], xi[b], xi[c]};
      x[0] = x[1] = x[2] = 0.0;
      for (int v = 0; v < 8; ++v) {
        const double Nv = 0.125 * (1.0 + ((v & 1) ? 1.0 : -1.0) * r[0]) *
                          (1.0 + ((v & 2) ? 1.0 : -1.0) * r[1]) * (1.0 + ((v & 4) ? 1.0 : -1.0) * r[2]);
        const double* xv = vert + 3 * (int64_t)ev[8 * e + v];
        x[0] += Nv * xv[0];
        x[1] += Nv * xv[1];
        x[2] += Nv * xv[2];
      }
    };
    map(ijk[0], ijk[1], ijk[2], x0);
    for (int d = 0; d < 3; ++d) {
      if (ijk[d] + 1 >= n) continue;
      int m[3] = {ijk[0], ijk[1], ijk[2]};
      m[d] += 1;
      double x1[3];
      map(m[0], m[1], m[2], x1);
      const double dist = sqrt((x1[0] - x0[0]) * (x1[0] - x0[0]) + (x1[1] - x0[1]) * (x1[1] - x0[1]) +
                               (x1[2] - x0[2]) * (x1[2] - x0[2]));
      best = fmin(best, dist);
    }
  }
  if (best < 1e300) atomicMin(out, (unsigned long long)__double_as_longlong(best));
}

// lambda W, mu W (FP32) and rho W per element-local point for every model,
// in launch order: position pos holds element order[pos] of the user arrays.
__global__ void material_kernel(int n3, int64_t nspec, int nmodels, const int32_t* __restrict__ order,
                                const double* __restrict__ lam, const double* __restrict__ mu,
                                const double* __restrict__ rho, const double* __restrict__ wdet,
                                float* __restrict__ mat, float* __restrict__ wrho) {
  const int64_t total = (int64_t)nmodels * nspec * n3;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t mp = t / n3;  // model * nspec + pos
    const int q = (int)(t - mp * n3);
    const int64_t model = mp / nspec;
    const int64_t pos = mp - model * nspec;
    const int64_t src = (model * nspec + order[pos]) * n3 + q;
    const double W = wdet[pos * n3 + q];
    mat[mp * 2 * n3 + q] = (float)(lam[src] * W);
    mat[mp * 2 * n3 + n3 + q] = (float)(mu[src] * W);
    wrho[t] = (float)(rho[src] * W);
  }
}

// Lumped mass over the launch positions [pbeg, pbeg + count) of one colour
// (no two elements of a colour share a node, so plain read-modify-write in
// FP64 is race free and deterministic).  ibool and wdet are in launch order,
// rho in user order.
__global__ void mass_color_kernel(int n3, int64_t nspec, int64_t nglob, int nmodels, int64_t pbeg,
                                  int64_t count, const int32_t* __restrict__ order,
                                  const int32_t* __restrict__ ibool, const double* __restrict__ rho,
                                  const double* __restrict__ wdet, double* __restrict__ mass) {
  const int64_t total = (int64_t)nmodels * count * n3;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t mp = t / n3;
    const int q = (int)(t - mp * n3);
    const int model = (int)(mp / count);
    const int64_t pos = pbeg + (mp - (int64_t)model * count);
    const int64_t pt = pos * n3 + q;
    mass[(int64_t)model * nglob + ibool[pt]] +=
        rho[((int64_t)model * nspec + order[pos]) * n3 + q] * wdet[pt];
  }
}

// Same sum by one thread in position order (meshes without a valid colouring).
__global__ void mass_serial_kernel(int n3, int64_t nspec, int64_t nglob, int nmodels,
                                   const int32_t* __restrict__ order, const int32_t* __restrict__ ibool,
                                   const double* __restrict__ rho, const double* __restrict__ wdet,
                                   double* __restrict__ mass) {
  for (int model = 0; model < nmodels; ++model)
    for (int64_t pt = 0; pt < nspec * n3; ++pt) {
      const int64_t pos = pt / n3;
      mass[(int64_t)model * nglob + ibool[pt]] +=
          rho[((int64_t)model * nspec + order[pos]) * n3 + (pt - pos * n3)] * wdet[pt];
    }
}

__global__ void minv_kernel(int64_t n, const double* __restrict__ mass, float* __restrict__ minv) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    minv[t] = mass[t] > 0.0 ? (float)(1.0 / mass[t]) : 0.0f;  // a node no element reaches stays at rest
}

__global__ void fill_f32(float* __restrict__ p, int64_t n, float v) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    p[t] = v;
}

__global__ void fill_f64(double* __restrict__ p, int64_t n, double v) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    p[t] = v;
}

// ---------------------------------------------------------------------------
// Explicit Newmark (beta = 0, gamma = 1/2) update, one thread per global node
// and model.  mode bit 1 (kCorrect): acc = M^{-1} f, v += dt/2 acc, and acc
// is stored to a if kStoreA; without it acc is read from a.  Bit 2
// (kPredict): u += dt v + dt^2/2 acc, v += dt/2 acc, f = 0 unless kKeepF
// (the coming force pass overwrites every node).  A step is "correct then
// predict" in one pass, so a never has to be written.
// ---------------------------------------------------------------------------
// kSeg (the adjoint's forward recomputation): also store acc to seg_a and the
// predicted u to seg_u, the segment buffers, in the same pass.
constexpr int kCorrect = 1, kPredict = 2, kStoreA = 4, kKeepF = 8, kSeg = 16;

// One entry (node, component) of the update: m = M^{-1} at the node, ff
// and aa its f and a; uu and vv are updated in place, the acceleration used
// is returned.  Both kernels below apply exactly this.
template <int MODE>
__device__ __forceinline__ float newmark_entry(float m, float ff, float aa, float dt, float hdt, float hdt2, float& uu,
                                               float& vv) {
  float acc;
  if constexpr ((MODE & kCorrect) != 0) {
    acc = m * ff;
    vv = vv + hdt * acc;
  } else {
    acc = aa;
  }
  if constexpr ((MODE & kPredict) != 0) {
    uu = uu + dt * vv + hdt2 * acc;
    vv = vv + hdt * acc;
  }
  return acc;
}

// NC: field components per node (3 elastic, 1 acoustic).  One entry per lane.
template <int MODE, int NC>
__global__ void newmark_kernel(int64_t nnodes, float dt, const float* __restrict__ minv, float* __restrict__ u,
                               float* __restrict__ v, float* __restrict__ a, float* __restrict__ f,
                               float* __restrict__ seg_u, float* __restrict__ seg_a) {
  const float hdt = 0.5f * dt, hdt2 = 0.5f * dt * dt;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < NC * nnodes;
       t += (int64_t)gridDim.x * blockDim.x) {
    constexpr bool C = (MODE & kCorrect) != 0, Pr = (MODE & kPredict) != 0;
    float vv = v[t], uu = Pr ? u[t] : 0.0f;
    const float acc = newmark_entry<MODE>(C ? minv[t / NC] : 0.0f, C ? f[t] : 0.0f, C ? 0.0f : a[t], dt, hdt, hdt2,
                                          uu, vv);
    if constexpr ((MODE & kStoreA) != 0) a[t] = acc;
    if constexpr (C && (MODE & kSeg) != 0) seg_a[t] = acc;
    if constexpr (Pr) {
      u[t] = uu;
      if constexpr ((MODE & kSeg) != 0) seg_u[t] = uu;
      if constexpr ((MODE & kKeepF) == 0) f[t] = 0.0f;
    }
    v[t] = vv;
  }
}

// The same update with four consecutive entries per lane (16-byte loads and
// stores; every array 16-byte aligned).  With NT (a state too large for the
// caches to keep between steps) v and f are streamed with non-temporal loads
// and v with a non-temporal store, so they do not evict u, which the force
// pass gathers next; a state that the caches hold keeps default caching.
// The last (NC nnodes) % 4 entries go to the first lanes, one each.
typedef float semx_f4 __attribute__((ext_vector_type(4)));
template <bool NT>
__device__ __forceinline__ semx_f4 stream_load(const float* p) {
  if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const semx_f4*>(p));
  else return *reinterpret_cast<const semx_f4*>(p);
}

template <int MODE, int NC, bool NT>
__global__ void newmark4_kernel(int64_t nnodes, float dt, const float* __restrict__ minv, float* __restrict__ u,
                                float* __restrict__ v, float* __restrict__ a, float* __restrict__ f,
                                float* __restrict__ seg_u, float* __restrict__ seg_a) {
  constexpr bool C = (MODE & kCorrect) != 0, Pr = (MODE & kPredict) != 0;
  const float hdt = 0.5f * dt, hdt2 = 0.5f * dt * dt;
  const int64_t len = NC * nnodes, len4 = len / 4;
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int64_t q = gid; q < len4; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t0 = 4 * q;
    semx_f4 vv = stream_load<NT>(v + t0);
    semx_f4 uu = {0.0f, 0.0f, 0.0f, 0.0f}, ff = uu, aa = uu, acc;
    if constexpr (Pr) uu = *reinterpret_cast<const semx_f4*>(u + t0);
    if constexpr (C) ff = stream_load<NT>(f + t0);
    else aa = *reinterpret_cast<const semx_f4*>(a + t0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float x = uu[e], y = vv[e];
      acc[e] = newmark_entry<MODE>(C ? minv[(t0 + e) / NC] : 0.0f, ff[e], aa[e], dt, hdt, hdt2, x, y);
      uu[e] = x;
      vv[e] = y;
    }
    if constexpr ((MODE & kStoreA) != 0) *reinterpret_cast<semx_f4*>(a + t0) = acc;
    if constexpr (C && (MODE & kSeg) != 0) *reinterpret_cast<semx_f4*>(seg_a + t0) = acc;
    if constexpr (Pr) {
      *reinterpret_cast<semx_f4*>(u + t0) = uu;
      if constexpr ((MODE & kSeg) != 0) *reinterpret_cast<semx_f4*>(seg_u + t0) = uu;
      if constexpr ((MODE & kKeepF) == 0) *reinterpret_cast<semx_f4*>(f + t0) = (semx_f4){0.0f, 0.0f, 0.0f, 0.0f};
    }
    if constexpr (NT) __builtin_nontemporal_store(vv, reinterpret_cast<semx_f4*>(v + t0));
    else *reinterpret_cast<semx_f4*>(v + t0) = vv;
  }
  const int64_t t = 4 * len4 + gid;
  if (t < len) {
    float vv = v[t], uu = Pr ? u[t] : 0.0f;
    const float acc = newmark_entry<MODE>(C ? minv[t / NC] : 0.0f, C ? f[t] : 0.0f, C ? 0.0f : a[t], dt, hdt, hdt2,
                                          uu, vv);
    if constexpr ((MODE & kStoreA) != 0) a[t] = acc;
    if constexpr (C && (MODE & kSeg) != 0) seg_a[t] = acc;
    if constexpr (Pr) {
      u[t] = uu;
      if constexpr ((MODE & kSeg) != 0) seg_u[t] = uu;
      if constexpr ((MODE & kKeepF) == 0) f[t] = 0.0f;
    }
    v[t] = vv;
  }
}

bool aligned16(const float* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// State arrays from this size up are streamed past the caches by the update.
constexpr int64_t kStreamBytes = int64_t(64) << 20;

template <int MODE, int NC>
void launch_newmark_nc(semx_ctx* c, int64_t nn, unsigned gb, float dt, const float* minv, float* u, float* v,
                       float* a, float* f, float* seg_u, float* seg_a) {
  const bool vec = aligned16(u) && aligned16(v) && aligned16(a) && aligned16(f) && (!seg_u || aligned16(seg_u)) &&
                   (!seg_a || aligned16(seg_a));
  if (vec) {
    const unsigned g4 = grid_for((NC * nn + 3) / 4, 1 << 30);
    // measured crossover: 26 MB per state array (32^3 NGLL 5) runs faster
    // with default caching, 86 MB (48^3) and up with the streaming hints
    if ((int64_t)sizeof(float) * NC * nn >= kStreamBytes)
      newmark4_kernel<MODE, NC, true><<<g4, kThreads, 0, c->stream>>>(nn, dt, minv, u, v, a, f, seg_u, seg_a);
    else
      newmark4_kernel<MODE, NC, false><<<g4, kThreads, 0, c->stream>>>(nn, dt, minv, u, v, a, f, seg_u, seg_a);
  } else {
    newmark_kernel<MODE, NC><<<gb, kThreads, 0, c->stream>>>(nn, dt, minv, u, v, a, f, seg_u, seg_a);
  }
}

// Launch one Newmark variant, with the segment stores when seg_u or seg_a is given.
template <int MODE>
void launch_newmark(semx_ctx* c, int64_t nn, unsigned gb, float dt, const float* minv, float* u, float* v, float* a,
                    float* f, float* seg_u, float* seg_a) {
  if (c->ncomp == 1)
    launch_newmark_nc<MODE, 1>(c, nn, gb, dt, minv, u, v, a, f, nullptr, nullptr);
  else if (seg_u || seg_a)
    launch_newmark_nc<MODE | kSeg, 3>(c, nn, gb, dt, minv, u, v, a, f, seg_u, seg_a);
  else
    launch_newmark_nc<MODE, 3>(c, nn, gb, dt, minv, u, v, a, f, nullptr, nullptr);
}

// a = M^{-1} f without touching v (initial acceleration).
__global__ void accel_kernel(int64_t nnodes, int nc, const float* __restrict__ minv, const float* __restrict__ f,
                             float* __restrict__ a) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nc * nnodes;
       t += (int64_t)gridDim.x * blockDim.x)
    a[t] = minv[t / nc] * f[t];
}

// Point sources at sample m: f[node][c] += sum over the (source s, point q)
// pairs that reach the node of stf[s][m] * l_q(x_s) dir_c (elastic, nc = 3;
// acoustic, nc = 1: l_q(x_s)), all models.  One thread per (model, source
// node, component) sums its pairs in a fixed order (source, then point), so
// the injection is deterministic even where sources share a node.  The
// sample is m, or *step + 1 when `step` is given (the device step counter
// of a graph-captured step: the injection at the end of step n uses sample
// n + 1).
__global__ void source_kernel(int nsn, const int32_t* __restrict__ snode, const int32_t* __restrict__ sptr,
                              const int32_t* __restrict__ sidx, int n3, int nc, int64_t nstf, int64_t m,
                              const int64_t* step, int nmodels, int64_t nglob, const float* __restrict__ wdir,
                              const float* __restrict__ stf, float* __restrict__ f) {
  if (step) m = *step + 1;
  const int64_t per = (int64_t)nsn * nc;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nmodels * per;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t % per;
    const int i = (int)(r / nc), cc = (int)(r % nc);
    float acc = 0.0f;
    for (int k = sptr[i]; k < sptr[i + 1]; ++k) {
      const int p = sidx[k];
      const float amp = (m >= 0 && m < nstf) ? stf[(int64_t)(p / n3) * nstf + m] : 0.0f;
      acc += amp * wdir[(int64_t)nc * p + cc];
    }
    const int64_t idx = ((t / per) * nglob + snode[i]) * nc + cc;
    f[idx] += acc;
  }
}

// Device step counter of graph-captured steps: set before a replay, advanced
// at the end of every captured step.
__global__ void step_set_kernel(int64_t* step, int64_t v) { *step = v; }
__global__ void step_incr_kernel(int64_t* step) { *step += 1; }

// FP64 block reductions accumulated with a double atomic into out[slot].
__device__ inline void block_sum_to(double v, double* out) {
  __shared__ double red[256];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(out, red[0]);
}

// out[0] += sum_g mass_g |x_g|^2 (FP64), over one model's nodes (nc components each).
__global__ void mnorm_kernel(int64_t nglob, int nc, const double* __restrict__ mass, const float* __restrict__ x,
                             double* __restrict__ out) {
  double s = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nc * nglob;
       t += (int64_t)gridDim.x * blockDim.x) {
    const double xv = x[t];
    s += mass[t / nc] * xv * xv;
  }
  block_sum_to(s, out);
}

// out[0] += sum x.y (FP64)
__global__ void dot_kernel(int64_t n, const float* __restrict__ x, const float* __restrict__ y,
                           double* __restrict__ out) {
  double s = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    s += (double)x[t] * (double)y[t];
  block_sum_to(s, out);
}

// flag[0] = 1 if any entry is NaN or Inf
__global__ void finite_kernel(int64_t n, const float* __restrict__ x, int* __restrict__ flag) {
  bool bad = false;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(x[t]);
  if (bad) atomicOr(flag, 1);
}

// power iteration helpers: y = -M^{-1} f (f = -K x), so y = M^{-1} K x
__global__ void neg_minv_kernel(int64_t nglob, int nc, const float* __restrict__ minv, const float* __restrict__ f,
                                float* __restrict__ y, float scale) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nc * nglob;
       t += (int64_t)gridDim.x * blockDim.x)
    y[t] = -minv[t / nc] * f[t] * scale;
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
int check_ctx(semx_ctx* c) {
  if (!c) return SEMX_EINVAL;
  return SEMX_OK;
}

int set_device(semx_ctx* c) {
  SEMX_HIP(c, hipSetDevice(c->device));
  return SEMX_OK;
}

// scratch layout: [0..7] doubles for reductions, then int flags
double* scratch_d(semx_ctx* c) { return c->d_scratch.as<double>(); }
int* scratch_i(semx_ctx* c) { return reinterpret_cast<int*>(c->d_scratch.as<double>() + 8); }


// Greedy first-fit colouring in element order (Sec. IV-C: element adjacency
// from the global-to-local map, colour by colour execution).  Two elements
// conflict when they share a global node; with `corners_only` the conflict
// test uses the 8 corner nodes (enough for a conforming hexahedral mesh,
// where shared edges and faces imply shared corners).
void greedy_color(int n, int64_t nspec, int64_t nglob, const int32_t* ibool, bool corners_only,
                  std::vector<int32_t>& color) {
  const int n3 = n * n * n;
  const int N = n - 1;
  std::vector<int> qs;
  if (corners_only) {
    for (int c = 0; c < 2; ++c)
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) qs.push_back(a * N + n * (b * N + n * c * N));
  } else {
    for (int q = 0; q < n3; ++q) qs.push_back(q);
  }
  // node -> elements (CSR) over the selected local points
  std::vector<int64_t> cnt(nglob + 1, 0);
  for (int64_t e = 0; e < nspec; ++e)
    for (int q : qs) cnt[ibool[e * n3 + q] + 1]++;
  for (int64_t g = 0; g < nglob; ++g) cnt[g + 1] += cnt[g];
  std::vector<int32_t> adj(cnt[nglob]);
  std::vector<int64_t> fillp(cnt.begin(), cnt.end() - 1);
  for (int64_t e = 0; e < nspec; ++e)
    for (int q : qs) adj[fillp[ibool[e * n3 + q]]++] = (int32_t)e;
  color.assign(nspec, -1);
  std::vector<int64_t> stamp(1024, -1);
  for (int64_t e = 0; e < nspec; ++e) {
    for (int q : qs) {
      const int64_t g = ibool[e * n3 + q];
      for (int64_t t = cnt[g]; t < cnt[g + 1]; ++t) {
        const int32_t o = adj[t];
        if (o != e && color[o] >= 0) stamp[color[o]] = e;
      }
    }
    int c = 0;
    while (c < (int)stamp.size() && stamp[c] == e) ++c;
    if (c >= (int)stamp.size()) stamp.resize(stamp.size() * 2, -1);
    color[e] = c;
  }
}

// True if no two elements of a colour share a global node and every element
// has distinct nodes.
bool coloring_valid(int n3, int64_t nspec, int64_t nglob, const int32_t* ibool, int ncolors,
                    const int32_t* cptr, const int32_t* order) {
  std::vector<int64_t> stamp(nglob, -1);
  for (int c = 0; c < ncolors; ++c) {
    for (int32_t t = cptr[c]; t < cptr[c + 1]; ++t) {
      const int64_t e = order[t];
      for (int q = 0; q < n3; ++q) {
        const int64_t g = ibool[e * n3 + q];
        if (stamp[g] == c) return false;
        stamp[g] = c;
      }
    }
  }
  return true;
}

// 2 x 2 x 2 element blocks for the FP32 elastic force at NGLL <= 5 (the
// block kernel, force_block.hip).  Built when every element is affine-numbered
// with the same strides, all elements are of one geometry kind, and the
// elements pair up into blocks: in element order, each element not yet taken
// opens a block with the seven elements whose first node lies one element
// step away along each combination of axes.  Blocks are coloured greedily by
// their eight corner nodes (a conforming structured mesh needs eight colours)
// and the colouring is checked on every node of every block.  `pos_of[e]` is
// element e's launch position.  On success the tables are on the device and
// c->nblocks > 0; otherwise c->nblocks = 0 and the per-element kernel runs.
int build_blocks(semx_ctx* c, const std::vector<int32_t>& pos_of, const std::vector<std::array<int32_t, 4>>& aff,
                 const std::vector<int32_t>& order) {
  c->nblocks = 0;
  c->block_launches.clear();
  for (DevBuf* b : {&c->d_bpos, &c->d_baff, &c->d_bfirst}) dev_free(*b);
  c->h_baff.clear();
  c->h_bfirst.clear();
  const int n = c->n;
  const int64_t nspec = c->nspec;
  if (n < 2 || n > kBlockMaxN || c->ncolors == 0 || nspec % 8 != 0) return SEMX_OK;
  const int64_t sx = aff[0][1], sy = aff[0][2], sz = aff[0][3];
  for (int64_t e = 0; e < nspec; ++e)
    if (aff[e][0] < 0 || aff[e][1] != sx || aff[e][2] != sy || aff[e][3] != sz ||
        c->h_regular[e] != c->h_regular[0])
      return SEMX_OK;
  const int nb1 = 2 * n - 1;
  if (((int64_t)(nb1 - 1) * (std::llabs(sx) + std::llabs(sy) + std::llabs(sz)) + 1) * 12 > INT32_MAX) return SEMX_OK;
  // first node -> element
  std::vector<std::pair<int64_t, int32_t>> first_node(nspec);
  for (int64_t e = 0; e < nspec; ++e) first_node[e] = {aff[e][0], (int32_t)e};
  std::sort(first_node.begin(), first_node.end());
  auto find = [&](int64_t g) -> int32_t {
    auto it = std::lower_bound(first_node.begin(), first_node.end(), std::make_pair(g, (int32_t)-1));
    return (it != first_node.end() && it->first == g) ? it->second : -1;
  };
  const int64_t step[3] = {(n - 1) * sx, (n - 1) * sy, (n - 1) * sz};
  std::vector<int32_t> taken(nspec, 0);
  std::vector<std::array<int32_t, 8>> blocks;
  blocks.reserve(nspec / 8);
  for (int64_t e = 0; e < nspec; ++e) {
    if (taken[e]) continue;
    std::array<int32_t, 8> mem;
    for (int m = 0; m < 8; ++m) {
      const int64_t g = aff[e][0] + (m & 1) * step[0] + ((m >> 1) & 1) * step[1] + (m >> 2) * step[2];
      const int32_t em = find(g);
      if (em < 0 || taken[em]) return SEMX_OK;
      mem[m] = em;
    }
    for (int m = 0; m < 8; ++m) taken[mem[m]] = 1;
    blocks.push_back(mem);
  }
  const int64_t nb = (int64_t)blocks.size();
  auto node = [&](int64_t b, int X, int Y, int Z) -> int64_t {
    return aff[blocks[b][0]][0] + X * sx + Y * sy + Z * sz;
  };
  // every node of a block must lie in the global range (a lattice numbering)
  for (int64_t b = 0; b < nb; ++b)
    for (int v = 0; v < 8; ++v) {
      const int64_t g = node(b, (v & 1) * (nb1 - 1), ((v >> 1) & 1) * (nb1 - 1), (v >> 2) * (nb1 - 1));
      if (g < 0 || g >= c->nglob) return SEMX_OK;
    }
  // greedy block colouring by corner nodes
  std::vector<std::pair<int64_t, int32_t>> corner(nb * 8);
  for (int64_t b = 0; b < nb; ++b)
    for (int v = 0; v < 8; ++v)
      corner[b * 8 + v] = {node(b, (v & 1) * (nb1 - 1), ((v >> 1) & 1) * (nb1 - 1), (v >> 2) * (nb1 - 1)), (int32_t)b};
  std::sort(corner.begin(), corner.end());
  std::vector<int32_t> bcol(nb, -1);
  std::vector<int64_t> stamp(64, -1);
  for (int64_t b = 0; b < nb; ++b) {
    for (int v = 0; v < 8; ++v) {
      const int64_t g = node(b, (v & 1) * (nb1 - 1), ((v >> 1) & 1) * (nb1 - 1), (v >> 2) * (nb1 - 1));
      for (auto it = std::lower_bound(corner.begin(), corner.end(), std::make_pair(g, (int32_t)-1));
           it != corner.end() && it->first == g; ++it)
        if (it->second != b && bcol[it->second] >= 0) stamp[bcol[it->second]] = b;
    }
    int k = 0;
    while (k < (int)stamp.size() && stamp[k] == b) ++k;
    if (k >= (int)stamp.size()) return SEMX_OK;
    bcol[b] = k;
  }
  int nbc = 0;
  for (auto k : bcol) nbc = std::max(nbc, k + 1);
  // launch order: colour-major, blocks in element order inside a colour;
  // check that no two blocks of a colour share any node
  std::vector<int64_t> border;
  border.reserve(nb);
  std::vector<int32_t> seen(c->nglob, -1);
  for (int k = 0; k < nbc; ++k) {
    const int64_t beg = (int64_t)border.size();
    for (int64_t b = 0; b < nb; ++b) {
      if (bcol[b] != k) continue;
      for (int Z = 0; Z < nb1; ++Z)
        for (int Y = 0; Y < nb1; ++Y)
          for (int X = 0; X < nb1; ++X) {
            const int64_t g = node(b, X, Y, Z);
            if (seen[g] == k) return SEMX_OK;
            seen[g] = k;
          }
      border.push_back(b);
    }
    c->block_launches.push_back({beg, (int64_t)border.size() - beg, c->h_regular[0] == 0, 0});
  }
  // tables in block launch order, and the first touch of each node in it
  const int nbn = nb1 * nb1 * nb1, nwb = (nbn + 31) / 32;
  std::vector<int32_t> bpos(nb * 8), baff(nb * 4);
  std::vector<uint32_t> bfirst(nb * nwb, 0u);
  std::vector<uint8_t> touched(c->nglob, 0);
  for (int64_t t = 0; t < nb; ++t) {
    const int64_t b = border[t];
    for (int m = 0; m < 8; ++m) bpos[t * 8 + m] = pos_of[blocks[b][m]];
    baff[t * 4 + 0] = aff[blocks[b][0]][0];
    baff[t * 4 + 1] = (int32_t)sx;
    baff[t * 4 + 2] = (int32_t)sy;
    baff[t * 4 + 3] = (int32_t)sz;
    for (int q = 0; q < nbn; ++q) {
      const int64_t g = node(b, q % nb1, (q / nb1) % nb1, q / (nb1 * nb1));
      if (!touched[g]) {
        touched[g] = 1;
        bfirst[t * nwb + q / 32] |= 1u << (q % 32);
      }
    }
  }
  (void)order;
  int rc = dev_alloc(c, c->d_bpos, sizeof(int32_t) * bpos.size());
  if (!rc) rc = dev_alloc(c, c->d_baff, sizeof(int32_t) * baff.size());
  if (!rc) rc = dev_alloc(c, c->d_bfirst, sizeof(uint32_t) * bfirst.size());
  if (rc) return rc;
  SEMX_HIP(c, hipMemcpy(c->d_bpos.p, bpos.data(), sizeof(int32_t) * bpos.size(), hipMemcpyHostToDevice));
  SEMX_HIP(c, hipMemcpy(c->d_baff.p, baff.data(), sizeof(int32_t) * baff.size(), hipMemcpyHostToDevice));
  SEMX_HIP(c, hipMemcpy(c->d_bfirst.p, bfirst.data(), sizeof(uint32_t) * bfirst.size(), hipMemcpyHostToDevice));
  c->h_baff = std::move(baff);
  c->h_bfirst = std::move(bfirst);
  c->nblocks = nb;
  c->blocks_irregular = c->h_regular[0] == 0;
  return SEMX_OK;
}

// Launch-ordered layout: every per-element array on the device is stored by
// launch position, positions sorted by (geometry kind, colour, element), so
// that each launch (one colour of one kind, or one kind for atomic assembly)
// streams one contiguous range with no element-list indirection.  Then the
// FP64 geometry kernel fills Gamma and W det J in that order.
int build_layout(semx_ctx* c) {
  const int n3 = c->n3;
  const int64_t nspec = c->nspec;
  std::vector<int32_t> order;
  order.reserve(nspec);
  struct Range { int64_t beg, cnt; bool irr; int color; int64_t naff; };
  // affine numbering: ibool(e, i, j, k) = g0 + i sx + j sy + k sz at every point
  // (a lattice numbering); aff[e] = {g0, sx, sy, sz}, g0 = -1 if not affine
  const int n = c->n;
  std::vector<std::array<int32_t, 4>> aff(nspec);
  for (int64_t e = 0; e < nspec; ++e) {
    const int32_t* ie = &c->h_ibool[e * n3];
    const int64_t g0 = ie[0];
    const int64_t sx = n > 1 ? (int64_t)ie[1] - g0 : 0, sy = n > 1 ? (int64_t)ie[n] - g0 : 0,
                  sz = n > 1 ? (int64_t)ie[n * n] - g0 : 0;
    bool ok = true;
    for (int k = 0; k < n && ok; ++k)
      for (int j = 0; j < n && ok; ++j)
        for (int i = 0; i < n && ok; ++i) ok = ie[i + n * (j + n * k)] == g0 + i * sx + j * sy + k * sz;
    // the force kernels read the prior force of an affine element through a
    // buffer over its node span, addressed with a 31-bit byte offset
    if (ok && ((n - 1) * (std::llabs(sx) + std::llabs(sy) + std::llabs(sz)) + 1) * 12 > INT32_MAX) ok = false;
#ifdef SEMX_NO_AFFINE_NUMBERING
    ok = false;
#endif
    aff[e] = ok ? std::array<int32_t, 4>{(int32_t)g0, (int32_t)sx, (int32_t)sy, (int32_t)sz}
                : std::array<int32_t, 4>{-1, 0, 0, 0};
  }
  std::vector<Range> col;
  const int nc = c->ncolors > 0 ? c->ncolors : 1;
  std::vector<int64_t> kind_beg(3, 0);
  for (int irr = 0; irr < 2; ++irr) {
    kind_beg[irr] = (int64_t)order.size();
    for (int k = 0; k < nc; ++k) {
      Range r{(int64_t)order.size(), 0, irr == 1, k, 0};
      if (c->ncolors > 0) {
        for (int32_t t = c->color_ptr[k]; t < c->color_ptr[k + 1]; ++t) {
          const int32_t e = c->elem_order[t];
          if ((c->h_regular[e] == 0) == (irr == 1)) order.push_back(e);
        }
      } else {
        for (int64_t e = 0; e < nspec; ++e)
          if ((c->h_regular[e] == 0) == (irr == 1)) order.push_back((int32_t)e);
      }
      r.cnt = (int64_t)order.size() - r.beg;
      // elements with an affine numbering first (stable): the FP32 force
      // kernel computes their node numbers instead of streaming them
      auto mid = std::stable_partition(order.begin() + r.beg, order.end(),
                                       [&](int32_t e) { return aff[e][0] >= 0; });
      r.naff = mid - (order.begin() + r.beg);
      if (r.cnt) col.push_back(r);
    }
  }
  kind_beg[2] = (int64_t)order.size();
  c->h_order = order;
  c->colored_launches.clear();
  c->atomic_launches.clear();
  // coloured: colour-major execution order, regular before irregular in a colour
  for (int k = 0; k < nc; ++k)
    for (const auto& r : col)
      if (r.color == k) c->colored_launches.push_back({r.beg, r.cnt, r.irr, r.naff});
  // atomic: one launch per kind; its affine elements are not contiguous, so
  // the whole range takes the node-number stream
  for (int irr = 0; irr < 2; ++irr)
    if (kind_beg[irr + 1] > kind_beg[irr])
      c->atomic_launches.push_back({kind_beg[irr], kind_beg[irr + 1] - kind_beg[irr], irr == 1, 0});

  std::vector<int32_t> ib((size_t)nspec * n3), affpos((size_t)nspec * 4);
  std::vector<float> gel((size_t)nspec * 9);
  // trilinear map x_a = sum_m c_m[a] b_m(r) with monomials
  // b = (1, rx, ry, rz, rx ry, rx rz, ry rz, rx ry rz); c_m[a] = 1/8 sum_v x_v[a] b_m(s_v)
  std::vector<float> tri((size_t)nspec * 24, 0.0f);
  for (int64_t pos = 0; pos < nspec; ++pos) {
    const int64_t e = order[pos];
    std::memcpy(&ib[pos * n3], &c->h_ibool[e * n3], sizeof(int32_t) * n3);
    std::memcpy(&affpos[pos * 4], aff[e].data(), sizeof(int32_t) * 4);
    std::memcpy(&gel[pos * 9], &c->h_gam_el[e * 9], sizeof(float) * 9);
    double cm[3][8] = {{0}};
    for (int v = 0; v < 8; ++v) {
      const double sx = (v & 1) ? 1.0 : -1.0, sy = (v & 2) ? 1.0 : -1.0, sz = (v & 4) ? 1.0 : -1.0;
      const double b[8] = {1.0, sx, sy, sz, sx * sy, sx * sz, sy * sz, sx * sy * sz};
      const double* x = &c->h_vert[3 * (int64_t)c->h_elem_vert[8 * e + v]];
      for (int a = 0; a < 3; ++a)
        for (int m = 0; m < 8; ++m) cm[a][m] += 0.125 * x[a] * b[m];
    }
    for (int a = 0; a < 3; ++a)
      for (int m = 0; m < 8; ++m) tri[pos * 24 + 8 * a + m] = (float)cm[a][m];
  }
  // first touch in coloured launch order (colour-major, regular then irregular)
  const int fw = (n3 + 31) / 32;
  std::vector<uint32_t> first;
  c->elem_cover = false;
  c->first_words = 0;
  if (c->ncolors > 0) {
    first.assign((size_t)nspec * fw, 0u);
    std::vector<uint8_t> touched(c->nglob, 0);
    for (const auto& L : c->colored_launches)
      for (int64_t pos = L.pos0; pos < L.pos0 + L.count; ++pos)
        for (int q = 0; q < n3; ++q) {
          const int32_t g = ib[pos * n3 + q];
          if (!touched[g]) {
            touched[g] = 1;
            first[pos * fw + q / 32] |= 1u << (q % 32);
          }
        }
    c->elem_cover = true;
    for (int64_t g = 0; g < c->nglob && c->elem_cover; ++g) c->elem_cover = touched[g] != 0;
    c->first_words = fw;
  }
  // element-interior points that are the only reference to their node
  {
    std::vector<uint8_t> refs(c->nglob, 0);
    for (int64_t t = 0; t < nspec * n3; ++t) refs[ib[t]] = refs[ib[t]] < 2 ? refs[ib[t]] + 1 : 2;
    bool excl = n > 2;
    for (int64_t pos = 0; pos < nspec && excl; ++pos)
      for (int q = 0; q < n3 && excl; ++q) {
        const int qi = q % n, qj = (q / n) % n, qk = q / (n * n);
        const bool interior = qi > 0 && qi < n - 1 && qj > 0 && qj < n - 1 && qk > 0 && qk < n - 1;
        if (interior) excl = refs[ib[pos * n3 + q]] == 1;
      }
    c->interior_exclusive = excl;
  }
  int rc = dev_alloc(c, c->d_order, sizeof(int32_t) * nspec);
  if (!rc && !first.empty()) rc = dev_alloc(c, c->d_first, sizeof(uint32_t) * first.size());
  if (!rc && first.empty()) dev_free(c->d_first);
  if (!rc) rc = dev_alloc(c, c->d_ibool, sizeof(int32_t) * nspec * n3);
  if (!rc) rc = dev_alloc(c, c->d_aff, sizeof(int32_t) * 4 * nspec);
  if (!rc) rc = dev_alloc(c, c->d_gam_el, sizeof(float) * 9 * nspec);
  if (!rc) rc = dev_alloc(c, c->d_tri, sizeof(float) * 24 * nspec);
  if (!rc) rc = dev_alloc(c, c->d_wdet, sizeof(double) * nspec * n3);
  if (!rc && c->nirregular > 0) rc = dev_alloc(c, c->d_gam_pt, sizeof(float) * 9 * nspec * n3);
  if (!rc && c->nirregular == 0) dev_free(c->d_gam_pt);
  if (rc) return rc;
  SEMX_HIP(c, hipMemcpy(c->d_order.p, order.data(), sizeof(int32_t) * nspec, hipMemcpyHostToDevice));
  SEMX_HIP(c, hipMemcpy(c->d_ibool.p, ib.data(), sizeof(int32_t) * nspec * n3, hipMemcpyHostToDevice));
  SEMX_HIP(c, hipMemcpy(c->d_aff.p, affpos.data(), sizeof(int32_t) * 4 * nspec, hipMemcpyHostToDevice));
  if (!first.empty())
    SEMX_HIP(c, hipMemcpy(c->d_first.p, first.data(), sizeof(uint32_t) * first.size(), hipMemcpyHostToDevice));
  c->h_first = std::move(first);
  c->first_tl_dirty = true;
  SEMX_HIP(c, hipMemcpy(c->d_gam_el.p, gel.data(), sizeof(float) * 9 * nspec, hipMemcpyHostToDevice));
  SEMX_HIP(c, hipMemcpy(c->d_tri.p, tri.data(), sizeof(float) * 24 * nspec, hipMemcpyHostToDevice));
  {
    std::vector<int32_t> pos_of(nspec);
    for (int64_t pos = 0; pos < nspec; ++pos) pos_of[order[pos]] = (int32_t)pos;
    rc = build_blocks(c, pos_of, aff, order);
    if (rc) return rc;
  }
  int* bad = scratch_i(c);
  SEMX_HIP(c, hipMemsetAsync(bad, 0, sizeof(int), c->stream));
  geom_kernel<<<grid_for(nspec * n3, 8192), kThreads, 0, c->stream>>>(
      c->n, nspec, c->d_vert.as<double>(), c->d_elem_vert.as<int32_t>(), c->d_order.as<int32_t>(),
      c->d_xi64.as<double>(), c->d_w64.as<double>(), c->d_gam_pt.as<float>(), c->d_wdet.as<double>(), bad,
      nullptr);
  SEMX_HIP(c, hipGetLastError());
  int hbad = 0;
  SEMX_HIP(c, hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  SEMX_HIP(c, hipStreamSynchronize(c->stream));
  if (hbad) return fail(c, SEMX_EGEOM, "upload_mesh: det J <= 0 at some GLL point");
  return SEMX_OK;
}

// Start of a timed force pass: record the opening event of a pair from the
// pool and hand back the closing one.
hipError_t time_pass_begin(semx_ctx* c, hipEvent_t* e1) {
  while (c->ev_pool.size() < c->ev_used + 2) {
    hipEvent_t ev;
    hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) return e;
    c->ev_pool.push_back(ev);
  }
  hipError_t e = hipEventRecord(c->ev_pool[c->ev_used], c->stream);
  *e1 = c->ev_pool[c->ev_used + 1];
  c->ev_used += 2;
  return e;
}

// f = -K u accumulated into f (f must already hold zeros or earlier sums).
// With `first_touch` (coloured per-element paths) the first point to
// reach each node stores instead of adding, so f's prior content is ignored.
// Kernel arguments of a per-element force pass (launch range left empty).
ForceArgs force_args(const semx_ctx* c, const float* u, float* f, bool first_touch) {
  ForceArgs a{};
  a.ibool = c->d_ibool.as<int32_t>();
  a.aff = c->d_aff.as<int32_t>();
  a.gam_pt = c->d_gam_pt.as<float>();
  a.gam_el = c->d_gam_el.as<float>();
  a.tri = c->d_tri.as<float>();
  a.xi = c->d_xi32.as<float>();
  a.mat = c->d_mat.as<float>();
  a.u = u;
  a.f = f;
  a.D = c->d_D.as<float>();
  a.Dh = c->d_Dh.p;
  a.nspec = c->nspec;
  a.nglob = c->nglob;
  a.nmodels = c->nmodels;
  if (first_touch && c->assembly != SEMX_ASM_ATOMIC && c->d_first.p) {
    a.first = c->d_first.as<uint32_t>();
    a.first_words = c->first_words;
  }
  return a;
}

// `f_zero`: f holds zeros on entry, so with atomic assembly the points that
// are their node's only reference may store instead of adding.
// nchunks x G steps through one captured graph of G steps: the steps are
// recorded once on the capture stream (with the device step counter in place
// of the host step index in the source, receiver and source-work kernels,
// and the counter advanced at the end of each step), then the graph is
// launched nchunks times on the context's stream, the counter set from the
// host index before each launch.  The captured steps are the ones
// step_once would launch directly: bitwise the same results.
bool prestores(const semx_ctx* c);
int build_first_tl(semx_ctx* c);

int run_graph_chunks(semx_ctx* c, int64_t nchunks, int64_t G) {
  int rc = SEMX_OK;
  // nothing may allocate or copy synchronously inside the capture
  if (prestores(c) && c->first_tl_dirty) rc = build_first_tl(c);
  if (!rc && !c->d_step.p) rc = dev_alloc(c, c->d_step, sizeof(int64_t));
  if (rc) return rc;
  if (!c->cap_stream) SEMX_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  int64_t* dstep = c->d_step.as<int64_t>();
  const int64_t it0 = c->it;
  const bool pend0 = c->pending_correct;
  hipStream_t home = c->stream;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  c->stream = c->cap_stream;
  hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
  for (int64_t s = 0; s < G && e == hipSuccess && !rc; ++s) {
    c->track_energy = false;
    rc = step_once(c, true, nullptr, nullptr, dstep);
  }
  const hipError_t e_end = e == hipSuccess ? hipStreamEndCapture(c->cap_stream, &graph) : e;
  c->stream = home;
  c->it = it0;  // the capture ran nothing
  c->pending_correct = pend0;
  if (rc || e_end != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc ? rc : hip_fail(c, e_end, "time-loop graph capture");
  }
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(c, e, "time-loop graph instantiate");
  for (int64_t k = 0; k < nchunks && e == hipSuccess; ++k) {
    step_set_kernel<<<1, 1, 0, c->stream>>>(dstep, c->it);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipGraphLaunch(exec, c->stream);
    c->it += G;
  }
  c->pending_correct = true;
  const hipError_t e_destroy = hipGraphExecDestroy(exec);
  if (e != hipSuccess) return hip_fail(c, e, "time-loop graph launch");
  if (e_destroy != hipSuccess) return hip_fail(c, e_destroy, "time-loop graph destroy");
  return SEMX_OK;
}

// True when the FP32 elastic coloured force runs on 2 x 2 x 2 element blocks.
// In the automatic mode only where the block kernel measured faster than the
// per-element kernel: the stored-Gamma path, which streams 36 B of Gamma per
// point and gains from the block's single pass over its nodes (0.583 against
// 0.603 ms per apply at 64^3).  On the trilinear and regular paths the
// per-element kernel keeps 16 elements per compute unit in flight against
// the blocks' two workgroups, and wins (0.42-0.44 against 0.50 ms, 0.49
// against 0.55 ms).
bool blocks_active(const semx_ctx* c) {
  if (c->blocks_mode == SEMX_BLOCKS_OFF || c->nblocks == 0 || c->physics != SEMX_ELASTIC ||
      c->storage != SEMX_F32 || c->contraction != SEMX_C_F32 || c->assembly != SEMX_ASM_COLORED ||
      c->n > kBlockMaxN)
    return false;
  return c->blocks_mode == SEMX_BLOCKS_ON || (c->blocks_irregular && c->irregular_geo == kStored);
}

// `tl`: the time loop's pass after the source force was stored into f
// (prestores()): the first-touch bits with the source nodes cleared.
int force_accumulate(semx_ctx* c, const float* u, float* f, bool first_touch = false, bool f_zero = false,
                     bool tl = false) {
  ForceArgs a = force_args(c, u, f, first_touch);
  if (tl && a.first) a.first = c->d_first_tl.as<uint32_t>();
  const bool atomic = c->assembly == SEMX_ASM_ATOMIC;
  a.excl_interior = atomic && f_zero && c->interior_exclusive ? 1 : 0;
  if (blocks_active(c)) {
    hipEvent_t e1 = nullptr;
    if (c->timing_stride > 0 && (c->timing_seq++ % c->timing_stride) == 0) {
      SEMX_HIP(c, time_pass_begin(c, &e1));
      c->timed_launches += (int64_t)c->block_launches.size();
    }
    const int geo = c->blocks_irregular ? c->irregular_geo : kRegular;
    for (const auto& L : c->block_launches) {
      const uint32_t* bf = !first_touch ? nullptr : tl ? c->d_bfirst_tl.as<uint32_t>() : c->d_bfirst.as<uint32_t>();
      const BlockArgs b{c->d_bpos.as<int32_t>(), c->d_baff.as<int32_t>(), bf, L.pos0, L.count};
      const hipError_t e = launch_force_block(c->n, geo, a, b, c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "force kernel launch");
    }
    if (e1) SEMX_HIP(c, hipEventRecord(e1, c->stream));
    return SEMX_OK;
  }
  const auto& launches = atomic ? c->atomic_launches : c->colored_launches;
  hipEvent_t e1 = nullptr;
  if (!launches.empty() && c->timing_stride > 0 && (c->timing_seq++ % c->timing_stride) == 0) {
    SEMX_HIP(c, time_pass_begin(c, &e1));
    c->timed_launches += (int64_t)launches.size();
  }
  for (const auto& L : launches) {
    a.pos0 = L.pos0;
    a.count = L.count;
    hipError_t e;
    const int geo = L.irregular ? c->irregular_geo : kRegular;
    if (c->physics == SEMX_ACOUSTIC && c->n >= kTileMinNAcoustic)
      e = launch_force_tile16_acoustic(c->n, geo, atomic, L.naff, a, c->stream);
    else if (c->physics == SEMX_ACOUSTIC)
      e = launch_force_acoustic(c->n, geo, atomic, L.naff, a, c->stream);
    else if (c->n >= kTileMinN || (c->n >= kTileMinNMixed && c->contraction != SEMX_C_F32) ||
             (c->n == kTileRegularN && geo == kRegular))
      e = launch_force_tile16(c->n, c->contraction, geo, atomic, L.naff, a, c->stream);
    else if (c->contraction == SEMX_C_F32 && c->n > kMaxNLow)
      e = launch_force_high(c->n, geo, atomic, a, c->stream);
    else if (c->contraction == SEMX_C_F32)
      e = launch_force_f32_split(c->n, geo, atomic, L.naff, a, c->stream);
    else
      e = launch_force_mfma(c->n, c->contraction, geo, atomic, a, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "force kernel launch");
  }
  if (e1) SEMX_HIP(c, hipEventRecord(e1, c->stream));
  return SEMX_OK;
}

int zero_f32(semx_ctx* c, float* p, int64_t n) {
  fill_f32<<<grid_for(n), kThreads, 0, c->stream>>>(p, n, 0.0f);
  SEMX_HIP(c, hipGetLastError());
  return SEMX_OK;
}

int64_t state_len(const semx_ctx* c) { return (int64_t)c->nmodels * c->nglob * c->ncomp; }

// Seismogram buffer [nmodels][nrec][ncomp][nt_max] in the storage precision, zeroed.
int alloc_seismograms(semx_ctx* c) {
  const int nm = c->nmodels > 0 ? c->nmodels : 1;
  const int64_t cnt = (int64_t)nm * c->rec.nrec * c->ncomp * c->rec.nt_max;
  if (c->storage == SEMX_F64) {
    dev_free(c->rec.seis);
    int rc = dev_alloc(c, c->rec.seis64, sizeof(double) * cnt);
    if (rc) return rc;
    fill_f64<<<grid_for(cnt), kThreads, 0, c->stream>>>(c->rec.seis64.as<double>(), cnt, 0.0);
    SEMX_HIP(c, hipGetLastError());
    return SEMX_OK;
  }
  dev_free(c->rec.seis64);
  int rc = dev_alloc(c, c->rec.seis, sizeof(float) * cnt);
  if (rc) return rc;
  return zero_f32(c, c->rec.seis.as<float>(), cnt);
}

// True when the force pass writes every node itself (coloured per-element
// passes with first-touch stores over a mesh whose nodes all belong to some
// element), so f needs no clearing before it.
bool force_overwrites(const semx_ctx* c) {
  return c->assembly == SEMX_ASM_COLORED && c->elem_cover && c->d_first.p != nullptr;
}

// f = -K u.  `f_zeroed`: f already holds zeros.  `tl`: see force_accumulate.
int force_into(semx_ctx* c, const float* u, float* f, bool f_zeroed, bool tl = false) {
  if (!f_zeroed && !force_overwrites(c)) {
    int rc = zero_f32(c, f, state_len(c));
    if (rc) return rc;
  }
  return force_accumulate(c, u, f, force_overwrites(c), !force_overwrites(c), tl);
}

// The time loop stores the source force into f before the force pass (in
// the bookkeeping launch) when the pass overwrites every node with
// first-touch stores: the source nodes' first touch then reads and adds to
// it, and no injection launch follows the pass.
bool prestores(const semx_ctx* c) { return c->src.nsrc > 0 && c->src.nsn > 0 && force_overwrites(c); }

// The time loop's first-touch bits: the bit of each source node's first
// touch (in launch order) cleared, per element and per block.
int build_first_tl(semx_ctx* c) {
  std::vector<uint8_t> src(c->nglob, 0);
  for (int32_t g : c->h_src_nodes)
    if (g < 0 || g >= c->nglob) return fail(c, SEMX_ESTATE, "sources do not belong to the current mesh");
  const int n3 = c->n3, fw = c->first_words;
  if (!c->h_first.empty()) {
    for (int32_t g : c->h_src_nodes) src[g] = 1;
    std::vector<uint32_t> bits = c->h_first;
    for (const auto& L : c->colored_launches)
      for (int64_t pos = L.pos0; pos < L.pos0 + L.count; ++pos) {
        const int32_t* ib = &c->h_ibool[(size_t)c->h_order[pos] * n3];
        for (int q = 0; q < n3; ++q)
          if (src[ib[q]] == 1) {
            src[ib[q]] = 0;
            bits[pos * fw + q / 32] &= ~(1u << (q % 32));
          }
      }
    int rc = dev_alloc(c, c->d_first_tl, sizeof(uint32_t) * bits.size());
    if (rc) return rc;
    SEMX_HIP(c, hipMemcpy(c->d_first_tl.p, bits.data(), sizeof(uint32_t) * bits.size(), hipMemcpyHostToDevice));
  }
  if (c->nblocks > 0 && !c->h_bfirst.empty()) {
    for (int32_t g : c->h_src_nodes) src[g] = 1;
    const int nb1 = 2 * c->n - 1, nbn = nb1 * nb1 * nb1, nwb = (nbn + 31) / 32;
    std::vector<uint32_t> bits = c->h_bfirst;
    for (int64_t t = 0; t < c->nblocks; ++t) {
      const int32_t* r = &c->h_baff[t * 4];
      for (int q = 0; q < nbn; ++q) {
        const int64_t g = r[0] + (int64_t)(q % nb1) * r[1] + (int64_t)((q / nb1) % nb1) * r[2] +
                          (int64_t)(q / (nb1 * nb1)) * r[3];
        if (src[g] == 1) {
          src[g] = 0;
          bits[t * nwb + q / 32] &= ~(1u << (q % 32));
        }
      }
    }
    int rc = dev_alloc(c, c->d_bfirst_tl, sizeof(uint32_t) * bits.size());
    if (rc) return rc;
    SEMX_HIP(c, hipMemcpy(c->d_bfirst_tl.p, bits.data(), sizeof(uint32_t) * bits.size(), hipMemcpyHostToDevice));
  }
  c->first_tl_dirty = false;
  return SEMX_OK;
}


int inject_sources(semx_ctx* c, int64_t m, float* f, const int64_t* dstep = nullptr) {
  if (c->src.nsrc == 0 || c->src.nsn == 0) return SEMX_OK;
  const SourceSet& S = c->src;
  const int64_t total = (int64_t)c->nmodels * S.nsn * c->ncomp;
  source_kernel<<<grid_for(total), kThreads, 0, c->stream>>>(
      S.nsn, S.snode.as<int32_t>(), S.sptr.as<int32_t>(), S.sidx.as<int32_t>(), c->n3, c->ncomp, S.nstf, m, dstep,
      c->nmodels, c->nglob, S.wdir.as<float>(), S.stf.as<float>(), f);
  SEMX_HIP(c, hipGetLastError());
  return SEMX_OK;
}

int finalize_state(semx_ctx* c, float* seg_a = nullptr) {
  if (c->storage == SEMX_F64) return f64_finalize(c);
  if (!c->pending_correct) return SEMX_OK;
  const int64_t nn = (int64_t)c->nmodels * c->nglob;
  launch_newmark<kCorrect | kStoreA>(c, nn, grid_for(c->ncomp * nn), (float)c->dt, c->d_minv.as<float>(),
                                     c->d_u.as<float>(), c->d_v.as<float>(), c->d_a.as<float>(),
                                     c->d_f.as<float>(), nullptr, seg_a);
  SEMX_HIP(c, hipGetLastError());
  c->pending_correct = false;
  return SEMX_OK;
}

int do_reset(semx_ctx* c) {
  c->run_gen++;
  c->ckpt_count = 0;
  if (c->storage == SEMX_F64) return f64_reset(c);
  const int64_t len = state_len(c);
  for (auto* b : {&c->d_u, &c->d_v, &c->d_a, &c->d_f}) {
    int rc = zero_f32(c, b->as<float>(), len);
    if (rc) return rc;
  }
  c->it = 0;
  c->pending_correct = false;
  if (c->rec.nrec > 0 && c->rec.seis.p) {
    int rc = zero_f32(c, c->rec.seis.as<float>(), c->rec.seis.bytes / sizeof(float));
    if (rc) return rc;
  }
  if (c->src.nsrc > 0) {
    int rc = inject_sources(c, 0, c->d_f.as<float>());
    if (rc) return rc;
    const int64_t nn = (int64_t)c->nmodels * c->nglob;
    accel_kernel<<<grid_for(c->ncomp * nn), kThreads, 0, c->stream>>>(nn, c->ncomp, c->d_minv.as<float>(),
                                                                       c->d_f.as<float>(), c->d_a.as<float>());
    SEMX_HIP(c, hipGetLastError());
    rc = zero_f32(c, c->d_f.as<float>(), len);
    if (rc) return rc;
  }
  int rc = energy_reset(c);
  // the forward run that the adjoint replays starts here
  if (!rc && c->ckpt_every > 0) rc = save_checkpoint(c);
  return rc;
}

int check_finite(semx_ctx* c, bool* ok) {
  if (c->storage == SEMX_F64) return f64_check_finite(c, ok);
  int* flag = scratch_i(c);
  hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "hipMemsetAsync flag");
  const int64_t len = state_len(c);
  finite_kernel<<<grid_for(len, 4096), kThreads, 0, c->stream>>>(len, c->d_u.as<float>(), flag);
  finite_kernel<<<grid_for(len, 4096), kThreads, 0, c->stream>>>(len, c->d_v.as<float>(), flag);
  int h = 0;
  e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "finite check");
  *ok = (h == 0);
  return SEMX_OK;
}

}  // namespace

// One explicit Newmark step (correct the pending step, predict, force,
// sources; optionally record receivers).  Leaves f = -K u + f_src pending.
int step_once(semx_ctx* c, bool record, float* seg_u, float* seg_a, const int64_t* dstep) {
  if (c->storage == SEMX_F64) return f64_step_once(c, record);
  const int64_t nn = (int64_t)c->nmodels * c->nglob;
  const float dt = (float)c->dt;
  float *u = c->d_u.as<float>(), *v = c->d_v.as<float>(), *a = c->d_a.as<float>(), *f = c->d_f.as<float>();
  const float* minv = c->d_minv.as<float>();
  const bool track = c->track_energy;
  c->track_energy = false;
  // a tracked step keeps f^n through the Newmark pass for the potential term;
  // without a pending force (first step after a reset or a new state) -K u^n
  // is computed into the work vector
  const bool keep = force_overwrites(c) || track;
  const float* f_pe = f;
  if (track && !c->pending_correct) {
    int rc = force_into(c, u, c->d_work.as<float>(), false);
    if (rc) return rc;
    f_pe = c->d_work.as<float>();
  }
  const unsigned gb = grid_for(c->ncomp * nn, 1 << 30);  // one pass per lane (streams faster than grid-stride)
  if (c->pending_correct) {
    if (keep) launch_newmark<kCorrect | kPredict | kKeepF>(c, nn, gb, dt, minv, u, v, a, f, seg_u, seg_a);
    else launch_newmark<kCorrect | kPredict>(c, nn, gb, dt, minv, u, v, a, f, seg_u, seg_a);
  } else {
    if (keep) launch_newmark<kPredict | kKeepF>(c, nn, gb, dt, minv, u, v, a, f, seg_u, nullptr);
    else launch_newmark<kPredict>(c, nn, gb, dt, minv, u, v, a, f, seg_u, nullptr);
  }
  SEMX_HIP(c, hipGetLastError());
  const bool src_in_f = c->pending_correct;
  if (track) {
    int rc = energy_track(c, f_pe, src_in_f);
    if (rc) return rc;
  }
  // source work and receivers read u^{n+1}, which the force pass leaves
  // alone; with prestores() the same launch stores f_src^{n+1} into f
  const bool pre = prestores(c);
  int rc = pre && c->first_tl_dirty ? build_first_tl(c) : SEMX_OK;
  if (!rc) rc = step_aux(c, c->it, track && src_in_f, record, dstep, pre);
  if (rc) return rc;
  // f is zero here only if the Newmark pass cleared it (untracked step on a
  // mesh the force pass does not overwrite)
  rc = force_into(c, u, f, !track && !force_overwrites(c), pre);
  if (!rc && !pre) rc = inject_sources(c, c->it + 1, f, dstep);
  if (rc) return rc;
  if (dstep) {
    step_incr_kernel<<<1, 1, 0, c->stream>>>(const_cast<int64_t*>(dstep));
    SEMX_HIP(c, hipGetLastError());
  }
  c->it++;
  c->pending_correct = true;
  if (track) c->energy_it = c->it;
  return SEMX_OK;
}

int apply_force_accumulate(semx_ctx* c, const float* u, float* f) { return force_accumulate(c, u, f); }
int fill_zero(semx_ctx* c, float* p, int64_t n) { return zero_f32(c, p, n); }
int complete_step(semx_ctx* c, float* seg_a) { return finalize_state(c, seg_a); }
// Point sources with the time function given in FP32 (stf32) or FP64
// (stf64); both precisions are kept on the device for the two storage modes.
int set_sources_impl(semx_ctx* c, int nsrc, const int32_t* elem, const double* xi, const double* dir,
                     int64_t nstf, const float* stf32, const double* stf64) {
  if (!c) return SEMX_EINVAL;
  if (!c->have_mesh) return fail(c, SEMX_ESTATE, "set_sources: no mesh");
  if (nsrc < 0) return fail(c, SEMX_EINVAL, "set_sources: nsrc < 0");
  if (nsrc == 0) {
    c->src.nsrc = 0;
    c->src.nsn = 0;
    c->h_src_nodes.clear();
    c->first_tl_dirty = true;
    c->run_gen++;
    c->ckpt_count = 0;
    return c->have_model && c->d_u.p ? energy_reset(c) : SEMX_OK;
  }
  const int nc = c->ncomp;
  if (!elem || !xi || (nc == 3 && !dir) || (!stf32 && !stf64) || nstf <= 0)
    return fail(c, SEMX_EINVAL, "set_sources: bad arguments");
  const int n = c->n, n3 = c->n3;
  std::vector<int32_t> nodes((size_t)nsrc * n3);
  std::vector<float> wdir((size_t)nsrc * n3 * nc);
  std::vector<double> wdir64((size_t)nsrc * n3 * nc);
  for (int s = 0; s < nsrc; ++s) {
    if (elem[s] < 0 || elem[s] >= c->nspec) return fail(c, SEMX_EINVAL, "set_sources: element out of range");
    for (int d = 0; d < 3; ++d)
      if (!(xi[3 * s + d] >= -1.0 && xi[3 * s + d] <= 1.0))
        return fail(c, SEMX_EINVAL, "set_sources: reference coordinate outside [-1, 1]");
    double lx[kMaxN], ly[kMaxN], lz[kMaxN];
    lagrange_at(n, c->xi, xi[3 * s + 0], lx);
    lagrange_at(n, c->xi, xi[3 * s + 1], ly);
    lagrange_at(n, c->xi, xi[3 * s + 2], lz);
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          const int q = i + n * (j + n * k);
          nodes[(size_t)s * n3 + q] = c->h_ibool[(size_t)elem[s] * n3 + q];
          const double wq = lx[i] * ly[j] * lz[k];
          for (int d = 0; d < nc; ++d) {
            const double v = nc == 3 ? wq * dir[3 * s + d] : wq;  // acoustic: no direction
            wdir64[((size_t)s * n3 + q) * nc + d] = v;
            wdir[((size_t)s * n3 + q) * nc + d] = (float)v;
          }
        }
  }
  const size_t ns = (size_t)nsrc * nstf;
  std::vector<float> s32(ns);
  std::vector<double> s64(ns);
  for (size_t t = 0; t < ns; ++t) {
    s64[t] = stf64 ? stf64[t] : (double)stf32[t];
    s32[t] = stf32 ? stf32[t] : (float)stf64[t];
  }
  // points that carry a nonzero weight (a source on a node has one per element)
  std::vector<int32_t> pts;
  for (size_t p = 0; p < (size_t)nsrc * n3; ++p) {
    bool nz = false;
    for (int d = 0; d < nc; ++d) nz |= wdir64[p * nc + d] != 0.0;
    if (nz) pts.push_back((int32_t)p);
  }
  if (pts.empty()) pts.push_back(0);
  // the nodes that receive a source force in FP32, each with its (source,
  // point) pairs in order: the injection's per-node sums
  std::vector<std::pair<int32_t, int32_t>> np_pairs;  // (node, s n3 + q)
  for (size_t p = 0; p < (size_t)nsrc * n3; ++p) {
    bool nz = false;
    for (int d = 0; d < nc; ++d) nz |= wdir[p * nc + d] != 0.0f;
    if (nz) np_pairs.push_back({nodes[p], (int32_t)p});
  }
  std::sort(np_pairs.begin(), np_pairs.end());
  std::vector<int32_t> sptr(1, 0), sidx, snode;
  for (size_t k = 0; k < np_pairs.size(); ++k) {
    if (k > 0 && np_pairs[k].first != np_pairs[k - 1].first) sptr.push_back((int32_t)k);
    if (k == 0 || np_pairs[k].first != np_pairs[k - 1].first) snode.push_back(np_pairs[k].first);
    sidx.push_back(np_pairs[k].second);
  }
  c->h_src_nodes = snode;
  c->first_tl_dirty = true;
  sptr.push_back((int32_t)np_pairs.size());
  if (sidx.empty()) sidx.push_back(0);
  int rc = dev_alloc(c, c->src.nodes, nodes.size() * sizeof(int32_t));
  if (!rc) rc = dev_alloc(c, c->src.snode, sizeof(int32_t) * std::max<size_t>(1, snode.size()));
  if (!rc) rc = dev_alloc(c, c->src.sptr, sizeof(int32_t) * sptr.size());
  if (!rc) rc = dev_alloc(c, c->src.sidx, sizeof(int32_t) * sidx.size());
  if (!rc) rc = dev_alloc(c, c->src.pts, pts.size() * sizeof(int32_t));
  if (!rc) rc = dev_alloc(c, c->src.wdir, wdir.size() * sizeof(float));
  if (!rc) rc = dev_alloc(c, c->src.stf, sizeof(float) * ns);
  if (!rc) rc = dev_alloc(c, c->src.wdir64, wdir64.size() * sizeof(double));
  if (!rc) rc = dev_alloc(c, c->src.stf64, sizeof(double) * ns);
  if (rc) return rc;
  SEMX_HIP(c, hipMemcpy(c->src.nodes.p, nodes.data(), nodes.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  if (!snode.empty())
    SEMX_HIP(c, hipMemcpy(c->src.snode.p, snode.data(), sizeof(int32_t) * snode.size(), hipMemcpyHostToDevice));
  SEMX_HIP(c, hipMemcpy(c->src.sptr.p, sptr.data(), sizeof(int32_t) * sptr.size(), hipMemcpyHostToDevice));
  SEMX_HIP(c, hipMemcpy(c->src.sidx.p, sidx.data(), sizeof(int32_t) * sidx.size(), hipMemcpyHostToDevice));
  c->src.nsn = (int)snode.size();
  SEMX_HIP(c, hipMemcpy(c->src.pts.p, pts.data(), pts.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  c->src.npts = (int)pts.size();
  SEMX_HIP(c, hipMemcpy(c->src.wdir.p, wdir.data(), wdir.size() * sizeof(float), hipMemcpyHostToDevice));
  SEMX_HIP(c, hipMemcpy(c->src.stf.p, s32.data(), sizeof(float) * ns, hipMemcpyHostToDevice));
  SEMX_HIP(c, hipMemcpy(c->src.wdir64.p, wdir64.data(), wdir64.size() * sizeof(double), hipMemcpyHostToDevice));
  SEMX_HIP(c, hipMemcpy(c->src.stf64.p, s64.data(), sizeof(double) * ns, hipMemcpyHostToDevice));
  c->src.nsrc = nsrc;
  c->src.nstf = nstf;
  c->run_gen++;  // checkpoints of a run with other sources are not replayable
  c->ckpt_count = 0;
  // the source work restarts with the new source set
  return c->have_model && c->d_u.p ? energy_reset(c) : SEMX_OK;
}

unsigned grid_1d(int64_t n, int cap) { return grid_for(n, cap); }

}  // namespace semx

using namespace semx;

extern "C" {

int semx_create(semx_ctx** out, int ngll, void* hip_stream) {
  if (!out) return SEMX_EINVAL;
  *out = nullptr;
  if (ngll < 2 || ngll > kMaxN) return SEMX_EINVAL;
  semx_ctx* c = new semx_ctx();
  c->n = ngll;
  c->n3 = ngll * ngll * ngll;
  c->stream = static_cast<hipStream_t>(hip_stream);
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess) {
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, c->device);
    if (e == hipSuccess) c->num_cu = prop.multiProcessorCount;
  }
  if (e != hipSuccess) {
    delete c;
    return SEMX_EHIP;
  }
  gll_nodes_weights(ngll, c->xi, c->w);
  deriv_matrix(ngll, c->xi, c->D);
  std::vector<float> Df(c->D.begin(), c->D.end());
  int rc = dev_alloc(c, c->d_D, Df.size() * sizeof(float));
  if (!rc) rc = dev_alloc(c, c->d_xi64, ngll * sizeof(double));
  if (!rc) rc = dev_alloc(c, c->d_w64, ngll * sizeof(double));
  if (!rc) rc = dev_alloc(c, c->d_xi32, ngll * sizeof(float));
  if (!rc) rc = dev_alloc(c, c->d_scratch, 8 * sizeof(double) + 64);
  if (rc) {
    semx_destroy(c);
    return rc;
  }
  e = hipMemcpy(c->d_D.p, Df.data(), Df.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->d_xi64.p, c->xi.data(), ngll * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->d_w64.p, c->w.data(), ngll * sizeof(double), hipMemcpyHostToDevice);
  std::vector<float> xi32(c->xi.begin(), c->xi.end());
  if (e == hipSuccess) e = hipMemcpy(c->d_xi32.p, xi32.data(), ngll * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    semx_destroy(c);
    return SEMX_EHIP;
  }
  *out = c;
  return SEMX_OK;
}

int semx_destroy(semx_ctx* c) {
  if (!c) return SEMX_OK;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  for (hipEvent_t ev : c->ev_pool) (void)hipEventDestroy(ev);
  for (DevBuf& b : c->ckpts) dev_free(b);
  for (DevBuf* b : {&c->d_bpos, &c->d_baff, &c->d_bfirst, &c->d_step, &c->d_first_tl, &c->d_bfirst_tl}) dev_free(*b);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  c->cap_stream = nullptr;
  for (DevBuf* b : {&c->d_D, &c->d_Dh, &c->d_xi64, &c->d_w64, &c->d_ibool, &c->d_vert, &c->d_elem_vert,
                    &c->d_gam_pt, &c->d_gam_el, &c->d_tri, &c->d_xi32, &c->d_wdet, &c->d_order, &c->d_mat, &c->d_minv,
                    &c->d_mass64, &c->d_wrho, &c->d_u, &c->d_v, &c->d_a, &c->d_f, &c->d_work, &c->d_scratch,
                    &c->src.nodes, &c->src.wdir, &c->src.stf, &c->src.pts, &c->src.snode, &c->src.sptr,
                    &c->src.sidx, &c->rec.nodes, &c->rec.wts,
                    &c->rec.seis,
                    &c->src.wdir64, &c->src.stf64, &c->rec.wts64, &c->rec.seis64, &c->d_gam64, &c->d_mat64,
                    &c->d_minv64, &c->d_D64,
                    &c->d_first, &c->d_aff})
    dev_free(*b);
  delete c;
  return SEMX_OK;
}

const char* semx_last_error(const semx_ctx* c) { return c ? c->err.c_str() : "null context"; }

int semx_upload_mesh(semx_ctx* c, int64_t nspec, int64_t nglob, const int32_t* ibool, int64_t nvert,
                     const double* vert_xyz, const int32_t* elem_vert) {
  if (!c) return SEMX_EINVAL;
  c->err.clear();
  if (nspec <= 0 || nglob <= 0 || nvert <= 0 || !ibool || !vert_xyz || !elem_vert)
    return fail(c, SEMX_EINVAL, "upload_mesh: empty mesh or null array");
  if (nspec * c->n3 >= ((int64_t)1 << 31) || 3 * nglob >= ((int64_t)1 << 31))
    return fail(c, SEMX_EINVAL, "upload_mesh: mesh exceeds 2^31 element-local points or 2^31/3 nodes");
  const int n = c->n, n3 = c->n3;
  for (int64_t t = 0; t < nspec * n3; ++t)
    if (ibool[t] < 0 || ibool[t] >= nglob)
      return fail(c, SEMX_EINVAL, "upload_mesh: ibool entry outside [0, nglob)");
  for (int64_t t = 0; t < nspec * 8; ++t)
    if (elem_vert[t] < 0 || elem_vert[t] >= nvert)
      return fail(c, SEMX_EINVAL, "upload_mesh: elem_vert entry outside [0, nvert)");
  for (int64_t t = 0; t < 3 * nvert; ++t)
    if (!std::isfinite(vert_xyz[t])) return fail(c, SEMX_EINVAL, "upload_mesh: non-finite vertex coordinate");
  int rc = set_device(c);
  if (rc) return rc;
  c->have_mesh = c->have_model = false;
  // sources and receivers live in elements of the previous mesh
  c->src.nsrc = 0;
  c->src.nsn = 0;
  c->h_src_nodes.clear();
  c->rec.nrec = 0;
  c->nspec = nspec;
  c->nglob = nglob;
  c->nvert = nvert;
  c->h_ibool.assign(ibool, ibool + nspec * n3);
  c->h_elem_vert.assign(elem_vert, elem_vert + nspec * 8);
  c->h_vert.assign(vert_xyz, vert_xyz + 3 * nvert);

  // regular (affine) elements: x_v - x_0 = a e1 + b e2 + c e3 for corner v = a + 2b + 4c
  c->h_regular.assign(nspec, 0);
  c->nregular = 0;
  std::vector<float> gam_el(9 * nspec, 0.0f);
  for (int64_t e = 0; e < nspec; ++e) {
    const double* x0 = vert_xyz + 3 * (int64_t)elem_vert[8 * e];
    double E[3][3];
    double scale = 0.0;
    for (int d = 0; d < 3; ++d) {
      const double* xd = vert_xyz + 3 * (int64_t)elem_vert[8 * e + (1 << d)];
      for (int a = 0; a < 3; ++a) {
        E[a][d] = xd[a] - x0[a];
        scale = std::max(scale, std::fabs(E[a][d]));
      }
    }
    bool affine = true;
    for (int v = 0; v < 8 && affine; ++v) {
      const double* xv = vert_xyz + 3 * (int64_t)elem_vert[8 * e + v];
      for (int a = 0; a < 3; ++a) {
        const double pred = x0[a] + ((v & 1) ? E[a][0] : 0.0) + ((v & 2) ? E[a][1] : 0.0) + ((v & 4) ? E[a][2] : 0.0);
        if (std::fabs(xv[a] - pred) > 1e-12 * scale) affine = false;
      }
    }
    if (!affine) continue;
    // J = E/2 (reference cube has side 2); Gamma = J^{-1}
    double J[3][3];
    for (int a = 0; a < 3; ++a)
      for (int d = 0; d < 3; ++d) J[a][d] = 0.5 * E[a][d];
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (!(det > 0.0)) continue;  // left to the device check, which reports it
    double G[3][3];
    G[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    G[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    G[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    G[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    G[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    G[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    G[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    G[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    G[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    for (int d = 0; d < 3; ++d)
      for (int b = 0; b < 3; ++b) gam_el[9 * e + 3 * d + b] = (float)G[d][b];
    c->h_regular[e] = 1;
    c->nregular++;
  }
  c->nirregular = nspec - c->nregular;

  c->h_gam_el = std::move(gam_el);
  rc = dev_alloc(c, c->d_vert, sizeof(double) * 3 * nvert);
  if (!rc) rc = dev_alloc(c, c->d_elem_vert, sizeof(int32_t) * 8 * nspec);
  if (rc) return rc;
  SEMX_HIP(c, hipMemcpy(c->d_vert.p, vert_xyz, sizeof(double) * 3 * nvert, hipMemcpyHostToDevice));
  SEMX_HIP(c, hipMemcpy(c->d_elem_vert.p, elem_vert, sizeof(int32_t) * 8 * nspec, hipMemcpyHostToDevice));
  unsigned long long* hmin_bits = reinterpret_cast<unsigned long long*>(scratch_d(c));
  const unsigned long long big = 0x7FEFFFFFFFFFFFFFull;
  SEMX_HIP(c, hipMemcpyAsync(hmin_bits, &big, sizeof(big), hipMemcpyHostToDevice, c->stream));
  spacing_kernel<<<grid_for(nspec * n3, 4096), kThreads, 0, c->stream>>>(
      n, nspec, c->d_vert.as<double>(), c->d_elem_vert.as<int32_t>(), c->d_xi64.as<double>(), hmin_bits);
  SEMX_HIP(c, hipGetLastError());
  unsigned long long hbits = 0;
  SEMX_HIP(c, hipMemcpyAsync(&hbits, hmin_bits, sizeof(hbits), hipMemcpyDeviceToHost, c->stream));
  SEMX_HIP(c, hipStreamSynchronize(c->stream));
  std::memcpy(&c->hmin, &hbits, sizeof(double));

  // colouring: corners first, full-node conflicts if that is not valid
  std::vector<int32_t> color;
  greedy_color(n, nspec, nglob, ibool, true, color);
  auto to_lists = [&](const std::vector<int32_t>& col) {
    int nc = 0;
    for (auto v : col) nc = std::max(nc, v + 1);
    c->ncolors = nc;
    c->color_ptr.assign(nc + 1, 0);
    for (auto v : col) c->color_ptr[v + 1]++;
    for (int k = 0; k < nc; ++k) c->color_ptr[k + 1] += c->color_ptr[k];
    c->elem_order.assign(nspec, 0);
    std::vector<int32_t> pos(c->color_ptr.begin(), c->color_ptr.end() - 1);
    for (int64_t e = 0; e < nspec; ++e) c->elem_order[pos[col[e]]++] = (int32_t)e;
  };
  to_lists(color);
  if (!coloring_valid(n3, nspec, nglob, ibool, c->ncolors, c->color_ptr.data(), c->elem_order.data())) {
    greedy_color(n, nspec, nglob, ibool, false, color);
    to_lists(color);
    if (!coloring_valid(n3, nspec, nglob, ibool, c->ncolors, c->color_ptr.data(), c->elem_order.data())) {
      // an element repeats a node (e.g. a periodic mesh one element wide): only atomics are exact
      c->ncolors = 0;
      c->assembly = SEMX_ASM_ATOMIC;
    }
  }
  rc = build_layout(c);
  if (rc) return rc;
  c->have_mesh = true;
  return SEMX_OK;
}

int semx_set_coloring(semx_ctx* c, int ncolors, const int32_t* color_ptr, const int32_t* elem_order) {
  if (!c) return SEMX_EINVAL;
  if (!c->have_mesh) return fail(c, SEMX_ESTATE, "set_coloring: no mesh");
  if (ncolors <= 0 || !color_ptr || !elem_order) return fail(c, SEMX_EINVAL, "set_coloring: bad arguments");
  if (color_ptr[0] != 0 || color_ptr[ncolors] != c->nspec)
    return fail(c, SEMX_EINVAL, "set_coloring: color_ptr must run from 0 to nspec");
  for (int k = 0; k < ncolors; ++k)
    if (color_ptr[k + 1] < color_ptr[k]) return fail(c, SEMX_EINVAL, "set_coloring: color_ptr decreasing");
  std::vector<char> seen(c->nspec, 0);
  for (int64_t t = 0; t < c->nspec; ++t) {
    const int32_t e = elem_order[t];
    if (e < 0 || e >= c->nspec || seen[e]) return fail(c, SEMX_EINVAL, "set_coloring: not a permutation");
    seen[e] = 1;
  }
  if (!coloring_valid(c->n3, c->nspec, c->nglob, c->h_ibool.data(), ncolors, color_ptr, elem_order))
    return fail(c, SEMX_EINVAL, "set_coloring: two elements of a colour share a node");
  c->ncolors = ncolors;
  c->color_ptr.assign(color_ptr, color_ptr + ncolors + 1);
  c->elem_order.assign(elem_order, elem_order + c->nspec);
  // the device layout follows the colouring: rebuild it; the model must be uploaded again
  c->have_model = false;
  return build_layout(c);
}

int semx_get_coloring(semx_ctx* c, int* ncolors, int32_t* color_ptr, int32_t* elem_order) {
  if (!c) return SEMX_EINVAL;
  if (!c->have_mesh) return fail(c, SEMX_ESTATE, "get_coloring: no mesh");
  if (ncolors) *ncolors = c->ncolors;
  if (color_ptr && c->ncolors) std::copy(c->color_ptr.begin(), c->color_ptr.end(), color_ptr);
  if (elem_order && c->ncolors) std::copy(c->elem_order.begin(), c->elem_order.end(), elem_order);
  return SEMX_OK;
}

int semx_mesh_info(semx_ctx* c, int64_t* nregular, int64_t* nirregular, int* ncolors) {
  if (!c) return SEMX_EINVAL;
  if (!c->have_mesh) return fail(c, SEMX_ESTATE, "mesh_info: no mesh");
  if (nregular) *nregular = c->nregular;
  if (nirregular) *nirregular = c->nirregular;
  if (ncolors) *ncolors = c->ncolors;
  return SEMX_OK;
}

namespace {

// Shared part of the model uploads: per-point force weights wl, wm (lambda,
// mu for the elastic operator; 1/rho, 0 for the acoustic one, whose force
// kernels read only the first), and the mass density md (rho; 1/kappa).
int upload_model_impl(semx_ctx* c, int nmodels, const double* lambda, const double* mu, const double* rho,
                      double vpmax) {
  const int64_t npt = (int64_t)nmodels * c->nspec * c->n3;
  int rc = set_device(c);
  if (rc) return rc;
  c->have_model = false;
  c->nmodels = nmodels;
  c->vp_max = vpmax;
  DevBuf dl, dm, dr;
  rc = dev_alloc(c, dl, sizeof(double) * npt);
  if (!rc) rc = dev_alloc(c, dm, sizeof(double) * npt);
  if (!rc) rc = dev_alloc(c, dr, sizeof(double) * npt);
  if (!rc) rc = dev_alloc(c, c->d_mat, sizeof(float) * 2 * npt);
  if (!rc) rc = dev_alloc(c, c->d_wrho, sizeof(float) * npt);
  if (!rc) rc = dev_alloc(c, c->d_mass64, sizeof(double) * nmodels * c->nglob);
  if (!rc) rc = dev_alloc(c, c->d_minv, sizeof(float) * nmodels * c->nglob);
  const int64_t len = c->ncomp * (int64_t)nmodels * c->nglob;
  const size_t es = c->storage == SEMX_F64 ? sizeof(double) : sizeof(float);
  if (!rc) rc = dev_alloc(c, c->d_u, es * len);
  if (!rc) rc = dev_alloc(c, c->d_v, es * len);
  if (!rc) rc = dev_alloc(c, c->d_a, es * len);
  if (!rc) rc = dev_alloc(c, c->d_f, es * len);
  if (!rc) rc = dev_alloc(c, c->d_work, es * len);
  if (!rc && c->storage == SEMX_F64) rc = dev_alloc(c, c->d_gam64, sizeof(double) * 9 * c->nspec * c->n3);
  if (!rc && c->storage != SEMX_F64)
    for (DevBuf* b : {&c->d_gam64, &c->d_mat64, &c->d_minv64}) dev_free(*b);
  auto cleanup = [&]() { dev_free(dl); dev_free(dm); dev_free(dr); };
  if (rc) { cleanup(); return rc; }
  hipError_t e = hipMemcpy(dl.p, lambda, sizeof(double) * npt, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dm.p, mu, sizeof(double) * npt, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dr.p, rho, sizeof(double) * npt, hipMemcpyHostToDevice);
  if (e != hipSuccess) { cleanup(); return hip_fail(c, e, "upload_model copies"); }
  material_kernel<<<grid_for(npt, 8192), kThreads, 0, c->stream>>>(
      c->n3, c->nspec, nmodels, c->d_order.as<int32_t>(), dl.as<double>(), dm.as<double>(), dr.as<double>(),
      c->d_wdet.as<double>(), c->d_mat.as<float>(), c->d_wrho.as<float>());
  fill_f64<<<grid_for(nmodels * c->nglob), kThreads, 0, c->stream>>>(c->d_mass64.as<double>(),
                                                                     nmodels * c->nglob, 0.0);
  // deterministic mass assembly, one coloured launch range at a time
  if (c->ncolors > 0) {
    for (const auto& L : c->colored_launches)
      mass_color_kernel<<<grid_for((int64_t)nmodels * L.count * c->n3, 8192), kThreads, 0, c->stream>>>(
          c->n3, c->nspec, c->nglob, nmodels, L.pos0, L.count, c->d_order.as<int32_t>(),
          c->d_ibool.as<int32_t>(), dr.as<double>(), c->d_wdet.as<double>(), c->d_mass64.as<double>());
  } else {
    // no valid colouring (an element repeats a node): one thread walks the
    // positions in order, which keeps the sum deterministic (tiny meshes only)
    mass_serial_kernel<<<1, 1, 0, c->stream>>>(c->n3, c->nspec, c->nglob, nmodels, c->d_order.as<int32_t>(),
                                               c->d_ibool.as<int32_t>(), dr.as<double>(), c->d_wdet.as<double>(),
                                               c->d_mass64.as<double>());
  }
  minv_kernel<<<grid_for(nmodels * c->nglob), kThreads, 0, c->stream>>>(nmodels * c->nglob,
                                                                        c->d_mass64.as<double>(),
                                                                        c->d_minv.as<float>());
  e = hipGetLastError();
  if (e == hipSuccess && c->storage == SEMX_F64) {
    // FP64 Gamma by launch position (the same map; W is recomputed bitwise equal)
    geom_kernel<<<grid_for(c->nspec * c->n3, 8192), kThreads, 0, c->stream>>>(
        c->n, c->nspec, c->d_vert.as<double>(), c->d_elem_vert.as<int32_t>(), c->d_order.as<int32_t>(),
        c->d_xi64.as<double>(), c->d_w64.as<double>(), nullptr, c->d_wdet.as<double>(), scratch_i(c),
        c->d_gam64.as<double>());
    e = hipGetLastError();
    if (e == hipSuccess) rc = f64_model_setup(c, dl.as<double>(), dm.as<double>());
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  cleanup();
  if (e != hipSuccess) return hip_fail(c, e, "upload_model kernels");
  if (rc) return rc;
  c->have_model = true;
  c->lambda_max = 0.0;
  // receivers depend on nmodels
  if (c->rec.nrec > 0) {
    rc = alloc_seismograms(c);
    if (rc) return rc;
  }
  return do_reset(c);
}

}  // namespace

int semx_upload_model(semx_ctx* c, int nmodels, const double* lambda, const double* mu, const double* rho) {
  if (!c) return SEMX_EINVAL;
  c->err.clear();
  if (!c->have_mesh) return fail(c, SEMX_ESTATE, "upload_model: no mesh");
  if (c->physics != SEMX_ELASTIC)
    return fail(c, SEMX_ESTATE, "upload_model: acoustic physics; use semx_upload_model_acoustic");
  if (nmodels <= 0 || !lambda || !mu || !rho) return fail(c, SEMX_EINVAL, "upload_model: bad arguments");
  const int64_t npt = (int64_t)nmodels * c->nspec * c->n3;
  if (npt >= ((int64_t)1 << 31) || 3 * (int64_t)nmodels * c->nglob >= ((int64_t)1 << 31))
    return fail(c, SEMX_EINVAL, "upload_model: batch too large");
  double vpmax = 0.0;
  for (int64_t t = 0; t < npt; ++t) {
    const double l = lambda[t], m = mu[t], r = rho[t];
    if (!(r > 0.0) || !(m > 0.0) || !(l + 2.0 * m / 3.0 > 0.0) || !std::isfinite(l) || !std::isfinite(m) ||
        !std::isfinite(r))
      return fail(c, SEMX_EINVAL, "upload_model: need rho > 0, mu > 0, lambda + 2 mu/3 > 0");
    vpmax = std::max(vpmax, std::sqrt((l + 2.0 * m) / r));
  }
  return upload_model_impl(c, nmodels, lambda, mu, rho, vpmax);
}

int semx_upload_model_acoustic(semx_ctx* c, int nmodels, const double* kappa, const double* rho) {
  if (!c) return SEMX_EINVAL;
  c->err.clear();
  if (!c->have_mesh) return fail(c, SEMX_ESTATE, "upload_model_acoustic: no mesh");
  if (c->physics != SEMX_ACOUSTIC)
    return fail(c, SEMX_ESTATE, "upload_model_acoustic: elastic physics; call semx_set_physics first");
  if (nmodels <= 0 || !kappa || !rho) return fail(c, SEMX_EINVAL, "upload_model_acoustic: bad arguments");
  const int64_t npt = (int64_t)nmodels * c->nspec * c->n3;
  if (npt >= ((int64_t)1 << 31) || (int64_t)nmodels * c->nglob >= ((int64_t)1 << 31))
    return fail(c, SEMX_EINVAL, "upload_model_acoustic: batch too large");
  std::vector<double> wl((size_t)npt), wm((size_t)npt, 0.0), md((size_t)npt);
  double vpmax = 0.0;
  for (int64_t t = 0; t < npt; ++t) {
    const double k = kappa[t], r = rho[t];
    if (!(r > 0.0) || !(k > 0.0) || !std::isfinite(k) || !std::isfinite(r))
      return fail(c, SEMX_EINVAL, "upload_model_acoustic: need kappa > 0, rho > 0");
    wl[t] = 1.0 / r;
    md[t] = 1.0 / k;
    vpmax = std::max(vpmax, std::sqrt(k / r));
  }
  return upload_model_impl(c, nmodels, wl.data(), wm.data(), md.data(), vpmax);
}

int semx_set_physics(semx_ctx* c, int physics) {
  if (!c) return SEMX_EINVAL;
  if (physics != SEMX_ELASTIC && physics != SEMX_ACOUSTIC) return fail(c, SEMX_EINVAL, "set_physics: unknown physics");
  if (c->have_model) return fail(c, SEMX_ESTATE, "set_physics: call before uploading a model");
  // the source weights are stored per field component
  if (c->src.nsrc > 0 && physics != c->physics)
    return fail(c, SEMX_ESTATE, "set_physics: call before semx_set_sources");
  if (physics == SEMX_ACOUSTIC) {
    if (c->storage != SEMX_F32) return fail(c, SEMX_EINVAL, "set_physics: acoustic physics runs in FP32 storage");
    if (c->contraction != SEMX_C_F32)
      return fail(c, SEMX_EINVAL, "set_physics: acoustic physics needs the SEMX_C_F32 contraction setting");
    if (c->ckpt_every > 0) return fail(c, SEMX_ESTATE, "set_physics: turn checkpointing off first");
  }
  c->physics = physics;
  c->ncomp = physics == SEMX_ACOUSTIC ? 1 : 3;
  if (c->rec.nrec > 0) return alloc_seismograms(c);
  return SEMX_OK;
}

int semx_gll(int ngll, double* xi, double* w) {
  if (ngll < 2 || ngll > kMaxN || !xi || !w) return SEMX_EINVAL;
  std::vector<double> x, ww;
  gll_nodes_weights(ngll, x, ww);
  for (int a = 0; a < ngll; ++a) {
    xi[a] = x[a];
    w[a] = ww[a];
  }
  return SEMX_OK;
}

int semx_set_mode(semx_ctx* c, int contraction, int assembly) {
  if (!c) return SEMX_EINVAL;
  if (contraction != SEMX_C_F32 && contraction != SEMX_C_BF16 && contraction != SEMX_C_F16 &&
      contraction != SEMX_C_MFMA_F32)
    return fail(c, SEMX_EINVAL, "set_mode: unknown contraction");
  if (assembly != SEMX_ASM_COLORED && assembly != SEMX_ASM_ATOMIC)
    return fail(c, SEMX_EINVAL, "set_mode: unknown assembly");
  if (contraction != SEMX_C_F32 && !mfma_supported(c->n, contraction))
    return fail(c, SEMX_EINVAL, "set_mode: MFMA contractions need 4 <= NGLL <= 8 or 11 <= NGLL <= 16");
  if (contraction != SEMX_C_F32 && c->storage == SEMX_F64)
    return fail(c, SEMX_EINVAL, "set_mode: FP64 storage contracts on the vector units (SEMX_C_F32 only)");
  if (contraction != SEMX_C_F32 && c->physics == SEMX_ACOUSTIC)
    return fail(c, SEMX_EINVAL, "set_mode: the acoustic operator contracts on the vector units (SEMX_C_F32 only)");
  if (assembly == SEMX_ASM_COLORED && c->have_mesh && c->ncolors == 0)
    return fail(c, SEMX_EINVAL, "set_mode: mesh has elements with repeated nodes; only atomic assembly is exact");
  c->contraction = contraction;
  c->assembly = assembly;
  return SEMX_OK;
}

int semx_apply_force(semx_ctx* c, const float* u_dev, float* f_dev) {
  if (!c) return SEMX_EINVAL;
  if (!c->have_mesh || !c->have_model) return fail(c, SEMX_ESTATE, "apply_force: mesh and model required");
  if (c->storage == SEMX_F64) return fail(c, SEMX_ESTATE, "apply_force: FP64 storage; use semx_apply_force_f64");
  if (!u_dev || !f_dev) return fail(c, SEMX_EINVAL, "apply_force: null pointer");
  const int64_t len = state_len(c);
  if (u_dev < f_dev + len && f_dev < u_dev + len) return fail(c, SEMX_EINVAL, "apply_force: u and f overlap");
  return force_into(c, u_dev, f_dev, false);
}

int semx_force_skeleton(semx_ctx* c, const float* u_dev, float* f_dev, int reps, double* ms_per_pass) {
  if (!c || !ms_per_pass) return SEMX_EINVAL;
  if (!c->have_mesh || !c->have_model) return fail(c, SEMX_ESTATE, "force_skeleton: mesh and model required");
  if (c->storage != SEMX_F32 || c->physics != SEMX_ELASTIC || c->contraction != SEMX_C_F32 ||
      c->assembly != SEMX_ASM_COLORED)
    return fail(c, SEMX_ESTATE, "force_skeleton: covers the FP32 elastic per-element kernels with coloured assembly");
  if (!u_dev || !f_dev || reps <= 0) return fail(c, SEMX_EINVAL, "force_skeleton: null pointer or reps <= 0");
  const int64_t len = state_len(c);
  if (u_dev < f_dev + len && f_dev < u_dev + len) return fail(c, SEMX_EINVAL, "force_skeleton: u and f overlap");
  ForceArgs a = force_args(c, u_dev, f_dev, force_overwrites(c));
  auto pass = [&]() -> hipError_t {
    if (blocks_active(c)) {
      const int geo = c->blocks_irregular ? c->irregular_geo : kRegular;
      for (const auto& L : c->block_launches) {
        const BlockArgs b{c->d_bpos.as<int32_t>(), c->d_baff.as<int32_t>(),
                          force_overwrites(c) ? c->d_bfirst.as<uint32_t>() : nullptr, L.pos0, L.count};
        const hipError_t e = launch_force_block_skeleton(c->n, geo, a, b, c->stream);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    }
    for (const auto& L : c->colored_launches) {
      a.pos0 = L.pos0;
      a.count = L.count;
      const int geo = L.irregular ? c->irregular_geo : kRegular;
      const hipError_t e = c->n > kMaxNLow ? launch_force_high_skeleton(c->n, geo, a, c->stream)
                                           : launch_force_skeleton(c->n, geo, L.naff, a, c->stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = pass();  // warm
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
  for (int k = 0; k < reps && e == hipSuccess; ++k) e = pass();
  if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(c, e, "force_skeleton");
  *ms_per_pass = (double)ms / reps;
  return SEMX_OK;
}



int semx_set_dt(semx_ctx* c, double dt) {
  if (!c) return SEMX_EINVAL;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, SEMX_EINVAL, "set_dt: dt must be positive");
  if (c->lambda_max > 0.0 && dt * std::sqrt(c->lambda_max) >= 2.0)
    return fail(c, SEMX_EUNSTABLE, "set_dt: dt above the stability bound 2/sqrt(lambda_max)");
  c->dt = dt;
  c->have_dt = true;
  return SEMX_OK;
}

int semx_cfl_dt(semx_ctx* c, double courant, double* dt_out) {
  if (!c || !dt_out) return SEMX_EINVAL;
  if (!c->have_mesh || !c->have_model) return fail(c, SEMX_ESTATE, "cfl_dt: mesh and model required");
  if (!(courant > 0.0)) return fail(c, SEMX_EINVAL, "cfl_dt: courant must be positive");
  *dt_out = courant * c->hmin / c->vp_max;
  return SEMX_OK;
}

int semx_max_eigenvalue(semx_ctx* c, int iters, double* lambda_max) {
  if (!c || !lambda_max) return SEMX_EINVAL;
  if (!c->have_mesh || !c->have_model) return fail(c, SEMX_ESTATE, "max_eigenvalue: mesh and model required");
  if (iters <= 0) return fail(c, SEMX_EINVAL, "max_eigenvalue: iters must be positive");
  // power iteration on M^{-1} K for model 0 (nmodels entries are independent)
  const int saved_models = c->nmodels;
  const int64_t n3g = c->ncomp * c->nglob;
  DevBuf x, y;
  int rc = dev_alloc(c, x, sizeof(float) * n3g * saved_models);
  if (!rc) rc = dev_alloc(c, y, sizeof(float) * n3g * saved_models);
  if (rc) { dev_free(x); dev_free(y); return rc; }
  // deterministic pseudo-random start vector (hash of the index)
  std::vector<float> h(n3g * saved_models, 0.0f);
  uint64_t s = 0x9E3779B97F4A7C15ull;
  for (int64_t t = 0; t < n3g; ++t) {
    s ^= s << 13; s ^= s >> 7; s ^= s << 17;
    h[t] = (float)((s >> 11) * (1.0 / 9007199254740992.0) - 0.5);
  }
  hipError_t e = hipMemcpy(x.p, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) { dev_free(x); dev_free(y); return hip_fail(c, e, "power iteration init"); }
  double lam = 0.0;
  for (int k = 0; k < iters && !rc; ++k) {
    rc = force_into(c, x.as<float>(), y.as<float>(), false);  // y = -K x
    if (rc) break;
    fill_f64<<<1, 64, 0, c->stream>>>(scratch_d(c), 8, 0.0);
    // Rayleigh quotient lam = (x^T K x)/(x^T M x) = -(x.y)/(x^T M x)
    dot_kernel<<<grid_for(n3g, 2048), kThreads, 0, c->stream>>>(n3g, x.as<float>(), y.as<float>(), scratch_d(c));
    mnorm_kernel<<<grid_for(n3g, 2048), kThreads, 0, c->stream>>>(c->nglob, c->ncomp, c->d_mass64.as<double>(),
                                                                  x.as<float>(), scratch_d(c) + 1);
    double hd[2];
    e = hipMemcpyAsync(hd, scratch_d(c), 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) { rc = hip_fail(c, e, "power iteration"); break; }
    lam = -hd[0] / hd[1];
    // x <- M^{-1} K x, normalised to unit M-norm scale
    const double nrm = std::sqrt(hd[1]);
    neg_minv_kernel<<<grid_for(n3g), kThreads, 0, c->stream>>>(c->nglob, c->ncomp, c->d_minv.as<float>(),
                                                               y.as<float>(), x.as<float>(),
                                                               (float)(1.0 / (lam * nrm)));
    e = hipGetLastError();
    if (e != hipSuccess) rc = hip_fail(c, e, "power iteration update");
  }
  dev_free(x);
  dev_free(y);
  if (rc) return rc;
  c->lambda_max = lam;
  *lambda_max = lam;
  return SEMX_OK;
}

int semx_set_sources(semx_ctx* c, int nsrc, const int32_t* elem, const double* xi, const double* dir,
                     int64_t nstf, const float* stf) {
  return set_sources_impl(c, nsrc, elem, xi, dir, nstf, stf, nullptr);
}

int semx_set_sources_f64(semx_ctx* c, int nsrc, const int32_t* elem, const double* xi, const double* dir,
                         int64_t nstf, const double* stf) {
  return set_sources_impl(c, nsrc, elem, xi, dir, nstf, nullptr, stf);
}

int semx_set_receivers(semx_ctx* c, int nrec, const int32_t* elem, const double* xi, int64_t nt_max) {
  if (!c) return SEMX_EINVAL;
  if (!c->have_mesh) return fail(c, SEMX_ESTATE, "set_receivers: no mesh");
  if (nrec < 0 || nt_max < 0) return fail(c, SEMX_EINVAL, "set_receivers: negative count");
  if (nrec == 0) {
    c->rec.nrec = 0;
    return SEMX_OK;
  }
  if (!elem || !xi || nt_max == 0) return fail(c, SEMX_EINVAL, "set_receivers: bad arguments");
  const int n = c->n, n3 = c->n3;
  std::vector<int32_t> nodes((size_t)nrec * n3);
  std::vector<float> wts((size_t)nrec * n3);
  std::vector<double> wts64((size_t)nrec * n3);
  for (int r = 0; r < nrec; ++r) {
    if (elem[r] < 0 || elem[r] >= c->nspec) return fail(c, SEMX_EINVAL, "set_receivers: element out of range");
    for (int d = 0; d < 3; ++d)
      if (!(xi[3 * r + d] >= -1.0 && xi[3 * r + d] <= 1.0))
        return fail(c, SEMX_EINVAL, "set_receivers: reference coordinate outside [-1, 1]");
    double lx[kMaxN], ly[kMaxN], lz[kMaxN];
    lagrange_at(n, c->xi, xi[3 * r + 0], lx);
    lagrange_at(n, c->xi, xi[3 * r + 1], ly);
    lagrange_at(n, c->xi, xi[3 * r + 2], lz);
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          const int q = i + n * (j + n * k);
          nodes[(size_t)r * n3 + q] = c->h_ibool[(size_t)elem[r] * n3 + q];
          wts64[(size_t)r * n3 + q] = lx[i] * ly[j] * lz[k];
          wts[(size_t)r * n3 + q] = (float)wts64[(size_t)r * n3 + q];
        }
  }
  int rc = dev_alloc(c, c->rec.nodes, nodes.size() * sizeof(int32_t));
  if (!rc) rc = dev_alloc(c, c->rec.wts, wts.size() * sizeof(float));
  if (!rc) rc = dev_alloc(c, c->rec.wts64, wts64.size() * sizeof(double));
  if (rc) return rc;
  SEMX_HIP(c, hipMemcpy(c->rec.nodes.p, nodes.data(), nodes.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  SEMX_HIP(c, hipMemcpy(c->rec.wts.p, wts.data(), wts.size() * sizeof(float), hipMemcpyHostToDevice));
  SEMX_HIP(c, hipMemcpy(c->rec.wts64.p, wts64.data(), wts64.size() * sizeof(double), hipMemcpyHostToDevice));
  c->rec.nrec = nrec;
  c->rec.nt_max = nt_max;
  return alloc_seismograms(c);
}

int semx_reset(semx_ctx* c) {
  if (!c) return SEMX_EINVAL;
  if (!c->have_mesh || !c->have_model) return fail(c, SEMX_ESTATE, "reset: mesh and model required");
  return do_reset(c);
}

int semx_step(semx_ctx* c, int64_t nsteps) {
  if (!c) return SEMX_EINVAL;
  if (!c->have_mesh || !c->have_model) return fail(c, SEMX_ESTATE, "step: mesh and model required");
  if (!c->have_dt) return fail(c, SEMX_ESTATE, "step: dt not set");
  if (nsteps < 0) return fail(c, SEMX_EINVAL, "step: nsteps < 0");
  // Graph-captured chunks for the untracked middle of a long call: FP32
  // storage, no force timing, no checkpoints, no watchdog; the first step
  // (if no corrector is pending) and the last (energy tracking) run directly.
  const int64_t G = c->graph_chunk;
  if (G > 0 && c->storage == SEMX_F32 && c->timing_stride == 0 && c->ckpt_every == 0 &&
      c->watchdog_every == 0 && nsteps >= 2 * G + 2) {
    int64_t done = 0;
    if (!c->pending_correct) {
      c->track_energy = false;
      int rc = step_once(c, true);
      if (rc) return rc;
      ++done;
    }
    const int64_t nchunks = (nsteps - done - 1) / G;
    if (nchunks >= 2) {
      int rc = run_graph_chunks(c, nchunks, G);
      if (rc) return rc;
      done += nchunks * G;
    }
    for (int64_t s = done; s < nsteps; ++s) {
      c->track_energy = s + 1 == nsteps;
      int rc = step_once(c, true);
      if (rc) return rc;
    }
    return SEMX_OK;
  }
  for (int64_t s = 0; s < nsteps; ++s) {
    // the discrete energy is tracked on the last step of the call and on the
    // watchdog's steps that check it
    const bool wd_step = c->watchdog_every > 0 && (c->it + 1) % c->watchdog_every == 0;
    c->track_energy = s + 1 == nsteps || (wd_step && c->watchdog_emax > 0.0);
    int rc = step_once(c, true);
    if (rc) return rc;
    if (c->ckpt_every > 0 && c->it % c->ckpt_every == 0) {
      rc = save_checkpoint(c);
      if (rc) return rc;
    }
    if (wd_step) {
      bool ok = true;
      rc = check_finite(c, &ok);
      if (rc) return rc;
      if (!ok) return fail(c, SEMX_ENUMERIC, "watchdog: non-finite displacement or velocity at step " + std::to_string(c->it));
      if (c->watchdog_emax > 0.0) {
        double k = 0, p = 0;
        rc = energy_read(c, &k, &p, nullptr);
        if (rc) return rc;
        if (!(k + p <= c->watchdog_emax))
          return fail(c, SEMX_ENUMERIC, "watchdog: discrete energy above the limit at step " + std::to_string(c->it));
      }
    }
  }
  return SEMX_OK;
}

int semx_time_index(semx_ctx* c, int64_t* it) {
  if (!c || !it) return SEMX_EINVAL;
  *it = c->it;
  return SEMX_OK;
}

int semx_read_seismograms(semx_ctx* c, float* out, int out_on_device) {
  if (!c || !out) return SEMX_EINVAL;
  if (c->storage == SEMX_F64) return fail(c, SEMX_ESTATE, "read_seismograms: FP64 storage; use semx_read_seismograms_f64");
  if (c->rec.nrec == 0 || !c->rec.seis.p) return fail(c, SEMX_ESTATE, "read_seismograms: no receivers");
  SEMX_HIP(c, hipMemcpyAsync(out, c->rec.seis.p, c->rec.seis.bytes,
                             out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  if (!out_on_device) SEMX_HIP(c, hipStreamSynchronize(c->stream));
  return SEMX_OK;
}

int semx_get_state(semx_ctx* c, float* u_dev, float* v_dev, float* a_dev, int64_t* it) {
  if (!c) return SEMX_EINVAL;
  if (!c->have_model) return fail(c, SEMX_ESTATE, "get_state: no model");
  if (c->storage == SEMX_F64) return fail(c, SEMX_ESTATE, "get_state: FP64 storage; use semx_get_state_f64");
  int rc = finalize_state(c);
  if (rc) return rc;
  const size_t bytes = sizeof(float) * state_len(c);
  if (u_dev) SEMX_HIP(c, hipMemcpyAsync(u_dev, c->d_u.p, bytes, hipMemcpyDeviceToDevice, c->stream));
  if (v_dev) SEMX_HIP(c, hipMemcpyAsync(v_dev, c->d_v.p, bytes, hipMemcpyDeviceToDevice, c->stream));
  if (a_dev) SEMX_HIP(c, hipMemcpyAsync(a_dev, c->d_a.p, bytes, hipMemcpyDeviceToDevice, c->stream));
  if (it) *it = c->it;
  return SEMX_OK;
}

int semx_set_state(semx_ctx* c, const float* u_dev, const float* v_dev, const float* a_dev, int64_t it) {
  if (!c) return SEMX_EINVAL;
  if (!c->have_model) return fail(c, SEMX_ESTATE, "set_state: no model");
  if (c->storage == SEMX_F64) return fail(c, SEMX_ESTATE, "set_state: FP64 storage; use semx_set_state_f64");
  if (!u_dev || !v_dev || !a_dev || it < 0) return fail(c, SEMX_EINVAL, "set_state: null pointer or negative index");
  const size_t bytes = sizeof(float) * state_len(c);
  SEMX_HIP(c, hipMemcpyAsync(c->d_u.p, u_dev, bytes, hipMemcpyDeviceToDevice, c->stream));
  SEMX_HIP(c, hipMemcpyAsync(c->d_v.p, v_dev, bytes, hipMemcpyDeviceToDevice, c->stream));
  SEMX_HIP(c, hipMemcpyAsync(c->d_a.p, a_dev, bytes, hipMemcpyDeviceToDevice, c->stream));
  int rc = zero_f32(c, c->d_f.as<float>(), state_len(c));
  if (rc) return rc;
  c->it = it;
  c->pending_correct = false;
  c->run_gen++;  // earlier checkpoints belong to another run
  c->ckpt_count = 0;
  return energy_reset(c);
}

int semx_energy(semx_ctx* c, double* kinetic, double* potential, double* source_work) {
  if (!c || !kinetic || !potential) return SEMX_EINVAL;
  if (!c->have_mesh || !c->have_model) return fail(c, SEMX_ESTATE, "energy: mesh and model required");
  return energy_read(c, kinetic, potential, source_work);
}

int semx_set_watchdog(semx_ctx* c, int64_t interval, double max_energy) {
  if (!c) return SEMX_EINVAL;
  if (interval < 0) return fail(c, SEMX_EINVAL, "set_watchdog: negative interval");
  c->watchdog_every = interval;
  c->watchdog_emax = max_energy;
  return SEMX_OK;
}

int semx_set_geometry(semx_ctx* c, int mode) {
  if (!c) return SEMX_EINVAL;
  if (mode == SEMX_GEOM_STORED) c->irregular_geo = kStored;
  else if (mode == SEMX_GEOM_TRILINEAR) c->irregular_geo = kTrilinear;
  else return fail(c, SEMX_EINVAL, "set_geometry: unknown mode");
  return SEMX_OK;
}

int semx_set_graphs(semx_ctx* c, int chunk) {
  if (!c) return SEMX_EINVAL;
  if (chunk < 0 || chunk > 4096) return fail(c, SEMX_EINVAL, "set_graphs: chunk outside [0, 4096]");
  c->graph_chunk = chunk;
  return SEMX_OK;
}

int semx_set_blocks(semx_ctx* c, int mode, int* active) {
  if (!c) return SEMX_EINVAL;
  if (mode != SEMX_BLOCKS_OFF && mode != SEMX_BLOCKS_AUTO && mode != SEMX_BLOCKS_ON)
    return fail(c, SEMX_EINVAL, "set_blocks: unknown mode");
  c->blocks_mode = mode;
  if (active) *active = blocks_active(c) ? 1 : 0;
  return SEMX_OK;
}

int semx_set_timing(semx_ctx* c, int stride) {
  if (!c) return SEMX_EINVAL;
  if (stride < 0) return fail(c, SEMX_EINVAL, "set_timing: negative stride");
  c->timing_stride = stride;
  c->timing_seq = 0;
  c->timed_launches = 0;
  c->ev_used = 0;
  return SEMX_OK;
}

int semx_force_timing(semx_ctx* c, int64_t* launches, double* total_ms) {
  if (!c || !launches || !total_ms) return SEMX_EINVAL;
  SEMX_HIP(c, hipStreamSynchronize(c->stream));
  double tot = 0.0;
  for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
    float ms = 0.0f;
    SEMX_HIP(c, hipEventElapsedTime(&ms, c->ev_pool[k], c->ev_pool[k + 1]));
    tot += ms;
  }
  *launches = c->timed_launches;
  *total_ms = tot;
  c->ev_used = 0;
  c->timed_launches = 0;
  return SEMX_OK;
}

int semx_set_storage(semx_ctx* c, int storage) {
  if (!c) return SEMX_EINVAL;
  if (storage != SEMX_F32 && storage != SEMX_F64) return fail(c, SEMX_EINVAL, "set_storage: unknown storage");
  if (c->have_model) return fail(c, SEMX_ESTATE, "set_storage: call before semx_upload_model");
  if (c->ckpt_every > 0) return fail(c, SEMX_ESTATE, "set_storage: turn checkpointing off first");
  if (storage == SEMX_F64 && c->contraction != SEMX_C_F32)
    return fail(c, SEMX_EINVAL, "set_storage: FP64 storage needs the SEMX_C_F32 contraction setting");
  if (storage == SEMX_F64 && c->n > kMaxNLow)
    return fail(c, SEMX_EINVAL, "set_storage: FP64 storage supports NGLL <= 10");
  if (storage == SEMX_F64 && c->physics == SEMX_ACOUSTIC)
    return fail(c, SEMX_EINVAL, "set_storage: the acoustic operator runs in FP32 storage");
  c->storage = storage;
  if (c->rec.nrec > 0) return alloc_seismograms(c);
  return SEMX_OK;
}

int semx_apply_force_f64(semx_ctx* c, const double* u_dev, double* f_dev) {
  if (!c) return SEMX_EINVAL;
  if (!c->have_mesh || !c->have_model) return fail(c, SEMX_ESTATE, "apply_force_f64: mesh and model required");
  if (c->storage != SEMX_F64) return fail(c, SEMX_ESTATE, "apply_force_f64: needs SEMX_F64 storage");
  if (!u_dev || !f_dev) return fail(c, SEMX_EINVAL, "apply_force_f64: null pointer");
  const int64_t len = state_len(c);
  if (u_dev < f_dev + len && f_dev < u_dev + len) return fail(c, SEMX_EINVAL, "apply_force_f64: u and f overlap");
  return f64_force_into(c, u_dev, f_dev, false);
}

int semx_read_seismograms_f64(semx_ctx* c, double* out, int out_on_device) {
  if (!c || !out) return SEMX_EINVAL;
  if (c->storage != SEMX_F64) return fail(c, SEMX_ESTATE, "read_seismograms_f64: needs SEMX_F64 storage");
  if (c->rec.nrec == 0 || !c->rec.seis64.p) return fail(c, SEMX_ESTATE, "read_seismograms_f64: no receivers");
  SEMX_HIP(c, hipMemcpyAsync(out, c->rec.seis64.p, c->rec.seis64.bytes,
                             out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  if (!out_on_device) SEMX_HIP(c, hipStreamSynchronize(c->stream));
  return SEMX_OK;
}

int semx_get_state_f64(semx_ctx* c, double* u_dev, double* v_dev, double* a_dev, int64_t* it) {
  if (!c) return SEMX_EINVAL;
  if (!c->have_model) return fail(c, SEMX_ESTATE, "get_state_f64: no model");
  if (c->storage != SEMX_F64) return fail(c, SEMX_ESTATE, "get_state_f64: needs SEMX_F64 storage");
  int rc = f64_finalize(c);
  if (rc) return rc;
  const size_t bytes = sizeof(double) * state_len(c);
  if (u_dev) SEMX_HIP(c, hipMemcpyAsync(u_dev, c->d_u.p, bytes, hipMemcpyDeviceToDevice, c->stream));
  if (v_dev) SEMX_HIP(c, hipMemcpyAsync(v_dev, c->d_v.p, bytes, hipMemcpyDeviceToDevice, c->stream));
  if (a_dev) SEMX_HIP(c, hipMemcpyAsync(a_dev, c->d_a.p, bytes, hipMemcpyDeviceToDevice, c->stream));
  if (it) *it = c->it;
  return SEMX_OK;
}

int semx_set_state_f64(semx_ctx* c, const double* u_dev, const double* v_dev, const double* a_dev, int64_t it) {
  if (!c) return SEMX_EINVAL;
  if (!c->have_model) return fail(c, SEMX_ESTATE, "set_state_f64: no model");
  if (c->storage != SEMX_F64) return fail(c, SEMX_ESTATE, "set_state_f64: needs SEMX_F64 storage");
  if (!u_dev || !v_dev || !a_dev || it < 0) return fail(c, SEMX_EINVAL, "set_state_f64: null pointer or negative index");
  const size_t bytes = sizeof(double) * state_len(c);
  SEMX_HIP(c, hipMemcpyAsync(c->d_u.p, u_dev, bytes, hipMemcpyDeviceToDevice, c->stream));
  SEMX_HIP(c, hipMemcpyAsync(c->d_v.p, v_dev, bytes, hipMemcpyDeviceToDevice, c->stream));
  SEMX_HIP(c, hipMemcpyAsync(c->d_a.p, a_dev, bytes, hipMemcpyDeviceToDevice, c->stream));
  fill_f64<<<grid_for(state_len(c)), kThreads, 0, c->stream>>>(c->d_f.as<double>(), state_len(c), 0.0);
  SEMX_HIP(c, hipGetLastError());
  c->it = it;
  c->pending_correct = false;
  return energy_reset(c);
}

}  // extern "C"
