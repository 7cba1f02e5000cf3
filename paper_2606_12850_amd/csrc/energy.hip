// Discrete energy of the explicit Newmark scheme and the work of the point
// sources (Sec. II-B weak form with the diagonal GLL mass; Sec. V-C
// second-order Newmark).  With K, M symmetric, the central-difference form of
// the scheme conserves
//   E^{n+1/2} = 1/2 (v^{n+1/2})^T M v^{n+1/2} + 1/2 (u^{n+1})^T K u^n,
// v^{n+1/2} = (u^{n+1} - u^n) / dt (the scheme's half-step velocity), up to the
// work of the sources: E^{n+1/2} - E^{n-1/2} = 1/2 (u^{n+1} - u^{n-1})^T f_src^n.
//
// Bookkeeping on the time loop, model 0 of the batch, FP64 sums:
//  * energy_track(): after the Newmark pass of step n (u holds u^{n+1}, v the
//    half-step velocity, f_pe the force f^n = -K u^n + f_src^n), one pass
//    sums v^T M v and u^{n+1} . f_pe in fixed-size blocks, reduced in a fixed
//    order (deterministic);
//  * energy_source_step(): every step, one workgroup over the source points
//    adds 1/2 (u^{n+1} - u^{n-1}) . f_src^n to the running source work and,
//    on tracked steps, sums u^{n+1} . f_src^n (the source part of f^n, which
//    the potential term must not see); it keeps u at the source points of
//    the last two steps.
// acc (double[8]): 0 sum M v^2, 1 sum u . f_pe, 2 sum u . f_src, 3 running
// source work.  The caller's state and kernels are not touched.
#include <algorithm>

#include "semx_internal.hpp"

namespace semx {
namespace {

constexpr int kEnergyBlocks = 1024;
constexpr int kT = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// part[b][0] = sum M v^2, part[b][1] = sum u . f over the entries of block b
// (grid-stride over nc * nglob entries of model 0).
template <class T>
__global__ __launch_bounds__(kT) void energy_pass_kernel(int64_t nglob, int nc, const double* __restrict__ mass,
                                                         const T* __restrict__ v, const T* __restrict__ u,
                                                         const T* __restrict__ f, double* __restrict__ part) {
  __shared__ double red[kT];
  double kin = 0.0, pot = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nc * nglob;
       t += (int64_t)gridDim.x * blockDim.x) {
    const double vv = v[t];
    kin += mass[t / nc] * vv * vv;
    pot += (double)u[t] * (double)f[t];
  }
  kin = block_sum(kin, red);
  pot = block_sum(pot, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = kin;
    part[2 * blockIdx.x + 1] = pot;
  }
}

// acc[0], acc[1] = sums of the block partials, in block order.
__global__ void energy_reduce_kernel(int nblk, const double* __restrict__ part, double* __restrict__ acc) {
  __shared__ double red[kT];
  double kin = 0.0, pot = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    kin += part[2 * b];
    pot += part[2 * b + 1];
  }
  kin = block_sum(kin, red);
  pot = block_sum(pot, red);
  if (threadIdx.x == 0) {
    acc[0] = kin;
    acc[1] = pot;
  }
}

// One workgroup over the source points with a nonzero weight (model 0):
// pts[k] = s n3 + q, f_src^n at that point, component c =
// stf[s][n] * wdir[(s n3 + q) nc + c]; hist is indexed by k.
// work: acc[3] += 1/2 sum (u^{n+1} - u^{n-1}) . f_src^n (with_work);
// corr: acc[2] = sum u^{n+1} . f_src^n; then hist[slot_new] = u^{n+1}.
// The step is n, or *step when `step` is given (graph-captured steps); the
// history slot of u^{n-1} (written two steps ago, overwritten with u^{n+1})
// and whether u^{n-1} is known (n > it0) follow from it.
template <class T>
__device__ __forceinline__ void source_energy_block(int npt, int n3, int nc, int64_t nstf, int64_t n,
                                                    const int64_t* step, int64_t it0, const int32_t* __restrict__ pts,
                                                    const int32_t* __restrict__ nodes, const T* __restrict__ wdir,
                                                    const T* __restrict__ stf, const T* __restrict__ u, T* hist,
                                                    size_t per, int with_corr, double* __restrict__ acc,
                                                    double* red) {
  if (step) n = *step;
  T* slot = hist + (size_t)((n + 1) & 1) * per;
  const T* hist_old = slot;
  T* hist_new = slot;
  const int with_work = n > it0 ? 1 : 0;
  double work = 0.0, corr = 0.0;
  for (int k = threadIdx.x; k < npt; k += blockDim.x) {
    const int p = pts[k];
    const int s = p / n3;
    const double amp = (n >= 0 && n < nstf) ? (double)stf[(int64_t)s * nstf + n] : 0.0;
    const int64_t g = nodes[p];
    for (int c = 0; c < nc; ++c) {
      const double un = u[nc * g + c];
      const double fs = amp * (double)wdir[(int64_t)nc * p + c];
      work += 0.5 * (un - (double)hist_old[(int64_t)nc * k + c]) * fs;
      corr += un * fs;
      hist_new[(int64_t)nc * k + c] = (T)un;
    }
  }
  work = block_sum(work, red);
  corr = block_sum(corr, red);
  if (threadIdx.x == 0) {
    if (with_work) acc[3] += work;
    if (with_corr) acc[2] = corr;
  }
}

template <class T>
__global__ __launch_bounds__(kT) void source_energy_kernel(int npt, int n3, int nc, int64_t nstf, int64_t n,
                                                           const int64_t* step, int64_t it0,
                                                           const int32_t* __restrict__ pts,
                                                           const int32_t* __restrict__ nodes,
                                                           const T* __restrict__ wdir, const T* __restrict__ stf,
                                                           const T* __restrict__ u, T* hist, size_t per,
                                                           int with_corr, double* __restrict__ acc) {
  __shared__ double red[kT];
  source_energy_block<T>(npt, n3, nc, nstf, n, step, it0, pts, nodes, wdir, stf, u, hist, per, with_corr, acc, red);
}

// Receivers (FP32 storage): receiver r of model `model` is
// sum_q l_q(x_r) u[node_q] per component (nc = 3 elastic, 1 acoustic),
// stored as sample `it` of seis [nmodels][nrec][nc][nt_max].  One block of
// kT lanes; the caller keeps samples outside [0, nt_max) away.
__device__ __forceinline__ void receiver_block(int r, int model, int nrec, int n3, int nc, int64_t nglob,
                                               int64_t nt_max, int64_t it, const int32_t* __restrict__ nodes,
                                               const float* __restrict__ wts, const float* __restrict__ u,
                                               float* __restrict__ seis, float (*red)[kT]) {
  const float* um = u + (int64_t)model * nglob * nc;
  float s[3] = {0.f, 0.f, 0.f};
  for (int q = threadIdx.x; q < n3; q += blockDim.x) {
    const float wq = wts[(int64_t)r * n3 + q];
    const int64_t g = nodes[(int64_t)r * n3 + q];
    for (int c = 0; c < nc; ++c) s[c] += wq * um[nc * g + c];
  }
  red[0][threadIdx.x] = s[0];
  red[1][threadIdx.x] = s[1];
  red[2][threadIdx.x] = s[2];
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + st];
    __syncthreads();
  }
  if ((int)threadIdx.x < nc)
    seis[(((int64_t)model * nrec + r) * nc + threadIdx.x) * nt_max + it] = red[threadIdx.x][0];
}

// The source force of sample m stored at the source nodes (all models): one
// thread per (model, source node, component) sums the (source, point) pairs
// that reach the node in a fixed order, as the injection after a force pass
// does, and stores the sum.
struct Prestore {
  int nsn;                    // source nodes; 0: nothing to store
  const int32_t* snode;       // [nsn] node numbers
  const int32_t* sptr;        // [nsn + 1]
  const int32_t* sidx;        // the points s n3 + q of each node
  float* f;                   // [nmodels][nglob][nc]
  int nmodels;
};

// The per-step bookkeeping before the force pass (FP32 storage), one launch
// after the Newmark pass: blocks x < nrec_blocks record receiver x of model
// y (sample it, or *step for graph-captured steps; nothing outside
// [0, nt_max)); block x = nrec_blocks of row y = 0, when `src` is set, is
// source_energy_block; the blocks after it in row 0 store the source force
// of sample it + 1 (P.nsn > 0).  All of them read u^{n+1}, which the force
// pass that follows leaves alone; the stores to f touch only source nodes,
// which nothing else in the launch reads.
__global__ __launch_bounds__(kT) void step_aux_kernel(int nrec_blocks, int nrec, int n3, int nc, int64_t nglob,
                                                      int64_t nt_max, int64_t it, const int64_t* step,
                                                      const int32_t* __restrict__ rnodes,
                                                      const float* __restrict__ rwts, float* __restrict__ seis,
                                                      int src, int npt, int64_t nstf, int64_t it0,
                                                      const int32_t* __restrict__ pts,
                                                      const int32_t* __restrict__ snodes,
                                                      const float* __restrict__ wdir, const float* __restrict__ stf,
                                                      float* hist, size_t per, int with_corr,
                                                      double* __restrict__ acc, const float* __restrict__ u,
                                                      Prestore P) {
  __shared__ float rred[3][kT];
  __shared__ double ered[kT];
  if ((int)blockIdx.x < nrec_blocks) {
    if (step) it = *step;
    if (it < 0 || it >= nt_max) return;  // uniform over the block
    receiver_block(blockIdx.x, blockIdx.y, nrec, n3, nc, nglob, nt_max, it, rnodes, rwts, u, seis, rred);
    return;
  }
  if (blockIdx.y != 0) return;
  if (src && (int)blockIdx.x == nrec_blocks) {
    source_energy_block<float>(npt, n3, nc, nstf, it, step, it0, pts, snodes, wdir, stf, u, hist, per, with_corr,
                               acc, ered);
    return;
  }
  const int64_t m = (step ? *step : it) + 1;
  const int64_t per_m = (int64_t)P.nsn * nc;
  const int64_t t = ((int64_t)blockIdx.x - nrec_blocks - src) * kT + threadIdx.x;
  if (t >= P.nmodels * per_m) return;
  const int64_t r = t % per_m;
  const int i = (int)(r / nc), cc = (int)(r % nc);
  float sum = 0.0f;
  for (int k = P.sptr[i]; k < P.sptr[i + 1]; ++k) {
    const int p = P.sidx[k];
    const float amp = (m >= 0 && m < nstf) ? stf[(int64_t)(p / n3) * nstf + m] : 0.0f;
    sum += amp * wdir[(int64_t)nc * p + cc];
  }
  P.f[((t / per_m) * nglob + P.snode[i]) * nc + cc] = sum;
}

// u at the source points (model 0) into hist (at a reset or a new state).
template <class T>
__global__ void source_gather_kernel(int npt, int nc, const int32_t* __restrict__ pts,
                                     const int32_t* __restrict__ nodes, const T* __restrict__ u,
                                     T* __restrict__ hist) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < npt; k += gridDim.x * blockDim.x)
    for (int c = 0; c < nc; ++c) hist[(int64_t)nc * k + c] = u[(int64_t)nc * nodes[pts[k]] + c];
}

__global__ void zero_doubles_kernel(double* __restrict__ p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0.0;
}

template <class T>
int source_step_t(semx_ctx* c, int64_t n, bool with_corr, const int64_t* dstep) {
  const int npt = c->src.npts;
  const size_t per = (size_t)npt * c->ncomp;
  T* hist = c->d_ehist.as<T>();
  const bool f64 = c->storage == SEMX_F64;
  const T* wdir = f64 ? (const T*)c->src.wdir64.p : (const T*)c->src.wdir.p;
  const T* stf = f64 ? (const T*)c->src.stf64.p : (const T*)c->src.stf.p;
  // the slot of u^{n-1} (stored two steps ago) is the slot u^{n+1} goes to;
  // u^{n-1} is known from the second step on (n > energy_it0)
  source_energy_kernel<T><<<1, kT, 0, c->stream>>>(npt, c->n3, c->ncomp, c->src.nstf, n, dstep, c->energy_it0,
                                                   c->src.pts.as<int32_t>(), c->src.nodes.as<int32_t>(), wdir, stf,
                                                   c->d_u.as<T>(), hist, per, with_corr ? 1 : 0,
                                                   c->d_eacc.as<double>());
  SEMX_HIP(c, hipGetLastError());
  return SEMX_OK;
}

}  // namespace

int energy_reset(semx_ctx* c) {
  int rc = SEMX_OK;
  if (!c->d_eacc.p) rc = dev_alloc(c, c->d_eacc, sizeof(double) * 8);
  if (!rc && !c->d_epart.p) rc = dev_alloc(c, c->d_epart, sizeof(double) * 2 * kEnergyBlocks);
  if (rc) return rc;
  zero_doubles_kernel<<<1, 64, 0, c->stream>>>(c->d_eacc.as<double>(), 8);
  SEMX_HIP(c, hipGetLastError());
  c->energy_it = -1;
  c->energy_it0 = c->it;
  const int npt = c->src.nsrc > 0 ? c->src.npts : 0;
  if (npt == 0) return SEMX_OK;
  const size_t tsz = c->storage == SEMX_F64 ? sizeof(double) : sizeof(float);
  const size_t bytes = 2 * (size_t)npt * c->ncomp * tsz;
  if (c->d_ehist.bytes != bytes) {
    rc = dev_alloc(c, c->d_ehist, bytes);
    if (rc) return rc;
  }
  SEMX_HIP(c, hipMemsetAsync(c->d_ehist.p, 0, bytes, c->stream));
  const size_t per = (size_t)npt * c->ncomp;
  const unsigned nb = (unsigned)std::min(1024, (npt + kT - 1) / kT);
  const size_t slot = (size_t)(c->it & 1) * per;
  if (c->storage == SEMX_F64)
    source_gather_kernel<double><<<nb, kT, 0, c->stream>>>(npt, c->ncomp, c->src.pts.as<int32_t>(),
                                                           c->src.nodes.as<int32_t>(),
                                                           c->d_u.as<double>(), c->d_ehist.as<double>() + slot);
  else
    source_gather_kernel<float><<<nb, kT, 0, c->stream>>>(npt, c->ncomp, c->src.pts.as<int32_t>(),
                                                          c->src.nodes.as<int32_t>(),
                                                          c->d_u.as<float>(), c->d_ehist.as<float>() + slot);
  SEMX_HIP(c, hipGetLastError());
  return SEMX_OK;
}

int step_aux(semx_ctx* c, int64_t n, bool with_corr, bool record, const int64_t* dstep, bool prestore) {
  const bool src = c->src.nsrc > 0 && c->d_ehist.p != nullptr;
  const bool rec = record && c->rec.nrec > 0 && (dstep || (n >= 0 && n < c->rec.nt_max));
  const bool pre = prestore && c->src.nsrc > 0 && c->src.nsn > 0;
  if (!src && !rec && !pre) return SEMX_OK;
  const int nrb = rec ? c->rec.nrec : 0;
  Prestore P{};
  int npb = 0;
  if (pre) {
    P = {c->src.nsn, c->src.snode.as<int32_t>(), c->src.sptr.as<int32_t>(), c->src.sidx.as<int32_t>(),
         c->d_f.as<float>(), c->nmodels};
    npb = (int)(((int64_t)c->nmodels * c->src.nsn * c->ncomp + kT - 1) / kT);
  }
  dim3 grid(nrb + (src ? 1 : 0) + npb, rec ? c->nmodels : 1);
  const size_t per = (size_t)c->src.npts * c->ncomp;
  step_aux_kernel<<<grid, kT, 0, c->stream>>>(
      nrb, c->rec.nrec, c->n3, c->ncomp, c->nglob, c->rec.nt_max, n, dstep, c->rec.nodes.as<int32_t>(),
      c->rec.wts.as<float>(), c->rec.seis.as<float>(), src ? 1 : 0, c->src.npts, c->src.nstf, c->energy_it0,
      c->src.pts.as<int32_t>(), c->src.nodes.as<int32_t>(), c->src.wdir.as<float>(), c->src.stf.as<float>(),
      c->d_ehist.as<float>(), per, with_corr ? 1 : 0, c->d_eacc.as<double>(), c->d_u.as<float>(), P);
  SEMX_HIP(c, hipGetLastError());
  return SEMX_OK;
}

int energy_source_step(semx_ctx* c, int64_t n, bool with_corr, const int64_t* dstep) {
  if (c->src.nsrc == 0 || !c->d_ehist.p) return SEMX_OK;
  return c->storage == SEMX_F64 ? source_step_t<double>(c, n, with_corr, dstep)
                                : source_step_t<float>(c, n, with_corr, dstep);
}

int energy_track(semx_ctx* c, const void* f_pe, bool source_in_f) {
  if (!c->d_eacc.p) return fail(c, SEMX_ESTATE, "energy: the run was not reset");
  double* part = c->d_epart.as<double>();
  if (c->storage == SEMX_F64)
    energy_pass_kernel<double><<<kEnergyBlocks, kT, 0, c->stream>>>(
        c->nglob, c->ncomp, c->d_mass64.as<double>(), c->d_v.as<double>(), c->d_u.as<double>(),
        static_cast<const double*>(f_pe), part);
  else
    energy_pass_kernel<float><<<kEnergyBlocks, kT, 0, c->stream>>>(c->nglob, c->ncomp, c->d_mass64.as<double>(),
                                                                  c->d_v.as<float>(), c->d_u.as<float>(),
                                                                  static_cast<const float*>(f_pe), part);
  SEMX_HIP(c, hipGetLastError());
  energy_reduce_kernel<<<1, kT, 0, c->stream>>>(kEnergyBlocks, part, c->d_eacc.as<double>());
  SEMX_HIP(c, hipGetLastError());
  if (!source_in_f) zero_doubles_kernel<<<1, 64, 0, c->stream>>>(c->d_eacc.as<double>() + 2, 1);
  SEMX_HIP(c, hipGetLastError());
  return SEMX_OK;
}

int energy_read(semx_ctx* c, double* kin, double* pot, double* work) {
  if (c->energy_it != c->it || !c->d_eacc.p)
    return fail(c, SEMX_ESTATE,
                "energy: no half step tracked at the current time index (call semx_step after a reset or a new state)");
  double h[4] = {0, 0, 0, 0};
  SEMX_HIP(c, hipMemcpyAsync(h, c->d_eacc.p, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  SEMX_HIP(c, hipStreamSynchronize(c->stream));
  *kin = 0.5 * h[0];
  *pot = -0.5 * (h[1] - h[2]);
  if (work) *work = h[3];
  return SEMX_OK;
}

}  // namespace semx
