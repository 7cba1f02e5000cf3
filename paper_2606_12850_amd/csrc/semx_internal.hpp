// Internal declarations of libsemx (not installed).  Context layout, error
// helpers and the launchers each kernel translation unit provides.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/semx.h"

namespace semx {

constexpr int kMaxN = 16;     // largest supported NGLL
constexpr int kMaxNLow = 10;  // largest NGLL of the one-point-per-lane kernels (FP64 storage, adjoint)
constexpr int kNumXcd = 8;  // MI355X: 8 accelerator complex dies, round-robin block dispatch
// Word 3 of a raw buffer resource on gfx9-family devices (gfx950): 32-bit
// data format, no swizzle, range-checked against num_records (out-of-range
// lanes read zeros and fetch nothing).
constexpr int kBufferWord3 = 0x00020000;

// geometry path of a force launch
constexpr int kRegular = 0;    // affine element: one Gamma per element
constexpr int kStored = 1;     // per-point Gamma streamed from memory
constexpr int kTrilinear = 2;  // J rebuilt per point from the trilinear map coefficients

// Device buffer owned by the library.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// One force launch: a contiguous range of launch positions (elements of one
// colour and one geometry kind, or of one kind for atomic assembly).
struct Launch {
  int64_t pos0 = 0;
  int64_t count = 0;
  bool irregular = false;  // geometry path: kRegular, else the context's irregular path
  int64_t naff = 0;        // leading elements whose node numbers are affine in (i, j, k)
};

struct SourceSet {
  int nsrc = 0;
  int64_t nstf = 0;
  DevBuf nodes;   // int32 [nsrc][n3]
  DevBuf wdir;    // float [nsrc][n3][3]: l_q(x_s) * dir_c
  DevBuf stf;     // float [nsrc][nstf]
  DevBuf wdir64;  // double copies of wdir and stf (FP64 storage)
  DevBuf stf64;
  DevBuf pts;     // int32 [npts]: the points (s n3 + q) with a nonzero weight (energy bookkeeping)
  int npts = 0;
  // the nodes that receive a source force (FP32 weights), ascending, and for
  // node i its points sidx[sptr[i] .. sptr[i + 1]) (s n3 + q, ascending)
  DevBuf snode, sptr, sidx;
  int nsn = 0;
};

struct ReceiverSet {
  int nrec = 0;
  int64_t nt_max = 0;
  DevBuf nodes;   // int32 [nrec][n3]
  DevBuf wts;     // float [nrec][n3]
  DevBuf seis;    // float [nmodels][nrec][3][nt_max] (FP32 storage)
  DevBuf wts64;   // double [nrec][n3]
  DevBuf seis64;  // double [nmodels][nrec][3][nt_max] (FP64 storage)
};

}  // namespace semx

struct semx_ctx {
  int n = 0, n3 = 0;
  hipStream_t stream = nullptr;
  // graph-captured time loop (semx_set_graphs): steps per captured chunk
  // (0: every step launched directly), the device step counter the captured
  // steps read, and the stream the capture is recorded on
  int graph_chunk = 0;
  semx::DevBuf d_step;
  hipStream_t cap_stream = nullptr;
  int device = 0;
  int num_cu = 256;
  std::string err;

  int contraction = SEMX_C_F32;
  int assembly = SEMX_ASM_COLORED;
  int storage = SEMX_F32;  // SEMX_F64: state, force and time loop in double (fp64.hip)
  int physics = SEMX_ELASTIC;  // SEMX_ACOUSTIC: scalar field (acoustic.hip)
  int ncomp = 3;               // field components per node: 3 elastic, 1 acoustic

  // GLL data (library's own, FP64 on host)
  std::vector<double> xi, w, D;  // D[a*n+b] = l'_b(xi_a)
  semx::DevBuf d_D;              // float [n][n]
  semx::DevBuf d_Dh;             // packed half/bfloat D tables for the MFMA paths
  semx::DevBuf d_xi64, d_w64;    // double [n]

  // mesh
  bool have_mesh = false;
  int64_t nspec = 0, nglob = 0, nvert = 0;
  std::vector<int32_t> h_ibool;     // kept for colouring checks and sources
  std::vector<int32_t> h_elem_vert;
  std::vector<double> h_vert;
  // per-element device arrays are stored by launch position; h_order[pos] =
  // element, positions sorted by (geometry kind, colour, element)
  std::vector<int32_t> h_order;
  semx::DevBuf d_order;     // int32 [nspec]
  std::vector<float> h_gam_el;  // [nspec][9] per-element Gamma of regular elements (user order)
  semx::DevBuf d_ibool;     // int32 [nspec][n3]
  semx::DevBuf d_aff;       // int32 [nspec][4]: g0, sx, sy, sz of affine-numbered elements (g0 = -1 otherwise)
  semx::DevBuf d_vert;      // double [nvert][3]
  semx::DevBuf d_elem_vert; // int32 [nspec][8]
  semx::DevBuf d_gam_pt;    // float [nspec][9][n3] (allocated if any irregular element)
  semx::DevBuf d_tri;       // float [nspec][3][8] trilinear map coefficients (irregular elements)
  semx::DevBuf d_xi32;      // float [n] GLL nodes
  int irregular_geo = semx::kStored;  // path for irregular elements (semx_set_geometry)
  semx::DevBuf d_gam_el;    // float [nspec][9]     (per-element Gamma of regular elements)
  semx::DevBuf d_wdet;      // double [nspec][n3]   w_i w_j w_k det J
  std::vector<uint8_t> h_regular;  // per element
  int64_t nregular = 0, nirregular = 0;
  double hmin = 0.0;               // min distance between adjacent GLL points

  // first touch of each node in coloured launch order, per launch position:
  // bit q of d_first[pos * first_words + q / 32] set when local point q is the
  // first to reach its node; elem_cover = every node is reached by an element
  semx::DevBuf d_first;
  int first_words = 0;
  std::vector<uint32_t> h_first;     // host copy of d_first
  // the time loop's first-touch bits (per element and per block): the same
  // with the bit of every node that receives a source force cleared, so the
  // pass adds to the source force stored there before it (built when the
  // sources or the mesh change)
  semx::DevBuf d_first_tl, d_bfirst_tl;
  bool first_tl_dirty = true;
  std::vector<int32_t> h_src_nodes;  // nodes with a source force (FP32 weights), ascending
  bool elem_cover = false;
  // every element-interior GLL point (local indices 1..n-2 in all three
  // directions) is the only reference to its node, as in any conforming mesh:
  // atomic assembly stores those points' forces without an atomic
  bool interior_exclusive = false;

  // colouring
  int ncolors = 0;
  std::vector<int32_t> color_ptr, elem_order;
  std::vector<semx::Launch> colored_launches;  // per colour: regular then irregular
  std::vector<semx::Launch> atomic_launches;   // regular list, irregular list
  // 2 x 2 x 2 element blocks (FP32 elastic force, NGLL <= 5, coloured):
  // built when every element is affine-numbered with common strides, of one
  // geometry kind, and belongs to a block; nblocks = 0 otherwise
  int64_t nblocks = 0;
  bool blocks_irregular = false;
  int blocks_mode = 1;                         // semx_set_blocks (SEMX_BLOCKS_AUTO)
  std::vector<semx::Launch> block_launches;    // per block colour: a range of the block tables
  semx::DevBuf d_bpos, d_baff, d_bfirst;
  std::vector<int32_t> h_baff;     // host copies of d_baff and d_bfirst
  std::vector<uint32_t> h_bfirst;

  // model
  bool have_model = false;
  int nmodels = 0;
  semx::DevBuf d_mat;      // float [nmodels][nspec][2][n3]: lambda*W, mu*W
  semx::DevBuf d_minv;     // float [nmodels][nglob]
  semx::DevBuf d_mass64;   // double [nmodels][nglob]
  semx::DevBuf d_wrho;     // float [nmodels][nspec][n3] rho * W (adjoint density kernel)
  double vp_max = 0.0;

  // FP64 storage: Gamma [nspec][9][n3], lambda W / mu W [nmodels][nspec][2][n3]
  // by launch position, M^{-1} [nmodels][nglob], D [n][n]
  semx::DevBuf d_gam64, d_mat64, d_minv64, d_D64;

  // time loop state, [nmodels][nglob][3], float or double by `storage`
  semx::DevBuf d_u, d_v, d_a, d_f;
  semx::DevBuf d_work;     // scratch vector of the same shape (energy, power iteration)
  semx::DevBuf d_scratch;  // double reduction scratch + flags
  double dt = 0.0;
  bool have_dt = false;
  double lambda_max = 0.0;  // power-iteration estimate (0 = unknown)
  int64_t it = 0;
  bool pending_correct = false;  // f holds -K u^n + f_src^n, a/v not yet corrected
  int64_t watchdog_every = 0;
  double watchdog_emax = 0.0;

  // discrete energy E^{n+1/2} and source work (energy.hip): tracked on the
  // last step of each semx_step call and on watchdog steps
  semx::DevBuf d_eacc;    // double [8] sums (see energy.hip)
  semx::DevBuf d_epart;   // double block partials
  semx::DevBuf d_ehist;   // u at the source points, last two steps [2][nsrc n3][ncomp]
  int64_t energy_it = -1; // time index whose E^{it-1/2} is in d_eacc (-1: none)
  int64_t energy_it0 = 0; // time index of the last reset / new state (the source work starts there)
  bool track_energy = false;  // track the energy on the coming step

  semx::SourceSet src;
  semx::ReceiverSet rec;

  // forward checkpoints for the adjoint: state (u, v, a) at it = k * ckpt_every
  int64_t ckpt_every = 0;
  int64_t ckpt_count = 0;
  std::vector<semx::DevBuf> ckpts;  // one buffer of 3 * state_len floats per checkpoint
  // run generation: bumped by every reset, new state, new sources or new
  // model; a checkpoint is usable only by the run that saved it
  int64_t run_gen = 0;
  std::vector<int64_t> ckpt_gen;    // generation of each saved checkpoint

  // optional event timing of force passes: every timing_stride-th pass
  // (0 = off) is bracketed by one event pair; timed_launches counts the
  // force launches inside the timed passes
  int timing_stride = 0;
  int64_t timing_seq = 0;
  int64_t timed_launches = 0;
  std::vector<hipEvent_t> ev_pool;  // 2 per recorded launch, reused
  size_t ev_used = 0;
};

namespace semx {

// ---- error helpers -------------------------------------------------------
int fail(semx_ctx* c, int code, const std::string& msg);
int hip_fail(semx_ctx* c, hipError_t e, const char* what);
#define SEMX_HIP(ctx, call)                                   \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return semx::hip_fail(ctx, e_, #call); \
  } while (0)

int dev_alloc(semx_ctx* c, DevBuf& b, size_t bytes);
void dev_free(DevBuf& b);

// ---- GLL basis (host, FP64) ---------------------------------------------
void gll_nodes_weights(int n, std::vector<double>& xi, std::vector<double>& w);
void deriv_matrix(int n, const std::vector<double>& xi, std::vector<double>& D);
void lagrange_at(int n, const std::vector<double>& xi, double x, double* l);

// ---- launchers (force_f32.hip, force_mfma.hip) -----------------------------

struct ForceArgs {
  const int32_t* ibool;
  const int32_t* aff;    // [nspec][4] affine numbering g = g0 + i sx + j sy + k sz
  const float* gam_pt;   // [nspec][9][n3]   (kStored)
  const float* gam_el;   // [nspec][9]       (kRegular)
  const float* tri;      // [nspec][3][8]    (kTrilinear: c0..c7 of each coordinate)
  const float* xi;       // [n] GLL nodes, FP32
  const float* mat;      // [nmodels][nspec][2][n3]
  const float* u;        // [nmodels][nglob][3]
  float* f;              // [nmodels][nglob][3]
  const float* D;        // [n][n] FP32
  const void* Dh;        // packed low-precision D tables (MFMA paths)
  const uint32_t* first; // coloured per-element paths: per-position bitmask of the points that
                         // reach their node first in launch order (store, no read), or null
  int first_words;       // 32-bit words per position in `first`
  int excl_interior;     // atomic assembly: element-interior points own their nodes (plain store)
  int64_t pos0;          // first launch position of this launch
  int64_t count;
  int64_t nspec, nglob;
  int nmodels;
};
hipError_t launch_force_f32(int n, int geo, bool atomic, const ForceArgs& a, hipStream_t s);
// The same over a launch whose first `naff` elements have an affine numbering:
// those compute their node numbers instead of reading ibool.
hipError_t launch_force_f32_split(int n, int geo, bool atomic, int64_t naff, const ForceArgs& a, hipStream_t s);
// Memory skeleton of the coloured launch_force_f32_split (same loads and stores, no arithmetic).
hipError_t launch_force_skeleton(int n, int geo, int64_t naff, const ForceArgs& a, hipStream_t s);

// force_block.hip: 2 x 2 x 2 element blocks, NGLL 2..5, coloured assembly.
// A launch covers blocks beg .. beg + count - 1 of the block tables (one
// block colour): bpos [nblocks][8] launch positions of the block's elements
// m = dx + 2 dy + 4 dz; baff [nblocks][4] the block's node numbering
// G0 + X sx + Y sy + Z sz (X, Y, Z = 0..2n-2); bfirst [nblocks][words] the
// first-touch bits of its nodes in block launch order (or null: every node
// reads its prior force).
struct BlockArgs {
  const int32_t* bpos;
  const int32_t* baff;
  const uint32_t* bfirst;
  int64_t beg, count;
};
hipError_t launch_force_block(int n, int geo, const ForceArgs& a, const BlockArgs& b, hipStream_t s);
hipError_t launch_force_block_skeleton(int n, int geo, const ForceArgs& a, const BlockArgs& b, hipStream_t s);
constexpr int kBlockMaxN = 5;  // eight elements of n^3 points in one 1024-lane workgroup

hipError_t launch_force_mfma(int n, int prec, int geo, bool atomic, const ForceArgs& a, hipStream_t s);
// force_high.hip: NGLL 11..16 (one lane per (i, j) column; the FP32 force pass uses it for 11..12)
hipError_t launch_force_high(int n, int geo, bool atomic, const ForceArgs& a, hipStream_t s);
// Memory skeleton of the coloured launch_force_high (same loads and stores, no arithmetic).
hipError_t launch_force_high_skeleton(int n, int geo, const ForceArgs& a, hipStream_t s);
// force_tile16.hip: NGLL 11..16 (16-point tiles, padded below 16), all six
// contractions on the matrix cores; prec SEMX_C_F32 / SEMX_C_MFMA_F32 (FP32
// operands), SEMX_C_BF16, SEMX_C_F16 (the launch's first naff elements have
// an affine numbering).  FP32 contractions take it from kTileMinN (below,
// the column kernel is faster: at NGLL 11-12 the padded tile does 2.4-3x the
// useful matrix work), the matrix-core modes from kTileMinNMixed.
constexpr int kTileMinN = 13;
constexpr int kTileMinNMixed = 11;
// FP32 at NGLL 12: the tile kernel for launches of regular elements (its
// persistent form, 0.754 against 0.917 ms per apply for the column kernel
// at 2e7 nodes); with per-point or trilinear geometry the column kernel
// stays faster (0.98 against 1.05-1.19 ms), as at NGLL 11 on every path.
constexpr int kTileRegularN = 12;
hipError_t launch_force_tile16(int n, int prec, int geo, bool atomic, int64_t naff, const ForceArgs& a,
                               hipStream_t s);
// The scalar (acoustic) operator, NGLL 12..16, on the same tiles (FP32; the
// first half of the material table is W / rho): u and f have one value per
// node.  Measured against the column kernel at 2e7 nodes: slower at NGLL 11
// (0.374 / 0.355 ms), faster from 12 (0.348 / 0.383) to 16 (0.195 / 0.383).
constexpr int kTileMinNAcoustic = 12;
hipError_t launch_force_tile16_acoustic(int n, int geo, bool atomic, int64_t naff, const ForceArgs& a,
                                        hipStream_t s);
// acoustic.hip: the scalar operator, NGLL 2..16 (u, f hold one value per node;
// the launch's first naff elements have an affine numbering)
hipError_t launch_force_acoustic(int n, int geo, bool atomic, int64_t naff, const ForceArgs& a, hipStream_t s);
// MFMA contraction modes: NGLL 4..8 and 13..16 (all three precisions).
bool mfma_supported(int n, int prec);

// ---- host helpers shared between translation units (api.hip) ----------------
// One explicit step.  seg_u / seg_a (the adjoint's forward recomputation,
// may be null): the Newmark pass also stores the predicted u and, when it
// corrects the previous step, that step's acceleration, into them.
// dstep: the device step counter when the step is captured into a graph
// (the step-indexed kernels read it; the step advances it), else null.
int step_once(semx_ctx* c, bool record, float* seg_u = nullptr, float* seg_a = nullptr,
              const int64_t* dstep = nullptr);
int apply_force_accumulate(semx_ctx* c, const float* u, float* f);
int fill_zero(semx_ctx* c, float* p, int64_t n);
// Apply the pending correction (a = M^{-1} f, v += dt/2 a); seg_a, if given,
// receives a as well.
int complete_step(semx_ctx* c, float* seg_a = nullptr);
unsigned grid_1d(int64_t n, int cap = 1 << 16);
// adjoint.hip
int save_checkpoint(semx_ctx* c);

// scratch layout: [0..7] doubles for reductions, then int flags
inline double* scratch_doubles(semx_ctx* c) { return c->d_scratch.as<double>(); }
inline int* scratch_flags(semx_ctx* c) { return reinterpret_cast<int*>(c->d_scratch.as<double>() + 8); }

// energy.hip: discrete energy and source work bookkeeping (model 0)
int energy_reset(semx_ctx* c);
// after the Newmark pass of step n: f_pe holds f^n (-K u^n + f_src^n when
// source_in_f, else -K u^n)
int energy_track(semx_ctx* c, const void* f_pe, bool source_in_f);
// every step n after the Newmark pass (u holds u^{n+1})
int energy_source_step(semx_ctx* c, int64_t n, bool with_corr, const int64_t* dstep = nullptr);
// FP32 storage: energy_source_step and, with `record`, the receivers' sample
// n (u^{n+1}), in one launch before the force pass (dstep: the device step
// counter of graph-captured steps, else null).  `prestore`: the same launch
// also stores the source force of sample n + 1 into f at the source nodes
// (the force pass then adds to it, through the time-loop first-touch bits).
int step_aux(semx_ctx* c, int64_t n, bool with_corr, bool record, const int64_t* dstep = nullptr,
             bool prestore = false);
int energy_read(semx_ctx* c, double* kin, double* pot, double* work);

// fp64.hip: the FP64 storage path (state buffers hold doubles)
int f64_model_setup(semx_ctx* c, const double* lam_dev, const double* mu_dev);
int f64_force_into(semx_ctx* c, const double* u, double* f, bool f_zeroed);
int f64_finalize(semx_ctx* c);
int f64_reset(semx_ctx* c);
int f64_step_once(semx_ctx* c, bool record);
int f64_check_finite(semx_ctx* c, bool* ok);

}  // namespace semx
