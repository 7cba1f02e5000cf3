/*
 * semx -- spectral-element elastic wave operator for AMD Instinct MI355X (gfx950).
 *
 * C interface of libsemx.so.  The library implements the matrix-free
 * element internal-force operator of the spectral-element method (SEM) for
 * isotropic elasticity and the explicit, diagonal-mass Newmark time loop
 * around it, following "High-Order Spectral Element Methods for Wave
 * Propagation on ARM Multicore CPU with SME" (Sec. II-B: GLL tensor-product
 * basis, elastic wave equation and weak form, diagonal mass, stiffness
 * applied as three forward and three transpose batched small contractions;
 * Sec. IV-C: graph-coloured assembly versus atomic updates; Sec. IV-D: fused
 * derivative/strain/stress traversal, regular/irregular element paths,
 * flattened gather/scatter; Sec. V-C: second-order Newmark, Ricker source).
 *
 * Conventions
 *   - Every function returns an int status: SEMX_OK (0) or a negative code.
 *     semx_last_error() returns a per-context text for the last failure.
 *   - Host arrays passed in are copied before the call returns; the caller
 *     keeps ownership.  Device pointers passed in (u_dev, f_dev, ...) stay
 *     owned by the caller and must hold at least the stated number of
 *     elements; the library never frees them.  Buffers the library allocates
 *     are freed by semx_destroy().
 *   - All GPU work is ordered on the HIP stream given to semx_create(); a
 *     call that returns data to host memory synchronises that stream.
 *     A context is not thread-safe; use one context per host thread.
 *   - ngll = n = N+1 GLL points per direction, 2 <= n <= 16 (N = polynomial
 *     degree up to 15).  From NGLL 11 the FP32 operator runs on a
 *     column-per-lane kernel (NGLL 11, and 12 on irregular elements) or on
 *     matrix-core tiles (the rest; the acoustic operator from 12), the
 *     adjoint on column-per-lane kernels; FP64 storage supports n <= 10
 *     (SEMX_EINVAL above), the 16-bit matrix-core contractions 4 <= n <= 8
 *     and 11 <= n <= 16.  Element-local point q = i + n*(j + n*k), i fastest
 *     (i along xi, j along eta, k along zeta).
 *   - Corner v = a + 2b + 4c of an 8-node hexahedron sits at reference
 *     coordinates (xi, eta, zeta) = (2a-1, 2b-1, 2c-1); the geometry is the
 *     trilinear map of the 8 corners.
 *   - Vectors over global nodes are FP32 [nmodels][nglob][3], component
 *     fastest (FP64 with SEMX_F64 storage, see semx_set_storage()).
 *     f = -K u is the internal force (the negative stiffness action), the
 *     right-hand-side term of the weak form.
 */
#ifndef SEMX_H
#define SEMX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct semx_ctx semx_ctx;

/* status codes */
#define SEMX_OK 0
#define SEMX_EINVAL -1     /* bad argument, size or shape */
#define SEMX_ESTATE -2     /* call out of order (e.g. step before upload) */
#define SEMX_EGEOM -3      /* det J <= 0 at some GLL point */
#define SEMX_EUNSTABLE -4  /* dt above the stability bound of the operator */
#define SEMX_EHIP -5       /* HIP runtime error; the text names the HIP call */
#define SEMX_ENOMEM -6     /* device allocation failed */
#define SEMX_ENUMERIC -7   /* NaN/Inf or energy blow-up detected by the watchdog */

/* contraction arithmetic of the force operator (mixed precision keeps the
 * geometry map, stress and assembly in FP32) */
#define SEMX_C_F32 0       /* FP32 contractions: vector units through LDS (NGLL 2..12),
                              FP32-operand MFMA tiles (NGLL 13..16) */
#define SEMX_C_BF16 1      /* BF16-operand MFMA contractions, FP32 accumulation */
#define SEMX_C_F16 2       /* FP16-operand MFMA contractions, FP32 accumulation */
#define SEMX_C_MFMA_F32 3  /* FP32-operand MFMA contractions (v_mfma_f32_16x16x4f32) */

/* assembly of element forces into the global vector (Sec. IV-C) */
#define SEMX_ASM_COLORED 0 /* colour by colour, plain read-modify-write, deterministic */
#define SEMX_ASM_ATOMIC 1  /* one launch, FP32 global atomic adds */

/* storage and arithmetic of the state vectors and the time loop */
#define SEMX_F32 0         /* FP32 fields, force and Newmark update (default) */
#define SEMX_F64 1         /* FP64 fields, FP64 force, Newmark, sources and receivers */

/* Create a context for n = ngll GLL points per direction whose GPU work runs
 * on hip_stream (a hipStream_t; NULL = the default stream) of the current
 * device.  Defaults: SEMX_C_F32, SEMX_ASM_COLORED. */
int semx_create(semx_ctx **out, int ngll, void *hip_stream);

/* Free every buffer of the context.  NULL is accepted. */
int semx_destroy(semx_ctx *ctx);

/* Text of the last error on this context ("" if none).  Valid until the next call. */
const char *semx_last_error(const semx_ctx *ctx);

/* Mesh (Sec. II-B; global-to-local map of Sec. IV-C).
 *   ibool     [nspec][n^3]  global node of each element-local point, 0 <= g < nglob;
 *   vert_xyz  [nvert][3]    FP64 corner coordinates;
 *   elem_vert [nspec][8]    corner vertex indices, order above.
 * The library computes J, det J and Gamma = J^{-1} at every GLL point in FP64
 * on the device, stores Gamma in FP32, classifies each element as regular
 * (affine map: Gamma constant) or irregular, and colours the elements by
 * greedy first-fit in element order so that no two elements of a colour share
 * a global node.  Returns SEMX_EGEOM if det J <= 0 anywhere.  Invalidates any
 * uploaded model and time-loop state, and removes the sources and receivers
 * (they are placed in elements of the previous mesh). */
int semx_upload_mesh(semx_ctx *ctx, int64_t nspec, int64_t nglob, const int32_t *ibool,
                     int64_t nvert, const double *vert_xyz, const int32_t *elem_vert);

/* Replace the colouring: elem_order [nspec] lists the elements colour by
 * colour, colour c owning elem_order[color_ptr[c] .. color_ptr[c+1]-1].
 * Rejected (SEMX_EINVAL) unless it is a permutation and no two elements of a
 * colour share a global node. */
int semx_set_coloring(semx_ctx *ctx, int ncolors, const int32_t *color_ptr, const int32_t *elem_order);

/* Read the current colouring.  color_ptr needs ncolors+1 entries and
 * elem_order nspec entries; either may be NULL to query ncolors only. */
int semx_get_coloring(semx_ctx *ctx, int *ncolors, int32_t *color_ptr, int32_t *elem_order);

/* Counts of the mesh: regular and irregular elements and colours. */
int semx_mesh_info(semx_ctx *ctx, int64_t *nregular, int64_t *nirregular, int *ncolors);

/* Isotropic elastic model per element-local point (Sec. II-B, T = C : grad s
 * with C isotropic), FP64 host arrays [nmodels][nspec][n^3]: Lame lambda,
 * mu and density rho.  nmodels > 1 uploads a batch of models sharing the
 * mesh; state vectors then hold nmodels stacked fields.  The library forms
 * lambda*w_i w_j w_k det J and mu*w_i w_j w_k det J (FP32) and the lumped
 * GLL mass M_g = sum rho w_i w_j w_k det J (FP64 accumulate, FP32 M^{-1}).
 * Requires rho > 0, mu > 0, lambda + 2 mu/3 > 0.  Resets the time loop. */
int semx_upload_model(semx_ctx *ctx, int nmodels, const double *lambda, const double *mu,
                      const double *rho);

/* Select the contraction arithmetic and the assembly (constants above).
 * The matrix-core contractions (SEMX_C_BF16, SEMX_C_F16, SEMX_C_MFMA_F32)
 * need 4 <= NGLL <= 8 or 11 <= NGLL <= 16 (at 13..16 SEMX_C_MFMA_F32 is the
 * FP32 path itself); SEMX_EINVAL otherwise, or for an unknown value, or for
 * coloured assembly on a mesh whose elements repeat a node. */
int semx_set_mode(semx_ctx *ctx, int contraction, int assembly);

/* Geometry path of irregular (non-affine) elements (Sec. IV-D keeps the
 * regular and irregular cases in separate code paths):
 *   SEMX_GEOM_STORED     Gamma = J^{-1} at every GLL point precomputed in FP64
 *                        and streamed from memory (9 floats per point);
 *   SEMX_GEOM_TRILINEAR  J rebuilt at every point inside the kernel from the
 *                        element's trilinear-map coefficients (computed in
 *                        FP64, stored FP32): the same operator with no
 *                        per-point geometry traffic.
 * Regular (affine) elements always use one Gamma per element.  Default STORED. */
#define SEMX_GEOM_STORED 0
#define SEMX_GEOM_TRILINEAR 1
int semx_set_geometry(semx_ctx *ctx, int mode);

/* Element blocks for the coloured FP32 elastic force at NGLL <= 5 (the
 * colouring of Sec. IV-C taken over 2 x 2 x 2 element blocks, with the
 * fused traversal of Sec. IV-D inside each): one workgroup per block of
 * eight face-adjacent elements gathers each of the block's (2 NGLL - 1)^3
 * nodes once and writes each once, the elements' shared nodes summed in a
 * fixed order (deterministic).  The library builds the blocks at mesh upload
 * when every element is affine-numbered with common strides, all elements
 * share one geometry kind, and the elements pair up into blocks (a
 * structured box with even element counts per side).  Modes:
 *   SEMX_BLOCKS_OFF   the per-element kernel;
 *   SEMX_BLOCKS_AUTO  blocks where they are built and measured faster than
 *                     the per-element kernel: irregular elements on the
 *                     stored-Gamma path (the default);
 *   SEMX_BLOCKS_ON    blocks wherever they are built (every geometry path).
 * The result equals the per-element pass up to the order of floating-point
 * summation.  *active (may be null) returns whether the next coloured FP32
 * force pass of this context, with its current geometry path, uses the
 * blocks.  SEMX_EINVAL for an unknown mode. */
#define SEMX_BLOCKS_OFF 0
#define SEMX_BLOCKS_AUTO 1
#define SEMX_BLOCKS_ON 2
int semx_set_blocks(semx_ctx *ctx, int mode, int *active);

/* f = -K u for every model: u_dev, f_dev device FP32 [nmodels][nglob][3].
 * f_dev is overwritten (not accumulated).  u_dev and f_dev must not overlap. */
int semx_apply_force(semx_ctx *ctx, const float *u_dev, float *f_dev);

/* Time step of the explicit Newmark loop (Sec. V-C).  Rejected with
 * SEMX_EUNSTABLE if dt exceeds 2/sqrt(lambda_max(M^{-1}K)) as estimated by
 * semx_max_eigenvalue() when that estimate has been made. */
int semx_set_dt(semx_ctx *ctx, double dt);

/* dt = courant * (min distance between adjacent GLL points) / (max P speed),
 * P speed sqrt((lambda + 2 mu)/rho) over all points of all models. */
int semx_cfl_dt(semx_ctx *ctx, double courant, double *dt_out);

/* Largest eigenvalue of M^{-1}K (model 0) by `iters` power iterations on the
 * device; the explicit scheme is stable for dt < 2/sqrt(lambda_max). */
int semx_max_eigenvalue(semx_ctx *ctx, int iters, double *lambda_max);

/* Point forces (Sec. V-C: Ricker source).  Source s acts at reference
 * coordinates xi[s][0..2] in [-1,1]^3 of element elem[s] with unit direction
 * dir[s][0..2] and time function stf[s][m], m = 0..nstf-1, sample m at
 * t_m = m dt (samples beyond nstf are 0).  It adds
 * stf[s][m] dir[s][c] l_i(xi) l_j(eta) l_k(zeta) to node (i,j,k) of elem[s]
 * (tensor-product interpolation weights, Sec. II-B).  Where several
 * sources reach one node their terms are summed in source order before the
 * node's force is updated, so the injection is deterministic.  With
 * nmodels > 1 the same sources act on every model.  nsrc = 0 removes all
 * sources. */
int semx_set_sources(semx_ctx *ctx, int nsrc, const int32_t *elem, const double *xi,
                     const double *dir, int64_t nstf, const float *stf);

/* Receivers: displacement interpolated at reference coordinates xi[r] of
 * element elem[r] (Sec. II-B interpolation) recorded after every step into
 * a device buffer [nmodels][nrec][3][nt_max]; steps beyond nt_max are not
 * recorded.  Clears earlier recordings. */
int semx_set_receivers(semx_ctx *ctx, int nrec, const int32_t *elem, const double *xi, int64_t nt_max);

/* u = v = 0, time index 0, a = M^{-1} f_src(t_0); clears seismograms. */
int semx_reset(semx_ctx *ctx);

/* Advance nsteps explicit Newmark steps (beta = 0, gamma = 1/2):
 *   u += dt v + dt^2/2 a;  v += dt/2 a;  f = -K u + f_src(t_{n+1});
 *   a = M^{-1} f;  v += dt/2 a;  record u at the receivers.
 * Requires mesh, model and dt.  If the watchdog interval is set, checks
 * every that many steps that the state is finite (SEMX_ENUMERIC otherwise). */
int semx_step(semx_ctx *ctx, int64_t nsteps);

/* Graph-captured time stepping: when chunk > 0, a semx_step() call of at
 * least 2 chunk + 2 steps with FP32 storage, no force timing, no
 * checkpoints and no watchdog records `chunk` steps once as a HIP graph and
 * launches it for the middle of the call (the first step of a fresh run and
 * the last, energy-tracked, step run directly).  The graph's kernels read
 * the time index from a device counter that the library sets before each
 * launch and advances after each step, so the results are bitwise those of
 * direct stepping; only the per-step launch cost goes.  The graph is built
 * per call and destroyed at its end.  chunk = 0 (the default) steps
 * directly.  SEMX_EINVAL outside [0, 4096]. */
int semx_set_graphs(semx_ctx *ctx, int chunk);

/* Current time index (number of steps taken since reset). */
int semx_time_index(semx_ctx *ctx, int64_t *it);

/* Copy the seismograms [nmodels][nrec][3][nt_max] (FP32) to out, which is a
 * device pointer if out_on_device != 0, else host memory (stream synchronised). */
int semx_read_seismograms(semx_ctx *ctx, float *out, int out_on_device);

/* Checkpoint: copy u, v, a ([nmodels][nglob][3] FP32, device pointers; any
 * may be NULL) and the time index out of / into the context.  Restoring a
 * state and stepping reproduces the uninterrupted run bitwise with
 * SEMX_ASM_COLORED. */
int semx_get_state(semx_ctx *ctx, float *u_dev, float *v_dev, float *a_dev, int64_t *it);
int semx_set_state(semx_ctx *ctx, const float *u_dev, const float *v_dev, const float *a_dev, int64_t it);

/* Discrete energy of the explicit Newmark scheme (Sec. II-B weak form with
 * the lumped GLL mass; Sec. V-C second-order Newmark), model 0, FP64 sums.
 * After semx_step() has brought the run to time index it = n+1:
 *   kinetic   = 1/2 (v^{n+1/2})^T M v^{n+1/2}, v^{n+1/2} the scheme's
 *               half-step velocity (u^{n+1} - u^n) / dt,
 *   potential = 1/2 (u^{n+1})^T K u^n,
 * so E^{n+1/2} = kinetic + potential, which the scheme conserves up to the
 * work of the sources: E^{n+1/2} - E^{n-1/2} = 1/2 (u^{n+1} - u^{n-1})^T f_src^n.
 *   source_work (may be NULL): that work summed over the steps since the
 *               last semx_reset(), semx_set_state() or semx_set_sources(),
 *               from the second of them on (E^{n+1/2} minus the first tracked
 *               E equals it in exact arithmetic).
 * The energy is evaluated on the last step of every semx_step() call (and on
 * the watchdog's steps): one extra read pass over v, u and f; the source
 * work is summed on every step over the source points only.
 * Errors: SEMX_ESTATE without mesh and model, or when no step was taken
 * since the last reset / new state (or since a call that moved the time
 * index otherwise, e.g. the adjoint's recomputation). */
int semx_energy(semx_ctx *ctx, double *kinetic, double *potential, double *source_work);

/* Watchdog: every `interval` steps (0 = off) semx_step checks that u and v
 * are finite, and (if max_energy > 0) that the discrete energy E^{n+1/2} of
 * semx_energy() stays below max_energy; a violation stops stepping and
 * returns SEMX_ENUMERIC. */
int semx_set_watchdog(semx_ctx *ctx, int64_t interval, double max_energy);

/* Forward checkpoints for the adjoint: with every > 0, semx_reset() and every
 * `every`-th semx_step() keep a copy of (u, v, a) on the device (3 vectors
 * per checkpoint, owned by the library).  0 turns checkpointing off and
 * frees the copies. */
int semx_set_checkpointing(semx_ctx *ctx, int64_t every);

/* Discrete adjoint of the explicit Newmark run (exact gradient of a
 * seismogram functional chi; the paper's weak form gives K linear in
 * lambda, mu and the lumped mass linear in rho).  gseis_dev holds
 * d chi / d seismogram, device FP32 [nmodels][nrec][3][nt_max] laid out like
 * semx_read_seismograms(); the first nt samples (steps 1..nt since reset)
 * are used, nt <= steps taken.  Writes d chi / d lambda, d chi / d mu and
 * d chi / d rho per element-local point to device FP64 arrays
 * [nmodels][nspec][n^3] (user element order, overwritten).  The adjoint runs
 * in FP32 with exact power-of-two normalisation of the adjoint source and of
 * the forward field; only the final rescaling is FP64, so gradients of
 * physically tiny misfits do not underflow.  Recomputes the
 * forward segment by segment from the checkpoints (coloured assembly makes
 * the recomputation bitwise equal to the first pass); the context's own
 * state is restored before return.  Needs semx_set_checkpointing() before the
 * semx_reset() that started the forward run. */
int semx_adjoint(semx_ctx *ctx, const float *gseis_dev, int64_t nt, double *g_lambda_dev,
                 double *g_mu_dev, double *g_rho_dev);

/* ---------------------------------------------------------------------------
 * FP64 storage.  The same operator (Sec. II-B) and time loop (Sec. V-C) with
 * state vectors, geometry map Gamma, lambda W, mu W, M^{-1}, the force and
 * all sums in FP64, for runs that must agree with an FP64 reference to FP64
 * rounding and for finite-difference checks.  Contractions run on the
 * vector units (SEMX_C_F32 is the only valid contraction setting; other
 * settings give SEMX_EINVAL); coloured and atomic assembly both work, the
 * atomic one with FP64 atomic adds.  In this mode the FP32 entry points that
 * move state vectors or seismograms (semx_apply_force, semx_get_state,
 * semx_set_state, semx_read_seismograms) and the adjoint
 * (semx_set_checkpointing, semx_adjoint) return SEMX_ESTATE; the _f64
 * variants below take their place.  Everything else (mesh, model, dt,
 * receivers, reset, step, energy, watchdog) works unchanged.
 * ------------------------------------------------------------------------- */

/* Select SEMX_F32 or SEMX_F64 (default SEMX_F32).  Allowed before
 * semx_upload_model() only (SEMX_ESTATE after it, and while checkpointing is
 * on); SEMX_EINVAL for an unknown value or, for SEMX_F64, while a
 * matrix-core contraction is selected. */
int semx_set_storage(semx_ctx *ctx, int storage);

/* f = -K u in FP64: u_dev, f_dev device FP64 [nmodels][nglob][3], f
 * overwritten, no overlap.  Needs SEMX_F64 storage. */
int semx_apply_force_f64(semx_ctx *ctx, const double *u_dev, double *f_dev);

/* semx_set_sources() with an FP64 time function stf [nsrc][nstf] (used
 * exactly by SEMX_F64 storage, rounded to FP32 for SEMX_F32). */
int semx_set_sources_f64(semx_ctx *ctx, int nsrc, const int32_t *elem, const double *xi,
                         const double *dir, int64_t nstf, const double *stf);

/* FP64 seismograms [nmodels][nrec][3][nt_max] to device (out_on_device != 0)
 * or host memory.  Needs SEMX_F64 storage. */
int semx_read_seismograms_f64(semx_ctx *ctx, double *out, int out_on_device);

/* FP64 checkpoint copies of u, v, a (device [nmodels][nglob][3]; NULL skips
 * one in get_state).  Needs SEMX_F64 storage. */
int semx_get_state_f64(semx_ctx *ctx, double *u_dev, double *v_dev, double *a_dev, int64_t *it);
int semx_set_state_f64(semx_ctx *ctx, const double *u_dev, const double *v_dev, const double *a_dev,
                       int64_t it);

/* -------------------------------------------------------------------------
 * Acoustic physics.  The paper selects its equal-accuracy (h, p) pairs with
 * an acoustic solver in a homogeneous medium (Sec. V-C).  With
 * SEMX_ACOUSTIC the context solves for a scalar field p,
 *     (1/kappa) p_tt = div(rho^-1 grad p) + sources,
 * discretised as the elastic operator is (Sec. II-B GLL weak form): lumped
 * mass M_g = sum w_i w_j w_k det J / kappa, force f = -K p with
 * K_gh = sum w_i w_j w_k det J rho^-1 grad phi_g . grad phi_h, the same
 * explicit Newmark loop.  Every state vector, force vector and seismogram
 * then has ONE component per node: u, v, a, f are [nmodels][nglob] and
 * seismograms [nmodels][nrec][1][nt_max] in the entry points above
 * (semx_apply_force, semx_get_state, semx_set_state, semx_read_seismograms,
 * semx_max_eigenvalue, semx_energy, semx_step, semx_cfl_dt with
 * c = sqrt(kappa/rho)).  semx_set_sources() ignores dir (it may be NULL):
 * a source adds stf[s][m] l_q(x_s) to the nodes of its element.  Both
 * assemblies, both geometry paths and NGLL 2..16 are supported; the
 * matrix-core contractions, FP64 storage and the adjoint are elastic only
 * (SEMX_EINVAL).
 * ------------------------------------------------------------------------- */
#define SEMX_ELASTIC 0   /* vector displacement, isotropic elasticity (default) */
#define SEMX_ACOUSTIC 1  /* scalar field, acoustic wave equation */

/* Select the physics.  Allowed before a model is uploaded and before
 * sources are set (SEMX_ESTATE otherwise, or while checkpointing is on:
 * source weights are stored per field component); SEMX_EINVAL for an
 * unknown value or, for SEMX_ACOUSTIC, with FP64 storage or a matrix-core
 * contraction.  Receivers may be set before it (their seismogram buffer is
 * re-sized). */
int semx_set_physics(semx_ctx *ctx, int physics);

/* Acoustic model per element-local point, FP64 host arrays
 * [nmodels][nspec][n^3]: bulk modulus kappa = rho c^2 and density rho, both
 * > 0 (SEMX_EINVAL otherwise).  The library forms w_i w_j w_k det J / rho
 * (FP32) and M_g = sum w_i w_j w_k det J / kappa (FP64 accumulate, FP32
 * M^{-1}).  SEMX_ESTATE unless the physics is SEMX_ACOUSTIC (and
 * semx_upload_model returns SEMX_ESTATE while it is).  Resets the time loop. */
int semx_upload_model_acoustic(semx_ctx *ctx, int nmodels, const double *kappa, const double *rho);

/* The library's GLL nodes (ascending) and weights for ngll points
 * (Sec. II-B), FP64, into host arrays of ngll entries; no context, no GPU
 * work.  For callers that place sources or receivers at nodes or weight them
 * by quadrature (e.g. a plane source on an element face).  SEMX_EINVAL
 * unless 2 <= ngll <= 16 and both pointers are non-NULL. */
int semx_gll(int ngll, double *xi, double *w);

/* Kernel timing.  With stride k > 0, every k-th force pass (one
 * semx_apply_force, or the force part of one time step: all its colour
 * launches back to back; the first, then k, 2k, ... counted from this call)
 * is bracketed by one pair of HIP events recorded on the context stream; 0
 * turns timing off, a negative stride is SEMX_EINVAL.  semx_force_timing()
 * synchronises the stream, returns the number of force-kernel launches
 * inside the timed passes and their summed event-measured duration in
 * milliseconds since the last read (so the average launch includes the
 * short gaps between launches, not the latency of an event per launch), and
 * clears the record. */
int semx_set_timing(semx_ctx *ctx, int stride);
int semx_force_timing(semx_ctx *ctx, int64_t *launches, double *total_ms);

/* Streaming reference: copy nbytes (a positive multiple of 16) between two
 * device buffers the library allocates and frees, reps times, with its own
 * copy kernel (one 16-byte element per lane, non-temporal) on the context
 * stream;
 * returns the read+write bandwidth 2 nbytes reps / time in GB/s (HIP
 * events).  A measured ceiling for HBM-bound kernels beside the published
 * peak.  SEMX_ENOMEM if the two buffers do not fit. */
int semx_stream_bandwidth(semx_ctx *ctx, int64_t nbytes, int reps, double *gbps);

/* Access-pattern reference for the force pass (Sec. II-B operator, Sec. IV-D
 * fused traversal): runs, reps times after one warm-up pass, the memory
 * skeleton of the FP32 per-element force pass that semx_apply_force and
 * semx_step launch with coloured assembly (one lane per point up to NGLL
 * 10, one lane per column from 11): the same colour launches, grid,
 * block-to-element mapping and per-point loads and stores (node numbers,
 * geometry, material, the gather of u, the first-touch bits, the read of f
 * where the point is not first and the store of f) without the
 * contractions, the stress arithmetic and the slice barriers.  The clearing of f that a pass
 * without first-touch coverage needs is not included.  Returns the average
 * milliseconds per pass (HIP events on the context stream); the force pass
 * cannot take less time than its skeleton.
 *   u_dev: device [nmodels][nglob][3] FP32, read only.
 *   f_dev: device [nmodels][nglob][3] FP32, overwritten with meaningless
 *          values; must not overlap u_dev.
 * Errors: SEMX_ESTATE without mesh and model, or unless the context runs the
 * FP32 elastic per-element kernels (FP32 storage and contraction, coloured
 * assembly); SEMX_EINVAL for null pointers,
 * overlapping buffers or reps <= 0. */
int semx_force_skeleton(semx_ctx *ctx, const float *u_dev, float *f_dev, int reps, double *ms_per_pass);

/* ---------------------------------------------------------------------------
 * Surrogate network: a multilayer perceptron that maps model parameters to
 * receiver seismograms, trained on SEM runs of this library (the SEM solve
 * stays the fallback and the reference for its error).  Layer l computes
 * Z_l = H_l W_l^T + b_l with W_l [out][in]; hidden layers apply SiLU, the
 * last layer is linear.  GEMMs run on BF16 matrix cores with FP32
 * accumulation from a BF16 copy of FP32 master weights; losses and the
 * optimiser are FP32.  Parameters are packed W_1, b_1, W_2, b_2, ...
 * (row-major, FP32).  All device pointers are caller-owned; work is ordered
 * on the stream given at creation.
 * ------------------------------------------------------------------------- */
typedef struct semx_mlp semx_mlp;

/* widths[0..nlayers]: input width, hidden widths, output width; batches up
 * to max_batch rows.  Parameters start at zero (set them before use). */
int semx_mlp_create(semx_mlp **out, int nlayers, const int *widths, int max_batch, void *hip_stream);
int semx_mlp_destroy(semx_mlp *net);
const char *semx_mlp_last_error(const semx_mlp *net);
int semx_mlp_num_params(semx_mlp *net, int64_t *nparams);
/* host FP32 parameter vector in/out; set also clears the Adam moments */
int semx_mlp_set_params(semx_mlp *net, const float *params);
int semx_mlp_get_params(semx_mlp *net, float *params);
int semx_mlp_get_grads(semx_mlp *net, float *grads);
/* y_dev [batch][width_out] = net(x_dev [batch][width_in]); keeps the
 * activations for semx_mlp_backward (x_dev must stay alive until then) */
int semx_mlp_forward(semx_mlp *net, const float *x_dev, int batch, float *y_dev);
/* Allocation-free inference forward, for callers that cannot allocate
 * device memory: code under HIP graph capture and tight serving loops (the
 * surrogate's batched inference).  Same result as semx_mlp_forward (the same
 * GEMM kernels and accumulation order), but the hidden activations live in a
 * workspace of 16 MB that the library holds in static device memory on each
 * GPU it runs on, not in the network's buffers, and nothing is kept for
 * semx_mlp_backward.  The call allocates and frees nothing.
 *   x_dev: device FP32 [batch][widths[0]], read only; y_dev: device FP32
 *   [batch][widths[nlayers]], overwritten.  batch is not limited by
 *   max_batch, only by the workspace: batch x (widest hidden layer) <= 2^21
 *   floats (e.g. 4096 x 512), else SEMX_EINVAL.
 * Every call on one GPU uses that GPU's single workspace: calls that overlap
 * on one GPU (several streams, several networks, several host threads) race
 * and must be serialised by the caller.  The workspace keeps the last call's
 * activations; nothing in it needs to start at zero.  (semx_mlp_create
 * resolves the workspace's device address and fails with SEMX_EHIP if it
 * cannot.) */
int semx_mlp_forward_noalloc(semx_mlp *net, const float *x_dev, int batch, float *y_dev);
/* parameter gradient of a scalar loss L given dy_dev = dL/dy (overwrites the
 * gradient buffer) for the batch of the last semx_mlp_forward call */
int semx_mlp_backward(semx_mlp *net, const float *dy_dev, int batch);
/* mean squared error over n values: loss (FP64, host, may be NULL) and
 * dy_dev = dloss/dy (may be NULL) */
int semx_mlp_mse(semx_mlp *net, const float *y_dev, const float *t_dev, int64_t n, float *dy_dev, double *loss);
/* one Adam step (bias-corrected, step >= 1) on the FP32 master parameters;
 * refreshes the BF16 working copy */
int semx_mlp_adam(semx_mlp *net, float lr, float beta1, float beta2, float eps, int64_t step);

/* Surrogate inference around the network (no counterpart in the paper; the
 * learned surrogate's input normalisation, ensemble mean and error
 * indicator), on the network's stream:
 * semx_mlp_affine: y_dev[r][c] = scale_dev[c] * x_dev[r][c] + shift_dev[c]
 *   for r < rows, c < cols (device FP32, row-major; x_dev and y_dev may be
 *   the same buffer).  Normalises inputs ((x - mean) / std as scale 1/std,
 *   shift -mean/std) and maps normalised outputs back to physical units. */
int semx_mlp_affine(semx_mlp *net, const float *x_dev, int64_t rows, int cols, const float *scale_dev,
                    const float *shift_dev, float *y_dev);
/* semx_mlp_ensemble: preds_dev [members][rows][cols] are the members'
 *   normalised predictions.  mean_dev [rows][cols] = scale * (mean over the
 *   members) + shift (physical units); indicator_dev [rows] = || scale * s ||
 *   / || mean_dev row || with s the unbiased standard deviation over the
 *   members (0 for one member), norms over the row accumulated in FP64 in a
 *   fixed order.  The indicator is the surrogate's fallback criterion.
 *   SEMX_EINVAL for a null pointer, members < 1 or cols < 1. */
int semx_mlp_ensemble(semx_mlp *net, const float *preds_dev, int members, int64_t rows, int cols,
                      const float *scale_dev, const float *shift_dev, float *mean_dev, float *indicator_dev);

#ifdef __cplusplus
}
#endif
#endif /* SEMX_H */
