/*
 * reco.h - C ABI of the MI355X wavelet-multigrid (WMG) preconditioned Krylov
 * CT reconstruction library (libreco.so).
 *
 * Problem (Section 2.1, eq. sys / eq. sys_ne): W x = b with x an n x n image on
 * [-1,1]^2 (pixel (ix,iy) at flat index iy*n + ix, y growing with iy) and b the
 * sinogram of m parallel-beam directions theta_k = k*pi/m, k = 0..m-1, times nb
 * detector bins of width one pixel centred on the origin (flat index k*nb + j).
 * Ray (k, j) is the line p.(cos theta_k, sin theta_k) = (j - (nb-1)/2) * 2/n and
 * w_ij is the exact length of ray i inside pixel j (a ray lying on a pixel edge
 * gives half of its length to each side), or, for geometries created with
 * RECO_PROJ_JOSEPH, the weight of Joseph's interpolation kernel (Section 2.1).
 * Either W is applied matrix-free, and its transpose is applied exactly.  Krylov methods solve the normal
 * equations (W^T W + lambda I) x = W^T b (eq. sys_ne, eq. sys_reg).
 *
 * Conventions for every entry point:
 *  - Array pointers are caller-owned HIP device memory, contiguous, with the
 *    element type selected by the geometry's dtype (float for RECO_F32,
 *    double for RECO_F64).  Images are [n][n], sinograms [m][nb].
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls that only enqueue work return before it finishes.
 *  - Arguments are validated before any launch; an invalid argument returns
 *    RECO_EINVAL and enqueues nothing.  HIP failures return RECO_EDEVICE.
 *    No call aborts or throws; reco_last_error() gives the thread's last
 *    message.
 *  - The library owns geometry tables, the packet diagonal and solver
 *    workspaces; it never frees caller memory.
 */
#ifndef RECO_H
#define RECO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t reco_status;
#define RECO_OK         0   /* success */
#define RECO_PENDING    1   /* request queued or running (reco_poll) */
#define RECO_ENOTCONV   2   /* iteration cap reached before tol; x holds the last iterate */
#define RECO_EINVAL    -1   /* invalid argument; nothing was enqueued */
#define RECO_ENOMEM    -2   /* device or host allocation failed */
#define RECO_EDEVICE   -3   /* a HIP call failed, or a device-side reduction never
                               received its partial sums (bounded wait) */
#define RECO_ENUMERIC  -4   /* a non-finite scalar appeared (e.g. NaN in b) */
#define RECO_ENOTFOUND -5   /* unknown ticket */

#define RECO_F32 0
#define RECO_F64 1

#define RECO_PRECOND_NONE 0
#define RECO_PRECOND_WMG  1   /* additive WMG, packet-diagonal coarsest solves */
#define RECO_PRECOND_WMG_HYBRID 2   /* the hybrid WMG cycle with exact coarsest
                                       solves (GMRES and BiCGStab only; see
                                       reco_wmg_hybrid_apply) */

/* Projection kernels (reco_geometry_desc.projector). */
#define RECO_PROJ_EXACT  0   /* exact ray-pixel intersection lengths */
#define RECO_PROJ_JOSEPH 1   /* Joseph's kernel (Section 2.1): along the image
                                axis closest to the ray, linear interpolation
                                between the two nearest pixel centres of each
                                row (column) crossed, times the ray length per
                                row (column), h / max(|cos|, |sin|) */

typedef struct reco_geometry_s* reco_geometry;
typedef struct reco_server_s* reco_server;

/* Geometry description.  n >= 2; n_angles >= 1; n_bins >= 1; the detector bins
 * are one pixel wide.  wmg_levels = ell >= 1 levels of the WMG hierarchy
 * (Section 3.1.3); the packet transform has L = ell - 1 levels, needs
 * n % 2^L == 0 and L <= 5.  dtype is RECO_F32 or RECO_F64.  Size limits (the
 * kernels use 32-bit byte offsets): (n + 32) * (n + 8) and n_angles * n_bins
 * elements each below 2^31 bytes, i.e. n <= 23150 in RECO_F32 (16364 in
 * RECO_F64); larger descriptions are rejected with RECO_EINVAL. */
typedef struct {
  int32_t n;
  int32_t n_angles;
  int32_t n_bins;
  int32_t wmg_levels;
  int32_t dtype;
  int32_t projector;  /* RECO_PROJ_EXACT (0) or RECO_PROJ_JOSEPH */
} reco_geometry_desc;

/* Solver options.  tol > 0 is the relative residual target (normal-equation
 * residual ||W^T (b - W x) - lambda x|| / ||W^T b|| for CGLS and GMRES; the
 * relative size of the last correction for SIRT).  max_iter >= 1.  restart is
 * the GMRES restart length (1..64).  lambda >= 0 is the Tikhonov weight
 * (CGLS/GMRES).  precond is RECO_PRECOND_NONE, RECO_PRECOND_WMG or (GMRES and
 * BiCGStab) RECO_PRECOND_WMG_HYBRID.
 * check_every is the host poll period in iterations (0 = adaptive).
 * history, if not NULL, receives up to history_cap relative residuals (host
 * memory).  fixed_iters > 0 runs exactly that many iterations, ignoring tol. */
typedef struct {
  double tol;
  int32_t max_iter;
  int32_t restart;
  double lambda;
  int32_t precond;
  int32_t check_every;
  double* history;
  int32_t history_cap;
  int32_t fixed_iters;
} reco_solve_opts;

/* Solver result.  iters = iterations done, matvecs = applications of W^T W
 * (one W plus one W^T each), relres = final relative residual,
 * status = RECO_OK / RECO_ENOTCONV / RECO_ENUMERIC, elapsed_ms = wall time of
 * the call (or, from reco_poll, of the request from admission to completion). */
typedef struct {
  int32_t iters;
  int32_t matvecs;
  double relres;
  reco_status status;
  int32_t reserved;
  double elapsed_ms;
} reco_solve_info;

/* Message of the calling thread's last failure ("" if none).  The pointer
 * stays valid until the thread's next failing call. */
const char* reco_last_error(void);

/* Library version string. */
const char* reco_version(void);

/* Build the geometry: per-angle tables (Section 2.1) and, for ell >= 1, the
 * packet diagonal d_q = ||W H_L^T e_q||^2 used by the WMG coarsest solves
 * (the Galerkin operators of eq. galerkin restricted to their diagonal in the
 * packet basis; Section 3.1.3).  Work is enqueued on `stream` and the call
 * waits for it.  *out receives an immutable handle that any stream may use
 * concurrently.  Errors: RECO_EINVAL (bad description), RECO_ENOMEM,
 * RECO_EDEVICE. */
reco_status reco_create_geometry(const reco_geometry_desc* desc, void* stream,
                                 reco_geometry* out);

/* Free a geometry.  The caller must ensure no work using it is in flight. */
reco_status reco_destroy_geometry(reco_geometry g);

/* Copy the geometry's parameters into *desc. */
reco_status reco_geometry_get_desc(reco_geometry g, reco_geometry_desc* desc);

/* Copy the packet diagonal (without lambda) into the HOST array d[n][n],
 * float64, in the quadrant layout of the full Haar packet transform: one level
 * maps an s x s block to quadrants [[LL, LH], [HL, HH]] (eq. 1of4 - 4of4, LH =
 * low-pass along y, high-pass along x) and each quadrant is split again,
 * L times.  Synchronous. */
reco_status reco_packet_diagonal(reco_geometry g, double* d_host);

/* Count the nonzero weights of W (the update count of one projection) into
 * *nnz.  Synchronous; runs a counting pass on the GPU. */
reco_status reco_count_nnz(reco_geometry g, void* stream, int64_t* nnz);

/* b = W x (Section 2.1, eq. sys).  x: image [n][n]; b: sinogram [m][nb]
 * (overwritten).  Asynchronous on `stream`. */
reco_status reco_project(reco_geometry g, const void* x, void* b, void* stream);

/* x = W^T b, the exact transpose of reco_project's matrix (Section 2.1).
 * b: sinogram [m][nb]; x: image [n][n] (overwritten).  Asynchronous. */
reco_status reco_backproject(reco_geometry g, const void* b, void* x, void* stream);

/* z = M^-1 r with the additive WMG preconditioner in packet-diagonal form,
 * M^-1 = H_L^T diag(1/(d + lambda)) H_L (Section 3.1; 1/0 := 0).
 * r, z: images [n][n]; they may not alias.  Asynchronous. */
reco_status reco_wmg_apply(reco_geometry g, const void* r, void* z, double lambda,
                           void* stream);

/* z = M^-1 r with the paper's hybrid wavelet multigrid cycle (Section 3.1.2,
 * hybrid variant, recursed over the wmg_levels - 1 levels of Section 3.1.3)
 * on K = W^T W + lambda I: at each node of the recursion the LL subproblem is
 * treated first, the residual is updated with the node's Galerkin operator
 * (eq. galerkin), and the LH, HL and HH subproblems are treated with that
 * residual; the coarsest subproblems (one Haar packet over all 2^L x 2^L
 * tiles) are solved exactly by Cholesky (Section 4.1), the factors being
 * built in float64 on first use for each lambda and kept with the geometry.
 * Reading for singular coarsest blocks (unseen pixels, too few rays): pivots
 * at most 1e-12 of the largest coarsest diagonal entry are dropped (zero
 * correction).  The cycle is not symmetric, so CGLS rejects it.  Limits:
 * 2 <= wmg_levels <= 4, at most 4096 unknowns per coarsest block and 8 GiB of
 * factors (16 n^4 / 4^L bytes), else RECO_EINVAL.  r, z: images [n][n] (no
 * aliasing).  Synchronous. */
reco_status reco_wmg_hybrid_apply(reco_geometry g, const void* r, void* z, double lambda,
                                  void* stream);

/* CGLS on (W^T W + lambda I) x = W^T b (a Krylov method of Section 2.3.1),
 * preconditioned by M^-1 when opts->precond == RECO_PRECOND_WMG.
 * b: sinogram; x: image, output
 * (the solve starts from x = 0).  Synchronous: returns when done.
 * Returns RECO_OK, RECO_ENOTCONV (x = last iterate), RECO_ENUMERIC, or an
 * error; *info (may be NULL) receives the counts and final relres. */
reco_status reco_solve_cgls(reco_geometry g, const void* b, void* x,
                            const reco_solve_opts* opts, reco_solve_info* info,
                            void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): reco_solve_cgls with every
 * solver buffer (residuals, direction, padded image copies, reduction
 * partials, device state, residual history) carved from one fixed device
 * array of RECO_NOALLOC_SCRATCH_BYTES that the library holds on each device
 * it runs on until the process ends, and the host copy of the solver state
 * on the caller's stack.  The call makes no device or host allocation; the
 * caller passes b and x as for reco_solve_cgls and gets the same result.
 * Limits: the geometry's CGLS buffers plus 8 bytes per history entry
 * (max_iter, or fixed_iters) must fit in the array (about 4 * (2 M + 4 N)
 * bytes for RECO_F32, twice that for RECO_F64: a 1024 x 1024 image with
 * 1448 angles of 1449 bins fits), else RECO_EINVAL with the sizes in the
 * message and nothing enqueued; per-kernel timing (reco_timing_enable) must
 * be off, else RECO_EINVAL.  All calls on one device share the array, so
 * calls that overlap on one device (other threads, other streams) race; the
 * array keeps the last call's contents, and each call re-initialises what
 * the kernels rely on before its first launch.  Synchronous. */
#define RECO_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
reco_status reco_solve_cgls_noalloc(reco_geometry g, const void* b, void* x,
                                    const reco_solve_opts* opts, reco_solve_info* info,
                                    void* stream);

/* GMRES(restart) on the right-preconditioned system (W^T W + lambda I) M^-1 u
 * = W^T b, x = M^-1 u (eq. sys_prec, second form).  Otherwise as
 * reco_solve_cgls. */
reco_status reco_solve_gmres(reco_geometry g, const void* b, void* x,
                             const reco_solve_opts* opts, reco_solve_info* info,
                             void* stream);

/* BiCGStab (the paper's primary Krylov solver, Section 2.3.1), right
 * preconditioned on (W^T W + lambda I) M^-1 u = W^T b, x = M^-1 u (eq.
 * sys_prec): van der Vorst's recursion with shadow vector r_0 = W^T b,
 * relres = ||r_k|| / ||r_0||, two matvecs (W and W^T each) per iteration.
 * opts->restart is ignored.  A breakdown (rho = 0, <r_0, v> = 0, or omega = 0
 * before tol is met) returns RECO_ENOTCONV with x = the last iterate.
 * Otherwise as reco_solve_cgls. */
reco_status reco_solve_bicgstab(reco_geometry g, const void* b, void* x,
                                const reco_solve_opts* opts, reco_solve_info* info,
                                void* stream);

/* SIRT, x <- x + C W^T R (b - W x) with R, C the inverse row and column sums
 * of W (eq. sys_sirt, eq. sirt_it; 1/0 := 0).  lambda and precond are
 * ignored.  Otherwise as reco_solve_cgls. */
reco_status reco_solve_sirt(reco_geometry g, const void* b, void* x,
                            const reco_solve_opts* opts, reco_solve_info* info,
                            void* stream);

/* Solve `count` independent CGLS problems (each with its own geometry, all of
 * dtype RECO_F32) together: every Krylov phase of all unfinished problems is
 * one launch over a shared work list, and chunks of iterations are captured
 * once in a HIP graph and replayed until every problem has converged.
 * geoms[i], b[i], x[i] describe problem i; opts[i] its options (precond,
 * tol, max_iter, lambda; history ignored); info[i] receives its result.
 * Each problem's result equals what reco_solve_cgls computes for it alone.
 * Synchronous. */
reco_status reco_solve_batch(int32_t count, const reco_geometry* geoms,
                             const void* const* b, void* const* x,
                             const reco_solve_opts* opts, reco_solve_info* info,
                             void* stream);

/* Serving: submitted requests are admitted in arrival order while their
 * geometry and Krylov state fit in hbm_budget_bytes and fewer than max_slots
 * run.  Requests are served in two tiers by the cost of one iteration
 * (n^2 * n_angles below or at least 1024^2 * 512), each with a scheduler
 * thread and a stream of its own: the small tier advances all its running
 * requests together (continuous batching; one batched CGLS iteration per
 * tick, requests join and leave between ticks), the large tier runs one
 * request at a time.  Geometries are created on first use (large ones on a
 * builder thread and stream of their own) and cached by description; the
 * server uses three streams.  Each result equals what reco_solve_cgls
 * computes for the request alone.  ENOMEM from reco_poll: the request alone
 * needs more than the budget. */
reco_status reco_server_create(size_t hbm_budget_bytes, int32_t max_slots,
                               reco_server* out);

/* Stop the scheduler (running requests are finished first) and free it. */
reco_status reco_server_destroy(reco_server s);

/* Queue a request: reconstruct x (device [n][n]) from b (device [m][nb]) for
 * the geometry `desc` (dtype RECO_F32) with `opts` (CGLS; history ignored).
 * b and x must stay valid until reco_poll reports a terminal status.
 * *ticket identifies the request. */
reco_status reco_submit(reco_server s, const reco_geometry_desc* desc, const void* b,
                        void* x, const reco_solve_opts* opts, uint64_t* ticket);

/* State of a request: RECO_PENDING while queued or running, else the final
 * status (RECO_OK, RECO_ENOTCONV, RECO_ENUMERIC, RECO_ENOMEM ...) with *info
 * filled.  t_submit_admit_done (may be NULL) receives the submit, admit and
 * completion times in seconds on the library's steady clock (-1 if not yet).
 * Terminal results remain readable until the server is destroyed. */
reco_status reco_poll(reco_server s, uint64_t ticket, reco_solve_info* info,
                      double t_submit_admit_done[3]);

/* Per-kernel timing (profiling aid).  While enabled, every launch of a timed
 * kernel family is bracketed by HIP events recorded on its launch stream.
 * Families: 0 forward projector, 1 backprojector, 2 WMG apply, 3 CGLS vector
 * update, 4 packet-diagonal setup, 5 image padding/transposition, 6 one replay
 * of a batched-iteration graph (reco_solve_batch and the server; the kernels
 * inside a graph are not timed individually).
 * reco_timing_read waits for the recorded events and returns the number of
 * timed launches and their summed duration in milliseconds since the last
 * reset.  Disabled by default. */
reco_status reco_timing_enable(int32_t on);
reco_status reco_timing_read(int32_t family, int64_t* launches, double* total_ms);
reco_status reco_timing_reset(void);

/* Current time of the library's steady clock in seconds (the clock of
 * reco_poll's timestamps). */
double reco_clock(void);

#ifdef __cplusplus
}
#endif

#endif /* RECO_H */
