/*
 * ridc.h -- C ABI of the MI355X (gfx950) semi-implicit RIDC library.
 *
 * Semi-implicit Revisionist Integral Deferred Correction (RIDC-FBE) of Ong, Melfi and
 * Christlieb, "Parallel Semi-Implicit Time Integrators" (arXiv:1209.4297), for
 *
 *     u_t = f_E(u) + f_I(u),     f_I(u) = nu * Lap_h u      (section II, eq. ode; section IV)
 *
 * on a uniform finite-difference grid.  Level 0 (the predictor) is first-order IMEX
 * forward-backward Euler (section II, eq. imex_diffusion; section III-B, eq. pred).  Level
 * j = 1..P-1 (a corrector) is an IMEX Euler step on the error equation plus the (j+1)-node
 * Lagrange quadrature of f along level j-1 (section III-C, eq. corr and the quadrature rule that
 * follows it).  All P levels advance together as the lagged pipeline of section III (Fig. 1):
 * at pipeline step s level j computes time index s - j(j+1)/2 (the start-up wait of section
 * III-E), so an integration of nt steps takes nt + P(P-1)/2 pipeline steps.  Every level starts
 * from u0 (section III-E, Fig. 2).  The result is the top level at t = nt*dt.
 *
 * Conventions shared by every entry point:
 *  - Every function returns an int status: RIDC_OK (0) or a negative RIDC_E_* code.  No C++
 *    exception crosses the ABI.  ridc_last_error() gives a message for the calling thread.
 *  - Arrays are contiguous FP64 in device memory (hipMalloc'd or torch CUDA tensors).  1D: n
 *    values.  2D: n*n values, row-major u[iy*n + ix].  Dirichlet grids hold the interior
 *    unknowns only (x_i = i*h, i = 1..n, h = length/(n+1), zero ghosts); periodic grids hold
 *    x_i = i*h, i = 0..n-1, h = length/n.
 *  - The caller owns every array it passes; the handle owns its level rings, transform
 *    matrices, weights and workspaces, and frees them in ridc_destroy.
 *  - Work is enqueued asynchronously on the HIP stream given to ridc_create (NULL = the null
 *    stream).  Input arrays must stay valid until the stream reaches the work; the caller
 *    synchronises (or calls ridc_sync) before reading outputs.
 *  - Device-side failures (a non-finite result) are reported by ridc_sync.
 */
#ifndef RIDC_H
#define RIDC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------------------ */
#define RIDC_OK             0
#define RIDC_E_INVAL       -1   /* bad argument: n < 2, dt <= 0, order outside 1..12, ...   */
#define RIDC_E_UNSUPPORTED -2   /* valid but not implemented (e.g. 2D periodic)            */
#define RIDC_E_NOMEM       -3   /* device allocation failed                                 */
#define RIDC_E_HIP         -4   /* a HIP runtime call failed                                */
#define RIDC_E_NONFINITE   -5   /* the result holds a NaN or Inf                            */
#define RIDC_E_STATE       -6   /* call out of order (e.g. ridc_read before the last step)  */

#define RIDC_MAX_ORDER 12       /* section III-E: orders 8 and 12 are usable in FP64         */

/* ---- problem description ------------------------------------------------------------------ */
typedef enum { RIDC_BC_PERIODIC = 0, RIDC_BC_DIRICHLET0 = 1 } ridc_bc;

/* Explicit (non-stiff) term f_E, section II: f^N.                                            */
typedef enum {
  RIDC_FE_NONE = 0,          /* f_E = 0                                                       */
  RIDC_FE_ADVECT_C2 = 1,     /* f_E = -a (u_{i+1} - u_{i-1}) / (2h), 1D only                  */
  RIDC_FE_LOGISTIC = 2,      /* f_E = u (1 - u), pointwise                                     */
  RIDC_FE_ADVECT_UPWIND = 3, /* f_E = -a (u_i - u_{i-1}) / h if a >= 0, else -a (u_{i+1} - u_i)
                                / h: first-order upwind (section IV-A), 1D only               */
  RIDC_FE_BURGERS = 4        /* f_E = -(1/2)(F_{i+1/2} - F_{i-1/2}) / h, F_{i+1/2} =
                                (u_{i+1}^2 + u_i^2)/2: the numerical flux of section IV-B, 1D */
} ridc_fe_kind;

/* Arithmetic of the implicit solve.  Quadrature sums and level differences are FP64 always.  */
typedef enum {
  RIDC_PREC_FP64 = 0,          /* every operation in FP64                                     */
  RIDC_PREC_FP32_REFINE = 1,   /* 2D: FP32 MFMA transforms, increment form, one FP64 residual
                                  refinement                                                  */
  RIDC_PREC_BF16X3_REFINE = 2  /* 2D: split-BF16 (hi/lo, three products) MFMA transforms with
                                  FP32 accumulation, increment form, one FP64 refinement      */
} ridc_prec;

typedef struct {
  int32_t dim;       /* 1 or 2                                                                */
  int32_t bc;        /* ridc_bc; 2D supports RIDC_BC_DIRICHLET0 only                          */
  int64_t n;         /* unknowns per axis, >= 2                                               */
  double length;     /* domain length per axis, > 0                                           */
  int32_t fe_kind;   /* ridc_fe_kind                                                           */
  int32_t order;     /* P = number of levels, 1..RIDC_MAX_ORDER (1 = plain IMEX Euler)        */
  double a;          /* advection speed (RIDC_FE_ADVECT_C2)                                   */
  double nu;         /* diffusion coefficient, >= 0; f_I = nu * Lap_h                         */
  double dt;         /* uniform time step, > 0 (section III-C: one weight table)              */
  int32_t prec;      /* ridc_prec; 1D always computes in FP64                                 */
  int32_t reserved;  /* must be 0                                                              */
} ridc_problem;

typedef struct ridc_handle ridc_handle;   /* opaque; owned by the library                     */

/* ---- extensions: a nonlinear stiff term and IMEX Runge-Kutta levels (1D) ------------------- */
/* Stiff term f^S = nu Lap_h u + kappa g(u).  With a reaction g the implicit equation of every
 * stage, y - tau f^S(y) = rhs, is nonlinear and is solved by Newton's method (section III-B,
 * after eq. pred), each iterate a tridiagonal solve with the Jacobian
 * I - tau (nu D2 + kappa diag g'(y)).                                                         */
typedef enum {
  RIDC_FS_DIFFUSION = 0,     /* g = 0 (linear: one solve per stage)                           */
  RIDC_FS_LOGISTIC = 1,      /* g(u) = u (1 - u)                                              */
  RIDC_FS_CUBIC = 2          /* g(u) = u - u^3                                                */
} ridc_fs_kind;

/* IMEX pair of one level (section II; section III-D, Thm 2).  The predictor takes one step of
 * its pair; a corrector applies its pair to the integral form of the error equation (section
 * III-A), the previous level interpolated through S_j = p_0 + ... + p_j stored nodes (the
 * section III-C window widened to S_j nodes), so level j has order S_j.                       */
typedef enum {
  RIDC_PAIR_FBE = 0,         /* forward-backward Euler as a two-stage pair, order 1           */
  RIDC_PAIR_ARK3 = 1,        /* the third-order pair of section II (5 stages)                 */
  RIDC_PAIR_ARK4 = 2         /* the fourth-order pair of section II (7 stages)                */
} ridc_pair;

typedef struct {
  int32_t fs_kind;               /* ridc_fs_kind; a reaction needs a Dirichlet grid            */
  int32_t newton_maxit;          /* Newton iterates allowed per stage (0 = 30); a stage that
                                    does not converge leaves NaN (RIDC_E_NONFINITE on sync)    */
  double kappa;                  /* reaction rate                                             */
  int32_t pair[RIDC_MAX_ORDER];  /* ridc_pair of level j = 0..order-1 (the predictor first)   */
  int32_t reserved;              /* must be 0                                                 */
} ridc_ext;

/* ---- lifetime ------------------------------------------------------------------------------ */
/* Validate *p, build the plan (exact quadrature weights of section III-C, the pipeline schedule,
 * level rings, solver data) and allocate device memory on the current HIP device.
 * hip_stream: a hipStream_t (NULL = null stream) on which all later work of the handle runs.
 * On success *out receives the handle.  Errors: RIDC_E_INVAL, RIDC_E_UNSUPPORTED,
 * RIDC_E_NOMEM, RIDC_E_HIP.                                                                  */
int ridc_create(const ridc_problem* p, void* hip_stream, ridc_handle** out);

/* ridc_create for a 1D problem whose levels are IMEX pairs and/or whose stiff term carries a
 * reaction (ridc_ext).  p->order is the number of levels P; level j has order
 * S_j = p_0 + ... + p_j (Thm 2), and the result, the top level, has order S_{P-1}.  Level j
 * computes t_m at pipeline step m + d_j, d_0 = 0, d_j = d_{j-1} + S_j - 1 (its first step needs
 * the previous level through the window's last start-up node); an integration of nt steps takes
 * nt + d_{P-1} pipeline steps and needs nt = 0 or nt >= S_{P-1} - 1.  Every entry point that
 * takes a handle accepts the result (tuning entry points: RIDC_E_UNSUPPORTED).  Limits: dim 1,
 * FP64, n <= 8192, S_{P-1} <= 12.  Errors: as ridc_create, and RIDC_E_UNSUPPORTED for a
 * reaction on a periodic grid.                                                                */
int ridc_create_ext(const ridc_problem* p, const ridc_ext* e, void* hip_stream,
                    ridc_handle** out);

/* Device bytes ridc_create_ext would allocate (0 if invalid).                                 */
size_t ridc_footprint_bytes_ext(const ridc_problem* p, const ridc_ext* e);

/* Interpolation and partial-interval quadrature weights of an IMEX corrector stage (section
 * III-C with S nodes): for the window of S equispaced nodes whose position r (0 <= r <= S-2)
 * holds t_n, interp[k] = l_k(t_n + c dt) and quad[k] = (1/dt) int_{t_n}^{t_n + c dt} l_k, with
 * c the abscissa of stage `stage` of `pair` and l_k the Lagrange basis (k = 0..S-1, ascending
 * nodes); exact rationals rounded once.  2 <= S <= 12.  Host only.                          */
int ridc_stage_weights(int32_t S, int32_t r, int32_t pair, int32_t stage, double* interp,
                       double* quad);

/* Free everything the handle owns (after synchronising its stream).  NULL-safe.              */
int ridc_destroy(ridc_handle* h);

/* Device bytes ridc_create would allocate for *p (rings, transforms, workspaces); 0 if *p is
 * invalid.  Used for admission control by HBM footprint.                                      */
size_t ridc_footprint_bytes(const ridc_problem* p);

/* ---- one-shot integration ------------------------------------------------------------------ */
/* Integrate from u0_dev for nsteps uniform steps (t = nsteps*dt): ridc_begin, all pipeline
 * steps, ridc_read.  nsteps == 0 returns u0; otherwise nsteps >= order-1 is required (the
 * start-up quadrature of the top corrector uses t_0..t_{P-1}).  uT_dev receives the top level;
 * levels_dev (nullable) receives every level's final value, level-major (P blocks).
 * u0_dev and uT_dev may be the same array.  Asynchronous; see ridc_sync.                      */
int ridc_integrate(ridc_handle* h, const double* u0_dev, int64_t nsteps, double* uT_dev,
                   double* levels_dev);

/* RIDC with restarts (section III-E): nsteps is split into `segments` equal intervals (nsteps
 * must be a multiple of segments, each segment >= order-1 steps); each interval is a full RIDC
 * integration restarted from the top level of the previous one.  segments = 1 is
 * ridc_integrate.  uT_dev receives the final top level (it may alias u0_dev).                 */
int ridc_integrate_restarts(ridc_handle* h, const double* u0_dev, int64_t nsteps,
                            int32_t segments, double* uT_dev);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same 1D integration as ridc_create +
 * ridc_integrate + ridc_destroy, with the same kernels and bitwise the same result, but with no
 * handle and no allocation of any kind on the device.  The level rings and the weight and PCR
 * tables live in a fixed 32 MiB array inside the library, one per GPU, which the GPU keeps until
 * the process ends.  p: as for ridc_create, dim 1 and order <= 6; the rings need
 * (sum over levels of ring slots) * n * 8 bytes plus 4 KiB, e.g. n <= 246,000 at order 4
 * (17 slots).  hip_stream: the stream of the work (NULL = null stream).  u0_dev, uT_dev: n
 * doubles on the current device, owned by the caller, may alias.  nonfinite_dev (nullable):
 * a device int the caller has cleared, set to 1 when the result holds a NaN or Inf.
 * Asynchronous; the caller synchronises the stream.  All calls on one GPU share its array:
 * calls whose work overlaps on that GPU (other streams, other threads) race and give wrong
 * results; calls in stream order on one stream are safe.  Errors (before any device work):
 * RIDC_E_INVAL, RIDC_E_UNSUPPORTED (2D, order > 6, or a problem larger than the array),
 * RIDC_E_HIP.                                                                                */
int ridc_integrate_noalloc(const ridc_problem* p, void* hip_stream, const double* u0_dev,
                           int64_t nsteps, double* uT_dev, int* nonfinite_dev);

/* Integrate `count` handles (any mix of sizes, orders, dims and precisions, all created on the
 * same stream) together: each pipeline step of every handle is grouped into shared launches.
 * u0[i], uT[i] and nsteps[i] as in ridc_integrate.  Each handle's result is bitwise the same
 * as when it is integrated alone.                                                             */
int ridc_integrate_batch(ridc_handle* const* hs, int32_t count, const double* const* u0,
                         const int64_t* nsteps, double* const* uT);

/* ---- stepping interface (continuous batching) ---------------------------------------------- */
/* Load u0 into every level and arm the handle for nsteps time steps (pipeline step 0).       */
int ridc_begin(ridc_handle* h, const double* u0_dev, int64_t nsteps);

/* Advance each armed handle by min(max_steps, its remaining) pipeline steps.  Handles that
 * share a pipeline step are grouped into shared launches.  All handles must share a stream.  */
int ridc_advance(ridc_handle* const* hs, int32_t count, int64_t max_steps);

/* Pipeline steps left before ridc_read may be called (0 when done; -1 if never armed).        */
int64_t ridc_remaining(const ridc_handle* h);

/* Copy the top level (uT_dev) and optionally every level (levels_dev, nullable, level-major)
 * out of a handle whose remaining() is 0.  Errors: RIDC_E_STATE if steps remain.              */
int ridc_read(ridc_handle* h, double* uT_dev, double* levels_dev);

/* Wait for the handle's stream; RIDC_E_NONFINITE if the last result read held a NaN/Inf.     */
int ridc_sync(ridc_handle* h);

/* Thread-local message for the last failing call on this thread ("" if none).                 */
const char* ridc_last_error(void);

/* ---- introspection (host only, no device work) --------------------------------------------- */
/* Quadrature weights of corrector j for start-up row r (0 <= r < j): the j+1 integrals, in
 * units of dt, of the Lagrange basis on nodes t_s..t_{s+j} over [t_{s+r}, t_{s+r+1}]
 * (section III-C; row r = j-1 is the steady-state trailing window).  out: j+1 doubles,
 * ascending node order.                                                                       */
int ridc_quadrature_weights(int32_t j, int32_t r, double* out);

/* Number of PCR stages and the final divisor the 1D solver uses for (I - r*D2) on a cycle of
 * length m (periodic: m = n; Dirichlet: m = 2n+2, odd extension), r = dt*nu/h^2.             */
int ridc_pcr_plan(double r, int64_t m, int32_t* stages, double* divisor);

/* Kernel names and per-launch algorithmic work of the handle's dominant kernel: bytes moved
 * per pipeline step at steady state (1D) or flops per step of the 2D transforms.             */
int ridc_step_cost(const ridc_handle* h, double* hbm_bytes, double* flops);

/* ---- tuning --------------------------------------------------------------------------------- */
/* Choose the handle's launch shape by measurement and record it in the tuning table (see
 * ridc_tune_save) for later handles with the same key:
 *  - 1D: candidate tilings (threads per workgroup; whole cycle per workgroup, or chunks of
 *    `rows` rows with a PCR halo; the whole-range workgroup), keyed by (n, boundary, PCR
 *    stages).  threads_out/rows_out/flags_out (nullable) receive the choice (rows 0 = whole
 *    cycle; flags as in ridc_set_tile).
 *  - 2D: the transform-pass shapes the handle's side and precision allow, keyed by (n,
 *    precision): 32- or 64-column waves (FP32/FP64 passes), 64- or 32-wide k-slices
 *    (split-BF16 pass), prefolded or row-major intermediates (n a multiple of 256), each
 *    timed over whole pipeline steps (10 at n <= 1024, fewer above; best of three rounds).
 *    threads_out receives the threads per block, rows_out 0, flags_out the shape bits as in
 *    ridc_set_tile.
 * A shape already recorded for the key (this process, or the tuning cache file) is applied
 * without measuring; ridc_tune_clear forgets the table.  Every shape performs the same
 * operations for every output value, so results are bitwise independent of the choice.  The
 * tuning launches overwrite the level rings: the handle must be re-armed (ridc_begin).
 * IMEX handles (ridc_create_ext): RIDC_E_UNSUPPORTED.                                        */
int ridc_autotune(ridc_handle* h, int32_t* threads_out, int32_t* rows_out, int32_t* flags_out);

/* 2D handles: set the transform-pass shape bits `flags` (1: 64-column waves, FP32/FP64 passes
 * with n/2 a multiple of 64 or no fold; 2: 32-wide k-slices, split-BF16 pass; 4: row-major
 * intermediates folded while staging, instead of the folded planes (sums and differences of
 * mirrored columns) that the passes exchange by default when n is a multiple of 256; 0: none
 * of these).  A handle with no recorded shape starts at 0, split-BF16 handles at 2 where 2 is
 * allowed.  rows must be 0 and threads is ignored; results do not depend on the shape.
 * 1D: force a tiling: threads in {64,128,256,512,1024}; rows = 0 for the whole cycle in one
 * workgroup, else chunks of `rows` rows (allowed when the PCR coupling vanishes within a halo
 * shorter than the system); flags bit 0 = write level values with nontemporal stores; flags
 * bit 1 = one workgroup of `threads` (512 or 1024, rows 0) runs every level and many pipeline
 * steps in one launch (needs the levels' cycles to fit one CU's LDS; order <= 6 with 512
 * threads, order <= 4 with 1024).
 * Errors: RIDC_E_INVAL if the tiling does not fit.                                            */
int ridc_set_tile(ridc_handle* h, int32_t threads, int32_t rows, int32_t flags);

/* Tiling of grouped 1D launches (ridc_advance or ridc_integrate_batch over several 1D handles),
 * process-wide: `threads` per workgroup (256, 512 or 1024; 1024 falls back to 512 for batches
 * holding an order above 6) and the most rows a workgroup holds in LDS: rows = 0 puts each
 * level's whole cycle in one workgroup whenever it fits; rows >= 256 cuts longer cycles into
 * chunks whose rows plus PCR halos stay within `rows` (systems whose halo is too long for that
 * keep whole cycles).  Like every tiling it does not change results (section III-E's pipeline
 * and the solves are computed the same way).  Default: 256 threads, rows 0.
 * Errors: RIDC_E_INVAL for other values.                                                      */
int ridc_set_batch_tile(int32_t threads, int32_t rows);

/* Time one grouped launch of the 1D handles among hs[0..count) for every candidate batch tiling
 * (threads x rows, 20 steady-state steps each, HIP events on the first 1D handle's stream) and
 * set the fastest as with ridc_set_batch_tile, recording it in the tuning table; a grouped
 * tiling already recorded there (this process or the cache file) is set without measuring.
 * The timed steps overwrite the level rings, so every 1D handle is left unarmed (call
 * ridc_begin again).  threads_out and rows_out (nullable) receive the choice.  Errors:
 * RIDC_E_INVAL for bad handles, RIDC_E_HIP on launch failures.                               */
int ridc_autotune_batch(ridc_handle* const* hs, int32_t count, int32_t* threads_out,
                        int32_t* rows_out);

/* Tuning table.  The autotuners record their choices in a process-wide table, loaded on first
 * use from a JSON file and rewritten after every new entry: $RIDC_TUNE_CACHE if set (empty or
 * "off": no file), else $XDG_CACHE_HOME/ridc/tune.json, else $HOME/.cache/ridc/tune.json.  The
 * file names the GPU it was measured on (architecture and compute units); entries of another
 * GPU are not loaded.  A cache that cannot be written is not an error.
 * ridc_tune_save: write the table to `path` (NULL = the default file).
 * ridc_tune_load: merge the entries of `path` (NULL = the default file) into the table.
 * ridc_tune_clear: forget every entry in memory (the file is kept; it is not reloaded).
 * Errors: RIDC_E_INVAL when the file cannot be written or read.                               */
int ridc_tune_save(const char* path);
int ridc_tune_load(const char* path);
int ridc_tune_clear(void);

/* Average duration of the dominant kernel per pipeline step, from HIP events on the handle's
 * stream, starting at the handle's next pipeline step (which must have every level active):
 *  - 1D, one launch per step: `reps` back-to-back launches of that step (each recomputes the
 *    same values; the handle does not advance);
 *  - 1D, whole-integration workgroup (systems that fit one CU's LDS): one launch running
 *    `reps` steps; the handle runs ahead and is left unarmed (call ridc_begin again);
 *  - 2D: `reps` launches of the second transform pass of that step over all levels (after its
 *    right-hand side and first pass once): the kind of most of a step's passes.  These launches
 *    rewrite only per-step intermediates (the right-hand side and transform buffers, which the
 *    step recomputes); the level rings and the handle's position are unchanged.
 * *work_per_launch (nullable) receives the algorithmic HBM bytes (1D, per step) or flops (2D,
 * per pass).  Errors: RIDC_E_STATE if the next step is not a full one or too few remain.     */
int ridc_kernel_time(ridc_handle* h, int32_t reps, double* us_per_launch,
                     double* work_per_launch);

/* Average duration of one grouped 1D launch (section III-E's pipeline step for every instance in
 * hs[0..count), with the current batch tiling), from HIP events around `reps` back-to-back
 * launches on the handles' stream.  Every handle must be armed, 1D, not set to the whole-range
 * workgroup, and have every level active in its next step, which each launch recomputes (the
 * handles do not advance).  *bytes_per_launch (nullable) receives the algorithmic HBM bytes of
 * that step summed over the instances (as ridc_step_cost).  Errors: RIDC_E_STATE,
 * RIDC_E_UNSUPPORTED, RIDC_E_INVAL, RIDC_E_HIP.                                              */
int ridc_batch_kernel_time(ridc_handle* const* hs, int32_t count, int32_t reps,
                           double* us_per_launch, double* bytes_per_launch);

/* 2D: average duration of the right-hand-side kernel (the stencils and the quadrature of
 * eq. (corr) over the window, section III-C, plus the explicit-term differences, for every
 * level) at the handle's next pipeline step, which must have every level active, from HIP events
 * around `reps` back-to-back launches on the handle's stream (each rewrites the same values; the
 * handle does not advance).  *bytes_per_launch (nullable) receives its algorithmic HBM bytes.
 * Errors: RIDC_E_UNSUPPORTED for 1D handles (their stencils are fused into the level step),
 * RIDC_E_STATE, RIDC_E_INVAL.                                                                */
int ridc_stencil_time(ridc_handle* h, int32_t reps, double* us_per_launch,
                      double* bytes_per_launch);

/* Library version string.                                                                     */
const char* ridc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RIDC_H */
