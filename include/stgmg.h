/*
 * stgmg -- space-time geometric-multigrid preconditioned flexible GMRES for the
 * dG(k) x Q_r^d / Q_{r-1} slab systems of dynamic poro-/thermoelasticity, on one
 * AMD MI355X (gfx950).
 *
 * Method: Anselmann, Bause, Margenberg, Shamko, "An energy-efficient
 * GMRES-Multigrid solver for space-time finite element computation of dynamic
 * poro- and thermoelasticity" (arXiv:2303.06742).
 *   - slab problem: Problem 3.1 (v-form, Eq:DPQ_A0), algebraic form Problem 4.1
 *     (Eq:ALS_In, Eq:DefAn, Eq:DefAab);
 *   - solver: flexible GMRES preconditioned by one geometric-multigrid V-cycle
 *     (Sec. 4), smoother = patchwise Vanka operator (Def:VankaOP, Eq:VankaOP0)
 *     applied by Algorithm 4.1, direct solve on the coarsest level.
 *
 * Vector layout (all vectors are FP64, on the device unless stated otherwise):
 *   X = (V_1, U_1, P_1, ..., V_{k+1}, U_{k+1}, P_{k+1})      (Eq:DefXn)
 *   time node outermost; inside a node V and U are node-major over the
 *   lexicographic Q_r lattice of (r N + 1)^d nodes (x fastest) with the d
 *   components interleaved (index d*node + c), and P is over the lexicographic
 *   Q_{r-1} lattice of ((r-1) N + 1)^d nodes.  A residual / right-hand side has
 *   the same layout with the rows (u-equation, v-equation, p-equation).
 *   n_s = 2 d (rN+1)^d + ((r-1)N+1)^d values per time node, n = (k+1) n_s.
 *
 * Ownership: the library owns handles and all hierarchy memory (operators,
 * patch inverses, Krylov bases) and frees them in stgmg_destroy.  The caller
 * owns every vector argument; the library never keeps a pointer past the call.
 * Device vectors must be 8-byte aligned, hold n doubles and must not alias
 * each other unless stated.  Every entry point that takes device vectors checks
 * them with hipPointerGetAttributes: a NULL vector is STGMG_ERR_INVALID_ARG; host
 * memory (pinned or not), a pointer the runtime does not know, or a misaligned one
 * is STGMG_ERR_BAD_POINTER, returned before anything is enqueued.
 *
 * Errors: every function returns a status; no C++ exception crosses this
 * interface.  stgmg_last_error() gives a thread-local text for the last
 * failure.  A handle may be used by one host thread / stream at a time.
 */
#ifndef STGMG_H
#define STGMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t stgmg_status;
#define STGMG_OK 0
#define STGMG_NOT_CONVERGED 1        /* x holds the last iterate */
#define STGMG_PENDING 2              /* server: the request has not finished yet */
#define STGMG_ERR_INVALID_ARG (-1)
#define STGMG_ERR_UNSUPPORTED (-2)
#define STGMG_ERR_OOM (-3)
#define STGMG_ERR_HIP (-4)
#define STGMG_ERR_SINGULAR_PATCH (-5) /* a patch matrix A_P had a zero pivot */
#define STGMG_ERR_NONFINITE (-6)      /* NaN/Inf in rhs, x0 or a residual */
#define STGMG_ERR_BAD_POINTER (-7)    /* a vector argument is not device memory, or not 8-byte aligned */

#define STGMG_PATCH_CELL 0   /* one patch per cell */
#define STGMG_PATCH_VERTEX 1 /* one patch per grid vertex: the cells that touch it (Eq:DefPlm) */

#define STGMG_FP64 0 /* patch inverses stored and applied in FP64 */
#define STGMG_FP32 1 /* patch inverses computed in FP64, stored and applied in FP32 */
#define STGMG_BF16 2 /* patch inverses computed in FP64, stored in BF16 (time_blocks = 3 only: the
                        symmetric tiles, four tiles per 8-byte unit, and the small reduced factors),
                        applied with FP64 sums */

/* pressure space Q_h of Def:VhQh / Eq:DefVhQh */
#define STGMG_PRESSURE_CONT 0 /* continuous Q_{r-1} (Taylor-Hood), B_gamma with Nitsche terms (Def:B, first option) */
#define STGMG_PRESSURE_DISC 1 /* broken P_{r-1}^disc: per cell the monomials prod (xi - 1/2)^a, |a| <= r-1, cell-major;
                                 B_gamma the symmetric interior penalty form (Def:B, second option) */

/* formulation of the third equation */
#define STGMG_FORM_V   0 /* Problem 3.1: -C(v, psi) */
#define STGMG_FORM_DTU 1 /* Problem B.1: -C(d_t u, psi), the jump of c0 p + alpha div u and
                            -alpha <u . n, psi> on the boundary (u_D(t_{n-1}) on the right) */

typedef struct stgmg_handle stgmg_handle;

/* Problem and solver parameters.  Fine level: coarse_cells << (levels-1) cells
 * per axis on the unit square/cube; level 0 is solved directly. */
typedef struct {
  int32_t dim;           /* 2 or 3 */
  int32_t coarse_cells;  /* cells per axis on level 0 (>= 1) */
  int32_t levels;        /* number of levels L+1 >= 1 */
  int32_t r;             /* displacement degree (Q_r^d); pressure degree r-1 (see pressure); 2 <= r <= 4 */
  int32_t k;             /* dG(k) in time, 0 <= k <= 3 */
  int32_t patch;         /* STGMG_PATCH_CELL or STGMG_PATCH_VERTEX */
  int32_t smoother_prec; /* STGMG_FP64, STGMG_FP32 or STGMG_BF16 */
  int32_t n_smooth;      /* J_max pre- and post-smoothing sweeps (paper: 4) */
  double omega;          /* Vanka under-relaxation (paper: 0.7) */
  double tau;            /* slab length */
  double rho, lambda, mu, alpha, c0; /* material parameters of Eq:HPS (isotropic C) */
  double K;              /* permeability K*I when K_cells == NULL */
  const double* K_cells; /* host, optional: K per fine cell, lexicographic (x fastest);
                            coarse cells take the mean of their 2^d children. Copied. */
  int32_t graph;         /* V-cycle as a captured HIP graph: 1 captures it inside stgmg_setup and
                            replays it in every solve; 0 and -1 (automatic, the default) launch
                            the kernels directly.  A process that set up, solved and released
                            several hundred graph-captured handles has seen every later solve
                            report non-finite Arnoldi values; the same work without graphs did
                            not, so capture is not automatic.  While a capture runs, null-stream
                            work from other threads of the process fails (a runtime rule), so
                            set up handles with graphs while no other thread uses the GPU
                            through the null stream (the server launches directly). */
  int32_t time_blocks;   /* how A_P^{-1} of Def:VankaOP is stored and applied (the same operator
                            in every mode, up to rounding):
                            0: the full space-time inverse (n_P^2 values);
                            1: through the eigen-decomposition of (M^t)^{-1} D^t, since
                               A_P = D^t (x) MM_P + M^t (x) KK_P: one spatial inverse of n_P/(k+1)
                               rows per eigenvalue ((k+1)x fewer values);
                            2: as 1, with the u-equation rows of each spatial block eliminated
                               (V = lam U - (rho M)^{-1} r_u): stored are (rho M)^{-1} on the
                               patch nodes, KK_pV (rho M)^{-1}, and one Schur complement inverse
                               of n_P/(k+1) - nU rows per eigenvalue (about 3x fewer again);
                            3: as 2, with each Schur inverse stored through its symmetric form:
                               X = (D1 S D2)^{-1}, D1 = diag(I, -lam^{-1/2}), D2 = diag(I, lam^{1/2})
                               on the (U, P) rows, is symmetric, and its lower triangle is kept in
                               64-value tiles: off-diagonal 8x8 tiles, the diagonal 8x8 blocks as
                               triangles two to a tile, a last block row of at most 4 rows in 4x16
                               tiles (about 0.52x the values of 2 at 59 rows; FP32 storage pairs the tiles
                               so that a lane loads 8 bytes, and keeps 2 for Schur blocks of
                               more than 96 rows, where the square layout measured faster).
                            Default of the Python workloads: 3. */
  int32_t pressure;      /* STGMG_PRESSURE_CONT (0, the zero-initialised default) or STGMG_PRESSURE_DISC */
  int32_t form;          /* STGMG_FORM_V (0, default) or STGMG_FORM_DTU */
  int32_t waves_per_patch; /* time_blocks = 3 only: wavefronts that apply one patch's tiles: 0 by the
                              patch count (4 on levels of fewer than 4,096 patches -- 8,192 for Schur
                              blocks of more than 96 rows -- and 1 on larger levels; see autotune), or
                              1, 2 or 4 on every level.  The same operator either way, up to the order
                              of the sums. */
  int32_t autotune;      /* 1: stgmg_setup times the candidate launch shapes on every level and keeps
                            the fastest -- the waves per patch of the tiled patch solve (1, 2 or 4,
                            when waves_per_patch is 0) and the lanes per node of the level operator
                            (2, 4, 8 or 16) -- adding a few milliseconds per level.  The results then
                            depend on the timing in their last bits (the order of sums), so two
                            handles of one problem may differ by rounding.  0: fixed rules. */
} stgmg_params;

typedef struct {
  int32_t iters;         /* FGMRES iterations = V-cycles applied */
  int32_t restarts;
  int32_t converged;     /* 1 if ||b - A x|| <= rtol ||b - A x0|| */
  double res0;           /* ||b - A x0||_2 */
  double rel_res_true;   /* ||b - A x||_2 / res0, recomputed at exit */
  double rel_res_est;    /* last Givens estimate */
  double t_solve_ms;     /* wall time of the solve (device synchronised) */
  double t_vcycle_ms;    /* device time inside the V-cycles of the solve (HIP events around each) */
} stgmg_info;

/* Build the level hierarchy for Problem 4.1 with the given parameters: level
 * operators (Eq:DefAab, re-assembled on every level), grid transfers, patch
 * tables, the patch inverses A_P^{-1} of Def:VankaOP (extracted from the
 * assembled level matrix and inverted on the GPU) and the coarse inverse.
 * hip_stream: the caller's hipStream_t (NULL = default stream).  The handle
 * runs on a stream of its own; every call first waits for the work already
 * enqueued on hip_stream and returns after its own work has completed.  Returns STGMG_ERR_SINGULAR_PATCH if any A_P is
 * singular, STGMG_ERR_OOM if device memory runs out. */
stgmg_status stgmg_setup(const stgmg_params* params, void* hip_stream, stgmg_handle** out);

/* Sizes of one level (level = 0..levels-1; -1 = finest): number of unknowns n,
 * number of patches, stored nonzeros of the level operator, and the device
 * bytes held by the whole handle. Any output pointer may be NULL. */
stgmg_status stgmg_query(const stgmg_handle* h, int32_t level, int64_t* n_dofs, int64_t* n_patches,
                         int64_t* nnz, int64_t* hbm_bytes);

/* Launch shapes that level `level` (as in stgmg_query) uses, after the setup's autotuning when
 * stgmg_params.autotune = 1: the wavefronts that apply one patch's symmetric tiles (1, 2 or 4; 0 where
 * the level has no tiled patch solve) and the lanes per Q_r node of the level-operator kernel
 * (2, 4, 8 or 16; 0 where the level applies its operator from the CSR matrices).  Either output
 * pointer may be NULL. */
stgmg_status stgmg_query_launch(const stgmg_handle* h, int32_t level, int32_t* waves_per_patch,
                                int32_t* node_lanes);

/* Solve A_n x = rhs (Problem 4.1, Eq:ALS_In) on the finest level with FGMRES
 * (right preconditioning, restart length `restart`, at most `max_iters`
 * iterations), one V-cycle per iteration (Sec. 4).  x: in = x0, out = solution.
 * Stops when ||rhs - A x||_2 <= rtol * ||rhs - A x0||_2, checked on the true
 * residual.  info may be NULL.  Returns STGMG_NOT_CONVERGED (x = last iterate)
 * or STGMG_ERR_NONFINITE (x unchanged) when applicable. */
stgmg_status stgmg_solve(stgmg_handle* h, const double* rhs_dev, double* x_dev, double rtol,
                         int32_t restart, int32_t max_iters, stgmg_info* info);

/* Allocation-free variant of stgmg_solve for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * FGMRES and V-cycle kernels, with the FGMRES workspace (bases V and Z, Arnoldi vector, dot
 * product partial sums, Hessenberg column, update coefficients: about (2 restart + 2) n doubles)
 * in a static device array of STGMG_NOALLOC_SCRATCH_BYTES, which each GPU the library runs on
 * holds until the process ends.  It calls no hipMalloc/hipFree (the hierarchy was allocated by
 * stgmg_setup).  Returns STGMG_ERR_UNSUPPORTED, before anything is enqueued, when the workspace
 * of n unknowns and `restart` does not fit (e.g. n above about 260,000 at restart 30).  All
 * calls on one GPU share that GPU's array, whose contents persist from the last call: calls
 * that overlap in time on one GPU (other threads, other handles) race and must be serialised
 * by the caller.  Arguments, result and statuses as for stgmg_solve. */
#define STGMG_NOALLOC_SCRATCH_BYTES (128LL << 20)
stgmg_status stgmg_solve_noalloc(stgmg_handle* h, const double* rhs_dev, double* x_dev, double rtol,
                                 int32_t restart, int32_t max_iters, stgmg_info* info);

/* y = A_level x (the assembled level operator of Eq:DefAn). level -1 = finest. */
stgmg_status stgmg_apply_operator(stgmg_handle* h, int32_t level, const double* x_dev, double* y_dev);

/* z = B r: one V-cycle with zero initial guess on the finest level (Sec. 4). */
stgmg_status stgmg_apply_vcycle(stgmg_handle* h, const double* r_dev, double* z_dev);

/* d <- `sweeps` steps of Algorithm 4.1 on level `level` (>= 1) for A_l d = b,
 * starting from the given d (Def:VankaOP with the handle's omega). */
stgmg_status stgmg_smooth(stgmg_handle* h, int32_t level, const double* b_dev, double* d_dev, int32_t sweeps);

/* Grid transfers between level l-1 and l (l >= 1): prolongation by
 * interpolation, d_fine += P e_coarse, and restriction by the transpose,
 * b_coarse = P^T r_fine (Sec. 4, list of GMRES-GMG ingredients). */
stgmg_status stgmg_prolongate_add(stgmg_handle* h, int32_t level, const double* e_coarse_dev, double* d_fine_dev);
stgmg_status stgmg_restrict(stgmg_handle* h, int32_t level, const double* r_fine_dev, double* b_coarse_dev);

/* Right-hand side of Problem 3.1 for the slab (t_start, t_start + tau] on the
 * finest level, for the built-in prescribed solution
 *   u_i = S(x) sin(t) (every component), p = S(x) cos(t), S = prod_j sin(pi x_j),
 * whose Dirichlet data vanish on the boundary of the unit square/cube:
 *   F[b] = tau/2 w_b S(t_{n,b}) + e_b MM x_prev_end          (Def:LG, Problem 3.1)
 * x_prev_end_dev: the previous slab's values at t_{n-1} (n_s doubles, one time
 * node block).  rhs_dev: n doubles. */
stgmg_status stgmg_slab_rhs(stgmg_handle* h, double t_start, const double* x_prev_end_dev, double* rhs_dev);

/* Time marching of Problem 3.1 (or B.1) with the built-in prescribed solution over n_slabs
 * slabs (t_start + s tau, t_start + (s+1) tau], s = 0 .. n_slabs-1, inside the library: for
 * every slab the right-hand side of stgmg_slab_rhs from the previous slab's end values (on the
 * device; a captured HIP graph for hierarchies that capture the V-cycle), x0 = 0, stgmg_solve
 * with rtol / restart / max_iters, and the last time-node block of the solution (the values at
 * t_n, the right Radau node) as the next slab's start values (Problem 3.1, the jump term of
 * Def:LG).  x_end_dev (n_s doubles): in = the values at t_start, out = those at
 * t_start + n_slabs tau.  x_dev (n doubles): workspace; out = the last slab's solution.
 * infos (n_slabs entries, may be NULL): per slab.  Returns STGMG_OK if every slab converged,
 * else the first non-OK status of a slab (marching continues after NOT_CONVERGED). */
stgmg_status stgmg_march(stgmg_handle* h, double t_start, int32_t n_slabs, double* x_end_dev, double* x_dev,
                         double rtol, int32_t restart, int32_t max_iters, stgmg_info* infos);

/* Nodal interpolant (V, U, P) of the built-in prescribed solution at time t,
 * n_s doubles (one time-node block), on the finest level. */
stgmg_status stgmg_interpolate_solution(stgmg_handle* h, double t, double* x_block_dev);

/* Copy the stored inverse of patch `patch` of level `level` (>= 1) to host
 * memory as a dense row-major FP64 matrix of n_P x n_P (the patch dofs in
 * increasing global order), and its global dof numbers (n_P int64).
 * Call with out == NULL to get n_P only.  For tests. */
stgmg_status stgmg_get_patch_inverse(stgmg_handle* h, int32_t level, int64_t patch, int32_t* n_p,
                                     double* out_host, int64_t* dofs_host);

/* Kernel timing with HIP events on the handle's stream, for roofline figures.
 * enable != 0 starts recording (clearing earlier records); stgmg_profile_get
 * returns, for `what` = STGMG_PROF_PATCH_APPLY (patch GEMV of Def:VankaOP on the
 * finest level) or STGMG_PROF_RESIDUAL (residual b - A d on the finest level),
 * the number of recorded launches, their summed duration in ms, and the
 * algorithmic bytes of one launch (stored inverse entries + gathered residual
 * + written images, resp. matrix values + x + b + y; index bytes excluded). */
#define STGMG_PROF_PATCH_APPLY 0
#define STGMG_PROF_RESIDUAL 1
stgmg_status stgmg_profile_enable(stgmg_handle* h, int32_t enable);
stgmg_status stgmg_profile_get(stgmg_handle* h, int32_t what, int64_t* launches, double* total_ms,
                               double* bytes_per_launch);

stgmg_status stgmg_destroy(stgmg_handle* h);

/* Closed-form sizes for admission control, without building anything: n (unknowns
 * of the finest level, the length of rhs and x), the device bytes a handle holds
 * after stgmg_setup plus the FGMRES workspace for `restart`, and the peak bytes
 * during setup (resident + temporary extraction/inversion buffers).  Exact up to
 * allocation granularity. */
stgmg_status stgmg_footprint(const stgmg_params* params, int32_t restart, int64_t* n_dofs, int64_t* resident_bytes,
                             int64_t* setup_peak_bytes);

/* Solve count independent problems (Problem 4.1 each) at the same time: every
 * handle runs on its own stream, driven by its own host thread (at most 16 at
 * once); kernels of different problems overlap on the GPU.  Each problem's result
 * is bitwise the same as that of stgmg_solve alone.  statuses[i] and infos[i]
 * (either may be NULL) receive the per-problem outcome; the return value is
 * STGMG_OK if every problem returned STGMG_OK, else the first non-OK status. */
stgmg_status stgmg_solve_batch(int32_t count, stgmg_handle* const* handles, const double* const* rhs_dev,
                               double* const* x_dev, double rtol, int32_t restart, int32_t max_iters,
                               stgmg_info* infos, stgmg_status* statuses);

/* Serving loop for a stream of solve requests (continuous batching): requests
 * are admitted as soon as their footprint fits in hbm_budget bytes next to the
 * running and resident problems; up to max_slots run at once, each with its own
 * stream and host thread; hierarchies of finished requests with a non-zero
 * problem_key stay resident (at most resident_max, least recently used evicted
 * first) and are reused by later requests with the same key (follow-on slabs). */
typedef struct stgmg_server stgmg_server;
stgmg_status stgmg_server_create(int64_t hbm_budget, int32_t max_slots, int32_t resident_max, stgmg_server** out);
/* Queue a request: params (copied, K_cells included), problem_key (0 = never
 * reused; equal keys must mean equal params), rhs_host (n doubles, copied; n from
 * stgmg_footprint), x0 = 0, relative tolerance rtol, restart 30.  STGMG_ERR_OOM if
 * the problem can never fit the budget. */
stgmg_status stgmg_server_submit(stgmg_server* srv, const stgmg_params* params, uint64_t problem_key,
                                 const double* rhs_host, double rtol, uint64_t* ticket);
/* STGMG_PENDING while the request is queued or running; otherwise its final
 * status, with x_host (n doubles, may be NULL), info and latency_ms (submit to
 * completion, may be NULL) filled.  A finished ticket can be polled again. */
stgmg_status stgmg_server_poll(stgmg_server* srv, uint64_t ticket, double* x_host, stgmg_info* info,
                               double* latency_ms);
/* The error text of a finished request that failed ("" otherwise, or for an
 * unknown ticket); it stays valid until stgmg_server_destroy.  (The worker that ran
 * the request is another thread, so stgmg_last_error does not see it.) */
const char* stgmg_server_message(stgmg_server* srv, uint64_t ticket);
/* Waits for all queued and running requests, then frees everything. */
stgmg_status stgmg_server_destroy(stgmg_server* srv);

const char* stgmg_status_string(stgmg_status s);
const char* stgmg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* STGMG_H */
