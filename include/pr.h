/*
 * pr.h -- C ABI of the MI355X (gfx950) library for the data-parallel hot path
 * of micro-macro parareal for slow-fast SDEs (Legoll, Lelievre, Myerscough,
 * Samaey, "Parareal computation of stochastic differential equations with
 * time-scale separation: a numerical study", arXiv 1912.09240).
 *
 * Conventions shared by every entry point
 *  - Return value: PR_OK (0) on success, a negative pr_status otherwise;
 *    pr_last_error() then returns a thread-local message.  Invalid arguments
 *    are rejected before anything is launched.
 *  - Pointers are DEVICE pointers (memory of the current HIP device) owned by
 *    the caller unless the comment says "host".  The library never frees or
 *    reallocates caller memory.  The only library-owned memory lives inside
 *    the opaque handles returned by the *_create calls and is released by the
 *    matching *_destroy call.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls enqueue work
 *    on it and return without waiting, except the *_create calls and
 *    pr_parareal_iterate when it is asked for host error values.
 *  - Layouts are structure-of-arrays, slice-major: x[k][n] is particle p of
 *    slice k at x[k*n + p]; the fast variables are y[k][d][n].
 *  - Symbols of the paper <-> names here: P particles = n, N slices =
 *    n_slices (k when a count of slices is passed), I cells = n_cells,
 *    delta t = dt, the levels p_j = j/Q of the quantile knots use Q = n_q.
 */
#ifndef PR_H
#define PR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PR_OK = 0,
    PR_E_INVALID = -1,     /* an argument is out of range or inconsistent   */
    PR_E_HIP = -2,         /* a HIP runtime call failed (message says which) */
    PR_E_NOMEM = -3,       /* workspace too small or device allocation failed */
    PR_E_UNSUPPORTED = -4  /* valid request that this build does not serve  */
} pr_status;

/* Precision of the particle state and of the Euler-Maruyama arithmetic.
 * Moments, knots, coarse model and matching offsets are always FP64. */
enum { PR_F64 = 64, PR_F32 = 32 };

/* Flags of pr_parareal_create. */
enum {
    PR_REUSE_COARSE = 1,   /* q_c^* = C(q_k^n) instead of C(R(X_k^n))          */
    PR_SKIP_CONVERGED = 2, /* do not re-run the fine propagator on slices whose
                              start is already exact (n < k, Sec. 3.3.3)       */
    PR_PROFILE = 4,        /* record HIP events around each phase of an
                              iteration (see pr_parareal_profile)              */
    PR_AUTOTUNE = 8        /* batched handle: time the fine kernel's shapes at
                              creation and keep the fastest                    */
};

/* Launch patterns of pr_parareal_batch_iterate (same results bitwise). */
enum {
    PR_LAUNCH_BATCHED = 0,      /* one launch per phase for all instances       */
    PR_LAUNCH_GRAPH = 1,        /* the batched sequence captured in a hipGraph   */
    PR_LAUNCH_PER_INSTANCE = 2  /* every phase launched instance by instance     */
};

/* Phases reported by pr_parareal_profile. */
enum {
    PR_PH_FINE = 0,        /* fine propagator, all slices: one kernel launch   */
    PR_PH_RESTRICT_FINE,   /* restriction of the fine results (full sort)      */
    PR_PH_COARSE,          /* coarse propagation of all slices in parallel     */
    PR_PH_CHAIN,           /* serial quantile-iterator chain                   */
    PR_PH_MATCH,           /* matching of all slices                           */
    PR_PH_RESTRICT_NEW,    /* knots of the new states (+ error)                */
    PR_PH_COUNT
};

/*
 * Slow-fast SDE (Sec. 2.1.1, eq. (SDEx)/(SDEy)) with tau_x = 1, D = E = 1/beta,
 * slow potential F = c3 x^4/4 + c1 x^2/2 + lambda (x - mean_i y_i)^2/2 and
 * fast potential G = sum_i (y_i - a_i x)^2/2:
 *   dX   = -(c3 X^3 + c1 X + lambda (X - mean_i Y_i)) dt + sqrt(2/beta) dW_0
 *   dY_i = -(1/eps) (Y_i - a_i X) dt + sqrt(2/(beta eps)) dW_{i+1}
 */
typedef struct pr_sde {
    int d_fast;        /* d >= 1; this build serves d in {1, 2, 3, 4, 8, 16, 32} */
    int precision;     /* PR_F64 or PR_F32                                     */
    double lambda;     /* coupling                                             */
    double eps;        /* time-scale separation, > 0                           */
    double beta;       /* inverse temperature, > 0                             */
    double c3, c1;     /* slow potential coefficients                          */
    const double *a;   /* device, d_fast coefficients a_i; NULL means all 1    */
} pr_sde;

/* Time slices (Sec. 3.1): S fine steps of dt split into n_slices slices;
 * slice n covers the global steps [floor(n S/N), floor((n+1) S/N)). */
typedef struct pr_schedule {
    int64_t total_steps;  /* S >= n_slices                                    */
    int n_slices;         /* N >= 1                                           */
    double dt;            /* fine step, > 0                                   */
} pr_schedule;

/* Coarse grid (Sec. 2.2.2): n_cells uniform cells on [x_lo, x_hi]; quantile
 * knots at p_j = j/n_q, j = 0..n_q (Sec. 4.4). */
typedef struct pr_grid {
    int n_cells;          /* I >= 3                                           */
    double x_lo, x_hi;    /* x_lo < x_hi                                      */
    int n_q;              /* Q >= 2                                           */
} pr_grid;

/* Thread-local message of the last failing call ("" if none). */
const char *pr_last_error(void);

/* Library ABI version (incremented on incompatible changes). */
int pr_version(void);

/*
 * Noise.  Every normal number comes from Philox4x32-10 (Salmon et al., SC'11)
 * with key (lo32(seed), hi32(seed)) and counter (m, p, tag<<16 | j, instance),
 * m the global step, p the particle, j the pair index.  A block (w0..w3)
 * gives two normals by Box-Muller from u = (k + 1/2) 2^-52 with
 * k = (w0 >> 12) 2^32 + w1 and the angle pi t, t = (i + f)/128 with
 * i = (w2 >> 4) mod 256 and f = ((w2 >> 12) 2^32 + w3) 2^-52; normal 2j and
 * 2j+1 of a particle use pair j.  Tags: 0 EM increments, 1 initial ensemble, 2 coefficients a_i,
 * 3 batched-instance parameters.  Noise therefore depends only on
 * (seed, instance, step, particle): a slice run twice uses the same numbers
 * (Sec. 6) and any subset of particles can be recomputed.
 */

/* a[i] = 0.5 + u, u = ((w2 >> 5) 2^26 + (w3 >> 6)) 2^-53 of block
 * (tag 2, m = 0, p = i), i < d.
 * a: device, d doubles. */
int pr_draw_coupling(uint64_t seed, uint32_t instance, int d, double *a, void *stream);

/* Initial ensemble: X0 = N(0, 1/4) (normal 0), Y0_i = a_i X0 + beta^-1/2 z
 * (normal i+1), tag 1, m = 0.  x: [n], y: [d][n], precision of sde. */
int pr_init_ensemble(const pr_sde *sde, uint64_t seed, uint32_t instance, int64_t n,
                     void *x, void *y, void *stream);

/*
 * Fine propagator F (Sec. 3.2.1): Euler-Maruyama, eq. (EMx)/(EMy), drift at
 * the old state, over every slice in [slice_first, slice_first+slice_count)
 * at once.  x: [slice_count][n], y: [slice_count][d][n], in place: on entry
 * the state at the start of each slice, on exit at its end.  Each particle
 * keeps its state in registers; normals are generated in the kernel.
 */
int pr_fine_propagate(const pr_sde *sde, const pr_schedule *sched, uint64_t seed,
                      uint32_t instance, int64_t n, int slice_first, int slice_count,
                      void *x, void *y, void *stream);

/*
 * Restriction R (Sec. 3.2.2) of k ensembles of n particles to the empirical
 * quantile function of the slow variable (Sec. 4.4).  x: [k][n] (FP64, or
 * FP32 when precision == PR_F32), read only.  Outputs (any may be NULL
 * except q):
 *   q        [k][n_q+1]  knots at p_j = j/Q, midpoint (Hazen) convention:
 *                        t = p_j n - 1/2, min at t <= 0, max at t >= n-1,
 *                        else linear between order statistics floor(t), +1;
 *   rank     [k][n]      position of particle p in the stable ascending
 *                        order by (value, p); -0.0 orders before +0.0;
 *   perm     [k][n]      particle at each position (inverse of rank);
 *   x_sorted [k][n]      values in that order (FP64);
 *   moments  [k][4]      (1/n) sum_p x_p^m, m = 1..4 (eq. (MCestimator));
 *   hist     [k][I]      counts in cells floor((x-x_lo) I/(x_hi-x_lo))
 *                        clamped to [0, I-1] (eq. (binning)); uses the
 *                        cells of hist_grid (n_q of hist_grid is ignored).
 * hist_grid may be NULL when hist is NULL.  n_q >= 1.
 * ws: device workspace of at least pr_restrict_workspace_size() bytes.
 */
size_t pr_restrict_workspace_size(int64_t n, int k, int precision);
int pr_restrict_quantiles(const void *x, int precision, int64_t n, int k, int n_q,
                          const pr_grid *hist_grid, double *q, uint32_t *rank, uint32_t *perm,
                          double *x_sorted, double *moments, uint32_t *hist,
                          void *ws, size_t ws_bytes, void *stream);

/*
 * Matching preserving the fast marginal (Sec. 5.1, eq. (transformation)) in
 * quantile add/subtract form: for every particle of each of the k ensembles,
 *   u = (rank + 1/2)/n, j = min(floor(u Q), Q-1), w = u Q - j,
 *   x_out = x_prior + (1-w) d_j + w d_{j+1},  d = q_target - q_prior.
 * The fast variables and weights are untouched.  With q_target == q_prior the
 * output equals the input bitwise (eq. (projection)).  x_out may alias
 * x_prior.  q_*: [k][n_q+1]; rank: [k][n] from pr_restrict_quantiles of
 * x_prior; x_*: [k][n] of the given precision.
 */
int pr_match_quantiles(const double *q_target, const double *q_prior, const uint32_t *rank,
                       int64_t n, int k, int n_q, const void *x_prior, void *x_out,
                       int precision, void *stream);

/*
 * pr_restrict_quantiles for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments and results, bit for bit, without ws and
 * ws_bytes.  The workspace is a static device array of
 * PR_STATIC_SCRATCH_BYTES inside the library, one per GPU, held until the
 * process ends; its device address is looked up once per GPU.  The call
 * allocates nothing.  Requests whose workspace (pr_restrict_workspace_size)
 * exceeds the array return PR_E_NOMEM before anything is launched (64 MiB:
 * about 2.7 million FP64 keys over all k ensembles).  Every call on one GPU
 * shares its array, so calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller; the call clears what
 * it needs cleared itself.
 */
#define PR_STATIC_SCRATCH_BYTES (64u << 20)
int pr_restrict_quantiles_static(const void *x, int precision, int64_t n, int k, int n_q,
                                 const pr_grid *hist_grid, double *q, uint32_t *rank, uint32_t *perm,
                                 double *x_sorted, double *moments, uint32_t *hist, void *stream);

/*
 * Knots (Sec. 4.4, midpoint convention) of the matched ensembles without
 * sorting them.  For the k ensembles X that pr_match_quantiles(q_target,
 * q_prior, rank, n, k, n_q, x_prior, ...) makes from the priors, q_out
 * (device, [k][n_q+1]) receives the knots that pr_restrict_quantiles of X
 * would give, bit for bit: matching moves every prior value by a smooth
 * function of its rank, so the matched values in the prior's rank order are
 * nearly sorted, and every order statistic the knots need is found between
 * the nearest positions before and after its rank where all values before
 * lie below all values after.  ws, ws_bytes: the workspace of the
 * pr_restrict_quantiles call on x_prior that produced rank (same n, k,
 * precision), not used since; its sorted keys are read and the rest of its
 * key storage is overwritten.  flag (device, one int) is set to 1, else 0,
 * where some order statistic could not be isolated (matched values far from
 * the prior's order): q_out is then incomplete and the knots are to be
 * taken by pr_restrict_quantiles of X.  Returns PR_E_UNSUPPORTED, launching
 * nothing, when n is too small for the workspace to hold the chunk extremes
 * (2 keys per 64 particles).
 */
int pr_match_knots(const double *q_target, const double *q_prior, int64_t n, int k, int n_q,
                   int precision, void *ws, size_t ws_bytes, double *q_out, int *flag, void *stream);

/*
 * Coarse propagator C (Sec. 2.2): finite volumes for the slow Fokker-Planck
 * equation eq. (FPz) with the effective drift of eq. (Fbar),
 * V' = c3 x^3 + (c1 + lambda (1 - mean a)) x, Dbar = 1/beta, zero flux at the
 * grid ends, advanced by the exact exponential E(tau) = exp(A tau) with tau
 * the slice length (Sec. 2.2.2).  pr_coarse_create builds A on the host and
 * E(tau) on the device for every distinct slice length (synchronous).
 * pr_coarse_fp_step maps knots -> cell masses (piecewise-linear cdf through
 * the knots, eq. (discr_cdf)) -> E masses, clipped at 0 -> knots (flat
 * stretches give their midpoint, end knots are the grid ends), for slices
 * [slice_first, slice_first+slice_count) in parallel.  q_in, q_out:
 * [count][n_q+1]; rho_out: [count][I] or NULL.
 */
int pr_coarse_create(const pr_sde *sde, const pr_schedule *sched, const pr_grid *grid,
                     void *stream, void **coarse);
int pr_coarse_fp_step(const void *coarse, int slice_first, int slice_count,
                      const double *q_in, double *q_out, double *rho_out, void *stream);
/* Device pointer to E of slice n ([I][I], row-major) for inspection. */
int pr_coarse_matrix(const void *coarse, int slice, const double **E);
int pr_coarse_destroy(void *coarse);

/*
 * Quantile iterator J alone (Sec. 4.4, eq. (quantile_reconstruction)) on k
 * independent rows of n_q+1 knots at the levels p_j = j/Q: for every row s
 *   q_out[s] = PAVA(q_f[s] + (q_c_next[s] - q_c_star[s]))
 * evaluated in the order shown, so that J(a, f, a) = f bit for bit
 * (eq. (iterator_property)), then made non-decreasing by the monotone repair
 * of Sec. 4.4 (crossing quantiles replaced by their average), read as
 * pool-adjacent-violators with equal weights whose pool sums accumulate in
 * the order of the serial stack form.  This is one link of the serial chain
 * of pr_parareal_iterate without its coarse step (q_c_next = C_n(q^n)).
 * Arrays: device, [k][n_q+1]; q_out may alias an input row for row.
 * 1 <= n_q <= 2047.  k = 0 launches nothing.
 */
int pr_quantile_jump(const double *q_c_next, const double *q_f, const double *q_c_star, int k, int n_q,
                     double *q_out, void *stream);

/*
 * Micro-macro parareal (Sec. 3.2.3-3.2.4) with the quantile iterator
 * (Sec. 4.4, eq. (quantile_reconstruction); PAVA monotone repair) and
 * fast-marginal matching.  pr_parareal_create draws the initial ensemble and
 * runs the zeroth iteration (coarse pass from R(X0), matching against X0);
 * it owns all state buffers.  pr_parareal_iterate runs n_iter iterations
 * k -> k+1: fine propagation of every slice, restriction, coarse correction,
 * serial J chain, matching.  If q_ref (device, [N+1][n_q+1], the knots of the
 * serial fine run) is given, err_out (host, [n_iter][2]) receives for each
 * iteration the RMS knot error at n = N and its maximum over n.
 * pr_parareal_state copies the state at time index t (0..N) out: x [n],
 * y [d][n], q [n_q+1] (knots of that state), any may be NULL.
 */
int pr_parareal_create(const pr_sde *sde, const pr_schedule *sched, const pr_grid *grid,
                       uint64_t seed, uint32_t instance, int64_t n, int flags, void *stream,
                       void **h);
int pr_parareal_iterate(void *h, int n_iter, const double *q_ref, double *err_out, void *stream);
int pr_parareal_state(void *h, int t, void *x, void *y, double *q, void *stream);
int pr_parareal_iteration(const void *h);
/* Iterations since creation whose new knots were taken by a sort of the new
 * states (when pr_match_knots could not isolate them), or -1 for h NULL.
 * pr_parareal_iterate waits for its stream once per iteration to decide
 * this. */
int pr_parareal_knot_sorts(const void *h);
/* With PR_PROFILE: ms_out (host, PR_PH_COUNT doubles) receives the summed
 * device time of each phase over all iterations since creation, measured by
 * HIP events recorded on the iteration's stream; iterations (host, may be
 * NULL) receives how many iterations were timed.  Without PR_PROFILE the call
 * fails with PR_E_INVALID. */
int pr_parareal_profile(const void *h, double *ms_out, int *iterations);
int pr_parareal_destroy(void *h);

/*
 * Batched micro-macro parareal over many independent instances (d = 1, FP64,
 * a = NULL), each with its own SDE parameters, particle count n[i] and
 * schedule, sharing the coarse grid.  Host arrays sde, sched, n have n_inst
 * entries; instance (host, may be NULL for 0..n_inst-1) gives the Philox
 * instance word of each.  Creation draws every initial ensemble, builds the
 * coarse exponentials of every distinct slice length and runs the zeroth
 * iteration (synchronous).  flags: PR_REUSE_COARSE, PR_AUTOTUNE.
 * pr_parareal_batch_iterate runs n_iter iterations with the given launch
 * pattern; ms_out (host, may be NULL) receives their device time (HIP events
 * on stream; the call then waits for them).  The fine propagation of all
 * slices of all instances is one persistent launch whose workgroups take
 * (instance, slice, particle tile) units from a queue in decreasing cost.
 * pr_parareal_batch_state copies the state of instance inst at time t.
 * pr_parareal_batch_info reports the tuned block size and particles per
 * thread, the number of fine work units, the fine particle-steps of one
 * iteration and how the fine results are sorted (1: ensembles of 2^16 to
 * 2^20 + 2^16 FP64 keys by splitters and buckets, the rest by radix passes;
 * 0: all by radix passes).  With PR_AUTOTUNE, creation times the fine
 * kernel's shapes (block {128, 256} x particles per thread {1, 2, 4}, kept
 * per device) and the two sorts on the batch's own states (kept per batch;
 * both give the same bits); without it the defaults are 256, 2 and 1.
 * Every output pointer (host) may be NULL.  pr_parareal_batch_knot_sorts returns the number of batched
 * iterations whose new knots needed a sort of some new states (where the
 * knots from the fine results' order could not isolate an order statistic),
 * or -1 for h NULL; segments (host, may be NULL) receives how many
 * ensembles those sorts covered (only the flagged ones are sorted).  The
 * batched launch modes wait for their stream once per iteration to decide
 * this.  pr_draw_instances writes, for instances 0..count-1, the
 * batched-workload draw of (eps, lambda, log2 n, slices) from the tag-3
 * block of each: eps = 10^(-3+2u0), lambda = 0.5+1.5u1, log2 n =
 * 12+floor(7u2), slices = 8+floor(57u3), u_k = (w_k + 1/2) 2^-32.
 * out: device [count][4].
 */
int pr_draw_instances(uint64_t seed, int count, double *out, void *stream);
int pr_parareal_batch_create(int n_inst, const pr_sde *sde, const pr_schedule *sched, const int64_t *n,
                             const pr_grid *grid, uint64_t seed, const uint32_t *instance, int flags,
                             void *stream, void **h);
int pr_parareal_batch_iterate(void *h, int n_iter, int mode, double *ms_out, void *stream);
int pr_parareal_batch_state(void *h, int inst, int t, void *x, void *y, double *q, void *stream);
int pr_parareal_batch_info(const void *h, int *tuned_block, int *tuned_ppt, int64_t *units,
                           int64_t *particle_steps, int *split_sort);
int pr_parareal_batch_knot_sorts(const void *h, int64_t *segments);
int pr_parareal_batch_destroy(void *h);

/*
 * Pathwise adjoint of the fine propagator (d = 1, FP64, a = NULL) with
 * respect to theta = (lambda, eps, beta, c3), noise held fixed (the same
 * Philox numbers), for observables of the slow variable at the final step.
 *
 * pr_fine_checkpoint: Euler-Maruyama over all global steps [0, S) of sched
 *   (its slice count is ignored) from the state in x, y ([n] each, updated in
 *   place to step S), writing the state at steps 0, E, 2E, ... into
 *   ckpt [ceil(S/E)][2][n] (x then y), E = ckpt_every.
 * pr_observables: obs[0] = (1/n) sum x^2; obs[1+a] = midpoint (Hazen)
 *   quantile of x at level alpha[a] (host, a < n_alpha <= 3).  If seed_x is
 *   given ([1+n_alpha][n]) it receives d obs / d x_p with the order frozen:
 *   2 x_p / n, and (1-f), f at the two order statistics of a quantile.
 * pr_fine_adjoint: reverse sweep over the checkpointed trajectory.  Segments
 *   are replayed from their checkpoints (the noise regenerated from Philox),
 *   with states every 8 steps kept in the workspace and 8-step tapes in
 *   registers; the per-step noise increments are recovered from consecutive
 *   states.  seed_x (and seed_y or NULL) [n_seed][n] are dL_k/dX_S,
 *   dL_k/dY_S; grad [n_seed][4] (device) receives dL_k/d(lambda, eps, beta,
 *   c3).  from_initial != 0 adds the dependence of the initial law
 *   Y0 = X0 + beta^-1/2 z on beta (the checkpoint at step 0 must then be the
 *   initial ensemble of pr_init_ensemble).  n_seed <= 4.  Workspace:
 *   pr_adjoint_workspace_size bytes.  Other d or precisions: PR_E_UNSUPPORTED.
 */
int pr_fine_checkpoint(const pr_sde *sde, const pr_schedule *sched, uint64_t seed, uint32_t instance,
                       int64_t n, void *x, void *y, double *ckpt, int ckpt_every, void *stream);
size_t pr_observables_workspace_size(int64_t n);
int pr_observables(const double *x, int64_t n, const double *alpha, int n_alpha, double *obs,
                   double *seed_x, void *ws, size_t ws_bytes, void *stream);
size_t pr_adjoint_workspace_size(int64_t n, int ckpt_every, int n_seed);
int pr_fine_adjoint(const pr_sde *sde, const pr_schedule *sched, uint64_t seed, uint32_t instance,
                    int64_t n, const double *ckpt, int ckpt_every, const double *seed_x,
                    const double *seed_y, int n_seed, int from_initial, double *grad, void *ws,
                    size_t ws_bytes, void *stream);

/*
 * Histogram-state micro-macro parareal (Sec. 4, Sec. 5): the macroscopic
 * state is the vector of cell masses rho[I] of the slow variable on the grid
 * (eq. (integral)); the ensembles are FP64 with optional particle weights.
 * Cell i is [x_i, x_{i+1}) with index floor((x - x_lo) I/(x_hi - x_lo))
 * clamped to the grid; at most 1024 cells.
 */
enum {                  /* iterators J(rho_c^{n+1}, rho_f^*, rho_c^*), Sec. 4    */
    PR_J_ADD = 0,       /* rho_f + (rho_c^{n+1} - rho_c^*); negative cells set to 0
                           and then the result scaled to the mass of rho_f      */
    PR_J_MULT = 1,      /* rho_f (rho_c^{n+1} / rho_c^*) where rho_c^* > 0, else 0,
                           scaled to the mass of rho_f                           */
    PR_J_ROT = 2,       /* rotation of sqrt(rho_f) in the plane of sqrt(rho_c^*)
                           and sqrt(rho_c^{n+1}) (Sec. 4.3, closed form)         */
    PR_J_QUANTILE = 3   /* quantile add/subtract on the union of the three cdfs'
                           edge levels, pool-adjacent-violators, back to masses  */
};
enum {                       /* matchings M(rho, prior), Sec. 5                   */
    PR_M_MARGINAL = 0,       /* X = q_rho(cbar(Xbar)) on piecewise-linear cdfs;
                                fast variables and weights unchanged            */
    PR_M_REWEIGHT = 1,       /* W = Wbar rho'_i / rhobar_i, rho' = rho with the
                                mass of cells without prior particles handed to
                                the nearest supported cells                    */
    PR_M_RESAMPLE = 2,       /* reweighting, then stratified resampling with
                                u_j = (j + U[0,1))/P drawn from the seed         */
    PR_M_RESAMPLE_DET = 3    /* the same with u_j = (j + 1/2)/P                   */
};

/* rho[s][I] (device) = weighted histogram of x[s][n] (device), s < k; w[s][n]
 * the weights or NULL for equal weights RN(1/n).  Each mass is the exact sum
 * of its cell's weights rounded once (weights in [2^-60, 2^15) or 0).
 * Workspace: pr_hist_workspace_size(k, n_cells) bytes. */
size_t pr_hist_workspace_size(int k, int n_cells);
int pr_hist_restrict(const double *x, const double *w, int64_t n, int k, const pr_grid *grid, double *rho,
                     void *ws, size_t ws_bytes, void *stream);

/* rho_out[s] = J(rho_c[s], rho_f[s], rho_cs[s]) for k independent triples of
 * histograms [k][I] (device); rho_out must not alias an input.  The quantile
 * iterator needs pr_hist_jump_workspace_size(k, n_cells) bytes of workspace
 * (the others accept ws = NULL).  Sums over the cells run left to right. */
size_t pr_hist_jump_workspace_size(int k, int n_cells);
int pr_hist_jump(int kind, const double *rho_c, const double *rho_f, const double *rho_cs, int k,
                 const pr_grid *grid, double *rho_out, void *ws, size_t ws_bytes, void *stream);

/* Matching of k ensembles of n particles.  rho_t [k][I] targets, rho_p [k][I]
 * the histograms of the priors (pr_hist_restrict of x, w); prior x [n] or
 * [k][n] (prior_stride 0 or n), y [D][n] or [k][D][n], w likewise or NULL
 * for equal weights.  Outputs [k][n], [k][D][n], [k][n]:
 *   MARGINAL writes x_out only (may equal x);
 *   REWEIGHT writes w_out only (may equal w);
 *   RESAMPLE(_DET) writes x_out, y_out, w_out (no aliasing with the prior);
 *     slot j of ensemble s takes the prior particle p whose cumulative
 *     fixed-point weight interval holds U_j (Philox block (tag 4, m = 0,
 *     p = j, pair = t_first + s, instance) for the random variant).
 * Workspace: pr_hist_match_workspace_size(n, k, n_cells) bytes. */
size_t pr_hist_match_workspace_size(int64_t n, int k, int n_cells);
int pr_hist_match(int kind, const double *rho_t, const double *rho_p, int64_t n, int k, int d,
                  const pr_grid *grid, const double *x, const double *y, const double *w, int64_t prior_stride,
                  double *x_out, double *y_out, double *w_out, uint64_t seed, uint32_t instance, int t_first,
                  void *ws, size_t ws_bytes, void *stream);

/* Histogram-state parareal driver (FP64).  create runs the zeroth iteration
 * (rho^0 = R(X0), rho^{n+1} = C_n(rho^n), X^n = M(rho^n; X0)); iterate runs
 * generic iterations: fine propagation of every slice, restriction of the
 * fine results and of the current states, coarse propagation, the serial
 * chain of coarse step and iterator, matching against the fine results.
 * Flags: PR_REUSE_COARSE (C of the previous macro states), PR_PROFILE.
 * rho_ref [K+1][I] (device) makes iterate compute the L2 error of the new
 * states' histograms per time point; err_out (host) receives [n_iter][2]:
 * the error at n = N and the maximum over n. */
int pr_parareal_hist_create(const pr_sde *sde, const pr_schedule *sched, const pr_grid *grid, uint64_t seed,
                            uint32_t instance, int64_t n, int iterator, int matching, int flags, void *stream,
                            void **h);
int pr_parareal_hist_iterate(void *h, int n_iter, const double *rho_ref, double *err_out, void *stream);
int pr_parareal_hist_state(void *h, int t, double *x, double *y, double *w, double *rho, void *stream);
int pr_parareal_hist_iteration(const void *h);
int pr_parareal_hist_profile(const void *h, double *ms_out, int *iterations);
int pr_parareal_hist_destroy(void *h);

/*
 * Chemical-reaction system (Sec. 2.1.2, the paper's own workload): slow X,
 * fast Y (d = 1), multiplicative noise, eq. (SDEx)/(SDEy) with
 *   D(x, y) = (k4 y + k5 x)/2,
 *   E(y)    = (k0 + k1 y + k2 y(y-1) + k3 y(y-1)(y-2))/2,
 * half the summed propensities of the reactions 0 -> Y (k0), Y -> 0 (k1 y),
 * 2Y -> 3Y (k2 y(y-1)), 3Y -> 2Y (k3 y(y-1)(y-2)), Y -> Y + X (k4 y),
 * X -> 0 (k5 x), and the drifts of those reactions (chemical Langevin form):
 *   -dF/dx = k4 y - k5 x,  -dG/dy = k0 - k1 y + k2 y(y-1) - k3 y(y-1)(y-2).
 * D and E enter the square roots as max(., 0).  Table 1 of the paper gives
 * tau_x = 25, eps = 2.5e-2, k = (60, 1, 4.8e-3, k3, 0.833, 1); with k3 read
 * as 0.666e-5 the fast variable is bistable (stable states near 105 and 408).
 * Initial law (Sec. 6): independent lognormal X0, Y0 with the given means
 * and standard deviations.
 */
typedef struct pr_chem {
    double tau_x;              /* slow time scale, > 0                          */
    double eps;                /* time-scale separation, > 0                    */
    double k[6];               /* reaction rates k0..k5, >= 0, k4, k5 > 0       */
    double x0_mean, x0_sd;     /* lognormal X0: mean > 0, sd >= 0               */
    double y0_mean, y0_sd;     /* lognormal Y0: mean > 0, sd >= 0               */
} pr_chem;

/* Initial ensemble: log X0 = mu_x + s_x z0, log Y0 = mu_y + s_y z1 with
 * s^2 = log(1 + sd^2/mean^2), mu = log(mean) - s^2/2, (z0, z1) the normal
 * pair (tag 1, m = 0, p, j = 0).  x, y: device, [n] FP64. */
int pr_chem_init_ensemble(const pr_chem *c, uint64_t seed, uint32_t instance, int64_t n, double *x, double *y,
                          void *stream);

/* Fine propagator of the chemical system: Euler-Maruyama (eq. (EMx)/(EMy)),
 * drift and diffusion at the old state, normals (z0, z1) of pair
 * (tag 0, m, p, j = 0):
 *   X' = X + (dt/tau_x)(k4 Y - k5 X) + sqrt(2 max(D, 0) dt/tau_x) z0
 *   Y' = Y + (dt/eps) b(Y)          + sqrt(2 max(E, 0) dt/eps) z1
 * over every slice in [slice_first, slice_first+slice_count) at once, in
 * place: x [slice_count][n], y [slice_count][n] (device, FP64). */
int pr_chem_fine_propagate(const pr_chem *c, const pr_schedule *sched, uint64_t seed, uint32_t instance, int64_t n,
                           int slice_first, int slice_count, double *x, double *y, void *stream);

/* ybar (host): the mean of the fast variable's equilibrium density
 * phi(y) ~ exp(int_0^y b(s)/E(s) ds)/E(y) (Sec. 2.2.1, the chemical
 * reactions example), both integrals by the trapezoidal rule on the uniform
 * grid of [0, 1000] with spacing 1e-2. */
int pr_chem_mean_fast(const pr_chem *c, double *ybar);

/* Coarse propagator of the chemical system: the finite-volume scheme of
 * Sec. 2.2.2 for eq. (FPz) with Fbar'(x) = -(k4 ybar - k5 x) and
 * Dbar(x) = (k4 ybar + k5 x)/2 (eq. (Fbar)/(Dbar) with phi independent of x),
 * rho_inf(x) = exp(-int_0^x Fbar'/Dbar ds)/Dbar(x), edge coefficients
 * Dbar(x_i) rho_inf(x_i)/(tau_x h), zero flux at the grid ends, advanced by
 * E(tau) = exp(A tau) per distinct slice length.  Needs k4 ybar + k5 x_lo
 * > 0.  The handle serves pr_coarse_fp_step, pr_coarse_matrix and
 * pr_coarse_destroy like that of pr_coarse_create (synchronous). */
int pr_chem_coarse_create(const pr_chem *c, const pr_schedule *sched, const pr_grid *grid, void *stream,
                          void **coarse);

/* Histogram-state parareal driver on the chemical system: as
 * pr_parareal_hist_create, with the chemical fine propagator, initial law
 * and coarse propagator (d = 1).  The handle is driven and released with the
 * pr_parareal_hist_* calls. */
int pr_parareal_hist_create_chem(const pr_chem *c, const pr_schedule *sched, const pr_grid *grid, uint64_t seed,
                                 uint32_t instance, int64_t n, int iterator, int matching, int flags, void *stream,
                                 void **h);

/*
 * Linear-advection study (Sec. 6, the linear advection case): the slow
 * Fokker-Planck equation eq. (FPz) with Fbar(x) = x/eps and Dbar = 1/beta
 * (tau_x = 1), discretised by the finite-volume scheme of Sec. 2.2.2 with
 * rho_inf(x) ~ exp(-beta x/eps) and zero flux at the grid ends, advanced by
 * E(tau) = exp(A tau) per distinct slice length.  eps, beta > 0.  The handle
 * serves pr_coarse_fp_step, pr_coarse_matrix, pr_coarse_destroy and the
 * deterministic parareal below (synchronous).
 */
int pr_advection_coarse_create(double eps, double beta, const pr_schedule *sched, const pr_grid *grid,
                               void *stream, void **coarse);

/*
 * Deterministic parareal on cell masses (Sec. 6, the linear advection case):
 * the fine and the coarse propagator are two coarse handles (any model) of
 * the same grid and slice count, each applying its E once per slice with
 * negative rounding residue clipped to 0; restriction and matching are the
 * identity; the iterator is one of PR_J_* (as in pr_hist_jump).  create
 * copies rho0 (device, [I]) and runs the zeroth iteration
 * rho^{n+1} = C_n(rho^n); iterate runs n_iter iterations
 * rho_{k+1}^{n+1} = J(C_n(rho_{k+1}^n), F_n(rho_k^n), C_n(rho_k^n)), the fine
 * and coarse propagation of all slices in one batched launch each and the
 * serial chain one link per slice.  With rho_ref (device, [N+1][I]),
 * err_out (host, [n_iter][2]) receives after each iteration the L2 error at
 * n = N and its maximum over n.  The handles must outlive the parareal
 * handle.  flags: 0.
 */
int pr_parareal_fp_create(const void *fine, const void *coarse, const pr_grid *grid, const double *rho0,
                          int iterator, int flags, void *stream, void **h);
int pr_parareal_fp_iterate(void *h, int n_iter, const double *rho_ref, double *err_out, void *stream);
int pr_parareal_fp_state(void *h, int t, double *rho, void *stream);
int pr_parareal_fp_iteration(const void *h);
int pr_parareal_fp_destroy(void *h);

#ifdef __cplusplus
}
#endif

#endif /* PR_H */
