/*
 * sp2dm.h -- C ABI of the MI355X (gfx950) SP2 / SP2ACC density-matrix library.
 *
 * The library computes the zero-temperature density matrix D = theta(mu I - F)
 * of a symmetric block-sparse Fock/Kohn-Sham matrix F by the recursive
 * second-order spectral projection expansion with scale-and-fold acceleration
 * and error-controlled truncation, following Kruchinina, Rudberg, Rubensson,
 * "Efficient computation of the density matrix with error control on
 * distributed computer systems" (arXiv:1909.12533):
 *   - problem statement: F symmetric, n_occ occupied orbitals, a non-zero
 *     homo-lumo gap, D = sum_{i<=n_occ} y_i y_i^T (section "Introduction");
 *   - Step 1 / Algorithm 1 / Algorithm 2 / Step 3 of section "Density matrix
 *     construction" (schedule, initialisation, iteration with truncation and
 *     parameterless stopping, homo/lumo estimates);
 *   - truncation thresholds of eq. (tau_trunc) and the bound on the
 *     occupied-subspace error (section "Error control");
 *   - Frobenius and Frob-Inf truncation norms (section "Upper bounds for the
 *     spectral norm");
 *   - symmetric storage of the upper triangle only (section "Implementation
 *     details").
 *
 * Every operation runs on the GPU in hand-written HIP kernels; the host only
 * sequences them and evaluates scalar formulas (schedule, stopping test,
 * homo/lumo back-propagation, error bookkeeping) in IEEE double precision.
 *
 * Conventions
 * -----------
 * Matrices are "upper BSR" (sp2_bsr): n x n, block size bs = 64 (the only
 * supported value), nbr = ceil(n / 64) block rows, nnzb stored blocks (I, J)
 * with J >= I, sorted by (I, J); row_ptr[nbr + 1] (int64), col_idx[nnzb]
 * (int32), val[nnzb * 64 * 64] (double, each block row-major).  A block below
 * the diagonal is the transpose of its stored mirror; diagonal blocks are
 * full symmetric 64 x 64 blocks.  When n is not a multiple of 64, rows and
 * columns >= n of the last block row/column are padding and must be 0.
 * All pointers inside sp2_bsr are DEVICE pointers on the context's device.
 *
 * Ownership: inputs are borrowed; they must stay valid until the call returns
 * (every call is synchronous with respect to the host: it returns after the
 * context's stream has finished the work it issued).  Matrices returned
 * through "sp2_bsr **out" are allocated by the library (through the allocator
 * installed with sp2_set_allocator, or hipMalloc) and released with
 * sp2_bsr_free.  A tape is released with sp2_tape_free.
 *
 * Return codes: 0 = success; negative = error, no output written (*out left
 * NULL), message in sp2_last_error; positive = warning, outputs valid.
 * A context is not thread-safe; use one context per host thread / stream.
 */
#ifndef SP2DM_H
#define SP2DM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SP2_OK 0
#define SP2_ERR_INVALID_ARG (-1) /* n_occ not in (0, n), bs != 64, lmin >= lmax, bad pattern ... */
#define SP2_ERR_BAD_BOUNDS (-2)  /* not (lmin <= homo_ub < lumo_lb <= lmax) */
#define SP2_ERR_NONFINITE (-3)   /* F (or another input) holds NaN / Inf */
#define SP2_ERR_OOM (-4)         /* device allocation failed */
#define SP2_ERR_HIP (-5)         /* HIP runtime error */
#define SP2_WARN_NOT_CONVERGED 1 /* n_max reached before the stopping criterion fired (not raised when a
                                    mixed run's FP64 tail reaches n_max before the criterion could be
                                    evaluated: its two e values must come from FP64 squares) */
#define SP2_WARN_TRACE 2         /* |tr D - n_occ| > 1/2: bounds wrong or gap closed */

#define SP2_BLOCK 64

/* precision of the bulk squares */
#define SP2_PREC_FP64 0   /* every square in FP64 MFMA (the plain FP64 square loads its operands straight
                             to LDS; SP2_F64_KERNEL=tile in the environment selects the register-staged
                             kernel, bit-identical) */
#define SP2_PREC_FP32 1   /* FP32 MFMA squares (FP32 storage) until e_i < switch_tol, then FP64 */
#define SP2_PREC_BF16X3 2 /* BF16 hi/lo split MFMA (hi*hi + hi*lo + lo*hi, FP32 accumulate), then FP64.
                             Products whose output pattern holds >= 35% of the upper blocks run on
                             4 x 4-block tiles, sparser ones on 2 x 2 (bit-identical results); the
                             environment variable SP2_BF16X3_TILE = 2 or 4 forces one of them. */

/* truncation norm (section "Upper bounds for the spectral norm") */
#define SP2_TRUNC_NONE 0
#define SP2_TRUNC_FROB 1
#define SP2_TRUNC_FROBINF 2

/* stop reasons */
#define SP2_STOP_CRITERION 1   /* e_i > C e_{i-2}^2 with p_i != p_{i-1} (Algorithm 2) */
#define SP2_STOP_IDEMPOTENCY 2 /* e_i <= idem_stop */
#define SP2_STOP_NMAX 3        /* i = n_max */
#define SP2_STOP_NOISE_FLOOR 4 /* low_floor_stop: a low-precision e_i below ten times its rounding noise */

typedef struct sp2_ctx sp2_ctx;
typedef struct sp2_tape sp2_tape;

typedef struct {
  int64_t n;        /* matrix dimension */
  int32_t bs;       /* block size, must be 64 */
  int32_t owned;    /* 1: allocated by the library, release with sp2_bsr_free */
  int64_t nbr;      /* ceil(n / bs) */
  int64_t nnzb;     /* stored blocks */
  int64_t *row_ptr; /* device, nbr + 1 */
  int32_t *col_idx; /* device, nnzb */
  double *val;      /* device, nnzb * bs * bs */
} sp2_bsr;

typedef struct {
  int32_t accel;        /* 1: SP2ACC (scale-and-fold), 0: SP2 (alpha_i = 1, n_min = 1) */
  int32_t precision;    /* SP2_PREC_* */
  double switch_tol;    /* mixed precision: FP64 from the first square after e_i < switch_tol;
                           < 0: no FP64 tail, the low precision to its own stopping criterion */
  int32_t trunc_norm;   /* SP2_TRUNC_* */
  int32_t n_max_cap;    /* cap of n_max, and n_max of the trace-correcting run (<= 1000) */
  int64_t coarse_bs;    /* Frob-Inf submatrix size, a multiple of 64 (paper: 4096) */
  double gamma;         /* allowed occupied-subspace error, eq. (tau_trunc); used when tau_fixed == 0 */
  double tau_fixed;     /* > 0: the same threshold tau for every iteration */
  double idem_stop;     /* > 0: also stop when e_i <= idem_stop */
  int32_t record_tape;  /* 1: keep the masks and checkpoints needed by vjp / jvp / replay */
  int32_t n_checkpoints;/* number of X~_i checkpoints in the tape; 0 = ceil(sqrt(n)); a checkpoint that
                           would take the tape beyond min(20% of the device, 30% of free memory) is
                           skipped (the adjoint then replays from an earlier one) */
  int32_t correct;      /* rounds of the FP64 occupied-subspace correction after the expansion (0 = none);
                           see "Subspace correction" below */
  int32_t corr_purify;  /* FP64 purification squares after each correction round (>= 1; default 2) */
  double corr_tol;      /* Frobenius budget for dropping small blocks of every intermediate of the
                           correction (0 = default 1e-9) */
  int64_t corr_mem;     /* device bytes for the copies of X~_i kept for the correction; the iterates
                           beyond that go to pinned host memory (corr_host_mem) or are recomputed
                           (0 = min(25% of the device, 35% of free memory)) */
  int32_t adjoint_precision; /* arithmetic of sp2_vjp / sp2_jvp steps at the iterations the forward ran in
                           low precision: -1 = the forward's (default), else SP2_PREC_* */
  double corr_deriv_tol;   /* the correction's derivative steps stop at the first X~_k with e_k below this
                              (0 = default 1e-2) */
  int32_t corr_mcweeny;    /* 1: each purification is one McWeeny step P' = 3P^2 - 2P^3 formed as
                              S - (P R + R P) with S = P^2 an FP64 square and R = S - P, the small product
                              P R + R P in the run's low arithmetic (corr_purify is then the number of such
                              steps); 0: corr_purify FP64 squares X^2, 2X - X^2, ... */
  int64_t corr_host_mem;   /* pinned host bytes for the copies of X~_i beyond corr_mem (written and read
                              back on a second stream, overlapped with the squares); 0 = 75% of the
                              available host memory, < 0 = none (those iterates are recomputed) */
  double low_start_xi;     /* mixed precision with homo/lumo bounds: the squares stay in FP64 until the
                              first X~_i whose gap image xi_i = 1 - q_i - l_i (section "Error control")
                              reaches this value, then run in the low precision (0 = from X~_0; must be
                              in [0, 1); ignored by the trace-correcting run) */
  int32_t tail_storage;    /* storage of the FP64 tail's iterates: 0 = FP64 (default); 1 = FP32, the tail's
                              squares multiplying the FP32-stored values in FP64 arithmetic (for expansions
                              whose FP64 iterates do not fit in device memory: the same memory as the FP32
                              squares, an idempotency floor of about the FP32 rounding of the iterate,
                              ~2^-24 ||X||_F, instead of the FP32 squares' accumulation noise); not
                              combined with the correction */
  int32_t low_floor_stop;  /* 1: an expansion that stays in the low precision to its end (switch_tol <= 0 with
                              the correction, or < 0) stops at the first e_i below ten times its rounding
                              noise (the level from which the FP64 tail would start: the low-precision
                              squares no longer resolve convergence), before the criterion of Algorithm 2,
                              which needs e_i to stop decreasing; 0 (default): by the criterion */
} sp2_options;

/* Per-run statistics.  Arrays are HOST arrays owned by the caller, each of
 * length `capacity` (>= n_max_cap + 1); entry i refers to X~_i.  Any array
 * pointer may be NULL. */
typedef struct {
  int32_t capacity;
  int32_t n_iter;       /* n: D = X~_n */
  int32_t n_max, n_min;
  int32_t stop_reason;  /* SP2_STOP_* */
  int32_t switch_iter;  /* mixed precision: first iteration squared in FP64 (-1: none) */
  double homo_ub_est;   /* Step 3 estimates (NaN when no iteration qualified) */
  double lumo_lb_est;
  double subspace_err_bound; /* sum_i ||E_i||_M / (xi_i - ||E_i||_M) ("Error control"); NaN without bounds */
  double time_s;        /* wall time of the expansion (device resident input to device resident D) */
  double alg_flops;     /* sum_i 2 * 64^3 * #{(I,K,J): I <= J, X~_IK != 0 != X~_KJ} */
  int64_t max_nnzb;
  double *e;            /* ||X~_i - X~_i^2||_F */
  double *t;            /* tr(X~_i - X~_i^2) */
  double *trace;        /* tr X~_i */
  double *alpha;
  double *tau;
  double *trunc_err_frob;  /* ||E_i||_F */
  double *trunc_err_mixed; /* ||E_i||_M */
  double *iter_time_s;
  double *iter_flops;
  int32_t *p;
  int32_t *precision;   /* precision of the square of X~_i */
  int64_t *nnzb;        /* stored upper blocks of X~_i */
  double *square_time_s;   /* device time of the MFMA square of X~_i (HIP events on the context stream) */
  double square_time_total_s; /* sum of square_time_s over the run */
  /* subspace correction (zero when opt->correct == 0) */
  int32_t corr_rounds;
  double corr_time_s;      /* wall time of all rounds (part of time_s) */
  double corr_flops;       /* algorithmic flops of their block products (part of alg_flops) */
  double corr_delta_norm;  /* ||Delta||_F of the last round, Delta = [D, [D, F]] */
  double corr_step_norm;   /* ||dD||_F of the last round (the first-order correction) */
  double corr_e_last;      /* ||P - P^2||_F of the input P of the last purification square */
  int64_t corr_max_nnzb;   /* largest pattern among the correction's intermediates */
  int64_t seq_bytes;       /* device bytes of the stored X~_i sequence the correction replays */
  int64_t seq_host_bytes;  /* pinned host bytes of the part of that sequence kept in host memory */
  int32_t corr_recomputed; /* iterates the correction recomputed (not stored) */
  int64_t device_peak_bytes; /* largest device memory the library held at once during the call */
} sp2_stats;

typedef void *(*sp2_alloc_fn)(size_t bytes, void *user);
typedef void (*sp2_free_fn)(void *ptr, void *user);

/* Library version string. */
const char *sp2_version(void);

/* Fill *opt with the defaults: SP2ACC, FP64, switch_tol 1e-3, Frob-Inf,
 * n_max_cap 100, coarse_bs 4096, gamma 1e-3, tau_fixed 0, idem_stop 0,
 * no tape, no subspace correction (corr_purify 2, corr_tol 1e-9, corr_mem 0),
 * adjoint_precision -1, corr_deriv_tol 0, corr_mcweeny 0, corr_host_mem 0, low_start_xi 0,
 * tail_storage 0, low_floor_stop 0. */
void sp2_options_default(sp2_options *opt);

/* Create a context on HIP device `device` issuing all work on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  Returns SP2_ERR_HIP when the
 * device cannot be used. */
int sp2_create(sp2_ctx **ctx, int device, void *hip_stream);
void sp2_destroy(sp2_ctx *ctx);

/* Route every device allocation of the library through (alloc, free_).
 * alloc must return device memory on the context's device usable on its
 * stream, or NULL on failure.  NULL restores hipMalloc / hipFree.  Buffers
 * cached by the context are released first. */
int sp2_set_allocator(sp2_ctx *ctx, sp2_alloc_fn alloc, sp2_free_fn free_, void *user);

/* Release device buffers cached between calls. */
void sp2_trim(sp2_ctx *ctx);

/* Message of the last error on this context ("" when none). */
const char *sp2_last_error(const sp2_ctx *ctx);

/* Gershgorin interval [lmin, lmax] containing the spectrum of F (Step 1:
 * lambda_min <= lambda_1 and lambda_max >= lambda_N). */
int sp2_gershgorin(sp2_ctx *ctx, const sp2_bsr *F, double *lmin, double *lmax);

/* Subspace correction (opt->correct > 0).  Squares in low precision perturb
 * the occupied subspace, and later iterations keep such a perturbation
 * instead of removing it (section "Error control": an error in the occupied
 * subspace is not recovered); an FP64 tail restores idempotency and trace but
 * not the subspace.  After the expansion, each round takes the current
 * D (a near-projector) and
 *   Delta = [D, [D, F]] = D F (I - D) + (I - D) F D          (C = [D, F] is
 *           accumulated in FP64; it is small, so it is stored and [D, C] is
 *           formed in the low precision)
 *   dD    = J Delta, J the derivative of the expansion's map F -> D
 *           (dX~_0 = -Delta / (lmax - lmin), dX~_i = b_i dX~_{i-1}
 *           + c_i (X~_{i-1} dX~_{i-1} + dX~_{i-1} X~_{i-1}) along the stored
 *           X~_0 .. X~_{n-1} with the run's polynomials)
 *   D     <- purified (D + dD): corr_purify FP64 steps X^2, 2X - X^2, ...
 * In the eigenbasis of F the occupied-virtual part of Delta is
 * (lambda_v - lambda_o) E_ov for D = theta + E, and J divides that part by
 * (lambda_o - lambda_v), so D + dD removes E to first order; the residual is
 * O(||E||^2 / gap).  Blocks of C, Delta and every dX~_i are dropped while the
 * Frobenius norm of the dropped part stays within corr_tol.  With
 * switch_tol = 0 the expansion runs in the low precision to its stopping
 * criterion (evaluated on the low-precision e_i) and the purification replaces
 * the FP64 tail.  Copies of X~_0, X~_1, ... are kept on the device within
 * corr_mem bytes (stats->seq_bytes), then in pinned host memory within
 * corr_host_mem bytes (stats->seq_host_bytes); iterates beyond both are
 * recomputed from their recorded masks and polynomials, bit for bit.
 * Derivative steps from the first iterate with e_i < corr_deriv_tol on are
 * skipped: near a projector they only keep the occupied-virtual part, which
 * the purification leaves in place. */

/* Density matrix by SP2 / SP2ACC (Steps 1-3, Algorithms 1-2).
 *   F         symmetric input in upper BSR (device)
 *   n_occ     number of occupied orbitals, 0 < n_occ < n
 *   lmin/lmax spectral bounds, lmin <= lambda_1, lmax >= lambda_N
 *   homo_ub, lumo_lb  pointers to bounds homo <= *homo_ub < *lumo_lb <= lumo,
 *             or both NULL: trace-correcting run (alpha = 1, p_i from traces,
 *             thresholds tau_fixed), the first run of the paper's protocol
 *   opt       options (NULL = defaults)
 *   D_out     receives D = X~_n (library-owned upper BSR)
 *   homo_est, lumo_est  receive updated bounds from Step 3 (NaN if none)
 *   stats     optional per-iteration statistics (caller-owned host arrays)
 *   tape      optional: receives the tape for sp2_vjp / sp2_jvp / sp2_replay
 *             (requires opt->record_tape = 1)
 * Returns 0, a warning (> 0) or an error (< 0). */
int sp2_density(sp2_ctx *ctx, const sp2_bsr *F, int64_t n_occ, double lmin, double lmax,
                const double *homo_ub, const double *lumo_lb, const sp2_options *opt,
                sp2_bsr **D_out, double *homo_est, double *lumo_est, sp2_stats *stats,
                sp2_tape **tape);

/* The expansion one unit of work at a time.  sp2_density_begin,
 * sp2_density_step and sp2_density_end perform exactly the work of
 * sp2_density (same arithmetic, same results), split so that a caller can run
 * it in pieces (interleave other work, watch progress, time single
 * iterations):
 *   begin  Step 1 (schedule) and Algorithm 1 (X_0 = (lmax I - F) / w and its
 *          truncation); arguments as sp2_density; *solver receives the handle;
 *   step   one iteration of Algorithm 2 (square of X~_i with the fused
 *          update, e_i and t_i, the stopping test, truncation of X_{i+1}) or,
 *          once the expansion has stopped, one block product of the subspace
 *          correction (opt->correct > 0); *info (may be NULL) describes the
 *          step, info->done = 1 when nothing is left; calling it after that
 *          is an error;
 *   end    Step 3 and the outputs (D_out, estimates, stats, tape) exactly as
 *          sp2_density; only valid after *done = 1.
 * F is borrowed until sp2_density_end returns.  The handle is released with
 * sp2_solver_free (also after end, and after any error: a failed step leaves
 * it unusable).  stats->time_s is the time spent inside the three calls. */
typedef struct sp2_solver sp2_solver;
#define SP2_STEP_ITERATION 1  /* one iteration of Algorithm 2 */
#define SP2_STEP_CORRECTION 2 /* one product of the subspace correction */
typedef struct {
  int32_t done;           /* 1: nothing left, call sp2_density_end */
  int32_t kind;           /* SP2_STEP_* */
  int32_t iteration;      /* i of the square of X~_i (SP2_STEP_ITERATION), else -1 */
  int32_t precision;      /* SP2_PREC_* of the step's dominant block products */
  double flops;           /* algorithmic flops of the step's block products (2 * 64^3 each) */
  double wall_s;          /* time spent in the call */
  double kernel_s[3];     /* device time of the MFMA product kernels by arithmetic (index SP2_PREC_*),
                             from HIP events on the context stream */
  double kernel_flops[3]; /* algorithmic flops of those launches, same index (a recomputed iterate's
                             square counts here but not in flops) */
  int32_t kernel_launches[3]; /* number of those launches, same index */
} sp2_step_info;
int sp2_density_begin(sp2_ctx *ctx, const sp2_bsr *F, int64_t n_occ, double lmin, double lmax,
                      const double *homo_ub, const double *lumo_lb, const sp2_options *opt, sp2_solver **solver);
int sp2_density_step(sp2_ctx *ctx, sp2_solver *solver, sp2_step_info *info);
int sp2_density_end(sp2_ctx *ctx, sp2_solver *solver, sp2_bsr **D_out, double *homo_est, double *lumo_est,
                    sp2_stats *stats, sp2_tape **tape);
void sp2_solver_free(sp2_ctx *ctx, sp2_solver *solver);

/* Vector-Jacobian product of the recorded (frozen schedule and masks) map
 * F -> D: Fbar = (dL/dF) for L = tr(W D), W symmetric in upper BSR on any
 * pattern.  X~_i are recomputed from the tape's checkpoints; recomputed
 * iterates are kept for the next steps within min(20% of the device, 30% of
 * free memory) and recomputed again beyond that.  Each step
 * Xbar <- cb G + cc (X~ G + G X~) runs in the arithmetic the forward used for
 * that X~_i (FP64, or FP32 values with FP32 / BF16x3 products for the
 * low-precision iterations of a mixed run), or in the one the forward's
 * options named in adjoint_precision.  The map excludes the subspace
 * correction (sp2_options.correct). */
int sp2_vjp(sp2_ctx *ctx, const sp2_tape *tape, const sp2_bsr *W, sp2_bsr **Fbar_out);

/* Jacobian-vector product dD = (dD/dF) dF of the recorded map (arithmetic
 * per step as in sp2_vjp). */
int sp2_jvp(sp2_ctx *ctx, const sp2_tape *tape, const sp2_bsr *dF, sp2_bsr **dD_out);

/* The recorded map applied to another F (same n): schedule, n and masks
 * frozen.  Used for finite differences. */
int sp2_replay(sp2_ctx *ctx, const sp2_tape *tape, const sp2_bsr *F, sp2_bsr **D_out);

/* Tape facts: number of iterations, checkpoints held, bytes held on the device. */
int sp2_tape_info(const sp2_tape *tape, int32_t *n_iter, int32_t *n_checkpoints, int64_t *device_bytes);

/* ---- host scalar control (no GPU involved) ------------------------------ */

/* Step 1 schedule from homo/lumo bounds (section "Density matrix
 * construction"): polynomial sequence p_i, scale-and-fold parameters alpha_i
 * (alpha_i = 1 for SP2, accel = 0), the bound images l_i (unoccupied images in
 * [0, l_i]) and q_i (occupied images in [1 - q_i, 1]), the gap bounds
 * xi_i = 1 - l_i - q_i and thresholds tau_i of eq. (tau_trunc) (or tau_fixed
 * when > 0).  Output arrays are host arrays of length n_max_cap + 1 (entry 0 of
 * p and alpha is unused: -1 and 1); n_max and n_min are returned.  The same
 * formulas drive sp2_density. */
int sp2_schedule(double lmin, double lmax, double homo_ub, double lumo_lb, int accel, double gamma, double tau_fixed,
                 int n_max_cap, int32_t *n_max, int32_t *n_min, int32_t *p, double *alpha, double *l, double *q,
                 double *xi, double *tau);

/* Step 3 homo/lumo estimates from e_i = ||X~_i - X~_i^2||_F and tr X~_i,
 * i = 0..n, of a finished run with polynomials p_i and alpha_i.  bounds_mode
 * = 1: the run used homo/lumo bounds and l, q are its schedule arrays;
 * bounds_mode = 0: trace-correcting run (l, q unused).  N = matrix size.
 * Writes NaN when no iteration qualifies.  Host arrays of length n + 1. */
int sp2_homo_lumo(int bounds_mode, int n, const double *e, const double *trace, const int32_t *p, const double *alpha,
                  const double *l, const double *q, double lmin, double lmax, int64_t N, int64_t n_occ,
                  double *homo_ub, double *lumo_lb);

/* ---- single steps of the hot path (kernel-level entry points) ---------- */

/* One square of Algorithm 2 on an upper-BSR X: S = X^2 on the block pattern
 * of the square (every (I, J), I <= J, with some K such that X_IK and X_KJ
 * are stored), and Xn = a I + b X + c S on that pattern, where the a I term
 * touches only the n real diagonal entries.  sums[0] = ||X - S||_F^2,
 * sums[1] = tr X, sums[2] = tr S, sums[3] = algorithmic flops
 * (2 * 64^3 per block product).  precision: SP2_PREC_* (FP32 and BF16X3 round X
 * to FP32 first and return Xn rounded to FP32 values). */
int sp2_square_step(sp2_ctx *ctx, const sp2_bsr *X, double a, double b, double c, int precision,
                    sp2_bsr **Xn_out, double sums[4]);

/* Pair product of upper-BSR operands:
 *   out = a I + b G + c (X Y + sign * Y X),  sign = +1 or -1,
 * on the block pattern of X Y + Y X (upper blocks; the a I term touches only
 * the n real diagonal entries).  sign = +1 is the anticommutator, the
 * derivative of the square X^2 along Y that the adjoint recursion of
 * Algorithm 2 applies (symmetric result); sign = -1 is the commutator
 * (antisymmetric result for symmetric X and Y, or symmetric for an
 * antisymmetric Y), as used by the subspace correction.  X is symmetric; Y is
 * symmetric, or antisymmetric when y_antisym = 1 (a block below the diagonal
 * is minus the transpose of its stored mirror, diagonal blocks are stored in
 * full); G (symmetric, may be NULL) enters only at the output blocks it
 * stores.  An antisymmetric result is returned as its upper blocks in the
 * same format.  precision as in sp2_square_step.  sums[0] = ||out||_F^2 of the
 * whole matrix, sums[1] = algorithmic flops (2 * 64^3 per block product). */
int sp2_pair_product(sp2_ctx *ctx, const sp2_bsr *X, const sp2_bsr *Y, const sp2_bsr *G, int sign, int y_antisym,
                     double a, double b, double c, int precision, sp2_bsr **out, double sums[2]);

/* ---- general (full-pattern) storage ------------------------------------
 * The format of the paper's general matrix wrapper (section "Implementation
 * details"), which section "Numerical experiments" compares with the
 * symmetric one: every present block of both triangles is stored as it is.
 * Same sp2_bsr struct; within a block row the columns are strictly
 * increasing, 0 <= col < nbr (any triangle).  No symmetry is assumed. */

/* General storage of the symmetric matrix held by the upper-BSR U: the
 * stored blocks and, below the diagonal, the transposes of their mirrors.
 * *G is owned by the caller (sp2_bsr_free). */
int sp2_general_from_upper(sp2_ctx *ctx, const sp2_bsr *U, sp2_bsr **G);

/* General product out = a I + b G + c A B of matrices in general storage, on
 * the block pattern of A B (every (I, J) with some K such that A_IK and B_KJ
 * are stored) joined with the pattern of G and, when a != 0, the diagonal
 * blocks; the a I term touches only the n real diagonal entries.  G may be
 * NULL (then b is ignored).  The result is in general storage, owned by the
 * caller.  sums (may be NULL): sums[0] = ||G - A B||_F^2 (G = 0 when NULL),
 * sums[1] = tr G, sums[2] = tr(A B), sums[3] = algorithmic flops (2 * 64^3
 * per block product).  With A = B = G = X (symmetric X in general storage)
 * this is the square of Algorithm 2 done on both triangles: about twice the
 * block products and the stored blocks of sp2_square_step.  precision:
 * SP2_PREC_FP64, or SP2_PREC_BF16X3 (operands rounded to FP32, then split,
 * FP32 accumulation; the result holds FP32 values); any other value is
 * SP2_ERR_INVALID_ARG. */
int sp2_general_product(sp2_ctx *ctx, const sp2_bsr *A, const sp2_bsr *B, const sp2_bsr *G, double a, double b,
                        double c, int precision, sp2_bsr **out, double sums[4]);

/* Truncation X~ = X + E with ||E|| <= tau in the chosen norm (section "Error
 * control"); diagonal blocks are never removed.  err[0] = ||E||_F,
 * err[1] = ||E||_M with submatrices of coarse_bs rows. */
int sp2_truncate(sp2_ctx *ctx, const sp2_bsr *X, double tau, int norm, int64_t coarse_bs,
                 sp2_bsr **Xt_out, double err[2]);

/* Norms of the symmetric matrix A held by its upper blocks (section "Upper
 * bounds for the spectral norm"): *frob = ||A||_F of the full matrix and
 * *frobinf = ||A||_M, the Frob-Inf mixed norm: the largest row sum of the
 * matrix of Frobenius norms of the coarse_bs x coarse_bs submatrices of the
 * full matrix (the last ones smaller when coarse_bs does not divide n), an
 * upper bound of the spectral norm.  coarse_bs is a positive multiple of 64
 * with at most 16384 submatrices per row (checked only when frobinf is
 * requested); either output pointer may be NULL.  Both are accumulated in
 * FP64 in a fixed order (bitwise reproducible). */
int sp2_matrix_norms(sp2_ctx *ctx, const sp2_bsr *A, int64_t coarse_bs, double *frob, double *frobinf);

/* sp2_matrix_norms without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results (bit for bit) as
 * sp2_matrix_norms; its block norms, row indices, flags and partial sums live
 * in a fixed device scratch array of 64 MiB that every device the library
 * runs on holds until the process ends.  A matrix needing more scratch than
 * that (about 5.5 million stored blocks) is rejected with
 * SP2_ERR_INVALID_ARG before any device work.  Every call on a device shares
 * that device's array: calls that overlap on one device (other host threads,
 * other contexts) race and must be serialised by the caller. */
int sp2_matrix_norms_noalloc(sp2_ctx *ctx, const sp2_bsr *A, int64_t coarse_bs, double *frob, double *frobinf);

/* Copy a library matrix into caller buffers (device pointers of sizes
 * nbr + 1, nnzb, nnzb * 64 * 64). */
int sp2_bsr_copy(sp2_ctx *ctx, const sp2_bsr *src, int64_t *row_ptr, int32_t *col_idx, double *val);

void sp2_bsr_free(sp2_ctx *ctx, sp2_bsr *m);
void sp2_tape_free(sp2_ctx *ctx, sp2_tape *tape);

#ifdef __cplusplus
}
#endif

#endif /* SP2DM_H */
