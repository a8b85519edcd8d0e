/*
 * qcqp.h -- C ABI of the MI355X (gfx950) rAPDB library for convex QCQPs.
 *
 * Paper: "Restarted Accelerated Primal-Dual Algorithms with Adaptive Stepsizes for Nonlinear
 * Conic Constrained Convex Optimization" (arXiv 2605.29291).
 *
 * Problem (eq. (QCQP), §2.1), K = R^m_+ :
 *     min_{x in X} 1/2 x'Q_0 x + q_0'x + c_0
 *     s.t.         g_i(x) = 1/2 x'Q_i x + q_i'x + c_i <= 0   (i = 1..m),   A x = b,
 * with X = {lb <= x <= ub} a box (compact, Assumption on the sets in §2) and every Q_i
 * symmetric positive semidefinite.  The paper writes the constants c_i as r_i.
 * Multipliers y = (v, lambda), v in R^p for Ax = b, lambda in R^m_+ (§2, coupling function
 * Phi(x,y) = f(x) + <v, Ax-b> + <lambda, g(x)>, eq. (qcqp-coupling)).
 *
 * Conventions for every call:
 *   - every function returns qcqp_status and never throws across the boundary; on failure
 *     qcqp_last_error() returns a thread-local message describing it;
 *   - "host or device" pointers: a handle created with problem.on_device = 1 takes and
 *     returns device pointers (e.g. torch tensors) in every call; otherwise host pointers;
 *   - all device work is ordered on options.stream (a hipStream_t; NULL = default stream);
 *     calls that return results synchronise that stream before returning;
 *   - one handle must not be used from two host threads at once; a handle admitted to a
 *     batch belongs to the batch until it is fetched.
 * Everything is computed on the GPU by hand-written HIP kernels; there is no CPU fallback.
 */
#ifndef QCQP_H
#define QCQP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QCQP_OK = 0,
    QCQP_E_INVALID = 1,        /* invalid sizes / options / non-finite data; nothing allocated */
    QCQP_E_NOMEM = 2,          /* device allocation failed */
    QCQP_E_DEVICE = 3,         /* a HIP runtime error; message in qcqp_last_error() */
    QCQP_E_NOT_CONVERGED = 4,  /* solve stopped at max_iter; outputs are still written */
    QCQP_E_NUMERICAL = 5,      /* NaN/Inf met, or the backtracking step underflowed */
    QCQP_E_NO_ROOM = 6         /* batch admission refused: no free slot or HBM budget */
} qcqp_status;

typedef enum { QCQP_F64 = 0, QCQP_F32 = 1, QCQP_BF16 = 2, QCQP_F16 = 3 } qcqp_dtype;
typedef enum { QCQP_YX = 0, QCQP_XY = 1 } qcqp_variant;
typedef enum { QCQP_RESTART_NONE = 0, QCQP_RESTART_FIXED = 1, QCQP_RESTART_ADAPTIVE = 2 } qcqp_restart;
/* How a trial point's Q-stack products are formed.
 *   DIRECT:      U+ = [Q_i x+] streamed in full, the accumulation precision of the storage
 *                (FP64 for FP64 storage, FP32 for 32/16-bit storage).
 *   INCREMENTAL: W = [Q_i d] for the step d = x+ - x^k, U+ = U^k + W in FP64; every restart
 *                and the start re-anchor U with a direct pass accumulated in FP64.
 *   AUTO:        DIRECT for FP64 storage, INCREMENTAL otherwise. */
typedef enum { QCQP_PASS_AUTO = 0, QCQP_PASS_DIRECT = 1, QCQP_PASS_INCREMENTAL = 2 } qcqp_pass_mode;
/* Where lambda ranges:
 *   NONNEG:  R^m_+, K* for the QCQP's constraints g(x) <= 0 (§2.1);
 *   SIMPLEX: the unit simplex, which turns the problem into
 *            min_x max_{lambda in simplex} f(x) + sum_i lambda_i g_i(x) + <v, Ax - b>
 *            (the kernel-learning form (min-max-KML) of §5);
 *   CONES:   R^{m0}_+ x Q^{k_1} x ... x Q^{k_r} for the conic constraint g(x) in -K with the
 *            same (self-dual) product of second-order cones Q^k = {(t, u): ||u|| <= t} placed
 *            at the end of lambda (the cone setting of §2.1; m0 = m - sum k_j).  Convexity of
 *            lambda'g(x) over K* is the caller's: e.g. g_1 convex quadratic and the other
 *            components of a cone affine. */
typedef enum { QCQP_LAMBDA_NONNEG = 0, QCQP_LAMBDA_SIMPLEX = 1, QCQP_LAMBDA_CONES = 2 } qcqp_lambda_set;
/* When a solve stops.
 *   KKT:   the relative KKT residual (built from r(x,v,lambda) of the Theorem in §4.3) <= tol.
 *   PAPER: the criterion of the experiments of §5.1 for a known optimal value f_star,
 *          max{ |f(x) - f*| / (1 + |f*|), (sum_i max(g_i(x), 0) + sum_l |(Ax - b)_l|) / (m + p) }
 *          <= tol (the printed mean violation when p = 0; with lambda on the simplex only the
 *          equalities count). */
typedef enum { QCQP_STOP_KKT = 0, QCQP_STOP_PAPER = 1 } qcqp_stop_rule;

typedef struct qcqp_handle qcqp_handle;
typedef struct qcqp_batch qcqp_batch;

/* Problem data, eq. (QCQP), or the saddle problem min_{x in X} max_{y in Y-hat} Phi(x, y) of
 * eq. (qcqp-coupling) restricted as in problem (R-min-max) of §3.2.  Ownership: qcqp_create
 * copies (and converts) everything into library-owned device memory; the caller may free its
 * buffers as soon as it returns.  A zero-initialised tail (lambda_set .. ball_lambda) gives the
 * plain QCQP. */
typedef struct {
    int64_t n, m, p;           /* n > 0, m >= 0, 0 <= p < n (rank(A) = p is assumed, not checked) */
    const void *Q;             /* the stored matrices (m + has_q0 of them, or as q_stored lists),
                                  each n rows of ldq elements, row-major, element type Q_dtype,
                                  in index order (Q_0 first when has_q0).  Must be finite
                                  and symmetric (the library uses Q_i x = Q_i' x): after
                                  conversion to the storage type, qcqp_create refuses a matrix
                                  with a non-finite entry or max |Q_rc - Q_cr| > 1e-12 max |Q_rc|
                                  (QCQP_E_INVALID). */
    qcqp_dtype Q_dtype;        /* element type of the caller's Q */
    int64_t ldq;               /* leading dimension in elements (>= n; 0 means n) */
    int has_q0;                /* 0: Q_0 = 0 and is neither stored nor streamed */
    const double *q;           /* (m+1) x n: q_0 then q_1..q_m */
    const double *c;           /* m+1: c_0 then c_1..c_m */
    const double *A;           /* p x n row-major, NULL iff p == 0 */
    const double *b;           /* p, NULL iff p == 0 */
    const double *lb, *ub;     /* n each, lb <= ub, lb < +inf, ub > -inf; infinite bounds are
                                  allowed (e.g. x >= 0), finite ones keep X compact as the
                                  paper assumes */
    int on_device;             /* 1: all pointers here and in later calls are device memory */
    qcqp_lambda_set lambda_set;  /* R^m_+ (default) or the unit simplex (needs m >= 1) */
    double q0_shift;           /* rho >= 0: the objective is 1/2 x'(Q_0 + rho I)x + q_0'x + c_0,
                                  so an identity part costs no stored matrix */
    double ball;               /* B > 0: y restricted to ||y|| <= B (eq. (defcalB)); 0: off */
    double ball_v, ball_lambda;  /* > 0: ||v|| <= B_v, ||lambda|| <= B_lambda, the separable
                                  form of the Remark after eq. (defcalB); 0: off.  Not combined
                                  with `ball`; with the simplex only ball_v is allowed.
                                  The experiments of §5 impose no ball. */
    const int *q_stored;       /* NULL, or m+1 flags 0/1: which Q_i are stored in Q; the others
                                  are 0 (affine constraints), stream no bytes and need no
                                  memory.  q_stored[0] must equal has_q0.  Host memory. */
    int64_t n_soc;             /* CONES: number of second-order cones r >= 1 */
    const int64_t *soc_dims;   /* CONES: k_1..k_r >= 1, sum <= m; host memory */
} qcqp_problem;

/* Method parameters (Algorithm 1, the APDB-yx rules of §3.2, Algorithm 2, eq. (ada_restart)).
 * qcqp_options_default fills the §5 settings for rAPDB-yx, non-monotone. */
typedef struct {
    qcqp_variant variant;      /* QCQP_YX: eq. (apdb-yx-y) of §3.2 (dual step first, default);
                                  QCQP_XY: Algorithm 1 (primal step first, momentum on
                                  grad_x Phi, test function of eq. (backtracking)) */
    int c_nm;                  /* 0 monotone, 1 non-monotone step rule (Remark in §3.1) */
    double eta;                /* backtracking factor, in (0,1) (0.7) */
    double tau_bar;            /* initial primal step; <= 0: 1/||Q_0||_2 estimated on the GPU
                                  (or 1/max_i||Q_i||_2 when Q_0 is absent) */
    double gamma0;             /* sigma/tau ratio gamma_0 > 0 (0.1) */
    double mu;                 /* strong-convexity modulus of f, >= 0 (0) */
    double c_alpha, c_beta, delta;  /* yx: c_alpha > 0, delta in [0,1), c_alpha + delta <= 1
                                       (c_beta unused); xy: c_alpha > 0, c_beta > 0, delta >= 0,
                                       c_alpha + c_beta + delta < 1 (§5 uses 0.25, 0.3, 0.4) */
    qcqp_restart restart;
    int64_t restart_every;     /* K-hat for fixed restarts (400) */
    int restart_from_average;  /* 0: restart at the last iterate (as in §5); 1: Algorithm 2's average */
    double xi;                 /* smoothing of G_xi (0.04) */
    double q_restart;          /* contraction q in (0,1) of eq. (ada_restart) (0.5) */
    int64_t ada_first;         /* first G_xi evaluation, global k (50) */
    int64_t ada_every;         /* later checks at global k % ada_every == 0 (500) */
    int64_t max_iter;          /* iteration cap (50000) */
    double tol;                /* tolerance of the stop rule (1e-6) */
    qcqp_dtype storage;        /* HBM storage type of the Q stack (F64) */
    qcqp_pass_mode pass_mode;  /* AUTO */
    int spec_trials;           /* backtracking candidates evaluated per Q pass, 1..4 (2) */
    int64_t poll_every;        /* trial groups launched between host status polls (0 = auto) */
    int timing;                /* 1: time every Q-pass launch with HIP events (qcqp_info) */
    double inner_tol;          /* G_xi inner box-QP tolerance (1e-12) */
    int64_t max_inner;         /* G_xi inner iteration cap (100000) */
    int use_graphs;            /* 1: replay HIP-graph-captured chunks of trial groups (1); the
                                  timing mode always launches eagerly */
    void *stream;              /* hipStream_t of the caller; the library works on its own
                                  stream of default priority, ordered after this one */
    qcqp_stop_rule stop_rule;  /* KKT (default) or PAPER */
    double f_star;             /* the optimal value the PAPER rule compares against */
    int sym_pass;              /* 1: the Q pass streams a second copy of the stack that holds
                                  only the upper-triangle tiles of each Q_i (about half the
                                  bytes): each off-diagonal tile serves both its rows
                                  (Q_IJ w_J) and, transposed, its columns (Q_IJ' w_I), and a
                                  second kernel sums the per-tile results in a fixed order.
                                  Uses only the upper triangle, so Q_i must be symmetric (as
                                  in the problem class).  F64 storage with direct passes
                                  (128 x 128 tiles, FP64 sums), or BF16 / F16 storage with
                                  incremental passes (256 x 256 tiles of the stored values,
                                  FP32 products and tile sums, FP64 sum of the tiles; the
                                  exact FP64 anchors stream the row-major stack; create
                                  refuses a diagonal entry whose half is not exact in the
                                  storage type).  Single-instance solves only (a batch
                                  refuses such a handle).  0: the row-major pass (default). */
} qcqp_options;

typedef struct {
    int64_t iters;             /* accepted iterations k */
    int64_t trials;            /* backtracking test evaluations (sequential-equivalent count) */
    int64_t q_passes;          /* Q-stack passes streamed (trial groups + anchors) */
    int64_t restarts;
    int64_t gap_evals;         /* G_xi evaluations */
    int64_t status;            /* qcqp_status of the run */
    double rel_kkt, rel_dual, rel_pri, rel_comp;  /* at the returned iterate */
    double f;                  /* objective at the returned x */
    double max_violation;      /* max(0, max_i g_i(x), max_l |(Ax-b)_l|) */
    double seconds;            /* wall time of the call */
    double pass_seconds;       /* summed Q-pass kernel time (only with options.timing) */
    double last_gap;           /* last G_xi value (NaN if none) */
    int64_t pass_bytes;        /* algorithmic HBM bytes of one Q pass: (m+has_q0) n^2 sizeof(storage);
                                  with sym_pass the upper triangles,
                                  (m+has_q0) n(n+1)/2 sizeof(storage) */
    int64_t timed_passes;      /* Q passes covered by pass_seconds */
    double stop_value;         /* the stop rule's value at the returned iterate */
} qcqp_info;

/* Fill *o with the defaults listed above.  Never fails. */
void qcqp_options_default(qcqp_options *o);

/* Thread-local description of the last failure on this thread ("" if none). */
const char *qcqp_last_error(void);

/* Create a handle: validate the problem and options (Assumption on the sets in §2:
 * lb <= ub finite; eta in (0,1); the parameter ranges of Algorithm 1 (xy) or of Lemma
 * (APDB-yx convergence) in §3.2 (yx)),
 * allocate device memory, copy the data and convert Q to options.storage once with
 * round-to-nearest-even.  Errors: QCQP_E_INVALID (nothing allocated), QCQP_E_NOMEM,
 * QCQP_E_DEVICE.  *out is set only on success. */
qcqp_status qcqp_create(const qcqp_problem *prob, const qcqp_options *opt, qcqp_handle **out);

/* Run rAPDB (Algorithm 2 around APDB-yx or APDB-xy) from x0 (n; NULL -> Pi_X(0)) and y0
 * (p+m in the order (v, lambda); NULL -> 0; lambda is projected onto R^m_+) until the relative KKT
 * residual is <= tol or max_iter iterations.  Writes x_out (n) and y_out (p+m, may be NULL),
 * and *info when non-NULL.  Returns QCQP_OK, QCQP_E_NOT_CONVERGED (outputs still written),
 * QCQP_E_NUMERICAL or an error code.  The iteration is device-resident: the host only
 * enqueues kernel groups and reads a status word every poll_every groups. */
qcqp_status qcqp_solve(qcqp_handle *h, const double *x0, const double *y0, double *x_out,
                       double *y_out, qcqp_info *info);

/* One evaluation of the coupling's operator at (x, y) (eq. (qcqp-coupling)): Qx = [Q_i x]
 * as (m+1) x n (row 0 = Q_0 x, zero when Q_0 is absent), g = g_1..g_m (m), f = f(x) (1),
 * grad_x = Q_0x + q_0 + sum_i lambda_i (Q_i x + q_i) + A'v (n).  Any output may be NULL.
 * The Q pass accumulates in FP64 whatever the storage type.  Must not overlap a solve on
 * the same handle. */
qcqp_status qcqp_eval_operator(qcqp_handle *h, const double *x, const double *y, double *Qx,
                               double *g, double *f, double *grad_x);

/* The Q pass of one backtracking trial group, exactly as qcqp_solve launches it (the same
 * kernels, grid, tiles, candidate count and accumulation type), on caller-given points: x is
 * the iterate x^k (n) and xc holds nb = options.spec_trials trial points x^{k+1}_b (nb x n,
 * row-major).  out (nb x (m+1) x n, row-major, rows of matrices that are not stored are 0)
 * receives per candidate
 *   - [Q_i x^{k+1}_b] for i = 0..m in the direct mode (FP64 storage), accumulated in FP64;
 *   - W_b = [Q_i (x^{k+1}_b - x^k)] in the incremental mode (the default for 32/16-bit
 *     storage): the step is rounded to FP32, each lane of the kernel sums its share of a row
 *     (at most ceil(n / 8) products) in FP32, and the lanes' partial sums are combined in FP64.
 * This is the product the test function E_k of §3.2 (eq. (apdb-yx-y)) and Algorithm 1 uses
 * through U^{k+1} = U^k + W.  Host or device pointers as for the handle.  Errors:
 * QCQP_E_INVALID (null pointer, nb != spec_trials, handle in a batch), QCQP_E_DEVICE.  Must not
 * overlap a solve on the same handle. */
qcqp_status qcqp_eval_trial_pass(qcqp_handle *h, const double *x, const double *xc, int64_t nb,
                                 double *out);

/* Relative KKT residual at (x, y) (the residual r(x,v,lambda) of the Theorem in §4.3 in
 * relative form): out6 = {rel_kkt, rel_dual, rel_pri, rel_comp, f, max_violation}; out6 is
 * always host memory. */
qcqp_status qcqp_eval_kkt(qcqp_handle *h, const double *x, const double *y, double *out6);

/* Self-centred smoothed duality gap G_xi(z) at z = (x, y) (Definition in §4; evaluation as
 * in the Remark of §4.2, Euclidean case): out4 = {G, Py, Px, inner_iterations}, host memory.
 * The x-part, a strongly convex box QP, is solved on the GPU by accelerated projected
 * gradient to options.inner_tol. */
qcqp_status qcqp_eval_gap(qcqp_handle *h, const double *x, const double *y, double xi,
                          double *out4);

/* Largest n that qcqp_eval_gap_noalloc serves. */
#define QCQP_NOALLOC_MAX_N 1024

/* qcqp_eval_gap for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and the
 * same result, but the G_xi scratch (H = Q(lambda) + 2 xi I as n x n FP64 plus a few
 * vectors, about 8.1 MiB at the limit) lives in a static device array that the library
 * holds on each GPU it runs on until the process ends, instead of memory the handle
 * allocates on its first qcqp_eval_gap.  The call itself allocates nothing.  Arguments,
 * pointer kinds and out4 as for qcqp_eval_gap.  Errors: QCQP_E_INVALID for n >
 * QCQP_NOALLOC_MAX_N, a null pointer, xi <= 0 or a handle in a batch; QCQP_E_DEVICE.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (from two
 * host threads, or on handles whose streams run concurrently) race and must be serialised
 * by the caller. */
qcqp_status qcqp_eval_gap_noalloc(qcqp_handle *h, const double *x, const double *y, double xi,
                                  double *out4);

/* Release all device memory of the handle.  NULL is accepted. */
qcqp_status qcqp_destroy(qcqp_handle *h);

/* ---- serving: continuous batching of independent solves (one GPU) --------------------
 * A batch owns up to max_slots resident solves.  qcqp_batch_step launches, per trial group,
 * ONE pass kernel covering the tiles of every running slot (plus one step, one epilogue and
 * one control kernel, each covering all slots).  Per-slot reductions are deterministic, so a
 * slot's result does not depend on which other slots share the launches.
 * All handles in a batch must share the batch's storage type, spec_trials and device. */

/* hbm_budget_bytes: admission refuses a handle whose resident bytes would push the sum over
 * the budget (0 = no budget); max_slots >= 1. */
qcqp_status qcqp_batch_create(const qcqp_options *opt, size_t hbm_budget_bytes,
                              int64_t max_slots, qcqp_batch **out);

/* Admit a created handle as a new slot, starting from x0/y0 (as in qcqp_solve); *slot gets
 * its id.  QCQP_E_NO_ROOM when no slot or budget is free (the handle stays with the caller). */
qcqp_status qcqp_batch_admit(qcqp_batch *bt, qcqp_handle *h, const double *x0,
                             const double *y0, int64_t *slot);

/* Launch `groups` trial groups for all running slots, then poll.  Returns after the stream
 * has drained the groups. */
qcqp_status qcqp_batch_step(qcqp_batch *bt, int64_t groups);

/* Ids of slots that finished (converged, hit max_iter or failed) and were not yet fetched;
 * writes at most cap ids into done_slots (host memory) and their number into *n_done. */
qcqp_status qcqp_batch_poll(qcqp_batch *bt, int64_t *done_slots, int64_t cap, int64_t *n_done);

/* Copy a finished slot's x (n), y (p+m) and info out, release the slot and return its handle
 * to the caller (*h_out may be NULL).  QCQP_E_INVALID if the slot is not finished. */
qcqp_status qcqp_batch_fetch(qcqp_batch *bt, int64_t slot, double *x_out, double *y_out,
                             qcqp_info *info, qcqp_handle **h_out);

/* Number of running slots and resident bytes. */
qcqp_status qcqp_batch_stats(qcqp_batch *bt, int64_t *running, size_t *resident_bytes);

/* Pass accounting of the batch since creation: summed pass-kernel seconds (only with
 * options.timing), algorithmic bytes streamed ((m + has_q0) n^2 sizeof(storage) per slot pass,
 * counted from the device pass counters) and the number of slot passes.  Any pointer may be
 * NULL. */
qcqp_status qcqp_batch_pass_stats(qcqp_batch *bt, double *pass_seconds, double *pass_bytes,
                                  int64_t *passes);

/* Destroy the batch; handles still admitted are destroyed with it. */
qcqp_status qcqp_batch_destroy(qcqp_batch *bt);

/* Device bytes a handle for this problem/options would hold (for admission control). */
size_t qcqp_handle_bytes(const qcqp_handle *h);

/* Time `reps` launches of the Q-pass kernel exactly as the solve launches it (direct
 * trial mode, options.spec_trials candidates) between HIP events on the handle's stream;
 * *avg_seconds gets the mean duration.  For measurement only. */
qcqp_status qcqp_time_pass(qcqp_handle *h, int64_t reps, double *avg_seconds);

#ifdef __cplusplus
}
#endif
#endif /* QCQP_H */
