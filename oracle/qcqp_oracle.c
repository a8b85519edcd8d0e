/*
 * Plain FP64 CPU oracle for rAPDB on convex QCQPs.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct reference that the GPU
 * path is checked against.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline leg may load it; the product library never links, loads or calls it, and shares no
 * code, header, table or helper with it.
 *
 * Paper: "Restarted Accelerated Primal-Dual Algorithms with Adaptive Stepsizes for Nonlinear
 * Conic Constrained Convex Optimization" (arXiv 2605.29291).
 *
 * What is computed, and where the paper defines it:
 *   - the QCQP data and the coupling Phi(x,y) = f(x) + <v, Ax-b> + <lambda, g(x)>:
 *     eq. (QCQP) and eq. (qcqp-coupling), §2.1; K = R^m_+ so K* = R^m_+ (§2.1);
 *   - Euclidean Bregman distances D = 1/2||.||^2 (Remark at the end of §2.2), which turn
 *     every argmin step into a projection;
 *   - APDB-xy: Algorithm 1 with the test function E_k of eq. (backtracking), §3.1;
 *   - APDB-yx: the replacement update rules eq. (apdb-yx-y) and its E_k, §3.2
 *     (the set B is not imposed, as in §5);
 *   - the non-monotone step rule c_nm = 1 (Remark in §3.1, eq. (nonmonotone-tau));
 *   - rAPDB with fixed-frequency restarts: Algorithm 2, §4.1;
 *   - rAPDB-ada: restart test eq. (ada_restart) on the self-centred smoothed duality gap
 *     (Definition "Smoothed duality gap", §4), evaluated as in the Remark of §4.2;
 *   - the KKT residual r(x,v,lambda) of Theorem (metric subregularity sufficient condition),
 *     §4.3, used in relative form for termination;
 *   - the restricted dual domain Y-hat = Y ∩ B of problem (R-min-max), §3.2: the ball of
 *     eq. (defcalB) or the separable balls of the Remark after it (off unless requested, as in
 *     the experiments of §5);
 *   - conic constraints g(x) in -K with K = R^{m0}_+ x Q^{k_1} x ... x Q^{k_r}, second-order
 *     cones (the cone setting of §2.1; K* = K); the closed-form value r* of the Remark after
 *     Lemma "dual bound" shows the same cone;
 *   - constraints without a stored matrix (Q_i = 0, affine g_i), listed by a 0/1 map;
 *   - a min-max problem whose lambda ranges over the unit simplex and whose objective carries
 *     rho ||x||^2 / 2 (the kernel-learning form (min-max-KML) of §5, rho = 2 lambda_KML), with
 *     its equality constraint b'x = 0 entering Phi through the multiplier v.
 *
 * Everything is naive loops in double precision: no blocking, no reordering beyond what the
 * definitions state.  Q may be supplied as float64, float32, bfloat16 or float16; each element
 * is upcast exactly to double when read, so a rounded instance is solved exactly as stored.
 *
 * Readings of points the paper leaves open (each is a choice, listed again in the design notes):
 *   (R1) x^0 = Pi_X(0), y^0 = 0 unless given; tau_bar and gamma_0 are inputs.
 *   (R2) alpha_0 = c_alpha / sigma_{-1} (yx) or c_alpha / tau_{-1} (xy), beta_0 = gamma_0 c_beta /
 *        sigma_{-1}, using tau_{-1}, sigma_{-1} of Algorithm 1's first line.
 *   (R3) a restart re-enters the routine, resetting tau, gamma, momentum and the averages.
 *   (R4) the restart point is the last iterate (as in §5) unless restart_from_average is set
 *        (Algorithm 2 as printed).
 *   (R5) adaptive schedule: G_ref = G_xi(z^k) at global k = ada_first (no restart); then at
 *        every global k > ada_first with k % ada_every == 0 the candidate (last iterate) is
 *        tested against q * G_ref; on success restart there and G_ref <- G_xi(candidate).
 *   (R6) G_xi's x-part (a strongly convex box QP) is solved by accelerated projected gradient
 *        with gradient restart, step 1/L with L a Gershgorin bound; tolerance inner_tol.
 *   (R7) termination: relative KKT residual (see orc_kkt) <= tol, checked at every iterate
 *        before an iteration is taken; or k >= max_iter.
 *   (R8) the projection onto Y-hat is the projection onto the cone R^p x R^m_+ scaled back onto
 *        the ball (exact for a cone and a ball centred at 0); with a simplex, only a ball on v.
 *   (R9) with lambda on the simplex, the lambda-part of the KKT residual is the natural residual
 *        || lambda - Pi_simplex(lambda + g(x)) || and g is no constraint (rel_pri covers Ax - b).
 *  (R11) with cones, the lambda-part of the KKT residual is || lambda - Pi_K*(lambda + g(x)) ||
 *        and the infeasibility is dist(g(x), -K) = || Pi_K*(g(x)) || (Moreau's decomposition);
 *        both reduce to (R7)'s formulas for R^m_+.  The criterion of (R10) counts one violation
 *        per scalar constraint of R^{m0}_+ and one, dist(g_c, -Q), per cone.
 *  (R10) the experiments' criterion of §5.1, for a known optimal value f*:
 *        max{ |f(x) - f*| / (1 + |f*|), (sum_i max(g_i(x), 0) + sum_l |(Ax - b)_l|) / (m + p) },
 *        which is the printed mean violation when p = 0 (with lambda on a simplex only the
 *        equalities count as constraints).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------------------------ */
/* data                                                                                        */

typedef struct {
    int64_t n, m, p;
    const void *Q;      /* (m + has_q0) matrices of n x n, row-major, element type q_dtype */
    int32_t q_dtype;    /* 0 float64, 1 float32, 2 bfloat16 (raw uint16), 3 float16 (raw uint16) */
    int32_t has_q0;     /* 0: Q_0 = 0 and Q holds Q_1..Q_m only */
    const double *q;    /* (m+1) x n */
    const double *c;    /* m+1: c[0] = r_0, c[i] = r_i */
    const double *A;    /* p x n or NULL */
    const double *b;    /* p or NULL */
    const double *lb, *ub;   /* lb <= ub; infinite entries allowed (e.g. x >= 0) */
    /* the dual domain Y-hat = Y ∩ B and the objective's identity part (all zero = plain QCQP) */
    int32_t lambda_set;      /* 0: lambda in R^m_+ (K* of the QCQP, §2.1); 1: unit simplex */
    int32_t pad0;
    double q0_shift;         /* rho >= 0: the objective's Hessian is Q_0 + rho I */
    double ball;             /* B > 0: ||y|| <= B, the set of eq. (defcalB); 0: none */
    double ball_v, ball_l;   /* > 0: ||v|| <= B_v, ||lambda|| <= B_lambda (the separable form of
                                the Remark after eq. (defcalB)); 0: none */
    const int32_t *q_stored; /* m+1 flags, 1 where Q_i is stored (Q holds those matrices in index
                                order; the others are 0, e.g. affine constraints); NULL: Q_1..Q_m
                                stored and Q_0 as has_q0 says */
    int64_t n_soc;           /* lambda_set 2: lambda in R^{m0}_+ x Q^{k_1} x ... x Q^{k_r}, the
                                second-order cones at the end of lambda (K* for g(x) in -K with K
                                the same product, which is self-dual) */
    const int64_t *soc_dims; /* k_1..k_r, each >= 1, sum <= m */
} orc_problem;

typedef struct {
    int32_t variant;              /* 0 = APDB-yx, 1 = APDB-xy */
    int32_t c_nm;                 /* 0 monotone, 1 non-monotone */
    int32_t restart;              /* 0 none, 1 fixed frequency, 2 adaptive */
    int32_t restart_from_average; /* 0 last iterate (R4) */
    int64_t restart_every;        /* K-hat */
    int64_t ada_first, ada_every;
    int64_t max_iter;
    int64_t max_inner;            /* cap on inner box-QP iterations for G_xi */
    double eta, tau_bar, gamma0, mu;
    double c_alpha, c_beta, delta;
    double xi, q_restart;
    double tol, inner_tol;
    int32_t stop_rule;            /* 0: relative KKT (R7); 1: the criterion of §5.1 (R10) */
    int32_t pad0;
    double f_star;                /* the optimal value that criterion compares against */
} orc_options;

typedef struct {
    int64_t iters, trials, restarts, gap_evals, status;
    double rel_kkt, rel_dual, rel_pri, rel_comp, f, max_violation, last_gap;
    double stop_value;            /* the stop rule's value at the returned point */
} orc_info;

enum { ORC_CONVERGED = 0, ORC_INVALID = 1, ORC_NOT_CONVERGED = 4, ORC_NUMERICAL = 5 };

/* exact upcast of one stored element to double */
static double f16_to_double(uint16_t h)
{
    int sign = (h >> 15) & 1, e = (h >> 10) & 31, mant = h & 1023;
    double v;
    if (e == 0) v = ldexp((double)mant, -24);                 /* subnormal: mant * 2^-24 */
    else if (e == 31) v = mant ? NAN : INFINITY;
    else v = ldexp((double)(mant + 1024), e - 25);            /* (1 + mant/1024) * 2^(e-15) */
    return sign ? -v : v;
}

static double bf16_to_double(uint16_t h)
{
    uint32_t bits = (uint32_t)h << 16;
    float f;
    memcpy(&f, &bits, 4);
    return (double)f;
}

/* position of Q_i (i = 0..m) among the stored matrices, or -1 when Q_i = 0 is not stored */
static int64_t stored_index(const orc_problem *P, int64_t i)
{
    if (P->q_stored) {
        if (!P->q_stored[i]) return -1;
        int64_t s = 0;
        for (int64_t k = 0; k < i; ++k) s += P->q_stored[k] ? 1 : 0;
        return s;
    }
    if (!P->has_q0) return i == 0 ? -1 : i - 1;
    return i;
}

/* element (r, j) of the stored matrix number s (see stored_index) */
static double qel(const orc_problem *P, int64_t s, int64_t r, int64_t j)
{
    int64_t idx = (s * P->n + r) * P->n + j;
    switch (P->q_dtype) {
    case 0: return ((const double *)P->Q)[idx];
    case 1: return (double)((const float *)P->Q)[idx];
    case 2: return bf16_to_double(((const uint16_t *)P->Q)[idx]);
    default: return f16_to_double(((const uint16_t *)P->Q)[idx]);
    }
}

static double dot(const double *a, const double *b, int64_t n)
{
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j) s += a[j] * b[j];
    return s;
}

static double nrm2sq(const double *a, int64_t n) { return dot(a, a, n); }

static double clip(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* ------------------------------------------------------------------------------------------ */
/* operator: U_i = Q_i x, g_i(x) = 1/2 x'Q_i x + q_i'x + r_i, f = g_0, h = Ax - b               */
/* eq. (QCQP) and eq. (qcqp-coupling), §2.1; gradient of g as printed in §2.1.                 */

static void stack_matvec(const orc_problem *P, const double *x, double *U)
{
    const int64_t n = P->n;
    for (int64_t i = 0; i <= P->m; ++i) {
        const int64_t si = stored_index(P, i);
        for (int64_t r = 0; r < n; ++r) {
            double s = 0.0;
            if (si >= 0) {
                for (int64_t j = 0; j < n; ++j) s += qel(P, si, r, j) * x[j];
            }
            if (i == 0) s += P->q0_shift * x[r];      /* (Q_0 + rho I) x */
            U[i * n + r] = s;
        }
    }
}

/* Gy = grad_y Phi(x, .) = (Ax - b, g(x)) in the order y = (v, lambda); fval = f(x) */
static void constraint_values(const orc_problem *P, const double *x, const double *U,
                              double *Gy, double *fval)
{
    const int64_t n = P->n, m = P->m, p = P->p;
    for (int64_t l = 0; l < p; ++l) Gy[l] = dot(P->A + l * n, x, n) - P->b[l];
    for (int64_t i = 0; i <= m; ++i) {
        double gi = 0.5 * dot(x, U + i * n, n) + dot(P->q + i * n, x, n) + P->c[i];
        if (i == 0) *fval = gi;
        else Gy[p + i - 1] = gi;
    }
}

/* grad_x Phi(x, y) = Q_0 x + q_0 + sum_i lambda_i (Q_i x + q_i) + A'v   (eq. (qcqp-coupling)) */
static void grad_x(const orc_problem *P, const double *U, const double *y, double *gx)
{
    const int64_t n = P->n, m = P->m, p = P->p;
    for (int64_t j = 0; j < n; ++j) gx[j] = U[j] + P->q[j];
    for (int64_t i = 1; i <= m; ++i) {
        double lam = y[p + i - 1];
        for (int64_t j = 0; j < n; ++j) gx[j] += lam * (U[i * n + j] + P->q[i * n + j]);
    }
    for (int64_t l = 0; l < p; ++l)
        for (int64_t j = 0; j < n; ++j) gx[j] += y[l] * P->A[l * n + j];
}

/* Euclidean projection of z (k entries) onto the unit simplex {w >= 0, sum w = 1}: sort z in
 * decreasing order u_1 >= ... >= u_k, take the largest j with u_j > (u_1 + ... + u_j - 1)/j,
 * theta = (u_1 + ... + u_j - 1)/j and w = max(z - theta, 0) (the sorting method of Held, Wolfe
 * and Crowder, 1974; also Duchi et al., 2008). */
static int cmp_desc(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return x < y ? 1 : (x > y ? -1 : 0);
}

static void project_simplex(double *z, int64_t k)
{
    if (k <= 0) return;
    double *u = malloc(sizeof(double) * k);
    if (!u) { for (int64_t i = 0; i < k; ++i) z[i] = NAN; return; }
    memcpy(u, z, sizeof(double) * k);
    qsort(u, (size_t)k, sizeof(double), cmp_desc);
    double cum = 0.0, theta = 0.0;
    for (int64_t j = 0; j < k; ++j) {
        cum += u[j];
        double t = (cum - 1.0) / (double)(j + 1);
        if (u[j] > t) theta = t;
    }
    free(u);
    for (int64_t i = 0; i < k; ++i) z[i] = z[i] > theta ? z[i] - theta : 0.0;
}

/* Euclidean projection of z = (t, u) (k entries) onto the second-order cone
 * Q^k = {(t, u): ||u|| <= t}: z itself inside, 0 inside the polar cone (||u|| <= -t), otherwise
 * ((t + ||u||) / 2) (1, u / ||u||) (the closed form for the second-order cone, e.g. Fukushima,
 * Luo and Tseng, 2002).  Q^1 is the half-line t >= 0. */
static void project_soc(double *z, int64_t k)
{
    double t = z[0];
    double un = k > 1 ? sqrt(nrm2sq(z + 1, k - 1)) : 0.0;
    if (un <= t) return;
    if (un <= -t) {
        for (int64_t i = 0; i < k; ++i) z[i] = 0.0;
        return;
    }
    double a = 0.5 * (t + un);
    z[0] = a;
    for (int64_t i = 1; i < k; ++i) z[i] *= a / un;
}

/* lambda (m entries) onto K*: R^m_+, the unit simplex, or R^{m0}_+ x Q^{k_1} x ... x Q^{k_r} */
static void project_kstar(const orc_problem *P, double *lam)
{
    const int64_t m = P->m;
    if (P->lambda_set == 1) {
        project_simplex(lam, m);
        return;
    }
    int64_t m0 = m;
    if (P->lambda_set == 2)
        for (int64_t c = 0; c < P->n_soc; ++c) m0 -= P->soc_dims[c];
    for (int64_t i = 0; i < m0; ++i)
        if (lam[i] < 0.0) lam[i] = 0.0;
    if (P->lambda_set == 2) {
        int64_t off = m0;
        for (int64_t c = 0; c < P->n_soc; ++c) {
            project_soc(lam + off, P->soc_dims[c]);
            off += P->soc_dims[c];
        }
    }
}

/* scale w (k entries) back onto the ball of radius r when it lies outside */
static void scale_to_ball(double *w, int64_t k, double r)
{
    double s = sqrt(nrm2sq(w, k));
    if (s > r) {
        double f = r / s;
        for (int64_t i = 0; i < k; ++i) w[i] *= f;
    }
}

/* Euclidean projection onto the dual domain Y-hat = Y ∩ B, y = (v, lambda):
 *   Y = R^p x K*, with K* = R^m_+ for the QCQP (§2.1), a product of R^{m0}_+ and second-order
 *   cones for a conic constraint g(x) in -K (the cone setting of §2.1), or R^p x (unit simplex)
 *   for a min-max problem whose lambda ranges over a simplex;
 *   B = {||y|| <= B} (eq. (defcalB)) or {||v|| <= B_v} x {||lambda|| <= B_lambda} (the Remark
 *   after it), or the whole space.
 * R^p x K* (not the simplex) is a closed convex cone, and the projection onto the intersection
 * of such a cone
 * with a ball centred at 0 is the cone projection scaled back onto the ball; the separable ball
 * treats v and lambda the same way one block at a time. */
static void project_y(const orc_problem *P, double *y)
{
    const int64_t p = P->p, m = P->m;
    double *lam = y + p;
    project_kstar(P, lam);
    if (P->ball > 0.0) scale_to_ball(y, p + m, P->ball);
    if (P->ball_v > 0.0) scale_to_ball(y, p, P->ball_v);
    if (P->ball_l > 0.0) scale_to_ball(lam, m, P->ball_l);
}

/* ------------------------------------------------------------------------------------------ */
/* relative KKT residual (R7).  Built from r(x,v,lambda) of the Theorem in §4.3:
 *   r_x = || x - Pi_X(x - grad_x Phi) ||      (natural residual of dist(0, grad + N_X(x)))
 *   r_l = || min(lambda, -g(x)) ||            (feasibility and complementarity for K = R^m_+)
 *   r_v = || Ax - b ||
 * rel_dual = r_x / (1 + ||Q_0x+q_0|| + ||sum lambda_i (Q_i x + q_i)|| + ||A'v||)
 * rel_comp = r_l / (1 + ||c_{1..m}||)
 * rel_pri  = || ([g]_+, Ax-b) || / (1 + ||c_{1..m}|| + ||b||)
 * When lambda ranges over the unit simplex, g is not a constraint: r_l is the natural residual
 * || lambda - Pi_simplex(lambda + g(x)) || of the inner maximisation (for R^m_+ the same formula
 * gives min(lambda, -g)), and rel_pri and max_violation cover Ax - b only.
 * The Q_0 and q_0 terms include the identity part rho x.
 * out = {rel_kkt, rel_dual, rel_pri, rel_comp, f, max_violation}                              */
static void kkt_eval(const orc_problem *P, const double *x, const double *y, const double *U,
                     const double *Gy, double fval, double *out)
{
    const int64_t n = P->n, m = P->m, p = P->p;
    double rx = 0, s0 = 0, s1 = 0, s2 = 0;
    for (int64_t j = 0; j < n; ++j) {
        double a0 = U[j] + P->q[j];
        double a1 = 0.0, a2 = 0.0;
        for (int64_t i = 1; i <= m; ++i) a1 += y[p + i - 1] * (U[i * n + j] + P->q[i * n + j]);
        for (int64_t l = 0; l < p; ++l) a2 += y[l] * P->A[l * n + j];
        double gj = a0 + a1 + a2;
        double r = x[j] - clip(x[j] - gj, P->lb[j], P->ub[j]);
        rx += r * r;
        s0 += a0 * a0;
        s1 += a1 * a1;
        s2 += a2 * a2;
    }
    double rl = 0, pri = 0, cn = 0, bn = 0, maxv = 0;
    if (P->lambda_set == 2) {
        /* cones: r_l = ||lambda - Pi_K*(lambda + g)||, infeasibility dist(g, -K) = ||Pi_K*(g)||
         * (Moreau), per block for the maximum */
        double *w = malloc(sizeof(double) * (m > 0 ? m : 1));
        double *gv = malloc(sizeof(double) * (m > 0 ? m : 1));
        if (!w || !gv) { free(w); free(gv); for (int k = 0; k < 6; ++k) out[k] = NAN; return; }
        for (int64_t i = 0; i < m; ++i) {
            w[i] = y[p + i] + Gy[p + i];
            gv[i] = Gy[p + i];
            cn += P->c[i + 1] * P->c[i + 1];
        }
        project_kstar(P, w);
        project_kstar(P, gv);
        int64_t m0 = m;
        for (int64_t c = 0; c < P->n_soc; ++c) m0 -= P->soc_dims[c];
        for (int64_t i = 0; i < m; ++i) {
            double d = y[p + i] - w[i];
            rl += d * d;
            pri += gv[i] * gv[i];
            if (i < m0 && gv[i] > maxv) maxv = gv[i];
        }
        int64_t off = m0;
        for (int64_t c = 0; c < P->n_soc; ++c) {
            double b = sqrt(nrm2sq(gv + off, P->soc_dims[c]));
            if (b > maxv) maxv = b;
            off += P->soc_dims[c];
        }
        free(w); free(gv);
    } else if (P->lambda_set == 1) {
        double *w = malloc(sizeof(double) * (m > 0 ? m : 1));
        if (!w) { for (int k = 0; k < 6; ++k) out[k] = NAN; return; }
        for (int64_t i = 0; i < m; ++i) w[i] = y[p + i] + Gy[p + i];
        project_simplex(w, m);
        for (int64_t i = 0; i < m; ++i) {
            double d = y[p + i] - w[i];
            rl += d * d;
            cn += P->c[i + 1] * P->c[i + 1];
        }
        free(w);
    } else {
        for (int64_t i = 0; i < m; ++i) {
            double g = Gy[p + i], lam = y[p + i];
            double mn = lam < -g ? lam : -g;
            rl += mn * mn;
            if (g > 0) { pri += g * g; if (g > maxv) maxv = g; }
            cn += P->c[i + 1] * P->c[i + 1];
        }
    }
    for (int64_t l = 0; l < p; ++l) {
        pri += Gy[l] * Gy[l];
        if (fabs(Gy[l]) > maxv) maxv = fabs(Gy[l]);
        bn += P->b[l] * P->b[l];
    }
    double rel_dual = sqrt(rx) / (1.0 + sqrt(s0) + sqrt(s1) + sqrt(s2));
    double rel_comp = sqrt(rl) / (1.0 + sqrt(cn));
    double rel_pri = sqrt(pri) / (1.0 + sqrt(cn) + sqrt(bn));
    double r = rel_dual;
    if (rel_pri > r) r = rel_pri;
    if (rel_comp > r) r = rel_comp;
    if (isnan(rel_dual) || isnan(rel_pri) || isnan(rel_comp)) r = NAN;
    out[0] = r; out[1] = rel_dual; out[2] = rel_pri; out[3] = rel_comp;
    out[4] = fval; out[5] = maxv;
}

/* (R10) the termination criterion of the experiments of §5.1 for a known optimal value f_star:
 * the larger of the relative suboptimality and the mean constraint violation */
static double paper_criterion(const orc_problem *P, const double *Gy, double fval, double f_star)
{
    const int64_t m = P->m, p = P->p;
    double viol = 0.0;
    int64_t cnt = p;
    for (int64_t l = 0; l < p; ++l) viol += fabs(Gy[l]);
    if (P->lambda_set == 0) {
        for (int64_t i = 0; i < m; ++i)
            if (Gy[p + i] > 0.0) viol += Gy[p + i];
        cnt += m;
    } else if (P->lambda_set == 2) {
        /* one violation per scalar constraint of R^{m0}_+ and one per cone, dist(g_c, -Q) */
        double *gv = malloc(sizeof(double) * (m > 0 ? m : 1));
        if (!gv) return NAN;
        memcpy(gv, Gy + p, sizeof(double) * m);
        project_kstar(P, gv);
        int64_t m0 = m;
        for (int64_t c = 0; c < P->n_soc; ++c) m0 -= P->soc_dims[c];
        for (int64_t i = 0; i < m0; ++i) viol += gv[i];
        int64_t off = m0;
        for (int64_t c = 0; c < P->n_soc; ++c) {
            viol += sqrt(nrm2sq(gv + off, P->soc_dims[c]));
            off += P->soc_dims[c];
        }
        cnt += m0 + P->n_soc;
        free(gv);
    }
    double sub = fabs(fval - f_star) / (1.0 + fabs(f_star));
    double mv = cnt > 0 ? viol / (double)cnt : 0.0;
    return sub > mv ? sub : mv;
}

/* ------------------------------------------------------------------------------------------ */
/* self-centred smoothed duality gap G_xi(z) (Definition in §4, Euclidean case, Remark in §4.2)
 *   G_xi(z) = sup_{y' in Y} { Phi(x,y') - xi||y'-y||^2 } - inf_{x' in X} { Phi(x',y) + xi||x'-x||^2 }
 *           = Py + Px, with
 *   Py = <grad_y Phi(x), y'-y> - xi||y'-y||^2,  y' = Pi_Y(y + grad_y Phi(x) / (2 xi))
 *   Px = -min_{x+D in X} { grad_x Phi(x,y)'D + 1/2 D'Q(lambda)D + xi||D||^2 },
 *        Q(lambda) = Q_0 + sum_i lambda_i Q_i.
 * The x-part is a strongly convex box QP (R6).  out = {G, Py, Px, inner_iters}.               */
static int gap_eval(const orc_problem *P, const double *x, const double *y, double xi,
                    double inner_tol, int64_t max_inner, double *out)
{
    const int64_t n = P->n, m = P->m, p = P->p;
    double *U = malloc(sizeof(double) * (m + 1) * n);
    double *Gy = malloc(sizeof(double) * (p + m + 1));
    double *gx = malloc(sizeof(double) * n);
    double *H = malloc(sizeof(double) * n * n);
    double *D = calloc(n, sizeof(double));
    double *Dn = malloc(sizeof(double) * n);
    double *Z = calloc(n, sizeof(double));
    double *gz = malloc(sizeof(double) * n);
    if (!U || !Gy || !gx || !H || !D || !Dn || !Z || !gz) {
        free(U); free(Gy); free(gx); free(H); free(D); free(Dn); free(Z); free(gz);
        return -1;
    }
    double fval;
    stack_matvec(P, x, U);
    constraint_values(P, x, U, Gy, &fval);
    grad_x(P, U, y, gx);

    /* y-part, closed form: the maximiser is y' = Pi_{Y-hat}(y + grad_y Phi / (2 xi)) */
    double Py = 0.0;
    {
        double *yp = malloc(sizeof(double) * (p + m + 1));
        if (!yp) { free(U); free(Gy); free(gx); free(H); free(D); free(Dn); free(Z); free(gz); return -1; }
        for (int64_t l = 0; l < p + m; ++l) yp[l] = y[l] + Gy[l] / (2.0 * xi);
        project_y(P, yp);
        for (int64_t l = 0; l < p + m; ++l) {
            double dl = yp[l] - y[l];
            Py += Gy[l] * dl - xi * dl * dl;
        }
        free(yp);
    }

    /* x-part: H = Q(lambda) + 2 xi I, with Q(lambda) = Q_0 + rho I + sum lambda_i Q_i */
    int64_t *sidx = malloc(sizeof(int64_t) * (m + 1));
    if (!sidx) { free(U); free(Gy); free(gx); free(H); free(D); free(Dn); free(Z); free(gz); return -1; }
    for (int64_t i = 0; i <= m; ++i) sidx[i] = stored_index(P, i);
    for (int64_t r = 0; r < n; ++r)
        for (int64_t j = 0; j < n; ++j) {
            double h = sidx[0] >= 0 ? qel(P, sidx[0], r, j) : 0.0;
            for (int64_t i = 1; i <= m; ++i)
                if (sidx[i] >= 0) h += y[p + i - 1] * qel(P, sidx[i], r, j);
            H[r * n + j] = h + (r == j ? 2.0 * xi + P->q0_shift : 0.0);
        }
    free(sidx);
    double L = 0.0;   /* Gershgorin bound on lambda_max(H) */
    for (int64_t r = 0; r < n; ++r) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) s += fabs(H[r * n + j]);
        if (s > L) L = s;
    }
    double gnorm = sqrt(nrm2sq(gx, n));
    double t = 1.0;
    int64_t it = 0;
    for (it = 0; it < max_inner; ++it) {
        /* gradient of h at Z */
        for (int64_t r = 0; r < n; ++r) gz[r] = gx[r] + dot(H + r * n, Z, n);
        double res = 0.0, dir = 0.0;
        for (int64_t r = 0; r < n; ++r) {
            Dn[r] = clip(Z[r] - gz[r] / L, P->lb[r] - x[r], P->ub[r] - x[r]);
            double a = Dn[r] - Z[r];
            res += a * a;
            dir += (Z[r] - Dn[r]) * (Dn[r] - D[r]);
        }
        double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
        if (dir > 0.0) {            /* gradient restart */
            tn = 1.0;
            for (int64_t r = 0; r < n; ++r) Z[r] = Dn[r];
        } else {
            double beta = (t - 1.0) / tn;
            for (int64_t r = 0; r < n; ++r) Z[r] = Dn[r] + beta * (Dn[r] - D[r]);
        }
        for (int64_t r = 0; r < n; ++r) D[r] = Dn[r];
        t = tn;
        if (L * sqrt(res) <= inner_tol * (1.0 + gnorm)) { ++it; break; }
    }
    /* h(D) at the final D */
    double hv = 0.0;
    for (int64_t r = 0; r < n; ++r) hv += gx[r] * D[r] + 0.5 * D[r] * dot(H + r * n, D, n);
    double Px = -hv;
    out[0] = Py + Px; out[1] = Py; out[2] = Px; out[3] = (double)it;
    free(U); free(Gy); free(gx); free(H); free(D); free(Dn); free(Z); free(gz);
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* exported: single evaluation of the operator at (x, y)                                       */

int orc_operator(const orc_problem *P, const double *x, const double *y, double *U, double *Gy,
                 double *fval, double *gx)
{
    stack_matvec(P, x, U);
    constraint_values(P, x, U, Gy, fval);
    if (gx) grad_x(P, U, y, gx);
    return 0;
}

/* projection of y (p + m entries) onto the dual domain Y-hat, in place (test access) */
int orc_project_dual(const orc_problem *P, double *y)
{
    project_y(P, y);
    return 0;
}

/* grad_x Phi from a given U (used by tests that form U independently) */
int orc_grad_from_u(const orc_problem *P, const double *U, const double *y, double *gx)
{
    grad_x(P, U, y, gx);
    return 0;
}

int orc_kkt(const orc_problem *P, const double *x, const double *y, double *out6)
{
    const int64_t n = P->n, m = P->m, p = P->p;
    double *U = malloc(sizeof(double) * (m + 1) * n);
    double *Gy = malloc(sizeof(double) * (p + m + 1));
    if (!U || !Gy) { free(U); free(Gy); return -1; }
    double fval;
    stack_matvec(P, x, U);
    constraint_values(P, x, U, Gy, &fval);
    kkt_eval(P, x, y, U, Gy, fval, out6);
    free(U); free(Gy);
    return 0;
}

int orc_gap(const orc_problem *P, const double *x, const double *y, double xi, double inner_tol,
            int64_t max_inner, double *out4)
{
    return gap_eval(P, x, y, xi, inner_tol, max_inner, out4);
}

/* ------------------------------------------------------------------------------------------ */
/* rAPDB (Algorithm 2) around APDB-yx (§3.2) or APDB-xy (Algorithm 1).                           */

typedef struct {
    const orc_problem *P;
    const orc_options *o;
    int64_t n, m, p, ny;
    /* current iterate and cached operator values */
    double *x, *y, *U, *Gy, f;
    double *gxk, *gxp;            /* xy: grad_x Phi(x^k,y^k), grad_x Phi(x^{k-1},y^{k-1}) */
    double *Gyp;                  /* yx: grad_y Phi(x^{k-1}) */
    /* trial point */
    double *xt, *yt, *Ut, *Gyt, ft;
    double *s, *gtmp, *gtmp2;
    /* averages */
    double *cx, *cy, T;
} orc_state;

static int alloc_state(orc_state *S)
{
    int64_t n = S->n, m = S->m, ny = S->ny;
    S->x = malloc(sizeof(double) * n);   S->xt = malloc(sizeof(double) * n);
    S->y = malloc(sizeof(double) * (ny + 1)); S->yt = malloc(sizeof(double) * (ny + 1));
    S->U = malloc(sizeof(double) * (m + 1) * n); S->Ut = malloc(sizeof(double) * (m + 1) * n);
    S->Gy = malloc(sizeof(double) * (ny + 1)); S->Gyt = malloc(sizeof(double) * (ny + 1));
    S->Gyp = malloc(sizeof(double) * (ny + 1));
    S->gxk = malloc(sizeof(double) * n); S->gxp = malloc(sizeof(double) * n);
    S->s = malloc(sizeof(double) * (n + ny + 1));
    S->gtmp = malloc(sizeof(double) * n); S->gtmp2 = malloc(sizeof(double) * n);
    S->cx = malloc(sizeof(double) * n); S->cy = malloc(sizeof(double) * (ny + 1));
    return (S->x && S->xt && S->y && S->yt && S->U && S->Ut && S->Gy && S->Gyt && S->Gyp &&
            S->gxk && S->gxp && S->s && S->gtmp && S->gtmp2 && S->cx && S->cy) ? 0 : -1;
}

static void free_state(orc_state *S)
{
    free(S->x); free(S->xt); free(S->y); free(S->yt); free(S->U); free(S->Ut);
    free(S->Gy); free(S->Gyt); free(S->Gyp); free(S->gxk); free(S->gxp); free(S->s);
    free(S->gtmp); free(S->gtmp2); free(S->cx); free(S->cy);
}

/* evaluate the operator at S->x and install U, Gy, f (and grad_x for xy) */
static void install_point(orc_state *S)
{
    stack_matvec(S->P, S->x, S->U);
    constraint_values(S->P, S->x, S->U, S->Gy, &S->f);
    grad_x(S->P, S->U, S->y, S->gxk);
}

/* one accepted APDB iteration with backtracking; returns number of trials, or -1 on failure.
 * Epoch scalars are passed by pointer: tau (in: tau_k initial guess; out: tau_{k+1}),
 * tau_prev (tau_{k-1}), sig_prev (sigma_{k-1}), gam (gamma_k), sig0, alpha_k, beta_k, ke.   */
typedef struct {
    double tau, tau_prev, sig_prev, gam, sig0, alpha_k, beta_k;
    int64_t ke;
} orc_epoch;

static int64_t apdb_iteration(orc_state *S, orc_epoch *ep, double *trace_row)
{
    const orc_problem *P = S->P;
    const orc_options *o = S->o;
    const int64_t n = S->n, m = S->m, p = S->p, ny = S->ny;
    int64_t trials = 0;
    double sig = 0, th = 0, E = 0, rhs = 0;
    for (;;) {
        ++trials;
        if (trials > 400) return -1;
        double tau = ep->tau;
        sig = ep->gam * tau;                 /* sigma_k = gamma_k tau_k */
        th = ep->sig_prev / sig;             /* theta_k = sigma_{k-1} / sigma_k */
        double dd, dyy;
        if (o->variant == 0) {
            /* ---- APDB-yx, eq. (apdb-yx-y): dual step with momentum on grad_y Phi ---- */
            double alpha_next = o->c_alpha / sig;                    /* alpha_{k+1} = c_a / sigma_k */
            for (int64_t l = 0; l < ny; ++l) {
                S->s[l] = (1.0 + th) * S->Gy[l] - th * S->Gyp[l];     /* s^k */
                S->yt[l] = S->y[l] + sig * S->s[l];                   /* argmin -<s,y> + D_d/sigma */
            }
            project_y(P, S->yt);                                      /* ... over Y */
            grad_x(P, S->U, S->yt, S->gtmp);                          /* grad_x Phi(x^k, y^{k+1}) */
            for (int64_t j = 0; j < n; ++j)
                S->xt[j] = clip(S->x[j] - tau * S->gtmp[j], P->lb[j], P->ub[j]);
            stack_matvec(P, S->xt, S->Ut);
            constraint_values(P, S->xt, S->Ut, S->Gyt, &S->ft);
            /* E_k of §3.2 at (x^{k+1}, y^{k+1}), y = y^{k+1}:
             *   Phi(x',y) - Phi(x^k,y) - <grad_x Phi(x^k,y), x'-x^k> = 1/2 d'Q(lambda)d, computed as
             *   1/2 [ d'(Q_0x' - Q_0x^k) + sum lambda_i d'(Q_i x' - Q_i x^k) ]  (Phi quadratic in x) */
            double quad = 0.0;
            dd = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                double d = S->xt[j] - S->x[j];
                dd += d * d;
            }
            for (int64_t i = 0; i <= m; ++i) {
                double w = (i == 0) ? 1.0 : S->yt[p + i - 1];
                double e = 0.0;
                for (int64_t j = 0; j < n; ++j)
                    e += (S->xt[j] - S->x[j]) * (S->Ut[i * n + j] - S->U[i * n + j]);
                quad += w * e;
            }
            quad *= 0.5;
            double dG = 0.0;                 /* ||grad_y Phi(x') - grad_y Phi(x^k)||^2 */
            dyy = 0.0;
            for (int64_t l = 0; l < ny; ++l) {
                double a = S->Gyt[l] - S->Gy[l];
                dG += a * a;
                double b = S->yt[l] - S->y[l];
                dyy += b * b;
            }
            double Dp = 0.5 * dd, Dd = 0.5 * dyy;
            E = quad - Dp / tau + dG / (2.0 * alpha_next) - (1.0 / sig - th * ep->alpha_k) * Dd;
            rhs = -(o->delta / tau) * Dp - (o->delta / sig) * Dd;
            if (E <= rhs) {
                ep->alpha_k = alpha_next;
                break;
            }
        } else {
            /* ---- APDB-xy, Algorithm 1: primal step with momentum on grad_x Phi ---- */
            double alpha_next = o->c_alpha / tau;                    /* alpha_{k+1} = c_a / tau_k */
            double beta_next = o->gamma0 * o->c_beta / sig;          /* beta_{k+1} = g0 c_b / sigma_k */
            for (int64_t j = 0; j < n; ++j) {
                S->s[j] = (1.0 + th) * S->gxk[j] - th * S->gxp[j];
                S->xt[j] = clip(S->x[j] - tau * S->s[j], P->lb[j], P->ub[j]);
            }
            stack_matvec(P, S->xt, S->Ut);
            constraint_values(P, S->xt, S->Ut, S->Gyt, &S->ft);      /* grad_y Phi(x^{k+1}, y^k) */
            for (int64_t l = 0; l < ny; ++l) S->yt[l] = S->y[l] + sig * S->Gyt[l];
            project_y(P, S->yt);
            /* grad_x Phi(x',y') - grad_x Phi(x',y^k) = sum (l'_i - l_i)(Q_i x' + q_i) + A'(v'-v) */
            for (int64_t j = 0; j < n; ++j) {
                double a = 0.0, b = S->Ut[j] - S->U[j];
                for (int64_t i = 1; i <= m; ++i) {
                    a += (S->yt[p + i - 1] - S->y[p + i - 1]) * (S->Ut[i * n + j] + P->q[i * n + j]);
                    b += S->y[p + i - 1] * (S->Ut[i * n + j] - S->U[i * n + j]);
                }
                for (int64_t l = 0; l < p; ++l) a += (S->yt[l] - S->y[l]) * P->A[l * n + j];
                S->gtmp[j] = a;      /* y-difference of grad_x Phi at x' */
                S->gtmp2[j] = b;     /* grad_x Phi(x',y^k) - grad_x Phi(x^k,y^k) */
            }
            dd = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                double d = S->xt[j] - S->x[j];
                dd += d * d;
            }
            dyy = 0.0;
            for (int64_t l = 0; l < ny; ++l) {
                double b = S->yt[l] - S->y[l];
                dyy += b * b;
            }
            double Dp = 0.5 * dd, Dd = 0.5 * dyy;
            /* E_k of eq. (backtracking) */
            E = nrm2sq(S->gtmp, n) / (2.0 * alpha_next) - Dd / sig +
                nrm2sq(S->gtmp2, n) / (2.0 * beta_next) -
                (1.0 / tau - th * (ep->alpha_k + ep->beta_k)) * Dp;
            rhs = -(o->delta / tau) * Dp - (o->delta / sig) * Dd;
            if (E <= rhs) {
                ep->alpha_k = alpha_next;
                ep->beta_k = beta_next;
                break;
            }
        }
        if (isnan(E) || isnan(rhs)) return -1;
        ep->tau *= o->eta;                   /* tau_k <- eta tau_k */
    }
    /* accepted: averages (Algorithm 1, after the loop) */
    double tau = ep->tau;
    if (ep->ke == 0) ep->sig0 = sig;
    double tk = sig / ep->sig0;
    for (int64_t j = 0; j < n; ++j) S->cx[j] += tk * S->xt[j];
    for (int64_t l = 0; l < ny; ++l) S->cy[l] += tk * S->yt[l];
    S->T += tk;
    /* step-size rule (Algorithm 1; non-monotone form eq. (nonmonotone-tau)) */
    double gam_next = ep->gam * (1.0 + o->mu * tau);
    double tau_next = tau * sqrt(ep->gam / gam_next * (1.0 + o->c_nm * tau / ep->tau_prev));
    if (trace_row) {
        trace_row[0] = tau; trace_row[1] = sig; trace_row[2] = (double)trials;
        trace_row[3] = E; trace_row[4] = rhs;
    }
    /* shift state */
    memcpy(S->Gyp, S->Gy, sizeof(double) * ny);
    memcpy(S->gxp, S->gxk, sizeof(double) * n);
    memcpy(S->x, S->xt, sizeof(double) * n);
    memcpy(S->y, S->yt, sizeof(double) * ny);
    memcpy(S->U, S->Ut, sizeof(double) * (m + 1) * n);
    memcpy(S->Gy, S->Gyt, sizeof(double) * ny);
    S->f = S->ft;
    grad_x(P, S->U, S->y, S->gxk);
    ep->sig_prev = sig;
    ep->tau_prev = tau;
    ep->tau = tau_next;
    ep->gam = gam_next;
    ep->ke += 1;
    return trials;
}

/* epoch initialisation (Algorithm 1, first line) */
static void epoch_init(orc_state *S, orc_epoch *ep)
{
    const orc_options *o = S->o;
    ep->tau = o->tau_bar;
    ep->tau_prev = o->tau_bar;
    ep->sig_prev = o->gamma0 * o->tau_bar;
    ep->gam = o->gamma0;
    ep->sig0 = 0.0;
    ep->ke = 0;
    /* (R2): alpha_0, beta_0 from tau_{-1}, sigma_{-1} */
    ep->alpha_k = (o->variant == 0) ? o->c_alpha / ep->sig_prev : o->c_alpha / ep->tau_prev;
    ep->beta_k = o->gamma0 * o->c_beta / ep->sig_prev;
    /* x^{-1} = x^0, y^{-1} = y^0 */
    memcpy(S->Gyp, S->Gy, sizeof(double) * S->ny);
    memcpy(S->gxp, S->gxk, sizeof(double) * S->n);
    memset(S->cx, 0, sizeof(double) * S->n);
    memset(S->cy, 0, sizeof(double) * S->ny);
    S->T = 0.0;
}

/* move to the restart point (R4) */
static void restart_point(orc_state *S)
{
    if (S->o->restart_from_average && S->T > 0.0) {
        for (int64_t j = 0; j < S->n; ++j) S->x[j] = S->cx[j] / S->T;
        for (int64_t l = 0; l < S->ny; ++l) S->y[l] = S->cy[l] / S->T;
        install_point(S);
    }
}

static int validate(const orc_problem *P, const orc_options *o)
{
    if (P->n <= 0 || P->m < 0 || P->p < 0) return -1;
    if (!(o->eta > 0 && o->eta < 1)) return -1;
    if (!(o->tau_bar > 0 && o->gamma0 > 0 && o->mu >= 0)) return -1;
    if (o->variant == 0) {
        if (!(o->c_alpha > 0 && o->delta >= 0 && o->delta < 1 && o->c_alpha + o->delta <= 1)) return -1;
    } else {
        double s = o->c_alpha + o->c_beta + o->delta;
        if (!(o->c_alpha >= 0 && o->c_beta > 0 && o->delta >= 0 && s > 0 && s < 1)) return -1;
    }
    for (int64_t j = 0; j < P->n; ++j)
        if (!(P->lb[j] <= P->ub[j]) || P->lb[j] == INFINITY || P->ub[j] == -INFINITY) return -1;
    if (P->lambda_set < 0 || P->lambda_set > 2) return -1;
    if (P->lambda_set == 2) {
        if (P->n_soc < 1 || !P->soc_dims) return -1;
        int64_t tot = 0;
        for (int64_t c = 0; c < P->n_soc; ++c) {
            if (P->soc_dims[c] < 1) return -1;
            tot += P->soc_dims[c];
        }
        if (tot > P->m) return -1;
    }
    if (P->q_stored) {
        if (P->q_stored[0] != (P->has_q0 ? 1 : 0)) return -1;
        for (int64_t i = 0; i <= P->m; ++i)
            if (P->q_stored[i] != 0 && P->q_stored[i] != 1) return -1;
    }
    if (P->lambda_set == 1 && (P->m < 1 || P->ball > 0.0 || P->ball_l > 0.0)) return -1;
    if (!(P->q0_shift >= 0.0 && P->ball >= 0.0 && P->ball_v >= 0.0 && P->ball_l >= 0.0)) return -1;
    if (P->ball > 0.0 && (P->ball_v > 0.0 || P->ball_l > 0.0)) return -1;
    if (o->restart == 1 && o->restart_every < 1) return -1;
    if (o->restart == 2 && (o->ada_every < 1 || !(o->xi > 0) || !(o->q_restart > 0 && o->q_restart < 1)))
        return -1;
    return 0;
}

/*
 * Solve with rAPDB.  x0 (n) / y0 (p+m, order (v, lambda)) may be NULL.
 * trace (optional): trace_cap rows of 5 doubles per accepted iteration
 *   {tau_k, sigma_k, trials_k, E_k, rhs_k}.
 */
int orc_solve(const orc_problem *P, const orc_options *o, const double *x0, const double *y0,
              double *x_out, double *y_out, orc_info *info, double *trace, int64_t trace_cap)
{
    memset(info, 0, sizeof(*info));
    if (validate(P, o)) { info->status = ORC_INVALID; return ORC_INVALID; }
    orc_state S;
    memset(&S, 0, sizeof(S));
    S.P = P; S.o = o; S.n = P->n; S.m = P->m; S.p = P->p; S.ny = P->p + P->m;
    if (alloc_state(&S)) { free_state(&S); info->status = ORC_INVALID; return ORC_INVALID; }
    for (int64_t j = 0; j < S.n; ++j) S.x[j] = clip(x0 ? x0[j] : 0.0, P->lb[j], P->ub[j]);
    for (int64_t l = 0; l < S.ny; ++l) S.y[l] = y0 ? y0[l] : 0.0;
    project_y(P, S.y);
    install_point(&S);

    int64_t k = 0, trials = 0, restarts = 0, gap_evals = 0, checked_k = -1;
    double Gref = NAN, last_gap = NAN, kk[6];
    int status = ORC_NOT_CONVERGED;
    orc_epoch ep;
    epoch_init(&S, &ep);
    double crit = NAN;
    for (;;) {
        kkt_eval(P, S.x, S.y, S.U, S.Gy, S.f, kk);
        crit = (o->stop_rule == 1) ? paper_criterion(P, S.Gy, S.f, o->f_star) : kk[0];
        if (isnan(kk[0]) || isnan(crit)) { status = ORC_NUMERICAL; break; }
        if (crit <= o->tol) { status = ORC_CONVERGED; break; }
        if (k >= o->max_iter) { status = ORC_NOT_CONVERGED; break; }
        int do_restart = 0;
        if (o->restart == 1 && ep.ke >= o->restart_every) do_restart = 1;
        if (o->restart == 2 && k != checked_k) {
            checked_k = k;    /* one schedule check per global k, also after a restart */
            if (k == o->ada_first) {
                double g4[4];
                if (gap_eval(P, S.x, S.y, o->xi, o->inner_tol, o->max_inner, g4)) { status = ORC_NUMERICAL; break; }
                Gref = g4[0]; last_gap = g4[0]; ++gap_evals;
            } else if (k > o->ada_first && (k % o->ada_every) == 0 && !isnan(Gref)) {
                double g4[4];
                const double *xc = S.x, *yc = S.y;
                double *ax = NULL, *ay = NULL;
                if (o->restart_from_average && S.T > 0.0) {
                    ax = malloc(sizeof(double) * S.n); ay = malloc(sizeof(double) * (S.ny + 1));
                    for (int64_t j = 0; j < S.n; ++j) ax[j] = S.cx[j] / S.T;
                    for (int64_t l = 0; l < S.ny; ++l) ay[l] = S.cy[l] / S.T;
                    xc = ax; yc = ay;
                }
                int rc = gap_eval(P, xc, yc, o->xi, o->inner_tol, o->max_inner, g4);
                free(ax); free(ay);
                if (rc) { status = ORC_NUMERICAL; break; }
                ++gap_evals; last_gap = g4[0];
                if (g4[0] <= o->q_restart * Gref) { do_restart = 1; Gref = g4[0]; }   /* eq. (ada_restart) */
            }
        }
        if (do_restart) {
            restart_point(&S);
            epoch_init(&S, &ep);
            ++restarts;
            continue;   /* re-check termination at the restart point */
        }
        double *row = (trace && k < trace_cap) ? trace + 5 * k : NULL;
        int64_t t = apdb_iteration(&S, &ep, row);
        if (t < 0) { status = ORC_NUMERICAL; break; }
        trials += t;
        ++k;
    }
    memcpy(x_out, S.x, sizeof(double) * S.n);
    if (y_out) memcpy(y_out, S.y, sizeof(double) * S.ny);
    info->iters = k; info->trials = trials; info->restarts = restarts; info->gap_evals = gap_evals;
    info->status = status;
    info->rel_kkt = kk[0]; info->rel_dual = kk[1]; info->rel_pri = kk[2]; info->rel_comp = kk[3];
    info->f = kk[4]; info->max_violation = kk[5]; info->last_gap = last_gap;
    info->stop_value = crit;
    free_state(&S);
    return status;
}
