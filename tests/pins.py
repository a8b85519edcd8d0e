"""Independent reference solvers used to pin the oracle (test infrastructure).

None of these share code with the oracle or the GPU path:
  * ball_qp_bisection: the single-ball-constrained QP solved by 1-D multiplier bisection on the
    eigendecomposition of Q_0 (trust-region subproblem, easy case);
  * kkt_enumerate: brute-force enumeration of active constraint sets x box faces for tiny n, m,
    with the multipliers found by (nested) bisection on the monotone map lambda -> g(x(lambda));
  * barrier_qcqp: a textbook log-barrier interior-point method (Newton with backtracking,
    equality-constrained Newton steps when p > 0) giving f* independently;
  * box_qp_enumerate: exact minimiser of a strictly convex box QP by enumerating faces;
  * smoothed_gap: the self-centred smoothed duality gap of a plain QCQP (lambda >= 0, no
    equalities) with the y-part in closed form and the x-part by box_qp_enumerate (tiny n).
"""
import itertools

import numpy as np


def ball_qp_bisection(Q0, q0, rho):
    """min 1/2 x'Q0 x + q0'x  s.t. 1/2||x||^2 <= rho  (Q0 positive definite)."""
    e, V = np.linalg.eigh(Q0)
    b = V.T @ q0

    def xnorm2(lam):
        return float(np.sum(b * b / (e + lam) ** 2))

    if xnorm2(0.0) <= 2 * rho:
        lam = 0.0
    else:
        lo, hi = 0.0, 1.0
        while xnorm2(hi) > 2 * rho:
            hi *= 2
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if xnorm2(mid) > 2 * rho:
                lo = mid
            else:
                hi = mid
        lam = 0.5 * (lo + hi)
    x = -V @ (b / (e + lam))
    return x, lam


def _solve_face(H, h, lb, ub, pattern):
    n = len(h)
    x = np.zeros(n)
    F = [j for j in range(n) if pattern[j] == 0]
    B = [j for j in range(n) if pattern[j] != 0]
    for j in B:
        x[j] = lb[j] if pattern[j] == 1 else ub[j]
    if F:
        HFF = H[np.ix_(F, F)]
        rhs = -(h[F] + (H[np.ix_(F, B)] @ x[B] if B else 0.0))
        try:
            x[F] = np.linalg.solve(HFF, rhs)
        except np.linalg.LinAlgError:
            return None
    return x


def kkt_enumerate(Q, q, c, lb, ub, tol=1e-8):
    """Global minimiser of a tiny convex QCQP (n <= 3, m <= 2, box X) by KKT enumeration."""
    m = q.shape[0] - 1
    n = q.shape[1]

    def g(i, x):
        return 0.5 * x @ Q[i] @ x + q[i] @ x + c[i]

    def x_of(lams, S, pattern):
        H = Q[0].copy()
        h = q[0].copy()
        for lam, i in zip(lams, S):
            H = H + lam * Q[i]
            h = h + lam * q[i]
        return _solve_face(H, h, lb, ub, pattern)

    def root(fun, hi0=1.0):
        """largest-region root of a non-increasing fun on [0, inf); None if fun(0) < 0."""
        f0 = fun(0.0)
        if f0 is None:
            return None
        if f0 <= 0:
            return 0.0
        hi = hi0
        while True:
            v = fun(hi)
            if v is None:
                return None
            if v < 0:
                break
            hi *= 2
            if hi > 1e12:
                return None
        lo = 0.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            v = fun(mid)
            if v is None:
                return None
            if v > 0:
                lo = mid
            else:
                hi = mid
        return 0.5 * (lo + hi)

    best = None
    for r in range(0, m + 1):
        for S in itertools.combinations(range(1, m + 1), r):
            for pattern in itertools.product((0, 1, 2), repeat=n):
                if r == 0:
                    lams = []
                elif r == 1:
                    def f1(l):
                        x = x_of([l], S, pattern)
                        return None if x is None else g(S[0], x)
                    l1 = root(f1)
                    if l1 is None:
                        continue
                    lams = [l1]
                else:
                    def inner(l1):
                        def f2(l2):
                            x = x_of([l1, l2], S, pattern)
                            return None if x is None else g(S[1], x)
                        return root(f2)

                    def f1(l1):
                        l2 = inner(l1)
                        if l2 is None:
                            return None
                        x = x_of([l1, l2], S, pattern)
                        return None if x is None else g(S[0], x)
                    l1 = root(f1)
                    if l1 is None:
                        continue
                    l2 = inner(l1)
                    if l2 is None:
                        continue
                    lams = [l1, l2]
                x = x_of(lams, S, pattern)
                if x is None:
                    continue
                # KKT checks
                ok = all(l >= -tol for l in lams)
                ok = ok and all(g(i, x) <= tol for i in range(1, m + 1))
                ok = ok and all(abs(g(i, x)) <= 1e-6 for i in S)
                ok = ok and np.all(x >= lb - tol) and np.all(x <= ub + tol)
                lam_full = np.zeros(m)
                for l, i in zip(lams, S):
                    lam_full[i - 1] = l
                grad = Q[0] @ x + q[0] + sum(lam_full[i - 1] * (Q[i] @ x + q[i]) for i in range(1, m + 1))
                for j in range(n):
                    if pattern[j] == 1:
                        ok = ok and grad[j] >= -1e-7
                    elif pattern[j] == 2:
                        ok = ok and grad[j] <= 1e-7
                if ok:
                    fval = 0.5 * x @ Q[0] @ x + q[0] @ x + c[0]
                    if best is None or fval < best[2] - 1e-12:
                        best = (x, lam_full, fval)
    return best


def barrier_qcqp(Q, q, c, lb, ub, A=None, b=None, x0=None, t0=1.0, mu=10.0, eps=1e-11):
    """Log-barrier method (feasible start x0, default 0) for min f s.t. g_i <= 0, Ax=b, box."""
    m = q.shape[0] - 1
    n = q.shape[1]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=float)
    p = 0 if A is None else A.shape[0]

    def phi_parts(x):
        gs = np.array([0.5 * x @ Q[i] @ x + q[i] @ x + c[i] for i in range(1, m + 1)])
        return gs

    def obj(x, t):
        gs = phi_parts(x)
        if np.any(gs >= 0) or np.any(x <= lb) or np.any(x >= ub):
            return np.inf
        f = 0.5 * x @ Q[0] @ x + q[0] @ x
        return t * f - np.sum(np.log(-gs)) - np.sum(np.log(x - lb)) - np.sum(np.log(ub - x))

    t = t0
    while True:
        for _ in range(200):
            gs = phi_parts(x)
            grad = t * (Q[0] @ x + q[0])
            H = t * Q[0].copy()
            for i in range(1, m + 1):
                gi = Q[i] @ x + q[i]
                grad += gi / (-gs[i - 1])
                H += np.outer(gi, gi) / gs[i - 1] ** 2 + Q[i] / (-gs[i - 1])
            grad += -1.0 / (x - lb) + 1.0 / (ub - x)
            H += np.diag(1.0 / (x - lb) ** 2 + 1.0 / (ub - x) ** 2)
            if p:
                K = np.block([[H, A.T], [A, np.zeros((p, p))]])
                sol = np.linalg.solve(K, np.concatenate([-grad, np.zeros(p)]))
                dx = sol[:n]
            else:
                dx = np.linalg.solve(H, -grad)
            lam2 = -grad @ dx
            if lam2 / 2 <= 1e-14:
                break
            s = 1.0
            f0 = obj(x, t)
            while obj(x + s * dx, t) > f0 + 0.25 * s * (grad @ dx):
                s *= 0.5
                if s < 1e-20:
                    break
            x = x + s * dx
        if (m + 2 * n) / t < eps:
            break
        t *= mu
    return x, 0.5 * x @ Q[0] @ x + q[0] @ x + c[0]


def box_qp_enumerate(H, h, lo, hi):
    """argmin_{lo<=D<=hi} h'D + 1/2 D'HD for strictly convex H (tiny n): enumerate faces."""
    n = len(h)
    best = None
    for pattern in itertools.product((0, 1, 2), repeat=n):
        D = _solve_face(H, h, lo, hi, pattern)
        if D is None:
            continue
        if np.any(D < lo - 1e-12) or np.any(D > hi + 1e-12):
            continue
        val = h @ D + 0.5 * D @ H @ D
        if best is None or val < best[1]:
            best = (D, val)
    return best


def smoothed_gap(Q, q, c, lb, ub, x, lam, xi):
    """G_xi(z; z) of the Definition "Smoothed duality gap" (§4) at z = (x, lambda), Euclidean
    distances, for min f s.t. g_i <= 0 over a box: sup over lambda' >= 0 of
    Phi(x, lambda') - xi ||lambda' - lambda||^2 minus inf over x' in X of
    Phi(x', lambda) + xi ||x' - x||^2, both centred at z.

    The y-part is concave and separable: lambda'_i = max(0, lambda_i + g_i(x) / (2 xi)).  The
    x-part is a strictly convex box QP in D = x' - x with Hessian Q(lambda) + 2 xi I and gradient
    grad_x Phi(x, lambda), minimised exactly by face enumeration (3^n faces)."""
    Q = np.asarray(Q, dtype=float)
    m = len(lam)
    g = np.array([0.5 * x @ Q[i] @ x + q[i] @ x + c[i] for i in range(1, m + 1)])
    lp = np.maximum(0.0, lam + g / (2.0 * xi))
    py = (lp - lam) @ g - xi * np.sum((lp - lam) ** 2)
    gx = Q[0] @ x + q[0] + sum(lam[i - 1] * (Q[i] @ x + q[i]) for i in range(1, m + 1))
    H = Q[0] + sum(lam[i - 1] * Q[i] for i in range(1, m + 1)) + 2.0 * xi * np.eye(len(x))
    _, val = box_qp_enumerate(H, gx, lb - x, ub - x)
    return py - val
