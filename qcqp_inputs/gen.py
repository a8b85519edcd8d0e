"""Seeded instance generators (numpy PCG64 on the host, torch Philox on a device).

Recipes (the workloads the method is measured on):

* random convex QCQP: A_i iid N(0,1) n x n, Q_i = sym(A_i A_i^T / n) + shift*I for i=0..m,
  q_i ~ N(0, I), c_0 = 0, c_i ~ U(-1, -0.1) so that x = 0 is strictly feasible (a Slater
  point), X = [-10, 10]^n.  With shift = 0.01 every Q_i is positive definite.
* kernel-learning QCQP (§5.2 stand-in): two Gaussian clusters in R^20, RBF Gram matrices,
  variables (alpha, t); see kml_qcqp.
* rounded instances: Q rounded once (round-to-nearest-even) to a 16/32-bit storage type; the
  rounded values, upcast exactly, ARE the instance that both the oracle and the GPU solve.
"""
from __future__ import annotations

import dataclasses
import numpy as np

BASE_SEED = 20260529


def config_seed(config: int, instance: int = 0) -> int:
    """Fixed seed per (workload number, instance index)."""
    return BASE_SEED + 1000 * config + instance


@dataclasses.dataclass
class Instance:
    n: int
    m: int
    p: int
    Q: object            # (m+1 or m, n, n) array (numpy or torch), dtype float64/float32/bf16/fp16
    q: np.ndarray        # (m+1, n) float64
    c: np.ndarray        # (m+1,) float64
    lb: np.ndarray       # (n,)
    ub: np.ndarray       # (n,)
    A: np.ndarray | None = None   # (p, n)
    b: np.ndarray | None = None   # (p,)
    has_q0: bool = True
    name: str = ""
    lambda_set: str = "nonneg"   # "nonneg" (QCQP), "simplex" (min-max over a simplex) or
                                 # "cones" (R^{m0}_+ x second-order cones of sizes soc_dims)
    q0_shift: float = 0.0        # the objective's Hessian is Q_0 + q0_shift I
    q_stored: object = None      # (m+1,) 0/1: which Q_i are stored in Q (None: all but Q_0 per has_q0)
    soc_dims: object = None      # second-order cone sizes at the end of lambda ("cones")

    def q_as_float64_numpy(self) -> np.ndarray:
        Q = self.Q
        if hasattr(Q, "detach"):
            Q = Q.detach().to("cpu")
            import torch
            return Q.to(torch.float64).numpy()
        return np.asarray(Q, dtype=np.float64)


def _box(n, lo=-10.0, hi=10.0):
    return np.full(n, lo), np.full(n, hi)


def random_qcqp(n: int, m: int, seed: int, shift: float = 0.0, box: float = 10.0,
                p: int = 0) -> Instance:
    """Random convex QCQP on the host with numpy PCG64 (float64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Q = np.empty((m + 1, n, n))
    for i in range(m + 1):
        Ai = rng.standard_normal((n, n))
        Qi = Ai @ Ai.T / n
        Qi = 0.5 * (Qi + Qi.T)
        if shift:
            Qi[np.diag_indices(n)] += shift
        Q[i] = Qi
    q = rng.standard_normal((m + 1, n))
    c = np.concatenate([[0.0], rng.uniform(-1.0, -0.1, m)])
    lb, ub = _box(n, -box, box)
    A = b = None
    if p > 0:
        A = rng.standard_normal((p, n)) / np.sqrt(n)
        b = np.zeros(p)          # x = 0 stays feasible (Slater point)
    return Instance(n, m, p, Q, q, c, lb, ub, A, b, True, f"rand_n{n}_m{m}_s{seed}")


def random_qcqp_torch(n: int, m: int, seed: int, shift: float = 0.0, box: float = 10.0,
                      device="cuda", store_dtype=None) -> Instance:
    """Same recipe drawn with torch's Philox generator on `device`.

    Q is produced matrix by matrix in float64 and stored in `store_dtype` (float64 if None),
    rounded once with round-to-nearest-even, so a 16-bit stack never exists in float64 at once.
    q and c are drawn on the device and returned as float64 numpy arrays.
    """
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    sd = store_dtype or torch.float64
    Q = torch.empty((m + 1, n, n), dtype=sd, device=device)
    eye = torch.eye(n, dtype=torch.float64, device=device)
    for i in range(m + 1):
        Ai = torch.randn((n, n), generator=g, dtype=torch.float64, device=device)
        Qi = Ai @ Ai.T / n
        Qi = 0.5 * (Qi + Qi.T)
        if shift:
            Qi = Qi + shift * eye
        Q[i].copy_(Qi.to(sd))
        del Ai, Qi
    q = torch.randn((m + 1, n), generator=g, dtype=torch.float64, device=device).cpu().numpy()
    u = torch.rand((m,), generator=g, dtype=torch.float64, device=device).cpu().numpy()
    c = np.concatenate([[0.0], -1.0 + 0.9 * u])
    lb, ub = _box(n, -box, box)
    return Instance(n, m, 0, Q, q, c, lb, ub, None, None, True, f"randT_n{n}_m{m}_s{seed}")


EXACT_FRAC_BITS = 16   # A entries are multiples of 2^-16 (random_qcqp_exact)


def _exact_gaussian(rng, n):
    """n x n standard normal draws rounded to multiples of 2^-16 and clipped to [-8, 8]: every
    product of two entries is an integer multiple of 2^-32 below 2^38 of those units, so the
    n-term sums of A A' stay below 2^53 units for n <= 2^15 and are exact in FP64 in any
    summation order."""
    scale = float(2 ** EXACT_FRAC_BITS)
    return np.clip(np.rint(rng.standard_normal((n, n)) * scale), -8 * scale, 8 * scale) / scale


def random_qcqp_exact(n: int, m: int, seed: int, shift: float = 0.0, box: float = 10.0,
                      device=None) -> Instance:
    """The random convex QCQP recipe with bitwise-reproducible matrices on any machine.

    A_i is drawn on the host (numpy PCG64) and rounded to multiples of 2^-16, so A_i A_i' is
    exact in FP64 whatever BLAS or GPU computes it; Q_i = (A_i A_i') / n (one correctly rounded
    division per entry) + shift I.  With device="cuda" the products run on the GPU (torch), the
    stack stays there, and the bytes equal the host version's.  q_i ~ N(0, I), c_0 = 0,
    c_i ~ U(-1, -0.1), X = [-box, box]^n, all host float64.
    """
    if n > 2 ** 15:
        raise ValueError("random_qcqp_exact needs n <= 32768 for exact products")
    rng = np.random.Generator(np.random.PCG64(seed))
    if device is None:
        Q = np.empty((m + 1, n, n))
        for i in range(m + 1):
            A = _exact_gaussian(rng, n)
            Qi = (A @ A.T) / float(n)
            if shift:
                Qi[np.diag_indices(n)] += shift
            Q[i] = Qi
    else:
        import torch
        Q = torch.empty((m + 1, n, n), dtype=torch.float64, device=device)
        # a device tensor divisor keeps the division a true per-element division
        nt = torch.tensor(float(n), dtype=torch.float64, device=device)
        for i in range(m + 1):
            A = torch.from_numpy(_exact_gaussian(rng, n)).to(device)
            Qi = torch.div(A @ A.T, nt)
            if shift:
                Qi.diagonal().add_(shift)
            Q[i].copy_(Qi)
            del A, Qi
    q = rng.standard_normal((m + 1, n))
    c = np.concatenate([[0.0], rng.uniform(-1.0, -0.1, m)])
    lb, ub = _box(n, -box, box)
    return Instance(n, m, 0, Q, q, c, lb, ub, None, None, True, f"randX_n{n}_m{m}_s{seed}")


def stack_sha256(Q) -> str:
    """sha256 of a Q stack's bytes (numpy or torch, any device), matrix by matrix."""
    import hashlib
    h = hashlib.sha256()
    for i in range(Q.shape[0]):
        Qi = Q[i]
        if hasattr(Qi, "detach"):
            Qi = Qi.detach().cpu().numpy()
        h.update(np.ascontiguousarray(Qi).tobytes())
    return h.hexdigest()


def paper_random_qcqp(n: int = 1000, m: int = 10, seed: int = 0) -> Instance:
    """The random QCQPs of the paper's first experiment (§5.1), drawn afresh (its instances and
    seeds are not published): Q_i = L_i' S_i L_i for i = 0..m with L_i the orthonormal factor of
    the QR decomposition of an n x n standard Gaussian matrix and S_i diagonal with entries
    U[0, 100], the smallest set to 0 (so mu = 0); q_i ~ N(0, I); c_0 = 0 and c_i = r_i with
    -r_i ~ U[0, 1]; X = [-10, 10]^n.  Host numpy PCG64, float64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Q = np.empty((m + 1, n, n))
    for i in range(m + 1):
        L, _ = np.linalg.qr(rng.standard_normal((n, n)))
        d = rng.uniform(0.0, 100.0, n)
        d[np.argmin(d)] = 0.0
        Qi = (L.T * d) @ L
        Q[i] = 0.5 * (Qi + Qi.T)
    q = rng.standard_normal((m + 1, n))
    c = np.concatenate([[0.0], -rng.uniform(0.0, 1.0, m)])
    lb, ub = _box(n)
    return Instance(n, m, 0, Q, q, c, lb, ub, None, None, True, f"paper_rand_n{n}_m{m}_s{seed}")


def random_conic_qcqp(n: int, m_lin: int, soc_dims, seed: int, p: int = 0,
                      box: float = 10.0) -> Instance:
    """Convex problem with the constraint g(x) in -K, K = R^{m_lin}_+ x Q^{k_1} x ... (second-order
    cones at the end).  Objective and the m_lin scalar constraints: Q_i = A_iA_i'/n (+0.1 I for Q_0),
    q_i ~ N(0, I), c_i ~ U(-1, -0.1).  Each cone: a convex quadratic leading component of the same
    kind and affine tail components q ~ N(0, I/n) with no stored matrix, constants chosen so that
    x = 0 lies strictly inside (-c_lead > ||c_tail||): a Slater point.  Host numpy PCG64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dims = [int(k) for k in soc_dims]
    m = m_lin + sum(dims)
    stored = np.zeros(m + 1, dtype=np.int32)
    stored[0] = 1
    stored[1:m_lin + 1] = 1
    off = m_lin + 1
    for k in dims:
        stored[off] = 1                        # the cone's leading component is quadratic
        off += k
    mats = []
    for i in range(m + 1):
        if stored[i]:
            A = rng.standard_normal((n, n))
            Qi = A @ A.T / n + (0.1 * np.eye(n) if i == 0 else 0.0)
            mats.append(0.5 * (Qi + Qi.T))
    Q = np.stack(mats)
    q = rng.standard_normal((m + 1, n))
    c = np.concatenate([[0.0], rng.uniform(-1.0, -0.1, m)])
    off = m_lin + 1
    for k in dims:
        q[off + 1:off + k] /= np.sqrt(n)
        tail = rng.uniform(-0.3, 0.3, k - 1)
        c[off + 1:off + k] = tail
        c[off] = -(0.5 + np.linalg.norm(tail))
        off += k
    lb, ub = _box(n, -box, box)
    A = rng.standard_normal((p, n)) if p else None
    b = (A @ rng.uniform(-0.1, 0.1, n)) if p else None
    return Instance(n, m, p, Q, q, c, lb, ub, A, b, True, f"conic_n{n}_m{m_lin}_k{dims}_s{seed}",
                    lambda_set="cones", q_stored=stored, soc_dims=dims)


def round_instance(inst: Instance, dtype: str) -> Instance:
    """Round Q once (RNE) to 'float32' | 'bfloat16' | 'float16' (torch tensors on Q's device)."""
    import torch
    tdt = {"float32": torch.float32, "bfloat16": torch.bfloat16, "float16": torch.float16,
           "float64": torch.float64}[dtype]
    Q = inst.Q if hasattr(inst.Q, "to") else torch.from_numpy(np.ascontiguousarray(inst.Q))
    return dataclasses.replace(inst, Q=Q.to(tdt), name=inst.name + "_" + dtype)


def kml_qcqp(npts: int = 8000, dim: int = 20, bandwidths=(0.5, 1.0, 2.0, 4.0, 8.0), seed: int = 0,
             C: float = 1.0, device=None, store_dtype=None) -> Instance:
    """Kernel-learning QCQP in variables z = (alpha, t), n = npts + 1.

    Two Gaussian clusters (means +-mu*1/sqrt(dim), identity covariance), labels +-1, features
    standardised per column.  K_j = exp(-||a-a'||^2 / (2 h_j^2)) (diag = 1, tr K_j = npts).
        min  -2 * 1'alpha + c * t
        s.t. g_j(z) = 1/2 z' Q_j z - t <= 0,  Q_j = blkdiag(2 diag(y) K_j diag(y) / tr K_j, 0)
             y'alpha = 0 (p = 1),  0 <= alpha <= C,  0 <= t <= npts * C^2
    with c = sum_j tr K_j.  Q_0 = 0 is not stored (has_q0 = False).
    """
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    half = npts // 2
    mu = np.ones(dim) / np.sqrt(dim)
    X = np.concatenate([rng.standard_normal((half, dim)) + mu,
                        rng.standard_normal((npts - half, dim)) - mu])
    y = np.concatenate([np.ones(half), -np.ones(npts - half)])
    perm = rng.permutation(npts)
    X, y = X[perm], y[perm]
    X = (X - X.mean(0)) / X.std(0)
    n = npts + 1
    m = len(bandwidths)
    dev = device or "cpu"
    sd = store_dtype or torch.float64
    Xt = torch.from_numpy(X).to(dev)
    yt = torch.from_numpy(y).to(dev)
    sq = (Xt * Xt).sum(1)
    D2 = (sq[:, None] + sq[None, :] - 2.0 * (Xt @ Xt.T)).clamp_min_(0.0)
    Q = torch.zeros((m, n, n), dtype=sd, device=dev)
    traces = []
    for j, h in enumerate(bandwidths):
        K = torch.exp(-D2 / (2.0 * h * h))
        tr = float(torch.diagonal(K).sum())
        traces.append(tr)
        H = (yt[:, None] * K * yt[None, :]) * (2.0 / tr)
        H = 0.5 * (H + H.T)
        Q[j, :npts, :npts] = H.to(sd)
        del K, H
    csum = float(sum(traces))
    q = np.zeros((m + 1, n))
    q[0, :npts] = -2.0
    q[0, npts] = csum
    q[1:, npts] = -1.0
    c = np.zeros(m + 1)
    lb = np.zeros(n)
    ub = np.concatenate([np.full(npts, C), [npts * C * C]])
    A = np.concatenate([y, [0.0]])[None, :]
    b = np.zeros(1)
    Qout = Q if (device is not None) else Q.numpy()
    return Instance(n, m, 1, Qout, q, c, lb, ub, A, b, False, f"kml_n{npts}_s{seed}")


def kml_minmax(npts: int = 4000, dim: int = 200, density: float = 0.1, lam: float = 1.0,
               seed: int = 0, device=None, store_dtype=None) -> Instance:
    """The kernel-learning min-max problem of §5 (min-max-KML) as a saddle problem of this form:

        min_{x >= 0}  max_{y in simplex, v}  lam ||x||^2 - 2 1'x + sum_i y_i (c / r_i) x'H(K_i)x + v b'x

    with H(K) = diag(b) K diag(b), the three kernels of §5 -- polynomial (1 + a'a')^2, Gaussian
    exp(-0.5 ||a - a'||^2 / 0.1) and linear a'a' -- each normalised to unit diagonal (so
    r_i = tr K_i = npts), c = sum_i r_i, and the constraint <b, x> = 0 entering through the free
    multiplier v (p = 1).  In the library's terms: has_q0 = False, q0_shift = 2 lam (the
    objective's Hessian 2 lam I costs no stored matrix), q_0 = -2 1, Q_i = 2 (c / r_i) H(K_i),
    q_i = 0, c_i = 0, lambda_set = "simplex", lb = 0, ub = +inf; strongly convex in x with
    mu = 2 lam.

    Data: a synthetic stand-in for the SIDO0 molecular descriptors (which are not available
    here): `dim` binary features per point, drawn Bernoulli with a rate that differs between the
    two classes (labels +-1, balanced), then mean-centred and divided by their standard
    deviation per column, as §5 describes.
    """
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    half = npts // 2
    base = rng.uniform(0.5 * density, 1.5 * density, dim)
    shift = rng.uniform(-0.5, 0.5, dim) * density
    p_pos = np.clip(base + shift, 0.01, 0.99)
    p_neg = np.clip(base - shift, 0.01, 0.99)
    X = np.concatenate([(rng.random((half, dim)) < p_pos).astype(float),
                        (rng.random((npts - half, dim)) < p_neg).astype(float)])
    lab = np.concatenate([np.ones(half), -np.ones(npts - half)])
    perm = rng.permutation(npts)
    X, lab = X[perm], lab[perm]
    sd_ = X.std(0)
    sd_[sd_ == 0] = 1.0
    X = (X - X.mean(0)) / sd_
    dev = device or "cpu"
    sd = store_dtype or torch.float64
    Xt = torch.from_numpy(X).to(dev)
    bt = torch.from_numpy(lab).to(dev)
    G = Xt @ Xt.T
    sq = torch.diagonal(G).clone()
    m = 3
    Q = torch.empty((m, npts, npts), dtype=sd, device=dev)
    c_total = 3.0 * npts             # sum of the traces of the normalised kernels
    for i in range(m):
        if i == 0:
            K = (1.0 + G) ** 2
        elif i == 1:
            K = torch.exp(-0.5 * (sq[:, None] + sq[None, :] - 2.0 * G).clamp_min_(0.0) / 0.1)
        else:
            K = G.clone()
        dg = torch.sqrt(torch.diagonal(K).clamp_min(1e-300))
        K = K / dg[:, None] / dg[None, :]
        H = bt[:, None] * K * bt[None, :]
        H = 0.5 * (H + H.T)
        Q[i] = (2.0 * c_total / npts * H).to(sd)
        del K, H
    q = np.zeros((m + 1, npts))
    q[0] = -2.0
    c = np.zeros(m + 1)
    lb = np.zeros(npts)
    ub = np.full(npts, np.inf)
    Qout = Q if (device is not None) else Q.numpy()
    return Instance(npts, m, 1, Qout, q, c, lb, ub, lab[None, :].copy(), np.zeros(1), False,
                    f"kmlmm_n{npts}_s{seed}", lambda_set="simplex", q0_shift=2.0 * lam)


def serving_trace(num: int, seed: int, n_range=(200, 3000), m_range=(5, 200), rate=None):
    """Request sizes (n_k, m_k), per-request seeds and Poisson arrival times (seconds).

    rate=None means closed loop (all arrivals at t = 0).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = rng.integers(n_range[0], n_range[1] + 1, size=num)
    ms = rng.integers(m_range[0], m_range[1] + 1, size=num)
    seeds = seed * 7919 + np.arange(num)
    if rate is None:
        arr = np.zeros(num)
    else:
        arr = np.cumsum(rng.exponential(1.0 / rate, size=num))
    return [dict(n=int(ns[k]), m=int(ms[k]), seed=int(seeds[k]), arrival=float(arr[k]))
            for k in range(num)]
