"""Plain FP64 CPU oracle for shifted Cholesky QR and the Cholesky QR block update.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP library.

Every routine is written from Bindhak, Pelling & Saak, "Towards an Efficient
Shifted Cholesky QR for Applications in Model Order Reduction using pyMOR"
(arXiv 2507.07788), in FP64 (the paper's precision, Sec. 3.1), with no
blocking, fusion or reordering beyond what the paper states.  numpy's matrix
product serves as the library primitive for Gram matrices and block products.

Readings of the paper taken here (each one is also listed in the design notes):
  * CholQR3 = one shifted Cholesky QR pass followed by CholeskyQR2 (Sec. 3.1,
    item 2 of the algorithm list); afterwards Algorithm 1's test-and-continue.
  * Stopping test ||X - I||_F < tol with tol = 1e-13 and at most 10 passes
    (Sec. 3.1, stopping criterion of the experiments), not u*sqrt(n).
  * If a shifted Cholesky factorisation in Algorithm 1 still breaks down, the
    shift grows by 10x as in Algorithm 2 (Sec. 2.2, shift workaround).
  * ||X|| in the shift is the 2-norm, estimated by power iteration from the
    all-ones start vector (Appendix A uses IRLM from ones with tol 1e-2).
  * Breakdown of chol() means a pivot that is not > 0 or is not finite
    (LAPACK potrf semantics).
  * Columns are never dropped on a lucky breakdown (Sec. 2.2): such a call ends
    as "not converged".

The mixed-precision form of ``orth`` (``precision=1``) is not in the paper;
it follows the reading taken here: Gramians of the shifted passes and of the
first unshifted pass are formed from the FP32-rounded iterate with FP32
accumulation, everything else (applies, shift estimate, Cholesky, the Gramian
that feeds the final pass and the stopping test) stays FP64.  An FP32 Gramian
never satisfies the stopping test; its shift is n * u32 * ||X|| (u32 = 2^-24,
floor 2 u32), escalated x10 on breakdown like Algorithm 2's.
"""
from __future__ import annotations

import math

import numpy as np

#: unit roundoff of IEEE FP64 (Sec. 3.1)
U64 = 2.0 ** -53
#: unit roundoff of IEEE FP32 (mixed form only)
U32 = 2.0 ** -24

OK = 0
NOT_CONVERGED = 1
BREAKDOWN = 2
ENONFINITE = 3


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------
def gram(Q: np.ndarray) -> np.ndarray:
    """X = Q^T Q (Algorithm 1, Gram steps).  Upper triangle, mirrored."""
    X = Q.T @ Q
    return np.triu(X) + np.triu(X, 1).T


def gram_fp32(Q: np.ndarray) -> np.ndarray:
    """Q^T Q of the FP32-rounded Q with FP32 accumulation, returned in FP64
    (mixed form)."""
    Q32 = np.asarray(Q, dtype=np.float64).astype(np.float32)
    G = Q32.T @ Q32
    G = np.triu(G) + np.triu(G, 1).T
    return G.astype(np.float64)


def shift_fp32(n: int, xnorm: float) -> float:
    """Shift of a pass driven by an FP32 Gramian: max(n u32 ||X||, 2 u32)."""
    return max(n * U32 * xnorm, 2.0 * U32)


def gram_append(Q_in: np.ndarray, W: np.ndarray):
    """B~ = Q_in^T W and G = W^T W (Algorithm 2, Gram steps; Prop. 2.1)."""
    Bt = Q_in.T @ W
    return Bt, gram(W)


def schur(G: np.ndarray, Bt: np.ndarray) -> np.ndarray:
    """X = W^T W - B~^T B~ (Prop. 2.1, the Pythagorean form of the Gramian)."""
    return G - Bt.T @ Bt


def fro_dist_identity(X: np.ndarray) -> float:
    """||X - I||_F, the stopping quantity of Algorithms 1 and 2."""
    return float(np.linalg.norm(X - np.eye(X.shape[0]), "fro"))


def lambda_max(X: np.ndarray, steps: int = 30) -> float:
    """Estimate ||X||_2 of a symmetric X by power iteration from v0 = ones.

    Appendix A asks only for a rough largest-magnitude eigenvalue (IRLM with
    k=1, tol=1e-2, start vector of ones).  Plain power iteration from the same
    start vector, followed by the magnitude of the Rayleigh quotient.
    """
    n = X.shape[0]
    v = np.ones(n) / math.sqrt(n)
    for _ in range(steps):
        w = X @ v
        nrm = float(np.linalg.norm(w))
        if not (nrm > 0.0) or not math.isfinite(nrm):
            return nrm if math.isfinite(nrm) else float("nan")
        v = w / nrm
    return abs(float(v @ (X @ v)))


def shift_orth(m: int, n: int, xnorm: float, u: float = U64) -> float:
    """sigma = max{11 (m n + n (n+1)) u ||X||, 2u} (Algorithm 1, shift step)."""
    return max(11.0 * float(m * n + n * (n + 1)) * u * xnorm, 2.0 * u)


def shift_append_first(m: int, q: int, xnorm: float, u: float = U64) -> float:
    """First shift of Algorithm 2: 11 (m q + q (q+1)) u ||X||, floored at 2u.

    Algorithm 2 uses q, the width of the existing basis, in this formula (the
    append driver's option append_shift_dim substitutes p or q + p).
    """
    return max(11.0 * float(m * q + q * (q + 1)) * u * xnorm, 2.0 * u)


def cholesky_upper(M: np.ndarray):
    """Upper-triangular R with R^T R = M, row by row.

    Returns (R, ok).  ok is False on breakdown: some pivot
    d_j = m_jj - sum_{k<j} r_kj^2 is not > 0 or is not finite.
    """
    n = M.shape[0]
    R = np.zeros_like(M)
    for j in range(n):
        d = M[j, j] - R[:j, j] @ R[:j, j]
        if not (d > 0.0) or not math.isfinite(d):
            return R, False
        r = math.sqrt(d)
        R[j, j] = r
        R[j, j + 1:] = (M[j, j + 1:] - R[:j, j] @ R[:j, j + 1:]) / r
    return R, True


def apply_inverse(T: np.ndarray, Rt: np.ndarray) -> np.ndarray:
    """Y = T Rt^{-1} by forward substitution on every row (Algorithm 1, the
    Q <- Q R~^{-1} step; Algorithm 2, the Q <- (Q - Q_in B~) R~^{-1} step).

    y_j = (t_j - sum_{k<j} y_k r~_kj) / r~_jj, with a true division.
    """
    p = T.shape[1]
    Y = np.empty_like(T)
    for j in range(p):
        Y[:, j] = (T[:, j] - Y[:, :j] @ Rt[:j, j]) / Rt[j, j]
    return Y


def _chol_with_escalation(X: np.ndarray, sigma0: float, u: float,
                          max_escalations: int, tries: list | None = None):
    """chol(X + sigma I) from sigma = max(sigma0, 2u); after each breakdown
    sigma <- max(10 sigma, 2u) (Algorithm 2, inner loop), at most
    max_escalations times.

    Returns (R~, sigma, attempts, ok); every shift tried is appended to
    `tries` when given."""
    n = X.shape[0]
    sigma = max(sigma0, 2.0 * u)
    attempts = 0
    while True:
        attempts += 1
        if tries is not None:
            tries.append(sigma)
        Rt, ok = cholesky_upper(X + sigma * np.eye(n))
        if ok:
            return Rt, sigma, attempts, True
        if attempts > max_escalations:
            return Rt, sigma, attempts, False
        sigma = max(10.0 * sigma, 2.0 * u)


# --------------------------------------------------------------------------
# drivers
# --------------------------------------------------------------------------
#: shift policies of the orth driver (option ``shift_policy``)
RECOMPUTE = 0   # Algorithm 1 (rsCholQR): recompute sigma from the current X
NO_SHIFT = 1    # CholQR / CholQR2 (and shiftedCholeskyQR3 after its first pass)
FIXED = 2       # isCholQR: sigma from the input Gramian, reapplied


def default_opts(**kw) -> dict:
    """Options of the drivers; defaults give CholQR3 (a shifted first pass,
    then CholeskyQR2, then Algorithm 1's continuation)."""
    opts = dict(first_pass_shift=1, min_passes=3, max_iter=10, tol=1e-13,
                unit_roundoff=U64, max_escalations=32, power_steps=30, precision=0,
                shift_policy=RECOMPUTE, append_shift_dim=0)
    opts.update(kw)
    return opts


#: option sets of the Cholesky QR variants compared in Sec. 3.2 (Fig. 1)
VARIANTS = {
    # one pass, no shift: a breakdown ends the call
    "CholQR": dict(first_pass_shift=0, min_passes=1, max_iter=1, shift_policy=NO_SHIFT),
    # two plain passes
    "CholQR2": dict(first_pass_shift=0, min_passes=2, max_iter=2, shift_policy=NO_SHIFT),
    # a shifted pass followed by two plain ones, nothing more
    "sCholQR3": dict(first_pass_shift=1, min_passes=3, max_iter=3, shift_policy=NO_SHIFT),
    # plain passes until the test holds, the shift from ||A||^2 on a breakdown
    "isCholQR": dict(first_pass_shift=0, min_passes=0, max_iter=10, shift_policy=FIXED),
    # Algorithm 1 as printed
    "rsCholQR": dict(first_pass_shift=0, min_passes=0, max_iter=10, shift_policy=RECOMPUTE),
    # the shifted pass, CholeskyQR2, then Algorithm 1's test and continuation
    "CholQR3": dict(first_pass_shift=1, min_passes=3, max_iter=10, shift_policy=RECOMPUTE),
}


def orth(A: np.ndarray, **kw):
    """Shifted Cholesky QR of a tall matrix A (m x n), out of place.

    Algorithm 1 (rsCholQR) with the CholQR3 start: pass 1 is shifted when
    ``first_pass_shift`` is set, the stopping test is skipped until
    ``min_passes`` passes are done, and every other pass shifts only when the
    plain Cholesky factorisation of the current Gramian breaks down, with the
    shift recomputed from the current Gramian (Algorithm 1, shift step).

    ``shift_policy`` selects the other variants of Sec. 3.1 (see VARIANTS):
    NO_SHIFT ends the call on a breakdown (and a shifted first pass does not
    escalate); FIXED computes sigma = max{11 (mn + n(n+1)) u ||X_0||, 2u} once
    from the input Gramian X_0 = A^T A (||X_0|| = ||A||^2) and factors
    X + sigma I with it whenever the plain factorisation breaks down, ending
    the call if that fails too.

    Returns (Q, R, info) with info = dict(status, passes, sigma, chol_attempts,
    orth_fro).  ``first_pass_shift=0, min_passes=0`` is Algorithm 1 as printed.
    """
    o = default_opts(**kw)
    u = o["unit_roundoff"]
    policy = int(o["shift_policy"])
    if policy not in (RECOMPUTE, NO_SHIFT, FIXED):
        raise ValueError("shift_policy")
    if policy != RECOMPUTE and int(o["precision"]) != 0:
        raise ValueError("the variants of shift_policy run in FP64 only")
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    Q = A.copy()
    R = np.eye(n)
    g32 = int(o["precision"]) == 1      # the Gramian at hand is an FP32 one
    X = gram_fp32(Q) if g32 else gram(Q)
    info = dict(status=OK, passes=0, sigma=[], chol_attempts=0, orth_fro=None,
                fp32_grams=int(g32), shift_tries=[])
    sigma_fixed = None
    if policy == FIXED:
        sigma_fixed = shift_orth(m, n, lambda_max(X, o["power_steps"]), u)
    passes = 0
    while True:
        err = fro_dist_identity(X)
        info["orth_fro"] = err
        if not math.isfinite(err):
            info["status"] = ENONFINITE
            break
        if not g32 and passes >= o["min_passes"] and err < o["tol"]:
            break
        if passes >= o["max_iter"]:
            info["status"] = NOT_CONVERGED
            break
        passes += 1
        shifted = passes == 1 and bool(o["first_pass_shift"])
        sigma = 0.0
        ok = True
        if not shifted:
            info["chol_attempts"] += 1
            Rt, ok = cholesky_upper(X)
            shifted = not ok and policy != NO_SHIFT
        if shifted and policy == FIXED:
            sigma = sigma_fixed
            info["shift_tries"].append(sigma)
            info["chol_attempts"] += 1
            Rt, ok = cholesky_upper(X + sigma * np.eye(n))
        elif shifted:
            lam = lambda_max(X, o["power_steps"])
            esc = o["max_escalations"] if policy == RECOMPUTE else 0
            if g32:
                Rt, sigma, att, ok = _chol_with_escalation(X, shift_fp32(n, lam), U32, esc,
                                                           info["shift_tries"])
            else:
                Rt, sigma, att, ok = _chol_with_escalation(X, shift_orth(m, n, lam, u), u, esc,
                                                           info["shift_tries"])
            info["chol_attempts"] += att
        if not ok:
            info["status"] = BREAKDOWN
            break
        info["sigma"].append(sigma)
        Q = apply_inverse(Q, Rt)
        R = Rt @ R
        g32 = g32 and shifted           # FP32 Gramians end after an unshifted pass
        info["fp32_grams"] += int(g32)
        X = gram_fp32(Q) if g32 else gram(Q)
    info["passes"] = passes
    return Q, R, info


def append(Q_in: np.ndarray, R_in: np.ndarray, A_in: np.ndarray, **kw):
    """Algorithm 2 (cholQRUpdate): extend Q_in R_in = A_prev by columns A_in.

    Returns (Q_out, R_out, info); Q_out = [Q_in, Q], R_out = [[R_in, B],[0, R]]
    (Prop. 2.1).  The loop tests only the Schur complement X of the new block.

    Reading: the stopping test is consulted only after the first pass.  Prop.
    2.1 forms the new columns by the projection (A_in - Q_in Q_in^T A_in) R^-1;
    the initial X can equal I while Q_in^T A_in is not zero (A_in = Q_in C + H
    with H orthonormal and orthogonal to Q_in gives X = I exactly), and the
    loop as printed would then return Q = A_in, which is not orthogonal to
    Q_in.  One pass always applies the projection.
    """
    o = default_opts(**kw)
    u = o["unit_roundoff"]
    Q_in = np.asarray(Q_in, dtype=np.float64)
    A_in = np.asarray(A_in, dtype=np.float64)
    m, q = Q_in.shape
    p = A_in.shape[1]
    Q = A_in.copy()
    B = np.zeros((q, p))
    R = np.eye(p)
    Bt, G = gram_append(Q_in, Q)
    X = schur(G, Bt)
    info = dict(status=OK, passes=0, sigma=[], chol_attempts=0, orth_fro=None,
                shift_tries=[])
    passes = 0
    while True:
        err = fro_dist_identity(X)
        info["orth_fro"] = err
        if not math.isfinite(err):
            info["status"] = ENONFINITE
            break
        if passes >= 1 and err < o["tol"]:
            break
        if passes >= o["max_iter"]:
            info["status"] = NOT_CONVERGED
            break
        passes += 1
        sigma = 0.0
        info["chol_attempts"] += 1
        Rt, ok = cholesky_upper(X)
        if not ok:
            lam = lambda_max(X, o["power_steps"])
            d = (q, p, q + p)[int(o["append_shift_dim"])]
            sigma0 = shift_append_first(m, d, lam, u)
            Rt, sigma, att, ok = _chol_with_escalation(X, sigma0, u,
                                                       o["max_escalations"],
                                                       info["shift_tries"])
            info["chol_attempts"] += att
            if not ok:
                info["status"] = BREAKDOWN
                break
        info["sigma"].append(sigma)
        Q = apply_inverse(Q - Q_in @ Bt, Rt)
        B = B + Bt @ R
        R = Rt @ R
        Bt, G = gram_append(Q_in, Q)
        X = schur(G, Bt)
    info["passes"] = passes
    Q_out = np.concatenate([Q_in, Q], axis=1)
    R_out = np.zeros((q + p, q + p))
    R_out[:q, :q] = R_in
    R_out[:q, q:] = B
    R_out[q:, q:] = R
    return Q_out, R_out, info


def panel(A: np.ndarray, r: int, **kw):
    """Algorithm 3 (pnCholQR): split A into r panels of (nearly) equal width
    and apply Algorithm 2 to each in turn, starting from an empty basis."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    edges = np.linspace(0, n, r + 1).round().astype(int)
    Q = np.zeros((m, 0))
    R = np.zeros((0, 0))
    infos = []
    for i in range(r):
        Q, R, info = append(Q, R, A[:, edges[i]:edges[i + 1]], **kw)
        infos.append(info)
        if info["status"] != OK:
            break
    return Q, R, infos


# --------------------------------------------------------------------------
# accuracy metrics (Sec. 3.1), Frobenius norms
# --------------------------------------------------------------------------
def loo(Q: np.ndarray) -> float:
    """Loss of orthogonality ||I - Q^T Q||_F."""
    return fro_dist_identity(gram(Q))


def rrr(A: np.ndarray, Q: np.ndarray, R: np.ndarray) -> float:
    """Relative reconstruction residual ||A - Q R||_F / ||A||_F."""
    return float(np.linalg.norm(A - Q @ R) / np.linalg.norm(A))


def rcr(A: np.ndarray, R: np.ndarray) -> float:
    """Relative Cholesky residual ||A^T A - R^T R||_F / ||A||_F^2."""
    return float(np.linalg.norm(A.T @ A - R.T @ R) / np.linalg.norm(A) ** 2)
