"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: exact
closed forms (Hadamard constructions), brute force on tiny integer inputs,
LAPACK / library special cases (Householder QR, potrf, trsm, eigvalsh), the
invariants of Prop. 2.1 and the behaviour the paper reports.  The last group
plants plausible mistakes in the oracle and checks that a pin catches each.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import cholqr as O
import synth as S

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                     "paper_claims.json")))
U = 2.0 ** -53


def _householder_R(A):
    """LAPACK Householder R with a positive diagonal (unique for full rank)."""
    _, Rh = np.linalg.qr(A)
    return np.sign(np.diag(Rh))[:, None] * Rh


def _int_upper(g, n, lo=-3, hi=4, diag_pow=(0, 3)):
    """Integer upper-triangular T with power-of-two diagonal."""
    T = np.triu(g.integers(lo, hi, size=(n, n)).astype(np.float64), 1)
    T += np.diag(2.0 ** g.integers(diag_pow[0], diag_pow[1] + 1, size=n))
    return T


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------
def test_gram_bruteforce_integers():
    g = np.random.default_rng(1)
    A = g.integers(-9, 10, size=(37, 6)).astype(np.float64)
    X = O.gram(A)
    for j in range(6):
        for k in range(6):
            exact = sum(int(A[i, j]) * int(A[i, k]) for i in range(37))
            assert X[j, k] == exact


def test_gram_hadamard_exact():
    H = S.hadamard(256)[:, :40]
    assert np.array_equal(O.gram(H), 256.0 * np.eye(40))


def test_gram_append_and_schur_bruteforce():
    g = np.random.default_rng(2)
    Qi = g.integers(-4, 5, size=(23, 5)).astype(np.float64)
    W = g.integers(-4, 5, size=(23, 3)).astype(np.float64)
    Bt, G = O.gram_append(Qi, W)
    X = O.schur(G, Bt)
    for a in range(3):
        for b in range(3):
            gab = sum(int(W[i, a]) * int(W[i, b]) for i in range(23))
            bb = sum(sum(int(Qi[i, c]) * int(W[i, a]) for i in range(23)) *
                     sum(int(Qi[i, c]) * int(W[i, b]) for i in range(23))
                     for c in range(5))
            assert G[a, b] == gab
            assert X[a, b] == gab - bb
    for c in range(5):
        for a in range(3):
            assert Bt[c, a] == sum(int(Qi[i, c]) * int(W[i, a])
                                   for i in range(23))


def test_cholesky_exact_integer_factor():
    g = np.random.default_rng(3)
    for n in (1, 2, 5, 12):
        T = _int_upper(g, n)
        R, ok = O.cholesky_upper(T.T @ T)
        assert ok
        assert np.array_equal(R, T)


def test_cholesky_matches_lapack_potrf():
    g = np.random.default_rng(4)
    for n in (3, 17, 64):
        B = g.standard_normal((3 * n, n))
        M = B.T @ B
        R, ok = O.cholesky_upper(M)
        assert ok
        L = np.linalg.cholesky(M)
        assert np.linalg.norm(R - L.T) <= 1e-13 * np.linalg.norm(L)
        assert np.allclose(np.tril(R, -1), 0.0)


@pytest.mark.parametrize("M", [
    np.ones((2, 2)) + np.array([[0.0, 0.0], [0.0, 0.0]]),  # pivot exactly 0
    np.array([[1.0, 2.0], [2.0, 1.0]]),                     # indefinite
    np.array([[-1.0]]),                                     # negative pivot
    np.zeros((3, 3)),                                       # zero matrix
    np.array([[1.0, np.nan], [np.nan, 1.0]]),               # NaN off-diagonal
    np.array([[np.inf, 0.0], [0.0, 1.0]]),                  # Inf pivot
    np.array([[4.0, np.inf], [np.inf, 4.0]]),               # Inf off-diagonal
])
def test_cholesky_breakdown(M):
    _, ok = O.cholesky_upper(M)
    assert not ok


def test_apply_inverse_exact():
    g = np.random.default_rng(5)
    T = _int_upper(g, 9)
    Y = g.integers(-20, 21, size=(50, 9)).astype(np.float64)
    assert np.array_equal(O.apply_inverse(Y @ T, T), Y)


def test_apply_inverse_matches_trsm():
    g = np.random.default_rng(6)
    R = np.triu(g.standard_normal((20, 20))) + 5 * np.eye(20)
    T = g.standard_normal((300, 20))
    ref = scipy.linalg.solve_triangular(R, T.T, trans="T", lower=False).T
    assert np.linalg.norm(O.apply_inverse(T, R) - ref) <= 1e-13 * np.linalg.norm(ref)


def test_lambda_max_exact_cases():
    # c I: every start vector is an eigenvector; equal up to normalisation
    # rounding (a few ulps)
    assert abs(O.lambda_max(3.5 * np.eye(7)) - 3.5) <= 4 * U * 3.5
    v = np.arange(1.0, 9.0)
    lam = O.lambda_max(np.outer(v, v))
    assert abs(lam - v @ v) <= 4 * U * (v @ v)
    assert O.lambda_max(np.zeros((4, 4))) == 0.0


def test_lambda_max_within_irlm_tolerance():
    # Appendix A: the shift needs |lambda_max| only to tol 1e-2.  Gramians of
    # the paper's test matrices (log-spaced singular values).
    for n, kappa in ((5, 1e2), (20, 1e6), (100, 1e12), (256, 1e15)):
        A = S.test_matrix(2 * n + 50, n, kappa, seed=(7,))
        X = A.T @ A
        ref = np.linalg.eigvalsh(X)[-1]
        assert abs(O.lambda_max(X) - ref) <= 1e-2 * ref


def test_lambda_max_is_lower_bound_on_clustered_spectrum():
    # A Rayleigh quotient never exceeds lambda_max; with a clustered top of
    # the spectrum (Wishart) 30 steps still land within 10 %.
    g = np.random.default_rng(7)
    for n in (5, 20, 100):
        B = g.standard_normal((2 * n, n))
        X = B.T @ B
        ref = np.linalg.eigvalsh(X)[-1]
        est = O.lambda_max(X)
        assert 0.9 * ref <= est <= ref * (1 + 1e-13)


def _lambda_by_squaring(X, steps=30):
    """The device's evaluation of the same estimate: the first step X 1
    explicitly (X 1 = 0 ends it with 0), then X^(steps-1) from powers X^(2^k)
    (each scaled to unit Frobenius norm), then the Rayleigh quotient."""
    v = X @ np.ones(X.shape[0])
    n1 = np.linalg.norm(v)
    if not (n1 > 0) or not np.isfinite(n1):
        return 0.0 if np.isfinite(n1) else float("nan")
    v, P, rest, k = v / n1, X / np.linalg.norm(X), steps - 1, 0
    while rest >> k:
        if (rest >> k) & 1:
            v = P @ v
        if rest >> (k + 1):
            P = P @ P
            P = P / np.linalg.norm(P)
        k += 1
    nv = np.linalg.norm(v)
    if not (nv > 0) or not np.isfinite(nv):
        return 0.0 if np.isfinite(nv) else float("nan")
    v = v / nv
    return abs(float(v @ (X @ v)))


def test_power_iteration_by_squaring_is_the_same_estimate():
    # The 30 normalised steps from the ones vector give X^30 1 / ||X^30 1||;
    # forming X^30 from X^2, X^4, X^8, X^16 changes rounding only.  Also the
    # degenerate cases: X = 0, and 1 in the null space of X (both give 0).
    g = np.random.default_rng(17)
    cases = []
    for n, kappa in ((5, 1e2), (16, 1e8), (20, 1e6), (64, 1e12), (100, 1e15)):
        A = S.test_matrix(2 * n + 50, n, kappa, seed=(8,))
        cases.append(A.T @ A)
    for n in (7, 33):
        B = g.standard_normal((2 * n, n))
        cases.append(B.T @ B * 1e6)
    for X in cases:
        for steps in (30, 1, 7):
            ref = O.lambda_max(X, steps)
            assert abs(_lambda_by_squaring(X, steps) - ref) <= 1e-12 * ref
    assert _lambda_by_squaring(np.zeros((6, 6))) == O.lambda_max(np.zeros((6, 6))) == 0.0
    C = np.eye(4) - np.ones((4, 4)) / 4.0        # C 1 = 0 exactly
    assert O.lambda_max(C) == 0.0 and _lambda_by_squaring(C) == 0.0


def test_shift_formulas_exact():
    # 11 (m n + n (n+1)) with m=1000, n=20 is 11 * 20420 = 224620; with
    # ||X|| = 1 the shift is that integer times 2^-53, exactly.
    assert O.shift_orth(1000, 20, 1.0) == math.ldexp(224620, -53)
    # ||X|| = 4 scales by a power of two, exactly.
    assert O.shift_orth(1000, 20, 4.0) == math.ldexp(224620, -51)
    # floor 2u (Algorithm 1 shift step) when ||X|| = 0
    assert O.shift_orth(1000, 20, 0.0) == 2 * U
    # Algorithm 2 uses q: m=500, q=7 gives 11 (3500 + 56) = 39116.
    assert O.shift_append_first(500, 7, 1.0) == math.ldexp(39116, -53)
    # empty basis (q = 0): the formula gives 0, the floor gives 2u
    assert O.shift_append_first(500, 0, 123.0) == 2 * U
    assert GOLDEN["shift_constant"]["value"] == 11


def test_metrics_exact():
    H = S.hadamard(64)[:, :8]
    Q = H / 8.0
    assert O.loo(Q) == 0.0
    R = 8.0 * np.eye(8)
    assert O.rrr(H, Q, R) == 0.0
    assert O.rcr(H, R) == 0.0


# --------------------------------------------------------------------------
# whole orth
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m,n,kappa", [(200, 5, 1.0), (1000, 16, 1e2),
                                       (2000, 32, 10.0), (64, 64, 1e2)])
def test_orth_matches_householder(m, n, kappa):
    A = S.test_matrix(m, n, kappa, seed=(10,))
    Q, R, info = O.orth(A)
    assert info["status"] == O.OK
    Rh = _householder_R(A)
    assert np.linalg.norm(R - Rh) <= 1e-12 * np.linalg.norm(Rh)
    assert np.allclose(np.tril(R, -1), 0.0)


@pytest.mark.parametrize("k,n", [(3, 8), (4, 16), (5, 32)])
def test_orth_hadamard_closed_form(k, n):
    """A = H T with H^T H = 4^k I: R = 2^k T and Q = H / 2^k, bit for bit."""
    m = 4 ** k
    H = S.hadamard(m)[:, :n]
    T = _int_upper(np.random.default_rng(k), n)
    A = H @ T
    for kw in (dict(first_pass_shift=0, min_passes=0),   # Algorithm 1 as printed
               dict(first_pass_shift=0, min_passes=3)):  # unshifted CholQR3
        Q, R, info = O.orth(A, **kw)
        assert info["status"] == O.OK
        assert np.array_equal(R, (2.0 ** k) * T)
        assert np.array_equal(Q, H / 2.0 ** k)
        assert info["orth_fro"] == 0.0
    _, _, info = O.orth(A, first_pass_shift=0, min_passes=0)
    assert info["passes"] == 1


@pytest.mark.parametrize("kappa", [1e2, 1e6, 1e10, 1e15])
def test_orth_invariants_kappa_sweep(kappa):
    A = S.test_matrix(3000, 16, kappa, seed=(11,))
    Q, R, info = O.orth(A)
    assert info["status"] == O.OK
    assert O.loo(Q) <= 1e-12
    assert O.rrr(A, Q, R) <= 1e-13
    assert O.rcr(A, R) <= GOLDEN["fig2_rcr_upper"]["value"]
    assert info["passes"] >= 3
    assert info["sigma"][0] > 0.0


def test_orth_first_pass_shift_value():
    # CholQR3's first pass uses the paper's shift of the input Gramian.
    A = S.test_matrix(5000, 12, 1e4, seed=(12,))
    _, _, info = O.orth(A)
    lam = np.linalg.eigvalsh(O.gram(A))[-1]
    sig = 11.0 * (5000 * 12 + 12 * 13) * U * lam
    assert abs(info["sigma"][0] - sig) <= 1e-2 * sig
    assert info["sigma"][1] == 0.0 and info["sigma"][2] == 0.0


def test_fig1_pattern_rscholqr_robust():
    """Algorithm 1 as printed reaches the paper's stopping tolerance for
    300 x 10 inputs up to kappa = 1e20, where the unshifted Gram breaks down."""
    m, n = GOLDEN["fig1_shape"]["m"], GOLDEN["fig1_shape"]["n"]
    tol = GOLDEN["stop_tol"]["value"]
    broke = []
    for e in range(0, 21, 2):
        A = S.test_matrix(m, n, 10.0 ** e, seed=(6,))
        Q, R, info = O.orth(A, first_pass_shift=0, min_passes=0)
        assert info["status"] == O.OK, e
        assert info["passes"] <= GOLDEN["max_iter"]["value"]
        assert O.loo(Q) <= tol
        assert O.rrr(A, Q, R) <= GOLDEN["fig2_rrr_upper"]["value"]
        _, ok = O.cholesky_upper(O.gram(A))
        broke.append(not ok)
        if 10.0 ** e <= 1e4:
            assert not broke[-1]
    assert all(broke[6:])  # kappa >= 1e12: plain CholQR cannot even start


def test_orth_nonfinite_and_not_converged():
    A = S.test_matrix(400, 6, 1e2, seed=(13,))
    A[17, 3] = np.nan
    _, _, info = O.orth(A)
    assert info["status"] == O.ENONFINITE
    A = S.test_matrix(400, 6, 1e12, seed=(13,))
    _, _, info = O.orth(A, max_iter=1, min_passes=0)
    assert info["status"] == O.NOT_CONVERGED
    assert info["passes"] == 1


def test_orth_zero_column_not_converged():
    # An exactly dependent column keeps a zero eigenvalue in every Gramian.
    A = S.test_matrix(400, 6, 1e2, seed=(14,))
    A[:, 2] = 0.0
    _, _, info = O.orth(A)
    assert info["status"] == O.NOT_CONVERGED
    assert info["passes"] == 10


# --------------------------------------------------------------------------
# whole append (Prop. 2.1, Algorithm 2) and panel scheme (Algorithm 3)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("k,q,p", [(3, 8, 4), (4, 20, 10), (5, 60, 16)])
def test_append_hadamard_closed_form(k, q, p):
    """Q_in = H_q/2^k, W = H_p T + H_q C: B = 2^k C, R = 2^k T, Q = H_p/2^k."""
    m = 4 ** k
    H = S.hadamard(m)
    Hq, Hp = H[:, :q], H[:, q:q + p]
    g = np.random.default_rng(100 + k)
    T = _int_upper(g, p)
    C = g.integers(-3, 4, size=(q, p)).astype(np.float64)
    Rin = _int_upper(g, q)
    W = Hp @ T + Hq @ C
    Qo, Ro, info = O.append(Hq / 2.0 ** k, Rin, W)
    assert info["status"] == O.OK and info["passes"] == 1
    assert info["sigma"] == [0.0]
    assert np.array_equal(Qo[:, :q], Hq / 2.0 ** k)
    assert np.array_equal(Qo[:, q:], Hp / 2.0 ** k)
    assert np.array_equal(Ro[:q, :q], Rin)
    assert np.array_equal(Ro[:q, q:], (2.0 ** k) * C)
    assert np.array_equal(Ro[q:, q:], (2.0 ** k) * T)
    assert np.array_equal(Ro[q:, :q], np.zeros((p, q)))


def test_append_orthogonal_block_has_zero_B():
    # Columns orthogonal to Q_in: B = Q_in^T A_in = 0 and X_jj = c_j^T c_j.
    m, q, p = 256, 12, 5
    H = S.hadamard(m)
    W = H[:, q:q + p] * np.arange(1.0, p + 1)
    Bt, G = O.gram_append(H[:, :q] / 16.0, W)
    X = O.schur(G, Bt)
    assert np.array_equal(np.diag(X), (W * W).sum(0))
    _, Ro, info = O.append(H[:, :q] / 16.0, np.eye(q), W)
    assert info["status"] == O.OK
    assert np.array_equal(Ro[:q, q:], np.zeros((q, p)))


def test_append_lucky_breakdown():
    """W = Q_in b: X = 0 exactly, the shift is the 2u floor, the new block
    stays zero and the update never converges."""
    m, q, p = 256, 10, 3
    Qin = S.hadamard(m)[:, :q] / 16.0
    b = np.random.default_rng(9).integers(-3, 4, size=(q, p)).astype(float)
    W = (16.0 * Qin) @ b
    Bt, G = O.gram_append(Qin, W)
    assert np.array_equal(O.schur(G, Bt), np.zeros((p, p)))
    Qo, Ro, info = O.append(Qin, np.eye(q), W)
    assert info["status"] == O.NOT_CONVERGED
    assert info["sigma"][0] == 2 * U
    assert np.array_equal(Qo[:, q:], np.zeros((m, p)))


@pytest.mark.parametrize("kappa", [1e2, 1e8, 1e12])
def test_append_prop21_identities(kappa):
    A1 = S.test_matrix(4000, 12, 1e2, seed=(20,))
    A2 = S.test_matrix(4000, 8, kappa, seed=(21,))
    Q1, R1, _ = O.orth(A1)
    Qo, Ro, info = O.append(Q1, R1, A2)
    assert info["status"] == O.OK
    Qn = Qo[:, 12:]
    assert np.linalg.norm(Q1.T @ Qn) <= 1e-13
    assert O.loo(Qn) <= 1e-13
    assert O.loo(Qo) <= 1e-12
    A = np.concatenate([A1, A2], axis=1)
    assert O.rrr(A, Qo, Ro) <= 1e-13


def test_append_equals_householder_of_concatenation():
    A1 = S.test_matrix(3000, 10, 10.0, seed=(22,))
    A2 = S.test_matrix(3000, 7, 1e2, seed=(23,))
    Q1, R1, _ = O.orth(A1)
    _, Ro, _ = O.append(Q1, R1, A2)
    Rh = _householder_R(np.concatenate([A1, A2], axis=1))
    assert np.linalg.norm(Ro - Rh) <= 1e-12 * np.linalg.norm(Rh)


@pytest.mark.parametrize("r", [1, 2, 3, 5])
def test_panel_scheme_matches_householder(r):
    A = S.test_matrix(2000, 30, 1e2, seed=(24,))
    Q, R, infos = O.panel(A, r)
    assert all(i["status"] == O.OK for i in infos)
    Rh = _householder_R(A)
    assert np.linalg.norm(R - Rh) <= 1e-12 * np.linalg.norm(Rh)
    assert O.loo(Q) <= 1e-12


@pytest.mark.parametrize("r", [1, 2, 3, 5, 37])
def test_panel_scheme_hadamard_closed_form(r):
    """Algorithm 3 on A = H T (H Hadamard columns, T a small integer upper
    triangle): every panel's Gram, Schur complement and factor are exact, so
    R = 2^k T and Q = H / 2^k bit for bit, one pass per panel, whatever r
    (the first panel is Algorithm 2 on an empty basis)."""
    k, n = 5, 37
    H = S.hadamard(4 ** k)[:, :n]
    g = np.random.default_rng(5)
    T = np.triu(g.integers(-1, 2, size=(n, n)).astype(np.float64), 1) + np.diag(2.0 ** g.integers(0, 3, size=n))
    Q, R, infos = O.panel(H @ T, r)
    assert len(infos) == r and all(i["status"] == O.OK and i["passes"] == 1 for i in infos)
    assert np.array_equal(R, 2.0 ** k * T)
    assert np.array_equal(Q, H / 2.0 ** k)


def test_panel_scheme_ill_conditioned():
    A = S.test_matrix(2000, 20, 1e15, seed=(25,))
    Q, R, infos = O.panel(A, 4)
    assert all(i["status"] == O.OK for i in infos)
    assert O.loo(Q) <= 1e-12
    assert O.rrr(A, Q, R) <= 1e-13


def test_growth_run_small():
    A0, Ws, _ = S.growth_blocks(5000, 10, 10, 6, 1e2, 1e12)
    Q, R, info = O.orth(A0)
    assert info["status"] == O.OK
    for W in Ws:
        Q, R, info = O.append(Q, R, W)
        assert info["status"] == O.OK
    A = np.concatenate([A0] + Ws, axis=1)
    assert O.loo(Q) <= 1e-12
    assert O.rrr(A, Q, R) <= 1e-13


# --------------------------------------------------------------------------
# shift escalation, its floor and cap (Algorithm 2, inner loop; read into
# Algorithm 1 for a shifted factorisation that still breaks down)
# --------------------------------------------------------------------------
def test_escalation_sequence_exact():
    """X = diag(1, -delta): chol(X + sigma I) succeeds exactly when
    sigma > delta, so the shifts tried are sigma0 f^k (f the paper's factor)
    up to the first one above delta."""
    f = GOLDEN["escalation_factor"]["value"]
    X = np.diag([1.0, -999.5])
    tries = []
    _, sig, att, ok = O._chol_with_escalation(X, 1.0, U, 32, tries)
    assert ok and att == 4 and sig == f ** 3
    assert tries == [1.0, f, f * f, f ** 3]
    tries = []
    _, sig, att, ok = O._chol_with_escalation(X, 0.3, U, 32, tries)
    want = [0.3]
    while want[-1] <= 999.5:
        want.append(want[-1] * f)
    assert ok and tries == want and att == 5 and sig == want[-1]


def test_escalation_cap():
    """max_escalations bounds the x10 steps: the call fails after 1 + cap
    attempts, and a cap of zero allows the first shifted attempt only."""
    X = np.diag([1.0, -999.5])
    tries = []
    _, _, att, ok = O._chol_with_escalation(X, 1.0, U, 2, tries)
    assert not ok and att == 3 and tries == [1.0, 10.0, 100.0]
    _, _, att, ok = O._chol_with_escalation(X, 1.0, U, 0)
    assert not ok and att == 1
    _, _, att, ok = O._chol_with_escalation(X, 1.0, U, 3)
    assert ok and att == 4


def test_escalation_floor():
    """The shift never starts below 2u (Algorithm 2, the max with 2u): a zero
    or tiny first estimate starts at 2u.  With X = diag(1, -5u) the tries are
    2u, 20u.  (The same max after a x10 step can never bind: every shift is
    already at least 2u, so ten times it is at least 20u.)"""
    X = np.diag([1.0, -5.0 * U])
    for s0 in (0.0, 1e-300, U):
        tries = []
        _, sig, att, ok = O._chol_with_escalation(X, s0, U, 32, tries)
        assert ok and att == 2 and tries == [2 * U, 20 * U] and sig == 20 * U


def _dup_hadamard(k=4):
    """[h1, h1, h2, h3] of a Sylvester Hadamard matrix of order 4^k: an exact
    integer Gramian with the zero pivot 256 - 16 * 16 = 0 in column 2."""
    H = S.hadamard(4 ** k)
    return np.stack([H[:, 1], H[:, 1], H[:, 2], H[:, 3]], axis=1)


def test_orth_breakdown_at_the_escalation_cap():
    """Algorithm 1 as printed on exactly dependent columns with u = 2^-80: the
    shifts sigma0 10^k stay below half an ulp of the Gramian's entries for
    k <= 3, so X + sigma I rounds to X and every factorisation meets the same
    exact zero pivot.  With a cap of c escalations the call ends with
    SQR_BREAKDOWN after 1 + (1 + c) factorisations; the shifts tried are
    sigma0, 10 sigma0, ... with sigma0 the Algorithm 1 shift of ||X||_2 = 512."""
    A = _dup_hadamard()
    m, n = A.shape
    u = 2.0 ** -80
    X = O.gram(A)
    assert X[0, 0] == X[0, 1] == X[1, 1] == 256.0
    sig0 = 11.0 * (m * n + n * (n + 1)) * u * 512.0
    for cap in (0, 1, 3):
        _, _, info = O.orth(A, first_pass_shift=0, min_passes=0, unit_roundoff=u,
                            max_escalations=cap)
        assert info["status"] == O.BREAKDOWN and info["passes"] == 1
        assert info["chol_attempts"] == 2 + cap
        assert len(info["shift_tries"]) == 1 + cap
        for k, s in enumerate(info["shift_tries"]):
            assert abs(s - sig0 * 10.0 ** k) <= 1e-12 * s
        # the shifted matrices really are X (sigma below half an ulp of 256)
        assert 256.0 + info["shift_tries"][-1] == 256.0
    # with the default cap the shift grows past the rounding level and the
    # factorisation succeeds
    _, _, info = O.orth(A, first_pass_shift=0, min_passes=0, unit_roundoff=u)
    assert info["status"] != O.BREAKDOWN


def test_append_breakdown_keeps_basis():
    """Two identical new columns orthogonal to Q_in: X = [[1, 1], [1, 1]]
    exactly, whose factorisation meets a zero pivot; with u = 2^-80 the shift
    stays below half an ulp of 1, so a cap of zero ends the call with
    SQR_BREAKDOWN after two factorisations, and Q_out/R_out are the input."""
    k, q = 4, 6
    H = S.hadamard(4 ** k)
    Qin = H[:, :q] / 2.0 ** k
    h = H[:, q] / 2.0 ** k
    W = np.stack([h, h], axis=1)
    for cap in (0, 2):
        Qo, Ro, info = O.append(Qin, np.eye(q), W, unit_roundoff=2.0 ** -80,
                                max_escalations=cap)
        assert info["status"] == O.BREAKDOWN and info["passes"] == 1
        assert info["chol_attempts"] == 2 + cap
        assert np.array_equal(Qo[:, :q], Qin)


def test_append_first_shift_dimension():
    """Algorithm 2's first shift 11 (m d + d (d+1)) u ||X|| with d = q as
    printed, or p, or q + p (option append_shift_dim).  The duplicated column
    pair above has ||X||_2 = 2, so each first shift is an integer times
    2^-52 (to the rounding of the power iteration's Rayleigh quotient)."""
    k, q = 4, 6
    m = 4 ** k
    H = S.hadamard(m)
    Qin = H[:, :q] / 2.0 ** k
    h = H[:, q] / 2.0 ** k
    W = np.stack([h, h], axis=1)
    for dim, d in ((0, q), (1, 2), (2, q + 2)):
        _, _, info = O.append(Qin, np.eye(q), W, append_shift_dim=dim)
        want = math.ldexp(11 * (m * d + d * (d + 1)), -52)
        assert abs(info["shift_tries"][0] - want) <= 8 * U * want


# --------------------------------------------------------------------------
# the stopping quantity and the metrics at exact non-zero values
# --------------------------------------------------------------------------
def test_fro_distance_exact_nonzero():
    # X - I = [[1, 2], [2, 4]]: squares sum to 25
    assert O.fro_dist_identity(np.array([[2.0, 2.0], [2.0, 5.0]])) == 5.0
    assert O.fro_dist_identity(np.diag([4.0, 1.0])) == 3.0
    assert O.fro_dist_identity(np.zeros((3, 3))) == math.sqrt(3.0)


def test_metrics_exact_nonzero():
    A = np.array([[6.0], [8.0]])
    Q = np.array([[1.0], [0.0]])
    R = np.array([[6.0]])
    assert O.rrr(A, Q, R) == 8.0 / 10.0              # ||[0, 8]|| / ||[6, 8]||
    assert O.rcr(A, R) == 64.0 / 100.0               # |100 - 36| / 10^2
    assert O.loo(np.array([[3.0, 0.0], [0.0, 2.0]])) == math.sqrt(64.0 + 9.0)


def test_stop_test_is_strict_on_the_frobenius_distance():
    """A = [2 h1, h2] / 8 (m = 64): X = diag(4, 1), ||X - I||_F = 3 exactly.
    With tol = 3.5 Algorithm 1 stops before any pass (Q = A, R = I); with
    tol = 3 the test ||X - I||_F < tol fails and one pass gives the exact QR
    R = diag(2, 1), Q = [h1, h2] / 8."""
    H = S.hadamard(64)
    A = np.stack([2.0 * H[:, 0], H[:, 1]], axis=1) / 8.0
    kw = dict(first_pass_shift=0, min_passes=0)
    Q, R, info = O.orth(A, tol=3.5, **kw)
    assert info["passes"] == 0 and info["orth_fro"] == 3.0 and info["status"] == O.OK
    assert np.array_equal(Q, A) and np.array_equal(R, np.eye(2))
    Q, R, info = O.orth(A, tol=3.0, **kw)
    assert info["passes"] == 1 and info["orth_fro"] == 0.0
    assert np.array_equal(R, np.diag([2.0, 1.0])) and np.array_equal(Q, H[:, :2] / 8.0)


def test_append_entry_case_projects_once():
    """A_in = Q_in C + H_p / 2^k with Q_in = H_q / 2^k: the initial Schur
    complement is I exactly although B~ = C is not zero.  Prop. 2.1's
    projection must still be applied: one pass gives Q = H_p / 2^k, B = C,
    R = I, all exact, and the full basis is orthonormal."""
    k, q, p = 4, 12, 5
    H = S.hadamard(4 ** k)
    Qin = H[:, :q] / 2.0 ** k
    C = np.random.default_rng(17).integers(-3, 4, size=(q, p)).astype(np.float64)
    W = Qin @ C + H[:, q:q + p] / 2.0 ** k
    Bt, G = O.gram_append(Qin, W)
    assert np.array_equal(Bt, C)
    assert np.array_equal(O.schur(G, Bt), np.eye(p))
    Qo, Ro, info = O.append(Qin, np.eye(q), W)
    assert info["status"] == O.OK and info["passes"] == 1
    assert np.array_equal(Qo[:, q:], H[:, q:q + p] / 2.0 ** k)
    assert np.array_equal(Ro[:q, q:], C)
    assert np.array_equal(Ro[q:, q:], np.eye(p))
    assert O.loo(Qo) == 0.0


# --------------------------------------------------------------------------
# the Cholesky QR variants of Sec. 3.1 and Fig. 1's robustness pattern
# --------------------------------------------------------------------------
def test_fig1_pattern_all_variants():
    """300 x 10 inputs, kappa = 10^0 .. 10^20 (Sec. 3.2): plain CholQR loses
    orthogonality as kappa^2 u and CholQR/CholQR2 cannot factor the Gramian
    above about 1/sqrt(u) (the paper: kappa >= 1e8); sCholQR3 holds for
    moderate kappa; Algorithm 1 (rsCholQR), isCholQR and CholQR3 reach the
    stopping tolerance up to kappa = 1e20."""
    m, n = GOLDEN["fig1_shape"]["m"], GOLDEN["fig1_shape"]["n"]
    tol = GOLDEN["stop_tol"]["value"]
    limit = GOLDEN["cholqr2_fails_above_kappa"]["value"]
    for e in range(0, 21):
        kappa = 10.0 ** e
        A = S.test_matrix(m, n, kappa, seed=(6,))
        res = {v: O.orth(A, **kw) for v, kw in O.VARIANTS.items()}
        loo = {v: O.loo(r[0]) for v, r in res.items()}
        st = {v: r[2]["status"] for v, r in res.items()}
        for v in ("rsCholQR", "isCholQR", "CholQR3"):
            assert st[v] == O.OK and loo[v] <= tol, (v, e)
        if kappa <= 1e12:
            assert st["sCholQR3"] == O.OK and loo["sCholQR3"] <= tol, e
        if kappa <= 1e7:
            assert st["CholQR2"] == O.OK and loo["CholQR2"] <= tol, e
        if kappa >= 100 * limit:
            assert st["CholQR"] == st["CholQR2"] == O.BREAKDOWN, e
        if 1e3 <= kappa <= 1e8:
            # one plain pass: LOO of the order kappa^2 u
            assert 1e-3 * kappa ** 2 * U <= loo["CholQR"] <= 1e3 * kappa ** 2 * U, e
        # a plain variant never shifts; CholQR2 makes exactly its two passes
        assert all(s == 0.0 for s in res["CholQR2"][2]["sigma"])
        if st["CholQR2"] == O.OK:
            assert res["CholQR2"][2]["passes"] == 2


def test_isCholQR_reuses_the_input_shift():
    """isCholQR computes sigma once from X_0 = A^T A and reapplies it on every
    breakdown: with A scaled by 2^20 (||X_0|| = 2^40) the shift on every
    shifted pass equals the one from the input Gramian."""
    A = S.test_matrix(300, 10, 1e16, seed=(6,)) * 2.0 ** 20
    _, _, info = O.orth(A, **O.VARIANTS["isCholQR"])
    lam = O.lambda_max(O.gram(A))
    want = O.shift_orth(300, 10, lam)
    shifted = [s for s in info["sigma"] if s > 0.0]
    assert shifted and all(s == want for s in shifted)
    assert info["shift_tries"] == shifted


# --------------------------------------------------------------------------
# planted mistakes: each plausible slip in the oracle must fail a pin above
# --------------------------------------------------------------------------
def _fails(pin, *args):
    try:
        pin(*args)
    except (AssertionError, ValueError, np.linalg.LinAlgError):
        return True
    return False


def test_planted_mistakes_are_caught(monkeypatch):
    import oracle.cholqr as C
    append_pin = lambda: test_append_hadamard_closed_form(4, 20, 10)
    orth_pin = lambda: test_orth_hadamard_closed_form(4, 16)
    hh_pin = lambda: test_orth_matches_householder(1000, 16, 1e2)
    shift_pin = test_orth_first_pass_shift_value
    for pin in (append_pin, orth_pin, hh_pin, shift_pin):
        assert not _fails(pin)
    mistakes = [
        # Schur complement without the B~^T B~ term
        ("schur", lambda G, Bt: G, append_pin),
        # wrong sign of that term
        ("schur", lambda G, Bt: G + Bt.T @ Bt, append_pin),
        # B~ taken as W^T Q_in (transposed operand)
        ("gram_append", lambda Qi, W: ((W.T @ Qi).T[::-1], C.gram(W)),
         append_pin),
        # transposed triangular factor in the apply
        ("apply_inverse", (lambda f: lambda T, Rt: f(T, Rt.T))(C.apply_inverse),
         orth_pin),
        # forgetting the division by the diagonal in the substitution
        ("apply_inverse", (lambda f: lambda T, Rt: f(T, Rt) * np.diag(Rt))(
            C.apply_inverse), orth_pin),
        # Gram of the rows instead of the columns (Q Q^T)
        ("gram", lambda Q: (Q @ Q.T)[:Q.shape[1], :Q.shape[1]], hh_pin),
        # ||X|| estimate off by a factor 100
        ("lambda_max", (lambda f: lambda X, steps=30: f(X, steps) / 100.0)(
            C.lambda_max), shift_pin),
        # shift formula with n instead of n(n+1)
        ("shift_orth", lambda m, n, x, u=U: max(11.0 * (m * n + n) * u * x,
                                                2 * u), test_shift_formulas_exact),
    ]
    for name, bad, pin in mistakes:
        with monkeypatch.context() as mp:
            mp.setattr(C, name, bad)
            assert _fails(pin), name
    # missing square root on the Cholesky pivot
    with monkeypatch.context() as mp:
        mp.setattr(C.math, "sqrt", lambda x: x)
        assert _fails(append_pin)


# ---------------------------------------------------------------------------
# mixed-precision form (precision=1): FP32 Gramians until the first unshifted
# pass, then FP64 (a reading taken here; the paper has no mixed form)
# ---------------------------------------------------------------------------
def test_shift_fp32_exact():
    assert O.shift_fp32(16, 1.0) == 16 * 2.0 ** -24
    assert O.shift_fp32(256, 0.5) == 128 * 2.0 ** -24
    assert O.shift_fp32(16, 0.0) == 2.0 ** -23          # floor 2 u32


def test_gram_fp32_rounds_the_iterate():
    # integer entries: FP32 rounding and accumulation are exact
    A = np.array([[1.0, 2.0], [3.0, -4.0], [5.0, 6.0]])
    assert np.array_equal(O.gram_fp32(A), A.T @ A)
    # 1 + 2^-30 is not an FP32 number: the FP32 Gramian sees 1
    B = np.array([[1.0 + 2.0 ** -30], [0.0]])
    assert O.gram_fp32(B)[0, 0] == 1.0
    assert O.gram(B)[0, 0] > 1.0


def test_mixed_orthonormal_input_needs_fp64_pass():
    # FP64 sees an orthonormal input and stops at once; an FP32 Gramian can
    # never stop the iteration, so the mixed form makes an unshifted pass on
    # it (an R~ accurate to FP32 only), one FP64 pass, and stops on the FP64
    # check Gramian.
    Q0 = S.orthonormal(S.rng(11), 5000, 12)
    _, _, i64 = O.orth(Q0, first_pass_shift=0, min_passes=0)
    assert i64["passes"] == 0
    _, _, im = O.orth(Q0, first_pass_shift=0, min_passes=0, precision=1)
    assert im["status"] == O.OK
    assert im["passes"] == 2 and im["fp32_grams"] == 1
    assert im["sigma"] == [0.0, 0.0]


@pytest.mark.parametrize("kappa", [1e4, 1e8, 1e12, 1e15])
def test_mixed_orth_is_the_qr(kappa):
    A = S.test_matrix(6000, 16, kappa, seed=(12,))
    Q, R, i64 = O.orth(A)
    Qm, Rm, im = O.orth(A, precision=1)
    assert im["status"] == O.OK
    assert O.loo(Qm) <= 1e-13 and O.rrr(A, Qm, Rm) <= 1e-14
    assert np.abs(Rm - R).max() <= 1e-10 * kappa * np.abs(R).max()
    # FP32 Gramians for every shifted pass and the first unshifted one, then
    # exactly one FP64 pass and the FP64 check
    assert im["fp32_grams"] == im["passes"] - 1
    assert im["passes"] >= i64["passes"]
    assert all(s > 0 for s in im["sigma"][:im["passes"] - 2])
    assert im["sigma"][im["passes"] - 1] == 0.0
    # ||A||_2 = 1 by construction, so the first FP32 shift is 16 u32 (to the
    # accuracy of the norm estimate) and no shifted factorisation escalates
    assert abs(im["sigma"][0] / (16 * 2.0 ** -24) - 1.0) < 1e-2
    nshift = sum(s > 0 for s in im["sigma"])
    assert im["chol_attempts"] == im["passes"] + nshift - 1


def test_planted_mixed_mistakes_are_caught(monkeypatch):
    import oracle.cholqr as C
    pin = test_mixed_orthonormal_input_needs_fp64_pass
    qr_pin = lambda: test_mixed_orth_is_the_qr(1e8)
    assert not _fails(pin) and not _fails(qr_pin)
    mistakes = [
        # FP64 Gramians throughout (the FP32 rounding left out)
        ("gram_fp32", C.gram, pin),
        # FP64 shift constant in the FP32 passes (shift far too small)
        ("shift_fp32", lambda n, x: max(n * C.U64 * x, 2 * C.U64), qr_pin),
    ]
    for name, bad, p in mistakes:
        with monkeypatch.context() as mp:
            mp.setattr(C, name, bad)
            assert _fails(p), name


# Source-level mutants of the oracle: each replaces one exact fragment of
# oracle/cholqr.py, is loaded as a separate module, and must fail the pin
# named beside it.  (Dropping the 2u floor after a x10 step is not among
# them: the shift already starts at or above 2u, so ten times it is at least
# 20u and that floor can never bind -- an equivalent mutant that no input can
# tell apart; the floor on the first shift is pinned by
# test_escalation_floor.)
_MUTANTS = [
    ("x2 escalation", "sigma = max(10.0 * sigma, 2.0 * u)",
     "sigma = max(2.0 * sigma, 2.0 * u)", "test_escalation_sequence_exact"),
    ("x100 escalation", "sigma = max(10.0 * sigma, 2.0 * u)",
     "sigma = max(100.0 * sigma, 2.0 * u)", "test_escalation_sequence_exact"),
    ("first shift not floored", "sigma = max(sigma0, 2.0 * u)", "sigma = sigma0",
     "test_escalation_floor"),
    ("cap raised by 5", "if attempts > max_escalations:", "if attempts > max_escalations + 5:",
     "test_escalation_cap"),
    ("cap raised by 5 (driver)", "if attempts > max_escalations:",
     "if attempts > max_escalations + 5:", "test_orth_breakdown_at_the_escalation_cap"),
    ("squared stopping distance",
     'return float(np.linalg.norm(X - np.eye(X.shape[0]), "fro"))',
     'return float(np.linalg.norm(X - np.eye(X.shape[0]), "fro")) ** 2',
     "test_stop_test_is_strict_on_the_frobenius_distance"),
    ("squared stopping distance (unit)",
     'return float(np.linalg.norm(X - np.eye(X.shape[0]), "fro"))',
     'return float(np.linalg.norm(X - np.eye(X.shape[0]), "fro")) ** 2',
     "test_fro_distance_exact_nonzero"),
    ("non-strict stopping test", 'passes >= o["min_passes"] and err < o["tol"]',
     'passes >= o["min_passes"] and err <= o["tol"]',
     "test_stop_test_is_strict_on_the_frobenius_distance"),
    ("squared RRR", "return float(np.linalg.norm(A - Q @ R) / np.linalg.norm(A))",
     "return float(np.linalg.norm(A - Q @ R) / np.linalg.norm(A)) ** 2",
     "test_metrics_exact_nonzero"),
    ("RCR over ||A||", "/ np.linalg.norm(A) ** 2)", "/ np.linalg.norm(A))",
     "test_metrics_exact_nonzero"),
    ("append stops before projecting", 'if passes >= 1 and err < o["tol"]:',
     'if err < o["tol"]:', "test_append_entry_case_projects_once"),
    ("append shift dimension ignored", 'd = (q, p, q + p)[int(o["append_shift_dim"])]',
     "d = q", "test_append_first_shift_dimension"),
    ("isCholQR recomputes its shift", "sigma = sigma_fixed",
     'sigma = shift_orth(m, n, lambda_max(X, o["power_steps"]), u)',
     "test_isCholQR_reuses_the_input_shift"),
    ("plain variants shift on breakdown", "shifted = not ok and policy != NO_SHIFT",
     "shifted = not ok", "test_fig1_pattern_all_variants"),
]


@pytest.mark.parametrize("name,old,new,pin", _MUTANTS, ids=[m[0] for m in _MUTANTS])
def test_source_mutant_is_caught(name, old, new, pin, monkeypatch):
    import types
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "oracle", "cholqr.py")
    src = open(path).read()
    assert src.count(old) == 1, name
    mod = types.ModuleType("oracle_mutant")
    exec(compile(src.replace(old, new), path, "exec"), mod.__dict__)
    pin_fn = globals()[pin]
    assert not _fails(pin_fn)                      # the pin holds on the oracle
    monkeypatch.setitem(globals(), "O", mod)
    assert _fails(pin_fn), name
