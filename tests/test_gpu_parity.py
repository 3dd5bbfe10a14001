"""GPU parity: libsqr (HIP, through the C ABI) against the FP64 oracle.

Tolerances (from the accuracy targets of the method and the arithmetic):
  * ||Q^T Q - I||_F <= 1e-12 and ||A - QR||_F / ||A||_F <= 1e-13;
  * R within 1e-10 * kappa (relative, Frobenius) of the oracle's R, element
    by element within 1e-10 * kappa * ||R||_F; Q the same relative to ||Q||_F.
    For kappa >= 1e12 the factors are not numerically unique in FP64, so only
    the invariants are graded there.
  * Exact closed forms (Hadamard constructions) must match bit for bit.
"""
import math

import numpy as np
import pytest
import torch

import synth as S
from oracle import cholqr as O

pytestmark = pytest.mark.gpu

import paper_2507_07788_amd as sq  # noqa: E402  (a missing library fails, not skips)
from gpu_util import dev, host  # noqa: E402


def _small_upper(g, n):
    """Integer upper triangle, entries in {-1,0,1}, diagonal in {1,2,4}: the
    inverses of its 16x16 diagonal blocks are exact dyadic numbers."""
    T = np.triu(g.integers(-1, 2, size=(n, n)).astype(np.float64), 1)
    T += np.diag(2.0 ** g.integers(0, 3, size=n))
    return T


def _check_factors(A, Qg, Rg, Qo, Ro, kappa):
    assert O.loo(Qg) <= 1e-12
    assert O.rrr(A, Qg, Rg) <= 1e-13
    assert np.array_equal(np.tril(Rg, -1), np.zeros_like(Rg))
    if kappa < 1e12:
        tolr = 1e-10 * kappa
        assert np.linalg.norm(Rg - Ro) <= tolr * np.linalg.norm(Ro)
        assert np.max(np.abs(Rg - Ro)) <= tolr * np.linalg.norm(Ro)
        assert np.linalg.norm(Qg - Qo) <= tolr * np.linalg.norm(Qo)
        assert np.max(np.abs(Qg - Qo)) <= tolr * np.linalg.norm(Qo)


# --------------------------------------------------------------------------
# exact closed forms
# --------------------------------------------------------------------------
@pytest.mark.parametrize("k,n", [(3, 8), (4, 16), (4, 20), (5, 37), (5, 64)])
@pytest.mark.parametrize("mode", ["alg1", "cholqr3_noshift"])
def test_orth_hadamard_bitwise(k, n, mode):
    m = 4 ** k
    H = S.hadamard(m)[:, :n]
    T = _small_upper(np.random.default_rng(k * 100 + n), n)
    A = H @ T
    kw = dict(first_pass_shift=0, min_passes=0 if mode == "alg1" else 3)
    Qo, Ro, io = O.orth(A, **kw)
    assert np.array_equal(Ro, 2.0 ** k * T)  # the oracle reaches the closed form
    b, info = sq.sqr_orth(dev(A), opts=sq.sqr_default_opts(**kw))
    assert info["status"] == 0 and info["passes"] == io["passes"]
    assert np.array_equal(host(b.r()), 2.0 ** k * T)
    assert np.array_equal(host(b.q()), H / 2.0 ** k)
    assert info["orth_fro"] == 0.0


@pytest.mark.parametrize("k,q,p", [(3, 8, 4), (4, 20, 10), (5, 60, 16), (5, 33, 40)])
def test_append_hadamard_bitwise(k, q, p):
    m = 4 ** k
    H = S.hadamard(m)
    g = np.random.default_rng(7 * k + q)
    Tq = _small_upper(g, q)
    T = _small_upper(g, p)
    C = g.integers(-3, 4, size=(q, p)).astype(np.float64)
    A0 = H[:, :q] @ Tq
    W = H[:, q:q + p] @ T + H[:, :q] @ C
    kw = dict(first_pass_shift=0, min_passes=0)
    b, info = sq.sqr_orth(dev(A0), cap=q + p, opts=sq.sqr_default_opts(**kw))
    assert info["status"] == 0
    info = sq.sqr_append(b, dev(W))
    assert info["status"] == 0 and info["passes"] == 1 and b.n == q + p
    Rg = host(b.r())
    assert np.array_equal(Rg[:q, :q], 2.0 ** k * Tq)
    assert np.array_equal(Rg[:q, q:], 2.0 ** k * C)
    assert np.array_equal(Rg[q:, q:], 2.0 ** k * T)
    assert np.array_equal(Rg[q:, :q], np.zeros((p, q)))
    assert np.array_equal(host(b.q()), H[:, :q + p] / 2.0 ** k)


# --------------------------------------------------------------------------
# orth parity against the oracle
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [5, 16, 20, 33, 64, 65, 100, 128, 129, 200])
def test_orth_first_shift_matches_oracle(n):
    """The first shift carries ||X||_2 from the device's power iteration (by
    squaring up to 64 columns, step by step above; X in LDS or in global
    memory): the same estimate as the oracle's 30 steps, to rounding."""
    A = S.test_matrix(4000, n, 1e8, seed=(60,))
    io = O.orth(A)[2]
    b, info = sq.sqr_orth(dev(A))
    assert info["status"] == 0
    assert abs(info["sigma"][0] - io["sigma"][0]) <= 1e-9 * io["sigma"][0]


def test_orth_parity_20000x20_kappa1e6():
    A = S.test_matrix(20000, 20, 1e6, seed=(1,))
    Qo, Ro, io = O.orth(A)
    b, info = sq.sqr_orth(dev(A))
    assert info["status"] == 0 and info["passes"] == io["passes"] == 3
    assert abs(info["sigma"][0] - io["sigma"][0]) <= 1e-2 * io["sigma"][0]
    _check_factors(A, host(b.q()), host(b.r()), Qo, Ro, 1e6)


@pytest.mark.parametrize("m,n", [(1000, 5), (4099, 16), (10007, 17), (5000, 33),
                                 (3001, 64), (2000, 100), (2500, 128), (4097, 113),
                                 (2600, 200), (3001, 256)])
@pytest.mark.parametrize("kappa", [1e2, 1e8, 1e12, 1e15])
def test_orth_parity_sweep(m, n, kappa):
    A = S.test_matrix(m, n, kappa, seed=(3,))
    Qo, Ro, io = O.orth(A)
    b, info = sq.sqr_orth(dev(A))
    assert info["status"] == 0
    assert abs(info["passes"] - io["passes"]) <= 1
    _check_factors(A, host(b.q()), host(b.r()), Qo, Ro, kappa)


@pytest.mark.parametrize("e", [0, 4, 8, 12, 16, 20])
def test_orth_algorithm1_literal_fig1_shape(e):
    A = S.test_matrix(300, 10, 10.0 ** e, seed=(6,))
    kw = dict(first_pass_shift=0, min_passes=0)
    Qo, Ro, io = O.orth(A, **kw)
    b, info = sq.sqr_orth(dev(A), opts=sq.sqr_default_opts(**kw))
    assert info["status"] == 0
    assert O.loo(host(b.q())) <= 1e-13
    assert O.rrr(A, host(b.q()), host(b.r())) <= 1e-13


@pytest.mark.parametrize("m,n", [(3000, 70), (2000, 100), (2100, 128), (2200, 160)])
def test_orth_breakdown_then_shift_wide(m, n):
    """Algorithm 1 as printed: the unshifted first factorisation of a kappa =
    1e15 Gramian breaks down and the shifted retry (power iteration, shift,
    factorisation) runs on the wide-block paths."""
    A = S.test_matrix(m, n, 1e15, seed=(9,))
    kw = dict(first_pass_shift=0, min_passes=0)
    Qo, Ro, io = O.orth(A, **kw)
    assert io["chol_attempts"] > io["passes"]          # the oracle broke down
    b, info = sq.sqr_orth(dev(A), opts=sq.sqr_default_opts(**kw))
    assert info["status"] == 0
    assert info["chol_attempts"] > info["passes"]
    assert abs(info["passes"] - io["passes"]) <= 1
    _check_factors(A, host(b.q()), host(b.r()), Qo, Ro, 1e15)


@pytest.mark.parametrize("m,n", [(1, 1), (5, 5), (16, 16), (17, 3), (33, 20), (31, 31)])
def test_orth_tiny_and_square(m, n):
    A = S.test_matrix(m, n, 10.0, seed=(4,))
    Qo, Ro, io = O.orth(A)
    b, info = sq.sqr_orth(dev(A))
    assert info["status"] == 0
    _check_factors(A, host(b.q()), host(b.r()), Qo, Ro, 10.0)


def test_orth_leading_dimensions_and_cap():
    A = S.test_matrix(3000, 12, 1e4, seed=(5,))
    Ad = dev(A, ld=3011)
    Q = sq.colmajor(3000, 20, ld=3005)
    R = sq.colmajor(20, 20, ld=23)
    b, info = sq.sqr_orth(Ad, cap=20, Q=Q, R=R)
    Qo, Ro, _ = O.orth(A)
    assert info["status"] == 0 and b.n == 12
    _check_factors(A, host(b.q()), host(b.r()), Qo, Ro, 1e4)
    assert np.array_equal(host(Ad), A)  # input untouched


def test_orth_deterministic():
    A = S.test_matrix(50000, 24, 1e10, seed=(8,))
    Ad = dev(A)
    b1, _ = sq.sqr_orth(Ad)
    b2, _ = sq.sqr_orth(Ad)
    assert torch.equal(b1.q(), b2.q()) and torch.equal(b1.r(), b2.r())


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("n", [5, 16])
def test_narrow_recomputed_passes_match_stored_passes(precision, n):
    """At most 16 columns, the passes before the first one that can end the
    call (min_passes = 3) recompute their input from A through the earlier
    inverse factors and write nothing; with min_passes = 1 every pass writes
    its result and the next reads it.  At kappa 1e10 the stopping test fails
    after passes 1 and 2 either way, so both calls take the same passes on
    the same values: Q and R are equal bit for bit."""
    A = S.test_matrix(40000, n, 1e10, seed=(31, n))
    Ad = dev(A)
    b3, i3 = sq.sqr_orth(Ad, opts=sq.sqr_default_opts(precision=precision))
    b1, i1 = sq.sqr_orth(Ad, opts=sq.sqr_default_opts(precision=precision, min_passes=1))
    assert i3["status"] == 0 and i1["status"] == 0
    assert i3["passes"] == i1["passes"] >= 3
    assert torch.equal(b3.q(), b1.q()) and torch.equal(b3.r(), b1.r())
    Qo, Ro, _ = O.orth(A)
    _check_factors(A, host(b3.q()), host(b3.r()), Qo, Ro, 1e10)


def test_orth_status_codes():
    A = S.test_matrix(400, 6, 1e2, seed=(13,))
    A[17, 3] = np.nan
    _, info = sq.sqr_orth(dev(A))
    assert info["status"] == sq.SQR_ENONFINITE
    A = S.test_matrix(400, 6, 1e2, seed=(14,))
    A[:, 2] = 0.0
    _, info = sq.sqr_orth(dev(A))
    assert info["status"] == sq.SQR_NOT_CONVERGED and info["passes"] == 10
    A = S.test_matrix(400, 6, 1e12, seed=(13,))
    _, info = sq.sqr_orth(dev(A), opts=sq.sqr_default_opts(max_iter=1, min_passes=0))
    assert info["status"] == sq.SQR_NOT_CONVERGED and info["passes"] == 1


def test_orth_async_then_last_info():
    A = S.test_matrix(8000, 16, 1e6, seed=(15,))
    b, info = sq.sqr_orth(dev(A), sync=False)
    assert info is None
    got = sq.sqr_last_info(b)
    _, _, io = O.orth(A)
    assert got["status"] == 0 and got["passes"] == io["passes"]


# --------------------------------------------------------------------------
# append parity (Algorithm 2) and the basis-growth run (Algorithm 3 shape)
# --------------------------------------------------------------------------
def _growth(m, nblocks, p=10):
    A0, Ws, _ = S.growth_blocks(m, 10, p, nblocks, 1e2, 1e12)
    Q, R, io = O.orth(A0)
    orc = [io["passes"]]
    for W in Ws:
        Q, R, io = O.append(Q, R, W)
        assert io["status"] == 0
        orc.append(io["passes"])
    b, info = sq.sqr_orth(dev(A0), cap=10 + p * nblocks)
    gp = [info["passes"]]
    for W in Ws:
        info = sq.sqr_append(b, dev(W))
        assert info["status"] == 0
        gp.append(info["passes"])
    A = np.concatenate([A0] + Ws, axis=1)
    return A, b, Q, R, orc, gp


def test_append_growth_parity_small():
    A, b, Qo, Ro, orc, gp = _growth(20000, 19)
    assert b.n == 200
    Qg, Rg = host(b.q()), host(b.r())
    assert O.loo(Qg) <= 1e-12
    assert O.rrr(A, Qg, Rg) <= 1e-13
    assert sum(abs(x - y) for x, y in zip(orc, gp)) <= 2
    # blocks reach kappa 1e12: R graded on its leading well-conditioned part
    assert np.linalg.norm(Rg[:10, :10] - Ro[:10, :10]) <= 1e-8 * np.linalg.norm(Ro[:10, :10])


@pytest.mark.parametrize("q,p", [(1, 1), (7, 3), (16, 16), (45, 13), (100, 40), (500, 16)])
def test_append_parity_shapes(q, p):
    m = 6007
    A1 = S.test_matrix(m, q, 1e3, seed=(30,))
    A2 = S.test_matrix(m, p, 1e5, seed=(31,))
    Q1, R1, _ = O.orth(A1)
    Qo, Ro, io = O.append(Q1, R1, A2)
    b, info = sq.sqr_orth(dev(A1), cap=q + p)
    info = sq.sqr_append(b, dev(A2, ld=m + 3))
    assert info["status"] == 0 and b.n == q + p
    A = np.concatenate([A1, A2], axis=1)
    _check_factors(A, host(b.q()), host(b.r()), Qo, Ro, 1e5)


@pytest.mark.parametrize("q,p,eps", [(500, 16, 1e-10), (500, 10, 1e-9), (300, 40, 1e-10), (90, 60, 1e-10)])
def test_append_nearly_dependent_shifts(q, p, eps):
    """A block almost inside the basis span: the unshifted factorisation of
    the Schur complement breaks down, so the shift (power iteration on X) and
    its x10 escalation run; with this q only the factor fits in LDS."""
    m = 3001
    A1 = S.test_matrix(m, q, 1e3, seed=(50,))
    Q1, R1, _ = O.orth(A1)
    rng = np.random.default_rng(51)
    W = Q1 @ rng.standard_normal((q, p)) + eps * rng.standard_normal((m, p))
    Qo, Ro, io = O.append(Q1, R1, W)
    assert io["status"] == 0 and io["chol_attempts"] > io["passes"]
    b, info = sq.sqr_orth(dev(A1), cap=q + p)
    info = sq.sqr_append(b, dev(W))
    assert info["status"] == 0 and b.n == q + p
    assert abs(info["passes"] - io["passes"]) <= 1
    # X is at the rounding level here, so where the x10 escalation first
    # factorises depends on rounding: one attempt, one factor of 10 in sigma
    assert abs(info["chol_attempts"] - io["chol_attempts"]) <= 1
    ratio = info["sigma"][0] / io["sigma"][0]
    assert min(abs(ratio - 1.0), abs(ratio - 10.0), abs(ratio - 0.1)) <= 1e-2 * max(ratio, 1.0)
    A = np.concatenate([A1, W], axis=1)
    Qg, Rg = host(b.q()), host(b.r())
    assert O.loo(Qg) <= 1e-12 and O.rrr(A, Qg, Rg) <= 1e-13
    Bo, Bg = Ro[:q, q:], Rg[:q, q:]
    assert np.linalg.norm(Bg - Bo) <= 1e-8 * np.linalg.norm(Bo)


def test_append_lucky_breakdown_keeps_width():
    m, q, p = 256, 10, 3
    H = S.hadamard(m)
    A1 = H[:, :q]
    b, info = sq.sqr_orth(dev(A1), cap=q + p,
                          opts=sq.sqr_default_opts(first_pass_shift=0, min_passes=0))
    assert info["status"] == 0
    W = A1 @ np.random.default_rng(9).integers(-3, 4, size=(q, p)).astype(float)
    _, _, io = O.append(H[:, :q] / 16.0, np.eye(q), W)
    info = sq.sqr_append(b, dev(W))
    assert info["status"] == io["status"] == sq.SQR_NOT_CONVERGED
    assert info["sigma"][0] == io["sigma"][0] == 2.0 ** -52
    assert b.n == q


def test_append_usage_errors():
    A = S.test_matrix(500, 8, 10.0, seed=(40,))
    b, _ = sq.sqr_orth(dev(A), cap=12)
    with pytest.raises(RuntimeError):
        sq.sqr_append(b, dev(S.test_matrix(500, 5, 10.0, seed=(41,))))  # n+p > cap
    assert b.n == 8


@pytest.mark.slow
def test_append_growth_parity_full_1e6():
    """Basis growth at full size: m = 1e6, 10 -> 200 columns in 19 appends."""
    A, b, Qo, Ro, orc, gp = _growth(1_000_000, 19)
    Qg, Rg = host(b.q()), host(b.r())
    assert O.loo(Qg) <= 1e-12
    assert O.rrr(A, Qg, Rg) <= 1e-13
    assert sum(abs(x - y) for x, y in zip(orc, gp)) <= 2
    rows = np.random.default_rng(0).choice(A.shape[0], 2000, replace=False)
    assert np.max(np.abs(Qg[rows, :10] - Qo[rows, :10])) <= 1e-8 * np.max(np.abs(Qo[:, :10]))


@pytest.mark.parametrize("m,n", [(6000, 10), (6000, 16), (5000, 64), (4001, 128), (3001, 160),
                                 (3000, 256)])
@pytest.mark.parametrize("kappa", [1e4, 1e8, 1e12, 1e15])
def test_orth_mixed_parity(m, n, kappa):
    """Mixed FP32/FP64 form against the oracle's mixed form and the FP64 QR."""
    A = S.test_matrix(m, n, kappa, seed=(13,))
    Qo, Ro, io = O.orth(A)
    Qm, Rm, im = O.orth(A, precision=1)
    b, info = sq.sqr_orth(dev(A), opts=sq.sqr_default_opts(precision=1))
    assert info["status"] == 0
    assert abs(info["passes"] - im["passes"]) <= 1
    # ||A||_2 = 1: the first (FP32) shift is n u32 to the norm estimate's accuracy
    assert abs(info["sigma"][0] / (n * 2.0 ** -24) - 1.0) < 2e-2
    assert info["sigma"][info["passes"] - 1] == 0.0
    _check_factors(A, host(b.q()), host(b.r()), Qo, Ro, kappa)


@pytest.mark.slow
def test_mixed_error_against_fp64_oracle_table():
    """Mixed and FP64 forms against the FP64 oracle over the C3 grid
    (n in {16, 64, 128}, kappa in {1e4, 1e8, 1e12, 1e15}) at m = 1e5: the
    relative error of R (graded where R is unique, kappa < 1e12), LOO and RRR
    of each result; the table is printed (pytest -s)."""
    m = 100_000
    rows = []
    for n in (16, 64, 128):
        for kappa in (1e4, 1e8, 1e12, 1e15):
            A = S.test_matrix(m, n, kappa, seed=(70, n))
            Qo, Ro, io = O.orth(A)
            line = [n, kappa, io["passes"]]
            for precision in (0, 1):
                b, info = sq.sqr_orth(dev(A), opts=sq.sqr_default_opts(precision=precision))
                assert info["status"] == 0
                Qg, Rg = host(b.q()), host(b.r())
                err = np.linalg.norm(Rg - Ro) / np.linalg.norm(Ro)
                loo, rrr = O.loo(Qg), O.rrr(A, Qg, Rg)
                assert loo <= 1e-12 and rrr <= 1e-13
                if kappa < 1e12:
                    assert err <= 1e-10 * kappa
                line += [info["passes"], err, loo, rrr]
                sq.sqr_free(b)
            rows.append(line)
    print("\n   n   kappa  oracle | FP64: passes  R err    LOO      RRR   | mixed: passes  R err    LOO      RRR")
    for r in rows:
        print("%4d %7.0e %5d   | %6d  %8.1e %8.1e %8.1e | %6d  %8.1e %8.1e %8.1e" % tuple(r))


@pytest.mark.parametrize("start", ["alg1", "cholqr3"])
def test_fig1_pattern_on_the_device(start):
    """Fig. 1's robustness pattern through the library: 300 x 10 inputs with
    kappa from 1 to 1e20 reach the stopping tolerance (LOO <= 1e-13, the
    Sec. 3.1 criterion), with Algorithm 1 as printed and with the CholQR3
    start, in as many passes as the oracle (+-1)."""
    kw = dict(first_pass_shift=0, min_passes=0) if start == "alg1" else {}
    for e in range(0, 21, 2):
        A = S.test_matrix(300, 10, 10.0 ** e, seed=(6,))
        _, _, io = O.orth(A, **kw)
        b, info = sq.sqr_orth(dev(A), opts=sq.sqr_default_opts(**kw))
        assert info["status"] == 0 and info["passes"] <= 10, e
        assert abs(info["passes"] - io["passes"]) <= 1, e
        Qg, Rg = host(b.q()), host(b.r())
        assert O.loo(Qg) <= 1e-13 and O.rrr(A, Qg, Rg) <= 1e-13, e
        sq.sqr_free(b)


def test_park_returns_workspace_and_results_are_unchanged():
    """sqr_park hands an idle handle's scratch back to the pool; the next call
    on the handle takes a workspace again.  Same kernels, same order: the
    parked run equals the unparked one bit for bit."""
    A = S.test_matrix(5000, 24, 1e5, seed=(80,))
    W = S.test_matrix(5000, 8, 1e3, seed=(81,))
    out = []
    for park in (False, True):
        b, info = sq.sqr_orth(dev(A), cap=32)
        assert info["status"] == 0
        if park:
            sq.sqr_park(b)
            sq.sqr_park(b)          # parking a parked handle does nothing
        info = sq.sqr_append(b, dev(W))
        assert info["status"] == 0 and b.n == 32
        out.append((host(b.q()), host(b.r())))
        sq.sqr_free(b)
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_prof_hooks_count_launches():
    """sqr_prof_enable / sqr_prof_read: HIP events around each streaming
    launch, folded into Gram-only and apply launches with their bytes."""
    m, n = 200_000, 48
    A = dev(S.test_matrix(m, n, 1e4, seed=(82,)))
    sq.sqr_prof_read()                      # drop earlier records
    sq.sqr_prof_enable(True)
    b, info = sq.sqr_orth(A)
    prof = sq.sqr_prof_read()
    sq.sqr_prof_enable(False)
    sq.sqr_free(b)
    ng, msg, bg = prof["gram"]
    na, msa, ba = prof["apply"]
    x = info["passes"]
    assert ng == 1 and na == x                     # one Gram-only pass, x applies
    assert bg == 8.0 * m * n and ba == x * 16.0 * m * n
    assert msg > 0 and msa > 0


def test_orth_mixed_limits():
    A = dev(S.test_matrix(1000, 257, 10.0, seed=(14,)))
    with pytest.raises(RuntimeError):
        sq.sqr_orth(A, opts=sq.sqr_default_opts(precision=1))
    with pytest.raises(RuntimeError):
        sq.sqr_orth(A[:, :20], opts=sq.sqr_default_opts(precision=2))


def test_serving_mix_matches_each_session_alone():
    """Serving loop: every session's final basis from a concurrent mix (four
    streams, Poisson arrivals) equals the basis of the same session's requests
    run alone on one stream, to the bit: kernel results do not depend on what
    else runs on the device."""
    from paper_2507_07788_amd import serve
    reqs = serve.synthetic_workload(48, 8, seed=21, m_range=(3000, 40000),
                                    n_range=(8, 40), p_range=(1, 16))
    serve.poisson_arrivals(reqs, 1e5, seed=22)       # all but at once: streams overlap
    mixed = {}
    keep = {s: (lambda s: lambda Q, R: mixed.__setitem__(s, (Q, R)))(s) for s in range(8)}
    res = serve.Server(workers=4, keep=keep).run(reqs)
    assert len(res) == 48 and all(r.status == 0 for r in res)
    assert any(a.start < b.end and b.start < a.end for a in res for b in res if a.rid != b.rid)
    for s in range(8):
        alone = {}
        mine = [serve.Request(**{**r.__dict__, "arrival": 0.0}) for r in reqs if r.session == s]
        serve.Server(workers=1, keep={s: lambda Q, R: alone.__setitem__(0, (Q, R))}).run(
            mine, seeds={r.rid: 1_000_003 * (r.rid + 1) for r in mine})
        Qm, Rm = mixed[s]
        Qa, Ra = alone[0]
        assert torch.equal(Qm, Qa) and torch.equal(Rm, Ra), s
        assert O.loo(Qm.numpy()) <= 1e-12


# --------------------------------------------------------------------------
# the panel scheme (Algorithm 3) on a given matrix
# --------------------------------------------------------------------------
@pytest.mark.parametrize("r", [1, 2, 3, 37])
def test_panel_hadamard_bitwise(r):
    """sqr_panel on A = H T reaches the closed form R = 2^k T, Q = H / 2^k
    bit for bit, one pass per panel, as the oracle's panel scheme does."""
    k, n = 5, 37
    H = S.hadamard(4 ** k)[:, :n]
    g = np.random.default_rng(5)
    T = np.triu(g.integers(-1, 2, size=(n, n)).astype(np.float64), 1) + np.diag(2.0 ** g.integers(0, 3, size=n))
    b, info = sq.sqr_panel(dev(H @ T), r)
    assert info["status"] == 0 and info["passes"] == 1 and b.n == n
    assert np.array_equal(host(b.r()), 2.0 ** k * T)
    assert np.array_equal(host(b.q()), H / 2.0 ** k)


@pytest.mark.parametrize("m,n,r,kappa", [(3000, 20, 2, 1e4), (5000, 64, 4, 1e8), (4097, 130, 3, 1e6),
                                         (2000, 300, 5, 1e3), (1000, 40, 40, 1e2), (20000, 100, 1, 1e10),
                                         (6000, 48, 3, 1e15)])
def test_panel_parity(m, n, r, kappa):
    """sqr_panel against the oracle's Algorithm 3: the same outcome, R and Q
    within the tolerances (invariants only at kappa >= 1e12)."""
    A = S.test_matrix(m, n, kappa, seed=(40, r))
    Qo, Ro, infos = O.panel(A, r)
    assert all(i["status"] == O.OK for i in infos)
    b, info = sq.sqr_panel(dev(A), r)
    assert info["status"] == 0 and b.n == n
    _check_factors(A, host(b.q()), host(b.r()), Qo, Ro, kappa)


# --------------------------------------------------------------------------
# appends with a wide basis (more S tiles than block_pass holds): the basis
# part of each pass runs in proj_pass / cross_pass / btb_pass / bacc_pass
# --------------------------------------------------------------------------
def _grow(widths, m, kappas, seed, **kw):
    """Orthogonalise the first panel and append the others, on the device
    and in the oracle (on the device's own basis before each append, so the
    comparison is per call).  Returns the device basis, the full input, and
    the list of (device info, oracle info, oracle Q_out, oracle R_out)."""
    mats = [S.test_matrix(m, w, k, seed=(seed, i)) for i, (w, k) in enumerate(zip(widths, kappas))]
    cap = sum(widths)
    b, info = sq.sqr_orth(dev(mats[0]), cap=cap, opts=sq.sqr_default_opts(**kw) if kw else None)
    assert info["status"] == 0
    steps = []
    for Wm in mats[1:]:
        q = b.n
        Qin, Rin = host(b.q()), host(b.r())
        Qo, Ro, io = O.append(Qin, Rin, Wm, **kw)
        info = sq.sqr_append(b, dev(Wm, ld=m + 5))
        steps.append((q, info, io, Qo, Ro))
    return b, np.concatenate(mats, axis=1), steps


@pytest.mark.parametrize("widths,kappas", [
    ([500, 100], [1e3, 1e5]),             # q 500 > 464 = widest basis on block_pass for p = 100
    ([300, 300, 37], [1e2, 1e4, 1e6]),    # two wide appends, ragged p
    ([528, 40, 1], [1e3, 1e5, 1e2]),      # p = 1
    ([400, 210, 130], [1e4, 1e8, 1e3]),   # p > 128: two column tiles in proj/cross
    ([528, 528], [1e3, 1e3]),             # the widest block
])
def test_append_wide_basis_parity(widths, kappas):
    """Each wide-basis append against the oracle's Algorithm 2 on the same
    basis: the same status, passes within one, the new columns Q, the block
    B = R[0:q, q:] and the diagonal block R[q:, q:] within the tolerances."""
    m = 4007
    b, A, steps = _grow(widths, m, kappas, seed=60)
    for (q, info, io, Qo, Ro), kap in zip(steps, kappas[1:]):
        p = Ro.shape[0] - q
        assert info["status"] == io["status"] == 0, (q, p)
        assert abs(info["passes"] - io["passes"]) <= 1
    assert b.n == sum(widths)
    Qg, Rg = host(b.q()), host(b.r())
    assert O.loo(Qg) <= 1e-12 and O.rrr(A, Qg, Rg) <= 1e-13
    assert np.array_equal(np.tril(Rg, -1), np.zeros_like(Rg))
    # the last append element by element against the oracle on its basis
    q, info, io, Qo, Ro = steps[-1]
    tol = 1e-10 * kappas[-1]
    for blk_g, blk_o in ((Rg[:q, q:], Ro[:q, q:]), (Rg[q:, q:], Ro[q:, q:]), (Qg[:, q:], Qo[:, q:])):
        assert np.max(np.abs(blk_g - blk_o)) <= tol * max(np.linalg.norm(blk_o), 1.0)


def test_append_wide_basis_element_wise_first_pass():
    """One wide append of a well-conditioned block (kappa 10, no shift): B,
    the new diagonal block of R and the new columns against the oracle
    element by element at a tight tolerance (the arithmetic differs only in
    the order of the summations)."""
    m, q, p = 3001, 600, 24
    A1 = S.test_matrix(m, 300, 10.0, seed=(61, 0))
    A2 = S.test_matrix(m, 300, 10.0, seed=(61, 1))
    W = S.test_matrix(m, p, 10.0, seed=(61, 2))
    b, _ = sq.sqr_orth(dev(A1), cap=q + p)
    assert sq.sqr_append(b, dev(A2))["status"] == 0 and b.n == q
    Qin, Rin = host(b.q()), host(b.r())
    Qo, Ro, io = O.append(Qin, Rin, W)
    info = sq.sqr_append(b, dev(W))
    assert info["status"] == 0 and info["passes"] == io["passes"]
    assert info["sigma"][:info["passes"]] == io["sigma"]
    Rg, Qg = host(b.r()), host(b.q())
    assert np.max(np.abs(Rg[:q, q:] - Ro[:q, q:])) <= 1e-13 * np.linalg.norm(Ro[:q, q:])
    assert np.max(np.abs(Rg[q:, q:] - Ro[q:, q:])) <= 1e-13 * np.linalg.norm(Ro[q:, q:])
    assert np.max(np.abs(Qg[:, q:] - Qo[:, q:])) <= 1e-12


def test_append_wide_basis_nearly_dependent_shift():
    """A block almost inside a 600-column basis: the unshifted factorisation
    breaks down, the shift from ||X||_2 and its x10 escalation run on the
    Schur complement that btb_pass and small_step form."""
    m, q, p, eps = 3001, 600, 12, 1e-10
    A1 = S.test_matrix(m, 300, 1e3, seed=(62, 0))
    A2 = S.test_matrix(m, 300, 1e3, seed=(62, 1))
    b, _ = sq.sqr_orth(dev(A1), cap=q + p)
    assert sq.sqr_append(b, dev(A2))["status"] == 0
    Qin, Rin = host(b.q()), host(b.r())
    rng = np.random.default_rng(63)
    W = Qin @ rng.standard_normal((q, p)) + eps * rng.standard_normal((m, p))
    Qo, Ro, io = O.append(Qin, Rin, W)
    assert io["status"] == 0 and io["chol_attempts"] > io["passes"]
    info = sq.sqr_append(b, dev(W))
    assert info["status"] == 0 and b.n == q + p
    assert abs(info["passes"] - io["passes"]) <= 1
    assert abs(info["chol_attempts"] - io["chol_attempts"]) <= 1
    Qg, Rg = host(b.q()), host(b.r())
    A = np.concatenate([Qin @ Rin, W], axis=1)
    assert O.loo(Qg) <= 1e-12 and O.rrr(A, Qg, Rg) <= 1e-13
    Bo, Bg = Ro[:q, q:], Rg[:q, q:]
    assert np.linalg.norm(Bg - Bo) <= 1e-8 * np.linalg.norm(Bo)


@pytest.mark.parametrize("cap", [0, 2])
def test_append_wide_basis_breakdown_keeps_width(cap):
    """The exact breakdown of test_append_breakdown_keeps_width on a
    600-column Hadamard basis (the wide-basis route): two identical new
    columns orthogonal to the basis give X = m [[1, 1], [1, 1]]; with
    u = 2^-100 every shift up to 100 sigma0 rounds away against m, so the
    append ends with SQR_BREAKDOWN after 2 + cap factorisations, as in the
    oracle; the width, Q and R are unchanged, and a NaN block then ends with
    SQR_ENONFINITE, also keeping the width."""
    k, q = 6, 600
    m = 4 ** k
    H = S.hadamard(m)
    kw = dict(unit_roundoff=2.0 ** -100, max_escalations=cap)
    opts = sq.sqr_default_opts(first_pass_shift=0, min_passes=0, **kw)
    b, info = sq.sqr_orth(dev(H[:, :300] * 3.0), cap=q + 3, opts=opts)
    assert info["status"] == 0
    assert sq.sqr_append(b, dev(H[:, 300:q] * 3.0))["status"] == 0 and b.n == q
    Q0, R0 = host(b.q()), host(b.r())
    assert np.array_equal(Q0, H[:, :q] / 2.0 ** k) and np.array_equal(R0, 3.0 * 2.0 ** k * np.eye(q))
    h = H[:, q]
    W = np.asfortranarray(np.stack([h, h], axis=1))
    _, _, io = O.append(Q0, R0, W, **kw)
    assert io["status"] == O.BREAKDOWN and io["chol_attempts"] == 2 + cap
    info = sq.sqr_append(b, dev(W))
    assert info["status"] == sq.SQR_BREAKDOWN
    assert info["chol_attempts"] == io["chol_attempts"]
    assert b.n == q
    assert np.array_equal(host(b.q()), Q0) and np.array_equal(host(b.r()), R0)
    Wn = H[:, q:q + 2].copy()
    Wn[17, 1] = np.nan
    _, _, io = O.append(Q0, R0, Wn, **kw)
    assert io["status"] == O.ENONFINITE
    info = sq.sqr_append(b, dev(Wn))
    assert info["status"] == sq.SQR_ENONFINITE and b.n == q
    # a regular block is then appended exactly: B = 0, R = 5 m^(1/2)
    info = sq.sqr_append(b, dev(H[:, q + 1:q + 2] * 5.0))
    assert info["status"] == 0 and b.n == q + 1
    Rg = host(b.r())
    assert np.array_equal(Rg[:q, q], np.zeros(q)) and Rg[q, q] == 5.0 * 2.0 ** k
    assert np.array_equal(host(b.q())[:, q], H[:, q + 1] / 2.0 ** k)


@pytest.mark.parametrize("m,n,r,kappa", [(3000, 800, 2, 1e4), (2500, 1200, 3, 1e6), (2000, 1100, 4, 1e3)])
def test_panel_wide_parity(m, n, r, kappa):
    """sqr_panel beyond 528 columns (panels of at most 528; from the second
    panel on the basis is wide) against the oracle's Algorithm 3."""
    A = S.test_matrix(m, n, kappa, seed=(66, r))
    Qo, Ro, infos = O.panel(A, r)
    assert all(i["status"] == O.OK for i in infos)
    b, info = sq.sqr_panel(dev(A), r)
    assert info["status"] == 0 and b.n == n
    _check_factors(A, host(b.q()), host(b.r()), Qo, Ro, kappa)


def test_batch_rejects_wide_basis_append():
    """sqr_batch runs appends on block_pass only: an append whose basis is too
    wide comes back with SQR_EDIM and leaves the basis as it was."""
    m = 2000
    A1 = S.test_matrix(m, 500, 1e2, seed=(67, 0))
    b, _ = sq.sqr_orth(dev(A1), cap=600)
    W = dev(S.test_matrix(m, 100, 1e2, seed=(67, 1)))
    res = sq.sqr_batch([("append", b, W)])
    assert res[0]["rc"] == sq.SQR_EDIM and b.n == 500
    assert sq.sqr_append(b, W)["status"] == 0 and b.n == 600


# --------------------------------------------------------------------------
# blocks wider than 528 columns: the apply in superblocks of 128 columns
# (proj_pass for the earlier superblocks), the Gramian from cross_pass, the
# small matrices of small_step in the workspace
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m,n,kappa,variant", [
    (3001, 529, 1e3, "CholQR3"), (4000, 600, 1e8, "CholQR3"), (3000, 1100, 1e5, "CholQR3"),
    (2500, 700, 1e15, "CholQR3"), (3001, 800, 1e5, "rsCholQR"), (2000, 1030, 1e12, "rsCholQR"),
])
def test_orth_wide_block_parity(m, n, kappa, variant):
    """sqr_orth beyond 528 columns against the oracle's Algorithm 1 (CholQR3
    start, or as printed): the same status, passes within one, R and Q within
    the tolerances (invariants only at kappa >= 1e12)."""
    kw = {} if variant == "CholQR3" else dict(first_pass_shift=0, min_passes=0)
    A = S.test_matrix(m, n, kappa, seed=(70, n))
    Qo, Ro, io = O.orth(A, **kw)
    b, info = sq.sqr_orth(dev(A, ld=m + 3), opts=sq.sqr_default_opts(**kw) if kw else None)
    assert info["status"] == io["status"] == 0
    assert abs(info["passes"] - io["passes"]) <= 1
    _check_factors(A, host(b.q()), host(b.r()), Qo, Ro, kappa)


@pytest.mark.parametrize("q,p,kappa", [(300, 600, 1e4), (17, 530, 1e6), (600, 1040, 1e3)])
def test_append_wide_block_parity(q, p, kappa):
    """An append of more than 528 columns on a basis (its B~, B~^T B~ and B
    outside small_step) against the oracle's Algorithm 2 on the same basis."""
    m = 3001
    A1 = S.test_matrix(m, min(q, 300), 1e2, seed=(71, 0))
    b, _ = sq.sqr_orth(dev(A1), cap=q + p)
    if q > 300:
        assert sq.sqr_append(b, dev(S.test_matrix(m, q - 300, 1e2, seed=(71, 1))))["status"] == 0
    assert b.n == q
    W = S.test_matrix(m, p, kappa, seed=(71, 2))
    Qin, Rin = host(b.q()), host(b.r())
    Qo, Ro, io = O.append(Qin, Rin, W)
    info = sq.sqr_append(b, dev(W, ld=m + 1))
    assert info["status"] == io["status"] == 0 and b.n == q + p
    assert abs(info["passes"] - io["passes"]) <= 1
    Qg, Rg = host(b.q()), host(b.r())
    A = np.concatenate([Qin @ Rin, W], axis=1)
    assert O.loo(Qg) <= 1e-12 and O.rrr(A, Qg, Rg) <= 1e-13
    assert np.array_equal(np.tril(Rg, -1), np.zeros_like(Rg))
    tol = 1e-10 * kappa
    for blk_g, blk_o in ((Rg[:q, q:], Ro[:q, q:]), (Rg[q:, q:], Ro[q:, q:]), (Qg[:, q:], Qo[:, q:])):
        assert np.max(np.abs(blk_g - blk_o)) <= tol * max(np.linalg.norm(blk_o), 1.0)


@pytest.mark.parametrize("m,n,r,kappa", [(3000, 1200, 2, 1e5), (2500, 1100, 1, 1e4), (2000, 1600, 3, 1e5)])
def test_panel_wide_block_parity(m, n, r, kappa):
    """sqr_panel with panels wider than 528 columns (r = 1: one append of
    1100 columns on an empty basis, wider than small_step's LDS vectors)
    against the oracle's Algorithm 3."""
    A = S.test_matrix(m, n, kappa, seed=(72, r))
    Qo, Ro, infos = O.panel(A, r)
    assert all(i["status"] == O.OK for i in infos)
    b, info = sq.sqr_panel(dev(A), r)
    assert info["status"] == 0 and b.n == n
    _check_factors(A, host(b.q()), host(b.r()), Qo, Ro, kappa)


def test_wide_block_breakdown_and_nonfinite_keep_width():
    """A block of 542 columns whose first two columns are the same Hadamard
    column: X has an exact zero pivot; with u = 2^-100 and no escalation the
    append ends with SQR_BREAKDOWN after two factorisations, as in the
    oracle, and the width is unchanged; a NaN block of 600 columns ends with
    SQR_ENONFINITE; then a block of 600 Hadamard columns is appended exactly
    (R~ = 64 I, so every step of the pass is exact in FP64)."""
    k, q = 5, 16
    m = 4 ** k
    H = S.hadamard(m)
    kw = dict(unit_roundoff=2.0 ** -100, max_escalations=0)
    b, info = sq.sqr_orth(dev(H[:, :q] * 2.0), cap=q + 600,
                          opts=sq.sqr_default_opts(first_pass_shift=0, min_passes=0, **kw))
    assert info["status"] == 0
    Q0, R0 = host(b.q()), host(b.r())
    W = np.asfortranarray(np.concatenate([H[:, q:q + 1], H[:, q:q + 1], H[:, q + 1:q + 541]], axis=1))
    _, _, io = O.append(Q0, R0, W, **kw)
    assert io["status"] == O.BREAKDOWN and io["chol_attempts"] == 2
    info = sq.sqr_append(b, dev(W))
    assert info["status"] == sq.SQR_BREAKDOWN and info["chol_attempts"] == 2 and b.n == q
    assert np.array_equal(host(b.q()), Q0) and np.array_equal(host(b.r()), R0)
    Wn = H[:, q:q + 600].copy()
    Wn[5, 333] = np.nan
    info = sq.sqr_append(b, dev(Wn))
    assert info["status"] == sq.SQR_ENONFINITE and b.n == q
    info = sq.sqr_append(b, dev(H[:, q:q + 600] * 2.0))
    assert info["status"] == 0 and b.n == q + 600
    Rg = host(b.r())
    assert np.array_equal(Rg[:q, q:], np.zeros((q, 600)))
    assert np.array_equal(Rg[q:, q:], 2.0 * 2.0 ** k * np.eye(600))
    assert np.array_equal(host(b.q()), H[:, :q + 600] / 2.0 ** k)


# --------------------------------------------------------------------------
# batched calls (sqr_batch): the same results as the calls made alone
# --------------------------------------------------------------------------
def _alone_and_batched(specs, opts=None):
    """specs: ("orth", m, n, kappa, cap) or ("append", index of an orth spec,
    p, kappa).  Every orth runs alone (sqr_orth) and in one batch; then every
    append runs alone (sqr_append) on the alone bases and in a second batch on
    the batched bases.  Returns the pairs of (Q, R, info)."""
    g = np.random.default_rng(31)
    A, W = {}, {}
    for i, sp in enumerate(specs):
        if sp[0] == "orth":
            A[i] = dev(S.test_matrix(sp[1], sp[2], sp[3], seed=(32, i)))
        else:
            m = specs[sp[1]][1]
            W[i] = dev(S.test_matrix(m, sp[2], sp[3], seed=(33, i)))
    alone, batched = {}, {}
    calls, orth_ids = [], []
    for i, sp in enumerate(specs):
        if sp[0] != "orth":
            continue
        b, info = sq.sqr_orth(A[i], cap=sp[4], opts=opts)
        alone[i] = (b, info)
        calls.append(("orth", A[i], sp[4], sq.colmajor(sp[1], sp[4]), sq.colmajor(sp[4], sp[4])))
        orth_ids.append(i)
    res = sq.sqr_batch(calls, opts=opts)
    for i, d in zip(orth_ids, res):
        assert d["rc"] == 0, (i, d)
        batched[i] = (d["basis"], d["info"])
    calls, app_ids = [], []
    for i, sp in enumerate(specs):
        if sp[0] != "append":
            continue
        alone[i] = (alone[sp[1]][0], sq.sqr_append(alone[sp[1]][0], W[i]))
        calls.append(("append", batched[sp[1]][0], W[i]))
        app_ids.append(i)
    if calls:
        res = sq.sqr_batch(calls)
        for i, d in zip(app_ids, res):
            assert d["rc"] == 0, (i, d)
            batched[i] = (batched[specs[i][1]][0], d["info"])
    return alone, batched


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_matches_calls_alone(precision):
    """Orthogonalisations of uneven m and n (one block, whole-pass, split and
    per-block routes) and appends of uneven p, batched, give the results of
    the same calls made alone, bit for bit, and the oracle's accuracy."""
    specs = [("orth", 3001, 7, 1e6, 20), ("orth", 20011, 20, 1e10, 36), ("orth", 9000, 40, 1e3, 56),
             ("orth", 5003, 130, 1e8, 130), ("orth", 4001, 230, 1e4, 230)]
    if precision == 0:
        specs.append(("orth", 2500, 300, 1e12, 300))
    specs += [("append", 0, 13, 1e4), ("append", 1, 16, 1e8), ("append", 2, 3, 1e2)]
    opts = sq.sqr_default_opts(precision=precision)
    alone, batched = _alone_and_batched(specs, opts)
    for i, sp in enumerate(specs):
        (ba, ia), (bb, ib) = alone[i], batched[i]
        assert ia["status"] == ib["status"] == 0, (i, ia, ib)
        assert ia["passes"] == ib["passes"] and ia["sigma"] == ib["sigma"], i
        assert torch.equal(ba.q(), bb.q()) and torch.equal(ba.r(), bb.r()), i
    for i, sp in enumerate(specs):
        if sp[0] == "orth":
            assert O.loo(host(batched[i][0].q())) <= 1e-12


def test_batch_item_errors_leave_the_others_running():
    """A bad item (a second append to the same basis, an append past the
    capacity) gets its usage code; the other items of the batch complete."""
    A = dev(S.test_matrix(5000, 12, 1e4, seed=(34,)))
    b, _ = sq.sqr_orth(A, cap=20)
    W1 = dev(S.test_matrix(5000, 4, 1e2, seed=(35,)))
    W2 = dev(S.test_matrix(5000, 9, 1e2, seed=(36,)))
    res = sq.sqr_batch([("append", b, W1), ("append", b, W1),
                        ("orth", A, 12, sq.colmajor(5000, 12), sq.colmajor(12, 12))])
    assert [d["rc"] for d in res] == [0, sq.SQR_EOPT, 0]
    assert res[0]["info"]["status"] == 0 and b.n == 16
    res = sq.sqr_batch([("append", b, W2)])
    assert res[0]["rc"] == sq.SQR_EDIM and b.n == 16


def test_serving_batched_mix_matches_each_session_alone():
    """Serving with batched launches (up to eight requests per sqr_batch, two
    streams): every session's final basis equals the basis of its requests
    run alone, one call at a time on one stream, to the bit."""
    from paper_2507_07788_amd import serve
    reqs = serve.synthetic_workload(64, 8, seed=23, m_range=(3000, 40000),
                                    n_range=(8, 40), p_range=(1, 16))
    serve.poisson_arrivals(reqs, 1e5, seed=24)
    mixed = {}
    keep = {s: (lambda s: lambda Q, R: mixed.__setitem__(s, (Q, R)))(s) for s in range(8)}
    res = serve.Server(workers=2, batch=8, keep=keep).run(reqs)
    assert len(res) == 64 and all(r.status == 0 for r in res)
    # some requests shared a batch (the same start and end)
    assert any(a.start == b.start and a.end == b.end for a in res for b in res if a.rid != b.rid)
    for s in range(8):
        alone = {}
        mine = [serve.Request(**{**r.__dict__, "arrival": 0.0}) for r in reqs if r.session == s]
        serve.Server(workers=1, keep={s: lambda Q, R: alone.__setitem__(0, (Q, R))}).run(
            mine, seeds={r.rid: 1_000_003 * (r.rid + 1) for r in mine})
        Qm, Rm = mixed[s]
        Qa, Ra = alone[0]
        assert torch.equal(Qm, Qa) and torch.equal(Rm, Ra), s


# --------------------------------------------------------------------------
# full sizes of the measured configurations (m = 4e6 and 2e7 rows)
# --------------------------------------------------------------------------
def _invariants_dev(A, Q, R, n):
    """LOO and RRR evaluated on the device in row blocks (any size)."""
    m = A.shape[0]
    G = torch.zeros((n, n), dtype=torch.float64, device=A.device)
    res = nrm = 0.0
    Rt = torch.triu(R[:n, :n]).contiguous()
    for r0 in range(0, m, 1 << 22):
        r1 = min(m, r0 + (1 << 22))
        Qb = Q[r0:r1, :n].contiguous()
        Ab = A[r0:r1].contiguous()
        G += Qb.t() @ Qb
        D = Ab - Qb @ Rt
        res += float((D * D).sum())
        nrm += float((Ab * Ab).sum())
    loo = float(torch.linalg.norm(G - torch.eye(n, dtype=G.dtype, device=G.device)))
    return loo, math.sqrt(res / nrm)


@pytest.mark.slow
def test_orth_full_size_m4e6_n64_against_oracle():
    """m = 4e6, n = 64, kappa = 1e4: the oracle runs at full size on the host."""
    A = S.test_matrix(4_000_000, 64, 1e4, seed=(3,))
    Qo, Ro, io = O.orth(A)
    b, info = sq.sqr_orth(dev(A))
    assert info["status"] == 0 and abs(info["passes"] - io["passes"]) <= 1
    Rg = host(b.r())
    assert np.max(np.abs(Rg - Ro)) <= 1e-10 * 1e4 * np.max(np.abs(Ro))
    rows = np.random.default_rng(1).choice(A.shape[0], 4000, replace=False)
    Qg = b.q()[torch.as_tensor(rows, device=b.Q.device)].cpu().numpy()
    assert np.max(np.abs(Qg - Qo[rows])) <= 1e-10 * 1e4 * np.max(np.abs(Qo[rows]))
    loo, rrr = _invariants_dev(dev(A), b.Q, b.R, 64)
    assert loo <= 1e-12 and rrr <= 1e-13


@pytest.mark.slow
@pytest.mark.parametrize("precision", [0, 1])
def test_orth_full_size_m4e6_n16_against_oracle(precision):
    """m = 4e6, n = 16, kappa = 1e4: the one-block route at its full launch
    shape (passes 1 and 2 recompute their input from A, 64-row steps dealt
    over the whole grid); R and sampled rows of Q against the oracle at full
    size, FP64 and the mixed form."""
    A = S.test_matrix(4_000_000, 16, 1e4, seed=(3,))
    Qo, Ro, io = O.orth(A)
    print(f"orth 4e6 x 16, precision {precision}", flush=True)
    b, info = sq.sqr_orth(dev(A), opts=sq.sqr_default_opts(precision=precision))
    assert info["status"] == 0 and abs(info["passes"] - io["passes"]) <= 1
    Rg = host(b.r())
    assert np.max(np.abs(Rg - Ro)) <= 1e-10 * 1e4 * np.max(np.abs(Ro))
    rows = np.random.default_rng(1).choice(A.shape[0], 4000, replace=False)
    Qg = b.q()[torch.as_tensor(rows, device=b.Q.device)].cpu().numpy()
    assert np.max(np.abs(Qg - Qo[rows])) <= 1e-10 * 1e4 * np.max(np.abs(Qo[rows]))
    loo, rrr = _invariants_dev(dev(A), b.Q, b.R, 16)
    assert loo <= 1e-12 and rrr <= 1e-13


@pytest.mark.parametrize("m,n", [(1_000_003, 16), (1_000_003, 11), (262_147, 40), (65_541, 16)])
def test_orth_ragged_row_steps_against_oracle(m, n):
    """Row counts whose 64-row steps do not divide evenly over the grid and
    whose last step and last tile are partial: every row enters the Gramian
    and the result once (one-block route for n <= 16, fused wide route at 40)."""
    A = S.test_matrix(m, n, 1e6, seed=(5,))
    Qo, Ro, io = O.orth(A)
    print(f"orth {m} x {n}", flush=True)
    b, info = sq.sqr_orth(dev(A))
    assert info["status"] == 0 and abs(info["passes"] - io["passes"]) <= 1
    _check_factors(A, host(b.q()), host(b.r()), Qo, Ro, 1e6)


@pytest.mark.slow
@pytest.mark.parametrize("precision", [0, 1])
def test_orth_full_size_m4e6_n128_kappa1e12(precision):
    A = S.test_matrix_device(4_000_000, 128, 1e12, (3,))
    b, info = sq.sqr_orth(A, opts=sq.sqr_default_opts(precision=precision))
    assert info["status"] == 0
    loo, rrr = _invariants_dev(A, b.Q, b.R, 128)
    assert loo <= 1e-12 and rrr <= 1e-13


@pytest.mark.slow
def test_orth_full_size_m2e7_n256_kappa1e15():
    """FP64, then the mixed form on the same matrix."""
    A = S.test_matrix_device(20_000_000, 256, 1e15, (3,))
    for precision in (0, 1):
        print(f"orth 2e7 x 256, precision {precision}", flush=True)
        b, info = sq.sqr_orth(A, opts=sq.sqr_default_opts(precision=precision))
        assert info["status"] == 0 and info["passes"] <= 10
        loo, rrr = _invariants_dev(A, b.Q, b.R, 256)
        assert loo <= 1e-12 and rrr <= 1e-13
        sq.sqr_free(b)
        del b
        torch.cuda.empty_cache()


def test_orth_maximum_width_528():
    """The widest basis a handle supports (33 blocks: per-block launches, the
    small matrices in workspace memory)."""
    A = S.test_matrix(3000, 528, 1e4, seed=(23,))
    Qo, Ro, io = O.orth(A)
    b, info = sq.sqr_orth(dev(A))
    assert info["status"] == 0 and abs(info["passes"] - io["passes"]) <= 1
    _check_factors(A, host(b.q()), host(b.r()), Qo, Ro, 1e4)


def test_append_fills_capacity_528():
    """Appends up to the 528-column capacity; one more column is refused."""
    A = S.test_matrix(2500, 528, 1e3, seed=(24,))
    b, info = sq.sqr_orth(dev(A[:, :400]), cap=528)
    for c0 in range(400, 528, 64):
        info = sq.sqr_append(b, dev(A[:, c0:c0 + 64]))
        assert info["status"] == 0
    assert b.n == 528
    Qo, Ro, _ = O.orth(A)
    _check_factors(A, host(b.q()), host(b.r()), Qo, Ro, 1e3)
    with pytest.raises(RuntimeError):
        sq.sqr_append(b, dev(A[:, :1]))


# --------------------------------------------------------------------------
# status paths: the escalation cap, non-finite appends, the append entry
# case, the stopping test at an exact non-zero distance
# --------------------------------------------------------------------------
def _dup_hadamard(k=4):
    """[h1, h1, h2, h3]: an exact Gramian with the zero pivot 256 - 16 * 16."""
    H = S.hadamard(4 ** k)
    return np.asfortranarray(np.stack([H[:, 1], H[:, 1], H[:, 2], H[:, 3]], axis=1))


@pytest.mark.parametrize("cap", [0, 1, 3])
def test_orth_breakdown_at_the_escalation_cap(cap):
    """Algorithm 1 as printed with u = 2^-80 on exactly dependent columns:
    every shift up to 1e3 sigma0 rounds away against the Gramian's entries,
    so each factorisation meets the same exact zero pivot and the call ends
    with SQR_BREAKDOWN after 2 + cap factorisations, as in the oracle."""
    A = _dup_hadamard()
    kw = dict(first_pass_shift=0, min_passes=0, unit_roundoff=2.0 ** -80, max_escalations=cap)
    _, _, io = O.orth(A, **kw)
    assert io["status"] == O.BREAKDOWN and io["chol_attempts"] == 2 + cap
    b, info = sq.sqr_orth(dev(A), opts=sq.sqr_default_opts(**kw))
    assert info["status"] == sq.SQR_BREAKDOWN
    assert info["chol_attempts"] == io["chol_attempts"] and info["passes"] == 0
    assert info["converged"] == 0


@pytest.mark.parametrize("cap", [0, 2])
def test_append_breakdown_keeps_width(cap):
    """Two identical new columns orthogonal to the basis: X = [[1, 1], [1, 1]]
    exactly; with u = 2^-80 and a small cap the append ends with
    SQR_BREAKDOWN, the width is unchanged, and the basis then takes a
    regular append."""
    k, q = 4, 6
    m = 4 ** k
    H = S.hadamard(m)
    A1 = H[:, :q] * 3.0
    h = H[:, q]
    W = np.asfortranarray(np.stack([h, h], axis=1))
    kw = dict(unit_roundoff=2.0 ** -80, max_escalations=cap)
    _, _, io = O.append(H[:, :q] / 16.0, 3.0 * 16.0 * np.eye(q), W, **kw)
    assert io["status"] == O.BREAKDOWN
    b, info = sq.sqr_orth(dev(A1), cap=q + 3, opts=sq.sqr_default_opts(first_pass_shift=0, min_passes=0, **kw))
    assert info["status"] == 0
    Q0, R0 = host(b.q()), host(b.r())
    info = sq.sqr_append(b, dev(W))
    assert info["status"] == sq.SQR_BREAKDOWN
    assert info["chol_attempts"] == io["chol_attempts"] == 2 + cap
    assert b.n == q
    assert np.array_equal(host(b.q()), Q0) and np.array_equal(host(b.r()), R0)
    info = sq.sqr_append(b, dev(H[:, q + 1:q + 2] * 5.0))
    assert info["status"] == 0 and b.n == q + 1
    assert np.array_equal(host(b.r())[:q, q], np.zeros(q))
    assert host(b.r())[q, q] == 5.0 * 16.0


def test_append_nonfinite_keeps_width():
    A1 = S.test_matrix(3000, 12, 1e3, seed=(90,))
    W = S.test_matrix(3000, 5, 1e2, seed=(91,))
    W[1234, 2] = np.nan
    _, _, io = O.append(*O.orth(A1)[:2], W)
    assert io["status"] == O.ENONFINITE
    b, info = sq.sqr_orth(dev(A1), cap=20)
    info = sq.sqr_append(b, dev(W))
    assert info["status"] == sq.SQR_ENONFINITE and b.n == 12
    W[1234, 2] = np.inf
    assert sq.sqr_append(b, dev(W))["status"] == sq.SQR_ENONFINITE and b.n == 12
    W[1234, 2] = 0.5
    assert sq.sqr_append(b, dev(W))["status"] == 0 and b.n == 17


@pytest.mark.parametrize("k,q,p", [(4, 12, 5), (5, 40, 16), (5, 20, 37)])
def test_append_entry_case_bitwise(k, q, p):
    """W = Q_in C + H_p / 2^k: the initial Schur complement is I exactly while
    B~ = C.  One pass applies the projection (Prop. 2.1): Q = H_p / 2^k,
    B = C, R = I bit for bit, on the device as in the oracle."""
    m = 4 ** k
    H = S.hadamard(m)
    Qin = H[:, :q] / 2.0 ** k
    C = np.random.default_rng(17 + q).integers(-3, 4, size=(q, p)).astype(np.float64)
    W = Qin @ C + H[:, q:q + p] / 2.0 ** k
    Qo, Ro, io = O.append(Qin, np.eye(q), W)
    assert io["passes"] == 1
    kw = dict(first_pass_shift=0, min_passes=0)
    b, info = sq.sqr_orth(dev(H[:, :q]), cap=q + p, opts=sq.sqr_default_opts(**kw))
    assert info["status"] == 0
    info = sq.sqr_append(b, dev(W))
    assert info["status"] == 0 and info["passes"] == 1 and b.n == q + p
    Rg = host(b.r())
    assert np.array_equal(host(b.q())[:, q:], H[:, q:q + p] / 2.0 ** k)
    assert np.array_equal(Rg[:q, q:], C * 2.0 ** k / 2.0 ** k)
    assert np.array_equal(Rg[q:, q:], np.eye(p))
    assert info["orth_fro"] == 0.0


@pytest.mark.parametrize("tol,passes", [(3.5, 0), (3.0, 1)])
def test_stop_test_is_strict_on_the_frobenius_distance(tol, passes):
    """A = [2 h1, h2] / 8: ||X - I||_F = 3 exactly.  tol 3.5 stops before any
    pass (Q = A, R = I), tol 3 does not (one exact pass)."""
    H = S.hadamard(64)
    A = np.asfortranarray(np.stack([2.0 * H[:, 0], H[:, 1]], axis=1) / 8.0)
    kw = dict(first_pass_shift=0, min_passes=0, tol=tol)
    Qo, Ro, io = O.orth(A, **kw)
    b, info = sq.sqr_orth(dev(A), opts=sq.sqr_default_opts(**kw))
    assert info["status"] == 0 and info["passes"] == io["passes"] == passes
    assert info["orth_fro"] == io["orth_fro"] == (3.0 if passes == 0 else 0.0)
    assert np.array_equal(host(b.q()), Qo) and np.array_equal(host(b.r()), Ro)


@pytest.mark.parametrize("dim", [0, 1, 2])
def test_append_first_shift_dimension(dim):
    """Algorithm 2's first shift with d = q (as printed), p or q + p: the
    duplicated column pair breaks down unshifted and factors at the first
    shift, which the device publishes."""
    k, q = 4, 6
    H = S.hadamard(4 ** k)
    W = np.asfortranarray(np.stack([H[:, q], H[:, q]], axis=1) / 16.0)
    _, _, io = O.append(H[:, :q] / 16.0, np.eye(q), W, append_shift_dim=dim)
    b, info = sq.sqr_orth(dev(H[:, :q] / 16.0), cap=q + 2,
                          opts=sq.sqr_default_opts(first_pass_shift=0, min_passes=0,
                                                   append_shift_dim=dim))
    info = sq.sqr_append(b, dev(W))
    want = io["shift_tries"][0]
    assert info["chol_attempts"] >= 2 and info["sigma"][0] > 0.0
    assert abs(info["sigma"][0] - want) <= 1e-12 * want


# --------------------------------------------------------------------------
# the Cholesky QR variants (Sec. 3.1) and Fig. 1's pattern on the device
# --------------------------------------------------------------------------
@pytest.mark.parametrize("variant", sorted(sq.VARIANTS))
def test_variants_fig1_pattern_on_the_device(variant):
    """Each variant on 300 x 10 inputs with kappa = 10^0 .. 10^20 through the
    library, against the oracle's variant: the same status wherever the
    oracle is away from its own transition (it reaches the same status at the
    neighbouring decades too), LOO and RRR of every successful call as in
    the oracle, and the robustness pattern of Fig. 1."""
    kw = sq.VARIANTS[variant]
    st, ost, loo = {}, {}, {}
    for e in range(0, 21):
        A = S.test_matrix(300, 10, 10.0 ** e, seed=(6,))
        Qo, Ro, io = O.orth(A, **kw)
        b, info = sq.sqr_orth(dev(A), opts=sq.sqr_default_opts(**kw))
        st[e], ost[e] = info["status"], io["status"]
        Qg, Rg = host(b.q()), host(b.r())
        loo[e] = O.loo(Qg)
        if info["status"] == 0:
            assert abs(info["passes"] - io["passes"]) <= 1, e
            assert loo[e] <= max(1e-13, 1e2 * O.loo(Qo)), e
            assert O.rrr(A, Qg, Rg) <= 1e-13, e
        sq.sqr_free(b)
    for e in range(0, 21):
        stable = all(ost.get(f, ost[e]) == ost[e] for f in (e - 1, e + 1))
        if stable:
            assert st[e] == ost[e], (variant, e, st, ost)
    if variant in ("rsCholQR", "isCholQR", "CholQR3"):
        assert all(v == 0 for v in st.values()) and max(loo.values()) <= 1e-13
    if variant in ("CholQR", "CholQR2"):
        # kappa = 1e10 is the oracle's own transition decade: the two
        # smallest eigenvalues of the Gramian (1e-20, 1.7e-18) lie below its
        # rounding noise (~u), so whether a pivot turns non-positive depends
        # on the summation order (a call that gets through is graded by the
        # LOO and RRR checks above).
        assert all(st[e] == sq.SQR_BREAKDOWN for e in range(11, 21)), st


# --------------------------------------------------------------------------
# one handle, calls on alternating streams
# --------------------------------------------------------------------------
def test_alternating_streams_match_one_stream():
    """Calls of one handle on two streams are ordered (the later call waits
    for the earlier call's stream): orth, then appends alternating between
    the streams, equals the single-stream run bit for bit."""
    A0, Ws, _ = S.growth_blocks(60_000, 10, 10, 8, 1e2, 1e10)
    A0d = dev(A0)
    Wd = [dev(W) for W in Ws]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    out = []
    for streams in ((s1, s1), (s1, s2)):
        b, info = sq.sqr_orth(A0d, cap=90, stream=streams[0])
        assert info["status"] == 0
        for i, W in enumerate(Wd):
            info = sq.sqr_append(b, W, stream=streams[(i + 1) % 2])
            assert info["status"] == 0
        torch.cuda.synchronize()
        out.append((b.q().clone(), b.r().clone()))
        sq.sqr_free(b)
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    assert O.loo(host(out[1][0])) <= 1e-12


@pytest.mark.slow
def test_append_growth_full_1e6_elementwise():
    """Basis growth at m = 1e6 (10 -> 200 columns) with block kappa up to 1e6.
    The accumulated matrix [A0 W_1 .. W_19] is numerically singular (its
    condition number passes 1e15 after a few blocks: every block is coupled to
    the span of the earlier ones), so the global factors are not unique; the
    block of each append is, given the basis it is appended to (Prop. 2.1).
    So every append of the device run is compared with the oracle's append on
    the device's own basis Q_in, R_in: B, the new diagonal block of R and the
    new columns of Q element by element within 1e-10 kappa_k times their norm.
    The whole basis is graded on LOO and RRR."""
    m, nb, p = 1_000_000, 19, 10
    A0, Ws, kap = S.growth_blocks(m, 10, p, nb, 1e2, 1e6, seed=3)
    b, info = sq.sqr_orth(dev(A0), cap=10 + p * nb)
    Qo0, Ro0, _ = O.orth(A0)
    _check_factors(A0, host(b.q()), host(b.r()), Qo0, Ro0, 1e2)
    for W in Ws:
        assert sq.sqr_append(b, dev(W))["status"] == 0
    Qg, Rg = host(b.q()), host(b.r())
    for k, W in enumerate(Ws):
        q = 10 + p * k
        Qn, Rn, io = O.append(Qg[:, :q], Rg[:q, :q], W)
        assert io["status"] == 0, k
        tol = 1e-10 * kap[k]
        nrm = np.linalg.norm(Rn[:, q:])
        assert np.max(np.abs(Rg[:q, q:q + p] - Rn[:q, q:])) <= tol * nrm, k        # B
        assert np.max(np.abs(Rg[q:q + p, q:q + p] - Rn[q:, q:])) <= tol * nrm, k   # R_kk
        assert np.max(np.abs(Qg[:, q:q + p] - Qn[:, q:])) <= tol, k                # Q_k
    assert O.loo(Qg) <= 1e-12
    A = np.concatenate([A0] + Ws, axis=1)
    assert O.rrr(A, Qg, Rg) <= 1e-13
