"""The allocation-free orthogonalisation (sqr_orth_noalloc) against sqr_orth,
through the C ABI: two calls in a row on the shared static scratch, the
second smaller, each bit for bit equal to sqr_orth on the same input (the
same kernels and slot counts) and within the oracle's tolerances."""
import numpy as np
import pytest
import torch

import synth as S
from oracle import cholqr as O

pytestmark = pytest.mark.gpu

import paper_2507_07788_amd as sq  # noqa: E402
from gpu_util import dev, host  # noqa: E402


def _one(m, n, kappa, seed):
    A = S.test_matrix(m, n, kappa, seed=seed)
    Ad = dev(A)
    Q = sq.colmajor(m, n)
    R = sq.colmajor(n, n)
    Q.fill_(np.nan)
    R.fill_(np.nan)
    info = sq.sqr_orth_noalloc(Ad, Q, R)
    b, ref = sq.sqr_orth(Ad)
    assert info["status"] == ref["status"] == 0, (info, ref)
    assert info["passes"] == ref["passes"]
    assert info["sigma"] == ref["sigma"]
    assert torch.equal(Q, b.q()) and torch.equal(R, b.r())
    Qo, Ro, _ = O.orth(A)
    Qg, Rg = host(Q), host(R)
    assert O.loo(Qg) <= 1e-12 and O.rrr(A, Qg, Rg) <= 1e-13
    assert np.linalg.norm(Rg - Ro) <= 1e-10 * kappa * np.linalg.norm(Ro)
    sq.sqr_free(b)


def test_noalloc_two_calls_match_sqr_orth():
    print("noalloc: 200000 x 64, then 30011 x 20", flush=True)
    _one(200000, 64, 1e8, (90,))
    _one(30011, 20, 1e4, (91,))


def test_noalloc_every_route_and_async():
    """One block (narrow), whole-pass (wide) and split (128 columns) routes,
    the mixed form, and a call without info followed by a stream sync."""
    for m, n, kw in [(5000, 7, {}), (7001, 40, {}), (9000, 128, {}),
                     (8000, 48, dict(precision=1))]:
        print("noalloc route", m, n, kw, flush=True)
        A = S.test_matrix(m, n, 1e6, seed=(92, n))
        Ad = dev(A)
        Q, R = sq.colmajor(m, n), sq.colmajor(n, n)
        opts = sq.sqr_default_opts(**kw)
        info = sq.sqr_orth_noalloc(Ad, Q, R, opts=opts)
        b, ref = sq.sqr_orth(Ad, opts=opts)
        assert info["status"] == ref["status"] == 0 and info["passes"] == ref["passes"]
        assert torch.equal(Q, b.q()) and torch.equal(R, b.r())
        Q2, R2 = sq.colmajor(m, n), sq.colmajor(n, n)
        assert sq.sqr_orth_noalloc(Ad, Q2, R2, opts=opts, sync=False) is None
        torch.cuda.synchronize()
        assert torch.equal(Q2, Q) and torch.equal(R2, R)
        sq.sqr_free(b)
