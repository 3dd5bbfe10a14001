"""Host-side checks of the C ABI: the library loads, exports every function
declared in include/sqr.h, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sq():
    import paper_2507_07788_amd as sq
    return sq


def test_header_symbols_exported(sq):
    import glob
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        names |= set(re.findall(r"^\s*(?:int|void|int64_t)\s+(sqr_\w+)\s*\(",
                                open(h).read(), re.M))
    assert {"sqr_orth", "sqr_append", "sqr_free", "sqr_prof_read"} <= names
    lib = ctypes.CDLL(sq.LIB_PATH)
    for nm in names:
        assert hasattr(lib, nm), nm


def test_default_opts_are_the_papers_settings(sq):
    o = sq.sqr_default_opts()
    assert o.max_iter == 10 and o.tol == 1e-13          # Sec. 3.1
    assert o.unit_roundoff == 2.0 ** -53
    assert o.first_pass_shift == 1 and o.min_passes == 3  # CholQR3 start
    assert o.precision == 0 and o.max_escalations == 32 and o.power_steps == 30
    assert o.shift_policy == 0 and o.append_shift_dim == 0  # Algorithms 1 and 2 as printed


def _orth(sq, m, n, lda, ldq, cap, ldr, A=1, Q=1, R=1, opts=None):
    h = ctypes.c_void_p()
    P = lambda v: ctypes.c_void_p(0x1000 if v else 0)  # never dereferenced
    return sq.lib.sqr_orth(ctypes.byref(h), ctypes.byref(opts) if opts else None, m, n,
                           P(A), lda, P(Q), ldq, cap, P(R), ldr, None, None)


def test_usage_errors_before_any_gpu_work(sq):
    assert _orth(sq, 100, 10, 100, 100, 10, 10, A=0) == sq.SQR_ENULL
    assert _orth(sq, 100, 10, 100, 100, 10, 10, Q=0) == sq.SQR_ENULL
    assert _orth(sq, 100, 10, 100, 100, 10, 10, R=0) == sq.SQR_ENULL
    assert _orth(sq, 10, 11, 10, 10, 11, 11) == sq.SQR_EDIM       # n > m
    assert _orth(sq, 0, 0, 1, 1, 1, 1) == sq.SQR_EDIM             # empty
    assert _orth(sq, 100, 10, 99, 100, 10, 10) == sq.SQR_EDIM     # lda < m
    assert _orth(sq, 100, 10, 100, 99, 10, 10) == sq.SQR_EDIM     # ldq < m
    assert _orth(sq, 100, 10, 100, 100, 9, 10) == sq.SQR_EDIM     # cap < n
    assert _orth(sq, 100, 10, 100, 100, 12, 11) == sq.SQR_EDIM    # ldr < cap
    assert _orth(sq, 40000, 10, 40000, 40000, 16385, 16385) == sq.SQR_EDIM  # cap above 16384
    bad = sq.sqr_default_opts(precision=7)
    assert _orth(sq, 100, 10, 100, 100, 10, 10, opts=bad) == sq.SQR_EOPT
    bad = sq.sqr_default_opts(max_iter=0)
    assert _orth(sq, 100, 10, 100, 100, 10, 10, opts=bad) == sq.SQR_EOPT
    for kw in (dict(shift_policy=3), dict(shift_policy=-1), dict(append_shift_dim=3),
               dict(shift_policy=1, precision=1), dict(shift_policy=2, precision=1)):
        assert _orth(sq, 100, 10, 100, 100, 10, 10, opts=sq.sqr_default_opts(**kw)) == sq.SQR_EOPT, kw
    assert sq.lib.sqr_append(None, ctypes.c_void_p(0x1000), 1, 1, None, None) == sq.SQR_ENULL
    assert sq.lib.sqr_cols(None) == 0
    sq.lib.sqr_free(None)


def test_serving_workload_recipe():
    """The serving workload's request plan (host logic, no GPU): sessions
    start with an orthogonalisation, reserve exactly the columns their
    appends need, never exceed 512 columns, and keep their order."""
    from paper_2507_07788_amd import serve
    reqs = serve.synthetic_workload(2000, 64)
    assert len(reqs) == 2000 and len({r.session for r in reqs}) == 64
    width, cap, seen = {}, {}, set()
    for r in sorted(reqs, key=lambda r: r.rid):
        if r.session not in seen:
            assert r.kind == "orth"
            seen.add(r.session)
        if r.kind == "orth":
            width[r.session], cap[r.session] = r.cols, r.cap
            assert r.cols <= r.cap <= 512 and r.cols <= r.m
        else:
            width[r.session] += r.cols
            assert width[r.session] <= cap[r.session]
            assert 1 <= r.cols <= 16
    serve.poisson_arrivals(reqs, 100.0)
    arr = [r.arrival for r in sorted(reqs, key=lambda r: r.rid)]
    assert all(b > a for a, b in zip(arr, arr[1:]))
    assert abs(arr[-1] / len(arr) - 0.01) < 0.002      # mean gap 1 / rate


def test_variant_options_match_the_oracle(sq):
    """The binding's variant table and the oracle's name the same settings."""
    from oracle import cholqr as O
    assert set(sq.VARIANTS) == set(O.VARIANTS)
    for name, kw in sq.VARIANTS.items():
        assert kw == O.VARIANTS[name], name


def test_wrapper_rejects_bad_shapes_before_the_library(sq):
    """The C ABI sees only pointers and leading dimensions, so the binding
    checks shapes and devices first (host tensors: nothing reaches a GPU)."""
    import torch
    A = torch.zeros(4, 10).t()                     # 10 x 4, column-major
    with pytest.raises(ValueError):
        sq.sqr_orth(A, cap=6, Q=torch.zeros(5, 10).t(), R=torch.zeros(6, 6))   # Q too narrow
    with pytest.raises(ValueError):
        sq.sqr_orth(A, cap=6, Q=torch.zeros(6, 9).t(), R=torch.zeros(6, 6))    # Q too short
    with pytest.raises(ValueError):
        sq.sqr_orth(A, cap=6, Q=torch.zeros(6, 10).t(), R=torch.zeros(6, 5))   # R too small
    with pytest.raises(ValueError):
        sq.sqr_orth(A, cap=6, Q=torch.zeros(6, 10, device="meta").t(), R=torch.zeros(6, 6))
    with pytest.raises(ValueError):
        sq.sqr_orth(A, cap=3)                                                   # cap < n
    b = sq.Basis(None, torch.zeros(8, 10).t(), torch.zeros(8, 8), 10, 8)
    with pytest.raises(ValueError):
        sq.sqr_append(b, torch.zeros(2, 9).t())                                 # W rows != m
    with pytest.raises(ValueError):
        sq.sqr_append(b, torch.zeros(2, 10, device="meta").t())


def _noalloc(sq, m, n, lda, ldq, ldr, A=1, Q=1, R=1, opts=None):
    P = lambda v: ctypes.c_void_p(0x1000 if v else 0)  # never dereferenced
    return sq.lib.sqr_orth_noalloc(ctypes.byref(opts) if opts else None, m, n, P(A), lda,
                                   P(Q), ldq, P(R), ldr, None, None)


def test_noalloc_usage_errors_and_limit_before_any_gpu_work(sq):
    """sqr_orth_noalloc rejects bad arguments and widths beyond its static
    scratch (SQR_NOALLOC_MAX_COLS) before any HIP call."""
    hdr = open(os.path.join(ROOT, "include", "sqr.h")).read()
    maxc = int(re.search(r"#define SQR_NOALLOC_MAX_COLS\s+(\d+)", hdr).group(1))
    assert maxc == 128
    assert _noalloc(sq, 100, 10, 100, 100, 10, A=0) == sq.SQR_ENULL
    assert _noalloc(sq, 100, 10, 100, 100, 10, R=0) == sq.SQR_ENULL
    assert _noalloc(sq, 10, 11, 10, 10, 11) == sq.SQR_EDIM        # n > m
    assert _noalloc(sq, 100, 10, 99, 100, 10) == sq.SQR_EDIM      # lda < m
    assert _noalloc(sq, 100, 10, 100, 100, 9) == sq.SQR_EDIM      # ldr < n
    assert _noalloc(sq, 10000, maxc + 1, 10000, 10000, maxc + 1) == sq.SQR_ELIMIT
    bad = sq.sqr_default_opts(max_iter=0)
    assert _noalloc(sq, 100, 10, 100, 100, 10, opts=bad) == sq.SQR_EOPT


def test_leading_dimension_limit(sq):
    """Leading dimensions of 2^25 rows or more are refused (lane offsets
    inside a 16-column tile must stay below 4 GiB)."""
    big = 1 << 25
    assert _orth(sq, 100, 10, big, 100, 10, 10) == sq.SQR_EDIM
    assert _orth(sq, 100, 10, 100, big, 10, 10) == sq.SQR_EDIM
    assert _noalloc(sq, 100, 10, big, 100, 10) == sq.SQR_EDIM


def test_batch_usage_errors_before_any_gpu_work(sq):
    """sqr_batch rejects a missing item list and gives every bad item its own
    usage code (the checks of sqr_orth / sqr_append) without touching a GPU
    when no item is left to run."""
    assert sq.lib.sqr_batch(None, None, 1, None) == sq.SQR_ENULL
    items = (sq.SqrBatchItem * 3)()
    assert sq.lib.sqr_batch(None, items, 0, None) == sq.SQR_ENULL
    items[0].kind = sq.SQR_BATCH_ORTH                 # null pointers
    items[1].kind = sq.SQR_BATCH_ORTH                 # n > m
    items[1].inp = items[1].Q = items[1].R = 0x1000
    items[1].m, items[1].cols, items[1].ld_in, items[1].ldq, items[1].cap, items[1].ldr = 10, 11, 10, 10, 11, 11
    items[2].kind = 7                                 # unknown kind
    assert sq.lib.sqr_batch(None, items, 3, None) == sq.SQR_OK
    assert [it.rc for it in items] == [sq.SQR_ENULL, sq.SQR_EDIM, sq.SQR_EOPT]
    bad = sq.sqr_default_opts(max_iter=0)
    assert sq.lib.sqr_batch(ctypes.byref(bad), items, 3, None) == sq.SQR_EOPT


def test_panel_usage_errors_before_any_gpu_work(sq):
    """sqr_panel (Algorithm 3) rejects r outside 1..n, a capacity above 16384
    and the mixed form before any HIP call."""
    h = ctypes.c_void_p()
    P = lambda: ctypes.c_void_p(0x1000)   # never dereferenced

    def panel(m, n, r, opts=None):
        return sq.lib.sqr_panel(ctypes.byref(h), ctypes.byref(opts) if opts else None, m, n, P(), m, r,
                                P(), m, n, P(), n, None, None)
    assert panel(100, 10, 0) == sq.SQR_EDIM
    assert panel(100, 10, 11) == sq.SQR_EDIM
    assert panel(10, 11, 2) == sq.SQR_EDIM
    assert panel(40000, 16385, 32) == sq.SQR_EDIM  # cap above 16384
    assert panel(100, 10, 2, sq.sqr_default_opts(precision=1)) == sq.SQR_EOPT
