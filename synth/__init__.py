"""Seeded synthetic inputs shaped like the paper's test matrices.

Shared by the tests, the benchmark and the smoke check, on both sides of every
parity comparison.  This module holds none of the Cholesky QR arithmetic: it
only draws Gaussian numbers and orthonormalises them with LAPACK's Householder
QR (numpy.linalg.qr), which the method under test does not use.

Recipe (Sec. 3.1, test matrices A := U Sigma V): U (m x n) and V (n x n) are the
positive-diagonal Q factors of seeded standard-normal matrices, Sigma holds
values log-spaced from 1 down to 1/kappa, and A = U diag(s) V^T in FP64.
"""
from __future__ import annotations

import math

import numpy as np


def rng(*key: int) -> np.random.Generator:
    """PCG64 generator seeded by SeedSequence(key)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(
        [int(k) for k in key])))


def orthonormal(g: np.random.Generator, m: int, n: int) -> np.ndarray:
    """Positive-diagonal Q factor of an m x n standard-normal matrix."""
    G = g.standard_normal((m, n))
    Q, R = np.linalg.qr(G)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


def singular_values(n: int, kappa: float) -> np.ndarray:
    """n values log-spaced from 1 down to 1/kappa."""
    if n == 1:
        return np.ones(1)
    return np.logspace(0.0, -math.log10(kappa), n)


def test_matrix(m: int, n: int, kappa: float, seed=(0,)) -> np.ndarray:
    """A = U diag(s) V^T with cond_2(A) = kappa (Fortran order, FP64)."""
    g = rng(*seed, m, n, int(round(math.log10(kappa) * 100)))
    U = orthonormal(g, m, n)
    V = orthonormal(g, n, n)
    s = singular_values(n, kappa)
    return np.asfortranarray((U * s) @ V.T)


def test_matrix_device(m: int, n: int, kappa: float, seed=(0,), device="cuda",
                       max_elems: int = (1 << 31) - 1):
    """The same recipe drawn and formed on a GPU, for sizes the host cannot
    hold comfortably (m up to 2e7): torch's Gaussian generator seeded from
    SeedSequence(seed, m, n, kappa), Householder QR (torch.linalg.qr) for the
    orthonormal factors, GEMMs for U diag(s) V^T.  Returns an m x n FP64
    column-major tensor (a transposed view of an n x m contiguous tensor).
    Not bit-identical to test_matrix (a different random stream).

    The QR and GEMM libraries behind torch index with 32-bit integers, so no
    operand handed to them exceeds 2^31 elements: the tall factor U is a
    two-level Householder QR over row blocks (QR of each block, QR of the
    stacked R factors, Q_i times its piece of the second Q), and the product
    is formed block by block (max_elems bounds every operand)."""
    import torch
    key = np.random.SeedSequence([int(k) for k in seed] + [m, n, int(round(math.log10(kappa) * 100))])
    gen = torch.Generator(device=device)
    gen.manual_seed(int(key.generate_state(1, dtype=np.uint64)[0] >> np.uint64(1)))
    f64 = torch.float64
    lim = max_elems

    def house(G):
        assert G.numel() <= lim
        Q, R = torch.linalg.qr(G)
        return Q, R

    V, Rv = house(torch.randn((n, n), generator=gen, device=device, dtype=f64))
    dv = torch.sign(torch.diagonal(Rv))
    dv[dv == 0] = 1.0
    V = V * dv
    s = torch.as_tensor(singular_values(n, kappa), device=device, dtype=f64)
    SVt = (s[:, None] * V.t()).contiguous()          # diag(s) V^T, n x n

    rows = max(n, min(m, lim // max(n, 1)))           # rows per block
    starts = list(range(0, m, rows))
    Qs, Rs = [], []
    for r0 in starts:
        r1 = min(m, r0 + rows)
        Qi, Ri = house(torch.randn((r1 - r0, n), generator=gen, device=device, dtype=f64))
        Qs.append(Qi)
        Rs.append(Ri)
    Q2, R2 = house(torch.cat(Rs, 0))                  # (blocks * n) x n
    d = torch.sign(torch.diagonal(R2))
    d[d == 0] = 1.0
    out = torch.empty((n, m), device=device, dtype=f64).t()
    for i, r0 in enumerate(starts):
        r1 = min(m, r0 + rows)
        Ui = Qs[i] @ (Q2[i * n:(i + 1) * n] * d)      # block of U, positive diag
        Qs[i] = None
        out[r0:r1] = Ui @ SVt
        del Ui
    return out


def growth_blocks(m: int, n0: int, p: int, nblocks: int, kappa_lo: float,
                  kappa_hi: float, coupling: float = 1e-3, seed: int = 2):
    """Inputs of an iterative basis-growth run.

    Returns (A0, [W_1..W_nblocks], kappas).  A0 (m x n0) has kappa = 1e2.
    Block k is U_k diag(s_k) V_k^T + coupling * [U_0 .. U_{k-1}] G_k, with
    kappa_k log-uniform in [kappa_lo, kappa_hi] and G_k Gaussian: the second
    term ties each block to the span of all earlier blocks, so new columns are
    nearly dependent on the basis grown so far.
    """
    g0 = rng(seed, 0, m, n0)
    U0 = orthonormal(g0, m, n0)
    V0 = orthonormal(g0, n0, n0)
    A0 = np.asfortranarray((U0 * singular_values(n0, 1e2)) @ V0.T)
    Uall = np.empty((m, n0 + nblocks * p), order="F")
    Uall[:, :n0] = U0
    blocks, kappas = [], []
    for k in range(1, nblocks + 1):
        g = rng(seed, k, m, p)
        lk = g.uniform(math.log10(kappa_lo), math.log10(kappa_hi))
        kappa = 10.0 ** lk
        Uk = orthonormal(g, m, p)
        Vk = orthonormal(g, p, p)
        q = n0 + (k - 1) * p
        Gk = g.standard_normal((q, p))
        W = (Uk * singular_values(p, kappa)) @ Vk.T + coupling * (Uall[:, :q] @ Gk)
        blocks.append(np.asfortranarray(W))
        kappas.append(kappa)
        Uall[:, q:q + p] = Uk
    return A0, blocks, kappas


def hadamard(m: int) -> np.ndarray:
    """Sylvester Hadamard matrix of order m (a power of two); H^T H = m I."""
    assert m >= 1 and (m & (m - 1)) == 0
    H = np.ones((1, 1))
    while H.shape[0] < m:
        H = np.block([[H, H], [H, -H]])
    return H
