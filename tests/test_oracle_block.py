"""Pins of the oracle's block GMRES: one column reduces to GMRES, the block
Arnoldi relation and orthonormality, the minimal-residual property over the
block space (never worse than GMRES on one column alone), an exact solve once
the block space fills the whole space, and per-column tolerances against dense
solves on a small coarse operator."""
import numpy as np
import pytest

import synth
from oracle import operator as dop
from oracle.block import block_arnoldi, block_gmres
from oracle.krylov import arnoldi, gmres


def _matrix(N=40, seed=0):
    rng = np.random.default_rng(seed)
    M = (2.5 * np.eye(N) + rng.standard_normal((N, N)) / np.sqrt(N)
         + 1j * rng.standard_normal((N, N)) / np.sqrt(N))
    return M, rng


def test_single_column_is_gmres():
    M, rng = _matrix()
    b = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    Xb, ib = block_gmres(lambda v: M @ v, b[:, None], [1e-10], 8, 200)
    xg, ig = gmres(lambda v: M @ v, b, 1e-10, 8, 200)
    assert ib["converged"] and ig.converged
    assert ib["cycles"] == ig.cycles
    assert np.linalg.norm(Xb[:, 0] - xg) <= 1e-9 * np.linalg.norm(xg)


def test_block_arnoldi_relation():
    M, rng = _matrix(seed=1)
    R0 = rng.standard_normal((40, 3)) + 1j * rng.standard_normal((40, 3))
    V, Hb, S0, j, _ = block_arnoldi(lambda W: M @ W, R0, 5)
    Vm = np.concatenate(V, axis=1)
    assert j == 5 and Vm.shape == (40, 18)
    assert np.abs(Vm.conj().T @ Vm - np.eye(18)).max() <= 1e-12
    assert np.abs(M @ Vm[:, :15] - Vm @ Hb).max() <= 1e-12 * np.abs(M).max()
    assert np.abs(V[0] @ S0 - R0).max() <= 1e-12 * np.abs(R0).max()
    # block upper Hessenberg: nothing below the first block subdiagonal
    assert np.abs(np.tril(Hb, -4)).max() == 0.0


def test_block_space_beats_single_column_gmres():
    """One cycle of m block steps from X = 0: each column's residual is the
    minimum over the block space, which contains that column's own Krylov
    space, so it is at most GMRES(m)'s after its first cycle."""
    M, rng = _matrix(N=60, seed=2)
    A = lambda v: M @ v
    B = rng.standard_normal((60, 4)) + 1j * rng.standard_normal((60, 4))
    m = 6
    Xb, _ = block_gmres(A, B, [1e-30] * 4, m, 1)
    for c in range(4):
        ar = arnoldi(A, B[:, c], m, "mgs")
        e1 = np.zeros(m + 1, dtype=np.complex128)
        e1[0] = np.linalg.norm(B[:, c])
        y = np.linalg.lstsq(ar.Hbar, e1, rcond=None)[0]
        xg = sum(y[i] * ar.V[i] for i in range(m))
        rb = np.linalg.norm(B[:, c] - M @ Xb[:, c])
        rg = np.linalg.norm(B[:, c] - M @ xg)
        assert rb <= rg * (1 + 1e-10)
        assert rb < 0.9 * rg      # and strictly better with 4 columns sharing the space


def test_exact_once_the_space_is_full():
    M, rng = _matrix(N=24, seed=3)
    B = rng.standard_normal((24, 4)) + 1j * rng.standard_normal((24, 4))
    X, info = block_gmres(lambda v: M @ v, B, [1e-13] * 4, 6, 1)   # 6 x 4 = 24
    assert np.abs(M @ X - B).max() <= 1e-11 * np.abs(B).max()


def test_per_column_tolerances_on_coarse_operator():
    dims, ntv = (2, 2, 2, 2), 4
    A = synth.self_blocks(dims, ntv, 3.0, 0).numpy()
    Bh = synth.hop_blocks(dims, ntv, 0).numpy()
    op = dop.build(dims, A, Bh, 0.1)
    D = dop.dense(op)
    rng = np.random.default_rng(4)
    N = op.V * op.n
    B = rng.standard_normal((N, 5)) + 1j * rng.standard_normal((N, 5))
    tols = np.array([1e-10, 1e-8, 1e-6, 1e-9, 1e-7])
    f = lambda v: dop.apply(op, v.reshape(op.V, op.n)).reshape(-1)
    X, info = block_gmres(f, B, tols, 20, 100)
    assert info["converged"]
    rel = np.linalg.norm(B - D @ X, axis=0) / np.linalg.norm(B, axis=0)
    assert np.all(rel <= tols)
    Xr = np.linalg.solve(D, B)
    assert np.linalg.norm(X[:, 0] - Xr[:, 0]) <= 1e-7 * np.linalg.norm(Xr[:, 0])
