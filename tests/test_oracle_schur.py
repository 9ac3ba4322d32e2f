"""Pins of the oracle's odd-even reduction (Sec. 2.2): the matrix-free Schur
apply against block elimination of the dense matrix, the reduced solve against
dense LU, Gamma5-hermiticity, and the compressed parity order."""
import numpy as np
import pytest

import synth
from oracle import operator as dop
from oracle import schur
from oracle.lattice import coords


def make(dims, ntv, m0=3.0, mu=0.0, seed=0):
    A = synth.self_blocks(dims, ntv, m0, seed).numpy()
    B = synth.hop_blocks(dims, ntv, seed).numpy()
    return dop.build(dims, A, B, mu)


def test_compressed_order_is_site_halving():
    dims = (4, 2, 2, 6)
    par = schur.parity(dims)
    c = coords(dims)
    assert np.array_equal(par, c.sum(axis=1) % 2)
    for p in (0, 1):
        s = schur.sites(dims, p)
        assert np.array_equal(s // 2, np.arange(len(s)))
    with pytest.raises(ValueError):
        schur.parity((3, 2, 2, 2))


@pytest.mark.parametrize("dims,mu", [((2, 2, 2, 2), 0.0), ((4, 2, 2, 2), 0.2), ((2, 4, 2, 4), 0.0)])
def test_apply_matches_dense_elimination(dims, mu):
    op = make(dims, 2, mu=mu)
    S = schur.dense(op)
    rng = np.random.default_rng(1)
    ne = op.V // 2
    x = rng.standard_normal((ne, op.n)) + 1j * rng.standard_normal((ne, op.n))
    assert np.allclose(schur.apply(op, x).reshape(-1), S @ x.reshape(-1), rtol=0, atol=1e-12)


def test_gamma5_hermiticity():
    op = make((2, 2, 2, 2), 3)
    S = schur.dense(op)
    g = np.tile(dop.gamma5(op.n), op.V // 2)
    assert np.allclose(g[:, None] * S * g[None, :], S.conj().T, rtol=0, atol=1e-12)


@pytest.mark.parametrize("mu", [0.0, 0.1])
def test_reduced_solve_matches_lu(mu):
    op = make((4, 2, 2, 2), 3, m0=3.2, mu=mu)
    rng = np.random.default_rng(2)
    b = rng.standard_normal((op.V, op.n)) + 1j * rng.standard_normal((op.V, op.n))
    x, info = schur.solve(op, b, 1e-12, m=20)
    xref = np.linalg.solve(dop.dense(op), b.reshape(-1)).reshape(op.V, op.n)
    r = b - dop.apply(op, x)
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(b) * 1.0001
    assert np.linalg.norm(x - xref) <= 1e-9 * np.linalg.norm(xref)
    # the odd rows of the residual vanish up to rounding
    _, r_o = schur.split(op, r)
    assert np.linalg.norm(r_o) <= 1e-13 * np.linalg.norm(b)
