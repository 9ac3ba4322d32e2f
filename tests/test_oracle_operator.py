"""Pins for the oracle's coarse-operator apply: FFT closed form, Gamma5
hermiticity, the adjoint identity, degenerate lattice extents."""
import numpy as np
import pytest

import synth
from oracle import operator as dop
from oracle.lattice import coords, neighbours


def random_op(dims, ntv, m0=3.0, mu=0.0, seed=0):
    A = synth.self_blocks(dims, ntv, m0, seed).numpy()
    B = synth.hop_blocks(dims, ntv, seed).numpy()
    return dop.build(dims, A, B, mu)


def test_neighbour_tables_periodic():
    dims = (3, 4, 2, 5)
    fwd, bwd = neighbours(dims)
    c = coords(dims)
    V = c.shape[0]
    for mu in range(4):
        # x + mu - mu = x and the coordinate moves by exactly one, periodically
        assert np.array_equal(bwd[mu][fwd[mu]], np.arange(V))
        d = (c[fwd[mu]] - c) % np.array(dims)
        e = np.zeros(4, dtype=np.int64)
        e[mu] = 1 % dims[mu]
        assert np.all(d == e)


@pytest.mark.parametrize("dims", [(4, 3, 2, 5), (2, 2, 2, 2), (1, 3, 2, 1)])
def test_apply_translation_invariant_fft(dims):
    """All A_x = A and B_{x,mu} = B_mu: the operator is diagonalised by the
    lattice Fourier transform, D(p) = A + sum_mu (B_mu e^{i p_mu}
    + G5 B_mu^H G5 e^{-i p_mu}), p_mu = 2 pi k_mu / L_mu."""
    rng = np.random.default_rng(11)
    n = 6
    V = int(np.prod(dims))
    A1 = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    B1 = rng.standard_normal((4, n, n)) + 1j * rng.standard_normal((4, n, n))
    mu_tm = 0.3
    op = dop.build(dims, np.broadcast_to(A1, (V, n, n)),
                   np.broadcast_to(B1, (V, 4, n, n)), mu_tm)
    psi = rng.standard_normal((V, n)) + 1j * rng.standard_normal((V, n))
    out = dop.apply(op, psi)
    # Fourier side.  Site order is x0 fastest: lattice array index [x3,x2,x1,x0].
    shape = tuple(reversed(dims))
    ph = np.fft.fftn(psi.reshape(shape + (n,)), axes=(0, 1, 2, 3))
    G = np.diag(np.r_[np.ones(n // 2), -np.ones(n // 2)])
    A_tm = A1 + 1j * mu_tm * G
    ks = np.meshgrid(*[np.arange(L) for L in shape], indexing="ij")
    res = np.einsum("ij,...j->...i", A_tm, ph)
    for mu in range(4):
        axis = 3 - mu
        p = 2 * np.pi * ks[axis] / shape[axis]
        fwd = np.einsum("ij,...j->...i", B1[mu], ph)
        bwd = np.einsum("ij,...j->...i", G @ B1[mu].conj().T @ G, ph)
        res += np.exp(1j * p)[..., None] * fwd + np.exp(-1j * p)[..., None] * bwd
    ref = np.fft.ifftn(res, axes=(0, 1, 2, 3)).reshape(V, n)
    assert np.allclose(out, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("dims", [(2, 3, 2, 2), (1, 2, 3, 1)])
def test_gamma5_hermiticity_dense(dims):
    ntv = 3
    op = random_op(dims, ntv, mu=0.0)
    D = dop.dense(op)
    G = np.kron(np.eye(op.V), np.diag(dop.gamma5(op.n)))
    if min(dims) >= 2:
        # exact: sign flips and two-term sums, which commute
        assert np.array_equal(G @ D @ G, D.conj().T)
    else:
        assert np.allclose(G @ D @ G, D.conj().T, rtol=0, atol=1e-15)
    # twisted mass: G5 D(mu) G5 = D(-mu)^H
    opm = random_op(dims, ntv, mu=0.25)
    Dm = dop.dense(opm)
    Dneg = dop.dense(dop.with_mu(opm, -0.25))
    assert np.allclose(G @ Dm @ G, Dneg.conj().T, rtol=0, atol=1e-15)


@pytest.mark.parametrize("dims", [(2, 3, 2, 2), (2, 1, 1, 3), (3, 3, 3, 3)])
def test_apply_equals_dense_and_bsr(dims):
    op = random_op(dims, 2, mu=0.1)
    rng = np.random.default_rng(2)
    psi = rng.standard_normal((op.V, op.n)) + 1j * rng.standard_normal((op.V, op.n))
    out = dop.apply(op, psi).reshape(-1)
    D = dop.dense(op)
    assert np.allclose(out, D @ psi.reshape(-1), rtol=0, atol=1e-13)
    assert np.allclose(out, dop.bsr(op) @ psi.reshape(-1), rtol=0, atol=1e-13)


def test_adjoint_identity():
    op = random_op((3, 2, 2, 2), 3, mu=0.2)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((op.V, op.n)) + 1j * rng.standard_normal((op.V, op.n))
    y = rng.standard_normal((op.V, op.n)) + 1j * rng.standard_normal((op.V, op.n))
    lhs = np.vdot(dop.apply_adjoint(op, y), x)
    rhs = np.vdot(y, dop.apply(op, x))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)
    D = dop.dense(op)
    assert np.allclose(dop.apply_adjoint(op, y).reshape(-1), D.conj().T @ y.reshape(-1),
                       atol=1e-13)


def test_block_jacobi_inverse():
    op = random_op((2, 2, 2, 2), 2, mu=0.3)
    Binv = dop.block_jacobi_inverse(op)
    eye = np.eye(op.n)
    assert np.allclose(np.einsum("sij,sjk->sik", Binv, op.A), eye, atol=1e-12)


@pytest.mark.parametrize("dims", [(3, 2, 4, 2), (2, 1, 3, 3)])
def test_apply_site_matches_dense_rows(dims):
    """The single-site stencil (used for sampled checks of large lattices)
    reproduces the rows of the assembled dense matrix, twisted mass and
    periodic wrap included."""
    ntv, mu = 3, 0.07
    A0 = synth.self_blocks(dims, ntv, 2.8, 4).numpy()
    B = synth.hop_blocks(dims, ntv, 4).numpy()
    op = dop.build(dims, A0, B, mu)
    D = dop.dense(op)
    rng = np.random.default_rng(5)
    psi = rng.standard_normal((op.V, op.n)) + 1j * rng.standard_normal((op.V, op.n))
    full = (D @ psi.reshape(-1)).reshape(op.V, op.n)
    fwd, bwd = neighbours(dims)
    for x in range(op.V):
        out = dop.apply_site(A0[x], B[x], np.stack([B[bwd[m, x], m] for m in range(4)]),
                             psi[x], psi[fwd[:, x]], psi[bwd[:, x]], mu)
        assert np.allclose(out, full[x], rtol=0, atol=1e-13)
