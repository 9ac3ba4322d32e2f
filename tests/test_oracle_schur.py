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


# ------------------------------------------------ block Jacobi on the reduced system

def _dense_bj(op):
    """B^{-1} S assembled densely: B = blockdiag(D_ee) inverted with
    numpy.linalg.inv on the assembled block diagonal (independent of dinv_ee)."""
    S = schur.dense(op)
    Ae = op.A[schur.sites(op.dims, 0)]
    n = op.n
    Bd = np.zeros_like(S)
    for i, a in enumerate(Ae):
        Bd[i * n:(i + 1) * n, i * n:(i + 1) * n] = a
    return np.linalg.inv(Bd) @ S, Bd


@pytest.mark.parametrize("mu", [0.0, 0.15])
def test_bj_apply_matches_dense(mu):
    """Sec. 3.2: B = D_ee for the reduced system; B^{-1} S against the dense
    block elimination and a dense inverse of the block diagonal."""
    op = make((2, 4, 2, 2), 2, mu=mu)
    M, Bd = _dense_bj(op)
    rng = np.random.default_rng(3)
    ne = op.V // 2
    x = rng.standard_normal((ne, op.n)) + 1j * rng.standard_normal((ne, op.n))
    assert np.allclose(schur.apply_bj(op, x).reshape(-1), M @ x.reshape(-1), rtol=0, atol=1e-12)
    assert np.allclose(schur.dinv_ee(op, x).reshape(-1), np.linalg.solve(Bd, x.reshape(-1)),
                       rtol=0, atol=1e-12)


def test_bj_polynomial_is_built_from_preconditioned_operator():
    """d = dim: the harmonic Ritz values of B^{-1} S are its exact eigenvalues
    (Sec. 3.3, polynomial of the left-preconditioned operator); they differ
    from the eigenvalues of S, so building q from S instead would fail."""
    from oracle import poly
    op = make((2, 2, 2, 2), 2, m0=2.6)
    M, _ = _dense_bj(op)
    S = schur.dense(op)
    N = M.shape[0]
    rng = np.random.default_rng(4)
    v0 = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    ne = op.V // 2
    At = lambda v: schur.apply_bj(op, v.reshape(ne, op.n)).reshape(-1)
    theta, _ = poly.build_polynomial(At, v0, N)
    ev = np.linalg.eigvals(M)
    # the N-th step's h_{N+1,N} is rounding (~1e-8), not zero: harmonic Ritz
    # values within ~1e-6 of the eigenvalues
    assert max(np.min(np.abs(ev - t)) for t in theta) <= 1e-5 * np.abs(ev).max()
    evs = np.linalg.eigvals(S)
    assert max(np.min(np.abs(evs - t)) for t in theta) > 1e-1


@pytest.mark.parametrize("mu,d", [(0.0, 4), (0.1, 4), (0.0, 1)])
def test_bj_poly_gcrodr_method_matches_lu(mu, d):
    """The paper's coarsest-level method on the reduced system (left block
    Jacobi + polynomial of B^{-1} S + GCRO-DR with recycling) against dense LU
    for three right-hand sides in a row, with the recycle invariants of the
    preconditioned operator A^ = B^{-1} S q(B^{-1} S): C = A^ U, C^H C = I."""
    from oracle import poly
    from oracle.gcrodr import RecycleState
    op = make((4, 2, 2, 2), 3, m0=3.1, mu=mu)
    Dm = dop.dense(op)
    M, _ = _dense_bj(op)
    rng = np.random.default_rng(5)
    st = RecycleState()
    ne = op.V // 2
    v0 = rng.standard_normal(ne * op.n) + 1j * rng.standard_normal(ne * op.n)
    for r in range(3):
        b = rng.standard_normal((op.V, op.n)) + 1j * rng.standard_normal((op.V, op.n))
        x, info, theta = schur.solve_method(op, b, 1e-11, m=16, k=4, d=d, u=10, state=st, v0=v0)
        assert info.converged
        xref = np.linalg.solve(Dm, b.reshape(-1))
        assert np.linalg.norm(b.reshape(-1) - Dm @ x.reshape(-1)) <= 1e-11 * np.linalg.norm(b) * 1.0001
        assert np.linalg.norm(x.reshape(-1) - xref) <= 1e-8 * np.linalg.norm(xref)
        assert np.allclose(st.C.conj().T @ st.C, np.eye(4), atol=1e-10)
        if d > 1:
            qU = np.stack([poly.q_apply(lambda v: M @ v, theta, st.U[:, i]) for i in range(4)], 1)
        else:
            qU = st.U
        assert np.linalg.norm(M @ qU - st.C) <= 1e-8 * np.linalg.norm(st.C)
