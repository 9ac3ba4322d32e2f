"""Pins for the oracle's Arnoldi, GMRES(m), polynomial and GCRO-DR: dense LU,
brute-force Krylov least squares, closed forms, invariants."""
import os

import numpy as np
import pytest

import synth
from oracle import operator as dop
from oracle import poly
from oracle.gcrodr import RecycleState, gcrodr
from oracle.krylov import arnoldi, gmres

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_op(dims=(2, 2, 2, 2), ntv=4, m0=None, mu=0.0, seed=0):
    A0 = synth.self_blocks(dims, ntv, 0.0, seed).numpy()
    B = synth.hop_blocks(dims, ntv, seed).numpy()
    op0 = dop.build(dims, A0, B, 0.0)
    if m0 is None:
        # shift so that min Re eig = 0.05 * max |eig| (exact, dense)
        from oracle.calibrate_m0 import m0_root
        m0 = m0_root(np.linalg.eigvals(dop.dense(op0)), 0.05)
    A = A0 + m0 * np.eye(2 * ntv)
    return dop.build(dims, A, B, mu)


def flat(op):
    return lambda v: dop.apply(op, v.reshape(op.V, op.n)).reshape(-1)


def krylov_lstsq_residual(Dm, b, j):
    """Brute force: min over x in K_j(D, b) of ||b - D x|| via an explicit
    (orthonormalised) power basis."""
    K = np.empty((b.size, j), dtype=np.complex128)
    v = b.copy()
    for i in range(j):
        K[:, i] = v
        v = Dm @ v
    Q, _ = np.linalg.qr(K)
    AQ = Dm @ Q
    c = np.linalg.lstsq(AQ, b, rcond=None)[0]
    return b - AQ @ c


def test_arnoldi_relation_and_orthonormality():
    op = small_op()
    A = flat(op)
    rng = np.random.default_rng(0)
    v = rng.standard_normal(op.N) + 1j * rng.standard_normal(op.N)
    for ortho in ("mgs", "cgs", "cgs2"):
        ar = arnoldi(A, v, 12, ortho)
        Vm = np.stack(ar.V, 1)
        AV = np.stack([A(ar.V[i]) for i in range(12)], 1)
        assert np.allclose(AV, Vm @ ar.Hbar, atol=1e-12)
        assert np.allclose(Vm.conj().T @ Vm, np.eye(13), atol=1e-12)
        assert np.allclose(np.tril(ar.Hbar, -2), 0)


@pytest.mark.parametrize("j", [1, 3, 6])
def test_gmres_steps_equal_bruteforce_krylov_minimum(j):
    op = small_op()
    Dm = dop.dense(op)
    rng = np.random.default_rng(1)
    b = rng.standard_normal(op.N) + 1j * rng.standard_normal(op.N)
    x, info = gmres(flat(op), b, 1e-30, m=j, max_cycles=1)
    ref = krylov_lstsq_residual(Dm, b, j)
    assert info.iters == j
    r = b - Dm @ x
    assert np.allclose(r, ref, atol=1e-9 * np.linalg.norm(b))


@pytest.mark.parametrize("ortho", ["mgs", "cgs2"])
def test_gmres_restarted_matches_dense_lu(ortho):
    op = small_op(dims=(3, 2, 2, 2), ntv=4, mu=0.02)
    Dm = dop.dense(op)
    rng = np.random.default_rng(2)
    b = rng.standard_normal(op.N) + 1j * rng.standard_normal(op.N)
    xref = np.linalg.solve(Dm, b)
    x, info = gmres(flat(op), b, 1e-10, m=10, max_cycles=2000, ortho=ortho)
    assert info.converged
    assert np.linalg.norm(b - Dm @ x) <= 1e-10 * np.linalg.norm(b)
    kappa = np.linalg.cond(Dm)
    assert np.linalg.norm(x - xref) <= 2 * kappa * 1e-10 * np.linalg.norm(xref)
    # residual history is non-increasing across restarts (minimal residual)
    h = np.array(info.history)
    assert np.all(h[1:] <= h[:-1] * (1 + 1e-12))


def test_gmres_c1_workload_against_lu():
    """The 4^4, N_tv = 8 workload with its calibrated m0, GMRES(30), tol 1e-10."""
    w = synth.WORKLOADS["c1"]
    A, B = synth.operator(w)
    op = dop.build(w.dims, A.numpy(), B.numpy(), w.mu)
    b = synth.rhs(w.dims, w.n_tv, 0).numpy().reshape(-1)
    x, info = gmres(flat(op), b, 1e-10, m=30, max_cycles=5000)
    assert info.converged
    xref = np.linalg.solve(dop.dense(op), b)
    assert np.linalg.norm(x - xref) <= 1e-6 * np.linalg.norm(xref)


# ---------------------------------------------------------------- polynomial

def test_leja_golden_examples():
    """Hand-worked Leja orders (Alg. 2), tests/golden/leja_examples.txt."""
    with open(os.path.join(GOLDEN, "leja_examples.txt")) as f:
        lines = [l for l in f if l.strip() and not l.startswith("#")]
    for line in lines:
        inp, out = line.split("->")
        theta = np.array([complex(t) for t in inp.split()])
        want = np.array([complex(t) for t in out.split()])
        assert np.array_equal(poly.leja_order(theta), want), line


def test_harmonic_ritz_generalized_form():
    """Harmonic Ritz values also solve Hbar^H Hbar g = theta H_d^H g (the
    generalised form of the same Petrov-Galerkin condition)."""
    op = small_op()
    rng = np.random.default_rng(3)
    v = rng.standard_normal(op.N) + 1j * rng.standard_normal(op.N)
    ar = arnoldi(flat(op), v, 8)
    th = poly.harmonic_ritz(ar.Hbar)
    Hd = ar.Hbar[:8, :8]
    alt = np.linalg.eigvals(np.linalg.solve(Hd.conj().T, ar.Hbar.conj().T @ ar.Hbar))
    assert max(np.min(np.abs(alt - t)) for t in th) <= 1e-10
    assert max(np.min(np.abs(th - a)) for a in alt) <= 1e-10


@pytest.mark.parametrize("d", [2, 4, 8])
def test_residual_polynomial_equals_gmres_residual(d):
    """p_d(A) v0 with the harmonic Ritz roots is the GMRES(d) residual for
    b = v0, x0 = 0 (Sec. 3.3)."""
    op = small_op()
    Dm = dop.dense(op)
    rng = np.random.default_rng(4)
    v0 = rng.standard_normal(op.N) + 1j * rng.standard_normal(op.N)
    theta, _ = poly.build_polynomial(flat(op), v0, d)
    pv = poly.p_apply(flat(op), theta, v0)
    ref = krylov_lstsq_residual(Dm, v0, d)
    assert np.allclose(pv, ref, atol=1e-9 * np.linalg.norm(v0))
    # and 1 - t q(t) = p(t): v0 - A q(A) v0 = p(A) v0
    qv = poly.q_apply(flat(op), theta, v0)
    assert np.allclose(v0 - Dm @ qv, pv, atol=1e-9 * np.linalg.norm(v0))


def test_full_degree_polynomial_is_inverse():
    """d = N: the harmonic Ritz values are the eigenvalues and q(A) = A^{-1}."""
    op = small_op(dims=(2, 1, 1, 1), ntv=3)     # N = 12
    Dm = dop.dense(op)
    rng = np.random.default_rng(5)
    v0 = rng.standard_normal(op.N) + 1j * rng.standard_normal(op.N)
    theta, _ = poly.build_polynomial(flat(op), v0, op.N)
    ev = np.linalg.eigvals(Dm)
    assert max(np.min(np.abs(ev - t)) for t in theta) <= 1e-8
    assert max(np.min(np.abs(theta - e)) for e in ev) <= 1e-8
    v = rng.standard_normal(op.N) + 1j * rng.standard_normal(op.N)
    assert np.allclose(poly.q_apply(flat(op), theta, v), np.linalg.solve(Dm, v),
                       atol=1e-7 * np.linalg.norm(np.linalg.solve(Dm, v)))


def test_q_independent_of_ordering():
    op = small_op()
    rng = np.random.default_rng(6)
    v0 = rng.standard_normal(op.N) + 1j * rng.standard_normal(op.N)
    theta, _ = poly.build_polynomial(flat(op), v0, 6)
    v = rng.standard_normal(op.N) + 1j * rng.standard_normal(op.N)
    a = poly.q_apply(flat(op), theta, v)
    b = poly.q_apply(flat(op), theta[::-1], v)
    assert np.allclose(a, b, atol=1e-10 * np.linalg.norm(a))


def test_pp_gmres_with_block_jacobi_converges():
    op = small_op(dims=(3, 2, 2, 2), ntv=4, mu=0.05)
    Dm = dop.dense(op)
    rng = np.random.default_rng(7)
    b = rng.standard_normal(op.N) + 1j * rng.standard_normal(op.N)
    Binv = dop.block_jacobi_inverse(op)
    Bi = lambda v: dop.apply_block_jacobi(Binv, v.reshape(op.V, op.n)).reshape(-1)
    At = lambda v: Bi(flat(op)(v))
    v0 = rng.standard_normal(op.N) + 1j * rng.standard_normal(op.N)
    theta, _ = poly.build_polynomial(At, v0, 4)
    x, info = poly.pp_gmres(flat(op), b, 1e-10, 10, 500, theta, Binv_apply=Bi)
    assert info.converged
    assert np.linalg.norm(b - Dm @ x) <= 1e-10 * np.linalg.norm(b)
    x2, info2 = gmres(flat(op), b, 1e-10, 10, 5000)
    assert info.iters < info2.iters          # fewer (preconditioned) iterations


# ---------------------------------------------------------------- GCRO-DR

def test_gcrodr_k0_is_gmres():
    op = small_op(dims=(3, 2, 2, 2), ntv=4)
    rng = np.random.default_rng(8)
    b = rng.standard_normal(op.N) + 1j * rng.standard_normal(op.N)
    x1, i1 = gmres(flat(op), b, 1e-10, 12, 500)
    x2, i2 = gcrodr(flat(op), b, 1e-10, 12, 0, 10, 500, RecycleState())
    assert i1.iters == i2.iters
    assert np.allclose(x1, x2, atol=1e-12 * np.linalg.norm(x1))


def test_gcrodr_invariants_and_recycling():
    op = small_op(dims=(3, 2, 2, 2), ntv=4, mu=0.01)
    Dm = dop.dense(op)
    A = flat(op)
    rng = np.random.default_rng(9)
    st = RecycleState()
    iters = []
    for r in range(3):
        b = rng.standard_normal(op.N) + 1j * rng.standard_normal(op.N)
        x, info = gcrodr(A, b, 1e-10, 20, 6, 10, 500, st)
        assert info.converged
        assert np.linalg.norm(b - Dm @ x) <= 1e-10 * np.linalg.norm(b)
        # C = A U with orthonormal columns
        assert np.allclose(st.C.conj().T @ st.C, np.eye(6), atol=1e-10)
        assert np.allclose(Dm @ st.U, st.C, atol=1e-9 * np.abs(st.C).max())
        iters.append(info.iters)
        # residual orthogonal to the deflation space after projection
        rr = b - Dm @ x
        c_proj = st.C.conj().T @ (rr - st.C @ (st.C.conj().T @ rr))
        assert np.linalg.norm(c_proj) <= 1e-10 * np.linalg.norm(rr)
    assert iters[2] < iters[0]                 # recycled space helps


def test_gcrodr_residual_orthogonal_to_c_each_cycle():
    """C^H r_hat = 0 after every cycle, for the C in use after that cycle
    (refreshed or frozen)."""
    op = small_op(dims=(3, 2, 2, 2), ntv=4)
    A = flat(op)
    rng = np.random.default_rng(10)
    for u in (10, 2):
        st = RecycleState()
        b = rng.standard_normal(op.N) + 1j * rng.standard_normal(op.N)
        for cyc in range(1, 6):
            st_c = RecycleState()
            st_c.U, st_c.C, st_c.updates = st.U, st.C, st.updates
            x, info = gcrodr(A, b, 1e-14, 16, 5, u, cyc, st_c)
            rh = info.final_rhat
            # rounding accumulates relative to the starting residual, not the current one
            assert np.linalg.norm(st_c.C.conj().T @ rh) <= 1e-12 * np.linalg.norm(b)
            assert np.linalg.norm(st_c.C.conj().T @ rh) <= 1e-6 * np.linalg.norm(rh)


def test_gcrodr_exact_eigenvectors_when_m_ge_N():
    op = small_op(dims=(2, 1, 1, 1), ntv=3)   # N = 12
    Dm = dop.dense(op)
    A = flat(op)
    rng = np.random.default_rng(11)
    b = rng.standard_normal(op.N) + 1j * rng.standard_normal(op.N)
    st = RecycleState()
    # first cycle runs at least k steps; m = N makes the Krylov space invariant
    x, info = gcrodr(A, b, 1e-13, op.N, 3, 10, 50, st)
    assert info.converged
    ev = np.linalg.eigvals(Dm)
    smallest = ev[np.argsort(np.abs(ev))[:3]]
    # span(U) is the invariant subspace of the 3 smallest-|lambda| eigenvalues
    U = st.U
    M = np.linalg.lstsq(U, Dm @ U, rcond=None)[0]
    assert np.linalg.norm(Dm @ U - U @ M) <= 1e-8 * np.linalg.norm(Dm @ U)
    got = np.linalg.eigvals(M)
    assert max(np.min(np.abs(smallest - g)) for g in got) <= 1e-8
    assert max(np.min(np.abs(got - s)) for s in smallest) <= 1e-8


def _refresh_subspace_error(eig_fn=None):
    """One GCRO-DR cycle whose Vhat = [U D_k, V_{m-k}] spans the whole space
    (m - k = N - k deflated Arnoldi steps, breaking down on the invariant
    complement of span(C)), followed by the recycle refresh from the
    generalised problem G^H G z = theta G^H (What^H Vhat) z.  With Vhat
    spanning C^N the harmonic Ritz pairs are exact eigenpairs, so the
    refreshed span(U) must be the invariant subspace of the k smallest-|lambda|
    eigenvalues.  Returns the largest of: the eigenvalue mismatch of U's
    Rayleigh-Ritz matrix and the relative invariance residual."""
    import oracle.gcrodr as gc
    op = small_op(dims=(3, 1, 1, 1), ntv=2)      # N = 12
    Dm = dop.dense(op)
    A = flat(op)
    N, k = op.N, 3
    rng = np.random.default_rng(21)
    st = RecycleState()
    # a recycle space that is not invariant: random U, C from qr(A U) (the
    # matrix-changed path), one update already counted
    st.U = rng.standard_normal((N, k)) + 1j * rng.standard_normal((N, k))
    st.C = np.zeros_like(st.U)
    st.updates = 1
    b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    saved = gc.sla
    if eig_fn is not None:
        class _Fake:
            eig = staticmethod(eig_fn)
        gc.sla = _Fake
    try:
        _, info = gcrodr(A, b, 1e-15, N, k, 10, 1, st, matrix_changed=True)
    finally:
        gc.sla = saved
    assert info.cycles == 1 and st.updates == 2
    ev = np.linalg.eigvals(Dm)
    smallest = ev[np.argsort(np.abs(ev))[:k]]
    U = st.U
    M = np.linalg.lstsq(U, Dm @ U, rcond=None)[0]
    inv_res = np.linalg.norm(Dm @ U - U @ M) / np.linalg.norm(Dm @ U)
    got = np.linalg.eigvals(M)
    mism = max(max(np.min(np.abs(smallest - g)) for g in got),
               max(np.min(np.abs(got - s_)) for s_ in smallest))
    return max(inv_res, mism / np.abs(smallest).max())


def test_gcrodr_refresh_recovers_invariant_subspace():
    """Pins the refresh step's generalised eigenproblem and its selection
    (Sec. 3.4; Parks et al. update): exact when Vhat spans everything."""
    assert _refresh_subspace_error() <= 1e-8


@pytest.mark.parametrize("mistake", ["no_rhs_matrix", "swapped", "conjugated"])
def test_gcrodr_refresh_pin_detects_wrong_eigenproblem(mistake):
    """Mistakes planted in the oracle's refresh (on the CPU) must fail the pin
    above: dropping What^H Vhat, swapping the two matrices (which selects the
    largest |theta|), or conjugating the problem."""
    import scipy.linalg as sla
    wrong = {"no_rhs_matrix": lambda a, b: sla.eig(a),
             "swapped": lambda a, b: sla.eig(b, a),
             "conjugated": lambda a, b: sla.eig(a.conj(), b.conj())}[mistake]
    assert _refresh_subspace_error(wrong) > 1e-3
