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


def _krylov_min(A, K, r):
    """min_y || r - A K y || by brute force (dense least squares)."""
    AK = np.stack([A(K[:, i]) for i in range(K.shape[1])], axis=1)
    y = np.linalg.lstsq(AK, r, rcond=None)[0]
    return np.linalg.norm(r - AK @ y)


def _dependent_block(N=60, seed=5):
    M, rng = _matrix(N=N, seed=seed)
    base = rng.standard_normal((N, 3)) + 1j * rng.standard_normal((N, 3))
    mix = rng.standard_normal((3, 4)) + 1j * rng.standard_normal((3, 4))
    # three independent columns and four combinations of them, each with a
    # part outside their span of relative size 1e-7 (dependent at 1e-12)
    noise = rng.standard_normal((N, 4)) + 1j * rng.standard_normal((N, 4))
    dep = base @ mix + 1e-7 * np.linalg.norm(base @ mix, axis=0) * noise / np.linalg.norm(noise, axis=0)
    return M, np.concatenate([base, dep], axis=1)


def test_dependent_columns_select_generators():
    from oracle.block import select_generators
    M, B = _dependent_block()
    picks = select_generators(B, 1e-12)
    assert picks.size == 3
    # the picks span the block to within the planted 1e-7 parts
    Q, _ = np.linalg.qr(B[:, picks])
    res = np.linalg.norm(B - Q @ (Q.conj().T @ B), axis=0) / np.linalg.norm(B, axis=0)
    assert res.max() <= 2e-7
    assert select_generators(B, 1e-16).size == 7       # a looser threshold keeps all


def test_dependent_columns_minimise_over_generated_space():
    """Residual columns that are numerically dependent generate the space from
    3 picks (the cycle runs 4 x 7 / 3 = 9 block steps, keeping the space's
    dimension); every one of the 7 columns gets its exact least-squares
    minimum over A times that space, including the parts of its residual
    outside the first block (brute-force least squares)."""
    from oracle.block import select_generators
    M, B = _dependent_block()
    A = lambda v: M @ v
    m = 4
    X, info = block_gmres(A, B, [1e-30] * 7, m, 1)
    assert info["generators"] == [3]
    assert info["steps"] == m * 7 // 3        # the space keeps dimension m x 7
    V0, _ = np.linalg.qr(B[:, select_generators(B, 1e-12)])
    K = [V0]
    for _ in range(info["steps"] - 1):
        Q, _ = np.linalg.qr(M @ K[-1])
        K.append(Q)
    K = np.concatenate(K, axis=1)
    for c in range(7):
        got = np.linalg.norm(B[:, c] - M @ X[:, c])
        best = _krylov_min(A, K, B[:, c])
        assert abs(got - best) <= 1e-8 * best + 1e-13 * np.linalg.norm(B[:, c])


def test_dropping_outside_parts_is_detected():
    """A mistake planted in the oracle (least squares with only the first
    block's coefficients V_0^H r, the parts of r outside V_0 dropped) leaves
    the dependent columns short of their minimum: the pin above catches it."""
    import oracle.block as ob
    M, B = _dependent_block()
    B = B.copy()
    nz = np.random.default_rng(9).standard_normal((60, 4))
    # parts of relative size 3e-2 outside the picks (dependent at sel_piv 1e-2)
    B[:, 3:] += 3e-2 * np.linalg.norm(B[:, 3:], axis=0) * nz / np.linalg.norm(nz, axis=0)
    A = lambda v: M @ v
    saved = ob.ls_rhs
    ob.ls_rhs = lambda V, R: np.concatenate(
        [V[0].conj().T @ R] + [np.zeros((Vb.shape[1], R.shape[1]), complex) for Vb in V[1:]], 0)
    try:
        X, info = ob.block_gmres(A, B, [1e-30] * 7, 4, 1, sel_piv=1e-2)
    finally:
        ob.ls_rhs = saved
    Xf, info_f = ob.block_gmres(A, B, [1e-30] * 7, 4, 1, sel_piv=1e-2)
    assert info["generators"] == info_f["generators"] == [3]
    worse = [np.linalg.norm(B[:, c] - M @ X[:, c]) / np.linalg.norm(B[:, c] - M @ Xf[:, c])
             for c in range(3, 7)]
    assert max(worse) > 1.2


def test_deflated_block_cycle_is_minimal_over_recycled_and_krylov_space():
    """Deflation against a recycled pair (U, C = A U orthonormal): after one
    cycle every column's residual is orthogonal to C and minimal over
    A span(U, K_m((I - C C^H) A, R_0 deflated)) (brute force)."""
    M, rng = _matrix(N=50, seed=6)
    A = lambda v: M @ v
    Uu = rng.standard_normal((50, 4)) + 1j * rng.standard_normal((50, 4))
    C, Rr = np.linalg.qr(M @ Uu)
    U = Uu @ np.linalg.inv(Rr)                      # C = A U exactly
    B = rng.standard_normal((50, 3)) + 1j * rng.standard_normal((50, 3))
    m = 3
    X, info = block_gmres(A, B, [1e-30] * 3, m, 1, U=U, C=C)
    R0 = B - C @ (C.conj().T @ B)
    P = lambda W: W - C @ (C.conj().T @ W)
    V0, _ = np.linalg.qr(R0)
    K = [V0]
    for _ in range(m - 1):
        K.append(P(M @ K[-1]))
    K = np.concatenate([U] + K, axis=1)
    for c in range(3):
        r = B[:, c] - M @ X[:, c]
        assert np.linalg.norm(C.conj().T @ r) <= 1e-12 * np.linalg.norm(B[:, c])
        best = _krylov_min(A, K, B[:, c])
        assert np.linalg.norm(r) <= best * (1 + 1e-8)


def test_deflated_block_gmres_converges_on_coarse_operator():
    """Recycle space from the oracle's GCRO-DR on a small coarse operator,
    then block GMRES deflated against it: every column to its tolerance, in
    fewer block steps than without deflation."""
    from oracle.gcrodr import RecycleState, gcrodr
    dims, ntv = (2, 2, 2, 2), 4
    A0 = synth.self_blocks(dims, ntv, 3.5, 0).numpy()
    Bh = synth.hop_blocks(dims, ntv, 0).numpy()
    op = dop.build(dims, A0, Bh, 0.05)
    f = lambda v: dop.apply(op, v.reshape(op.V, op.n)).reshape(-1)
    D = dop.dense(op)
    rng = np.random.default_rng(8)
    N = op.V * op.n
    st = RecycleState()
    for r in range(2):
        b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        gcrodr(f, b, 1e-10, 24, 8, 10, 200, st)
    B = rng.standard_normal((N, 4)) + 1j * rng.standard_normal((N, 4))
    tols = np.array([1e-10, 1e-8, 1e-9, 1e-7])
    X, info = block_gmres(f, B, tols, 6, 400, U=st.U, C=st.C)
    X0, info0 = block_gmres(f, B, tols, 6, 400)
    assert info["converged"] and info0["converged"]
    rel = np.linalg.norm(B - D @ X, axis=0) / np.linalg.norm(B, axis=0)
    assert np.all(rel <= tols)
    assert info["steps"] < info0["steps"]


def _invariant_error(U, M, k):
    """How far span(U) is from the invariant subspace of M's k smallest-|lambda|
    eigenvalues: the larger of the invariance residual of U and the mismatch
    of the eigenvalues of U's Rayleigh-Ritz matrix (relative)."""
    ev = np.linalg.eigvals(M)
    smallest = ev[np.argsort(np.abs(ev))[:k]]
    Mr = np.linalg.lstsq(U, M @ U, rcond=None)[0]
    inv_res = np.linalg.norm(M @ U - U @ Mr) / np.linalg.norm(M @ U)
    got = np.linalg.eigvals(Mr)
    mism = max(max(np.min(np.abs(smallest - g)) for g in got),
               max(np.min(np.abs(got - s)) for s in smallest))
    return max(inv_res, mism / np.abs(smallest).max())


def _block_recycle_error(stage, eig_fn=None):
    """Block recycling on a 12 x 12 matrix with 3 right-hand sides, where one
    block cycle spans the whole space: "build" -- 4 block steps from zero
    (12 basis vectors), the space built from the block Hessenberg matrix;
    "refresh" -- a random recycle pair that is not invariant (C = A U from a
    QR of A U), then one deflated cycle of 3 block steps (which with U spans
    C^12) and the refresh from G^H G z = theta G^H (What^H Vhat) z.  Either
    way the harmonic Ritz pairs are exact eigenpairs, so span(U) must be the
    invariant subspace of the 3 smallest-|lambda| eigenvalues."""
    import oracle.block as ob
    from oracle.gcrodr import RecycleState
    M, rng = _matrix(N=12, seed=31)
    A = lambda v: M @ v
    B = rng.standard_normal((12, 3)) + 1j * rng.standard_normal((12, 3))
    st = RecycleState()
    m = 4
    if stage == "refresh":
        Uu = rng.standard_normal((12, 3)) + 1j * rng.standard_normal((12, 3))
        C, Rr = np.linalg.qr(M @ Uu)
        st.U, st.C, st.updates = Uu @ np.linalg.inv(Rr), C, 1
        m = 3
    saved = ob.sla
    if eig_fn is not None:
        class _Fake:
            eig = staticmethod(eig_fn)
        ob.sla = _Fake
    try:
        _, info = block_gmres(A, B, [1e-30] * 3, m, 1, recycle=st, k=3, u=10)
    finally:
        ob.sla = saved
    assert info["cycles"] == 1 and st.updates == (2 if stage == "refresh" else 1)
    # the pair's own relations hold for any choice of vectors
    assert np.linalg.norm(st.C.conj().T @ st.C - np.eye(3)) <= 1e-12
    assert np.linalg.norm(M @ st.U - st.C) <= 1e-10 * np.linalg.norm(st.C)
    return _invariant_error(st.U, M, 3)


@pytest.mark.parametrize("stage", ["build", "refresh"])
def test_block_recycle_space_is_exact_when_the_cycle_spans_everything(stage):
    """Pins the block form of the GCRO-DR space construction and refresh
    (Sec. 3.4, with the block Arnoldi relation)."""
    assert _block_recycle_error(stage) <= 1e-8


@pytest.mark.parametrize("stage", ["build", "refresh"])
@pytest.mark.parametrize("mistake", ["no_rhs_matrix", "swapped", "conjugated"])
def test_block_recycle_pin_detects_wrong_eigenproblem(stage, mistake):
    """Mistakes planted in the oracle's block recycling (on the CPU) fail the
    pin above: dropping G^H What^H Vhat, swapping the two matrices (which
    selects the largest |theta|), or conjugating the problem."""
    import scipy.linalg as sla
    wrong = {"no_rhs_matrix": lambda a, b: sla.eig(a),
             "swapped": lambda a, b: sla.eig(b, a),
             "conjugated": lambda a, b: sla.eig(a.conj(), b.conj())}[mistake]
    assert _block_recycle_error(stage, wrong) > 1e-3


def test_block_recycling_cuts_block_steps_on_coarse_operator():
    """Block GMRES that builds and refreshes its own recycle space (k = 8,
    u = 4) over two batches of right-hand sides of a small coarse operator:
    every column to its tolerance, the second batch in fewer block steps than
    without recycling, and the space it leaves satisfies C = A U, C^H C = I."""
    from oracle.gcrodr import RecycleState
    dims, ntv = (2, 2, 2, 2), 4
    A0 = synth.self_blocks(dims, ntv, 3.5, 0).numpy()
    Bh = synth.hop_blocks(dims, ntv, 0).numpy()
    op = dop.build(dims, A0, Bh, 0.05)
    f = lambda v: dop.apply(op, v.reshape(op.V, op.n)).reshape(-1)
    D = dop.dense(op)
    rng = np.random.default_rng(9)
    N = op.V * op.n
    st = RecycleState()
    tols = np.array([1e-10, 1e-8, 1e-9, 1e-7])
    B1 = rng.standard_normal((N, 4)) + 1j * rng.standard_normal((N, 4))
    B2 = rng.standard_normal((N, 4)) + 1j * rng.standard_normal((N, 4))
    X1, i1 = block_gmres(f, B1, tols, 6, 400, recycle=st, k=8, u=4)
    X2, i2 = block_gmres(f, B2, tols, 6, 400, recycle=st, k=8, u=4)
    X0, i0 = block_gmres(f, B2, tols, 6, 400)
    assert i1["converged"] and i2["converged"] and i0["converged"]
    for X, B in ((X1, B1), (X2, B2)):
        rel = np.linalg.norm(B - D @ X, axis=0) / np.linalg.norm(B, axis=0)
        assert np.all(rel <= tols)
    assert st.updates == 4
    assert i2["steps"] < i0["steps"]
    assert np.linalg.norm(st.C.conj().T @ st.C - np.eye(8)) <= 1e-10
    assert np.linalg.norm(D @ st.U - st.C) <= 1e-8 * np.linalg.norm(st.C)
