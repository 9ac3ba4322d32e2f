"""Pins of the oracle's pipelined (Alg. 4 / Alg. 5, Sec. 3.5) and single-sync
Arnoldi processes: their Hessenberg matrices and deflation coefficients against
modified Gram-Schmidt Arnoldi (a different formulation, equal in exact
arithmetic), the Arnoldi relation, exact solves, the breakdown on an invariant
subspace and the operator-application count."""
import numpy as np
import pytest

from oracle.gcrodr import RecycleState, gcrodr
from oracle.krylov import arnoldi
from oracle.pipelined import p1_arnoldi, p1_gmres


def _problem(N=48, seed=0):
    rng = np.random.default_rng(seed)
    M = (3.0 * np.eye(N) + rng.standard_normal((N, N)) / np.sqrt(N)
         + 1j * rng.standard_normal((N, N)) / np.sqrt(N))
    v = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    return M, v, rng


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("ortho", ["p1", "ss"])
def test_hessenberg_matches_mgs(ortho):
    M, v, _ = _problem()
    A = lambda x: M @ x
    ref = arnoldi(A, v, 6, "mgs")
    got = arnoldi(A, v, 6, ortho)
    assert got.steps == 6 and not got.breakdown
    assert _rel(got.Hbar, ref.Hbar) <= 1e-10


@pytest.mark.parametrize("ortho", ["p1", "ss"])
def test_deflated_coefficients_match_mgs(ortho):
    """With recycled C: Hbar and B_k = C^H A V of the deflated process; the
    start vector is orthogonal to C, as GCRO-DR's residual is."""
    M, v, rng = _problem(seed=1)
    A = lambda x: M @ x
    Q, _ = np.linalg.qr(rng.standard_normal((M.shape[0], 4)) + 1j * rng.standard_normal((M.shape[0], 4)))
    C = [Q[:, i] for i in range(4)]
    v = v - Q @ (Q.conj().T @ v)
    ref = arnoldi(A, v, 6, "mgs", C=C)
    got = arnoldi(A, v, 6, ortho, C=C)
    assert _rel(got.Hbar, ref.Hbar) <= 1e-10
    assert np.abs(got.Bk - ref.Bk).max() <= 1e-10 * np.abs(ref.Bk).max()
    # the deflated Arnoldi relation A V_j = C B_k + V_{j+1} Hbar
    V = np.stack(got.V, 1)
    lhs = M @ V[:, :got.steps]
    rhs = Q @ got.Bk + V @ got.Hbar
    assert np.abs(lhs - rhs).max() <= 1e-10 * np.abs(lhs).max()


def test_p1_counts_operator_applications():
    """One application per step plus v^a_0 = A v_0 and the k products A c_j."""
    M, v, rng = _problem(seed=2)
    calls = []
    A = lambda x: (calls.append(1), M @ x)[1]
    Q, _ = np.linalg.qr(rng.standard_normal((M.shape[0], 3)) + 0j)
    v = v - Q @ (Q.conj().T @ v)
    _, _, _, steps, _, applies = p1_arnoldi(A, v, 5, C=[Q[:, i] for i in range(3)])
    assert steps == 5 and applies == 5 + 1 + 3 == len(calls)


def test_p1_gmres_solves():
    M, _, rng = _problem(seed=3)
    b = rng.standard_normal(M.shape[0]) + 1j * rng.standard_normal(M.shape[0])
    x, cycles, rel = p1_gmres(lambda v: M @ v, b, 1e-10, 6, 200)
    assert rel <= 1e-10 and cycles > 1
    xr = np.linalg.solve(M, b)
    assert np.linalg.norm(x - xr) <= 1e-8 * np.linalg.norm(xr)


@pytest.mark.parametrize("ortho", ["p1", "ss"])
def test_breakdown_on_invariant_subspace(ortho):
    """v_0 in a 3-dimensional invariant subspace: the third step finds
    h_{4,3} = 0 (t at rounding level) and the 3-step solve is exact."""
    rng = np.random.default_rng(4)
    N = 20
    M = np.zeros((N, N), dtype=np.complex128)
    M[:3, :3] = np.diag([2.0, 3.0 + 1j, 5.0]) + 0.3 * rng.standard_normal((3, 3))
    M[3:, 3:] = 4.0 * np.eye(N - 3) + rng.standard_normal((N - 3, N - 3)) / np.sqrt(N)
    b = np.zeros(N, dtype=np.complex128)
    b[:3] = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    ar = arnoldi(lambda x: M @ x, b, 10, ortho, breakdown_rel=1e-7)
    assert ar.breakdown and ar.steps == 3
    e1 = np.zeros(4, dtype=np.complex128)
    e1[0] = np.linalg.norm(b)
    y = np.linalg.lstsq(ar.Hbar, e1, rcond=None)[0]
    x = sum(y[i] * ar.V[i] for i in range(3))
    assert np.linalg.norm(M @ x - b) <= 1e-10 * np.linalg.norm(b)


def test_pipelined_gcrodr_matches_gcrodr():
    """GCRO-DR with the pipelined Arnoldi (Alg. 5) follows the same iteration:
    same cycle count, solutions equal to the tolerance, recycle spaces
    spanning the same directions."""
    M, _, rng = _problem(N=64, seed=5)
    D = lambda v: M @ v
    b1 = rng.standard_normal(64) + 1j * rng.standard_normal(64)
    b2 = rng.standard_normal(64) + 1j * rng.standard_normal(64)
    out = {}
    for ortho in ("mgs", "p1"):
        st = RecycleState()
        _, i1 = gcrodr(D, b1, 1e-10, 10, 4, 10, 500, st, ortho=ortho)
        x2, i2 = gcrodr(D, b2, 1e-10, 10, 4, 10, 500, st, ortho=ortho)
        out[ortho] = (i1, i2, x2, st.C)
    (a1, a2, xa, Ca), (p1_, p2, xp, Cp) = out["mgs"], out["p1"]
    assert a1.converged and a2.converged and p1_.converged and p2.converged
    assert abs(a1.cycles - p1_.cycles) <= 1 and abs(a2.cycles - p2.cycles) <= 1
    xr = np.linalg.solve(M, b2)
    assert np.linalg.norm(xp - xr) <= 1e-8 * np.linalg.norm(xr)
    # the recycled subspaces agree: the projection of one basis on the other
    s = np.linalg.svd(Ca.conj().T @ Cp, compute_uv=False)
    assert s.min() >= 1 - 1e-6
