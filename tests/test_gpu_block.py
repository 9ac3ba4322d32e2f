"""Block GMRES with one shared Krylov space (solve_coarse_block) against the
oracle's block GMRES and dense LU."""
import numpy as np
import pytest
import torch

import synth
from oracle import operator as dop
from oracle.block import block_gmres

from .helpers import log, make_pair, oracle_relres, rand_vec, rel, workload_pair

pytestmark = pytest.mark.gpu


def _rhs(dims, ntv, R, seed0):
    return torch.stack([synth.rhs(dims, ntv, seed0 + r) for r in range(R)])


def test_first_cycle_matches_oracle():
    """One cycle of m block steps from zero, no early stop: every column is the
    least-squares minimiser over the same block space as the oracle's."""
    from paper_2205_09104_amd import Opts
    log("block gmres one cycle")
    gop, oop = make_pair((4, 2, 2, 4), 6, 3.0, mu=0.1)
    R, m = 3, 6
    B = _rhs(oop.dims, 6, R, 40)
    X, st, rc = gop.solve_block(B.cuda(), 1e-30, Opts(m=m, max_cycles=1))
    assert rc != 0 and all(s["iters"] == m for s in st)
    N = oop.V * oop.n
    f = lambda v: dop.apply(oop, v.reshape(oop.V, oop.n)).reshape(-1)
    Bn = B.numpy().reshape(R, N).T
    Xr, info = block_gmres(f, Bn, [1e-30] * R, m, 1)
    Xg = X.cpu().numpy().reshape(R, N).T
    assert rel(Xg, Xr) <= 1e-10
    for c in range(R):
        assert abs(st[c]["rel_res_true"] - info["relres"][c]) <= 1e-8 * info["relres"][c]


@pytest.fixture(scope="module")
def c1():
    gop, oop, w = workload_pair("c1", store=("f64", "f32", "f16s"))
    D = dop.dense(oop)
    return gop, oop, w, D


@pytest.mark.parametrize("cfg", ["f64", "f64_poly", "f32", "f16s"])
def test_block_solve_per_column_tolerances(c1, cfg):
    from paper_2205_09104_amd import Opts
    gop, oop, w, D = c1
    log("block gmres solve", cfg)
    R = 6
    B = _rhs(w.dims, w.n_tv, R, 50)
    tols = np.array(synth.tolerances_loguniform(R, 1e-10, 1e-6, seed=3))
    o = {"f64": Opts(m=20),
         "f64_poly": Opts(m=12, d=4, seed=1),
         "f32": Opts(m=12, d=4, seed=1, prec="f32", inner_tol=1e-3, max_outer=40),
         "f16s": Opts(m=12, d=4, seed=1, prec="f16s", inner_tol=1e-2, max_outer=40)}[cfg]
    X, st, rc = gop.solve_block(B.cuda(), tols, o)
    assert rc == 0, st
    Xh = X.cpu().numpy()
    for c in range(R):
        assert st[c]["rel_res_true"] <= tols[c]
        assert oracle_relres(oop, Xh[c], B[c].numpy()) <= tols[c] * 1.0001
    xr = np.linalg.solve(D, B[int(np.argmin(tols))].numpy().reshape(-1))
    assert rel(Xh[int(np.argmin(tols))].reshape(-1), xr) <= 1e-6


def test_block_solve_deflated_by_recycle_space(c1):
    """After a single-RHS GCRO-DR solve has built the recycle space, block
    cycles deflated against it converge to every column's tolerance in fewer
    block steps than without it."""
    from paper_2205_09104_amd import Opts
    gop, oop, w, D = c1
    log("block gmres deflated")
    R = 4
    B = _rhs(w.dims, w.n_tv, R, 80)
    tols = np.array([1e-10, 1e-8, 1e-9, 1e-7])
    o = Opts(m=12, k=8, d=4, seed=1, u=3)
    for r in range(3):   # builds and refreshes the recycle space of the variant
        gop.solve(synth.rhs(w.dims, w.n_tv, 90 + r).cuda(), 1e-10, Opts(m=30 + 8, k=8, d=4, seed=1, u=3))
    Xd, sd, rcd = gop.solve_block(B.cuda(), tols, o)
    X0, s0, rc0 = gop.solve_block(B.cuda(), tols, Opts(m=12, d=4, seed=1))
    assert rcd == 0 and rc0 == 0
    Xh = Xd.cpu().numpy()
    for c in range(R):
        assert oracle_relres(oop, Xh[c], B[c].numpy()) <= tols[c] * 1.0001
    assert max(s["iters"] for s in sd) < max(s["iters"] for s in s0)


@pytest.mark.parametrize("prec", ["f64", "f16s"])
def test_block_solve_continues_from_start_vector(c1, prec):
    """A solve stopped early (bounded refinement / cycles) continues from its x:
    the second call meets the tolerances relative to b."""
    from paper_2205_09104_amd import Opts
    gop, oop, w, D = c1
    log("block gmres continued", prec)
    R = 3
    B = _rhs(w.dims, w.n_tv, R, 100).cuda()
    tols = np.array([1e-10, 1e-9, 1e-8])
    if prec == "f64":
        o1, o2 = Opts(m=8, max_cycles=2), Opts(m=12)
    else:
        o1 = Opts(m=8, d=4, seed=1, prec="f16s", inner_tol=1e-2, max_outer=2)
        o2 = Opts(m=8, d=4, seed=1, prec="f16s", inner_tol=1e-2, max_outer=40)
    X1, s1, rc1 = gop.solve_block(B, tols, o1)
    assert rc1 != 0
    X2, s2, rc2 = gop.solve_block(B, tols, o2, x0=X1)
    assert rc2 == 0
    Xh = X2.cpu().numpy()
    for c in range(R):
        assert s2[c]["rel_res_true"] <= tols[c]
        assert oracle_relres(oop, Xh[c], B[c].cpu().numpy()) <= tols[c] * 1.0001


@pytest.mark.parametrize("prec,eps", [("f64", 1e-13), ("f16s", 1e-7)])
def test_block_solve_with_dependent_columns(c1, prec, eps):
    """Right-hand sides that are numerically dependent (two columns within eps
    of two others): the space grows from a well-conditioned subset of the
    residual columns and every column still meets its tolerance."""
    from paper_2205_09104_amd import Opts
    gop, oop, w, D = c1
    log("block gmres dependent columns", prec)
    b = [synth.rhs(w.dims, w.n_tv, 110 + r) for r in range(4)]
    B = torch.stack([b[0], b[1], b[0] + eps * b[2], b[1] - eps * b[3]]).cuda()
    tols = np.array([1e-10, 1e-9, 1e-10, 1e-8])
    o = (Opts(m=12) if prec == "f64" else
         Opts(m=8, d=4, seed=1, prec="f16s", inner_tol=1e-2, max_outer=40))
    X, st, rc = gop.solve_block(B, tols, o)
    assert rc == 0, st
    Xh = X.cpu().numpy()
    Bh = B.cpu().numpy()
    for c in range(4):
        assert oracle_relres(oop, Xh[c], Bh[c]) <= tols[c] * 1.0001


def test_single_column_is_gmres(c1):
    """With one right-hand side the block process is GMRES(m): the same number
    of Arnoldi steps as the single-RHS solver (to a step or two of rounding)."""
    from paper_2205_09104_amd import Opts
    gop, oop, w, D = c1
    log("block with one column")
    b = synth.rhs(w.dims, w.n_tv, 60)
    _, s1, rc1 = gop.solve_block(b[None].cuda(), 1e-9, Opts(m=12, d=4, seed=1))
    _, sg, rcg = gop.solve(b.cuda(), 1e-9, Opts(m=12, d=4, seed=1))
    assert rc1 == 0 and rcg == 0
    assert abs(s1[0]["iters"] - sg[0]["iters"]) <= 2


def test_block_solver_rejects_bad_options(c1):
    from paper_2205_09104_amd import Opts
    from paper_2205_09104_amd._lib import DcError
    gop, oop, w, D = c1
    B = _rhs(w.dims, w.n_tv, 2, 70).cuda()
    for o in (Opts(m=10, schur=1), Opts(m=10, block_jacobi=1), Opts(m=0)):
        with pytest.raises(DcError):
            gop.solve_block(B, 1e-8, o)
    with pytest.raises(DcError):
        gop.solve_block(B, [1e-8, 0.0], Opts(m=10))


def test_dependent_columns_cycle_matches_oracle():
    """Residual columns that are numerically dependent (three columns and
    three combinations of them, each with a part of relative size 5e-7
    outside their span): the library generates the space from the picked
    columns, runs m x 6 / 3 block steps, and gives every column the exact
    least-squares minimiser over that space, the parts of its residual outside
    the first block included -- the same as the oracle's block GMRES."""
    from paper_2205_09104_amd import Opts
    log("block gmres dependent columns, one cycle")
    gop, oop = make_pair((4, 2, 2, 4), 6, 3.0, mu=0.1)
    N = oop.V * oop.n
    m = 3
    base = _rhs(oop.dims, 6, 3, 60).numpy().reshape(3, N)
    rng = np.random.default_rng(11)
    mix = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    dep = mix @ base
    nz = rng.standard_normal((3, N)) + 1j * rng.standard_normal((3, N))
    # parts of relative size 5e-7 outside the span: dependent at the FP64
    # selection threshold (squared part 2.5e-13 < 1e-12), large enough that
    # leaving them out of the least squares would show at 1e-9
    dep = dep + 5e-7 * (np.linalg.norm(dep, axis=1) / np.linalg.norm(nz, axis=1))[:, None] * nz
    Bn = np.concatenate([base, dep], axis=0)
    B = torch.from_numpy(Bn.reshape(6, oop.V, oop.n)).cuda()
    X, st, rc = gop.solve_block(B, 1e-30, Opts(m=m, max_cycles=1))
    f = lambda v: dop.apply(oop, v.reshape(oop.V, oop.n)).reshape(-1)
    Xr, info = block_gmres(f, Bn.T, [1e-30] * 6, m, 1)
    assert info["generators"] == [3] and info["steps"] == 6
    assert all(s["iters"] == 6 for s in st)
    Xg = X.cpu().numpy().reshape(6, N).T
    log(f"  difference to the oracle: {rel(Xg, Xr):.2e}")
    assert rel(Xg, Xr) <= 1e-9
    for c in range(6):
        assert abs(st[c]["rel_res_true"] - info["relres"][c]) <= 1e-7 * info["relres"][c]


def test_refinement_stops_on_stagnation(c1):
    """FP16-stored inner block solves too short to make progress: the FP64
    refinement stops once a column's residual has not fallen below 0.9 of its
    best for three steps, and reports it (stagnated, DC_NOT_CONVERGED)."""
    from paper_2205_09104_amd import Opts
    gop, oop, w, D = c1
    log("block gmres stagnation stop")
    B = _rhs(w.dims, w.n_tv, 2, 90)
    o = Opts(m=1, prec="f16s", inner_tol=1e-12, max_cycles=1, max_outer=200)
    X, st, rc = gop.solve_block(B.cuda(), 1e-12, o)
    assert rc == 1
    for s in st:
        assert s["status"] == 1
        assert s["stagnated"] == 1 or s["outer_iters"] >= 200
    assert any(s["stagnated"] == 1 for s in st)
    assert max(s["outer_iters"] for s in st) < 200


@pytest.mark.parametrize("dims,ntv,R,m", [((3, 3, 2, 2), 7, 20, 4),
                                          ((4, 4, 2, 4), 6, 40, 3),
                                          ((2, 2, 2, 2), 12, 70, 1)])
def test_wide_block_cycle_matches_oracle(dims, ntv, R, m):
    """Blocks of more than 16 columns take the MFMA Gram kernel: one cycle
    with ragged row chunks (N = 504, not a multiple of 32 or 64), ragged
    output tiles (20 and 40 columns, Krylov blocks of 20..120 vectors) and
    more than one 64-column tile (70 columns) gives every column the oracle's
    least-squares minimiser."""
    from paper_2205_09104_amd import Opts
    log("wide block cycle", dims, ntv, R, m)
    gop, oop = make_pair(dims, ntv, 3.0, mu=0.1)
    N = oop.V * oop.n
    B = _rhs(oop.dims, ntv, R, 200)
    X, st, rc = gop.solve_block(B.cuda(), 1e-30, Opts(m=m, max_cycles=1))
    assert all(s["iters"] == m for s in st)
    f = lambda v: dop.apply(oop, v.reshape(oop.V, oop.n)).reshape(-1)
    Bn = B.numpy().reshape(R, N).T
    Xr, info = block_gmres(f, Bn, [1e-30] * R, m, 1)
    Xg = X.cpu().numpy().reshape(R, N).T
    log(f"  difference to the oracle: {rel(Xg, Xr):.2e}")
    assert rel(Xg, Xr) <= 1e-10
    for c in range(R):
        assert abs(st[c]["rel_res_true"] - info["relres"][c]) <= 1e-8 * info["relres"][c]


@pytest.mark.parametrize("prec", ["f32", "f16s"])
def test_wide_block_reduced_precision_solve(prec):
    """24 columns in FP32 / FP16-stored inner block solves (MFMA Gram and
    update kernels in FP32) inside the FP64 refinement: every column meets its
    tolerance by the oracle's residual."""
    from paper_2205_09104_amd import Opts
    log("wide block reduced precision", prec)
    gop, oop = make_pair((4, 4, 2, 4), 6, 3.0, mu=0.1, store=("f64", "f32", "f16s"))
    R = 24
    B = _rhs(oop.dims, 6, R, 300)
    tols = np.array(synth.tolerances_loguniform(R, 1e-10, 1e-6, seed=5))
    o = Opts(m=6, d=3, seed=1, prec=prec, inner_tol=1e-3, max_outer=40)
    X, st, rc = gop.solve_block(B.cuda(), tols, o)
    assert rc == 0, st
    Xh = X.cpu().numpy()
    for c in range(R):
        assert oracle_relres(oop, Xh[c], B[c].numpy()) <= tols[c] * 1.0001


def _principal_sines(X, Y):
    """Sine of the largest principal angle between span(X) and span(Y)."""
    qx, _ = np.linalg.qr(X)
    qy, _ = np.linalg.qr(Y)
    c = np.linalg.svd(qx.conj().T @ qy, compute_uv=False).min()
    return float(np.sqrt(max(0.0, 1.0 - c * c)))


@pytest.mark.parametrize("d", [0, 3])
def test_block_recycling_matches_oracle(d):
    """Block GMRES that builds its recycle space from its first cycle and
    refreshes it from the next two (k = 6, u = 3, FP64, a tolerance never
    met): after 1, 2 and 3 cycles the iterate matches the oracle's block
    recycling from the same inputs (the polynomial of degree d from the same
    start vector), and so do span(U) and span(C)."""
    from oracle import poly as opoly
    from oracle.gcrodr import RecycleState
    from paper_2205_09104_amd import Opts
    log("block recycling vs oracle, d", d)
    gop, oop = make_pair((4, 2, 2, 4), 6, 3.0, mu=0.1)
    N = oop.V * oop.n
    R, m, k = 4, 6, 6
    B = _rhs(oop.dims, 6, R, 400)
    Bn = B.numpy().reshape(R, N).T
    f = lambda v: dop.apply(oop, v.reshape(oop.V, oop.n)).reshape(-1)
    v0 = rand_vec(oop.V, oop.n, 401)
    right = None
    if d > 1:
        th, _ = opoly.build_polynomial(f, v0.numpy().reshape(-1), d)
        right = lambda v: opoly.q_apply(f, th, v)
    for cycles in (1, 2, 3):
        gop.update(torch.as_tensor(oop.A0).cuda(), torch.as_tensor(oop.B).cuda())  # no space yet
        o = Opts(m=m, k=k, u=3, d=d, v0=v0.cuda() if d > 1 else None, max_cycles=cycles)
        X, st, rc = gop.solve_block(B.cuda(), 1e-30, o)
        sr = RecycleState()
        Xr, info = block_gmres(f, Bn, [1e-30] * R, m, cycles, right=right, recycle=sr, k=k, u=3)
        Xg = X.cpu().numpy().reshape(R, N).T
        U, Cm = gop.export_recycle(o)
        su = _principal_sines(U.cpu().numpy().reshape(k, -1).T, sr.U)
        sc = _principal_sines(Cm.cpu().numpy().reshape(k, -1).T, sr.C)
        log(f"  cycles {cycles}: iterate {rel(Xg, Xr):.2e}, span U {su:.2e}, span C {sc:.2e}, "
            f"updates {sr.updates}")
        assert rel(Xg, Xr) <= 1e-9
        assert su <= 1e-7 and sc <= 1e-7
        assert all(s["refresh_failed"] == 0 for s in st)


def test_block_recycling_cuts_block_steps(c1):
    """Mixed precision (FP16-stored inner block solves): a second batch of
    right-hand sides with the space the first batch built and refreshed
    needs fewer block steps than the same batch without recycling; every
    column meets its tolerance by the oracle's residual."""
    from paper_2205_09104_amd import Opts
    gop, oop, w, D = c1
    log("block recycling, step count")
    R = 6
    tols = np.array(synth.tolerances_loguniform(R, 1e-10, 1e-6, seed=9))
    B1 = _rhs(w.dims, w.n_tv, R, 500).cuda()
    B2 = _rhs(w.dims, w.n_tv, R, 600).cuda()
    base = dict(m=8, d=4, seed=1, prec="f16s", inner_tol=1e-2, max_outer=40)
    X0, s0, rc0 = gop.solve_block(B2, tols, Opts(**base))
    gop.update(torch.as_tensor(oop.A0).cuda(), torch.as_tensor(oop.B).cuda())
    o = Opts(k=16, u=4, **base)
    _, s1, rc1 = gop.solve_block(B1, tols, o)
    X2, s2, rc2 = gop.solve_block(B2, tols, o)
    assert rc0 == 0 and rc1 == 0 and rc2 == 0
    it0, it2 = max(s["iters"] for s in s0), max(s["iters"] for s in s2)
    log(f"  block steps without recycling {it0}, with {it2}")
    assert it2 < it0
    Xh = X2.cpu().numpy()
    for c in range(R):
        assert oracle_relres(oop, Xh[c], B2[c].cpu().numpy()) <= tols[c] * 1.0001
