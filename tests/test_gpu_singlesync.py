"""Single-sync Arnoldi (Sec. 3.5; option ortho = 1) on the GPU against the
oracle's latency-1 pipelined process (Alg. 4 / Alg. 5), which is a different
formulation with the same Hessenberg matrix in exact arithmetic."""
import numpy as np
import torch
import pytest

import synth
from oracle import operator as dop
from oracle import schur
from oracle.pipelined import p1_arnoldi

from .helpers import log, make_pair, oracle_relres, rand_vec, rel, workload_pair

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("reduced", [0, 1])
def test_single_sync_hessenberg_matches_pipelined_oracle(reduced):
    from paper_2205_09104_amd import Opts
    log("single-sync arnoldi", reduced)
    gop, oop = make_pair((4, 2, 2, 4), 6, 3.0, mu=0.1)
    rows = oop.V // 2 if reduced else oop.V
    v = rand_vec(rows, oop.n, 80)
    steps = 6
    H, s = gop.arnoldi(v.cuda(), steps, Opts(m=steps, ortho=1, schur=reduced))
    if reduced:
        f = lambda u: schur.apply(oop, u.reshape(rows, oop.n)).reshape(-1)
    else:
        f = lambda u: dop.apply(oop, u.reshape(rows, oop.n)).reshape(-1)
    _, Hb, _, st, brk, _ = p1_arnoldi(f, v.numpy().reshape(-1), steps)
    assert s == st == steps and not brk
    assert np.abs(H - Hb).max() <= 1e-9 * np.abs(Hb).max()


@pytest.fixture(scope="module")
def c1():
    gop, oop, w = workload_pair("c1", store=("f64", "f32", "f16s"))
    b = synth.rhs(w.dims, w.n_tv, 0)
    xref = np.linalg.solve(dop.dense(oop), b.numpy().reshape(-1)).reshape(oop.V, oop.n)
    return gop, oop, w, b, xref


@pytest.mark.parametrize("cfg", ["gmres", "poly", "gcrodr", "f16s", "reduced_f16s"])
def test_single_sync_solves(c1, cfg):
    """Every single-RHS solver option with the single-sync process reaches its
    tolerance on the FP64 true residual (re-checked with the oracle's apply)."""
    from paper_2205_09104_amd import Opts
    gop, oop, w, b, xref = c1
    log("single-sync solve", cfg)
    o = {"gmres": Opts(m=16, ortho=1),
         "poly": Opts(m=12, d=4, seed=1, ortho=1),
         "gcrodr": Opts(m=20, k=8, d=4, seed=1, ortho=1),
         "f16s": Opts(m=20, k=8, d=4, prec="f16s", outer=1, inner_tol=1e-2, seed=1, ortho=1),
         "reduced_f16s": Opts(m=20, k=8, d=4, prec="f16s", outer=1, inner_tol=1e-2, seed=1,
                              ortho=1, schur=1)}[cfg]
    for _ in range(2):      # the second solve reuses the polynomial and recycle space
        x, st, rc = gop.solve(b.cuda(), 1e-10, o)
        assert rc == 0 and st[0]["rel_res_true"] <= 1e-10, st
        xh = x.cpu().numpy()
        assert oracle_relres(oop, xh, b.numpy()) <= 1e-10
        assert rel(xh, xref) <= 1e-6


def test_single_sync_iterations_close_to_gram_schmidt_twice(c1):
    """Equal in exact arithmetic: on a well-conditioned problem the single-sync
    process needs about as many Arnoldi steps as Gram-Schmidt twice."""
    from paper_2205_09104_amd import Opts
    gop, oop, w, b, xref = c1
    log("single-sync steps")
    _, s2, _ = gop.solve(b.cuda(), 1e-8, Opts(m=30, d=4, seed=1))
    _, s1, _ = gop.solve(b.cuda(), 1e-8, Opts(m=30, d=4, seed=1, ortho=1))
    assert s1[0]["status"] == 0 and s2[0]["status"] == 0
    assert s1[0]["iters"] <= 1.5 * s2[0]["iters"] + 3


def test_single_sync_rejected_where_unsupported(c1):
    from paper_2205_09104_amd import Opts
    from paper_2205_09104_amd._lib import DcError
    gop, oop, w, b, xref = c1
    with pytest.raises(DcError):
        gop.solve_batch(b[None].cuda(), 1e-8, Opts(m=10, ortho=1))
    with pytest.raises(DcError):
        gop.solve(b.cuda(), 1e-8, Opts(m=10, ortho=2))


def test_single_sync_recycle_space_from_gram_schmidt_twice(c1):
    """The recycle space is built and refreshed from Gram-Schmidt-twice cycles
    even when the solve asks for the single-sync process, so C stays
    orthonormal and C = A~ q(A~) U holds with the oracle's operator."""
    from paper_2205_09104_amd import Opts
    gop, oop, w, b, xref = c1
    log("single-sync recycle space")
    k, d = 40, 6
    o = Opts(m=30 + k, k=k, d=d, u=3, seed=2, ortho=1)
    for r in range(3):
        x, st, rc = gop.solve(synth.rhs(w.dims, w.n_tv, 20 + r).cuda(), 1e-10, o)
        assert rc == 0, st
    U, Cm = gop.export_recycle(o)
    assert U.shape[0] == k
    Ch = Cm.cpu().numpy().reshape(k, -1)
    assert np.abs(Ch.conj() @ Ch.T - np.eye(k)).max() <= 1e-10
    Uq = [gop.poly_apply(U[i], o).cpu().numpy().reshape(-1) for i in range(k)]
    AU = np.stack([dop.apply(oop, u.reshape(oop.V, oop.n)).reshape(-1) for u in Uq])
    assert np.abs(AU - Ch).max() <= 1e-8 * np.abs(Ch).max()


@pytest.mark.parametrize("cfg", ["reduced_bj_ss", "full_cgs2", "f16s_outer"])
def test_graph_replayed_cycles_match_eager(cfg):
    """Arnoldi cycles recorded once as HIP graphs and replayed (opts.graphs =
    1) give the same iterates as the eager launches: several solves in a row,
    each replaying the cycle graphs several times, with eager work and host
    synchronisation between the replays, every solve's solution identical to
    the eager solve's."""
    from paper_2205_09104_amd import CoarseOp, Opts
    log("graph cycles", cfg)
    w = synth.WORKLOADS["c1"]
    A, B = synth.operator(w)
    base = {"reduced_bj_ss": dict(m=28, k=8, d=4, seed=1, schur=1, block_jacobi=1, ortho=1),
            "full_cgs2": dict(m=30, d=3, seed=2),
            "f16s_outer": dict(m=28, k=8, d=4, prec="f16s", outer=1, inner_tol=1e-1, seed=1,
                               schur=1, block_jacobi=1, ortho=1)}[cfg]
    store = ("f64", "f32", "f16s")
    opg = CoarseOp(A.cuda(), B.cuda(), w.dims, mu=w.mu, store=store)
    ope = CoarseOp(A.cuda(), B.cuda(), w.dims, mu=w.mu, store=store)
    for r in range(4):
        b = synth.rhs(w.dims, w.n_tv, r).cuda()
        xg, sg, rcg = opg.solve(b, 1e-10, Opts(**base, graphs=1))
        xe, se, rce = ope.solve(b, 1e-10, Opts(**base, graphs=0))
        torch.cuda.synchronize()
        assert rcg == rce == 0
        assert sg[0]["iters"] == se[0]["iters"] and sg[0]["matvecs"] == se[0]["matvecs"]
        assert torch.equal(xg, xe), r
    cap, launched = opg.graph_stats()
    log(f"  graphs captured {cap}, launched {launched}")
    assert cap >= 1 and launched > cap
    assert ope.graph_stats() == (0, 0)
    opg.close()
    ope.close()
