"""Single-sync Arnoldi (Sec. 3.5; option ortho = 1) on the GPU against the
oracle's latency-1 pipelined process (Alg. 4 / Alg. 5), which is a different
formulation with the same Hessenberg matrix in exact arithmetic."""
import numpy as np
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
