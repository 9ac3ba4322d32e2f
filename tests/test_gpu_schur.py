"""Odd-even reduced system (Sec. 2.2) on the GPU against the oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle import operator as dop
from oracle import poly as opoly
from oracle import schur
from oracle.krylov import arnoldi as o_arnoldi

from .helpers import log, make_pair, oracle_relres, rand_vec, rel, workload_pair

pytestmark = pytest.mark.gpu


def row_err(y, ref):
    """Largest per-row error relative to that row's norm."""
    num = np.linalg.norm(y - ref, axis=-1)
    den = np.maximum(np.linalg.norm(ref, axis=-1), 1e-300)
    return float((num / den).max())


@pytest.mark.parametrize("dims,ntv,mu", [((2, 2, 2, 2), 4, 0.0), ((4, 2, 2, 4), 6, 0.2),
                                         ((4, 4, 4, 4), 24, 0.0), ((2, 4, 2, 2), 32, 0.1),
                                         ((2, 2, 2, 2), 1, 0.3)])
def test_reduced_apply_matches_oracle(dims, ntv, mu):
    log("reduced apply", dims, ntv, mu)
    gop, oop = make_pair(dims, ntv, 2.8, mu=mu, store=("f64", "f32", "f16s"))
    ne = oop.V // 2
    x = rand_vec(ne, oop.n, 70, 0)
    ref = schur.apply(oop, x.numpy())
    y = gop.apply_reduced(x.cuda()).cpu().numpy()
    assert rel(y, ref) <= 1e-13
    # adjoint: <S^H z, x> = <z, S x>
    z = rand_vec(ne, oop.n, 71, 0)
    yh = gop.apply_reduced(z.cuda(), adjoint=True).cpu().numpy()
    lhs = np.vdot(yh.reshape(-1), x.numpy().reshape(-1))
    rhs = np.vdot(z.numpy().reshape(-1), ref.reshape(-1))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)
    x32 = x.to(torch.complex64).cuda()
    y32 = gop.apply_reduced(x32, prec="f32").cpu().numpy()
    assert rel(y32, ref) <= 1e-5
    assert row_err(y32, ref) <= 1e-4      # every row, not only the global norm
    y16 = gop.apply_reduced(x32, prec="f16s").cpu().numpy()
    assert rel(y16, ref) <= 5e-3          # FP16 blocks and inverse blocks, 2^-11 per entry
    assert row_err(y16, ref) <= 2e-2


def test_reduced_arnoldi_matches_oracle():
    from paper_2205_09104_amd import Opts
    log("reduced arnoldi")
    gop, oop = make_pair((4, 2, 2, 2), 4, 3.0, mu=0.1)
    ne = oop.V // 2
    v = rand_vec(ne, oop.n, 72, 0)
    H, s = gop.arnoldi(v.cuda(), 12, Opts(m=12, schur=1))
    f = lambda u: schur.apply(oop, u.reshape(ne, oop.n)).reshape(-1)
    ref = o_arnoldi(f, v.numpy().reshape(-1), 12, "mgs")
    assert s == 12
    assert np.abs(H - ref.Hbar).max() <= 1e-10 * np.abs(ref.Hbar).max()


@pytest.fixture(scope="module")
def c1():
    gop, oop, w = workload_pair("c1", store=("f64", "f32", "f16s"))
    b = synth.rhs(w.dims, w.n_tv, 0)
    xref = np.linalg.solve(dop.dense(oop), b.numpy().reshape(-1)).reshape(oop.V, oop.n)
    return gop, oop, w, b, xref


@pytest.mark.parametrize("cfg", ["gmres", "poly", "gcrodr", "f32", "f16s"])
def test_reduced_solves(c1, cfg):
    from paper_2205_09104_amd import Opts
    gop, oop, w, b, xref = c1
    log("reduced solve", cfg)
    opts = {"gmres": Opts(m=30, schur=1),
            "poly": Opts(m=20, d=4, seed=1, schur=1),
            "gcrodr": Opts(m=28, k=8, d=4, seed=1, schur=1),
            "f32": Opts(m=20, d=4, prec="f32", outer=1, inner_tol=1e-3, seed=1, schur=1),
            "f16s": Opts(m=20, d=4, prec="f16s", outer=1, inner_tol=1e-3, seed=1, schur=1)}[cfg]
    for rep in range(2):       # second solve reuses polynomial and recycle space
        x, st, rc = gop.solve(b.cuda(), 1e-10, opts)
        assert rc == 0 and st[0]["rel_res_true"] <= 1e-10, st
        xh = x.cpu().numpy()
        assert oracle_relres(oop, xh, b.numpy()) <= 1e-10
        assert rel(xh, xref) <= 1e-6
    if cfg == "gmres":
        # the reduced system needs fewer iterations than the full one
        _, sf, _ = gop.solve(b.cuda(), 1e-10, Opts(m=30))
        log(f"  iterations: reduced {st[0]['iters']}, full {sf[0]['iters']}")
        assert st[0]["iters"] < sf[0]["iters"]


@pytest.mark.parametrize("mu", [0.0, 0.07])
def test_reduced_adjoint_solve(mu):
    from paper_2205_09104_amd import Opts
    log("reduced adjoint", mu)
    gop, oop = make_pair((4, 2, 2, 2), 4, 3.2, mu=mu)
    b = rand_vec(oop.V, oop.n, 73, 0)
    x, st, rc = gop.solve(b.cuda(), 1e-11, Opts(m=20, d=4, seed=2, schur=1), adjoint=True)
    assert rc == 0
    assert oracle_relres(oop, x.cpu().numpy(), b.numpy(), adjoint=True) <= 1e-11


def test_reduced_rejects_bad_input():
    from paper_2205_09104_amd import Opts
    from paper_2205_09104_amd._lib import DcError
    log("reduced errors")
    gop, oop = make_pair((3, 2, 2, 2), 2, 3.0)
    b = rand_vec(oop.V, oop.n, 74, 0).cuda()
    with pytest.raises(DcError):
        gop.solve(b, 1e-8, Opts(m=10, schur=1))          # odd extent
    with pytest.raises(DcError):
        gop.apply_reduced(torch.zeros(oop.V // 2, oop.n, dtype=torch.complex128, device="cuda"))
    gop2, oop2 = make_pair((2, 2, 2, 2), 2, 3.0)
    b2 = rand_vec(oop2.V, oop2.n, 75, 0).cuda()
    with pytest.raises(DcError):
        gop2.solve_batch(b2[None], 1e-8, Opts(m=10, schur=1))


def test_reduced_profile_counts_stage_launches(c1):
    """Each reduced matvec runs one D_oe and one D_eo stage launch; the
    profiler counts exactly those that did work."""
    from paper_2205_09104_amd import Opts
    gop, oop, w, b, xref = c1
    log("reduced profile")
    for o in (Opts(m=30, schur=1), Opts(m=20, d=4, seed=1, schur=1)):
        gop.solve(b.cuda(), 1e-10, o)     # builds the polynomial (its applies are not matvecs)
        gop.profile_apply(1)
        _, st, rc = gop.solve(b.cuda(), 1e-10, o)
        n1, _ = gop.profile_apply_read("f64", kernel=1)
        n2, ms2 = gop.profile_apply_read("f64", kernel=2)
        n0, _ = gop.profile_apply_read("f64", kernel=0)
        assert rc == 0 and n1 == n2 == st[0]["matvecs"] and ms2 > 0.0
        assert n0 == 1          # the closing FP64 residual check on the full lattice
    gop.profile_apply(0)


def s_flat(oop):
    ne = oop.V // 2
    return lambda u: schur.apply(oop, u.reshape(ne, oop.n)).reshape(-1)


@pytest.mark.parametrize("d", [2, 5])
def test_reduced_polynomial_chain(c1, d):
    """The reduced apply's chain epilogues (first and later steps of q(S))
    against the oracle's chain with the same roots -- the oracle's, installed
    in the handle (to 1e-12) -- and the roots the library builds against the
    oracle's own (same v0, Leja order, 1e-8)."""
    from paper_2205_09104_amd import Opts
    gop, oop, w, b, xref = c1
    log("reduced poly chain", d)
    ne = oop.V // 2
    v0 = rand_vec(ne, oop.n, 73)
    opts = Opts(d=d, v0=v0.cuda(), schur=1)
    th = gop.poly_setup(opts)
    th_ref, _ = opoly.build_polynomial(s_flat(oop), v0.numpy().reshape(-1), d)
    assert len(th) == d
    assert np.max(np.abs(th - th_ref)) <= 1e-8 * np.abs(th_ref).max()
    x = rand_vec(ne, oop.n, 74)
    gop.poly_set(th_ref, opts)
    got = gop.poly_apply(x.cuda(), opts).cpu().numpy()
    want = opoly.q_apply(s_flat(oop), th_ref, x.numpy().reshape(-1)).reshape(ne, oop.n)
    assert rel(got, want) <= 1e-12


def test_reduced_recycle_invariants(c1):
    """GCRO-DR on S: C^H C = I and C = S q(S) U with the oracle's S."""
    from paper_2205_09104_amd import Opts
    gop, oop, w, b, xref = c1
    log("reduced recycle invariants")
    k, d = 6, 3
    opts = Opts(m=24 + k, k=k, d=d, u=10, seed=3, schur=1)
    for r in range(2):
        x, st, rc = gop.solve(synth.rhs(w.dims, w.n_tv, 10 + r).cuda(), 1e-10, opts)
        assert rc == 0
    U, Cm = gop.export_recycle(opts)
    assert U.shape[0] == k and U.shape[1] == oop.V // 2
    Ch = Cm.cpu().numpy().reshape(k, -1)
    assert np.allclose(Ch.conj() @ Ch.T, np.eye(k), atol=1e-10)
    Uq = [gop.poly_apply(U[i], opts).cpu().numpy().reshape(-1) for i in range(k)]
    SU = np.stack([s_flat(oop)(u) for u in Uq])
    assert np.max(np.abs(SU - Ch)) <= 1e-8 * np.abs(Ch).max()


def test_reduced_profile_vector_passes(c1):
    """The reduced kernels report their algorithmic vector passes: 2 for the
    A_o^{-1} D_oe kernel; for the A_e - D_eo kernel 3 when storing, 4 / 5 in
    the first / later chain steps and 4 for the residual."""
    from paper_2205_09104_amd import Opts
    gop, oop, w, b, xref = c1
    log("reduced profile passes")
    gop.profile_apply(1)
    ne = oop.V // 2
    x = rand_vec(ne, oop.n, 75).cuda()
    gop.apply_reduced(x)
    assert gop.profile_apply_read("f64", kernel=1)[0] == 1
    assert gop.profile_apply_passes("f64", 1) == 2
    assert gop.profile_apply_passes("f64", 2) == 3
    o = Opts(d=4, v0=rand_vec(ne, oop.n, 76).cuda(), schur=1)
    gop.poly_setup(o)
    gop.profile_apply(1)
    gop.poly_apply(x, o)                    # q of degree 3: one first and two later steps
    assert gop.profile_apply_read("f64", kernel=2)[0] == 3
    assert gop.profile_apply_passes("f64", 2) == 4 + 5 + 5
    assert gop.profile_apply_passes("f64", 1) == 2 * 3
    gop.profile_apply(0)
