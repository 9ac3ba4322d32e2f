"""Block-Jacobi preconditioning of the odd-even reduced system on the GPU
against the oracle.  Sec. 3.2 takes B = D_ee (the even sites' self blocks)
for the reduced operator S = D_ee - D_eo D_oo^{-1} D_oe and applies it from
the left; Sec. 3.3 builds the polynomial from B^{-1} S; Sec. 3.6 combines both
with GCRO-DR."""
import numpy as np
import pytest
import torch

import synth
from oracle import mixed
from oracle import operator as dop
from oracle import poly as opoly
from oracle import schur
from oracle.gcrodr import RecycleState
from oracle.krylov import arnoldi as o_arnoldi

from .helpers import log, make_pair, oracle_relres, rand_vec, rel, workload_pair

pytestmark = pytest.mark.gpu


def _coded(M, store):
    """M in the storage precision (decoded to complex128)."""
    if store == "f32":
        return mixed.round_fp32(M).astype(np.complex128)
    if store == "f16s":
        return mixed.dequantize_fp16(*mixed.quantize_fp16(M)).astype(np.complex128)
    return M


def bj_reduced_lowprec(dims, A0, B, mu, xe, store):
    """D_ee^{-1} S x_e with the blocks the kernels use in storage precision
    `store`: hop blocks coded, the self-block inverses (A_x + i mu Gamma5)^{-1}
    formed in FP64 and then coded; arithmetic in FP64 (the kernels accumulate
    in FP32, so they differ from this by FP32 rounding only)."""
    opc = dop.build(dims, np.zeros_like(A0), _coded(B, store), mu)
    n = A0.shape[1]
    tm = 1j * mu * np.diag(dop.gamma5(n))
    ev, od = schur.sites(dims, 0), schur.sites(dims, 1)
    inv_o = [_coded(np.linalg.inv(A0[y] + tm), store) for y in od]
    inv_e = [_coded(np.linalg.inv(A0[s] + tm), store) for s in ev]
    u = schur.d_oe(opc, xe)
    t = np.stack([inv_o[i] @ u[i] for i in range(len(od))])
    w = schur.d_eo(opc, t)
    return xe - np.stack([inv_e[i] @ w[i] for i in range(len(ev))])


def row_err(y, ref):
    """Largest per-row error relative to that row's norm."""
    num = np.linalg.norm(y - ref, axis=1)
    den = np.maximum(np.linalg.norm(ref, axis=1), 1e-300)
    return float((num / den).max())


@pytest.mark.parametrize("dims,ntv,mu", [((2, 2, 2, 2), 4, 0.0), ((4, 2, 2, 4), 6, 0.2),
                                         ((4, 4, 4, 4), 24, 0.0), ((2, 4, 2, 2), 32, 0.1),
                                         ((2, 2, 2, 2), 1, 0.3)])
def test_reduced_bj_apply_matches_oracle(dims, ntv, mu):
    """B^{-1} S x: FP64 against the oracle's definition (block solves after S)
    to 1e-13 overall and 1e-12 in every row; FP32 and FP16 storage against the
    same operator coded in that precision, row by row."""
    log("reduced bj apply", dims, ntv, mu)
    A0 = synth.self_blocks(dims, ntv, 2.8, 0)
    B = synth.hop_blocks(dims, ntv, 0)
    gop, oop = make_pair(dims, ntv, 2.8, mu=mu, store=("f64", "f32", "f16s"))
    ne = oop.V // 2
    x = rand_vec(ne, oop.n, 80, 0)
    ref = schur.apply_bj(oop, x.numpy())
    y = gop.apply_reduced(x.cuda(), block_jacobi=True).cpu().numpy()
    assert rel(y, ref) <= 1e-13
    assert row_err(y, ref) <= 1e-12
    x32 = x.to(torch.complex64)
    xh32 = x32.numpy().astype(np.complex128)
    for prec in ("f32", "f16s"):
        y = gop.apply_reduced(x32.cuda(), prec=prec, block_jacobi=True).cpu().numpy()
        refc = bj_reduced_lowprec(dims, A0.numpy(), B.numpy(), mu, xh32, prec)
        e = row_err(y.astype(np.complex128), refc)
        log(f"  {prec}: per-row error against the coded operator {e:.2e}")
        assert e <= 1e-5


def test_reduced_bj_arnoldi_matches_oracle():
    """Arnoldi Hessenberg of B^{-1} S (d = 0) and of B^{-1} S q(B^{-1} S) with
    the polynomial the library built (its harmonic Ritz values fed to the
    oracle's chain) against the oracle's MGS Arnoldi to 1e-10."""
    from paper_2205_09104_amd import Opts
    log("reduced bj arnoldi")
    gop, oop = make_pair((4, 2, 2, 2), 4, 3.0, mu=0.1)
    ne = oop.V // 2
    f = lambda u: schur.apply_bj(oop, u.reshape(ne, oop.n)).reshape(-1)
    v = rand_vec(ne, oop.n, 81, 0)
    H, s = gop.arnoldi(v.cuda(), 12, Opts(m=12, schur=1, block_jacobi=1))
    ref = o_arnoldi(f, v.numpy().reshape(-1), 12, "mgs")
    assert s == 12
    assert np.abs(H - ref.Hbar).max() <= 1e-10 * np.abs(ref.Hbar).max()
    v0 = rand_vec(ne, oop.n, 82, 0)
    o = Opts(m=10, d=4, v0=v0.cuda(), schur=1, block_jacobi=1)
    th, _ = opoly.build_polynomial(f, v0.numpy().reshape(-1), 4)
    gop.poly_set(th, o)                  # the oracle's roots, installed in the handle
    H, s = gop.arnoldi(v.cuda(), 10, o)
    fq = lambda u: f(opoly.q_apply(f, th, u))
    ref = o_arnoldi(fq, v.numpy().reshape(-1), 10, "mgs")
    assert s == 10
    assert np.abs(H - ref.Hbar).max() <= 1e-10 * np.abs(ref.Hbar).max()


@pytest.mark.parametrize("d", [2, 6])
def test_reduced_bj_polynomial(d):
    """Harmonic Ritz values of B^{-1} S in Leja order against the oracle's
    (same v0) to 1e-8, and the fused chain q(B^{-1} S) x with the oracle's
    values installed in the handle against the oracle's chain to 1e-12."""
    from paper_2205_09104_amd import Opts
    log("reduced bj polynomial", d)
    gop, oop = make_pair((4, 2, 2, 2), 4, 3.0, mu=0.05)
    ne = oop.V // 2
    f = lambda u: schur.apply_bj(oop, u.reshape(ne, oop.n)).reshape(-1)
    v0 = rand_vec(ne, oop.n, 83, 0)
    o = Opts(d=d, v0=v0.cuda(), schur=1, block_jacobi=1)
    th = gop.poly_setup(o)
    th_ref, _ = opoly.build_polynomial(f, v0.numpy().reshape(-1), d)
    assert len(th) == d
    assert np.max(np.abs(th - th_ref)) <= 1e-8 * np.abs(th_ref).max()
    x = rand_vec(ne, oop.n, 84, 0)
    gop.poly_set(th_ref, o)
    got = gop.poly_apply(x.cuda(), o).cpu().numpy()
    want = opoly.q_apply(f, th_ref, x.numpy().reshape(-1)).reshape(ne, oop.n)
    assert rel(got, want) <= 1e-12


@pytest.fixture(scope="module")
def c1():
    gop, oop, w = workload_pair("c1", store=("f64", "f32", "f16s"))
    b = synth.rhs(w.dims, w.n_tv, 0)
    xref = np.linalg.solve(dop.dense(oop), b.numpy().reshape(-1)).reshape(oop.V, oop.n)
    return gop, oop, w, b, xref


@pytest.mark.parametrize("cfg", ["gmres", "poly", "gcrodr", "gcrodr_ss", "f32", "f16s"])
def test_reduced_bj_solves(c1, cfg):
    """Every solver option with B = D_ee on the reduced system reaches 1e-10
    on the full-lattice residual of the oracle's FP64 apply, with the solution
    within 1e-6 of dense LU, twice in a row (the second reusing the
    polynomial and recycle space)."""
    from paper_2205_09104_amd import Opts
    gop, oop, w, b, xref = c1
    log("reduced bj solve", cfg)
    opts = {"gmres": Opts(m=30, schur=1, block_jacobi=1),
            "poly": Opts(m=20, d=4, seed=1, schur=1, block_jacobi=1),
            "gcrodr": Opts(m=28, k=8, d=4, seed=1, schur=1, block_jacobi=1),
            "gcrodr_ss": Opts(m=28, k=8, d=4, seed=1, schur=1, block_jacobi=1, ortho=1),
            "f32": Opts(m=28, k=8, d=4, prec="f32", outer=1, inner_tol=1e-3, seed=1, schur=1,
                        block_jacobi=1),
            "f16s": Opts(m=28, k=8, d=4, prec="f16s", outer=1, inner_tol=1e-1, seed=1,
                         schur=1, block_jacobi=1, ortho=1)}[cfg]
    for rep in range(2):
        x, st, rc = gop.solve(b.cuda(), 1e-10, opts)
        assert rc == 0 and st[0]["rel_res_true"] <= 1e-10, st
        xh = x.cpu().numpy()
        assert oracle_relres(oop, xh, b.numpy()) <= 1e-10
        assert rel(xh, xref) <= 1e-6


def test_reduced_bj_gmres_iterations_match_oracle(c1):
    """Plain GMRES(30) on B^{-1} S in FP64: the library's iteration count
    (Gram-Schmidt twice) equals the oracle's (modified Gram-Schmidt) to within
    one step, and the oracle converges to the same tolerance."""
    from paper_2205_09104_amd import Opts
    from oracle.krylov import gmres
    gop, oop, w, b, xref = c1
    log("reduced bj gmres iterations")
    x, st, rc = gop.solve(b.cuda(), 1e-10, Opts(m=30, schur=1, block_jacobi=1))
    assert rc == 0
    bh = schur.rhs(oop, b.numpy()).reshape(-1)
    ne = oop.V // 2
    S = lambda u: schur.apply(oop, u.reshape(ne, oop.n)).reshape(-1)
    L = lambda u: schur.dinv_ee(oop, u.reshape(ne, oop.n)).reshape(-1)
    tol_s = 1e-10 * np.linalg.norm(b.numpy()) / np.linalg.norm(bh)
    _, info = gmres(S, bh, tol_s, 30, 10000, left=L)
    log(f"  iterations: library {st[0]['iters']}, oracle {info.iters}")
    assert info.converged and abs(st[0]["iters"] - info.iters) <= 1


def test_reduced_bj_recycle_invariants(c1):
    """GCRO-DR on B^{-1} S q(B^{-1} S): C^H C = I and C = A^ U with the oracle's
    B^{-1} S and the oracle's polynomial roots installed in the handle."""
    from paper_2205_09104_amd import Opts
    gop, oop, w, b, xref = c1
    log("reduced bj recycle invariants")
    k, d = 6, 3
    ne = oop.V // 2
    f = lambda u: schur.apply_bj(oop, u.reshape(ne, oop.n)).reshape(-1)
    opts = Opts(m=24 + k, k=k, d=d, u=10, seed=3, schur=1, block_jacobi=1)
    # the polynomial: the oracle's roots from a fixed start vector, installed
    th, _ = opoly.build_polynomial(f, rand_vec(ne, oop.n, 85, 0).numpy().reshape(-1), d)
    gop.poly_set(th, opts)
    for r in range(2):
        x, st, rc = gop.solve(synth.rhs(w.dims, w.n_tv, 10 + r).cuda(), 1e-10, opts)
        assert rc == 0
    U, Cm = gop.export_recycle(opts)
    Ch = Cm.cpu().numpy().reshape(k, -1)
    assert np.allclose(Ch.conj() @ Ch.T, np.eye(k), atol=1e-10)
    AU = np.stack([f(opoly.q_apply(f, th, u)) for u in U.cpu().numpy().reshape(k, -1)])
    assert np.max(np.abs(AU - Ch)) <= 1e-8 * np.abs(Ch).max()


@pytest.mark.parametrize("mu", [0.0, 0.07])
def test_reduced_bj_adjoint_solve(mu):
    from paper_2205_09104_amd import Opts
    log("reduced bj adjoint", mu)
    gop, oop = make_pair((4, 2, 2, 2), 4, 3.2, mu=mu)
    b = rand_vec(oop.V, oop.n, 85, 0)
    o = Opts(m=24, k=4, d=4, seed=2, schur=1, block_jacobi=1)
    for rep in range(2):
        x, st, rc = gop.solve(b.cuda(), 1e-11, o, adjoint=True)
        assert rc == 0
        assert oracle_relres(oop, x.cpu().numpy(), b.numpy(), adjoint=True) <= 1e-11


def _principal_cosines(X, Y):
    """Cosines of the principal angles between span(X) and span(Y) (columns)."""
    qx, _ = np.linalg.qr(X)
    qy, _ = np.linalg.qr(Y)
    return np.linalg.svd(qx.conj().T @ qy, compute_uv=False)


@pytest.mark.parametrize("bj,k,m", [(0, 5, 25), (1, 5, 25), (1, 18, 32)])
def test_recycle_space_matches_oracle(bj, k, m):
    """The recycle space itself against the oracle's, from the same polynomial
    start vector and right-hand side (FP64, Gram-Schmidt twice against the
    oracle's modified Gram-Schmidt): after the construction cycle (harmonic
    Ritz vectors of H_m) and after one GCRO-DR cycle with its refresh
    (generalised problem of the deflated cycle), span(C) and span(U) agree
    to principal angles below 1e-5.  Twisted mass 0.1 keeps the spectrum
    free of the conjugate pairs that would make the k-th smallest |theta|
    ambiguous.  With k = 18 the new U and C are formed by the MFMA block
    update (16 or more outputs) with FP64 products."""
    from paper_2205_09104_amd import Opts
    log("recycle space vs oracle, bj", bj, "k", k)
    dims, ntv, mu = (4, 4, 2, 2), 4, 0.1
    gop, oop = make_pair(dims, ntv, 3.0, mu=mu)
    ne = oop.V // 2
    b = rand_vec(oop.V, oop.n, 86, 0)
    v0 = rand_vec(ne, oop.n, 87, 0)
    d = 3
    for cycles in (1, 2):
        o = Opts(m=m, k=k, d=d, u=10, schur=1, block_jacobi=bj, v0=v0.cuda(),
                 max_cycles=cycles)
        gop.update(torch.as_tensor(oop.A0).cuda(), torch.as_tensor(oop.B).cuda())  # fresh space
        gop.solve(b.cuda(), 1e-15, o)
        U, Cm = gop.export_recycle(o)
        st = RecycleState()
        schur.solve_method(oop, b.numpy(), 1e-15, m=m, k=k, d=d, u=10, state=st,
                           v0=v0.numpy().reshape(-1), bj=bool(bj), max_cycles=cycles)
        cc = _principal_cosines(Cm.cpu().numpy().reshape(k, -1).T, st.C)
        cu = _principal_cosines(U.cpu().numpy().reshape(k, -1).T, st.U)
        log(f"  cycles {cycles}: min cos C {cc.min():.12f}, U {cu.min():.12f}")
        assert np.sqrt(max(0.0, 1.0 - cc.min() ** 2)) <= 1e-5
        assert np.sqrt(max(0.0, 1.0 - cu.min() ** 2)) <= 1e-5
