"""The two kernel forms of the odd-even reduced operator S = D_ee - D_eo
D_oo^{-1} D_oe (Sec. 2.2, factored form).  The single-read pair (one kernel
over the odd rows that reads every hop block once and forms both D_oe and D_eo
products from that read, one that sums the products per even row) adds the
same terms in the same order as the two-kernel form, so every result must be
equal bit for bit; the two-kernel form itself is checked against the oracle
in test_gpu_schur.py / test_gpu_schur_bj.py, and the single-read form (the
default) is what those tests now run for FP32 / FP16 blocks with n a multiple
of 8."""
import numpy as np
import pytest
import torch

import synth

from .helpers import log, make_pair, rand_vec

pytestmark = pytest.mark.gpu

STORE = ("f64", "f32", "f16s")


def _both(fn):
    """fn() under the two-kernel form, then under the single-read form."""
    import paper_2205_09104_amd as dc
    try:
        dc.set_reduced_kernels(1)
        a = fn()
        torch.cuda.synchronize()
        dc.set_reduced_kernels(0)
        b = fn()
        torch.cuda.synchronize()
    finally:
        dc.set_reduced_kernels(0)
    return a, b


# n = 2 N_tv = 8, 16, 48, 64; extents of 2 make x + mu and x - mu the same site
@pytest.mark.parametrize("dims,ntv,mu", [((2, 2, 2, 2), 4, 0.0), ((4, 2, 2, 4), 8, 0.2),
                                         ((4, 4, 4, 4), 24, 0.0), ((2, 4, 2, 2), 32, 0.1),
                                         ((4, 4, 2, 6), 24, 0.05)])
def test_single_read_equals_two_kernel_form(dims, ntv, mu):
    gop, oop = make_pair(dims, ntv, 3.0, mu=mu, store=STORE)
    ne = oop.V // 2
    log("reduced forms", dims, ntv, mu)
    for prec in ("f32", "f16s"):
        x = rand_vec(ne, oop.n, 91, 0).to(torch.complex64).cuda()
        for kw in (dict(), dict(adjoint=True), dict(block_jacobi=True)):
            a, b = _both(lambda: gop.apply_reduced(x, prec=prec, **kw))
            d = float((a - b).abs().max())
            log(f"  {prec} {kw}: max |difference| {d:.1e}")
            assert torch.equal(a, b), (prec, kw, d)
            assert bool(torch.isfinite(b).all()) and float(b.abs().max()) > 0.0
    gop.close()


@pytest.mark.parametrize("bj", [0, 1])
def test_single_read_chain_epilogues_equal(bj):
    """q(S) and q(B^{-1} S) chains (first and later chain-step epilogues)."""
    from paper_2205_09104_amd import Opts
    w = synth.WORKLOADS["c1"]
    A, B = synth.operator(w)
    from paper_2205_09104_amd import CoarseOp
    op = CoarseOp(A.cuda(), B.cuda(), w.dims, mu=w.mu, store=STORE)
    ne = w.V // 2
    n = 2 * w.n_tv
    log("reduced forms, chains", bj)
    for prec in ("f32", "f16s"):
        v0 = rand_vec(ne, n, 92, 0).cuda()
        opts = Opts(d=6, v0=v0, schur=1, block_jacobi=bj, prec=prec, seed=1)
        op.poly_setup(opts)
        x = rand_vec(ne, n, 93, 0).to(torch.complex64).cuda()
        a, b = _both(lambda: op.poly_apply(x, opts))
        assert torch.equal(a, b), prec
    op.close()


@pytest.mark.parametrize("prec", ["f32", "f16s"])
def test_single_read_solves_equal(prec):
    """A mixed-precision reduced solve (block Jacobi, polynomial, GCRO-DR with
    refreshes, FP64 outer loop with the residual epilogue) takes the same
    iterates under both forms."""
    from paper_2205_09104_amd import CoarseOp, Opts
    w = synth.WORKLOADS["c1"]
    A, B = synth.operator(w)
    log("reduced forms, solves", prec)
    res = []
    for mode in (1, 0):
        import paper_2205_09104_amd as dc
        dc.set_reduced_kernels(mode)
        try:
            op = CoarseOp(A.cuda(), B.cuda(), w.dims, mu=w.mu, store=STORE)
            o = Opts(m=38, k=8, d=4, u=3, prec=prec, outer=1, inner_tol=1e-1, seed=1, schur=1,
                     block_jacobi=1, ortho=1)
            xs = []
            for r in range(3):
                x, st, rc = op.solve(synth.rhs(w.dims, w.n_tv, r).cuda(), 1e-10, o)
                assert rc == 0, st
                xs.append((x.cpu(), st[0]["matvecs"]))
            op.close()
        finally:
            dc.set_reduced_kernels(0)
        res.append(xs)
    for (xa, ma), (xb, mb) in zip(*res):
        log(f"  matvecs {ma} / {mb}")
        assert ma == mb
        assert torch.equal(xa, xb)


def test_single_read_profile_and_errors(c1_pair):
    """Under the single-read form the profiler's first and second reduced
    kernel slots count the scatter and gather launches (one each per matvec);
    the scatter kernel reports x_e plus the eight partial vectors (9 passes);
    bad mode values are refused."""
    import paper_2205_09104_amd as dc
    from paper_2205_09104_amd import Opts
    from paper_2205_09104_amd._lib import DcError
    gop, oop = c1_pair
    ne = oop.V // 2
    x = rand_vec(ne, oop.n, 94, 0).to(torch.complex64).cuda()
    gop.profile_apply(1)
    gop.apply_reduced(x, prec="f16s")
    assert gop.profile_apply_read("f16s", kernel=1)[0] == 1
    assert gop.profile_apply_read("f16s", kernel=2)[0] == 1
    assert gop.profile_apply_passes("f16s", 1) == 9
    assert gop.profile_apply_passes("f16s", 2) == 10      # 8 partials, x_e, out
    gop.profile_apply(0)
    for bad in (-1, 2, 7):
        with pytest.raises(DcError):
            dc.set_reduced_kernels(bad)
    o = Opts(m=20, d=4, seed=1, schur=1, block_jacobi=1, prec="f16s", outer=1, inner_tol=1e-1)
    gop.profile_apply(1)
    _, st, rc = gop.solve(synth.rhs((4, 4, 4, 4), 8, 0).cuda(), 1e-9, o)
    assert rc == 0
    n1 = gop.profile_apply_read("f16s", kernel=1)[0]
    n2 = gop.profile_apply_read("f16s", kernel=2)[0]
    assert n1 == n2 and n1 > 0
    gop.profile_apply(0)


@pytest.fixture(scope="module")
def c1_pair():
    gop, oop = make_pair((4, 4, 4, 4), 8, 3.0, mu=0.0, store=STORE)
    yield gop, oop
    gop.close()
