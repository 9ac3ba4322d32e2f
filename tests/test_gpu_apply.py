"""GPU parity of the D_c apply and the operator build against the oracle:
neighbour table and FP16 codes bit-exact, basis-vector columns bit-exact in
FP64, random vectors within rounding, every storage precision, degenerate
lattice extents, ragged block sizes (n not a multiple of 8)."""
import numpy as np
import pytest
import torch

import synth
from oracle import lattice, mixed
from oracle import operator as dop

from .helpers import log, make_pair, rand_vec, rel

pytestmark = pytest.mark.gpu

SHAPES = [  # (dims, n_tv): several tiles, ragged n, degenerate extents
    ((2, 3, 2, 2), 4),
    ((4, 4, 4, 4), 8),
    ((3, 2, 1, 2), 5),      # n = 10: T = 2 with a ragged tail
    ((1, 1, 2, 1), 1),      # n = 2: one element per lane tile row
    ((2, 2, 2, 3), 20),     # n = 40: T = 5
    ((2, 2, 2, 2), 32),     # n = 64: largest block
]


@pytest.mark.parametrize("dims,ntv", SHAPES)
def test_neighbours_bit_exact(dims, ntv):
    log("neighbours", dims, ntv)
    gop, oop = make_pair(dims, ntv, 3.0)
    nb = gop.neighbours()
    fwd, bwd = lattice.neighbours(dims)
    assert np.array_equal(nb[:4], fwd.astype(np.int32))
    assert np.array_equal(nb[4:], bwd.astype(np.int32))


@pytest.mark.parametrize("dims,ntv", SHAPES)
@pytest.mark.parametrize("mu", [0.0, 0.37])
def test_apply_f64_basis_columns_bit_exact(dims, ntv, mu):
    log("apply f64 basis", dims, ntv, mu)
    gop, oop = make_pair(dims, ntv, 2.5, mu=mu)
    V, n = oop.V, oop.n
    rng = np.random.default_rng(0)
    picks = rng.choice(V * n, size=min(12, V * n), replace=False)
    for p in picks:
        e = np.zeros((V, n), dtype=np.complex128)
        e.reshape(-1)[p] = 1.0
        got = gop.apply(torch.from_numpy(e).cuda()).cpu().numpy()
        want = dop.apply(oop, e)
        if min(dims) >= 2:
            # every output entry is one product (plus exact zeros, or a second
            # product when an extent is 2, and a + b = b + a): bit-exact
            assert np.array_equal(got, want), (dims, ntv, p)
        else:
            # extent 1: three or more couplings land on the same entry, and the
            # summation order is not fixed by the definition
            assert np.max(np.abs(got - want)) <= 4e-16 * np.abs(want).max(), (dims, ntv, p)


def row_err(y, ref):
    """Largest per-site error relative to that site's norm."""
    num = np.linalg.norm(y - ref, axis=-1)
    den = np.maximum(np.linalg.norm(ref, axis=-1), 1e-300)
    return float((num / den).max())


@pytest.mark.parametrize("dims,ntv", SHAPES)
@pytest.mark.parametrize("mu", [0.0, 0.21])
def test_apply_all_precisions_random(dims, ntv, mu):
    log("apply random", dims, ntv, mu)
    gop, oop = make_pair(dims, ntv, 2.5, mu=mu, store=("f64", "f32", "f16s"))
    x = rand_vec(oop.V, oop.n, 7).numpy()
    xg = torch.from_numpy(x).cuda()
    ref = dop.apply(oop, x)
    assert rel(gop.apply(xg).cpu().numpy(), ref) <= 1e-13
    refa = dop.apply_adjoint(oop, x)
    assert rel(gop.apply(xg, adjoint=True).cpu().numpy(), refa) <= 1e-13
    # reduced precision against the oracle's reduced-precision apply of the same
    # storage: globally and row by row (no single site far off)
    for prec in ("f32", "f16s"):
        lo = mixed.lowprec_apply(oop, prec)(x)
        got = gop.apply(xg.to(torch.complex64), prec=prec).cpu().numpy()
        assert rel(got, lo) <= 2e-6, prec
        assert row_err(got, lo) <= 1e-5, prec
        gota = gop.apply(xg.to(torch.complex64), prec=prec, adjoint=True).cpu().numpy()
        assert rel(gota, refa) <= (2e-6 if prec == "f32" else 3e-3), prec
    assert rel(gop.apply(xg.to(torch.complex64), prec="f16s").cpu().numpy(), ref) <= 3e-3


@pytest.mark.parametrize("dims,ntv", SHAPES[:4])
def test_f16_codes_bit_exact(dims, ntv):
    log("f16 codes", dims, ntv)
    gop, oop = make_pair(dims, ntv, 2.5, mu=0.4, store=("f16s",))
    codes, scales = gop.export_f16()
    blocks = np.concatenate([oop.A0[:, None], oop.B], axis=1)      # [V, 5, n, n]
    cre, cim, s = mixed.quantize_fp16(blocks)
    assert np.array_equal(scales, s)
    assert np.array_equal(codes[..., 0], cre.view(np.uint16))
    assert np.array_equal(codes[..., 1], cim.view(np.uint16))


def test_apply_workload_c2_full_size():
    """The 8^4, N_tv = 24 operator (the benchmark workload) at full size."""
    w = synth.WORKLOADS["c2"]
    if "c2" not in synth.load_m0_table():
        pytest.skip("m0 of workload c2 not calibrated")
    log("apply c2 full", w.dims)
    gop, oop = make_pair(w.dims, w.n_tv, w.m0(), w.mu, w.seed, store=("f64", "f32", "f16s"))
    x = rand_vec(oop.V, oop.n, 3).numpy()
    xg = torch.from_numpy(x).cuda()
    ref = dop.apply(oop, x)
    assert rel(gop.apply(xg).cpu().numpy(), ref) <= 1e-13
    assert rel(gop.apply(xg.to(torch.complex64), prec="f32").cpu().numpy(), ref) <= 1e-6
    assert rel(gop.apply(xg.to(torch.complex64), prec="f16s").cpu().numpy(), ref) <= 2e-3


def test_apply_rejects_bad_arguments():
    from paper_2205_09104_amd import DcError
    gop, oop = make_pair((2, 2, 2, 2), 2, 2.0)
    x = torch.zeros((oop.V, oop.n), dtype=torch.complex64, device="cuda")
    with pytest.raises(DcError):
        gop.apply(x, prec="f32")          # FP32 storage not requested


@pytest.mark.parametrize("dims,ntv,R", [((2, 3, 2, 2), 4, 5), ((4, 4, 4, 4), 8, 12),
                                        ((3, 2, 1, 2), 5, 17), ((2, 2, 2, 3), 24, 64),
                                        ((2, 2, 2, 2), 32, 70)])
@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_apply_multi_matches_oracle(dims, ntv, R, mu):
    log("apply multi", dims, ntv, R, mu)
    gop, oop = make_pair(dims, ntv, 2.5, mu=mu, store=("f64", "f32", "f16s"))
    X = np.stack([rand_vec(oop.V, oop.n, 80, r).numpy() for r in range(R)])
    Xg = torch.from_numpy(X).cuda()
    ref = np.stack([dop.apply(oop, x) for x in X])
    refa = np.stack([dop.apply_adjoint(oop, x) for x in X])
    assert rel(gop.apply_multi(Xg).cpu().numpy(), ref) <= 1e-13
    assert rel(gop.apply_multi(Xg, adjoint=True).cpu().numpy(), refa) <= 1e-13
    X32 = Xg.to(torch.complex64)
    lo = np.stack([mixed.lowprec_apply(oop, "f32")(x) for x in X])
    assert rel(gop.apply_multi(X32, prec="f32").cpu().numpy(), lo) <= 2e-6
    lo16 = np.stack([mixed.lowprec_apply(oop, "f16s")(x) for x in X])
    assert rel(gop.apply_multi(X32, prec="f16s").cpu().numpy(), lo16) <= 2e-6
    # same result as R single applies through the other kernel
    single = torch.stack([gop.apply(X32[r], prec="f32") for r in range(R)])
    assert rel(gop.apply_multi(X32, prec="f32").cpu().numpy(), single.cpu().numpy()) <= 2e-6


def test_apply_multi_tiles_agree_bitwise():
    """FP64: every right-hand-side tile of the multi-apply does the same
    arithmetic per output entry (bitwise equal results).  FP32: the tiles
    split the k range of the products differently between the waves (so that
    every wave has the same MFMA work), so they agree to rounding (1e-6
    relative).  The autotuner picks one of them and its result is that
    tile's."""
    import paper_2205_09104_amd as dc
    log("apply multi tiles")
    gop, oop = make_pair((3, 2, 2, 2), 24, 2.5, mu=0.1, store=("f64", "f32"))
    R = 40
    X = torch.stack([rand_vec(oop.V, oop.n, 81, r) for r in range(R)]).cuda()
    X32 = X.to(torch.complex64)
    outs = {}
    try:
        for mode in (16, 32, 64):
            dc.set_multi_tile_mode(mode)
            outs[mode] = (gop.apply_multi(X).cpu(), gop.apply_multi(X32, prec="f32").cpu())
        dc.set_multi_tile_mode(0)       # back to autotuning, table cleared
        auto = (gop.apply_multi(X).cpu(), gop.apply_multi(X32, prec="f32").cpu())
        tiles = (dc.multi_tile("f64", oop.n, R, oop.V), dc.multi_tile("f32", oop.n, R, oop.V))
        with pytest.raises(Exception):
            dc.set_multi_tile_mode(48)
    finally:
        dc.set_multi_tile_mode(0)
    for mode in (32, 64):
        assert torch.equal(outs[mode][0], outs[16][0])
        assert rel(outs[mode][1].numpy(), outs[16][1].numpy()) <= 1e-6
    assert tiles[0] in (16, 32, 64) and tiles[1] in (16, 32, 64)
    assert torch.equal(auto[0], outs[16][0]) and torch.equal(auto[1], outs[tiles[1]][1])
