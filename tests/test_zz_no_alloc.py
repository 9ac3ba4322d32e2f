"""dc_apply_reduced_noalloc: the reduced apply for callers that cannot
allocate, against dc_apply_reduced (same kernels: identical results), through
the C ABI, on two handles in a row with the second smaller than the first."""
import ctypes as C

import pytest
import torch

import synth

from .helpers import log, rand_vec

pytestmark = pytest.mark.gpu


def _noalloc(op, x, prec, adjoint):
    from paper_2205_09104_amd import PREC, _ptr, _stream_ptr
    from paper_2205_09104_amd._lib import check, load
    out = torch.empty_like(x)
    check(load().dc_apply_reduced_noalloc(op._h, PREC[prec], int(adjoint), _ptr(x), _ptr(out),
                                          _stream_ptr(None)))
    return out


def _handle(dims, ntv, mu):
    from paper_2205_09104_amd import CoarseOp
    A = synth.self_blocks(dims, ntv, 2.9, 0)
    B = synth.hop_blocks(dims, ntv, 0)
    return CoarseOp(A.cuda(), B.cuda(), dims, mu=mu, store=("f64", "f32", "f16s"))


def test_noalloc_reduced_apply_matches_and_allocates_nothing():
    from paper_2205_09104_amd import device_allocations
    from paper_2205_09104_amd._lib import DC_ERR_STATE, DcError
    big = _handle((8, 8, 4, 4), 24, 0.01)      # 512 even rows, n = 48
    small = _handle((4, 2, 2, 2), 3, 0.2)      # 16 even rows, n = 6 (ragged tiles)
    # before any reduced apply the odd inverses do not exist: refused
    x = rand_vec(small.V // 2, small.n, 90).cuda()
    with pytest.raises(DcError) as e:
        _noalloc(small, x, "f64", False)
    assert e.value.code == DC_ERR_STATE
    for op, seed in ((big, 91), (small, 92)):          # second call: smaller input
        for prec in ("f64", "f32", "f16s"):
            for adjoint in (False, True):
                log("noalloc", op.dims, prec, adjoint)
                x = rand_vec(op.V // 2, op.n, seed).cuda()
                if prec != "f64":
                    x = x.to(torch.complex64)
                ref = op.apply_reduced(x, prec=prec, adjoint=adjoint)   # builds the inverses
                torch.cuda.synchronize()
                n0, b0 = device_allocations()
                for rep in range(2):
                    y = _noalloc(op, x, prec, adjoint)
                    torch.cuda.synchronize()
                    assert torch.equal(y, ref), (op.dims, prec, adjoint, rep)
                assert device_allocations() == (n0, b0)
    # an update makes the inverses stale again until a reduced apply rebuilds them
    A = synth.self_blocks(small.dims, small.n // 2, 3.1, 1)
    B = synth.hop_blocks(small.dims, small.n // 2, 1)
    small.update(A.cuda(), B.cuda())
    x = rand_vec(small.V // 2, small.n, 93).cuda()
    with pytest.raises(DcError) as e:
        _noalloc(small, x, "f64", False)
    assert e.value.code == DC_ERR_STATE
    ref = small.apply_reduced(x)
    assert torch.equal(_noalloc(small, x, "f64", False), ref)
    big.close()
    small.close()
