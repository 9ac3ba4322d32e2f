"""Shared helpers of the GPU parity tests: build the same seeded operator for the
GPU library (device tensors) and for the oracle (host arrays)."""
import sys

import numpy as np
import torch

import synth
from oracle import operator as dop


def log(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def make_pair(dims, ntv, m0, mu=0.0, seed=0, store=("f64",)):
    """(gpu CoarseOp, oracle CoarseOp, A host, B host) for a seeded operator."""
    from paper_2205_09104_amd import CoarseOp
    A = synth.self_blocks(dims, ntv, m0, seed)
    B = synth.hop_blocks(dims, ntv, seed)
    gop = CoarseOp(A.cuda(), B.cuda(), dims, mu=mu, store=store)
    oop = dop.build(dims, A.numpy(), B.numpy(), mu)
    return gop, oop


def workload_pair(name, store=("f64",)):
    import pytest
    w = synth.WORKLOADS[name]
    if name not in synth.load_m0_table():
        pytest.skip(f"m0 of workload {name} not calibrated")
    return make_pair(w.dims, w.n_tv, w.m0(), w.mu, w.seed, store) + (w,)


def rand_vec(V, n, seed, sub=0):
    idx = torch.arange(V * n, dtype=torch.int64)
    return synth.complex_normal(idx, synth.STREAM_AUX, seed, sub).reshape(V, n)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def oracle_relres(oop, x, b, adjoint=False):
    x = np.asarray(x).reshape(oop.V, oop.n)
    b = np.asarray(b).reshape(oop.V, oop.n)
    Dx = dop.apply_adjoint(oop, x) if adjoint else dop.apply(oop, x)
    return float(np.linalg.norm(b - Dx) / np.linalg.norm(b))
