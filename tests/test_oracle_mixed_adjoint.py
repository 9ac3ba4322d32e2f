"""Pins for FP16 quantisation (round-to-nearest-even by exact rational brute
force), the FP64 flexible outer loop, adjoint solves and gradients (central
finite differences of a dense solve)."""
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import adjoint as adj
from oracle import mixed
from oracle import operator as dop
from oracle.krylov import gmres

_F16 = np.arange(65536, dtype=np.uint16).view(np.float16)
_F16 = np.unique(_F16[np.isfinite(_F16)].astype(np.float64))


def rne_half_bruteforce(q: float) -> float:
    """Nearest float16 value to q with ties to the even significand, by exact
    rational comparison against every finite float16 value."""
    i = np.searchsorted(_F16, q)
    cands = [_F16[j] for j in (i - 1, i) if 0 <= j < _F16.size]
    fq = Fraction(q)
    best = min(abs(Fraction(c) - fq) for c in cands)
    ties = [c for c in cands if abs(Fraction(c) - fq) == best]
    if len(ties) == 1:
        return ties[0]
    even = [c for c in ties if (np.float16(c).view(np.uint16) & 1) == 0]
    return even[0]


def test_fp16_quantisation_is_rne():
    rng = np.random.default_rng(0)
    vals = list(rng.uniform(-1, 1, 3000))
    vals += list(rng.uniform(-1, 1, 500) * 2.0 ** -16)          # subnormal range
    # exact midpoints between neighbouring halves, and one float64 ulp either side
    for k in range(200):
        a = _F16[_F16.size // 2 + k * 37 % 30000]
        b = _F16[_F16.size // 2 + k * 37 % 30000 + 1]
        if abs(a) > 1 or abs(b) > 1:
            continue
        mid = (a + b) / 2
        vals += [mid, np.nextafter(mid, 2.0), np.nextafter(mid, -2.0), -mid]
    vals = np.array(vals)
    n = 8
    per = n * n - 1                     # entry (0, 0) of each block holds 1 + 1j
    nb = len(vals) // per + 1
    padded = np.zeros(nb * per)
    padded[:len(vals)] = vals
    blocks = np.zeros((nb, n * n), dtype=np.complex128)
    blocks[:, 0] = 1.0 + 1.0j           # scale exactly 1: codes = entries rounded
    blocks[:, 1:] = (padded + 1j * padded[::-1]).reshape(nb, per)
    blocks = blocks.reshape(nb, n, n)
    cre, cim, s = mixed.quantize_fp16(blocks)
    assert np.all(s == 1.0)
    got_re = cre.reshape(nb, n * n)[:, 1:].reshape(-1).astype(np.float64)
    got_im = cim.reshape(nb, n * n)[:, 1:].reshape(-1).astype(np.float64)
    want_re = np.array([rne_half_bruteforce(v) for v in padded])
    want_im = np.array([rne_half_bruteforce(v) for v in padded[::-1]])
    assert np.array_equal(got_re, want_re)
    assert np.array_equal(got_im, want_im)


def test_fp16_quantisation_error_bound_and_zero_block():
    A = synth.self_blocks((2, 2, 2, 2), 4, 2.5, seed=3).numpy()
    A[3] = 0.0
    cre, cim, s = mixed.quantize_fp16(A)
    assert s[3] == 0 and not np.any(cre[3]) and not np.any(cim[3])
    dq = mixed.dequantize_fp16(cre, cim, s).astype(np.complex128)
    err = np.maximum(np.abs(dq.real - A.real), np.abs(dq.imag - A.imag))
    bound = (2.0 ** -11 + 2.0 ** -22) * s.astype(np.float64)[:, None, None]
    assert np.all(err <= bound)
    # the scale is the largest |Re| or |Im| of the block, rounded to FP32
    ref = np.maximum(np.abs(A.real).max(axis=(1, 2)), np.abs(A.imag).max(axis=(1, 2)))
    assert np.array_equal(s, ref.astype(np.float32))


def tiny_op(mu=0.0, dims=(2, 2, 2, 2), ntv=3, seed=0):
    A = synth.self_blocks(dims, ntv, 3.6, seed).numpy()
    B = synth.hop_blocks(dims, ntv, seed).numpy()
    return dop.build(dims, A, B, mu)


def test_fgmres_exact_and_identity_preconditioner():
    op = tiny_op(mu=0.1)
    Dm = dop.dense(op)
    rng = np.random.default_rng(1)
    b = rng.standard_normal(op.N) + 1j * rng.standard_normal(op.N)
    A = lambda v: Dm @ v
    Dinv = np.linalg.inv(Dm)
    x, info = mixed.fgmres(A, b, 1e-12, 10, 5, lambda v: Dinv @ v)
    assert info.converged and info.iters == 1
    x1, i1 = mixed.fgmres(A, b, 1e-10, 8, 500, lambda v: v)
    x2, i2 = gmres(A, b, 1e-10, 8, 500)
    assert i1.iters == i2.iters
    assert np.allclose(x1, x2, atol=1e-12 * np.linalg.norm(x2))


@pytest.mark.parametrize("store", ["f32", "f16s"])
def test_mixed_precision_reaches_fp64_accuracy(store):
    op = tiny_op(mu=0.05, dims=(3, 2, 2, 2), ntv=4)
    Dm = dop.dense(op)
    rng = np.random.default_rng(2)
    b = rng.standard_normal(op.N) + 1j * rng.standard_normal(op.N)
    x, info = mixed.mixed_solve(op, b, 1e-10, store=store, inner_tol=1e-3)
    assert info.converged
    assert np.linalg.norm(b - Dm @ x) <= 1e-10 * np.linalg.norm(b)
    xref = np.linalg.solve(Dm, b)
    assert np.linalg.norm(x - xref) <= 1e-6 * np.linalg.norm(xref)


def test_lowprec_apply_close_to_fp64():
    op = tiny_op(mu=0.05)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal((op.V, op.n)) + 1j * rng.standard_normal((op.V, op.n))
    ref = dop.apply(op, psi)
    for store, tol in (("f32", 1e-6), ("f16s", 2e-3)):
        got = mixed.lowprec_apply(op, store)(psi)
        assert np.linalg.norm(got - ref) <= tol * np.linalg.norm(ref)


# ------------------------------------------------------------- adjoint / grads

def test_adjoint_solve_identity():
    op = tiny_op(mu=0.2)
    rng = np.random.default_rng(4)
    b = rng.standard_normal((op.V, op.n)) + 1j * rng.standard_normal((op.V, op.n))
    c = rng.standard_normal((op.V, op.n)) + 1j * rng.standard_normal((op.V, op.n))
    x, _ = adj.solve(op, b, 1e-13)
    lam, _ = adj.solve_adjoint(op, c, 1e-13)
    lhs = np.vdot(c, x)
    rhs = np.vdot(lam, b)
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def _loss_dense(op, b, c):
    return float(np.real(np.vdot(c.reshape(-1), np.linalg.solve(dop.dense(op), b.reshape(-1)))))


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_gradients_match_central_differences(mu):
    op = tiny_op(mu=mu)
    rng = np.random.default_rng(5)
    b = rng.standard_normal((op.V, op.n)) + 1j * rng.standard_normal((op.V, op.n))
    c = rng.standard_normal((op.V, op.n)) + 1j * rng.standard_normal((op.V, op.n))
    L, x, lam, gb, gB = adj.loss_grads(op, b, c, tol=1e-13)
    h = 1e-6
    # right-hand side entries
    for (s, i) in [(0, 0), (5, 3), (11, 5)]:
        for part, unit in (("re", 1.0), ("im", 1j)):
            bp = b.copy(); bp[s, i] += h * unit
            bm = b.copy(); bm[s, i] -= h * unit
            fd = (_loss_dense(op, bp, c) - _loss_dense(op, bm, c)) / (2 * h)
            want = gb[s, i].real if part == "re" else gb[s, i].imag
            assert abs(fd - want) <= 1e-6 * max(1.0, abs(want))
    # tied forward hop entries: perturbing B moves both couplings
    for (s, mu_d, i, j) in [(0, 0, 0, 1), (7, 2, 4, 2), (13, 3, 5, 5)]:
        for part, unit in (("re", 1.0), ("im", 1j)):
            Bp = op.B.copy(); Bp[s, mu_d, i, j] += h * unit
            Bm = op.B.copy(); Bm[s, mu_d, i, j] -= h * unit
            opp = dop.CoarseOp(op.dims, op.n, op.A, Bp, op.mu, op.fwd, op.bwd)
            opm = dop.CoarseOp(op.dims, op.n, op.A, Bm, op.mu, op.fwd, op.bwd)
            fd = (_loss_dense(opp, b, c) - _loss_dense(opm, b, c)) / (2 * h)
            g = gB[s, mu_d, i, j]
            want = g.real if part == "re" else g.imag
            assert abs(fd - want) <= 1e-6 * max(1.0, abs(want))


def test_untied_gradient_matches_single_coupling_difference():
    op = tiny_op(mu=0.1, dims=(3, 3, 2, 2))
    rng = np.random.default_rng(6)
    b = rng.standard_normal((op.V, op.n)) + 1j * rng.standard_normal((op.V, op.n))
    c = rng.standard_normal((op.V, op.n)) + 1j * rng.standard_normal((op.V, op.n))
    Dm = dop.dense(op)
    x = np.linalg.solve(Dm, b.reshape(-1)).reshape(op.V, op.n)
    lam = np.linalg.solve(Dm.conj().T, c.reshape(-1)).reshape(op.V, op.n)
    G = adj.grad_hops_untied(op, lam, x)
    n = op.n
    h = 1e-6
    for (s, d, i, j) in [(1, 0, 2, 3), (4, 5, 0, 0), (9, 7, 5, 1)]:
        y = op.fwd[d, s] if d < 4 else op.bwd[d - 4, s]
        for unit in (1.0, 1j):
            E = np.zeros_like(Dm)
            E[s * n + i, y * n + j] = h * unit
            lp = np.real(np.vdot(c.reshape(-1), np.linalg.solve(Dm + E, b.reshape(-1))))
            lm = np.real(np.vdot(c.reshape(-1), np.linalg.solve(Dm - E, b.reshape(-1))))
            fd = (lp - lm) / (2 * h)
            want = G[s, d, i, j].real if unit == 1.0 else G[s, d, i, j].imag
            assert abs(fd - want) <= 1e-6 * max(1.0, abs(want))
