"""Reduced-precision storage and the FP64 flexible outer loop (oracle; test
infrastructure only).

The paper runs its coarsest level in single precision and names half-precision
storage as a further step (Sec. 4.2, closing remarks).  The reading used here:

* FP32 storage: each block entry rounded to complex64.
* FP16 storage with a per-block scale: s = FP32(max over the block of
  max(|Re|, |Im|)); code = FP16(entry / s) with round-to-nearest-even, computed
  from the FP64 quotient; decode = FP32(code) * s.  A zero block has s = 0 and
  zero codes.
* Outer loop: flexible GMRES (Saad, SIAM J. Sci. Comput. 14, 1993) in FP64.
  Each outer step applies a variable preconditioner z_j = M_j(v_j), here an
  inner solve with the reduced-precision operator, and keeps Z for the update
  x = x_0 + Z_m y.
"""
from __future__ import annotations

import numpy as np

from .krylov import SolveInfo


def quantize_fp16(blocks: np.ndarray):
    """(code_re, code_im, scale) for complex128 blocks [..., n, n]."""
    re = np.ascontiguousarray(blocks.real)
    im = np.ascontiguousarray(blocks.imag)
    s64 = np.maximum(np.abs(re).max(axis=(-1, -2)), np.abs(im).max(axis=(-1, -2)))
    s = s64.astype(np.float32)
    sd = s.astype(np.float64)
    safe = np.where(sd > 0.0, sd, 1.0)[..., None, None]
    cre = (re / safe).astype(np.float16)
    cim = (im / safe).astype(np.float16)
    zero = (sd == 0.0)[..., None, None]
    cre = np.where(zero, np.float16(0.0), cre)
    cim = np.where(zero, np.float16(0.0), cim)
    return cre, cim, s


def dequantize_fp16(cre, cim, s) -> np.ndarray:
    """complex64 blocks decoded as FP32(code) * s."""
    sf = s.astype(np.float32)[..., None, None]
    return (cre.astype(np.float32) * sf) + 1j * (cim.astype(np.float32) * sf)


def round_fp32(blocks: np.ndarray) -> np.ndarray:
    return blocks.astype(np.complex64)


def fgmres(A, b, tol, m, max_cycles, precond, x0=None):
    """Flexible GMRES(m) in FP64 with a (possibly varying) preconditioner."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    bn = np.linalg.norm(b)
    info = SolveInfo()
    if bn == 0.0:
        info.converged, info.relres = True, 0.0
        return np.zeros_like(b), info
    while True:
        r = b - A(x)
        info.matvecs += 1
        rel = np.linalg.norm(r) / bn
        info.history.append(rel)
        info.relres = rel
        if rel <= tol:
            info.converged = True
            break
        if info.cycles >= max_cycles:
            break
        beta = np.linalg.norm(r)
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m), dtype=np.complex128)
        j_done = 0
        for j in range(m):
            z = precond(V[j])
            Z.append(z)
            w = A(z)
            info.matvecs += 1
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            j_done = j + 1
            e1 = np.zeros(j + 2, dtype=np.complex128)
            e1[0] = beta
            y = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)[0]
            est = np.linalg.norm(e1 - H[:j + 2, :j + 1] @ y)
            if H[j + 1, j] == 0.0 or est <= tol * bn:
                break
            V.append(w / H[j + 1, j])
        e1 = np.zeros(j_done + 1, dtype=np.complex128)
        e1[0] = beta
        y = np.linalg.lstsq(H[:j_done + 1, :j_done], e1, rcond=None)[0]
        for i in range(j_done):
            x = x + y[i] * Z[i]
        info.cycles += 1
        info.iters += j_done
    return x, info


def lowprec_apply(op, store: str):
    """The operator with blocks stored in reduced precision ('f32' or 'f16s'),
    applied in complex64 arithmetic (FP32 accumulation); input and output are
    complex128 [V, n] (cast on the way in and out).

    Reading: the self blocks are stored as given, without the twisted-mass
    term, and i*mu*Gamma5 psi is added in the accumulation precision.  (In FP16
    with a per-block scale, mu ~ 1e-3 would otherwise fall below the
    quantisation step of blocks whose entries are O(1).)"""
    from .operator import gamma5
    A0 = op.A0 if op.A0 is not None else op.A
    if store == "f32":
        A = round_fp32(A0)
        B = round_fp32(op.B)
    elif store == "f16s":
        A = dequantize_fp16(*quantize_fp16(A0))
        B = dequantize_fp16(*quantize_fp16(op.B))
    else:
        raise ValueError(store)
    g5 = gamma5(op.n).astype(np.float32)
    tm = np.float32(op.mu)

    def apply(psi):
        p = psi.astype(np.complex64)
        out = np.einsum("sij,sj->si", A, p) + (1j * tm) * (g5 * p)
        for mu in range(4):
            f = op.fwd[mu]
            b = op.bwd[mu]
            out += np.einsum("sij,sj->si", B[:, mu], p[f])
            Bh = np.conj(np.swapaxes(B[b, mu], 1, 2))
            out += g5 * np.einsum("sij,sj->si", Bh, g5 * p[b])
        return out.astype(np.complex128)
    return apply


def mixed_solve(op, b, tol, store="f32", inner_tol=1e-4, m_inner=30,
                m_outer=10, max_outer=50):
    """FP64 flexible GMRES whose preconditioner is a GMRES(m_inner) solve with
    the reduced-precision operator to relative residual inner_tol."""
    from .krylov import gmres
    from .operator import apply
    shape = (op.V, op.n)
    lo = lowprec_apply(op, store)
    A64 = lambda v: apply(op, v.reshape(shape)).reshape(-1)
    Alo = lambda v: lo(v.reshape(shape)).reshape(-1)

    def precond(v):
        z, _ = gmres(Alo, v, inner_tol, m_inner, 100000)
        return z
    return fgmres(A64, b.reshape(-1), tol, m_outer, max_outer, precond)
