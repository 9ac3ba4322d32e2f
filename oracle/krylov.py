"""Arnoldi and restarted GMRES(m) (oracle; test infrastructure only).

Sec. 3.1: GMRES takes x_m from x_0 + K_m(A, r_0) with minimal residual 2-norm.
The Arnoldi process (Alg. 1) builds an orthonormal basis V and the
(m+1) x m Hessenberg matrix Hbar with h_ij = (A v_j, v_i) = v_i^H A v_j; the
modified Gram-Schmidt variant uses the partially orthogonalised vector for each
coefficient.  The iterate is x_0 + V_m z with z = argmin ||beta e_1 - Hbar z||.
GMRES(m) restarts from the last iterate after m steps.

Vectors are flat complex128 arrays; operators are callables flat -> flat.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def dot(a, b):
    """(a, b) = b^H a, the inner product used by the paper."""
    return np.vdot(b, a)


def orthogonalise(w, basis, ortho: str):
    """Orthogonalise w against the list `basis` (orthonormal vectors).

    Returns (w', h) with h[i] the accumulated coefficient of basis[i].
    'cgs'  : classical Gram-Schmidt, all coefficients from the same w (Alg. 1).
    'mgs'  : modified Gram-Schmidt, each coefficient from the updated w.
    'cgs2' : classical Gram-Schmidt applied twice, coefficients summed.
    'ss'   : classical Gram-Schmidt once (the coefficients of the single-sync
             process; its norm is formed in `arnoldi`).
    """
    h = np.zeros(len(basis), dtype=np.complex128)
    if ortho == "mgs":
        for i, v in enumerate(basis):
            h[i] = dot(w, v)
            w = w - h[i] * v
        return w, h
    passes = 2 if ortho == "cgs2" else 1   # 'cgs' and 'ss': one pass
    for _ in range(passes):
        hp = np.array([dot(w, v) for v in basis], dtype=np.complex128)
        for i, v in enumerate(basis):
            w = w - hp[i] * v
        h += hp
    return w, h


@dataclass
class ArnoldiResult:
    V: list                  # j+1 basis vectors
    Hbar: np.ndarray         # (j+1) x j
    Bk: np.ndarray | None    # k x j deflation coefficients C^H A V_j
    steps: int
    breakdown: bool


def arnoldi(A, v1, m: int, ortho: str = "mgs", C=None, rhs_norm=None,
            est_target=None, min_steps: int = 0, breakdown_rel: float = 1e-14):
    """Up to m Arnoldi steps from v1 (normalised inside).

    If C (list of orthonormal vectors) is given, each new vector is first made
    orthogonal to C (the deflated operator (I - C C^H) A of Sec. 3.4) and the
    coefficients C^H A v_j are returned as Bk.
    If est_target is given, stop as soon as the GMRES least-squares residual
    (with right-hand side rhs_norm * e_1) drops to est_target, but not before
    min_steps steps.
    Breakdown: stop when h_{j+1,j} <= breakdown_rel * ||A v_j|| (the exact-zero
    test of Alg. 1 with a rounding threshold).

    ortho='ss' is the single-sync process of Sec. 3.5 without the lag: the
    coefficients of one classical Gram-Schmidt pass and ||A v_j||^2 come from
    the same reduction, h_{j+1,j}^2 = ||A v_j||^2 - sum |h|^2 - sum |b|^2
    (breakdown when that is <= (breakdown_rel ||A v_j||)^2), and the new
    vector is the orthogonalised one divided by that h.  ortho='p1' runs the
    latency-1 pipelined process of Alg. 4 / Alg. 5 (pipelined.p1_arnoldi).
    """
    if ortho == "p1":
        from .pipelined import p1_arnoldi
        V, Hb, Bk, steps, brk, _ = p1_arnoldi(A, v1, m, C=C, rhs_norm=rhs_norm,
                                              est_target=est_target, min_steps=min_steps,
                                              breakdown_rel=breakdown_rel)
        return ArnoldiResult(V, Hb, Bk if C is not None else None, steps, brk)
    beta = np.linalg.norm(v1)
    V = [v1 / beta]
    H = np.zeros((m + 1, m), dtype=np.complex128)
    k = 0 if C is None else len(C)
    Bk = np.zeros((k, m), dtype=np.complex128)
    steps = 0
    breakdown = False
    for j in range(m):
        w = A(V[j])
        wnorm0 = np.linalg.norm(w)
        if k:
            w, b = orthogonalise(w, C, ortho)
            Bk[:, j] = b
        w, h = orthogonalise(w, V, ortho)
        H[:j + 1, j] = h
        if ortho == "ss":
            t = wnorm0 ** 2 - np.sum(np.abs(h) ** 2) - (np.sum(np.abs(Bk[:, j]) ** 2) if k else 0.0)
            hn = np.sqrt(t) if t > (breakdown_rel * wnorm0) ** 2 else 0.0
        else:
            hn = np.linalg.norm(w)
        H[j + 1, j] = hn
        steps = j + 1
        if hn <= breakdown_rel * wnorm0:
            # invariant subspace: A V_j = V_j H_j exactly; a zero v_{j+1} keeps
            # the relation A V_j = V_{j+1} Hbar_j with a zero last row
            H[j + 1, j] = 0.0
            V.append(np.zeros_like(w))
            breakdown = True
            break
        V.append(w / hn)
        if est_target is not None and steps >= min_steps:
            e1 = np.zeros(steps + 1, dtype=np.complex128)
            e1[0] = rhs_norm
            z = np.linalg.lstsq(H[:steps + 1, :steps], e1, rcond=None)[0]
            est = np.linalg.norm(e1 - H[:steps + 1, :steps] @ z)
            if est <= est_target:
                break
    return ArnoldiResult(V, H[:steps + 1, :steps], Bk[:, :steps], steps, breakdown)


@dataclass
class SolveInfo:
    converged: bool = False
    cycles: int = 0
    iters: int = 0
    matvecs: int = 0
    relres: float = np.inf
    history: list = field(default_factory=list)
    final_rhat: object = None     # last (recursively updated) preconditioned residual


class Counted:
    """Wraps an operator and counts its applications."""

    def __init__(self, f):
        self.f = f
        self.count = 0

    def __call__(self, v):
        self.count += 1
        return self.f(v)


def identity(v):
    return v


def gmres(A, b, tol: float, m: int, max_cycles: int, x0=None,
          left=None, right=None, ortho: str = "mgs"):
    """Restarted GMRES(m) for A x = b with optional left preconditioner L and
    right preconditioner R: Arnoldi runs on L A R, the start residual is
    L (b - A x), and the iterate is updated by x += R(V z).

    Stops when the true residual ||b - A x|| / ||b|| <= tol (checked in FP64 at
    every cycle end); inside a cycle it stops early when the least-squares
    residual estimate reaches the target, and the true residual then decides.
    """
    L = left or identity
    R = right or identity
    Ac = Counted(A)
    Ahat = lambda v: L(Ac(R(v)))
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    bn = np.linalg.norm(b)
    info = SolveInfo()
    if bn == 0.0:
        info.converged = True
        info.relres = 0.0
        return np.zeros_like(b), info
    safety = 1.0
    while True:
        r = b - Ac(x)
        rel = np.linalg.norm(r) / bn
        info.relres = rel
        info.history.append(rel)
        if rel <= tol:
            info.converged = True
            break
        if info.cycles >= max_cycles:
            break
        rhat = L(r)
        beta = np.linalg.norm(rhat)
        target = tol * bn * (beta / np.linalg.norm(r)) * safety
        ar = arnoldi(Ahat, rhat, m, ortho, rhs_norm=beta, est_target=target)
        j = ar.steps
        e1 = np.zeros(j + 1, dtype=np.complex128)
        e1[0] = beta
        z = np.linalg.lstsq(ar.Hbar, e1, rcond=None)[0]
        upd = np.zeros_like(b)
        for i in range(j):
            upd += z[i] * ar.V[i]
        x = x + R(upd)
        info.cycles += 1
        info.iters += j
        est = np.linalg.norm(e1 - ar.Hbar @ z)
        if est <= target:
            safety *= 0.5
    info.matvecs = Ac.count
    return x, info
