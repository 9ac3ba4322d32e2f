"""Latency-1 pipelined Arnoldi, GMRES and GCRO-DR (oracle; test infrastructure
only).

Sec. 3.5, Alg. 4 (pipelined GMRES) and Alg. 5 (pipelined GCRO-DR), with all
shifts sigma_j = 0 as in the paper.  Besides the orthonormal basis v_j the
process carries precomputed products v^a_j = A v_j (v^a_0 = A v_0 is formed
before the loop, and every later one by the recurrence, so that the only
operator application of step i is w = A v^a_{i-1}).  Step i takes all
coefficients from the one vector v^a_{i-1}:
    b_j = (v^a_{i-1}, c_j),  h_{j,i-1} = (v^a_{i-1}, v_j),
    t   = ||v^a_{i-1}||^2 - sum |h_{j,i-1}|^2 - sum |b_j|^2   (breakdown if t <= 0),
    h_{i,i-1} = sqrt(t),
    v_i   = (v^a_{i-1} - sum v_j h_{j,i-1} - sum c_j b_j) / h_{i,i-1},
    v^a_i = (w - sum v^a_j h_{j,i-1} - sum v^c_j b_j) / h_{i,i-1},
with v^c_j = A c_j for the recycled vectors (recomputed for every cycle, as the
paper does whenever C changes).  In exact arithmetic this is classical
Gram-Schmidt Arnoldi on (I - C C^H) A, so the Hessenberg matrix and the
coefficients B_k are those of the unpipelined process.

Readings: the squares in the expression for t are squared magnitudes (the
coefficients are complex); the text's v^a_0 = v_0 conflicts with the
algorithm, which forms v^a_0 = A v_0, and the latter is what makes
v^a_j = A v_j hold for every j, so it is the one used; the sum over b runs over
all k recycled vectors.
"""
from __future__ import annotations

import numpy as np

from .krylov import dot


def p1_arnoldi(A, v1, m: int, C=None, rhs_norm=None, est_target=None,
               min_steps: int = 0, breakdown_rel: float = 1e-14):
    """Up to m pipelined Arnoldi steps from v1 (normalised inside), deflated
    against the orthonormal vectors C (list) when given.  Returns
    (V, Hbar, Bk, steps, breakdown, applies) with V the steps+1 basis vectors
    and applies the number of applications of A (steps + 1, plus k for the
    v^c_j).  Early stop on the least-squares estimate and the breakdown rule
    as in krylov.arnoldi; breakdown here is t <= (breakdown_rel ||A v_j||)^2."""
    beta = np.linalg.norm(v1)
    C = [] if C is None else list(C)
    k = len(C)
    VC = [A(c) for c in C]
    V = [v1 / beta]
    VA = [A(V[0])]
    applies = k + 1
    H = np.zeros((m + 1, m), dtype=np.complex128)
    Bk = np.zeros((k, m), dtype=np.complex128)
    steps = 0
    breakdown = False
    for i in range(1, m + 1):
        va = VA[i - 1]
        w = A(va)
        applies += 1
        b = np.array([dot(va, c) for c in C], dtype=np.complex128)
        h = np.array([dot(va, v) for v in V[:i]], dtype=np.complex128)
        nrm2 = np.vdot(va, va).real
        t = nrm2 - np.sum(np.abs(h) ** 2) - np.sum(np.abs(b) ** 2)
        H[:i, i - 1] = h
        Bk[:, i - 1] = b
        steps = i
        if t <= (breakdown_rel ** 2) * nrm2:
            H[i, i - 1] = 0.0
            V.append(np.zeros_like(va))
            breakdown = True
            break
        hn = np.sqrt(t)
        H[i, i - 1] = hn
        vi = va - sum(h[j] * V[j] for j in range(i)) - sum(b[j] * C[j] for j in range(k))
        vai = w - sum(h[j] * VA[j] for j in range(i)) - sum(b[j] * VC[j] for j in range(k))
        V.append(vi / hn)
        VA.append(vai / hn)
        if est_target is not None and steps >= min_steps:
            e1 = np.zeros(steps + 1, dtype=np.complex128)
            e1[0] = rhs_norm
            z = np.linalg.lstsq(H[:steps + 1, :steps], e1, rcond=None)[0]
            if np.linalg.norm(e1 - H[:steps + 1, :steps] @ z) <= est_target:
                break
    return V, H[:steps + 1, :steps], Bk[:, :steps], steps, breakdown, applies


def p1_gmres(A, b, tol: float, m: int, max_cycles: int):
    """Restarted pipelined GMRES(m) (Alg. 4 per cycle): x += V_m y with
    y = argmin ||beta e_1 - Hbar y||, restarted from the true residual.
    Returns (x, cycles, relres)."""
    x = np.zeros_like(b)
    bn = np.linalg.norm(b)
    cycles = 0
    while True:
        r = b - A(x)
        rel = np.linalg.norm(r) / bn
        if rel <= tol or cycles >= max_cycles:
            return x, cycles, rel
        beta = np.linalg.norm(r)
        V, Hb, _, j, _, _ = p1_arnoldi(A, r, m, rhs_norm=beta, est_target=tol * bn)
        e1 = np.zeros(j + 1, dtype=np.complex128)
        e1[0] = beta
        y = np.linalg.lstsq(Hb, e1, rcond=None)[0]
        x = x + sum(y[i] * V[i] for i in range(j))
        cycles += 1
