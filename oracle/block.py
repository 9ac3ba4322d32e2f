"""Block GMRES with a shared Krylov space (oracle; test infrastructure only).

The batching configuration asks for block GMRES over many right-hand sides:
one Krylov space K_m(A, R_0) = span{R_0, A R_0, ..., A^{m-1} R_0} built from
the block of current residuals R_0 (N x r), in which every column takes its
minimal-residual correction.  Block Arnoldi keeps an orthonormal basis of
blocks V_0, ..., V_m (each N x r) and the block upper-Hessenberg matrix
Hbar ((m+1) r x m r) with A V_j = sum_{i <= j+1} V_i H_{i,j}; R_0 = V_0 S_0 is
a thin QR.  Column c of the correction is V_m y_c with
y_c = argmin || E_1 S_0 e_c - Hbar y ||, E_1 the first r columns of the
identity.  Restarted from the true residual of the columns that have not met
their own tolerance (the block shrinks as columns converge).  With a right
preconditioner M (the GMRES polynomial q(A) of Sec. 3.3) the space is built
with A M and the correction is M V_m y_c.

Gram-Schmidt between blocks is classical, applied twice; the new block is
orthonormalised by a QR factorisation (H_{j+1,j} its triangular factor).  A
rank-deficient new block (an invariant subspace reached by some combination of
columns) ends the cycle.
"""
from __future__ import annotations

import numpy as np


def block_arnoldi(A, R0, m: int, targets=None, rank_tol: float = 1e-12):
    """Up to m block steps from R0 (N x r).  A maps N x r blocks to N x r.
    If targets (length r) is given, stop once every column's least-squares
    residual is at or below its target.  Returns (V list of blocks, Hbar,
    S0, steps, residual estimates per column)."""
    N, r = R0.shape
    V0, S0 = np.linalg.qr(R0)
    V = [V0]
    H = np.zeros(((m + 1) * r, m * r), dtype=np.complex128)
    steps = 0
    est = np.linalg.norm(R0, axis=0)
    for j in range(m):
        W = A(V[j])
        hcol = np.zeros(((j + 1) * r, r), dtype=np.complex128)
        for _ in range(2):
            for i in range(j + 1):
                h = V[i].conj().T @ W
                W = W - V[i] @ h
                hcol[i * r:(i + 1) * r] += h
        Q, Rj = np.linalg.qr(W)
        H[:(j + 1) * r, j * r:(j + 1) * r] = hcol
        H[(j + 1) * r:(j + 2) * r, j * r:(j + 1) * r] = Rj
        V.append(Q)
        steps = j + 1
        # least squares of every column over the first steps blocks
        Hs = H[:(steps + 1) * r, :steps * r]
        E = np.zeros(((steps + 1) * r, r), dtype=np.complex128)
        E[:r] = S0
        Y = np.linalg.lstsq(Hs, E, rcond=None)[0]
        est = np.linalg.norm(E - Hs @ Y, axis=0)
        if np.min(np.abs(np.diag(Rj))) <= rank_tol * max(np.abs(np.diag(S0)).max(), 1e-300):
            break
        if targets is not None and np.all(est <= targets):
            break
    return V, H[:(steps + 1) * r, :steps * r], S0, steps, est


def block_gmres(A, B, tols, m: int, max_cycles: int, right=None):
    """Solve A X = B (N x R, per-column relative tolerances) with restarted
    block GMRES(m).  A and right act on single vectors.  Returns (X, info)
    with info = dict(cycles, steps, relres per column, converged)."""
    N, R = B.shape
    M = right or (lambda v: v)
    apply_block = lambda Vb: np.stack([A(M(Vb[:, c])) for c in range(Vb.shape[1])], axis=1)
    X = np.zeros_like(B)
    bn = np.linalg.norm(B, axis=0)
    tols = np.asarray(tols, dtype=np.float64)
    cycles = steps = 0
    rel = np.ones(R)
    while True:
        Rm = B - np.stack([A(X[:, c]) for c in range(R)], axis=1)
        rel = np.linalg.norm(Rm, axis=0) / np.where(bn > 0, bn, 1.0)
        active = np.where(rel > tols)[0]
        if active.size == 0 or cycles >= max_cycles:
            break
        R0 = Rm[:, active]
        V, Hs, S0, j, _ = block_arnoldi(apply_block, R0, m, targets=tols[active] * bn[active])
        r = active.size
        E = np.zeros(((j + 1) * r, r), dtype=np.complex128)
        E[:r] = S0
        Y = np.linalg.lstsq(Hs, E, rcond=None)[0]
        Vm = np.concatenate(V[:j], axis=1)
        U = Vm @ Y
        for a, c in enumerate(active):
            X[:, c] += M(U[:, a])
        cycles += 1
        steps += j
    return X, {"cycles": cycles, "steps": steps, "relres": rel,
               "converged": bool(np.all(rel <= tols))}
