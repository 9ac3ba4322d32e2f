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

Numerically dependent residual columns (restarts of many columns whose
residuals have collapsed onto a few slow directions) cannot all generate the
space: the generating block is the orthonormalised set of columns picked
greedily, each having the largest part outside the span of the earlier picks
(pivoting on the column-scaled block), while that part's squared relative
size exceeds sel_piv.  Every column still takes its least-squares
minimiser over the space those picks generate (the cycle then runs up to
m c / (picks) block steps, so that its space keeps the dimension m c that c
independent columns would give): with R_0 = [r_1 .. r_c] and
orthonormal blocks V_0 .. V_{j+1}, column a minimises
|| g_a - Hbar y || with g_a = [V_0^H r_a; V_1^H r_a; ...; V_{j+1}^H r_a] --
the parts of r_a outside V_0 are not orthogonal to the later blocks -- and
its residual norm is sqrt(|| g_a - Hbar y_a ||^2 + ||r_a||^2 - ||g_a||^2).

Deflation against a recycled pair (U, C) with C = A M U orthonormal (the
GCRO-DR space of Sec. 3.4): every new residual block starts with
x += M U C^H r, r -= C C^H r, the block Arnoldi runs on (I - C C^H) A M with
B_k = C^H A M V, and column a's correction M (V y_a - U B_k y_a) leaves the
residual r_a - V Hbar y_a (the C components cancel).

Block recycling (the GCRO-DR update of Sec. 3.4 with the block relation in
place of the single-vector one): a cycle of s = j nb basis vectors gives
A M [U D, V_s] = [C, V_{s+nb}] G with D = diag(1 / ||u_i||) and
G = [[D, B_k], [0, Hbar]] (without a recycle space G = Hbar).  The new space
takes the k harmonic Ritz vectors of that relation with the smallest |theta|:
G^H G z = theta G^H (What^H Vhat) z with Vhat = [U D, V_s], What =
[C, V_{s+nb}] (What^H Vhat = [I_s; 0] without a recycle space); P_k their
eigenvectors, [Q, R] = qr(G P_k), C = What Q, U = Vhat P_k R^{-1}.  It is
built after the first cycle that has at least k basis vectors and refreshed
after each later cycle until it has been updated u times.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


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


def select_generators(R0, sel_piv: float):
    """Indices of the residual columns that generate the space, in pick order
    (greedy pivoting on the column-scaled block, written out as Gram-Schmidt
    twice): each pick is the column with the largest squared part outside the
    span of the earlier picks (the lowest index among parts equal to a relative
    1e-10, so the unit columns' first pick is column 0), kept while that part
    exceeds sel_piv."""
    d = np.linalg.norm(R0, axis=0)
    cols = [R0[:, i] / d[i] if d[i] > 0 else None for i in range(R0.shape[1])]
    Q, picks = [], []
    while True:
        rests = {}
        for i, c in enumerate(cols):
            if c is None or i in picks:
                continue
            w = c.copy()
            for _ in range(2):
                for q in Q:
                    w = w - np.vdot(q, w) * q
            rests[i] = float(np.vdot(w, w).real)
        if not rests:
            break
        top = max(rests.values())
        # parts within a relative 1e-10 of the largest count as equal
        best = min(i for i, r in rests.items() if r >= top * (1.0 - 1e-10))
        if not rests[best] > sel_piv:
            break
        w = cols[best].copy()
        for _ in range(2):
            for q in Q:
                w = w - np.vdot(q, w) * q
        Q.append(w / np.linalg.norm(w))
        picks.append(best)
    return np.array(picks, dtype=np.int64)


def ls_rhs(Vblocks, R):
    """Right-hand sides of every column's least squares: the coefficients of
    the residual columns R on each basis block, stacked (V_i^H R)."""
    return np.concatenate([Vb.conj().T @ R for Vb in Vblocks], axis=0)


def _cycle(Ablk, R, m, targets, sel_piv, C):
    """One block cycle for the residual block R (N x c, already deflated when
    C is given).  Returns (Vblocks, Hbar, Y, steps, est, Bk, picks)."""
    N, c = R.shape
    picks = select_generators(R, sel_piv)
    if picks.size == 0:
        return [], None, None, 0, np.linalg.norm(R, axis=0), None, picks
    V0, _ = np.linalg.qr(R[:, picks])
    nb = V0.shape[1]
    V = [V0]
    H = np.zeros(((m + 1) * nb, m * nb), dtype=np.complex128)
    k = 0 if C is None else C.shape[1]
    Bk = np.zeros((k, m * nb), dtype=np.complex128)
    rn2 = np.linalg.norm(R, axis=0) ** 2
    steps, Y = 0, None
    est = np.sqrt(rn2)
    for j in range(m):
        W = Ablk(V[j])
        hcol = np.zeros(((j + 1) * nb, nb), dtype=np.complex128)
        for _ in range(2):
            if k:
                b = C.conj().T @ W
                W = W - C @ b
                Bk[:, j * nb:(j + 1) * nb] += b
            for i in range(j + 1):
                h = V[i].conj().T @ W
                W = W - V[i] @ h
                hcol[i * nb:(i + 1) * nb] += h
        Q, Rj = np.linalg.qr(W)
        H[:(j + 1) * nb, j * nb:(j + 1) * nb] = hcol
        H[(j + 1) * nb:(j + 2) * nb, j * nb:(j + 1) * nb] = Rj
        V.append(Q)
        steps = j + 1
        Hs = H[:(steps + 1) * nb, :steps * nb]
        G = ls_rhs(V, R)
        Y = np.linalg.lstsq(Hs, G, rcond=None)[0]
        inside = np.linalg.norm(G - Hs @ Y, axis=0) ** 2
        outside = np.maximum(rn2 - np.linalg.norm(G, axis=0) ** 2, 0.0)
        est = np.sqrt(inside + outside)
        if np.min(np.abs(np.diag(Rj))) <= 1e-12 * max(np.linalg.norm(R, axis=0).max(), 1e-300):
            break
        if targets is not None and np.all(est <= targets):
            break
    return V, H[:(steps + 1) * nb, :steps * nb], Y, steps, est, Bk[:, :steps * nb], picks


def harmonic_space(G, What, Vhat, k: int):
    """The k harmonic Ritz vectors of A M Vhat = What G with the smallest
    |theta| (G^H G z = theta G^H (What^H Vhat) z), as the recycle pair
    (U, C): [Q, R] = qr(G P_k), C = What Q, U = Vhat P_k R^{-1}."""
    WV = What.conj().T @ Vhat
    theta, Z = sla.eig(G.conj().T @ G, G.conj().T @ WV)
    mag = np.abs(theta)
    mag[~np.isfinite(mag)] = np.inf
    P = Z[:, np.argsort(mag, kind="stable")[:k]]
    Q, Rr = np.linalg.qr(G @ P)
    return Vhat @ P @ np.linalg.inv(Rr), What @ Q


def block_gmres(A, B, tols, m: int, max_cycles: int, right=None, U=None, C=None,
                sel_piv: float = 1e-12, recycle=None, k: int = 0, u: int = 0):
    """Solve A X = B (N x R, per-column relative tolerances) with restarted
    block GMRES(m).  A and right act on single vectors.  U, C: an optional
    frozen recycle space (C = A right(U), orthonormal columns) to deflate
    against.  recycle: a state with fields U, C, updates (None: no
    recycling) that the cycles build and refresh (k vectors, u updates) and
    deflate against.  Returns (X, info) with info = dict(cycles, steps,
    relres per column, converged, generators: the generating-block size of
    each cycle)."""
    N, R = B.shape
    M = right or (lambda v: v)
    apply_block = lambda Vb: np.stack([A(M(Vb[:, c])) for c in range(Vb.shape[1])], axis=1)
    Mblk = lambda Vb: np.stack([M(Vb[:, c]) for c in range(Vb.shape[1])], axis=1)
    X = np.zeros_like(B)
    bn = np.linalg.norm(B, axis=0)
    tols = np.asarray(tols, dtype=np.float64)
    cycles = steps = 0
    gens = []
    rel = np.ones(R)
    while True:
        Rm = B - np.stack([A(X[:, c]) for c in range(R)], axis=1)
        rel = np.linalg.norm(Rm, axis=0) / np.where(bn > 0, bn, 1.0)
        active = np.where(rel > tols)[0]
        if active.size == 0 or cycles >= max_cycles:
            break
        R0 = Rm[:, active]
        if recycle is not None:
            U, C = recycle.U, recycle.C
        if C is not None:
            coef = C.conj().T @ R0
            X[:, active] += Mblk(U @ coef)
            R0 = R0 - C @ coef
        # a block with fewer generators than columns keeps the dimension of
        # the cycle's space: up to m * (columns) / (generators) block steps
        npick = select_generators(R0, sel_piv).size
        m_eff = m if npick in (0, R0.shape[1]) else (m * R0.shape[1]) // npick
        V, Hs, Y, j, _, Bk, picks = _cycle(apply_block, R0, m_eff, tols[active] * bn[active],
                                           sel_piv, C)
        gens.append(int(picks.size))
        cycles += 1
        steps += j
        if j == 0:
            break
        Vm = np.concatenate(V[:j], axis=1)
        corr = Vm @ Y
        if C is not None:
            corr = corr - U @ (Bk @ Y)
        X[:, active] += Mblk(corr)
        if recycle is not None and k > 0:
            Vw = np.concatenate(V[:j + 1], axis=1)
            if C is None and Vm.shape[1] >= k:
                recycle.U, recycle.C = harmonic_space(Hs, Vw, Vm, k)
                recycle.updates = 1
            elif C is not None and recycle.updates < u:
                kk = U.shape[1]
                dk = 1.0 / np.linalg.norm(U, axis=0)
                G = np.zeros((kk + Hs.shape[0], kk + Hs.shape[1]), dtype=np.complex128)
                G[:kk, :kk] = np.diag(dk)
                G[:kk, kk:] = Bk
                G[kk:, kk:] = Hs
                recycle.U, recycle.C = harmonic_space(
                    G, np.concatenate([C, Vw], axis=1),
                    np.concatenate([U * dk[None, :], Vm], axis=1), kk)
                recycle.updates += 1
    return X, {"cycles": cycles, "steps": steps, "relres": rel,
               "converged": bool(np.all(rel <= tols)), "generators": gens}
