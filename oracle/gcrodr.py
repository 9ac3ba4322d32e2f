"""GCRO-DR: deflated restarts with Krylov-subspace recycling (oracle; test
infrastructure only).

Sec. 3.4 describes one cycle: keep k approximate small eigenmodes as U_k with
C_k = A U_k orthonormal; run m-k Arnoldi steps on (I - C_k C_k^H) A from the
current residual, giving A [U_k V_{m-k}] = [C_k V_{m-k+1}] G_m with
G_m = [[I_k, B_k], [0, Hbar_{m-k}]], B_k = C_k^H A V_{m-k}; minimise the residual
over span(U_k, V_{m-k}) through a least-squares problem with G_m; refresh U_k,
C_k from harmonic Ritz vectors.  The first cycle without a recycle space is a
GMRES(m) cycle.  U_k and C_k carry over to later right-hand sides (same
matrix), and after u updates they are frozen (Sec. 4.1.1, parameter u).  The
step-by-step algorithm is that of Parks, de Sturler, Mackey, Johnson and Maiti
(SIAM J. Sci. Comput. 28, 2006), restated here:

  construction cycle (no U):  GMRES(m) cycle; P_k = eigenvectors of
      H_m + |h_{m+1,m}|^2 H_m^{-H} e_m e_m^T for the k smallest |theta|;
      [Q, R] = qr(Hbar_m P_k); C = V_{m+1} Q; U = V_m P_k R^{-1}.
  new right-hand side with U:  (matrix changed: [Q,R] = qr(A U), C = Q,
      U = U R^{-1})  x += U C^H r;  r -= C C^H r.
  cycle:  v_1 = r/||r||; m-k deflated Arnoldi steps -> V, Hbar, B_k;
      D_k = diag(1/||u_i||); Uh = U D_k; Vhat = [Uh V_{m-k}];
      What = [C V_{m-k+1}]; G = [[D_k, B_k], [0, Hbar]];
      y = argmin || ||r|| e_{k+1} - G y ||; x += Vhat y; r -= What G y;
      update (if fewer than u updates so far): solve
      G^H G z = theta G^H What^H Vhat z, P_k = eigenvectors of the k smallest
      |theta|; [Q, R] = qr(G P_k); C = What Q; U = Vhat P_k R^{-1}.

Here A is the fully preconditioned operator L D R (Sec. 3.3, Sec. 3.2), the
residual is the left-preconditioned one L(b - D x), and every update of x is
passed through the right preconditioner R = q(.).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from .krylov import Counted, SolveInfo, arnoldi, identity
from .poly import harmonic_ritz_pairs


@dataclass
class RecycleState:
    U: np.ndarray | None = None     # N x k
    C: np.ndarray | None = None     # N x k, C = A U, C^H C = I
    updates: int = 0                # number of builds/refreshes so far


def _smallest(theta, vecs, k):
    mag = np.abs(theta)
    mag[~np.isfinite(mag)] = np.inf
    order = np.argsort(mag, kind="stable")[:k]
    return vecs[:, order]


def _combine(vectors, coeffs):
    """sum_i vectors[i] * coeffs[i, :] for a list of vectors -> N x c array."""
    M = np.stack(vectors, axis=1)
    return M @ coeffs


def gcrodr(D, b, tol, m, k, u, max_cycles, state: RecycleState,
           left=None, right=None, x0=None, matrix_changed=False,
           ortho="mgs"):
    """Solve D x = b to true relative residual tol with GCRO-DR(m, k) on the
    preconditioned operator, reusing/refreshing `state` (modified in place)."""
    L = left or identity
    R = right or identity
    Dc = Counted(D)
    A = lambda v: L(Dc(R(v)))
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    bn = np.linalg.norm(b)
    info = SolveInfo()
    if bn == 0.0:
        info.converged, info.relres = True, 0.0
        return np.zeros_like(b), info

    def true_rel(x):
        return np.linalg.norm(b - Dc(x)) / bn

    rel = true_rel(x)
    info.history.append(rel)
    info.relres = rel
    if rel <= tol:
        info.converged = True
        info.matvecs = Dc.count
        return x, info
    rhat = L(b - Dc(x))
    ratio = np.linalg.norm(rhat) / (rel * bn)   # preconditioned / true residual

    if state.U is not None and k > 0:
        if matrix_changed:
            AU = np.stack([A(state.U[:, i]) for i in range(state.U.shape[1])], 1)
            Q, Rr = np.linalg.qr(AU)
            state.C = Q
            state.U = state.U @ np.linalg.inv(Rr)
        c = state.C.conj().T @ rhat
        x = x + R(state.U @ c)
        rhat = rhat - state.C @ c
    elif k > 0:
        beta = np.linalg.norm(rhat)
        ar = arnoldi(A, rhat, m, ortho, rhs_norm=beta,
                     est_target=tol * bn * ratio, min_steps=k)
        j = ar.steps
        e1 = np.zeros(j + 1, dtype=np.complex128)
        e1[0] = beta
        y = np.linalg.lstsq(ar.Hbar, e1, rcond=None)[0]
        x = x + R(_combine(ar.V[:j], y[:, None])[:, 0])
        rhat = _combine(ar.V[:j + 1], (e1 - ar.Hbar @ y)[:, None])[:, 0]
        info.cycles += 1
        info.iters += j
        if j >= k:
            theta, Z = harmonic_ritz_pairs(ar.Hbar)
            P = _smallest(theta, Z, k)
            Q, Rr = np.linalg.qr(ar.Hbar @ P)
            state.C = _combine(ar.V[:j + 1], Q)
            state.U = _combine(ar.V[:j], P) @ np.linalg.inv(Rr)
            state.updates = 1

    while True:
        rel = true_rel(x)
        info.history.append(rel)
        info.relres = rel
        if rel <= tol:
            info.converged = True
            break
        if info.cycles >= max_cycles:
            break
        beta = np.linalg.norm(rhat)
        if state.U is None or k == 0:
            # plain GMRES(m) cycle (k = 0 reduces GCRO-DR to GMRES(m))
            ar = arnoldi(A, rhat, m, ortho, rhs_norm=beta,
                         est_target=tol * bn * ratio)
            j = ar.steps
            e1 = np.zeros(j + 1, dtype=np.complex128)
            e1[0] = beta
            y = np.linalg.lstsq(ar.Hbar, e1, rcond=None)[0]
            x = x + R(_combine(ar.V[:j], y[:, None])[:, 0])
            rhat = _combine(ar.V[:j + 1], (e1 - ar.Hbar @ y)[:, None])[:, 0]
            info.cycles += 1
            info.iters += j
            continue
        kk = state.U.shape[1]
        Clist = [state.C[:, i] for i in range(kk)]
        ar = arnoldi(A, rhat, m - kk, ortho, C=Clist, rhs_norm=beta,
                     est_target=tol * bn * ratio)
        j = ar.steps
        dk = 1.0 / np.linalg.norm(state.U, axis=0)
        Uh = state.U * dk[None, :]
        Vhat = np.concatenate([Uh, np.stack(ar.V[:j], 1)], axis=1)
        What = np.concatenate([state.C, np.stack(ar.V[:j + 1], 1)], axis=1)
        G = np.zeros((kk + j + 1, kk + j), dtype=np.complex128)
        G[:kk, :kk] = np.diag(dk)
        G[:kk, kk:] = ar.Bk
        G[kk:, kk:] = ar.Hbar
        rhs = np.zeros(kk + j + 1, dtype=np.complex128)
        rhs[kk] = beta
        y = np.linalg.lstsq(G, rhs, rcond=None)[0]
        x = x + R(Vhat @ y)
        rhat = rhat - What @ (G @ y)
        info.cycles += 1
        info.iters += j
        if state.updates < u:
            WV = What.conj().T @ Vhat
            theta, Z = sla.eig(G.conj().T @ G, G.conj().T @ WV)
            P = _smallest(theta, Z, kk)
            Q, Rr = np.linalg.qr(G @ P)
            state.C = What @ Q
            state.U = Vhat @ P @ np.linalg.inv(Rr)
            state.updates += 1
    info.matvecs = Dc.count
    info.final_rhat = rhat
    return x, info
