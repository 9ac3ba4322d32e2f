"""GMRES-polynomial preconditioning (oracle; test infrastructure only).

Sec. 3.3: after d Arnoldi steps of A from a random start vector, the harmonic
Ritz values theta_1..theta_d are the eigenvalues of H_d + h_{d+1,d}^2 f e_d^T
with f = H_d^{-H} e_d.  The GMRES residual polynomial is
p_d(t) = prod_i (1 - t/theta_i), and q_{d-1}, with p_d(t) = 1 - t q_{d-1}(t),
has the Newton-like form  q(t) = sum_i (1/theta_i) prod_{j<i} (1 - t/theta_j)
(empty product = 1), which costs d-1 products with A.  The values are taken in
Leja order (Alg. 2).  Alg. 3 then runs GMRES(m) right-preconditioned by q(A).
With the block-Jacobi preconditioner (Sec. 3.2) the polynomial is built for
B^{-1} D_c and the system is (B^{-1}D_c) q(B^{-1}D_c) y = B^{-1} b,
x = q(B^{-1}D_c) y.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .krylov import arnoldi, gmres


def harmonic_ritz(Hbar: np.ndarray) -> np.ndarray:
    """Harmonic Ritz values from the (d+1) x d Hessenberg matrix of d Arnoldi
    steps: eig(H_d + |h_{d+1,d}|^2 f e_d^T), f = H_d^{-H} e_d."""
    d = Hbar.shape[1]
    Hd = Hbar[:d, :d]
    h = Hbar[d, d - 1]
    ed = np.zeros(d, dtype=np.complex128)
    ed[-1] = 1.0
    f = np.linalg.solve(Hd.conj().T, ed)
    return sla.eigvals(Hd + (abs(h) ** 2) * np.outer(f, ed))


def harmonic_ritz_pairs(Hbar: np.ndarray):
    """Harmonic Ritz values and the eigenvectors z of the same matrix."""
    d = Hbar.shape[1]
    Hd = Hbar[:d, :d]
    h = Hbar[d, d - 1]
    ed = np.zeros(d, dtype=np.complex128)
    ed[-1] = 1.0
    f = np.linalg.solve(Hd.conj().T, ed)
    return sla.eig(Hd + (abs(h) ** 2) * np.outer(f, ed))


def leja_order(theta) -> np.ndarray:
    """Leja ordering (Alg. 2): the first value has the largest modulus; each next
    value maximises the product of distances to those already taken.

    Products are compared as sums of logarithms (no overflow at large d).
    Scores within a relative 1e-10 of the best count as ties, resolved by
    larger imaginary part, then larger real part, then lower index.
    Repeated values are kept (their score is -inf once one copy is taken).
    """
    theta = np.asarray(theta, dtype=np.complex128)
    d = theta.size
    remaining = list(range(d))
    order = []

    def pick(scores):
        best = max(scores[i] for i in remaining)
        if np.isfinite(best):
            tol = 1e-10 * max(1.0, abs(best))
            cand = [i for i in remaining if scores[i] >= best - tol]
        else:
            cand = [i for i in remaining if scores[i] == best]
        cand.sort(key=lambda i: (-theta[i].imag, -theta[i].real, i))
        return cand[0]

    scores = np.log(np.abs(theta) + 0.0)
    with np.errstate(divide="ignore"):
        while remaining:
            i = pick(scores)
            order.append(i)
            remaining.remove(i)
            dist = np.abs(theta - theta[i])
            scores = (scores if len(order) > 1 else np.zeros(d)) + np.log(dist)
    return theta[np.array(order, dtype=np.int64)]


def q_apply(A, theta, v):
    """q(A) v in the Newton-like form: d-1 products with A.
    prod <- v;  y <- prod/theta_1;
    for i = 2..d: prod <- prod - A(prod)/theta_{i-1};  y <- y + prod/theta_i."""
    prod = np.array(v, dtype=np.complex128, copy=True)
    y = prod / theta[0]
    for i in range(1, len(theta)):
        prod = prod - A(prod) / theta[i - 1]
        y = y + prod / theta[i]
    return y


def p_apply(A, theta, v):
    """p_d(A) v = prod_i (I - A/theta_i) v (the GMRES residual polynomial)."""
    out = np.array(v, dtype=np.complex128, copy=True)
    for t in theta:
        out = out - A(out) / t
    return out


def build_polynomial(A, v0, d: int, ortho: str = "mgs"):
    """Alg. 3, first three steps: d Arnoldi steps from v0, harmonic Ritz values,
    Leja order.  If Arnoldi breaks down after j < d steps, the Krylov space is
    invariant and the j eigenvalues of H_j (exact eigenvalues of A) are used."""
    ar = arnoldi(A, v0, d, ortho)
    if ar.breakdown:
        j = ar.steps
        theta = sla.eigvals(ar.Hbar[:j, :j])
    else:
        theta = harmonic_ritz(ar.Hbar)
    return leja_order(theta), ar


def pp_gmres(D, b, tol, m, max_cycles, theta, Binv_apply=None, x0=None,
             ortho="mgs"):
    """Alg. 3 with the block-Jacobi left preconditioner of Sec. 3.2 when
    Binv_apply is given: GMRES(m) on (B^{-1}D) q(B^{-1}D), x = q(B^{-1}D) y."""
    if Binv_apply is None:
        At = D
        left = None
    else:
        At = lambda v: Binv_apply(D(v))
        left = Binv_apply
    right = lambda v: q_apply(At, theta, v)
    return gmres(D, b, tol, m, max_cycles, x0=x0, left=left, right=right,
                 ortho=ortho)
