"""Adjoint solves and gradients of x = D_c^{-1} b (oracle; test infrastructure
only).

The adjoint system D^H lambda = g is solved with GMRES on the adjoint apply
written from its definition (operator.apply_adjoint).  For a real loss L of x,
with g = dL/dx in the convention grad = dL/dRe + i dL/dIm:
    grad_b = lambda,
    grad of an entry D[p, q] = -lambda_p conj(x_q),
so the gradient of the hop block coupling x to x+mu is -lambda_x x_{x+mu}^H
("untied": each of the 8 directed couplings taken as independent).  With the
backward coupling tied to the forward block, D[x+mu, x] = Gamma5 B[x,mu]^H
Gamma5, the forward block's gradient also receives -Gamma5 x_x lambda_{x+mu}^H
Gamma5.
"""
from __future__ import annotations

import numpy as np

from .krylov import gmres
from .operator import CoarseOp, apply, apply_adjoint, gamma5


def solve(op: CoarseOp, b, tol=1e-12, m=60, max_cycles=10000):
    shape = b.shape
    x, info = gmres(lambda v: apply(op, v.reshape(shape)).reshape(-1),
                    b.reshape(-1), tol, m, max_cycles)
    return x.reshape(shape), info


def solve_adjoint(op: CoarseOp, g, tol=1e-12, m=60, max_cycles=10000):
    shape = g.shape
    lam, info = gmres(lambda v: apply_adjoint(op, v.reshape(shape)).reshape(-1),
                      g.reshape(-1), tol, m, max_cycles)
    return lam.reshape(shape), info


def grad_hops_untied(op: CoarseOp, lam, x) -> np.ndarray:
    """[V, 8, n, n]: direction mu < 4 is the coupling x -> x+mu
    (-lambda_x x_{x+mu}^H); direction 4+mu the coupling x -> x-mu
    (-lambda_x x_{x-mu}^H)."""
    V, n = lam.shape
    G = np.empty((V, 8, n, n), dtype=np.complex128)
    for mu in range(4):
        G[:, mu] = -lam[:, :, None] * np.conj(x[op.fwd[mu]])[:, None, :]
        G[:, 4 + mu] = -lam[:, :, None] * np.conj(x[op.bwd[mu]])[:, None, :]
    return G


def grad_hops_tied(op: CoarseOp, lam, x) -> np.ndarray:
    """[V, 4, n, n]: gradient w.r.t. the forward block B[x, mu] when the backward
    coupling is Gamma5 B[x,mu]^H Gamma5:
    -lambda_x x_{x+mu}^H - Gamma5 x_x lambda_{x+mu}^H Gamma5."""
    V, n = lam.shape
    g5 = gamma5(n)
    G = np.empty((V, 4, n, n), dtype=np.complex128)
    for mu in range(4):
        y = op.fwd[mu]
        G[:, mu] = (-lam[:, :, None] * np.conj(x[y])[:, None, :]
                    - (g5 * x)[:, :, None] * np.conj(g5 * lam[y])[:, None, :])
    return G


def loss_grads(op: CoarseOp, b, c, tol=1e-12):
    """L = Re(c^H x), x = D^{-1} b.  Returns (L, x, lambda, grad_b, grad_B tied)."""
    x, _ = solve(op, b, tol)
    lam, _ = solve_adjoint(op, c, tol)
    L = float(np.real(np.vdot(c.reshape(-1), x.reshape(-1))))
    return L, x, lam, lam.copy(), grad_hops_tied(op, lam, x)
