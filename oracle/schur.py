"""Odd-even reduction of the coarse operator (oracle; test infrastructure only).

Sec. 2.2: the coarsest-level system is solved in its odd-even reduced form.
With the sites split by parity (x0 + x1 + x2 + x3 even or odd) and the
nearest-neighbour stencil coupling only sites of opposite parity, D has the
block form [[D_ee, D_eo], [D_oe, D_oo]] with block-diagonal D_ee = A_e and
D_oo = A_o (the self blocks, twisted mass included).  Eliminating the odd
sites gives the Schur complement

    S = D_ee - D_eo D_oo^{-1} D_oe

on the even sites: D x = b is solved as S x_e = b_e - D_eo D_oo^{-1} b_o,
then x_o = D_oo^{-1} (b_o - D_oe x_e).

Sec. 3.2 takes the block-Jacobi preconditioner of the reduced system to be
B = D_ee, the even sites' self blocks (not the block diagonal of S itself, which
the paper notes and accepts), applied from the left, and Sec. 3.3 builds the
polynomial from B^{-1} S: the system solved is B^{-1} S q(B^{-1} S) y = B^{-1} b_e
with x_e = q(B^{-1} S) y (the form written out in the paper for both
preconditioners together).

Vectors of one parity are stored compressed: the even (odd) sites in
increasing site order, which for an even extent L0 puts site x at position
x // 2.  Every extent must be even for the checkerboard to be consistent with
the periodic boundaries.
"""
from __future__ import annotations

import numpy as np

from . import operator as dop
from .krylov import gmres
from .lattice import coords


def parity(dims) -> np.ndarray:
    """0 for even sites, 1 for odd sites, in site order."""
    if any(int(d) % 2 for d in dims):
        raise ValueError("odd-even reduction needs every lattice extent even")
    return (coords(dims).sum(axis=1) % 2).astype(np.int64)


def sites(dims, p: int) -> np.ndarray:
    """Sites of parity p in increasing order (the compressed order)."""
    return np.where(parity(dims) == p)[0]


def split(op: dop.CoarseOp, v: np.ndarray):
    """(v_e, v_o) of a full-lattice vector [V, n]."""
    return v[sites(op.dims, 0)], v[sites(op.dims, 1)]


def merge(op: dop.CoarseOp, v_e: np.ndarray, v_o: np.ndarray) -> np.ndarray:
    v = np.zeros((op.V, op.n), dtype=np.complex128)
    v[sites(op.dims, 0)] = v_e
    v[sites(op.dims, 1)] = v_o
    return v


def _embed(op, v, p):
    v_full = np.zeros((op.V, op.n), dtype=np.complex128)
    v_full[sites(op.dims, p)] = v
    return v_full


def d_oe(op, x_e):
    """D_oe x_e: the odd rows of D applied to x_e on the even sites."""
    return dop.apply(op, _embed(op, x_e, 0))[sites(op.dims, 1)]


def d_eo(op, x_o):
    """D_eo x_o: the even rows of D applied to x_o on the odd sites."""
    return dop.apply(op, _embed(op, x_o, 1))[sites(op.dims, 0)]


def dinv_oo(op, v_o):
    """D_oo^{-1} v_o with D_oo the odd sites' self blocks."""
    Ao = op.A[sites(op.dims, 1)]
    return np.stack([np.linalg.solve(Ao[i], v_o[i]) for i in range(Ao.shape[0])])


def apply(op, x_e):
    """S x_e = A_e x_e - D_eo D_oo^{-1} D_oe x_e."""
    Ae = op.A[sites(op.dims, 0)]
    return np.einsum("sij,sj->si", Ae, x_e) - d_eo(op, dinv_oo(op, d_oe(op, x_e)))


def dinv_ee(op, v_e):
    """B^{-1} v_e with B = D_ee, the even sites' self blocks (Sec. 3.2)."""
    Ae = op.A[sites(op.dims, 0)]
    return np.stack([np.linalg.solve(Ae[i], v_e[i]) for i in range(Ae.shape[0])])


def apply_bj(op, x_e):
    """B^{-1} S x_e: the reduced operator with the block-Jacobi preconditioner
    B = D_ee applied from the left (Sec. 3.2)."""
    return dinv_ee(op, apply(op, x_e))


def rhs(op, b):
    """Reduced right-hand side b_e - D_eo D_oo^{-1} b_o."""
    b_e, b_o = split(op, b)
    return b_e - d_eo(op, dinv_oo(op, b_o))


def recover(op, b, x_e):
    """Full solution from x_e: x_o = D_oo^{-1} (b_o - D_oe x_e)."""
    _, b_o = split(op, b)
    return merge(op, x_e, dinv_oo(op, b_o - d_oe(op, x_e)))


def solve(op, b, tol: float, m: int = 30, max_cycles: int = 10000):
    """D x = b through the reduced system, GMRES(m) on S to the relative
    tolerance that makes ||b - D x|| <= tol ||b|| (the odd rows of the
    residual vanish exactly, the even rows are the reduced residual)."""
    bh = rhs(op, b).reshape(-1)
    n_e = bh.shape[0] // op.n
    f = lambda v: apply(op, v.reshape(n_e, op.n)).reshape(-1)
    tol_s = tol * np.linalg.norm(b) / max(np.linalg.norm(bh), 1e-300)
    xe, info = gmres(f, bh, tol_s, m, max_cycles)
    return recover(op, b, xe.reshape(n_e, op.n)), info


def solve_method(op, b, tol: float, m: int, k: int, d: int, u: int, state,
                 v0=None, bj: bool = True, max_cycles: int = 10000, seed: int = 0,
                 ortho: str = "mgs"):
    """D x = b through the reduced system with the paper's solver (Sec. 3.6):
    left block Jacobi B = D_ee (bj), the GMRES polynomial q of degree d - 1
    built from B^{-1} S (Sec. 3.3, random start v0), and GCRO-DR(m, k) with
    recycling through `state` (Sec. 3.4).  The reduced system is solved to
    the relative tolerance that makes ||b - D x|| <= tol ||b||.
    Returns (x, info, theta)."""
    from . import gcrodr as gc
    from . import poly

    bh = rhs(op, b).reshape(-1)
    n_e = bh.shape[0] // op.n
    shape = (n_e, op.n)
    S = lambda v: apply(op, v.reshape(shape)).reshape(-1)
    Binv = (lambda v: dinv_ee(op, v.reshape(shape)).reshape(-1)) if bj else None
    At = (lambda v: Binv(S(v))) if bj else S
    theta = None
    right = None
    if d > 1:
        if v0 is None:
            rng = np.random.default_rng(seed)
            v0 = rng.standard_normal(bh.shape[0]) + 1j * rng.standard_normal(bh.shape[0])
        theta, _ = poly.build_polynomial(At, np.asarray(v0).reshape(-1), d, ortho)
        right = lambda v: poly.q_apply(At, theta, v)
    tol_s = tol * np.linalg.norm(b) / max(np.linalg.norm(bh), 1e-300)
    xe, info = gc.gcrodr(S, bh, tol_s, m, k, u, max_cycles, state, left=Binv, right=right,
                         ortho=ortho)
    return recover(op, b, xe.reshape(shape)), info, theta


def dense(op) -> np.ndarray:
    """S assembled by block elimination of the dense D (tiny lattices only):
    an independent construction for checking `apply`."""
    D = dop.dense(op)
    n = op.n
    ev = np.concatenate([np.arange(x * n, (x + 1) * n) for x in sites(op.dims, 0)])
    od = np.concatenate([np.arange(x * n, (x + 1) * n) for x in sites(op.dims, 1)])
    return D[np.ix_(ev, ev)] - D[np.ix_(ev, od)] @ np.linalg.solve(D[np.ix_(od, od)],
                                                                   D[np.ix_(od, ev)])
