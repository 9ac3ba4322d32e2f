"""The coarse operator D_c as a 9-point block stencil (oracle; test infrastructure only).

Sec. 2.2 (coarsest-level structure): the coarsest-level matrix couples each
site to itself through a dense self-coupling block and to its 8 nearest
neighbours through hop blocks; with the spin-preserving aggregation each site
carries n = 2*n_tv variables and Gamma5 acts as +1 on the first n_tv and -1 on
the last n_tv of them.  Wilson-type operators are Gamma5-hermitian, so the hop
from x+mu back to x is Gamma5 B[x,mu]^H Gamma5 when B[x,mu] is the hop from x
to x+mu.  Sec. 2.1 (twisted mass): D_TM(mu) = D + i mu Gamma5.

Definition used throughout (rows are outputs):
    D[x, x]      = A[x] + i*mu*Gamma5
    D[x, x+mu]  += B[x, mu]
    D[x+mu, x]  += Gamma5 B[x, mu]^H Gamma5
so (D psi)_x = A'_x psi_x + sum_mu B[x,mu] psi_{x+mu}
                          + sum_mu Gamma5 B[x-mu,mu]^H Gamma5 psi_{x-mu}.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .lattice import neighbours


def gamma5(n: int) -> np.ndarray:
    """Diagonal of Gamma5 on one site: +1 for the first n/2, -1 for the rest."""
    g = np.ones(n)
    g[n // 2:] = -1.0
    return g


@dataclass
class CoarseOp:
    dims: tuple
    n: int
    A: np.ndarray        # [V, n, n] self blocks including i*mu*Gamma5
    B: np.ndarray        # [V, 4, n, n] forward hops
    mu: float
    fwd: np.ndarray      # [4, V]
    bwd: np.ndarray      # [4, V]
    A0: np.ndarray | None = None   # self blocks as given (without i*mu*Gamma5)

    @property
    def V(self):
        return self.A.shape[0]

    @property
    def N(self):
        return self.V * self.n


def build(dims, self_blocks, hop_blocks, mu: float = 0.0) -> CoarseOp:
    """Assemble the operator: copy the blocks and add i*mu*Gamma5 to A."""
    A0 = np.array(self_blocks, dtype=np.complex128, copy=True)
    B = np.array(hop_blocks, dtype=np.complex128, copy=True)
    A = A0.copy()
    V, n, _ = A.shape
    g5 = gamma5(n)
    idx = np.arange(n)
    A[:, idx, idx] += 1j * mu * g5
    fwd, bwd = neighbours(dims)
    return CoarseOp(tuple(int(d) for d in dims), n, A, B, float(mu), fwd, bwd, A0)


def with_mu(op: CoarseOp, mu_new: float) -> CoarseOp:
    """Same blocks, twisted mass replaced by mu_new."""
    A0 = op.A0 if op.A0 is not None else op.A
    A = A0.copy()
    idx = np.arange(op.n)
    A[:, idx, idx] += 1j * mu_new * gamma5(op.n)
    return CoarseOp(op.dims, op.n, A, op.B, float(mu_new), op.fwd, op.bwd, A0)


def apply(op: CoarseOp, psi: np.ndarray) -> np.ndarray:
    """(D psi) for psi of shape [V, n]: the 9-point stencil written out."""
    g5 = gamma5(op.n)
    out = np.einsum("sij,sj->si", op.A, psi)
    for mu in range(4):
        f = op.fwd[mu]
        b = op.bwd[mu]
        # forward: B[x, mu] psi_{x+mu}
        out += np.einsum("sij,sj->si", op.B[:, mu], psi[f])
        # backward: Gamma5 B[x-mu, mu]^H Gamma5 psi_{x-mu}
        Bh = np.conj(np.swapaxes(op.B[b, mu], 1, 2))
        out += g5 * np.einsum("sij,sj->si", Bh, g5 * psi[b])
    return out


def apply_site(A_x, B_x, B_back, psi_x, psi_fwd, psi_bwd, mu: float = 0.0) -> np.ndarray:
    """(D psi)_x at one site from the blocks it touches (for sampled checks of
    lattices too large to hold on the host): A_x [n, n] (without the twisted
    mass), B_x [4, n, n] = B[x, mu], B_back [4, n, n] = B[x - mu, mu],
    psi_x [n], psi_fwd [4, n] = psi_{x+mu}, psi_bwd [4, n] = psi_{x-mu}."""
    n = A_x.shape[0]
    g5 = gamma5(n)
    out = A_x @ psi_x + 1j * mu * g5 * psi_x
    for m in range(4):
        out = out + B_x[m] @ psi_fwd[m]
        out = out + g5 * (np.conj(B_back[m]).T @ (g5 * psi_bwd[m]))
    return out


def apply_adjoint(op: CoarseOp, psi: np.ndarray) -> np.ndarray:
    """(D^H psi), written from the definition D^H[y, x] = D[x, y]^H:
    (D^H psi)_x = A'_x^H psi_x + sum_mu Gamma5 B[x,mu] Gamma5 psi_{x+mu}
                               + sum_mu B[x-mu,mu]^H psi_{x-mu}."""
    g5 = gamma5(op.n)
    Ah = np.conj(np.swapaxes(op.A, 1, 2))
    out = np.einsum("sij,sj->si", Ah, psi)
    for mu in range(4):
        f = op.fwd[mu]
        b = op.bwd[mu]
        out += g5 * np.einsum("sij,sj->si", op.B[:, mu], g5 * psi[f])
        Bh = np.conj(np.swapaxes(op.B[b, mu], 1, 2))
        out += np.einsum("sij,sj->si", Bh, psi[b])
    return out


def dense(op: CoarseOp) -> np.ndarray:
    """The full N x N matrix (tiny lattices only)."""
    V, n = op.V, op.n
    D = np.zeros((V * n, V * n), dtype=np.complex128)
    g5 = gamma5(n)
    G = np.diag(g5)
    for x in range(V):
        D[x * n:(x + 1) * n, x * n:(x + 1) * n] += op.A[x]
        for mu in range(4):
            y = op.fwd[mu, x]
            D[x * n:(x + 1) * n, y * n:(y + 1) * n] += op.B[x, mu]
            D[y * n:(y + 1) * n, x * n:(x + 1) * n] += G @ op.B[x, mu].conj().T @ G
    return D


def bsr(op: CoarseOp) -> sp.bsr_matrix:
    """Block-sparse (BSR, block size n) assembly, for library cross-checks."""
    V, n = op.V, op.n
    G = np.diag(gamma5(n))
    rows, cols, blocks = [], [], []
    for x in range(V):
        rows.append(x)
        cols.append(x)
        blocks.append(op.A[x])
        for mu in range(4):
            y = op.fwd[mu, x]
            rows.append(x)
            cols.append(y)
            blocks.append(op.B[x, mu])
            rows.append(y)
            cols.append(x)
            blocks.append(G @ op.B[x, mu].conj().T @ G)
    # duplicates (extent-1/2 directions) are summed by the COO -> BSR conversion
    coo = sp.coo_matrix(
        (np.concatenate([b.reshape(-1) for b in blocks]),
         (np.concatenate([np.repeat(np.arange(n) + r * n, n) for r in rows]),
          np.concatenate([np.tile(np.arange(n) + c * n, n) for c in cols]))),
        shape=(V * n, V * n))
    return coo.tocsr().tobsr(blocksize=(n, n))


def block_jacobi_inverse(op: CoarseOp) -> np.ndarray:
    """B_x^{-1} for the block-diagonal preconditioner of Sec. 3.2: the inverse of
    each site's self-coupling block (here the full n x n self block)."""
    return np.linalg.inv(op.A)


def apply_block_jacobi(Binv: np.ndarray, psi: np.ndarray) -> np.ndarray:
    return np.einsum("sij,sj->si", Binv, psi)
