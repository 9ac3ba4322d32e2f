"""Periodic 4D lattice indexing (oracle; test infrastructure only).

The lattice is periodic in all four directions (Sec. 2.1: indices x +- mu-hat
are taken periodically).  Site numbering: x = x0 + L0*(x1 + L1*(x2 + L2*x3)).
"""
from __future__ import annotations

import numpy as np


def coords(dims):
    """[V, 4] integer coordinates of every site, in site order."""
    L0, L1, L2, L3 = (int(d) for d in dims)
    V = L0 * L1 * L2 * L3
    s = np.arange(V, dtype=np.int64)
    x0 = s % L0
    x1 = (s // L0) % L1
    x2 = (s // (L0 * L1)) % L2
    x3 = s // (L0 * L1 * L2)
    return np.stack([x0, x1, x2, x3], axis=1)


def site_index(dims, c):
    """Site number of coordinates c [..., 4] (taken modulo the extents)."""
    L = np.asarray(dims, dtype=np.int64)
    c = np.mod(np.asarray(c, dtype=np.int64), L)
    return c[..., 0] + L[0] * (c[..., 1] + L[1] * (c[..., 2] + L[2] * c[..., 3]))


def neighbours(dims):
    """(fwd, bwd): int64 [4, V] tables with fwd[mu, x] = x + mu-hat and
    bwd[mu, x] = x - mu-hat, periodic."""
    c = coords(dims)
    V = c.shape[0]
    fwd = np.empty((4, V), dtype=np.int64)
    bwd = np.empty((4, V), dtype=np.int64)
    for mu in range(4):
        step = np.zeros(4, dtype=np.int64)
        step[mu] = 1
        fwd[mu] = site_index(dims, c + step)
        bwd[mu] = site_index(dims, c - step)
    return fwd, bwd
