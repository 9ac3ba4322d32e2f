"""Seeded synthetic inputs for the coarse-operator solver: operator blocks and
right-hand sides.  Shared by the oracle and by the GPU path; holds none of the
solver's arithmetic.

Operator recipe (a random stand-in for the coarsest-level matrix of an
aggregation multigrid for clover-Wilson / twisted-mass fermions, whose gauge
configurations are not available):

* lattice: periodic L0 x L1 x L2 x L3, site = x0 + L0*(x1 + L1*(x2 + L2*x3));
* n = 2*n_tv variables per site, Gamma5 = diag(+1 (n_tv times), -1 (n_tv times));
* forward hop blocks B[x, mu] = Z / sqrt(n), Z standard complex Gaussian
  (E|z|^2 = 1); the backward coupling is Gamma5 B^H Gamma5 (derived, not drawn);
* self blocks A[x] = m0*I + Gamma5 H[x], H = (G + G^H)/2, G = Z'/sqrt(n);
  the twisted-mass term i*mu*Gamma5 is NOT included here: the operator build
  adds it;
* right-hand sides: standard complex Gaussian per entry.

Every entry comes from the counter-based Philox4x32-10 stream
(counter = (flat index, stream id, sub-stream), key = seed), so any site can be
regenerated alone.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field

import torch

from .philox import complex_normal, philox4x32_10  # noqa: F401

STREAM_HOPS = 0
STREAM_H = 1
STREAM_RHS = 2
STREAM_AUX = 3      # second vectors (loss weights, lambda/x for kernel tests)
STREAM_V0 = 4       # random start vector of the polynomial construction

_HERE = os.path.dirname(os.path.abspath(__file__))
M0_TABLE = os.path.join(_HERE, "m0.json")


def volume(dims) -> int:
    v = 1
    for d in dims:
        v *= int(d)
    return v


@dataclass
class Workload:
    """One synthetic coarse-operator configuration."""
    name: str
    dims: tuple
    n_tv: int
    rho: float            # target min Re(eig) / max |eig| of the mu = 0 operator
    mu: float = 0.0       # twisted mass added by the operator build
    seed: int = 0
    notes: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return 2 * self.n_tv

    @property
    def V(self) -> int:
        return volume(self.dims)

    @property
    def N(self) -> int:
        return self.V * self.n

    def m0(self) -> float:
        tab = load_m0_table()
        if self.name not in tab:
            raise KeyError(f"no calibrated m0 for workload {self.name}; "
                           f"run oracle/calibrate_m0.py")
        return float(tab[self.name]["m0"])


WORKLOADS = {
    # 4^4, N_tv = 8: small clover-Wilson case, min Re / max|eig| = 1e-2
    "c1": Workload("c1", (4, 4, 4, 4), 8, 1e-2),
    # 8^4, N_tv = 24: small-mass clover-Wilson case, ratio 1e-4
    "c2": Workload("c2", (8, 8, 8, 8), 24, 1e-4),
    # 16^3 x 32, N_tv = 24, twisted mass mu = 1e-3 (no coarse mu boost)
    "c3": Workload("c3", (16, 16, 16, 32), 24, 1e-4, mu=1e-3),
    # 16^4, N_tv = 24, clover-Wilson, ratio 1e-3 (batched right-hand sides)
    "c4": Workload("c4", (16, 16, 16, 16), 24, 1e-3),
    # 8^4, N_tv = 16, twisted mass mu = 1e-2 (differentiation)
    "c5": Workload("c5", (8, 8, 8, 8), 16, 1e-2, mu=1e-2),
    # small mixed-batch members (4^4 / 8^4 / 12^4, N_tv = 24)
    "mb4": Workload("mb4", (4, 4, 4, 4), 24, 1e-3),
    "mb8": Workload("mb8", (8, 8, 8, 8), 24, 1e-3),
    "mb12": Workload("mb12", (12, 12, 12, 12), 24, 1e-3),
}


def load_m0_table() -> dict:
    if not os.path.exists(M0_TABLE):
        return {}
    with open(M0_TABLE) as f:
        return json.load(f)


def _gamma5(n: int, device, dtype=torch.float64):
    g = torch.ones(n, dtype=dtype, device=device)
    g[n // 2:] = -1.0
    return g


def hop_blocks(dims, n_tv: int, seed: int = 0, sites=None, device="cpu"):
    """Forward hop blocks B[x, mu] as complex128 [len(sites)][4][n][n]."""
    n = 2 * n_tv
    V = volume(dims)
    if sites is None:
        sites = torch.arange(V, device=device, dtype=torch.int64)
    sites = torch.as_tensor(sites, dtype=torch.int64, device=device)
    out = torch.empty((sites.numel(), 4, n, n), dtype=torch.complex128, device=device)
    per_site = 4 * n * n
    local = torch.arange(per_site, device=device, dtype=torch.int64)
    chunk = max(1, (1 << 24) // per_site)
    for s in range(0, sites.numel(), chunk):
        sl = sites[s:s + chunk]
        idx = (sl[:, None] * per_site + local[None, :]).reshape(-1)
        z = complex_normal(idx, STREAM_HOPS, seed)
        out[s:s + chunk] = (z / (n ** 0.5)).reshape(-1, 4, n, n)
    return out


def self_blocks(dims, n_tv: int, m0: float, seed: int = 0, sites=None, device="cpu"):
    """Self blocks A[x] = m0 I + Gamma5 H[x] as complex128 [len(sites)][n][n]."""
    n = 2 * n_tv
    V = volume(dims)
    if sites is None:
        sites = torch.arange(V, device=device, dtype=torch.int64)
    sites = torch.as_tensor(sites, dtype=torch.int64, device=device)
    out = torch.empty((sites.numel(), n, n), dtype=torch.complex128, device=device)
    per_site = n * n
    local = torch.arange(per_site, device=device, dtype=torch.int64)
    g5 = _gamma5(n, device).to(torch.complex128)
    eye = torch.eye(n, dtype=torch.complex128, device=device)
    chunk = max(1, (1 << 24) // per_site)
    for s in range(0, sites.numel(), chunk):
        sl = sites[s:s + chunk]
        idx = (sl[:, None] * per_site + local[None, :]).reshape(-1)
        G = (complex_normal(idx, STREAM_H, seed) / (n ** 0.5)).reshape(-1, n, n)
        H = 0.5 * (G + G.conj().transpose(1, 2))
        out[s:s + chunk] = m0 * eye + g5[None, :, None] * H
    return out


def vector(dims, n_tv: int, stream: int, seed: int = 0, sub: int = 0,
           device="cpu"):
    """A standard complex Gaussian field [V][n] (complex128)."""
    n = 2 * n_tv
    V = volume(dims)
    idx = torch.arange(V * n, device=device, dtype=torch.int64)
    return complex_normal(idx, stream, seed, sub).reshape(V, n)


def rhs(dims, n_tv: int, r: int = 0, seed: int = 0, device="cpu"):
    """Right-hand side number r (sub-stream r of the RHS stream)."""
    return vector(dims, n_tv, STREAM_RHS, seed, r, device)


def operator(w: Workload, device="cpu", m0=None):
    """(self_blocks, hop_blocks) of workload w, complex128."""
    if m0 is None:
        m0 = w.m0()
    A = self_blocks(w.dims, w.n_tv, m0, w.seed, device=device)
    B = hop_blocks(w.dims, w.n_tv, w.seed, device=device)
    return A, B


def tolerances_loguniform(count: int, lo: float = 1e-10, hi: float = 1e-6,
                          seed: int = 0):
    """Per-RHS tolerances 10^U(log10 lo, log10 hi), seeded (Philox stream 5)."""
    import math
    idx = torch.arange(count, dtype=torch.int64)
    c = philox4x32_10(idx, torch.zeros_like(idx), torch.full_like(idx, 5),
                      torch.zeros_like(idx), seed, 0)
    u = (c[0].to(torch.float64) + 0.5) / 2.0 ** 32
    return [10.0 ** (math.log10(lo) + float(x) * (math.log10(hi) - math.log10(lo)))
            for x in u]
