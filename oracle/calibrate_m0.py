"""Calibrate the mass shift m0 of each synthetic workload (oracle script; test
infrastructure only).  Writes synth/m0.json.

Target: for the mu = 0 operator D(m0) = D_0 + m0 I (D_0 = the stencil with
A = Gamma5 H), m0 solves  min Re eig(D(m0)) = rho * max |eig(D(m0))|.

Two readings, by size:

* exact (lattices with at most `dense_limit` unknowns): every eigenvalue of
  D_0 from a dense eigendecomposition;
  f(m0) = m0 + min Re eig(D_0) - rho * max |m0 + eig(D_0)| has slope >= 1 - rho
  > 0, so the root is unique and bisection finds it;
* limiting disk (larger lattices): the spectrum of this random family fills a
  disk about the origin whose radius r follows from the entry variances: each
  row of D_0 carries variance 1/2 in the self block (H = (G + G^H)/2 with
  E|G_ij|^2 = 1/n gives E|H_ij|^2 = 1/(2n) on all n entries of a row) and 1 in
  each of the 8 hop couplings (E|B_ij|^2 = 1/n), so r^2 = 1/2 + 8.  For the
  disk of radius r centred at m0, min Re = m0 - r and max |.| = m0 + r, hence
  m0 = r (1 + rho) / (1 - rho).  The leftmost eigenvalue of a finite lattice
  sits in a dense edge (eigenvalue spacing there ~1e-3 at 2e5 unknowns) that
  restarted Krylov eigensolvers do not resolve to the 1e-4 level in hours, so
  the ratio is imposed on the limiting spectrum; the few finite-size
  eigenvalues just outside the disk then lie at or across the origin's side
  of m0 - r, which is the near-null-mode situation the deflation targets.

How close the limiting-disk reading comes on a given lattice is estimated
(not calibrated) from the Ritz values of a k-step Arnoldi process (modified
Gram-Schmidt, seeded Gaussian start) on D(m0): the leftmost Ritz value and
the largest Ritz modulus give rho_ritz = min Re / max |.|, recorded with the
residual norm |h_{k+1,k} e_k^T y| of the leftmost Ritz pair (how far it is
from an eigenpair).

Usage: python -m oracle.calibrate_m0 c1 c2 ...
       python -m oracle.calibrate_m0 --ritz STEPS c2 ...   (adds the estimate)
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np
import scipy.linalg as sla

from . import operator as dop


# per-row variance of D_0: self block 1/2, eight hop couplings 1 each
ROW_VARIANCE = 0.5 + 8.0


def limiting_radius() -> float:
    """Radius of the disk that the spectrum of D_0 fills for large lattices."""
    return float(np.sqrt(ROW_VARIANCE))


def m0_disk(rho: float) -> float:
    """m0 with (m0 - r) = rho (m0 + r) for the limiting disk of radius r."""
    r = limiting_radius()
    return r * (1.0 + rho) / (1.0 - rho)


def m0_root(eigs: np.ndarray, rho: float) -> float:
    lo = -float(eigs.real.min())
    f = lambda m0: m0 + eigs.real.min() - rho * np.abs(m0 + eigs).max()
    hi = lo + 1.0
    while f(hi) < 0:
        hi = lo + 2 * (hi - lo)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) < 0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def calibrate(name: str, dense_limit: int = 8192):
    import torch  # noqa: F401  (synth uses torch)
    import synth
    w = synth.WORKLOADS[name]
    N = synth.volume(w.dims) * 2 * w.n_tv
    t0 = time.time()
    if N > dense_limit:
        m0 = m0_disk(w.rho)
        return {"m0": m0, "rho_target": w.rho, "method": "limiting disk",
                "radius": limiting_radius(), "seconds": time.time() - t0}
    A0 = synth.self_blocks(w.dims, w.n_tv, 0.0, w.seed).numpy()
    B = synth.hop_blocks(w.dims, w.n_tv, w.seed).numpy()
    op = dop.build(w.dims, A0, B, 0.0)
    ev = sla.eigvals(dop.dense(op))
    m0 = m0_root(ev, w.rho)
    shifted = ev + m0
    return {"m0": m0, "rho_target": w.rho, "method": "dense eig",
            "rho_achieved": float(shifted.real.min() / np.abs(shifted).max()),
            "min_re_D0": float(ev.real.min()), "max_re_D0": float(ev.real.max()),
            "seconds": time.time() - t0}


def ritz_estimate(name: str, steps: int, seed: int = 7):
    """Leftmost Ritz value, largest Ritz modulus and their ratio for D(m0) of
    workload `name` (its calibrated m0) from `steps` Arnoldi steps."""
    import torch  # noqa: F401  (synth uses torch)
    import synth
    from .krylov import arnoldi
    w = synth.WORKLOADS[name]
    t0 = time.time()
    A, B = synth.operator(w)
    op = dop.build(w.dims, A.numpy(), B.numpy(), 0.0)
    f = lambda v: dop.apply(op, v.reshape(op.V, op.n)).reshape(-1)
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(op.V * op.n) + 1j * rng.standard_normal(op.V * op.n)
    ar = arnoldi(f, v, steps, "mgs")
    j = ar.steps
    theta, Y = sla.eig(ar.Hbar[:j, :j])
    i = int(np.argmin(theta.real))
    res = abs(ar.Hbar[j, j - 1]) * abs(Y[j - 1, i]) / np.linalg.norm(Y[:, i])
    return {"rho_ritz": float(theta.real.min() / np.abs(theta).max()),
            "ritz_min_re": float(theta.real.min()), "ritz_max_abs": float(np.abs(theta).max()),
            "ritz_steps": int(j), "ritz_left_residual": float(res),
            "ritz_seconds": time.time() - t0}


def main(names):
    import synth
    path = synth.M0_TABLE
    tab = synth.load_m0_table()
    ritz = 0
    if names and names[0] == "--ritz":
        ritz = int(names[1])
        names = names[2:]
    for name in names:
        if ritz:
            tab[name].update(ritz_estimate(name, ritz))
        else:
            tab[name] = calibrate(name)
        print(name, tab[name], flush=True)
        with open(path + ".tmp", "w") as f:
            json.dump(tab, f, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)


if __name__ == "__main__":
    main(sys.argv[1:])
