"""Calibrate the mass shift m0 of each synthetic workload (oracle script; test
infrastructure only).  Writes synth/m0.json.

Reading: for the mu = 0 operator D(m0) = D_0 + m0 I (D_0 = the stencil with
A = Gamma5 H), m0 solves  min Re eig(D(m0)) = rho * max |eig(D(m0))|.
f(m0) = m0 + min Re eig(D_0) - rho * max |m0 + eig(D_0)| has slope >= 1 - rho
> 0, so the root is unique and bisection finds it.  Small lattices use every
eigenvalue (dense eig); larger ones use ARPACK (scipy.sparse.linalg.eigs) for
the eigenvalues of smallest and largest real part, the only ones that decide
f for a spectrum symmetric about the real axis shifted to the right.

Usage: python -m oracle.calibrate_m0 c1 c2 ...
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from . import operator as dop


def _torch_matvec(op):
    """The same 9-point stencil as operator.apply, with the block products done
    by torch.bmm on the host's cores (calibration speed only)."""
    import torch
    g5 = torch.from_numpy(dop.gamma5(op.n)).to(torch.complex128)
    A = torch.from_numpy(op.A)
    B = [torch.from_numpy(np.ascontiguousarray(op.B[:, mu])) for mu in range(4)]
    Bh = [torch.from_numpy(np.ascontiguousarray(np.conj(np.swapaxes(op.B[op.bwd[mu], mu], 1, 2))))
          for mu in range(4)]
    fwd = [torch.from_numpy(op.fwd[mu]) for mu in range(4)]
    bwd = [torch.from_numpy(op.bwd[mu]) for mu in range(4)]

    def mv(v):
        psi = torch.from_numpy(np.ascontiguousarray(v.reshape(op.V, op.n)))
        out = torch.bmm(A, psi[:, :, None])[:, :, 0]
        for mu in range(4):
            out += torch.bmm(B[mu], psi[fwd[mu]][:, :, None])[:, :, 0]
            out += g5 * torch.bmm(Bh[mu], (g5 * psi[bwd[mu]])[:, :, None])[:, :, 0]
        return out.numpy().reshape(-1)
    return mv


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


def calibrate(name: str, dense_limit: int = 8192, arpack_tol: float = 1e-6, ncv: int = 300):
    import torch  # noqa: F401  (synth uses torch)
    import synth
    w = synth.WORKLOADS[name]
    A0 = synth.self_blocks(w.dims, w.n_tv, 0.0, w.seed).numpy()
    B = synth.hop_blocks(w.dims, w.n_tv, w.seed).numpy()
    op = dop.build(w.dims, A0, B, 0.0)
    t0 = time.time()
    if op.N <= dense_limit:
        ev = sla.eigvals(dop.dense(op))
        method = "dense eig"
    else:
        N = op.N
        lin = spla.LinearOperator((N, N), matvec=_torch_matvec(op), dtype=np.complex128)
        sr = spla.eigs(lin, k=2, which="SR", tol=arpack_tol, ncv=ncv,
                       maxiter=100000, return_eigenvectors=False)
        lr = spla.eigs(lin, k=2, which="LR", tol=arpack_tol, ncv=ncv,
                       maxiter=100000, return_eigenvectors=False)
        ev = np.concatenate([sr, lr])
        method = f"ARPACK SR/LR (k=2, ncv={ncv}, tol={arpack_tol:g})"
    m0 = m0_root(ev, w.rho)
    shifted = ev + m0
    return {"m0": m0, "rho_target": w.rho,
            "rho_achieved": float(shifted.real.min() / np.abs(shifted).max()),
            "min_re_D0": float(ev.real.min()), "max_re_D0": float(ev.real.max()),
            "method": method, "seconds": time.time() - t0}


def main(names):
    import synth
    path = synth.M0_TABLE
    tab = synth.load_m0_table()
    for name in names:
        tab[name] = calibrate(name)
        print(name, tab[name], flush=True)
        with open(path + ".tmp", "w") as f:
            json.dump(tab, f, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)


if __name__ == "__main__":
    main(sys.argv[1:])
