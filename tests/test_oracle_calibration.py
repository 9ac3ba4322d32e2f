"""Pins of the m0 calibration readings (oracle side, CPU).

The limiting-disk reading rests on two facts about the random operator family:
the mean row variance of D_0 (1/2 from the self block, 1 from each of the 8
hop couplings) and a spectrum that fills a disk of radius sqrt(that variance)
uniformly (circular law).  Both are checked on a small lattice by direct
computation, and the closed-form m0 is checked against the exact bisection
applied to a spectrum that is the limiting disk's boundary.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import operator as dop
from oracle.calibrate_m0 import ROW_VARIANCE, limiting_radius, m0_disk, m0_root


@pytest.fixture(scope="module")
def small_spectrum():
    dims, ntv = (3, 3, 3, 3), 8
    A0 = synth.self_blocks(dims, ntv, 0.0, 0).numpy()
    B = synth.hop_blocks(dims, ntv, 0).numpy()
    D = dop.dense(dop.build(dims, A0, B, 0.0))
    return D, sla.eigvals(D)


def test_row_variance_matches_frobenius_norm(small_spectrum):
    D, _ = small_spectrum
    fro = np.linalg.norm(D) ** 2 / D.shape[0]
    assert abs(fro / ROW_VARIANCE - 1.0) < 0.02


def test_spectrum_fills_the_disk_uniformly(small_spectrum):
    _, ev = small_spectrum
    r = limiting_radius()
    # uniform disk of radius r: E|lambda|^2 = r^2 / 2, P(|lambda| < r/2) = 1/4
    assert abs(np.mean(np.abs(ev) ** 2) / (r * r / 2) - 1.0) < 0.04
    assert abs(np.mean(np.abs(ev) < 0.5 * r) - 0.25) < 0.04
    # Gamma5-hermiticity: the spectrum is closed under conjugation
    assert np.max(np.min(np.abs(ev[:, None] - ev.conj()[None, :]), axis=1)) < 1e-8
    # edge: no eigenvalue far outside the disk
    assert np.abs(ev).max() < 1.1 * r


@pytest.mark.parametrize("rho", [1e-2, 1e-3, 1e-4])
def test_disk_formula_matches_bisection_on_the_disk(rho):
    r = limiting_radius()
    phi = np.linspace(0.0, 2 * np.pi, 4001)
    circle = r * np.exp(1j * phi)
    m_exact = m0_root(circle, rho)
    m = m0_disk(rho)
    assert abs(m - m_exact) < 1e-9
    assert abs((m - r) / (m + r) - rho) < 1e-14


def test_table_entries_follow_their_reading():
    tab = synth.load_m0_table()
    for name, e in tab.items():
        w = synth.WORKLOADS[name]
        assert e["rho_target"] == w.rho
        if e["method"] == "limiting disk":
            assert abs(e["m0"] - m0_disk(w.rho)) < 1e-12
        else:
            assert e["method"] == "dense eig"
            assert abs(e["rho_achieved"] - w.rho) < 1e-9
