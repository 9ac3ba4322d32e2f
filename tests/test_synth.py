"""Seeded input generator: Philox known answers, distribution, site regeneration."""
import os

import numpy as np
import pytest
import torch

import synth
from synth.philox import complex_normal, philox4x32_10

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(t, 16) for t in line.split()])
    return rows


@pytest.mark.parametrize("row", _kat_rows())
def test_philox_known_answers(row):
    t = lambda v: torch.tensor([v], dtype=torch.int64)
    out = philox4x32_10(t(row[0]), t(row[1]), t(row[2]), t(row[3]), row[4], row[5])
    assert [int(o) for o in out] == row[6:10]


def test_complex_normal_moments():
    z = complex_normal(torch.arange(400000), stream=7, seed=3).numpy()
    assert abs(z.mean()) < 5e-3
    assert abs(np.mean(np.abs(z) ** 2) - 1.0) < 1e-2
    assert abs(np.mean(z.real ** 2) - 0.5) < 1e-2
    assert abs(np.mean(z.real * z.imag)) < 5e-3
    assert abs(np.mean(z * z)) < 1e-2          # circular: E z^2 = 0


def test_site_regeneration_matches_full():
    dims, ntv = (3, 2, 2, 4), 4
    B = synth.hop_blocks(dims, ntv, seed=5)
    A = synth.self_blocks(dims, ntv, 1.5, seed=5)
    sites = torch.tensor([0, 7, 13, 47])
    assert torch.equal(synth.hop_blocks(dims, ntv, seed=5, sites=sites), B[sites])
    assert torch.equal(synth.self_blocks(dims, ntv, 1.5, seed=5, sites=sites), A[sites])


def test_self_block_structure():
    dims, ntv = (2, 2, 2, 2), 3
    n = 2 * ntv
    A = synth.self_blocks(dims, ntv, 0.7, seed=1).numpy()
    g5 = np.r_[np.ones(ntv), -np.ones(ntv)]
    H = g5[None, :, None] * (A - 0.7 * np.eye(n))
    assert np.allclose(H, np.conj(np.swapaxes(H, 1, 2)), atol=1e-15)


def test_tolerances_loguniform_range():
    t = np.array(synth.tolerances_loguniform(64, 1e-10, 1e-6, seed=0))
    assert t.min() >= 1e-10 and t.max() <= 1e-6
    assert np.log10(t).std() > 0.8      # spread over the decades, not clustered at 1e-6
