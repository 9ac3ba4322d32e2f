"""C ABI checks that need no GPU: the library loads, exports every symbol the
headers declare, and its host-side dense linear algebra matches numpy/scipy."""
import os
import re

import numpy as np
import pytest
import scipy.linalg as sla

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for h in ("dcsolve.h", "dcsolve_dense.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\*?\s+\*?([a-z_0-9]+)\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2205_09104_amd import _lib
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    from paper_2205_09104_amd import _lib
    names = _declared_functions()
    assert len(names) >= 20
    for nm in names:
        assert hasattr(lib, nm), nm
        assert nm in _lib.SIGNATURES, nm


def test_default_opts_and_error_paths(lib):
    import ctypes as C
    from paper_2205_09104_amd import _lib
    o = _lib.SolveOpts()
    assert lib.dc_default_opts(C.byref(o)) == 0
    assert (o.m, o.k, o.d, o.u, o.prec, o.m_outer) == (30, 0, 0, 10, 0, 10)
    # invalid descriptor is rejected before any device work
    desc = _lib.OpDesc()
    h = C.c_void_p()
    assert lib.build_coarse_op(C.byref(desc), None, None, None, C.byref(h)) == _lib.DC_ERR_INVALID
    assert lib.dc_last_error().decode()
    assert lib.dc_apply(None, 0, 0, None, None, None) == _lib.DC_ERR_INVALID
    assert lib.solve_coarse(None, None, 1, None, None, None, 0, None, None) == _lib.DC_ERR_INVALID


def test_dense_eig_matches_scipy():
    from paper_2205_09104_amd import dense_eig
    rng = np.random.default_rng(0)
    for n in (1, 2, 5, 17, 40, 64):
        A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        ev, Z = dense_eig(A, vectors=True)
        ref = sla.eigvals(A)
        assert max(np.min(np.abs(ref - e)) for e in ev) <= 1e-10 * max(1, np.abs(ref).max())
        assert max(np.min(np.abs(ev - r)) for r in ref) <= 1e-10 * max(1, np.abs(ref).max())
        # eigenvectors: A z = lambda z, unit norm
        assert np.allclose(np.linalg.norm(Z, axis=0), 1.0)
        assert np.linalg.norm(A @ Z - Z * ev[None, :]) <= 1e-9 * np.linalg.norm(A) * n


def test_dense_eig_hessenberg_and_degenerate():
    from paper_2205_09104_amd import dense_eig
    # upper Hessenberg with a zero subdiagonal and repeated eigenvalues
    H = np.triu(np.ones((6, 6)), -1).astype(complex)
    H[3, 2] = 0.0
    ref = np.linalg.eigvals(H)
    ev = dense_eig(H)
    assert max(np.min(np.abs(ref - e)) for e in ev) <= 1e-6
    J = np.diag(np.full(5, 2.0 + 1j))          # multiple eigenvalue, diagonal
    assert np.allclose(dense_eig(J), 2 + 1j)


def test_dense_lstsq_matches_numpy():
    from paper_2205_09104_amd import dense_lstsq
    rng = np.random.default_rng(1)
    for (r, c) in ((5, 3), (31, 30), (63, 62), (10, 10)):
        A = rng.standard_normal((r, c)) + 1j * rng.standard_normal((r, c))
        b = rng.standard_normal(r) + 1j * rng.standard_normal(r)
        x, rn = dense_lstsq(A, b)
        ref = np.linalg.lstsq(A, b, rcond=None)[0]
        assert np.allclose(x, ref, atol=1e-10 * np.linalg.norm(ref))
        assert abs(rn - np.linalg.norm(b - A @ ref)) <= 1e-10 * np.linalg.norm(b)


def test_harmonic_ritz_and_leja_match_oracle():
    """Host library vs the oracle (numpy/scipy) on the same Hessenberg data."""
    from oracle import poly as opoly
    from paper_2205_09104_amd import harmonic_ritz, leja_order
    rng = np.random.default_rng(2)
    for d in (2, 4, 8, 16, 20):
        H = np.triu(rng.standard_normal((d + 1, d)) + 1j * rng.standard_normal((d + 1, d)), -1)
        th = harmonic_ritz(H)
        ref = opoly.harmonic_ritz(H)
        assert max(np.min(np.abs(ref - t)) for t in th) <= 1e-9 * np.abs(ref).max()
        # Leja order of identical inputs is identical
        assert np.array_equal(leja_order(ref), opoly.leja_order(ref))
    with open(os.path.join(ROOT, "tests", "golden", "leja_examples.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            inp, out = line.split("->")
            theta = np.array([complex(t) for t in inp.split()])
            want = np.array([complex(t) for t in out.split()])
            assert np.array_equal(leja_order(theta), want), line
