"""Host logic of the library (no GPU): the tridiagonal eigen-solver behind the
Krylov spectral functions, against LAPACK on random, split, clustered and
nearly diagonal matrices; weights are checked through the resolvent identity
sum_m w_m / (z - theta_m) = [(z - T)^-1]_00, which is unique even where
eigenvalues are degenerate."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def edx():
    from paper_2105_06806_amd import edx as E
    return E


def test_tridiag_spectrum_against_lapack(edx):
    rng = np.random.default_rng(1)
    for trial in range(200):
        m = int(rng.integers(1, 50))
        a = rng.normal(size=m)
        b = np.abs(rng.normal(size=max(m - 1, 0)))
        if trial % 4 == 1 and m > 3:
            b[rng.integers(0, m - 1)] = 1e-17        # a split block
        if trial % 4 == 2:
            a[:] = 0.7                               # clustered spectrum
        if trial % 4 == 3:
            b *= 1e-9                                # nearly diagonal
        th, w = edx.tridiag_spectrum(a, b)
        T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        ev = np.linalg.eigvalsh(T)
        assert np.abs(th - ev).max() <= 1e-13 * max(1.0, np.abs(ev).max())
        assert abs(w.sum() - 1) < 1e-13 and np.all(w >= 0)
        for z in (0.3 + 0.7j, -1.1 + 0.05j):
            g = np.linalg.inv(z * np.eye(m) - T)[0, 0]
            assert abs((w / (z - th)).sum() - g) < 1e-11 * max(1.0, abs(g))


def test_tridiag_spectrum_rejects(edx):
    with pytest.raises(ValueError):
        edx.tridiag_spectrum([1.0, 2.0], [])
