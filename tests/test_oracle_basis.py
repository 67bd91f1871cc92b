"""Pins of the oracle's sector basis and per-spin tables (CPU only).

* The basis is built two independent ways: the build_sector listing (loop over
  every integer, keep popcount == N; Sec. 6 "Sector construction") and sorted
  combinations; both must agree and have length C(Ns, N) (eq. nud_dimension).
* Sector order: i = i_up + i_dw * D_up (eq. Vmatrix) equals ascending order of
  the Fock integer I = I_up + I_dw 2**Ns (eq. Irelation).
* Per-spin hop signs equal the 'bits strictly between' closed form, computed
  here by brute force on single strings.
"""
import math

import numpy as np
import pytest

from oracle import fock, rng
from paper_2105_06806_amd import inputs


@pytest.mark.parametrize("ns", range(1, 13))
def test_listing_equals_combinations(ns):
    for n in range(ns + 1):
        a = fock.spin_strings_listing(ns, n)
        b = fock.spin_strings(ns, n)
        assert a.size == math.comb(ns, n)
        assert np.array_equal(a, b)
        assert np.all(np.diff(a.astype(np.int64)) > 0)


def test_invalid_counts_empty():
    assert fock.spin_strings(6, 7).size == 0
    assert fock.spin_strings(6, -1).size == 0
    assert fock.sector_dim(6, 7, 3) == 0


@pytest.mark.parametrize("ns,nup,ndw", [(4, 2, 2), (6, 3, 2), (8, 4, 4), (7, 0, 7)])
def test_sector_order_is_fock_order(ns, nup, ndw):
    up, dw, I = fock.sector_states(ns, nup, ndw)
    assert I.size == math.comb(ns, nup) * math.comb(ns, ndw)
    assert np.all(np.diff(I.astype(np.int64)) > 0)
    i = np.arange(I.size)
    assert np.array_equal(I, up[i % len(up)] + (dw[i // len(up)] << np.uint64(ns)))


def test_dimension_formula_headline():
    # D = C(16,8)^2 for the half-filled Ns=16 sector
    assert math.comb(16, 8) ** 2 == 165636900
    assert fock.sector_dim(12, 6, 6) == 924 ** 2


def _brute_sign(s, a, b):
    """(-1)**(occupied levels strictly between a and b) for a single string."""
    lo, hi = min(a, b), max(a, b)
    return (-1) ** sum((s >> k) & 1 for k in range(lo + 1, hi))


@pytest.mark.parametrize("spin", [0, 1])
@pytest.mark.parametrize("norb,nbath,n", [(1, 5, 3), (2, 2, 3), (3, 1, 2), (1, 7, 4)])
def test_spin_hop_sign_between_rule(spin, norb, nbath, n):
    m = inputs.make_model(norb, nbath, 2.0, seed=3, symmetric=False)
    ns = fock.ns_of(m)
    off, col, sgn, amp = fock.spin_hop_csr(m, n, spin)
    strings = fock.spin_strings(ns, n)
    pairs = {}
    for (a, b, V) in fock.hop_pairs(m):
        pairs[(a, b)] = V
    for i in range(len(strings)):
        s = int(strings[i])
        expect = {}
        for (a, b), V in pairs.items():
            if ((s >> a) & 1) != ((s >> b) & 1):
                t = s ^ (1 << a) ^ (1 << b)
                j = int(np.searchsorted(strings, np.uint64(t)))
                expect[j] = (_brute_sign(s, a, b), V)
        got = {int(col[k]): (int(sgn[k]), float(amp[k])) for k in range(off[i], off[i + 1])}
        assert got == expect


def test_splitmix64_published_outputs():
    # Reference outputs of splitmix64 seeded with 0 (Vigna's public-domain
    # splitmix64.c): 0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4, 0x06c45d188009454f.
    assert [rng.splitmix64_scalar(0, k) for k in range(3)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    z = rng.splitmix64(12345, 1000)
    assert all(int(z[k]) == rng.splitmix64_scalar(12345, k) for k in (0, 1, 17, 999))
    u = rng.uniform_pm1(5, 100000)
    assert u.min() >= -1.0 and u.max() < 1.0 and abs(u.mean()) < 0.01
