"""Pins of the oracle's row-by-row product ``fock.hv_rows`` on the paths the
large-sector GPU checks rely on (CPU only).

``hv_rows`` is the reference for output rows of sectors whose matrix is too
large to store.  Besides the total-N density-density sectors (pinned in
test_oracle_hamiltonian.py) it has two more paths:

  * the spin-exchange and pair-hopping terms of eq. Ham1 (Jx, Jp != 0): every
    row is compared with the Jordan-Wigner build (an independent construction
    from 2x2 Kronecker factors, Ns <= 5) and, on larger sectors, with the
    explicit sector matrix (itself pinned to Jordan-Wigner), for both signs of
    each coupling and for Norb = 2 and 3;
  * orbital-resolved sectors (Sec. 2.2 with N_ud = N_alpha): the sector's
    states are a subset of the total-N sector's, and a density-density model
    with orbital-diagonal hybridisation leaves that subset invariant, so H of
    the orbital sector is the restriction of the total-N matrix.  Every row of
    hv_rows is compared with the total-N explicit product of the embedded
    vector, which must also vanish outside the subset.

A planted mistake (a dropped pair-hopping term in the row product) is caught.
"""
import itertools

import numpy as np
import pytest

from oracle import fock, jw
from paper_2105_06806_amd import inputs


def _model(norb, nbath, jx, jp, seed):
    return inputs.make_model(norb, nbath, 3.0, Jh=0.6, seed=seed, symmetric=False,
                             elo=-1.0, ehi=1.0, vlo=0.2, vhi=0.6, Jx=jx, Jp=jp, xmu=0.13)


SIGNS = [(0.45, 0.35), (-0.45, 0.35), (0.45, -0.35), (-0.3, -0.5), (0.5, 0.0), (0.0, 0.5)]


@pytest.mark.parametrize("jx,jp", SIGNS)
@pytest.mark.parametrize("norb,nbath,sec", [(2, 1, (2, 2)), (2, 1, (3, 1)), (2, 1, (1, 2)),
                                            (3, 0, (2, 1)), (3, 0, (2, 2)), (3, 0, (1, 1))])
def test_nondiag_rows_equal_jordan_wigner(norb, nbath, sec, jx, jp):
    m = _model(norb, nbath, jx, jp, seed=11)
    A = jw.sector_block(m, *sec)
    x = np.random.default_rng(3).standard_normal(A.shape[0])
    rows = np.arange(A.shape[0])
    got = fock.hv_rows(m, *sec, x, rows)
    assert np.abs(got - A @ x).max() <= 1e-13 * max(1.0, np.abs(A @ x).max())


@pytest.mark.parametrize("jx,jp", SIGNS[:4])
@pytest.mark.parametrize("norb,nbath,sec", [(2, 3, (4, 4)), (2, 3, (5, 3)), (3, 2, (4, 5)),
                                            (3, 2, (5, 5)), (2, 4, (5, 4))])
def test_nondiag_rows_equal_explicit(norb, nbath, sec, jx, jp):
    m = _model(norb, nbath, jx, jp, seed=12)
    H = fock.explicit_hamiltonian(m, *sec)
    x = np.random.default_rng(4).standard_normal(H.shape[0])
    ref = H @ x
    got = fock.hv_rows(m, *sec, x, np.arange(H.shape[0]))
    assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    # the spin-exchange / pair-hopping part is really exercised
    m0 = dict(m, Jx=0.0, Jp=0.0)
    ref0 = fock.explicit_hamiltonian(m0, *sec) @ x
    assert np.abs(ref - ref0).max() > 1e-3


def test_planted_missing_pair_hopping_is_caught():
    m = _model(2, 1, 0.45, 0.35, seed=11)
    sec = (2, 2)
    A = jw.sector_block(m, *sec)
    x = np.random.default_rng(3).standard_normal(A.shape[0])
    orig = fock.nondiagonal_terms
    try:
        # drop the pair-hopping operators from the term list
        fock.nondiagonal_terms = lambda mm: [t for t in orig(mm) if t[0] < 0]
        bad = fock.hv_rows(m, *sec, x, np.arange(A.shape[0]))
    finally:
        fock.nondiagonal_terms = orig
    assert np.abs(bad - A @ x).max() > 1e-3


def _orbital_cases():
    out = []
    for (norb, nbath, cup, cdw) in [(2, 2, (1, 2), (2, 1)), (2, 2, (3, 0), (1, 1)),
                                    (3, 1, (1, 0, 2), (2, 1, 1)), (2, 3, (2, 2), (1, 3)),
                                    (3, 2, (1, 2, 1), (2, 1, 2)), (2, 4, (2, 3), (3, 2))]:
        out.append((norb, nbath, cup, cdw))
    return out


@pytest.mark.parametrize("norb,nbath,cup,cdw", _orbital_cases())
def test_orbital_rows_equal_total_sector_restriction(norb, nbath, cup, cdw):
    m = inputs.make_model(norb, nbath, 2.5, Jh=0.4, seed=21, symmetric=False, xmu=0.2)
    ns = fock.ns_of(m)
    _, _, I_orb = fock.sector_states(ns, list(cup), list(cdw), m)
    nu, nd = sum(cup), sum(cdw)
    _, _, I_tot = fock.sector_states(ns, nu, nd)
    order = np.argsort(I_tot)
    pos = order[np.searchsorted(I_tot[order], I_orb)]
    assert np.array_equal(I_tot[pos], I_orb)          # every orbital state is in the total sector
    Htot = fock.explicit_hamiltonian(m, nu, nd)
    x = np.random.default_rng(5).standard_normal(I_orb.size)
    xt = np.zeros(I_tot.size)
    xt[pos] = x
    yt = Htot @ xt
    outside = np.ones(I_tot.size, dtype=bool)
    outside[pos] = False
    assert np.abs(yt[outside]).max(initial=0.0) == 0.0   # the subset is invariant
    got = fock.hv_rows(m, list(cup), list(cdw), x, np.arange(I_orb.size))
    assert np.abs(got - yt[pos]).max() <= 1e-13 * max(1.0, np.abs(yt).max())


def test_orbital_rows_cover_every_count_split():
    """All orbital sectors of one total-N sector together reproduce its product."""
    m = inputs.make_model(2, 2, 2.0, Jh=0.3, seed=22, symmetric=False)
    ns, nbit = fock.ns_of(m), 3
    nu, nd = 3, 2
    _, _, I_tot = fock.sector_states(ns, nu, nd)
    order = np.argsort(I_tot)
    x_tot = np.random.default_rng(6).standard_normal(I_tot.size)
    y_tot = fock.explicit_hamiltonian(m, nu, nd) @ x_tot
    y = np.full(I_tot.size, np.nan)
    splits = lambda n: [c for c in itertools.product(range(nbit + 1), repeat=2) if sum(c) == n]
    for cu in splits(nu):
        for cd in splits(nd):
            _, _, I_orb = fock.sector_states(ns, list(cu), list(cd), m)
            pos = order[np.searchsorted(I_tot[order], I_orb)]
            y[pos] = fock.hv_rows(m, list(cu), list(cd), x_tot[pos], np.arange(I_orb.size))
    assert not np.isnan(y).any()
    assert np.abs(y - y_tot).max() <= 1e-13 * np.abs(y_tot).max()
