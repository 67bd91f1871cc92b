"""Oracle pins for orbital-resolved quantum numbers (Sec. 2.2: with the
density-density interaction and orbital-diagonal hybridisation the number of
electrons of each spin is conserved per orbital, N_ud = Norb).

  * the per-orbital basis follows eq. SectorIndxDecomp (mixed radix, orbital 1
    fastest, each orbital's Nbit-bit string at its position in the ascending
    listing), checked against a brute-force filter of all strings;
  * the spectra of all orbital-resolved sectors with sum_a N_a,s = N_s together
    are the spectrum of the total-N sector (as multisets);
  * the ground state's G from its orbital-resolved sector equals G from the
    total-N sector (exact Lehmann sums, non-degenerate ground state);
  * spin exchange mixes orbital counts (so such models need the total-N form).
"""
import itertools

import numpy as np
import pytest

from oracle import fock, green
from paper_2105_06806_amd import inputs


def _brute_basis(model, counts):
    norb, nbath = model["norb"], model["nbath"]
    ns = fock.ns_of(model)
    nbit = nbath + 1
    out = []
    for s in range(1 << ns):
        idx, radix, ok = 0, 1, True
        for a in range(norb):
            lv = fock.orbital_levels(model, a)
            loc = sum(((s >> l) & 1) << k for k, l in enumerate(lv))
            if bin(loc).count("1") != counts[a]:
                ok = False
                break
            lst = [int(x) for x in fock.spin_strings_listing(nbit, counts[a])]
            idx += lst.index(loc) * radix
            radix *= len(lst)
        if ok:
            out.append((idx, s))
    out.sort()
    return np.array([s for _, s in out], dtype=np.uint64)


@pytest.mark.parametrize("norb,nbath,counts", [(2, 2, (1, 2)), (2, 2, (3, 0)), (3, 1, (1, 0, 2)),
                                                (2, 3, (2, 2))])
def test_basis_order(norb, nbath, counts):
    m = inputs.make_model(norb, nbath, 2.0, Jh=0.3, seed=3, symmetric=False)
    assert np.array_equal(fock.orbital_spin_strings(m, counts), _brute_basis(m, counts))


def _orbital_specs(norb, nbit, n):
    return [c for c in itertools.product(range(nbit + 1), repeat=norb) if sum(c) == n]


@pytest.mark.parametrize("norb,nbath,sec", [(2, 2, (3, 3)), (3, 1, (3, 2)), (2, 1, (2, 1))])
def test_spectra_union(norb, nbath, sec):
    m = inputs.make_model(norb, nbath, 3.0, Jh=0.5, seed=4, symmetric=False)
    full = np.sort(np.linalg.eigvalsh(fock.explicit_hamiltonian(m, *sec).toarray()))
    parts = []
    for cu in _orbital_specs(norb, nbath + 1, sec[0]):
        for cd in _orbital_specs(norb, nbath + 1, sec[1]):
            H = fock.explicit_hamiltonian(m, cu, cd).toarray()
            assert np.abs(H - H.T).max() == 0.0
            parts.append(np.linalg.eigvalsh(H))
    parts = np.sort(np.concatenate(parts))
    assert parts.size == full.size
    assert np.abs(parts - full).max() < 1e-11


def test_green_from_orbital_sector():
    m = inputs.make_model(2, 2, 3.0, Jh=0.5, seed=9, symmetric=False)
    sec = (3, 3)
    z = 1j * green.matsubara(30.0, 64)
    best = None
    for cu in _orbital_specs(2, 3, 3):
        for cd in _orbital_specs(2, 3, 3):
            w = np.linalg.eigvalsh(fock.explicit_hamiltonian(m, cu, cd).toarray())
            if best is None or w[0] < best[0]:
                best = (w[0], cu, cd)
    wf = np.linalg.eigvalsh(fock.explicit_hamiltonian(m, *sec).toarray())
    assert wf[1] - wf[0] > 1e-6 and abs(wf[0] - best[0]) < 1e-11
    for orb in (0, 1):
        for spin in (0, 1):
            Gf, Ef = green.lehmann_exact(m, *sec, orb, spin, z)
            Go, Eo = green.lehmann_exact(m, best[1], best[2], orb, spin, z)
            assert abs(Ef - Eo) < 1e-11
            assert np.abs(Gf - Go).max() < 1e-11 * np.abs(Gf).max()


def test_spin_exchange_mixes_orbital_counts():
    m = inputs.make_model(2, 1, 3.0, Jh=0.5, seed=2, symmetric=False, Jx=0.5, Jp=0.5)
    H = fock.explicit_hamiltonian(m, 2, 2).toarray()
    up, dw, I = fock.sector_states(fock.ns_of(m), 2, 2)
    lab = [tuple(bin(int(s) & mask).count("1") for mask in (0b0101, 0b1010)) for s in up]
    # some nonzero element connects different orbital occupations of spin up
    iu = np.arange(H.shape[0]) % len(up)
    r, c = np.nonzero(H)
    assert any(lab[iu[a]] != lab[iu[b]] for a, b in zip(r, c))
