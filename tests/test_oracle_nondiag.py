"""Oracle pins for the spin-exchange and pair-hopping terms of eq. Ham1.

  * the bit-string build equals the Jordan-Wigner matrix build (an independent
    construction from 2x2 Kronecker factors) on small systems, and differs
    from it if the sign of either coupling is flipped;
  * the isolated two-orbital atom with the Kanamori choice U' = U - 2J,
    Jx = Jp = J has the textbook two-electron spectrum: U - 3J (triplet, three
    states), U - J (two singlets), U + J (one singlet);
  * with a bath, the three-orbital Kanamori impurity is spin-rotation
    invariant: every level of the S_z = 1 sector is also a level of the
    S_z = 0 sector with the same electron count.  This fails for Jx = 0 (only
    the density-density part) and for the opposite sign of Jx, so it fixes
    that sign; the sign of Jp is fixed by the Jordan-Wigner comparison.
"""
import numpy as np
import pytest

from oracle import fock, jw
from paper_2105_06806_amd import inputs


def _model(norb, nbath, U, J, jx, jp, seed=1):
    m = inputs.make_model(norb, nbath, U, Jh=J, seed=seed, symmetric=False,
                          elo=-1.0, ehi=1.0, vlo=0.2, vhi=0.6, Jx=jx, Jp=jp)
    return m


@pytest.mark.parametrize("norb,nbath,sec", [(2, 1, (2, 2)), (2, 1, (3, 1)), (2, 1, (1, 2)),
                                            (3, 0, (2, 1)), (3, 0, (2, 2))])
def test_bits_equal_jordan_wigner(norb, nbath, sec):
    m = _model(norb, nbath, 3.0, 0.6, 0.45, 0.35)
    H = fock.explicit_hamiltonian(m, *sec).toarray()
    Hjw = jw.sector_block(m, *sec)
    assert np.abs(H - Hjw).max() < 1e-13
    assert np.abs(H - H.T).max() == 0.0
    for key in ("Jx", "Jp"):
        bad = dict(m)
        bad[key] = -m[key]
        Hb = fock.explicit_hamiltonian(bad, *sec).toarray()
        if np.abs(Hb - Hjw).max() < 1e-9:
            # the flipped coupling has no matrix element in this sector
            assert np.abs(fock.explicit_hamiltonian(dict(m, **{key: 0.0}), *sec).toarray()
                          - Hjw).max() < 1e-13
        else:
            assert np.abs(Hb - Hjw).max() > 0.1


def test_two_orbital_atom_spectrum():
    U, J = 4.0, 0.7
    m = {"norb": 2, "nbath": 0, "eps_imp": np.zeros(2), "xmu": 0.0,
         "eps_bath": np.zeros((2, 0)), "vhyb": np.zeros((2, 0)),
         "U": U, "Ust": U - 2 * J, "Jh": J, "Jx": J, "Jp": J}
    ev = []
    for sec in [(2, 0), (1, 1), (0, 2)]:
        ev += list(np.linalg.eigvalsh(fock.explicit_hamiltonian(m, *sec).toarray()))
    ev = np.sort(ev)
    ref = np.sort([U - 3 * J] * 3 + [U - J] * 2 + [U + J])
    assert np.allclose(ev, ref, atol=1e-12)


def _levels(m, sec):
    return np.linalg.eigvalsh(fock.explicit_hamiltonian(m, *sec).toarray())


@pytest.mark.parametrize("jx_sign,ok", [(1.0, True), (0.0, False), (-1.0, False)])
def test_kanamori_spin_rotation_invariance(jx_sign, ok):
    """Three orbitals: with two, flipping the sign of Jx is undone by a gauge
    change of one orbital's spin-up operators (which also flips Jp, and the
    spin-rotation test is blind to the sign of Jp); with three orbitals the
    product of the exchange signs around the orbital triangle is gauge
    invariant, so only the printed sign gives multiplets."""
    U, J = 3.0, 0.5
    m = inputs.make_model(3, 1, U, Jh=J, seed=7, symmetric=False, elo=-1, ehi=1, vlo=0.3, vhi=0.7,
                          Jx=jx_sign * J, Jp=J)
    a = _levels(m, (4, 2))                 # S_z = 1, N = 6
    b = _levels(m, (3, 3))                 # S_z = 0, N = 6
    d = np.array([np.abs(b - x).min() for x in a])
    if ok:
        assert d.max() < 1e-10
    else:
        assert d.min() > 1e-6 or (d > 1e-6).sum() > len(d) // 2
