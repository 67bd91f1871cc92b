"""Oracle pins for the electron-phonon (Holstein) impurity (Sec. "Electron-phonon
coupling", eq. HephBuild).

  * g = 0: the spectrum is the electronic one plus w0 p for every p (phonons
    decouple), and G equals the purely electronic G;
  * atomic limit (no bath hybridisation, one orbital): the independent-boson
    closed form E = E_el + w0 k - g^2 n^2 / w0 per occupation n, reached as the
    phonon cutoff grows;
  * the matrix equals a dense Kronecker build from the printed operators with
    the phonon index slowest, and a transposed factor order is caught;
  * sampled rows equal the explicit product.
"""
import numpy as np
import pytest

from oracle import eph, fock, green
from paper_2105_06806_amd import inputs


def _ph(m, nph, w0, g):
    m = dict(m)
    m.update(nph=nph, w0=w0, g=np.asarray(g, float))
    return m


def test_decoupled_spectrum_and_g():
    m0 = inputs.make_model(1, 3, 2.0, seed=101, symmetric=False)
    m = _ph(m0, 4, 0.7, [0.0])
    sec = (2, 2)
    we = np.linalg.eigvalsh(fock.explicit_hamiltonian(m0, *sec).toarray())
    w = np.linalg.eigvalsh(eph.explicit_hamiltonian(m, *sec).toarray())
    ref = np.sort(np.concatenate([we + 0.7 * p for p in range(5)]))
    assert np.abs(w - ref).max() < 1e-12
    z = 1j * green.matsubara(30.0, 16)
    g1, _ = eph.lehmann_exact(m, *sec, 0, 0, z)
    g2, _ = green.lehmann_exact(m0, *sec, 0, 0, z)
    assert np.abs(g1 - g2).max() < 1e-10


def test_atomic_limit_independent_boson():
    """V = 0: each electronic Fock state with impurity occupation n has phonon
    levels w0 k - g^2 n^2 / w0 (displaced oscillator), exact as N_ph grows."""
    m0 = inputs.make_model(1, 2, 1.5, seed=102, symmetric=False)
    m0["vhyb"] = np.zeros_like(m0["vhyb"])
    w0, g = 1.0, 0.3
    sec = (1, 1)
    He = fock.explicit_hamiltonian(m0, *sec).toarray()
    ns = fock.ns_of(m0)
    _, _, I = fock.sector_states(ns, *sec)
    nimp = fock.occupations(I, ns)[0] + fock.occupations(I, ns)[ns]
    ref = np.sort(np.concatenate([np.diag(He) + w0 * k - g * g * nimp ** 2 / w0 for k in range(4)]))
    w = np.linalg.eigvalsh(eph.explicit_hamiltonian(_ph(m0, 40, w0, [g]), *sec).toarray())
    assert np.abs(w[:ref.size // 2] - ref[:ref.size // 2]).max() < 1e-10
    # a small cutoff is visibly off: the truncation is real
    w5 = np.linalg.eigvalsh(eph.explicit_hamiltonian(_ph(m0, 1, w0, [g]), *sec).toarray())
    assert abs(w5[0] - ref[0]) > 1e-4


def test_dense_kronecker_build_and_order():
    m = _ph(inputs.make_model(2, 1, 2.0, Jh=0.3, seed=103, symmetric=False), 3, 0.6, [0.25, -0.4])
    sec = (2, 1)
    He = fock.explicit_hamiltonian(m, *sec).toarray()
    ns = fock.ns_of(m)
    _, _, I = fock.sector_states(ns, *sec)
    occ = fock.occupations(I, ns)
    G = np.diag(0.25 * (occ[0] + occ[ns]) - 0.4 * (occ[1] + occ[ns + 1]))
    b = np.diag(np.sqrt(np.arange(1, 4)), 1)
    ref = np.kron(np.eye(4), He) + 0.6 * np.kron(np.diag(np.arange(4.0)), np.eye(len(He))) + \
        np.kron(b + b.T, G)
    H = eph.explicit_hamiltonian(m, *sec).toarray()
    assert np.abs(H - ref).max() < 1e-14
    wrong = np.kron(He, np.eye(4)) + 0.6 * np.kron(np.eye(len(He)), np.diag(np.arange(4.0))) + \
        np.kron(G, b + b.T)
    assert np.abs(H - wrong).max() > 0.1


def test_sampled_rows():
    m = _ph(inputs.make_model(1, 4, 2.0, seed=104, symmetric=False), 5, 0.8, [0.5])
    sec = (3, 2)
    H = eph.explicit_hamiltonian(m, *sec)
    v = np.random.default_rng(1).standard_normal(H.shape[0])
    rows = np.arange(H.shape[0])
    assert np.abs(eph.hv_rows(m, *sec, v, rows) - H @ v).max() < 1e-12
