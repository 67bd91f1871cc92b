"""Pins of the oracle's eigen-solvers (CPU only).

* Dense LAPACK eigh, Lanczos with full re-orthogonalisation and ARPACK agree
  on the Ns=8 half-filled sector (D=4900, fully dense-checkable).
* U=0: ground energy = sum of the lowest N_up + N_dw one-body eigenvalues.
* V=0: ground energy = atomic-limit minimum (multi-orbital included).
* Particle-hole symmetry of the symmetrised bath: E0(Nu,Nd) = E0(Ns-Nu,Ns-Nd).
* Twin sectors (Sec. 6 "Diagonalization"): E0(a,b) = E0(b,a).
* The plain-recurrence ground energy (the paper's Lanczos) reaches the exact
  value within its stop rule.
"""
import numpy as np
import pytest

from oracle import closed, fock, kron, rng, spectra
from paper_2105_06806_amd import inputs


def _e0_dense(m, sec):
    """Dense LAPACK for D <= 2500, ARPACK above (ARPACK itself is pinned to
    LAPACK in test_three_solvers_agree_ns8)."""
    H = fock.explicit_hamiltonian(m, *sec)
    if H.shape[0] <= 2500:
        return spectra.dense_lowest(H)[0][0]
    return spectra.arpack_lowest(H)[0]


def test_three_solvers_agree_ns8():
    m, [sec] = inputs.workload("ns8")
    H = fock.explicit_hamiltonian(m, *sec)
    Ed = spectra.dense_lowest(H)[0][0]
    El, psi, _ = spectra.lanczos_full_reorth(lambda x: H @ x, rng.start_vector(1, H.shape[0]))
    Ea, _ = spectra.arpack_lowest(H)
    assert abs(El - Ed) <= 1e-12 * abs(Ed)
    assert abs(Ea - Ed) <= 1e-12 * abs(Ed)
    assert np.linalg.norm(H @ psi - Ed * psi) < 1e-8


@pytest.mark.parametrize("norb,nbath,sec", [(1, 7, (4, 4)), (1, 7, (3, 5)), (2, 3, (4, 3)), (1, 9, (2, 3))])
def test_noninteracting_closed_form(norb, nbath, sec):
    m = inputs.make_model(norb, nbath, 0.0, seed=17, symmetric=False, eps_imp=0.13)
    m["xmu"] = -0.05
    assert abs(_e0_dense(m, sec) - closed.e0_noninteracting(m, *sec)) < 1e-11


@pytest.mark.parametrize("norb,nbath,U,J,sec", [(1, 7, 2.0, 0.0, (4, 4)), (2, 3, 3.0, 0.5, (4, 4)),
                                               (2, 3, 3.0, 0.5, (2, 6)), (3, 2, 3.0, 0.5, (4, 5))])
def test_atomic_closed_form(norb, nbath, U, J, sec):
    m = inputs.make_model(norb, nbath, U, Jh=J, seed=19, symmetric=False)
    m["vhyb"][:] = 0.0
    assert abs(_e0_dense(m, sec) - closed.e0_atomic(m, *sec)) < 1e-12


def test_particle_hole_symmetry():
    m, _ = inputs.workload("ns8")
    ns = 8
    for (a, b) in [(4, 4), (5, 4), (5, 3), (6, 4)]:
        assert abs(_e0_dense(m, (a, b)) - _e0_dense(m, (ns - a, ns - b))) < 1e-12
    # multi-orbital with the Hartree-shifted impurity level and a symmetrised bath
    m2 = inputs.make_model(2, 3, 3.0, Jh=0.5, seed=23, symmetric=True)
    assert abs(_e0_dense(m2, (5, 3)) - _e0_dense(m2, (3, 5))) < 1e-12
    assert abs(_e0_dense(m2, (5, 4)) - _e0_dense(m2, (3, 4))) < 1e-12


def test_twin_sectors():
    m = inputs.make_model(1, 7, 2.5, seed=29, symmetric=False)
    for (a, b) in [(5, 3), (2, 4)]:
        assert abs(_e0_dense(m, (a, b)) - _e0_dense(m, (b, a))) < 1e-12


def test_plain_lanczos_ground_energy():
    m, [sec] = inputs.workload("ns8")
    H = fock.explicit_hamiltonian(m, *sec)
    Ed = spectra.dense_lowest(H)[0][0]
    E, steps = spectra.lanczos_ground_energy_plain(lambda x: H @ x, rng.start_vector(3, H.shape[0]), 200, 1e-12)
    assert abs(E - Ed) <= 1e-10 * abs(Ed)
    assert steps < 200


def test_kron_form_lanczos_matches_explicit():
    m = inputs.make_model(2, 3, 3.0, Jh=0.5, seed=31, symmetric=False)
    K = kron.KronH(m, 4, 4)
    Ed = _e0_dense(m, (4, 4))
    E, _, _ = spectra.lanczos_full_reorth(K.matvec, rng.start_vector(2, K.dim))
    assert abs(E - Ed) < 1e-11
