"""Oracle pins for several low-lying states and finite temperature (Sec. 6
"Eigenspace class" and the thermal form of "Dynamical correlation functions").

  * the per-state thermal sum over every eigenstate equals the textbook
    Lehmann double sum, and both equal a Jordan-Wigner build on the whole Fock
    space (no sectors, no sector signs);
  * U = 0: the thermal G over the whole Fock space is the Dyson closed form
    (independent of temperature) at two temperatures;
  * beta -> infinity: the thermal G is the T = 0 G of the unique ground state;
  * truncation by the Boltzmann cutoff and the annealing rule on hand-worked
    examples, and the truncation error stays within its bound;
  * the k lowest states of a sector are the lowest k of the whole-Fock-space
    spectrum restricted to that sector's quantum numbers.
"""
import math

import numpy as np
import pytest

from oracle import closed, fock, green, jw, thermal
from paper_2105_06806_amd import inputs


def _tiny(norb, nbath, U, seed, **kw):
    return inputs.make_model(norb, nbath, U, seed=seed, symmetric=False, **kw)


def _jw_thermal_g(model, orb, spin, z, beta):
    """Whole-Fock-space Lehmann double sum with Jordan-Wigner matrices."""
    ns = fock.ns_of(model)
    H, c = jw.fock_hamiltonian(model)
    w, V = np.linalg.eigh(H)
    cd = V.T @ c[orb + spin * ns].T @ V            # <m|c+|n>
    b = np.exp(-beta * (w - w[0]))
    num = cd ** 2 * (b[None, :] + b[:, None])
    G = np.zeros(len(z), dtype=complex)
    den = w[:, None] - w[None, :]
    mask = num > 0
    for k, zz in enumerate(z):
        G[k] = (num[mask] / (zz - den[mask])).sum()
    return G / b.sum()


@pytest.mark.parametrize("norb,nbath,spin,orb", [(1, 2, 0, 0), (2, 1, 1, 1), (1, 3, 1, 0)])
def test_per_state_equals_double_sum_and_jordan_wigner(norb, nbath, spin, orb):
    m = _tiny(norb, nbath, 2.5, seed=61 + norb, Jh=0.3)
    beta = 4.0
    z = 1j * green.matsubara(beta, 16)
    g1 = thermal.green_states_exact(m, thermal.all_states(m), orb, spin, z, beta)
    g2 = thermal.green_double_sum(m, orb, spin, z, beta)
    g3 = _jw_thermal_g(m, orb, spin, z, beta)
    assert np.abs(g1 - g2).max() < 1e-12
    assert np.abs(g1 - g3).max() < 1e-12
    # sum rule: i w_n G -> 1 (total spectral weight one)
    zz = np.array([1e6j])
    assert abs(zz[0] * thermal.green_double_sum(m, orb, spin, zz, beta)[0] - 1) < 1e-5


def test_jordan_wigner_catches_a_sign_error(monkeypatch):
    """A planted sign error in the operator application is caught by the
    Jordan-Wigner comparison."""
    m = _tiny(2, 1, 2.0, seed=65, Jh=0.3)
    beta = 3.0
    z = 1j * green.matsubara(beta, 8)
    ref = _jw_thermal_g(m, 1, 1, z, beta)
    orig = fock.apply_cdag

    def bad(I, mode):
        valid, Inew, sgn = orig(I, mode)
        return valid, Inew, np.ones_like(sgn)        # drop the fermionic sign
    monkeypatch.setattr(fock, "apply_cdag", bad)
    got = thermal.green_states_exact(m, thermal.all_states(m), 1, 1, z, beta)
    assert np.abs(got - ref).max() > 1e-3


@pytest.mark.parametrize("beta", [2.0, 15.0])
def test_noninteracting_closed_form_any_temperature(beta):
    m = _tiny(1, 3, 0.0, seed=66, eps_imp=0.3)
    z = 1j * green.matsubara(beta, 32)
    g = thermal.green_states_exact(m, thermal.all_states(m), 0, 0, z, beta)
    assert np.abs(g - closed.g_noninteracting(m, 0, z)).max() < 1e-12


def test_large_beta_is_ground_state_g():
    m = inputs.make_model(1, 3, 2.0, seed=67)          # particle-hole symmetric, Ns = 4
    states = thermal.all_states(m)
    e = np.array([s[0] for s in states])
    order = np.argsort(e)
    assert e[order[1]] - e[order[0]] > 0.05            # unique ground state
    gs_sec = states[order[0]][1]
    beta = 600.0
    z = 1j * green.matsubara(beta, 16)
    g = thermal.green_states_exact(m, states, 0, 0, z, beta)
    g0, _ = green.lehmann_exact(m, *gs_sec, 0, 0, z)
    assert np.abs(g - g0).max() < 1e-9


def test_espace_select_by_hand():
    # (E, sector, state); beta = 10: factors 1, e^-1, e^-5, e^-30
    ent = [(0.5, 1, 0), (0.0, 0, 0), (3.0, 2, 0), (0.1, 0, 1)]
    assert thermal.espace_select(ent, 10.0, 1e-9, 10) == [(0.0, 0, 0), (0.1, 0, 1), (0.5, 1, 0)]
    assert thermal.espace_select(ent, 10.0, 1e-9, 2) == [(0.0, 0, 0), (0.1, 0, 1)]
    assert thermal.espace_select(ent, 10.0, 1e-2, 10) == [(0.0, 0, 0), (0.1, 0, 1)]
    assert thermal.espace_select(ent, 10.0, 1e-20, 10) == sorted(ent)
    assert thermal.espace_select([], 10.0, 1e-9, 10) == []


def test_anneal_by_hand():
    # sector 0 kept everything it computed -> grows; 1 lost one -> cut to 1;
    # 2 kept nothing -> stays at one state
    assert thermal.anneal([2, 2, 2], [2, 2, 1], [2, 1, 0], 2) == [4, 1, 1]
    assert thermal.anneal([3], [3], [3], 1) == [4]


def test_truncation_error_bound():
    """Dropping the states under the cutoff changes G by at most
    2 * (dropped Boltzmann fraction) / omega_0 (each |G_n(i w)| <= 1/w)."""
    m = _tiny(1, 3, 2.0, seed=68)
    beta = 3.0
    z = 1j * green.matsubara(beta, 8)
    states = thermal.all_states(m)
    full = thermal.green_states_exact(m, states, 0, 0, z, beta)
    ent = [(s[0], i, 0) for i, s in enumerate(states)]
    cutoff = 5e-3
    kept = thermal.espace_select(ent, beta, cutoff, len(ent))
    assert 0 < len(kept) < len(ent)
    sub = [states[k[1]] for k in kept]
    trunc = thermal.green_states_exact(m, sub, 0, 0, z, beta)
    b = thermal.boltzmann([s[0] for s in states], beta)
    dropped = 1.0 - sum(b[k[1]] for k in kept) / b.sum()
    err = np.abs(trunc - full).max()
    assert 0 < err <= 2 * dropped / z[0].imag


def test_lowest_states_are_lowest_of_fock_space_block():
    m = _tiny(2, 1, 2.5, seed=69, Jh=0.4)
    H, _ = jw.fock_hamiltonian(m)
    ns = fock.ns_of(m)
    for sec in [(2, 1), (2, 2), (0, 3)]:
        _, _, I = fock.sector_states(ns, *sec)
        # the block of the Fock-space H on the sector's states, independently built
        blk = H[np.ix_(I.astype(np.int64), I.astype(np.int64))]
        ref = np.linalg.eigvalsh(blk)
        k = min(5, len(ref))
        e, V = thermal.lowest_states(m, sec, 5)
        assert np.allclose(e, ref[:k], atol=1e-12)
        assert np.allclose(V.T @ V, np.eye(k), atol=1e-12)
        Hs = fock.explicit_hamiltonian(m, *sec)
        assert np.abs(Hs @ V - V * e[None, :]).max() < 1e-11
