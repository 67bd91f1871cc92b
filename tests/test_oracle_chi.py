"""Oracle pins for the density-type susceptibilities (eq. KLgf with the bosonic
sign, O diagonal in the occupation basis).

  * the sector form equals a Jordan-Wigner build on the whole Fock space
    (O from the number operators, the ground state of the sector embedded in
    the Fock space), for spin and charge operators, and a flipped bosonic sign
    is caught;
  * U = 0: the charge susceptibility of one orbital and spin is the bubble of
    the one-body eigenvectors (occupied -> empty transitions);
  * the Krylov form equals the exact sum once the Krylov space is exhausted;
  * chi(i nu) is real and positive-definite in the sense -C(i nu) >= 0 and
    decreases with nu (a sum of 2 d / (nu^2 + d^2) terms);
  * finite temperature: the per-state thermal sum over every eigenstate equals
    the textbook bosonic double sum;
  * excitonic and pair functions against Jordan-Wigner builds on the whole
    Fock space and against U = 0 closed forms (particle-hole and
    particle-particle bubbles of the one-body eigenvectors).
"""
import numpy as np
import pytest

from oracle import chi, closed, fock, jw
from paper_2105_06806_amd import inputs


def _jw_chi(model, sec, cu, cd, z):
    ns = fock.ns_of(model)
    H, c = jw.fock_hamiltonian(model)
    n = [c[m].T @ c[m] for m in range(2 * ns)]
    O = sum(cu[a] * n[a] + cd[a] * n[ns + a] for a in range(model["norb"]))
    _, _, I = fock.sector_states(ns, *sec)
    idx = I.astype(np.int64)
    w0, V0 = np.linalg.eigh(H[np.ix_(idx, idx)])
    psi = np.zeros(H.shape[0])
    psi[idx] = V0[:, 0]
    w, V = np.linalg.eigh(H)
    amp = V.T @ (O @ psi)
    return chi.spectral(w, amp ** 2, w0[0], z)


@pytest.mark.parametrize("kind", ["spin", "charge"])
@pytest.mark.parametrize("norb,nbath,sec,orb", [(1, 3, (2, 2), 0), (2, 1, (2, 1), 1)])
def test_sector_form_equals_jordan_wigner(kind, norb, nbath, sec, orb):
    m = inputs.make_model(norb, nbath, 2.5, Jh=0.3, seed=81 + norb, symmetric=False)
    cu = np.zeros(norb)
    cd = np.zeros(norb)
    cu[orb], cd[orb] = (0.5, -0.5) if kind == "spin" else (1.0, 1.0)
    z = 1j * chi.bosonic(5.0, 12)
    got, _ = chi.chi_exact(m, *sec, cu, cd, z)
    ref = _jw_chi(m, sec, cu, cd, z)
    assert np.abs(got - ref).max() < 1e-12
    assert np.abs(got.imag).max() < 1e-12
    assert np.all(got.real <= 1e-14) and np.all(np.diff(got.real) >= -1e-14)


def test_flipped_bosonic_sign_is_caught(monkeypatch):
    m = inputs.make_model(1, 3, 2.0, seed=84, symmetric=False)
    z = 1j * chi.bosonic(4.0, 6)
    ref = _jw_chi(m, (2, 2), [0.5], [-0.5], z)

    def wrong(poles, weights, e0, zz):
        d = np.asarray(poles) - e0
        keep = np.abs(d) > 1e-10
        d, w = d[keep], np.asarray(weights)[keep]
        return (w[None, :] * (1 / (zz[:, None] - d) + 1 / (zz[:, None] + d))).sum(axis=1)
    monkeypatch.setattr(chi, "spectral", wrong)
    got, _ = chi.chi_exact(m, 2, 2, [0.5], [-0.5], z)
    assert np.abs(got - ref).max() > 1e-3


def test_noninteracting_bubble():
    """U = 0, one spin: C_{n n}(z) = sum_{k occ, l empty} |phi_k(0) phi_l(0)|^2
    [1/(z - (e_l - e_k)) - 1/(z + (e_l - e_k))]."""
    m = inputs.make_model(1, 4, 0.0, seed=85, symmetric=False, eps_imp=0.2)
    ns = fock.ns_of(m)
    nup, ndw = 2, 3
    e, U = np.linalg.eigh(closed.onebody_matrix(m))
    z = 1j * chi.bosonic(6.0, 10)
    got, _ = chi.chi_exact(m, nup, ndw, [1.0], [0.0], z)
    ref = np.zeros(len(z), dtype=complex)
    for k in range(nup):
        for l in range(nup, ns):
            w = (U[0, k] * U[0, l]) ** 2
            d = e[l] - e[k]
            ref += w * (1 / (z - d) - 1 / (z + d))
    assert np.abs(got - ref).max() < 1e-12


def test_krylov_exhausted_equals_exact():
    m = inputs.make_model(2, 1, 2.5, Jh=0.4, seed=86, symmetric=False)
    sec = (2, 2)
    H = fock.explicit_hamiltonian(m, *sec)
    w, V = np.linalg.eigh(H.toarray())
    z = 1j * chi.bosonic(8.0, 16)
    cu, cd = [0.5, 0.0], [-0.5, 0.0]
    ref, _ = chi.chi_exact(m, *sec, cu, cd, z)
    got, wgt, _ = chi.chi_krylov(m, *sec, V[:, 0], w[0], cu, cd, H.shape[0], z, lambda x: H @ x)
    assert np.abs(got - ref).max() < 1e-9 * np.abs(ref).max()


def test_thermal_per_state_equals_double_sum():
    from oracle import thermal
    m = inputs.make_model(1, 3, 2.0, seed=87, symmetric=False)
    secs = thermal.all_sectors(m)
    beta = 3.0
    z = 1j * chi.bosonic(beta, 10)
    cu, cd = [0.5], [-0.5]
    got = chi.chi_thermal_states(m, thermal.all_states(m), cu, cd, z, beta)
    ref = chi.chi_double_sum(m, secs, cu, cd, z, beta)
    assert np.abs(got - ref).max() < 1e-12


def _jw_general(model, sec, O, z, bosonic_pair=False):
    """sum over every Fock eigenstate m of the sector ground state |0> embedded
    in the Fock space: |<m|O+|0>|^2/(z - d) - |<m|O|0>|^2/(z + d) (pair), or the
    Hermitian form with O."""
    ns = fock.ns_of(model)
    H, c = jw.fock_hamiltonian(model)
    _, _, I = fock.sector_states(ns, *sec)
    idx = I.astype(np.int64)
    w0, V0 = np.linalg.eigh(H[np.ix_(idx, idx)])
    psi = np.zeros(H.shape[0])
    psi[idx] = V0[:, 0]
    w, V = np.linalg.eigh(H)
    if not bosonic_pair:
        amp = V.T @ (O @ psi)
        return chi.spectral(w, amp ** 2, w0[0], z)
    ap = (V.T @ (O.T @ psi)) ** 2
    ah = (V.T @ (O @ psi)) ** 2
    d = w - w0[0]
    zz = np.asarray(z)[:, None]
    kp, kh = ap > 1e-28, ah > 1e-28                  # states the operator reaches
    return (ap[kp][None, :] / (zz - d[kp][None, :])).sum(axis=1) - \
        (ah[kh][None, :] / (zz + d[kh][None, :])).sum(axis=1)


@pytest.mark.parametrize("sec", [(2, 1), (2, 2), (1, 3)])
def test_exciton_and_pair_equal_jordan_wigner(sec):
    m = inputs.make_model(2, 1, 2.5, Jh=0.4, seed=88, symmetric=False)
    ns = fock.ns_of(m)
    z = 1j * chi.bosonic(5.0, 10)
    _, c = jw.fock_hamiltonian(m)
    cd = [x.T for x in c]
    Oe = sum(cd[0 + s * ns] @ c[1 + s * ns] + cd[1 + s * ns] @ c[0 + s * ns] for s in (0, 1))
    got, _ = chi.chi_exciton_exact(m, *sec, 0, 1, z)
    assert np.abs(got - _jw_general(m, sec, Oe, z)).max() < 1e-12
    for a in (0, 1):
        Op = c[a + ns] @ c[a]                        # c_{a dw} c_{a up}
        got, _ = chi.chi_pair_exact(m, *sec, a, z)
        ref = _jw_general(m, sec, Op, z, bosonic_pair=True)
        assert np.abs(got - ref).max() < 1e-12, a


def test_pair_and_exciton_noninteracting_bubbles():
    m = inputs.make_model(2, 2, 0.0, Jh=0.0, Ust=0.0, seed=89, symmetric=False, eps_imp=0.15)
    ns = fock.ns_of(m)
    nup, ndw = 3, 2
    e, U = np.linalg.eigh(closed.onebody_matrix(m))
    z = 1j * chi.bosonic(6.0, 8)
    # pair of orbital 0: add up in l >= nup and down in k >= ndw, or remove from occupied
    ref = np.zeros(len(z), dtype=complex)
    for l in range(nup, ns):
        for k in range(ndw, ns):
            ref += (U[0, l] * U[0, k]) ** 2 / (z - (e[l] + e[k]))
    for l in range(nup):
        for k in range(ndw):
            ref -= (U[0, l] * U[0, k]) ** 2 / (z + (-e[l] - e[k]))
    got, _ = chi.chi_pair_exact(m, nup, ndw, 0, z)
    assert np.abs(got - ref).max() < 1e-12
    # exciton 0-1: particle-hole pairs of each spin
    ref = np.zeros(len(z), dtype=complex)
    for n in (nup, ndw):
        for k in range(n):
            for l in range(n, ns):
                amp = U[0, l] * U[1, k] + U[1, l] * U[0, k]
                d = e[l] - e[k]
                ref += amp ** 2 * (1 / (z - d) - 1 / (z + d))
    got, _ = chi.chi_exciton_exact(m, nup, ndw, 0, 1, z)
    assert np.abs(got - ref).max() < 1e-12


def test_thermal_pair_per_state_equals_double_sum():
    """Pair function at finite temperature: the per-state sum over every
    eigenstate of the Fock space equals the bosonic double sum (z != 0)."""
    from oracle import thermal
    m = inputs.make_model(1, 2, 2.0, seed=90, symmetric=False)
    secs = thermal.all_sectors(m)
    beta = 2.5
    z = 1j * chi.bosonic(beta, 8)[1:]
    got = chi.thermal_states_sum(thermal.all_states(m), beta,
                                 lambda sec, psi, e: chi.pair_state(m, sec, psi, e, 0, z))
    ref = chi.pair_double_sum(m, secs, 0, z, beta)
    assert np.abs(got - ref).max() < 1e-12


def test_thermal_exciton_per_state_equals_double_sum():
    from oracle import thermal
    m = inputs.make_model(2, 1, 2.0, Jh=0.3, seed=91, symmetric=False)
    beta = 2.0
    z = 1j * chi.bosonic(beta, 8)[1:]
    states = thermal.all_states(m)
    got = chi.thermal_states_sum(states, beta,
                                 lambda sec, psi, e: chi.exciton_state(m, sec, psi, e, 0, 1, z))
    # double sum with the Hermitian exciton operator, sector by sector
    e0 = min(s[0] for s in states)
    Z = sum(np.exp(-beta * (s[0] - e0)) for s in states)
    ref = np.zeros(len(z), dtype=complex)
    for sec in thermal.all_sectors(m):
        H = fock.explicit_hamiltonian(m, *sec).toarray()
        w, V = np.linalg.eigh(H)
        M = np.column_stack([V.T @ chi.exciton_apply(m, sec[0], sec[1], V[:, k], 0, 1)
                             for k in range(len(w))])
        b = np.exp(-beta * (w - e0))
        d = w[:, None] - w[None, :]
        keep = np.abs(d) > 1e-9
        num = M ** 2 * (b[None, :] - b[:, None])
        for q, zz in enumerate(z):
            ref[q] += (num[keep] / (zz - d[keep])).sum()
    assert np.abs(got - ref / Z).max() < 1e-12
