"""Several low-lying states and finite temperature (test infrastructure, FP64).

Sec. 6 "Eigenspace class": the solver keeps an ordered list of eigenstates
(energy, vector, quantum numbers).  At T = 0 only ground states enter; at
T > 0 each sector contributes its lanc_nstates_sector lowest states, the list
holds at most lanc_nstates_total of them, and it is truncated to the states
whose Boltzmann factor exp(-beta (E_i - E_0)) is not below `cutoff` (the
printed inequality reads the other way round; a truncation that kept only
the negligible states would be pointless, so it is read as "drop the states
below the cutoff").  Annealing over successive diagonalisations: a sector all
of whose computed states survived asks for nstates_step more next time, any
other sector is cut back to the number it kept (at least one, so that a
sector whose ground state later moves into the window is still seen).

Sec. 6 "Dynamical correlation functions" (thermal form): with the kept
states |n>, weights w_n = exp(-beta (E_n - E_0)) / Z, Z = sum of the kept
factors,
  G(z) = sum_n w_n G_n(z),
  G_n(z) = sum_m |<m|c+|n>|^2 / (z - (E_m - E_n)) + |<m|c|n>|^2 / (z + (E_m - E_n)),
both terms with + for fermions (as at T = 0).  ``green_states_exact`` is that
sum with every G_n taken exactly from the neighbouring sectors' spectra;
``green_double_sum`` is the textbook Lehmann double sum over all eigenstates
of a closed set of sectors,
  G(z) = (1/Z) sum_{n,m} |<m|c+|n>|^2 (exp(-beta E_n) + exp(-beta E_m)) / (z - (E_m - E_n)),
an independent expression the per-state form must reproduce when every state
is kept.
"""
from __future__ import annotations

import math

import numpy as np

from . import fock, green


def sector_spectrum(model, sec):
    """All eigenpairs of one sector (dense)."""
    H = fock.explicit_hamiltonian(model, *sec).toarray()
    return np.linalg.eigh(H)


def lowest_states(model, sec, k):
    """The k lowest eigenpairs of a sector (dense; k clipped to the dimension)."""
    w, V = sector_spectrum(model, sec)
    k = min(k, len(w))
    return w[:k], V[:, :k]


def boltzmann(energies, beta, e0=None):
    """exp(-beta (E - E0)), E0 = min(E) unless given."""
    e = np.asarray(energies, float)
    if e0 is None:
        e0 = e.min()
    return np.exp(-beta * (e - e0))


def espace_select(entries, beta, cutoff, ntotal):
    """Truncation of the eigenstate list (Sec. 6 "Eigenspace class").

    entries: list of (E, sector_index, state_index).  Sorted by energy (ties:
    sector, then state index); the states with exp(-beta (E - E0)) >= cutoff
    are kept, at most ntotal of them (the lowest)."""
    if not entries:
        return []
    ent = sorted(entries, key=lambda t: (t[0], t[1], t[2]))
    e0 = ent[0][0]
    kept = [t for t in ent if math.exp(-beta * (t[0] - e0)) >= cutoff]
    return kept[:ntotal]


def anneal(nstates, computed, kept, step):
    """Next per-sector state counts: +step where every computed state was kept,
    else the number kept (at least 1)."""
    out = []
    for n, c, k in zip(nstates, computed, kept):
        out.append(n + step if (c > 0 and k == c) else max(1, k))
    return out


def green_state(model, sec, psi, e, orb, spin, z):
    """G_n(z) of one eigenstate |n> (energy e) of sector `sec`, exact over the
    neighbouring sectors."""
    G = np.zeros(len(z), dtype=complex)
    for kind, sgn in (("cdag", -1.0), ("c", +1.0)):
        tgt, phi = green.apply_operator(model, sec[0], sec[1], psi, orb, spin, kind)
        if phi.size == 0 or not np.any(phi):
            continue
        wt, Vt = sector_spectrum(model, tgt)
        amp2 = (Vt.T @ phi) ** 2
        G += (amp2[None, :] / (z[:, None] + sgn * (wt[None, :] - e))).sum(axis=1)
    return G


def green_states_exact(model, states, orb, spin, z, beta):
    """Thermal G from a list of (E, sec, psi): sum_n w_n G_n (weights
    normalised over the list)."""
    e = np.array([s[0] for s in states])
    w = boltzmann(e, beta)
    w = w / w.sum()
    G = np.zeros(len(z), dtype=complex)
    for wn, (en, sec, psi) in zip(w, states):
        G += wn * green_state(model, sec, psi, en, orb, spin, z)
    return G


def all_sectors(model):
    """Every (N_up, N_dw) sector of the model (the whole Fock space)."""
    ns = fock.ns_of(model)
    return [(a, b) for a in range(ns + 1) for b in range(ns + 1)]


def all_states(model, sectors=None):
    """(E, sec, psi) of every eigenstate of the listed sectors."""
    out = []
    for sec in sectors or all_sectors(model):
        w, V = sector_spectrum(model, sec)
        for k in range(len(w)):
            out.append((w[k], sec, V[:, k]))
    return out


def green_double_sum(model, orb, spin, z, beta):
    """Textbook Lehmann double sum over every eigenstate of the whole Fock space
    (closed under c and c+): matrix elements of c+ between the eigenstates of
    sectors (N_up, N_dw) and their neighbours."""
    ns = fock.ns_of(model)
    spec = {sec: sector_spectrum(model, sec) for sec in all_sectors(model)}
    e0 = min(w[0] for w, _ in spec.values())
    Z = sum(np.exp(-beta * (w - e0)).sum() for w, _ in spec.values())
    G = np.zeros(len(z), dtype=complex)
    for sec, (wn, Vn) in spec.items():
        tgt = (sec[0] + 1, sec[1]) if spin == 0 else (sec[0], sec[1] + 1)
        if tgt[0] > ns or tgt[1] > ns:
            continue
        wm, Vm = spec[tgt]
        # <m|c+|n> for all n (columns of Vn) and m (columns of Vm)
        M = np.zeros((len(wm), len(wn)))
        for k in range(len(wn)):
            t2, phi = green.apply_operator(model, sec[0], sec[1], Vn[:, k], orb, spin, "cdag")
            assert tuple(t2) == tgt
            M[:, k] = Vm.T @ phi
        bn = np.exp(-beta * (wn - e0))
        bm = np.exp(-beta * (wm - e0))
        num = (M ** 2) * (bn[None, :] + bm[:, None])               # [m, n]
        den = z[:, None, None] - (wm[None, :, None] - wn[None, None, :])
        G += (num[None, :, :] / den).sum(axis=(1, 2))
    return G / Z
