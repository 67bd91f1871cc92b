"""Electron-phonon (Holstein) impurity (test infrastructure, FP64).

Sec. "Electron-phonon coupling": H = H_e + w0 b+b + sum_{a sigma} g_a
n_{a sigma} (b + b+) (one local mode, taken as printed: the density enters
without a shift), the phonon space truncated at N_ph quanta, D_ph = N_ph + 1.
A sector is an electronic sector times the phonon space; its index is
  i = i_e + p * D_up * D_dw       (phonon index slowest),
and eq. HephBuild gives
  H_S = 1_ph (x) H_e + (w0 N) (x) 1_e + (b + b+) (x) G_e,
with N = diag(0 .. N_ph) and G_e = diag(sum_a g_a (n_{a up} + n_{a dw})).
Model keys: "nph" (N_ph, 0 = no phonons), "w0", "g" ([norb]).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fock, green


def dph(model):
    return int(model.get("nph", 0)) + 1


def phonon_ops(nph):
    """b (annihilation, b|p> = sqrt(p)|p-1>) and the number operator on 0..nph."""
    d = nph + 1
    b = np.zeros((d, d))
    for p in range(1, d):
        b[p - 1, p] = np.sqrt(p)
    return b, np.diag(np.arange(d, dtype=float))


def coupling_diagonal(model, nup, ndw):
    """sum_a g_a (n_{a up} + n_{a dw}) in the electronic sector's order."""
    ns = fock.ns_of(model)
    _, _, I = fock.sector_states(ns, nup, ndw, model)
    occ = fock.occupations(I, ns)
    g = np.asarray(model.get("g", np.zeros(model["norb"])), float)
    d = np.zeros(I.size)
    for a in range(model["norb"]):
        d += g[a] * (occ[a] + occ[ns + a])
    return d


def explicit_hamiltonian(model, nup, ndw):
    """Sector matrix of eq. HephBuild (sparse), phonon index slowest."""
    He = fock.explicit_hamiltonian(model, nup, ndw)
    nph = int(model.get("nph", 0))
    b, N = phonon_ops(nph)
    Ge = sp.diags(coupling_diagonal(model, nup, ndw))
    Ie = sp.identity(He.shape[0], format="csr")
    Ip = sp.identity(nph + 1, format="csr")
    H = sp.kron(Ip, He) + float(model.get("w0", 0.0)) * sp.kron(sp.csr_matrix(N), Ie) + \
        sp.kron(sp.csr_matrix(b + b.T), Ge)
    return H.tocsr()


def hv_rows(model, nup, ndw, v, rows):
    """(H v)[rows] from the three terms of eq. HephBuild, for sectors too large
    for the explicit matrix: the electronic part row by row (fock.hv_rows on
    the row's phonon slice), the phonon terms from their definitions."""
    nph = int(model.get("nph", 0))
    De = len(fock.spin_basis(model, nup)) * len(fock.spin_basis(model, ndw))
    v = np.asarray(v, float)
    rows = np.asarray(rows, np.int64)
    p, ie = rows // De, rows % De
    out = np.zeros(rows.size)
    for q in np.unique(p):
        k = np.nonzero(p == q)[0]
        out[k] = fock.hv_rows(model, nup, ndw, v[q * De:(q + 1) * De], ie[k])
    gd = coupling_diagonal(model, nup, ndw)[ie]
    out += float(model.get("w0", 0.0)) * p * v[rows]
    lo = p > 0
    out[lo] += gd[lo] * np.sqrt(p[lo]) * v[rows[lo] - De]
    hi = p < nph
    out[hi] += gd[hi] * np.sqrt(p[hi] + 1) * v[rows[hi] + De]
    return out


def apply_operator(model, nup, ndw, psi, orb, spin, kind):
    """c+ / c of (orb, spin) on every phonon slice (the operator acts on the
    electrons only)."""
    D = dph(model)
    De = psi.size // D
    outs, tgt = [], None
    for q in range(D):
        tgt, phi = green.apply_operator(model, nup, ndw, psi[q * De:(q + 1) * De], orb, spin, kind)
        if phi.size == 0:
            return tgt, np.zeros(0)
        outs.append(phi)
    return tgt, np.concatenate(outs)


def lehmann_exact(model, nup, ndw, orb, spin, z):
    """T = 0 Lehmann sum over the e-ph sectors (dense)."""
    H0 = explicit_hamiltonian(model, nup, ndw).toarray()
    w0, V0 = np.linalg.eigh(H0)
    E0, psi = w0[0], V0[:, 0]
    G = np.zeros(len(z), dtype=complex)
    for kind, sgn in (("cdag", -1.0), ("c", +1.0)):
        tgt, phi = apply_operator(model, nup, ndw, psi, orb, spin, kind)
        if phi.size == 0:
            continue
        Ht = explicit_hamiltonian(model, *tgt).toarray()
        wt, Vt = np.linalg.eigh(Ht)
        amp2 = (Vt.T @ phi) ** 2
        G += (amp2[None, :] / (z[:, None] + sgn * (wt[None, :] - E0))).sum(axis=1)
    return G, E0
