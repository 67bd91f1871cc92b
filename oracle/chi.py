"""Density-type susceptibilities (test infrastructure, FP64).

Sec. 5 "Dynamical correlation functions" (eq. KLgf) with a bosonic operator:
the time ordering carries the minus sign, so for a Hermitian O
  C_O(z) = <O 1/(z - (H - E0)) O> - <O 1/(z + (H - E0)) O>
         = sum_m |<m|O|0>|^2 [1/(z - (E_m - E0)) - 1/(z + (E_m - E0))].
O is diagonal in the occupation basis and keeps the sector:
  O = sum_a (c_up[a] n_{a up} + c_dw[a] n_{a dw})
(spin: c_up = 1/2, c_dw = -1/2 on one orbital; charge: 1, 1; a cross-orbital
function follows from O = A + B as the paper describes).  Terms with
E_m = E0 contribute 1/z - 1/z = 0 at z != 0 and are dropped (also at z = 0,
the T = 0 limit); "E_m = E0" means within the ground-state degeneracy
threshold gs_threshold = 1e-9 of the input table (times max(1, |E0|)).
Bosonic Matsubara grid: nu_n = 2 n pi / beta.

``chi_exact`` sums over every eigenstate of the sector (dense).  ``chi_krylov``
is the Krylov form: start from O|psi0>, run N plain Lanczos steps in the same
sector, and use the eigenpairs (theta_m, first components u_m) of the
tridiagonal matrix:
  C(z) = |O psi0|^2 sum_m u_m^2 [1/(z - (theta_m - E0)) - 1/(z + (theta_m - E0))].
"""
from __future__ import annotations

import numpy as np

from . import fock, spectra

DROP_REL = 1e-9      # |E_m - E0| <= DROP_REL * max(1, |E0|): a zero-energy pole


def bosonic(beta, lmats):
    return 2 * np.arange(lmats) * np.pi / beta


def diag_operator(model, nup, ndw, coef_up, coef_dw):
    """Diagonal of O in the sector's index order."""
    ns = fock.ns_of(model)
    _, _, I = fock.sector_states(ns, nup, ndw, model)
    occ = fock.occupations(I, ns)               # [2 ns, D]
    d = np.zeros(I.size)
    for a in range(model["norb"]):
        d += coef_up[a] * occ[a] + coef_dw[a] * occ[ns + a]
    return d


def spectral(poles, weights, e0, z):
    """sum_m w_m [1/(z - d_m) - 1/(z + d_m)], d_m = poles - e0, zero poles dropped."""
    d = np.asarray(poles, float) - e0
    w = np.asarray(weights, float)
    keep = np.abs(d) > DROP_REL * max(1.0, abs(e0))
    d, w = d[keep], w[keep]
    z = np.asarray(z)[:, None]
    return (w[None, :] * (1.0 / (z - d[None, :]) - 1.0 / (z + d[None, :]))).sum(axis=1)


def chi_exact(model, nup, ndw, coef_up, coef_dw, z):
    H = fock.explicit_hamiltonian(model, nup, ndw).toarray()
    w, V = np.linalg.eigh(H)
    o = diag_operator(model, nup, ndw, coef_up, coef_dw)
    amp = V.T @ (o * V[:, 0])                   # <m|O|0>
    return spectral(w, amp ** 2, w[0], z), w[0]


def chi_krylov(model, nup, ndw, psi0, e0, coef_up, coef_dw, ngf, z, matvec):
    o = diag_operator(model, nup, ndw, coef_up, coef_dw)
    phi = o * np.asarray(psi0, float)
    wgt = float(phi @ phi)
    if wgt == 0.0:
        return np.zeros(len(z), dtype=complex), 0.0, (np.zeros(0), np.zeros(0))
    a, b = spectra.plain_lanczos(matvec, phi, ngf)
    th, U = spectra.tridiag_eigh(a, b)
    return spectral(th, wgt * U[0, :] ** 2, e0, z), wgt, (a, b)


def chi_thermal_states(model, states, coef_up, coef_dw, z, beta):
    """Thermal form: sum_n w_n C_n(z) over a list of (E, sec, psi), C_n the exact
    per-state function with E_n as reference, w_n normalised over the list."""
    e = np.array([t[0] for t in states])
    w = np.exp(-beta * (e - e.min()))
    w = w / w.sum()
    out = np.zeros(len(z), dtype=complex)
    for wn, (en, sec, psi) in zip(w, states):
        H = fock.explicit_hamiltonian(model, *sec).toarray()
        wm, V = np.linalg.eigh(H)
        o = diag_operator(model, sec[0], sec[1], coef_up, coef_dw)
        amp = V.T @ (o * np.asarray(psi, float))
        out += wn * spectral(wm, amp ** 2, en, z)
    return out


def chi_double_sum(model, sectors, coef_up, coef_dw, z, beta):
    """Textbook bosonic Lehmann double sum over every eigenstate of the listed
    sectors (O keeps the sector):
      C(z) = (1/Z) sum_{n,m} |<m|O|n>|^2 (e^{-beta E_n} - e^{-beta E_m}) / (z - (E_m - E_n)),
    pairs with |E_m - E_n| within the zero-pole threshold left out."""
    spec = []
    for sec in sectors:
        H = fock.explicit_hamiltonian(model, *sec).toarray()
        w, V = np.linalg.eigh(H)
        o = diag_operator(model, sec[0], sec[1], coef_up, coef_dw)
        spec.append((w, V.T @ (o[:, None] * V)))
    e0 = min(w[0] for w, _ in spec)
    Z = sum(np.exp(-beta * (w - e0)).sum() for w, _ in spec)
    out = np.zeros(len(z), dtype=complex)
    for w, M in spec:
        b = np.exp(-beta * (w - e0))
        d = w[:, None] - w[None, :]                       # E_m - E_n  [m, n]
        keep = np.abs(d) > DROP_REL * max(1.0, abs(e0))
        num = (M ** 2) * (b[None, :] - b[:, None])
        for k, zz in enumerate(z):
            out[k] += (num[keep] / (zz - d[keep])).sum()
    return out / Z
