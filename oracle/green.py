"""Impurity Green's function at T = 0 (test infrastructure, FP64).

Reading of eq. KLgf for fermions (the printed sign is inconsistent): both
terms enter with +, energies are measured from the ground energy E0:

  G(z) = sum_m |<m|c+|0>|^2 / (z - (E_m - E0)) + sum_m |<m|c|0>|^2 / (z + (E_m - E0)).

``lehmann_exact`` is that definition summed over every eigenstate of the
(N_up +- 1) sectors (dense diagonalisation, tiny sectors only).
``krylov_gf`` is the Krylov approximation of Sec. 6 "Dynamical correlation
functions": start from O+|psi0>/|O+|psi0>|, run N plain Lanczos steps, and use
the eigenpairs (theta_m, first components u_m) of the tridiagonal matrix as
poles and weights:
  G_p(z) = w_p sum_m u_m^2 / (z - (theta_m - E0)),
  G_h(z) = w_h sum_m u_m^2 / (z + (theta_m - E0)),
with w_p = |c+ psi0|^2, w_h = |c psi0|^2.
Matsubara grid (not defined in the paper): omega_n = (2n+1) pi / beta.
"""
from __future__ import annotations

import numpy as np

from . import fock, spectra


def matsubara(beta, lmats):
    return (2 * np.arange(lmats) + 1) * np.pi / beta


def apply_operator(model, nup, ndw, psi, orb, spin, kind):
    """phi = c+_{orb,spin} psi (kind='cdag') or c_{orb,spin} psi (kind='c').

    Computed on full 2Ns-bit strings with the full-string sign.  Returns
    ((nup', ndw'), phi) in the target sector's index order."""
    ns = fock.ns_of(model)
    m = orb + spin * ns
    d = 1 if kind == "cdag" else -1

    def shifted(spec):
        if np.ndim(spec) == 0:
            return spec + d
        t = list(spec)
        t[orb] += d                     # orbital-resolved: only orbital orb changes
        return tuple(t)

    tgt = (shifted(nup), ndw) if spin == 0 else (nup, shifted(ndw))
    bad = lambda spec: (np.ndim(spec) == 0 and not 0 <= spec <= ns) or \
        (np.ndim(spec) > 0 and not all(0 <= x <= model["nbath"] + 1 for x in spec))
    if bad(tgt[0]) or bad(tgt[1]):
        return tgt, np.zeros(0)
    up, dw, I = fock.sector_states(ns, nup, ndw, model)
    tup, tdw, _ = fock.sector_states(ns, *tgt, model)
    Dt = len(tup) * len(tdw)
    phi = np.zeros(Dt)
    if Dt == 0:
        return tgt, phi
    if kind == "cdag":
        valid, Inew, sgn = fock.apply_cdag(I, m)
    else:
        valid, Inew, sgn = fock.apply_c(I, m)
    j = np.nonzero(valid)[0]
    idx = fock._index_of(tup, tdw, ns, Inew[j])
    np.add.at(phi, idx, sgn[j] * np.asarray(psi, float)[j])
    return tgt, phi


def lehmann_exact(model, nup, ndw, orb, spin, z):
    """Exact T=0 Lehmann sum from dense diagonalisation of the three sectors."""
    H0 = fock.explicit_hamiltonian(model, nup, ndw).toarray()
    w0, V0 = np.linalg.eigh(H0)
    E0, psi = w0[0], V0[:, 0]
    G = np.zeros(len(z), dtype=complex)
    for kind, sgn in (("cdag", -1.0), ("c", +1.0)):
        tgt, phi = apply_operator(model, nup, ndw, psi, orb, spin, kind)
        if phi.size == 0:
            continue
        Ht = fock.explicit_hamiltonian(model, *tgt).toarray()
        wt, Vt = np.linalg.eigh(Ht)
        amp2 = (Vt.T @ phi) ** 2
        for Em, a2 in zip(wt, amp2):
            G += a2 / (z + sgn * (Em - E0))
    return G, E0


def gf_from_coeffs(alpha, beta, weight, e0, z, particle):
    """Spectral form of one Krylov branch from its tridiagonal coefficients."""
    if weight == 0.0 or len(alpha) == 0:
        return np.zeros(len(z), dtype=complex)
    th, U = spectra.tridiag_eigh(alpha, beta)
    u2 = U[0, :] ** 2
    s = -1.0 if particle else 1.0
    return weight * (u2[None, :] / (z[:, None] + s * (th[None, :] - e0))).sum(axis=1)


def krylov_gf(model, nup, ndw, psi0, e0, orb, spin, ngf, z, matvec_factory):
    """Krylov Green's function.  ``matvec_factory(nup, ndw)`` returns H.v for a
    sector.  Returns (G, w_p, w_h, (alpha_p, beta_p), (alpha_h, beta_h))."""
    out = np.zeros(len(z), dtype=complex)
    info = {}
    for kind in ("cdag", "c"):
        tgt, phi = apply_operator(model, nup, ndw, psi0, orb, spin, kind)
        w = float(phi @ phi) if phi.size else 0.0
        if w > 0.0:
            a, b = spectra.plain_lanczos(matvec_factory(*tgt), phi, ngf)
        else:
            a, b = np.zeros(0), np.zeros(0)
        out += gf_from_coeffs(a, b, w, e0, z, particle=(kind == "cdag"))
        info[kind] = (w, a, b)
    return out, info["cdag"][0], info["c"][0], info["cdag"][1:], info["c"][1:]
