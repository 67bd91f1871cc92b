"""Density-type susceptibilities (test infrastructure, FP64).

Sec. 6 "Dynamical correlation functions" (eq. KLgf) with a bosonic operator:
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

The paper also names excitonic and pair susceptibilities.  Here:
  * excitonic (orbitals a != b): O = sum_sigma (c+_{a sigma} c_{b sigma} +
    c+_{b sigma} c_{a sigma}), Hermitian and within the sector, so the same
    form as above;
  * pair (orbital a): O = c_{a dw} c_{a up}, which leaves the sector: with the
    bosonic sign of eq. KLgf,
      C(z) = <O 1/(z - (H - E0)) O+> - <O+ 1/(z + (H - E0)) O>
           = sum_m |<m|O+|0>|^2 / (z - (E_m - E0))        (m in N_up+1, N_dw+1)
             - sum_m |<m|O|0>|^2 / (z + (E_m - E0))       (m in N_up-1, N_dw-1).
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


def _apply_ops(model, nup, ndw, psi, ops, tgt):
    """phi = (product of ops, rightmost first) psi into sector tgt (full-string
    signs); ops as (mode, creator?) left to right."""
    ns = fock.ns_of(model)
    up, dw, I = fock.sector_states(ns, nup, ndw, model)
    tup, tdw, _ = fock.sector_states(ns, tgt[0], tgt[1], model)
    phi = np.zeros(len(tup) * len(tdw))
    if phi.size == 0:
        return phi
    valid, Inew, sgn = fock.apply_product(I, ops)
    j = np.nonzero(valid)[0]
    idx = fock._index_of(tup, tdw, ns, Inew[j])
    np.add.at(phi, idx, sgn[j] * np.asarray(psi, float)[j])
    return phi


def exciton_apply(model, nup, ndw, psi, a, b):
    """O psi for O = sum_sigma (c+_a c_b + c+_b c_a) on both spins."""
    ns = fock.ns_of(model)
    out = np.zeros(np.asarray(psi).size)
    for sg in (0, 1):
        ma, mb = a + sg * ns, b + sg * ns
        for (x, y) in ((ma, mb), (mb, ma)):
            out += _apply_ops(model, nup, ndw, psi, [(x, True), (y, False)], (nup, ndw))
    return out


def chi_exciton_exact(model, nup, ndw, a, b, z):
    H = fock.explicit_hamiltonian(model, nup, ndw).toarray()
    w, V = np.linalg.eigh(H)
    amp = V.T @ exciton_apply(model, nup, ndw, V[:, 0], a, b)
    return spectral(w, amp ** 2, w[0], z), w[0]


def _shift(spec, d, a):
    if np.ndim(spec) == 0:
        return int(spec) + d
    t = list(spec)
    t[a] += d
    return tuple(t)


def _valid(model, spec):
    if np.ndim(spec) == 0:
        return 0 <= spec <= fock.ns_of(model)
    return all(0 <= x <= model["nbath"] + 1 for x in spec)


def pair_apply(model, nup, ndw, psi, a, create):
    """O+ psi = c+_{a up} c+_{a dw} psi (create) or O psi = c_{a dw} c_{a up} psi;
    returns (target sector, phi) or (target, empty) when it does not exist."""
    ns = fock.ns_of(model)
    d = 1 if create else -1
    tgt = (_shift(nup, d, a), _shift(ndw, d, a))
    if not (_valid(model, tgt[0]) and _valid(model, tgt[1])):
        return tgt, np.zeros(0)
    ops = [(a, True), (a + ns, True)] if create else [(a + ns, False), (a, False)]
    return tgt, _apply_ops(model, nup, ndw, psi, ops, tgt)


def chi_pair_exact(model, nup, ndw, a, z):
    """Pair susceptibility at T = 0 from the dense spectra of the three sectors."""
    H = fock.explicit_hamiltonian(model, nup, ndw).toarray()
    w0, V0 = np.linalg.eigh(H)
    E0, psi = w0[0], V0[:, 0]
    out = np.zeros(len(z), dtype=complex)
    for create, sgn in ((True, -1.0), (False, +1.0)):
        tgt, phi = pair_apply(model, nup, ndw, psi, a, create)
        if phi.size == 0:
            continue
        wt, Vt = np.linalg.eigh(fock.explicit_hamiltonian(model, *tgt).toarray())
        amp2 = (Vt.T @ phi) ** 2
        term = (amp2[None, :] / (np.asarray(z)[:, None] + sgn * (wt[None, :] - E0))).sum(axis=1)
        out += term if create else -term
    return out, E0


def exciton_state(model, sec, psi, e, a, b, z):
    """T = 0 excitonic function of one eigenstate (energy e) of sector sec."""
    H = fock.explicit_hamiltonian(model, *sec).toarray()
    w, V = np.linalg.eigh(H)
    amp = V.T @ exciton_apply(model, sec[0], sec[1], psi, a, b)
    return spectral(w, amp ** 2, e, z)


def pair_state(model, sec, psi, e, a, z):
    """Pair function of one eigenstate (energy e): both branches, no pole dropped."""
    out = np.zeros(len(z), dtype=complex)
    for create, sgn in ((True, -1.0), (False, +1.0)):
        tgt, phi = pair_apply(model, sec[0], sec[1], psi, a, create)
        if phi.size == 0:
            continue
        wt, Vt = np.linalg.eigh(fock.explicit_hamiltonian(model, *tgt).toarray())
        amp2 = (Vt.T @ phi) ** 2
        term = (amp2[None, :] / (np.asarray(z)[:, None] + sgn * (wt[None, :] - e))).sum(axis=1)
        out += term if create else -term
    return out


def thermal_states_sum(states, beta, per_state):
    """sum_n w_n C_n over (E, sec, psi) with w_n normalised over the list;
    per_state(sec, psi, e) gives C_n."""
    e = np.array([t[0] for t in states])
    w = np.exp(-beta * (e - e.min()))
    w = w / w.sum()
    return sum(wn * per_state(sec, psi, en) for wn, (en, sec, psi) in zip(w, states))


def pair_double_sum(model, sectors, a, z, beta):
    """Bosonic Lehmann double sum of the pair operator O = c_{a dw} c_{a up} over
    every eigenstate of a set of sectors closed under O and O+:
      C(z) = (1/Z) sum_{n,m} |<m|O+|n>|^2 (e^{-beta E_n} - e^{-beta E_m}) / (z - (E_m - E_n))."""
    spec = {}
    for sec in sectors:
        H = fock.explicit_hamiltonian(model, *sec).toarray()
        spec[sec] = np.linalg.eigh(H)
    e0 = min(w[0] for w, _ in spec.values())
    Z = sum(np.exp(-beta * (w - e0)).sum() for w, _ in spec.values())
    out = np.zeros(len(z), dtype=complex)
    for sec, (wn, Vn) in spec.items():
        tgt = (sec[0] + 1, sec[1] + 1)
        if tgt not in spec:
            continue
        wm, Vm = spec[tgt]
        M = np.zeros((len(wm), len(wn)))
        for k in range(len(wn)):
            t2, phi = pair_apply(model, sec[0], sec[1], Vn[:, k], a, True)
            M[:, k] = Vm.T @ phi
        bn = np.exp(-beta * (wn - e0))
        bm = np.exp(-beta * (wm - e0))
        num = (M ** 2) * (bn[None, :] - bm[:, None])
        d = wm[:, None] - wn[None, :]
        for q, zz in enumerate(z):
            out[q] += (num / (zz - d)).sum()
    return out / Z
