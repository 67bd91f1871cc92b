"""Closed forms that pin the oracle (test infrastructure, FP64).

* Non-interacting limit (U = U' = J = 0): the Hamiltonian of eq. Ham1 is a
  quadratic form h (Ns x Ns per spin, star geometry impurity-bath).  The sector
  ground energy is the sum of the N_up lowest plus the N_dw lowest eigenvalues
  of h, and the impurity Green's function is the Dyson form
  G(z) = 1 / (z - e_imp - sum_nu V_nu^2 / (z - eps_nu)) with e_imp = eps_imp - xmu.
* Atomic limit (V = 0): impurity and bath decouple; the ground energy is the
  minimum over impurity occupation patterns of the impurity energy plus the
  sum of the lowest bath levels filled by the remaining electrons.
"""
from __future__ import annotations

from itertools import product

import numpy as np

from . import fock


def onebody_matrix(model):
    ns = fock.ns_of(model)
    h = np.diag(fock.level_energies(model))
    for (a, b, V) in fock.hop_pairs(model):
        h[a, b] = h[b, a] = V
    return h


def e0_noninteracting(model, nup, ndw):
    e = np.linalg.eigvalsh(onebody_matrix(model))
    return float(e[:nup].sum() + e[:ndw].sum())


def g_noninteracting(model, orb, z):
    norb, nbath = model["norb"], model["nbath"]
    e_imp = float(np.asarray(model["eps_imp"])[orb]) - model["xmu"]
    eb = np.asarray(model["eps_bath"]).reshape(norb, nbath)[orb]
    V = np.asarray(model["vhyb"]).reshape(norb, nbath)[orb]
    delta = (V[None, :] ** 2 / (z[:, None] - eb[None, :])).sum(axis=1)
    return 1.0 / (z - e_imp - delta)


def e0_atomic(model, nup, ndw):
    norb, nbath = model["norb"], model["nbath"]
    e_imp = np.asarray(model["eps_imp"], float) - model["xmu"]
    bath = np.sort(np.asarray(model["eps_bath"], float).ravel())
    U, Ust, J = model["U"], model["Ust"], model["Jh"]
    best = np.inf
    for pu in product((0, 1), repeat=norb):
        for pd in product((0, 1), repeat=norb):
            ku, kd = nup - sum(pu), ndw - sum(pd)
            if not (0 <= ku <= norb * nbath and 0 <= kd <= norb * nbath):
                continue
            e = sum(e_imp[a] * (pu[a] + pd[a]) for a in range(norb))
            e += sum(U * pu[a] * pd[a] for a in range(norb))
            e += sum(Ust * pu[a] * pd[b] for a in range(norb) for b in range(norb) if a != b)
            e += sum((Ust - J) * (pu[a] * pu[b] + pd[a] * pd[b])
                     for a in range(norb) for b in range(a + 1, norb))
            e += bath[:ku].sum() + bath[:kd].sum()
            best = min(best, e)
    return float(best)
