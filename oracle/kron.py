"""Second oracle form: H = H_d + H_up (x) 1 + 1 (x) H_dw with SciPy sparse factors.

Oracle (test infrastructure).  This is the decomposition of eq. Hdecomp /
eq. Hbuild written with library sparse products, used only where the explicit
sector matrix of ``fock.explicit_hamiltonian`` is too large to store.  It is
pinned to the explicit matrix entry for entry on small sectors
(tests/test_oracle_hamiltonian.py).

Vector layout: v[i_up + i_dw * D_up]; as a matrix M[i_dw, i_up] (row-major
reshape) the spin-up operator acts on the second index and the spin-down
operator on the first (eq. Vmatrix is the transpose of this view).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fock


def spin_hamiltonian(model, n, spin):
    """Hopping operator of one spin species on its D_sigma strings (CSR)."""
    off, col, sgn, amp = fock.spin_hop_csr(model, n, spin)
    D = len(off) - 1
    rows = np.repeat(np.arange(D), np.diff(off))
    return sp.csr_matrix((amp * sgn, (rows, col)), shape=(D, D))


def spin_diagonal(model, n):
    """E_sigma[s]: one-body energy plus same-spin inter-orbital interaction of a
    single spin string, and p[s]: the impurity occupation pattern (bits 0..norb-1)."""
    ns, norb = fock.ns_of(model), model["norb"]
    strings = fock.spin_strings(ns, n)
    occ = ((strings[None, :] >> np.arange(ns, dtype=np.uint64)[:, None]) & np.uint64(1)).astype(float)
    e = fock.level_energies(model)
    E = (e[:, None] * occ).sum(axis=0)
    for a in range(norb):
        for b in range(a + 1, norb):
            E += (model["Ust"] - model["Jh"]) * occ[a] * occ[b]
    p = (strings & np.uint64((1 << norb) - 1)).astype(np.int64)
    return E, p


def pattern_interaction(model):
    """W[p, q] = U sum_a p_a q_a + U' sum_{a != b} p_a q_b for impurity patterns."""
    norb = model["norb"]
    P = 1 << norb
    W = np.zeros((P, P))
    for p in range(P):
        for q in range(P):
            pb = [(p >> a) & 1 for a in range(norb)]
            qb = [(q >> a) & 1 for a in range(norb)]
            w = 0.0
            for a in range(norb):
                w += model["U"] * pb[a] * qb[a]
                for b in range(norb):
                    if a != b:
                        w += model["Ust"] * pb[a] * qb[b]
            W[p, q] = w
    return W


class KronH:
    """Matrix-free H for one sector built from the per-spin factors."""

    def __init__(self, model, nup, ndw):
        if model.get("Jx", 0.0) != 0.0 or model.get("Jp", 0.0) != 0.0:
            # spin exchange and pair hopping move electrons of both spins at once:
            # not a Kronecker sum (use fock.explicit_hamiltonian / hv_rows)
            raise ValueError("KronH covers the density-density interaction only")
        self.Hup = spin_hamiltonian(model, nup, 0)
        self.Hdw = spin_hamiltonian(model, ndw, 1)
        Eu, pu = spin_diagonal(model, nup)
        Ed, pd = spin_diagonal(model, ndw)
        W = pattern_interaction(model)
        self.Dup, self.Ddw = len(Eu), len(Ed)
        self.dim = self.Dup * self.Ddw
        # Hd as a (D_dw, D_up) matrix
        self.Hd = Ed[:, None] + Eu[None, :] + W[pu[None, :], pd[:, None]]

    def matvec(self, v):
        M = np.asarray(v, dtype=np.float64).reshape(self.Ddw, self.Dup)
        out = self.Hd * M
        out += (self.Hup @ M.T).T
        out += self.Hdw @ M
        return out.ravel()

    def diagonal(self):
        return self.Hd.ravel().copy()
