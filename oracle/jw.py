"""Jordan-Wigner Fock-space operators for tiny systems (test infrastructure).

An independent construction of the Hamiltonian: each annihilator is a
Kronecker product of 2x2 matrices, c_m = Z (x) ... (x) Z (x) a (x) 1 (x) ... (x) 1
with the Z string on every mode ordered before m (Sec. 2.3), so the
anticommutation relations hold by construction.  H of eq. Ham1 is assembled
by matrix products over the whole 4**Ns Fock space and then restricted to a
sector.  Only for Ns <= 5.
"""
from __future__ import annotations

from functools import reduce

import numpy as np

from . import fock

_A = np.array([[0.0, 1.0], [0.0, 0.0]])     # |1> -> |0>, basis (|0>, |1>)
_Z = np.diag([1.0, -1.0])
_I2 = np.eye(2)


def annihilator(m, nmodes):
    """c_m on the Fock space with basis index I = sum_k n_k 2**k.

    np.kron puts its first factor on the most significant bit, so factors are
    listed from mode nmodes-1 down to mode 0."""
    facs = []
    for k in range(nmodes - 1, -1, -1):
        facs.append(_I2 if k > m else (_A if k == m else _Z))
    return reduce(np.kron, facs)


def fock_hamiltonian(model):
    ns = fock.ns_of(model)
    M = 2 * ns
    c = [annihilator(m, M) for m in range(M)]
    cd = [x.T for x in c]
    n = [cd[m] @ c[m] for m in range(M)]
    e = fock.level_energies(model)
    H = np.zeros((2 ** M, 2 ** M))
    for s in (0, 1):
        for k in range(ns):
            H += e[k] * n[k + s * ns]
        for (a, b, V) in fock.hop_pairs(model):
            H += V * (cd[a + s * ns] @ c[b + s * ns] + cd[b + s * ns] @ c[a + s * ns])
    norb = model["norb"]
    for a in range(norb):
        H += model["U"] * n[a] @ n[ns + a]
        for b in range(norb):
            if a != b:
                H += model["Ust"] * n[a] @ n[ns + b]
        for b in range(a + 1, norb):
            H += (model["Ust"] - model["Jh"]) * (n[a] @ n[b] + n[ns + a] @ n[ns + b])
    # spin exchange and pair hopping (eq. Ham1), products of the matrices above
    jx, jp = model.get("Jx", 0.0), model.get("Jp", 0.0)
    for a in range(norb):
        for b in range(norb):
            if a != b:
                H -= jx * cd[a] @ c[ns + a] @ cd[ns + b] @ c[b]
                H += jp * cd[a] @ cd[ns + a] @ c[ns + b] @ c[b]
    return H, c


def sector_block(model, nup, ndw):
    ns = fock.ns_of(model)
    H, _ = fock_hamiltonian(model)
    _, _, I = fock.sector_states(ns, nup, ndw)
    idx = I.astype(np.int64)
    return H[np.ix_(idx, idx)]
