"""Sector basis and the explicit sector Hamiltonian on full 2Ns-bit Fock strings.

Oracle (test infrastructure).  Conventions (readings of Sec. 2.3, listed in the
design notes):
  * level k (0-based) of spin sigma is fermionic mode m = k + sigma*Ns, with all
    spin-up modes before all spin-down modes (the state order of Sec. 2.3);
  * Fock index I = I_up + I_dw * 2**Ns (eq. Irelation), bit m of I = n_m;
  * c_m |I> = (-1)**(number of occupied modes m' < m) |I - 2**m>  (Sec. 2.3);
  * impurity orbital a sits at level a, bath level (a, nu) at level
    norb + a*nbath + nu;
  * sector index i = i_up + i_dw * D_up (0-based; eq. SectorIndxDecomp read
    with the spin-down offset that eq. Vmatrix states);
  * H is eq. Ham1 restricted to the normal bath, with plain U n_up n_dw (no
    Hartree constant) and the chemical potential acting on the impurity only;
    the spin-exchange and pair-hopping terms of eq. Ham1 (couplings Jx, Jp,
    default 0) act on the impurity orbitals exactly as printed there:
      - Jx sum_{a != b} d+_{a up} d_{a dw} d+_{b dw} d_{b up}
      + Jp sum_{a != b} d+_{a up} d+_{a dw} d_{b dw} d_{b up}.
"""
from __future__ import annotations

from itertools import combinations

import numpy as np
import scipy.sparse as sp


def ns_of(model):
    return model["norb"] * (model["nbath"] + 1)


def level_energies(model):
    """One-body level energies e_k, k < Ns (impurity levels shifted by -xmu)."""
    norb, nbath = model["norb"], model["nbath"]
    e = np.zeros(ns_of(model))
    e[:norb] = np.asarray(model["eps_imp"], float) - model["xmu"]
    e[norb:] = np.asarray(model["eps_bath"], float).reshape(norb * nbath)
    return e


def hop_pairs(model):
    """(impurity level a, bath level b, V) for every hybridisation term of eq. Ham1."""
    norb, nbath = model["norb"], model["nbath"]
    V = np.asarray(model["vhyb"], float).reshape(norb, nbath)
    out = []
    for a in range(norb):
        for nu in range(nbath):
            out.append((a, norb + a * nbath + nu, float(V[a, nu])))
    return out


def spin_strings_listing(nbit, n):
    """The build_sector listing (Sec. 6, "Sector construction"): loop over every
    integer 0..2**nbit-1 and append those whose popcount equals n."""
    out = []
    for i in range(2 ** nbit):
        if bin(i).count("1") == n:
            out.append(i)
    return np.array(out, dtype=np.uint64)


def spin_strings(nbit, n):
    """Same set built independently from combinations, sorted ascending."""
    if n < 0 or n > nbit:
        return np.zeros(0, dtype=np.uint64)
    vals = sorted(sum(1 << k for k in c) for c in combinations(range(nbit), n))
    return np.array(vals, dtype=np.uint64)


def orbital_levels(model, a):
    """The Nbit = Nbath + 1 levels of orbital a: its impurity level, then its
    bath levels in order (orbital-resolved quantum numbers, Sec. 2.2)."""
    norb, nbath = model["norb"], model["nbath"]
    return [a] + [norb + a * nbath + nu for nu in range(nbath)]


def orbital_spin_strings(model, counts):
    """Strings of one spin with counts[a] electrons in orbital a's levels, in the
    order of eq. SectorIndxDecomp: i = i_1 + D_1 (i_2 + D_2 (...)), i_a the
    position of orbital a's Nbit-bit string in that orbital's ascending
    listing (orbital 1 fastest)."""
    norb, nbath = model["norb"], model["nbath"]
    per = []
    for a in range(norb):
        lv = orbital_levels(model, a)
        loc = spin_strings(nbath + 1, counts[a])          # ascending Nbit-bit strings
        full = []
        for x in loc:
            f = 0
            for k in range(nbath + 1):
                if (int(x) >> k) & 1:
                    f |= 1 << lv[k]
            full.append(f)
        per.append(full)
    out = [0]
    for a in range(norb):                                  # orbital a varies slower than a-1
        out = [prev | x for x in per[a] for prev in out]
    return np.array(out, dtype=np.uint64)


def spin_basis(model, spec):
    """Strings of one spin for a sector spec: an int N (total-N sector,
    ascending listing) or a sequence of per-orbital counts."""
    if np.ndim(spec) == 0:
        return spin_strings(ns_of(model), int(spec))
    return orbital_spin_strings(model, [int(x) for x in spec])


def sector_states(ns, nup, ndw, model=None):
    """Full Fock integers of the sector in sector order (i_up fastest).  With a
    model, nup/ndw may be per-orbital count sequences."""
    if model is None:
        up = spin_strings(ns, nup)
        dw = spin_strings(ns, ndw)
    else:
        up = spin_basis(model, nup)
        dw = spin_basis(model, ndw)
    I = (up[None, :] + (dw[:, None] << np.uint64(ns))).ravel()
    return up, dw, I


def _parity_below(I, m):
    """(-1)**(number of set bits of I below bit m) for an array of uint64."""
    mask = np.uint64((1 << m) - 1)
    return 1 - 2 * (np.bitwise_count(I & mask).astype(np.int64) & 1)


def apply_cdag_c(I, a, b):
    """c+_a c_b applied to |I> for an array of Fock integers I.

    Returns (valid, I_new, sign).  The annihilator acts first, then the creator,
    each with its own string sign (Sec. 2.3)."""
    one = np.uint64(1)
    bb, ba = np.uint64(b), np.uint64(a)
    has_b = ((I >> bb) & one).astype(bool)
    s1 = _parity_below(I, b)
    I1 = I ^ (one << bb)
    has_a = ((I1 >> ba) & one).astype(bool)
    s2 = _parity_below(I1, a)
    I2 = I1 | (one << ba)
    valid = has_b & ~has_a
    return valid, I2, s1 * s2


def apply_cdag(I, m):
    one = np.uint64(1)
    occ = ((I >> np.uint64(m)) & one).astype(bool)
    return ~occ, I | (one << np.uint64(m)), _parity_below(I, m)


def apply_c(I, m):
    one = np.uint64(1)
    occ = ((I >> np.uint64(m)) & one).astype(bool)
    return occ, I & ~(one << np.uint64(m)), _parity_below(I, m)


def occupations(I, ns):
    """n[m, state] for m < 2*Ns as float64."""
    ms = np.arange(2 * ns, dtype=np.uint64)
    return ((I[None, :] >> ms[:, None]) & np.uint64(1)).astype(np.float64)


def diagonal(model, I):
    """<I|H|I>: one-body levels plus the density-density interaction of eq. Ham1."""
    ns, norb = ns_of(model), model["norb"]
    n = occupations(I, ns)
    e = level_energies(model)
    d = (e[:, None] * (n[:ns] + n[ns:])).sum(axis=0)
    U, Ust, J = model["U"], model["Ust"], model["Jh"]
    for a in range(norb):
        d += U * n[a] * n[ns + a]
    for a in range(norb):
        for b in range(norb):
            if a != b:
                d += Ust * n[a] * n[ns + b]
    for a in range(norb):
        for b in range(a + 1, norb):
            d += (Ust - J) * (n[a] * n[b] + n[ns + a] * n[ns + b])
    return d


def _lookup(strings, x):
    """Positions of the values x in the (not necessarily sorted) string list."""
    order = np.argsort(strings, kind="stable")
    return order[np.searchsorted(strings[order], x)]


def _index_of(up, dw, ns, Inew):
    """Sector index i_up + i_dw*D_up of Fock integers known to lie in the sector."""
    mask = np.uint64((1 << ns) - 1)
    iu = _lookup(up, Inew & mask)
    idw = _lookup(dw, Inew >> np.uint64(ns))
    return iu.astype(np.int64) + idw.astype(np.int64) * len(up)


def hopping_terms(model):
    """Every off-diagonal operator c+_a c_b (with amplitude) of eq. Ham1, both
    directions and both spins, as (mode_a, mode_b, amplitude)."""
    ns = ns_of(model)
    out = []
    for (a, b, V) in hop_pairs(model):
        for s in (0, 1):
            out.append((a + s * ns, b + s * ns, V))
            out.append((b + s * ns, a + s * ns, V))
    return out


def nondiagonal_terms(model):
    """The spin-exchange and pair-hopping operators of eq. Ham1 as
    (amplitude, [(mode, creator?), ...] listed left to right), for every
    ordered pair of distinct impurity orbitals."""
    ns, norb = ns_of(model), model["norb"]
    jx, jp = float(model.get("Jx", 0.0)), float(model.get("Jp", 0.0))
    up = lambda a: a
    dw = lambda a: a + ns
    out = []
    for a in range(norb):
        for b in range(norb):
            if a == b:
                continue
            if jx != 0.0:
                out.append((-jx, [(up(a), True), (dw(a), False), (dw(b), True), (up(b), False)]))
            if jp != 0.0:
                out.append((jp, [(up(a), True), (dw(a), True), (dw(b), False), (up(b), False)]))
    return out


def apply_product(I, ops):
    """A product of creators/annihilators (listed left to right) applied to
    |I>: the rightmost acts first.  Returns (valid, I_new, sign)."""
    valid = np.ones(I.shape, dtype=bool)
    sign = np.ones(I.shape, dtype=np.int64)
    cur = I.copy()
    for (m, creator) in reversed(ops):
        ok, nxt, sg = (apply_cdag if creator else apply_c)(cur, m)
        valid &= ok
        sign *= sg
        cur = np.where(ok, nxt, cur)
    return valid, cur, sign


def explicit_hamiltonian(model, nup, ndw):
    """Sector Hamiltonian H_S as CSR, built term by term on full 2Ns-bit strings.

    Does not use the spin factorisation: every sign is the full-string sign of
    Sec. 2.3.  H[i, j] = <i|H|j>.  nup/ndw: electron counts, or per-orbital
    count sequences (orbital-resolved sector)."""
    ns = ns_of(model)
    up, dw, I = sector_states(ns, nup, ndw, model)
    D = I.size
    rows, cols, vals = [np.arange(D)], [np.arange(D)], [diagonal(model, I)]
    for (ma, mb, V) in hopping_terms(model):
        valid, Inew, sgn = apply_cdag_c(I, ma, mb)
        j = np.nonzero(valid)[0]
        rows.append(_index_of(up, dw, ns, Inew[j]))
        cols.append(j)
        vals.append(V * sgn[j].astype(np.float64))
    for (amp, ops) in nondiagonal_terms(model):
        valid, Inew, sgn = apply_product(I, ops)
        j = np.nonzero(valid)[0]
        rows.append(_index_of(up, dw, ns, Inew[j]))
        cols.append(j)
        vals.append(amp * sgn[j].astype(np.float64))
    H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(D, D)).tocsr()
    H.sum_duplicates()
    return H


def hv_rows(model, nup, ndw, v, rows):
    """(H v)[rows] computed row by row from second quantisation, for sectors too
    large to store H.  H is real symmetric, so row i of H is H|i>."""
    ns = ns_of(model)
    up = spin_basis(model, nup)
    dw = spin_basis(model, ndw)
    rows = np.asarray(rows, dtype=np.int64)
    iu, idw = rows % len(up), rows // len(up)
    I = up[iu] + (dw[idw] << np.uint64(ns))
    v = np.asarray(v, dtype=np.float64)
    out = diagonal(model, I) * v[rows]
    for (ma, mb, V) in hopping_terms(model):
        valid, Inew, sgn = apply_cdag_c(I, ma, mb)
        k = np.nonzero(valid)[0]
        j = _index_of(up, dw, ns, Inew[k])
        out[k] += V * sgn[k] * v[j]
    # H is symmetric: row i of the interaction terms is the operator applied to |i>
    for (amp, ops) in nondiagonal_terms(model):
        valid, Inew, sgn = apply_product(I, ops)
        k = np.nonzero(valid)[0]
        j = _index_of(up, dw, ns, Inew[k])
        out[k] += amp * sgn[k] * v[j]
    return out


def sector_dim(ns, nup, ndw):
    """Number of states of the sector, by counting the enumerated strings."""
    return len(spin_strings(ns, nup)) * len(spin_strings(ns, ndw))


def spin_hop_csr(model, n, spin):
    """Per-spin hopping list of one spin species as (off, col, sign, amp),
    rows in ascending string order, entries sorted by column.

    Derived from second quantisation on the full 2Ns-bit string with the other
    spin species empty.  That the sign does not depend on the other species'
    string is checked separately: the explicit H must equal the Kronecker
    assembly of these lists entry for entry."""
    ns = ns_of(model)
    strings = spin_strings(ns, n)
    shift = np.uint64(ns * spin)
    I = strings << shift
    rows, cols, sgns, amps = [], [], [], []
    for (a, b, V) in hop_pairs(model):
        for (x, y) in ((a, b), (b, a)):
            valid, Inew, sg = apply_cdag_c(I, x + ns * spin, y + ns * spin)
            j = np.nonzero(valid)[0]
            # H[i, j] = <i|c+_x c_y|j>: row is the new string
            r = np.searchsorted(strings, Inew[j] >> shift)
            rows.append(r)
            cols.append(j)
            sgns.append(sg[j])
            amps.append(np.full(j.size, V))
    if not rows:                       # no bath levels: no hopping at all
        rows = cols = sgns = [np.zeros(0, dtype=np.int64)]
        amps = [np.zeros(0)]
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    sgns = np.concatenate(sgns)
    amps = np.concatenate(amps)
    order = np.lexsort((cols, rows))
    rows, cols, sgns, amps = rows[order], cols[order], sgns[order], amps[order]
    off = np.zeros(len(strings) + 1, dtype=np.int64)
    np.add.at(off, rows + 1, 1)
    off = np.cumsum(off)
    return off, cols.astype(np.int64), sgns.astype(np.int8), amps
