"""Seeded synthetic Anderson-impurity inputs shared by the oracle tests and the GPU path.

This module only draws parameters; it contains none of the method's arithmetic
(no basis, no Hamiltonian, no Lanczos).  Both the CPU oracle (through the tests)
and the HIP path (through the binding and ``bench.py``) receive the same
dictionaries from here.

Model (normal bath, Sec. 2.1 eq. Ham1, density-density part only):
  * ``norb`` impurity orbitals, ``nbath`` bath levels per orbital,
    Ns = norb * (nbath + 1) levels per spin.
  * ``eps_imp[norb]`` impurity levels, ``xmu`` chemical potential (impurity only).
  * ``eps_bath[norb, nbath]`` bath levels, ``vhyb[norb, nbath]`` hybridisations,
    orbital-major.
  * ``U`` intra-orbital, ``Ust`` inter-orbital opposite-spin (U'), ``Jh`` Hund (J):
    same-spin inter-orbital coupling is U' - J.

Workload recipes (the paper's benchmark draws random bath energies and averages
over 10 realisations, Sec. 5 "Benchmarks"; the sizes below are the ones this
implementation is measured on):

  ``ns8``   Norb=1, Nbath=7  (Ns=8),  U=2, eps_imp=-U/2, symmetrised bath.
  ``ns12``  Norb=1, Nbath=11 (Ns=12), same distributions; GF workload.
  ``ns15o3`` Norb=3, Nbath=4 (Ns=15), U=3, J=0.5, U'=U-2J, Hartree-shifted
            eps_imp, eps_bath ~ U[-2,2], V ~ U[0.1,0.5].
  ``ns16``  Norb=1, Nbath=15 (Ns=16), symmetrised bath (the H.v headline sector).
  ``ns16o2`` Norb=2, Nbath=7 (Ns=16), as ns15o3 with J=U/6.
  ``batch`` 64 sets, Ns = [10,12,14][k % 3], U=2, symmetrised bath, all sectors
            N_up, N_dw in [Ns/2-2, Ns/2+2].
  ``serve`` Norb in {1,2}, Ns in 10..16 (Norb=2: even Ns only), U ~ U[1,6].

Seeds: realisation r of workload w uses seed = SEED_BASE[w] + r.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = {"ns8": 1000, "ns12": 2000, "ns15o3": 3000, "batch": 4000,
             "serve": 5000, "ns16": 6000, "ns16o2": 7000}


def _symmetrised_bath(rng, nbath, elo, ehi, vlo, vhi):
    """Particle-hole symmetric bath: pairs {x, -x} sharing one V, plus a level
    at 0 with its own V when nbath is odd.  Draw order: energies, then V."""
    m = nbath // 2
    x = rng.uniform(elo, ehi, size=m)
    v = rng.uniform(vlo, vhi, size=m + (nbath % 2))
    eps = np.concatenate([x, -x, np.zeros(nbath % 2)])
    vh = np.concatenate([v[:m], v[:m], v[m:]])
    return eps, vh


def _plain_bath(rng, nbath, elo, ehi, vlo, vhi):
    eps = rng.uniform(elo, ehi, size=nbath)
    vh = rng.uniform(vlo, vhi, size=nbath)
    return eps, vh


def make_model(norb, nbath, U, Ust=None, Jh=0.0, eps_imp=None, xmu=0.0,
               seed=0, symmetric=True, elo=-1.0, ehi=1.0, vlo=0.2, vhi=0.6, Jx=0.0, Jp=0.0,
               nph=0, w0=0.0, g=None):
    """Draw one bath realisation.  ``eps_imp`` defaults to the half-filling
    Hartree shift -(U/2 + (norb-1)(2U'-J)/2), which is -U/2 for norb=1.
    ``Jx``, ``Jp``: spin-exchange and pair-hopping couplings (0: density-density
    interaction only).  ``nph``, ``w0``, ``g``: Holstein phonon cutoff, frequency
    and per-orbital couplings (nph = 0: no phonons)."""
    rng = np.random.default_rng(seed)
    if Ust is None:
        Ust = U - 2.0 * Jh
    if eps_imp is None:
        eps_imp = -(U / 2.0 + (norb - 1) * (2.0 * Ust - Jh) / 2.0)
    eb = np.zeros((norb, nbath))
    vb = np.zeros((norb, nbath))
    for a in range(norb):
        draw = _symmetrised_bath if symmetric else _plain_bath
        eb[a], vb[a] = draw(rng, nbath, elo, ehi, vlo, vhi)
    return {
        "norb": int(norb), "nbath": int(nbath),
        "eps_imp": np.full(norb, float(eps_imp)), "xmu": float(xmu),
        "eps_bath": eb, "vhyb": vb,
        "U": float(U), "Ust": float(Ust), "Jh": float(Jh),
        "Jx": float(Jx), "Jp": float(Jp),
        "nph": int(nph), "w0": float(w0),
        "g": np.zeros(norb) if g is None else np.broadcast_to(np.asarray(g, float), (norb,)).copy(),
    }


def ns_of(model):
    return model["norb"] * (model["nbath"] + 1)


def workload(name, r=0):
    """Model plus the sector(s) of a named workload, realisation ``r``."""
    seed = SEED_BASE[name] + r
    if name == "ns8":
        m = make_model(1, 7, 2.0, seed=seed)
        return m, [(4, 4)]
    if name == "ns12":
        m = make_model(1, 11, 2.0, seed=seed)
        return m, [(6, 6)]
    if name == "ns16":
        m = make_model(1, 15, 2.0, seed=seed)
        return m, [(8, 8)]
    if name == "ns15o3":
        m = make_model(3, 4, 3.0, Jh=0.5, seed=seed, symmetric=False,
                       elo=-2.0, ehi=2.0, vlo=0.1, vhi=0.5)
        return m, [(7, 7)]
    if name == "ns16o2":
        m = make_model(2, 7, 3.0, Jh=0.5, seed=seed, symmetric=False,
                       elo=-2.0, ehi=2.0, vlo=0.1, vhi=0.5)
        return m, [(8, 8)]
    raise KeyError(name)


def batch_jobs(nsets=64, seed_base=SEED_BASE["batch"], ns_cycle=(10, 12, 14),
               spread=2, U=2.0):
    """Bath sets k < nsets with Ns = ns_cycle[k % len], each solved in every
    sector N_up, N_dw in [Ns/2 - spread, Ns/2 + spread]."""
    jobs = []
    for k in range(nsets):
        ns = ns_cycle[k % len(ns_cycle)]
        m = make_model(1, ns - 1, U, seed=seed_base + k)
        h = ns // 2
        for nup in range(h - spread, h + spread + 1):
            for ndw in range(h - spread, h + spread + 1):
                jobs.append((k, m, nup, ndw))
    return jobs


def serve_requests(n, seed=SEED_BASE["serve"], ns_lo=10, ns_hi=16):
    """Request mix: Norb in {1,2}; Norb=1 draws Ns in ns_lo..ns_hi, Norb=2
    draws an even Ns; U ~ U[1,6]; half filling N = floor(Ns/2)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        norb = int(rng.integers(1, 3))
        if norb == 1:
            ns = int(rng.integers(ns_lo, ns_hi + 1))
        else:
            ns = int(rng.choice([x for x in range(ns_lo, ns_hi + 1) if x % 2 == 0]))
        U = float(rng.uniform(1.0, 6.0))
        sub = int(rng.integers(0, 2**31 - 1))
        if norb == 1:
            m = make_model(1, ns - 1, U, seed=sub)
        else:
            m = make_model(2, ns // 2 - 1, U, Jh=U / 6.0, seed=sub, symmetric=False,
                           elo=-2.0, ehi=2.0, vlo=0.1, vhi=0.5)
        reqs.append((m, ns // 2, ns // 2))
    return reqs


def poisson_arrivals(n, rate, seed):
    """Arrival times (seconds) of a Poisson stream with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def random_vector(dim, seed, dtype=np.float64):
    """Uniform [-1, 1) test vector (not normalised)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=dim).astype(dtype)
