"""Writes the oracle reference values stored under tests/golden/ (calls only oracle/).

    python tests/golden/make_golden.py [ns12|ns15o3|all]

ns12.npz   Ns=12 half filling (Norb=1, Nbath=11, sector 6/6, D=853,776):
           E0 from the explicit sector matrix (ARPACK and Lanczos with full
           re-orthogonalisation), spin-up impurity G(i w_n) on 4096 Matsubara
           frequencies at beta=200 by the Krylov form at depth 200 from the
           oracle's ground vector, and the same at depth 400 (truncation check).
ns15o3.npz Ns=15, Norb=3, Nbath=4, sector 7/7 (D=41,409,225): E0 and the
           ground vector's G for orbital 0, spin up and spin down, with the
           Kronecker form of H (the explicit matrix does not fit), ARPACK for
           the ground state, plain Lanczos (depth 200) for G on 1024 Matsubara
           frequencies.  The ground level of this sector is doubly degenerate
           (the density-density interaction conserves every orbital's
           occupation per spin, and exchanging the spins maps one such
           occupation pattern onto another of the same sector), so G of one
           spin depends on which ground vector is found; G_up + G_dw does not
           (the two degenerate vectors lie in decoupled subspaces).
ns15o3_orb.npz the same sector and ground-state solve, G_up + G_dw for each of
           the three orbitals (the quantity that does not depend on which
           vector of the degenerate ground level is found); the six
           (orbital, spin) Krylov runs share the ground vector and run in
           forked worker processes.
Inputs come from the seeded generator (paper_2105_06806_amd.inputs, seeds
2000 and 3000), which holds no arithmetic of the method.
"""
import os
import sys
import time

import numpy as np
import scipy.sparse.linalg as spla

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import fock, green, kron, rng, spectra  # noqa: E402
from paper_2105_06806_amd import inputs  # noqa: E402


def ns12():
    t0 = time.time()
    m, [sec] = inputs.workload("ns12")
    H = fock.explicit_hamiltonian(m, *sec)
    Ea, _ = spectra.arpack_lowest(H)
    E, psi, it = spectra.lanczos_full_reorth(lambda x: H @ x, rng.start_vector(1, H.shape[0]),
                                              maxiter=400, tol=1e-14)
    beta, lmats = 200.0, 4096
    z = 1j * green.matsubara(beta, lmats)

    def factory(a, b):
        Ht = fock.explicit_hamiltonian(m, a, b)
        return lambda x: Ht @ x

    G, wp, wh, (ap, bp), (ah, bh) = green.krylov_gf(m, *sec, psi, E, 0, 0, 200, z, factory)
    G4, _, _, _, _ = green.krylov_gf(m, *sec, psi, E, 0, 0, 400, z, factory)
    np.savez(os.path.join(HERE, "ns12.npz"), e0=E, e0_arpack=Ea, lanczos_iters=it, beta=beta,
             lmats=lmats, g=G, g400=G4, wp=wp, wh=wh, alpha_p=ap, beta_p=bp, alpha_h=ah,
             beta_h=bh)
    print(f"ns12: E0 {E:.15f} arpack {Ea:.15f} |G200-G400| {np.abs(G - G4).max():.2e} "
          f"({time.time() - t0:.0f} s)")


def ns15o3():
    t0 = time.time()
    m, [sec] = inputs.workload("ns15o3")
    K = kron.KronH(m, *sec)
    op = spla.LinearOperator((K.dim, K.dim), matvec=K.matvec, dtype=np.float64)
    w, V = spla.eigsh(op, k=1, which="SA", tol=1e-13, ncv=24,
                      v0=rng.start_vector(3, K.dim))
    E, psi = float(w[0]), V[:, 0]
    print(f"ns15o3: E0 {E:.15f} ({time.time() - t0:.0f} s)", flush=True)
    beta, lmats = 200.0, 1024
    z = 1j * green.matsubara(beta, lmats)

    def factory(a, b):
        Kt = kron.KronH(m, a, b)
        return Kt.matvec

    G, wp, wh, _, _ = green.krylov_gf(m, *sec, psi, E, 0, 0, 200, z, factory)
    Gd, wpd, whd, _, _ = green.krylov_gf(m, *sec, psi, E, 0, 1, 200, z, factory)
    np.savez(os.path.join(HERE, "ns15o3.npz"), e0=E, beta=beta, lmats=lmats, g_up=G, g_dw=Gd,
             wp_up=wp, wh_up=wh, wp_dw=wpd, wh_dw=whd)
    print(f"ns15o3: G done ({time.time() - t0:.0f} s)")


_ORB = {}


def _orb_gf(job):
    orb, spin = job
    m, sec, psi, E, z = (_ORB[k] for k in ("m", "sec", "psi", "E", "z"))

    def factory(a, b):
        return kron.KronH(m, a, b).matvec

    G, wp, wh, _, _ = green.krylov_gf(m, *sec, psi, E, orb, spin, 200, z, factory)
    return orb, spin, G, wp, wh


def ns15o3_orb():
    import multiprocessing as mp
    t0 = time.time()
    m, [sec] = inputs.workload("ns15o3")
    K = kron.KronH(m, *sec)
    op = spla.LinearOperator((K.dim, K.dim), matvec=K.matvec, dtype=np.float64)
    w, V = spla.eigsh(op, k=1, which="SA", tol=1e-13, ncv=24,
                      v0=rng.start_vector(3, K.dim))
    E, psi = float(w[0]), np.ascontiguousarray(V[:, 0])
    del V, op
    print(f"ns15o3_orb: E0 {E:.15f} ({time.time() - t0:.0f} s)", flush=True)
    beta, lmats = 200.0, 1024
    _ORB.update(m=m, sec=sec, psi=psi, E=E, z=1j * green.matsubara(beta, lmats))
    jobs = [(orb, spin) for orb in range(m["norb"]) for spin in (0, 1)]
    with mp.get_context("fork").Pool(len(jobs)) as pool:
        res = pool.map(_orb_gf, jobs)
    g = np.zeros((m["norb"], lmats), complex)
    wts = np.zeros((m["norb"], 2, 2))
    for orb, spin, G, wp, wh in res:
        g[orb] += G
        wts[orb, spin] = (wp, wh)
    np.savez(os.path.join(HERE, "ns15o3_orb.npz"), e0=E, beta=beta, lmats=lmats, g_sum=g,
             weights=wts)
    print(f"ns15o3_orb: G done ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    if which in ("ns12", "all"):
        ns12()
    if which in ("ns15o3", "all"):
        ns15o3()
    if which in ("ns15o3_orb", "all"):
        ns15o3_orb()
