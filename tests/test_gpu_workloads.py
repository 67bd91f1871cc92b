"""GPU runs of the full-size workloads against stored oracle values.

tests/golden/ns12.npz and ns15o3.npz are written by tests/golden/make_golden.py,
which calls only the CPU oracle (explicit sector matrix / Kronecker form, ARPACK,
Krylov Green's function).

Bars: E0 FP64 1e-10 relative; G(i w_n) FP64 1e-8 * max|G|.  FP32 precision mode
is not fixed by the paper (parity unpinned): its errors are printed and only a
loose sanity bound is asserted.
"""
import os

import numpy as np
import pytest

from paper_2105_06806_amd import inputs

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def edx():
    import torch
    from paper_2105_06806_amd import edx as E
    assert torch.cuda.is_available()
    return E


def _gold(name):
    p = os.path.join(GOLD, name)
    if not os.path.exists(p):
        pytest.skip(f"{name} not generated (run tests/golden/make_golden.py)")
    return np.load(p)


def test_ns12_ground_state_and_green(edx):
    g = _gold("ns12.npz")
    m, [sec] = inputs.workload("ns12")
    S = edx.build_sector(m, *sec)
    e0, psi, rep, _ = edx.lanczos_ground_state(S, niter=512, tol=1e-14, rtol=1e-10, seed=21)
    assert abs(e0 - g["e0"]) <= 1e-10 * abs(g["e0"]), (e0, float(g["e0"]))
    G, gr = edx.green_cf(S, psi, e0, 0, 0, ngf=200, beta=float(g["beta"]), lmats=int(g["lmats"]))
    ref = g["g"]
    err = np.abs(G - ref).max() / np.abs(ref).max()
    print(f"ns12: |dE0|/|E0| = {abs(e0 - g['e0']) / abs(g['e0']):.2e}, max|dG|/max|G| = {err:.2e}")
    assert err <= 1e-8
    assert abs(gr["wp"] + gr["wh"] - 1.0) < 1e-12
    assert abs(gr["wp"] - float(g["wp"])) < 1e-10


def test_ns12_particle_hole_and_twin(edx):
    m, _ = inputs.workload("ns12")
    e = {}
    for sec in [(7, 6), (5, 6), (6, 7), (6, 5)]:
        S = edx.build_sector(m, *sec)
        e[sec] = edx.lanczos_ground_state(S, want_psi=False, niter=512, tol=1e-14, seed=3)[0]
    assert abs(e[(7, 6)] - e[(5, 6)]) < 1e-10 * abs(e[(7, 6)])    # particle-hole
    assert abs(e[(7, 6)] - e[(6, 7)]) < 1e-10 * abs(e[(7, 6)])    # twin sectors
    assert abs(e[(5, 6)] - e[(6, 5)]) < 1e-10 * abs(e[(5, 6)])


def _gsum(edx, S, psi, e0, lm, beta, orb=0):
    """G_up + G_dw of one orbital: independent of which vector of a degenerate
    ground level was found (see tests/golden/make_golden.py)."""
    Gu, ru = edx.green_cf(S, psi, e0, orb, 0, ngf=200, beta=beta, lmats=lm)
    Gd, rd = edx.green_cf(S, psi, e0, orb, 1, ngf=200, beta=beta, lmats=lm)
    return Gu + Gd, ru["wp"] + rd["wp"]


def test_ns15o3_every_orbital(edx):
    """Norb=3, D=41.4M, FP64: G_up + G_dw of each orbital against the
    oracle's (ns15o3_orb.npz, its own ground-state solve), 1e-8 * max|G|,
    and the particle weights."""
    path = os.path.join(GOLD, "ns15o3_orb.npz")
    if not os.path.exists(path):
        pytest.skip("ns15o3_orb.npz not written")
    g = np.load(path)
    m, [sec] = inputs.workload("ns15o3")
    S = edx.build_sector(m, *sec)
    E = float(g["e0"])
    lm, beta = int(g["lmats"]), float(g["beta"])
    e64, psi, rep, st = edx.lanczos_ground_state(S, niter=600, tol=1e-14, rtol=1e-10, seed=4,
                                                 allow=(edx.EDX_E_DEGENERATE,))
    assert abs(e64 - E) <= 1e-10 * abs(E), (e64, E)
    for orb in range(m["norb"]):
        G, wp = _gsum(edx, S, psi, e64, lm, beta, orb)
        ref = g["g_sum"][orb]
        err = np.abs(G - ref).max() / np.abs(ref).max()
        print(f"ns15o3 orbital {orb}: dG {err:.2e}")
        assert err <= 1e-8, (orb, err)
        assert abs(wp - float(g["weights"][orb, :, 0].sum())) < 1e-9, orb


def test_ns15o3_precision_mode(edx):
    """Norb=3, D=41.4M: FP64 against the oracle; FP32 vectors with FP64
    recurrence (none / local / full re-orthogonalisation), errors reported."""
    g = _gold("ns15o3.npz")
    if "g_up" not in g:
        pytest.skip("ns15o3.npz predates the two-spin reference")
    m, [sec] = inputs.workload("ns15o3")
    S = edx.build_sector(m, *sec)
    E = float(g["e0"])
    lm, beta = int(g["lmats"]), float(g["beta"])
    gref = g["g_up"] + g["g_dw"]
    e64, psi64, rep, st = edx.lanczos_ground_state(S, niter=600, tol=1e-14, rtol=1e-10, seed=4,
                                                   allow=(edx.EDX_E_DEGENERATE,))
    assert abs(e64 - E) <= 1e-10 * abs(E), (e64, E)
    # the 7/7 ground level is two-fold (the spin swap maps one vector of it
    # onto another): the deflated check must see the second copy
    assert st == edx.EDX_E_DEGENERATE and rep["degenerate"] == 1, (st, rep)
    assert abs(rep["e1"] - e64) <= 1e-9 * abs(E), rep
    G64, wp64 = _gsum(edx, S, psi64, e64, lm, beta)
    gerr64 = np.abs(G64 - gref).max() / np.abs(gref).max()
    print(f"ns15o3 f64: dE0 {abs(e64 - E) / abs(E):.2e} dG {gerr64:.2e} iters {rep['iters']}")
    assert gerr64 <= 1e-8
    assert abs(wp64 - float(g["wp_up"] + g["wp_dw"])) < 1e-9
    del psi64
    for reorth in (0, 1, 2):
        e32, psi32, rep32, st = edx.lanczos_ground_state(
            S, vtype="f32", reorth=reorth, niter=400, tol=1e-9, seed=4,
            allow=(edx.EDX_E_NOCONV, edx.EDX_E_DEGENERATE))
        G32, _ = _gsum(edx, S, psi32, e32, lm, beta)
        de = abs(e32 - E) / abs(E)
        dg = np.abs(G32 - gref).max() / np.abs(gref).max()
        print(f"ns15o3 f32 reorth={reorth}: dE0 {de:.2e} dG {dg:.2e} iters {rep32['iters']} status {st}")
        assert de < 1e-5
        assert dg < 5e-2
        del psi32


MO_CASES = [(2, 3, (4, 3), False), (3, 1, (3, 2), False), (3, 1, (2, 4), False),
            (2, 3, (3, 3), True), (3, 1, (3, 3), True)]


@pytest.mark.parametrize("norb,nbath,sec,degenerate", MO_CASES)
def test_green_multiorbital_small(edx, norb, nbath, sec, degenerate):
    """Every orbital of small multi-orbital sectors against the exact Lehmann
    sum.  Non-degenerate ground level: each spin separately.  Spin-swap
    degenerate ground level (checked here with the oracle): G_up + G_dw, which
    does not depend on the ground vector found."""
    from oracle import fock, green, spectra
    m = inputs.make_model(norb, nbath, 3.0, Jh=0.5, seed=55, symmetric=False, elo=-2, ehi=2,
                          vlo=0.1, vhi=0.5)
    H = fock.explicit_hamiltonian(m, *sec)
    w = np.linalg.eigvalsh(H.toarray())[:2]
    assert (w[1] - w[0] < 1e-9) == degenerate
    S = edx.build_sector(m, *sec)
    e0, psi, rep, st = edx.lanczos_ground_state(S, niter=400, tol=1e-14, rtol=1e-11, seed=8,
                                                allow=(edx.EDX_E_DEGENERATE,))
    assert abs(e0 - w[0]) <= 1e-10 * abs(w[0])
    # the deflated check (gs_threshold) flags exactly the degenerate levels
    assert (st == edx.EDX_E_DEGENERATE) == degenerate, (st, rep)
    beta, lm = 40.0, 128
    z = 1j * green.matsubara(beta, lm)
    for orb in range(norb):
        G = [edx.green_cf(S, psi, e0, orb, sp, ngf=300, beta=beta, lmats=lm)[0] for sp in (0, 1)]
        if degenerate:
            got = G[0] + G[1]
            ref = sum(green.lehmann_exact(m, *sec, orb, sp, z)[0] for sp in (0, 1))
            assert np.abs(got - ref).max() <= 1e-8 * np.abs(ref).max(), orb
        else:
            for sp in (0, 1):
                ref = green.lehmann_exact(m, *sec, orb, sp, z)[0]
                assert np.abs(G[sp] - ref).max() <= 1e-8 * np.abs(ref).max(), (orb, sp)
