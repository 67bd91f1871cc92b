"""GPU parity of the sector tables at full size and over every sector shape,
and of the whole Ns=16 product element by element (through the C ABI).

Bars: the string map, the inverse rank over all 2^Ns integers, the hop
columns, signs and signed amplitudes and the impurity patterns are compared
bit for bit with the oracle (Sec. 6 "Sector construction" listing order,
Sec. 2.3 fermionic sign); the one-body diagonal to 1e-14 relative.  The Ns=16
products are compared on every one of the 165,636,900 output elements with the
oracle's Kronecker form H_d o V + H_up V + V H_dw^T (pinned entry for entry to
the explicit second-quantised matrix), FP64 at 1e-13 of the row-sum bound of
|H| times max|v|, FP32 at 2e-6 of it.
"""
import math

import numpy as np
import pytest

from oracle import fock, kron
from paper_2105_06806_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def edx():
    import torch
    from paper_2105_06806_amd import edx as E
    assert torch.cuda.is_available()
    return E


def _rank_ref(ns, strings):
    r = np.full(1 << ns, -1, dtype=np.int32)
    r[strings.astype(np.int64)] = np.arange(strings.size, dtype=np.int32)
    return r


def _check_spin(S, m, spin, n, listing):
    ns = fock.ns_of(m)
    t = S.tables(spin)
    strings = (fock.spin_strings_listing(ns, n) if listing else fock.spin_strings(ns, n))
    assert np.array_equal(t["map"], strings.astype(np.uint32))
    assert np.array_equal(S.rank(spin), _rank_ref(ns, strings))
    off, col, sgn, amp = fock.spin_hop_csr(m, n, spin)
    assert np.array_equal(t["hop_off"], off)
    assert np.array_equal(t["hop_col"], col.astype(np.int32))
    assert np.array_equal(t["hop_sign"], sgn)
    assert np.array_equal(t["hop_amp"], amp * sgn)
    E, p = kron.spin_diagonal(m, n)
    assert np.array_equal(t["diag_p"], p.astype(np.uint8))
    assert np.abs(t["diag_e"] - E).max(initial=0.0) <= 1e-14 * max(1.0, np.abs(E).max(initial=0.0))


@pytest.mark.parametrize("wl", ["ns16", "ns16o2"])
def test_headline_tables_bit_exact(edx, wl):
    """The Ns=16 half-filled sectors of the H.v headline (Norb = 1 and 2), both
    spins, against the build_sector listing itself (loop over every integer)."""
    m, [sec] = inputs.workload(wl)
    S = edx.build_sector(m, *sec)
    assert S.dup == S.ddw == math.comb(16, 8)
    for spin in (0, 1):
        _check_spin(S, m, spin, sec[spin], listing=True)


def _sweep_models():
    out = []
    for ns in range(1, 17):
        out.append((1, ns - 1))
    for ns in range(2, 17, 2):
        out.append((2, ns // 2 - 1))
    for ns in (3, 6, 9, 12, 15):
        out.append((3, ns // 3 - 1))
    return out


@pytest.mark.parametrize("norb,nbath", _sweep_models(),
                         ids=[f"o{a}b{b}" for a, b in _sweep_models()])
def test_tables_every_sector_shape(edx, norb, nbath):
    """Every electron count N = 0..Ns of both spins (sector (N, Ns - N)) for
    Ns = 1..16 with one orbital, even Ns with two and Ns = 3..15 with three."""
    m = inputs.make_model(norb, nbath, 2.5, Jh=0.4 if norb > 1 else 0.0, seed=300 + 17 * norb + nbath,
                          symmetric=False, xmu=0.1)
    ns = fock.ns_of(m)
    for n in range(ns + 1):
        S = edx.build_sector(m, n, ns - n)
        assert S.dup == math.comb(ns, n) and S.ddw == math.comb(ns, ns - n)
        _check_spin(S, m, 0, n, listing=ns <= 12)
        _check_spin(S, m, 1, ns - n, listing=ns <= 12)


@pytest.mark.parametrize("norb,nbath,cup,cdw", [(2, 7, (4, 4), (4, 4)), (2, 7, (3, 5), (5, 2)),
                                                (3, 4, (2, 3, 2), (3, 2, 2))])
def test_orbital_rank_bit_exact(edx, norb, nbath, cup, cdw):
    """Orbital-resolved sectors (Sec. 2.2): the map and inverse rank follow the
    mixed-radix listing (pinned against a brute-force filter on the CPU)."""
    m = inputs.make_model(norb, nbath, 3.0, Jh=0.5, seed=71, symmetric=False)
    ns = fock.ns_of(m)
    S = edx.build_sector_orbital(m, cup, cdw)
    for spin, counts in ((0, cup), (1, cdw)):
        strings = fock.orbital_spin_strings(m, list(counts))
        t = S.tables(spin)
        assert np.array_equal(t["map"], strings.astype(np.uint32))
        assert np.array_equal(S.rank(spin), _rank_ref(ns, strings))


def _hscale(m):
    """Bound on the row sums of |H| (as in test_gpu_parity)."""
    e = np.abs(fock.level_energies(m)).sum() * 2
    return e + abs(m["U"]) * m["norb"] + abs(m["Ust"]) * m["norb"] ** 2 + \
        2 * np.abs(m["vhyb"]).sum() * 2 + 1.0


def _full_product(edx, wl, dtype, seed):
    import torch
    m, [sec] = inputs.workload(wl)
    S = edx.build_sector(m, *sec)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    gen = torch.Generator(device="cuda").manual_seed(seed)
    vd = torch.rand(S.dim, dtype=tdt, device="cuda", generator=gen) * 2 - 1
    v = edx.pad(S, vd)
    w = torch.full_like(v, float("nan"))
    edx.hv(S, v, w, ld=S.ld)
    torch.cuda.synchronize()
    got = w.view(S.ddw, S.ld)
    assert bool((got[:, S.dup:] == 0).all())
    got = got[:, :S.dup].double().cpu().numpy().ravel()
    del w, v
    x = vd.double().cpu().numpy()
    del vd
    ref = kron.KronH(m, *sec).matvec(x)
    return m, np.abs(got - ref).max(), _hscale(m) * np.abs(x).max()


@pytest.mark.parametrize("wl", ["ns16", "ns16o2"])
def test_hv_ns16_every_element_fp64(edx, wl):
    m, err, scale = _full_product(edx, wl, "f64", seed=12)
    assert err <= 1e-13 * scale, err


def test_hv_ns16_every_element_fp32(edx):
    m, err, scale = _full_product(edx, "ns16", "f32", seed=13)
    assert err <= 2e-6 * scale, err
