"""Several bath sets of one sector shape at once (edx_hv_multi and the
multi-set groups of edx_batch_ground_state) through the C ABI.

Bars: each set's product against the oracle's explicit sector matrix of its
own model (FP64 1e-13, FP32 2e-6 of the row-sum bound of |H| times max|v|),
and bit for bit equal to edx_hv with the one-column fused plan (the multi-set
pass sums every set exactly as that pass does); at Ns=14 against the oracle's
Kronecker form; padding rows of w zero.  Batched ground energies of grouped
jobs: FP64 within 1e-10 relative of the oracle spectrum (dense up to 2500
rows, ARPACK on the sparse matrix above) and of the plain single-job path.
"""
import numpy as np
import pytest

from oracle import fock, kron, spectra
from paper_2105_06806_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def edx():
    import torch
    from paper_2105_06806_amd import edx as E
    assert torch.cuda.is_available()
    return E


def _hscale(m):
    e = np.abs(fock.level_energies(m)).sum() * 2
    return e + abs(m["U"]) * m["norb"] + abs(m["Ust"]) * m["norb"] ** 2 + \
        2 * np.abs(m["vhyb"]).sum() * 2 + 1.0


def _models(norb, nbath, k, seed0):
    out = []
    for b in range(k):
        if norb == 1:
            out.append(inputs.make_model(1, nbath, 1.0 + 0.7 * b, seed=seed0 + b))
        else:
            out.append(inputs.make_model(norb, nbath, 2.0 + 0.5 * b, Jh=0.3, seed=seed0 + b,
                                         symmetric=False, elo=-2, ehi=2, vlo=0.1, vhi=0.5))
    return out


CASES = [("o1_ns10", 1, 9, (5, 5)), ("o1_ns10_ragged", 1, 9, (4, 6)), ("o2_ns10", 2, 4, (5, 4))]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("k", [1, 2, 4, 8])
@pytest.mark.parametrize("name,norb,nbath,sec", CASES, ids=[c[0] for c in CASES])
def test_hv_multi_against_oracle_and_single(edx, name, norb, nbath, sec, k, dtype):
    import torch
    tdt = torch.float64 if dtype == "f64" else torch.float32
    ms = _models(norb, nbath, k, seed0=500 + 10 * k)
    Ss = [edx.build_sector(m, *sec) for m in ms]
    xs = [torch.as_tensor(inputs.random_vector(Ss[0].dim, seed=700 + b), dtype=tdt, device="cuda")
          for b in range(k)]
    v = edx.interleave(Ss[0], xs)
    w = torch.full_like(v, float("nan"))
    edx.hv_multi(Ss, v, w)
    torch.cuda.synchronize()
    assert bool((w.view(Ss[0].ddw, Ss[0].ld, k)[:, Ss[0].dup:, :] == 0).all())
    ys = edx.deinterleave(Ss[0], w, k)
    tol = 1e-13 if dtype == "f64" else 2e-6
    for b in range(k):
        H = fock.explicit_hamiltonian(ms[b], *sec)
        ref = H @ xs[b].double().cpu().numpy()
        err = np.abs(ys[b].double().cpu().numpy() - ref).max()
        assert err <= tol * _hscale(ms[b]), (b, err)
        # the single-vector fused pass with one column per workgroup
        assert edx.set_plan(Ss[b], dtype, raise_on_error=False, mode=2, col_cols=1,
                            col_threads=256, row_rows=64, row_cols=16, col_order=0) == 0
        w1 = torch.empty_like(xs[b])
        edx.hv(Ss[b], xs[b], w1)
        torch.cuda.synchronize()
        assert bool(torch.equal(w1, ys[b])), (b, float((w1 - ys[b]).abs().max()))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_hv_multi_ns14_against_kron(edx, dtype):
    """The batch workload's largest shape (Ns=14 7/7, D=11,778,624), four bath sets: the
    first and last set against the oracle's Kronecker form."""
    import torch
    tdt = torch.float64 if dtype == "f64" else torch.float32
    ms = _models(1, 13, 4, seed0=4100)
    Ss = [edx.build_sector(m, 7, 7) for m in ms]
    gen = torch.Generator(device="cuda").manual_seed(3)
    xs = [torch.rand(Ss[0].dim, dtype=tdt, device="cuda", generator=gen) * 2 - 1
          for _ in range(4)]
    v = edx.interleave(Ss[0], xs)
    w = torch.empty_like(v)
    edx.hv_multi(Ss, v, w)
    ys = edx.deinterleave(Ss[0], w, 4)
    tol = 1e-13 if dtype == "f64" else 2e-6
    for b in (0, 3):
        ref = kron.KronH(ms[b], 7, 7).matvec(xs[b].double().cpu().numpy())
        err = np.abs(ys[b].double().cpu().numpy() - ref).max()
        assert err <= tol * _hscale(ms[b]), (b, err)


@pytest.mark.parametrize("dtype,k", [("f32", 8), ("f64", 8), ("f64", 4)])
def test_hv_multi_ns12_equals_single(edx, dtype, k):
    """The shape the batch groups (Ns=12 6/6, D=853,776), up to eight sets:
    every set bit for bit equal to the one-column fused pass on its own."""
    import torch
    tdt = torch.float64 if dtype == "f64" else torch.float32
    ms = _models(1, 11, k, seed0=1200 + k)
    Ss = [edx.build_sector(m, 6, 6) for m in ms]
    gen = torch.Generator(device="cuda").manual_seed(4)
    xs = [torch.rand(Ss[0].dim, dtype=tdt, device="cuda", generator=gen) * 2 - 1 for _ in range(k)]
    w = edx.hv_multi(Ss, edx.interleave(Ss[0], xs), torch.empty(Ss[0].ld * Ss[0].ddw * k, dtype=tdt,
                                                                  device="cuda"))
    ys = edx.deinterleave(Ss[0], w, k)
    for b in range(k):
        assert edx.set_plan(Ss[b], dtype, raise_on_error=False, mode=2, col_cols=1,
                            col_threads=256, row_rows=64, row_cols=16, col_order=0) == 0
        w1 = torch.empty_like(xs[b])
        edx.hv(Ss[b], xs[b], w1)
        torch.cuda.synchronize()
        assert bool(torch.equal(w1, ys[b])), (b, float((w1 - ys[b]).abs().max()))


def test_hv_multi_refusals(edx):
    import torch
    ms = _models(1, 7, 3, seed0=900)
    Ss = [edx.build_sector(m, 4, 4) for m in ms]
    v = torch.zeros(Ss[0].ld * Ss[0].ddw * 3, dtype=torch.float64, device="cuda")
    w = torch.zeros_like(v)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    st = edx.lib.edx_hv_multi(edx._handles(Ss), 3, edx.F64, edx._P(v.data_ptr()),
                              edx._P(w.data_ptr()), edx._P(ws.data_ptr()), ws.numel(), None)
    assert st == edx.EDX_E_INVALID                       # k = 3
    other = edx.build_sector(ms[0], 5, 3)                # another shape
    with pytest.raises(edx.EdxError) as ei:
        edx.hv_multi([Ss[0], other], torch.zeros(Ss[0].ld * Ss[0].ddw * 2, dtype=torch.float64,
                                                 device="cuda"),
                     torch.zeros(Ss[0].ld * Ss[0].ddw * 2, dtype=torch.float64, device="cuda"))
    assert ei.value.status == edx.EDX_E_INVALID
    nd = [edx.build_sector(inputs.make_model(2, 2, 3.0, Jh=0.5, seed=s, symmetric=False, Jx=0.5,
                                             Jp=0.5), 3, 3) for s in (1, 2)]
    with pytest.raises(edx.EdxError) as ei:
        edx.hv_multi(nd, torch.zeros(nd[0].ld * nd[0].ddw * 2, dtype=torch.float64, device="cuda"),
                     torch.zeros(nd[0].ld * nd[0].ddw * 2, dtype=torch.float64, device="cuda"))
    assert ei.value.status == edx.EDX_E_UNSUPPORTED


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_groups_same_shape_jobs(edx, dtype):
    """Jobs of two shapes, five bath sets each, forced through the whole-GPU
    path (wide_min_dim 1000): groups of four run through the multi-set pass,
    the fifth alone; energies against the dense oracle (FP64) and the plain
    path, with grouping on and off."""
    print("batch grouping", dtype, flush=True)
    jobs, ms = [], []
    for ns in (8, 10):
        for m in _models(1, ns - 1, 5, seed0=300 + ns):
            h = ns // 2
            for sec in ((h, h), (h - 1, h)):
                jobs.append(edx.build_sector(m, *sec))
                ms.append((m, sec))
    kw = dict(vtype=dtype, niter=400, tol=1e-12 if dtype == "f64" else 1e-8, seed=9, check_every=4)
    tiles = {"lane_wgs": 8, "ccols": np.ones(len(jobs), np.int32), "rcols": np.full(len(jobs), 32, np.int32),
             "wide_min_dim": 1000, "multi_k": 4}
    res, _ = edx.batch_ground_state(jobs, tiles=tiles, **kw)
    res_off, _ = edx.batch_ground_state(jobs, tiles=dict(tiles, multi_k=1), **kw)
    for (m, sec), S, r, r1 in zip(ms, jobs, res, res_off):
        assert r["status"] == 0 and r1["status"] == 0, (sec, r, r1)
        plain = edx.lanczos_ground_state(S, want_psi=False, allow=(edx.EDX_E_DEGENERATE,), **kw)[0]
        if dtype == "f64":
            H = fock.explicit_hamiltonian(m, *sec)
            E0 = spectra.dense_lowest(H)[0][0] if H.shape[0] <= 2500 else spectra.arpack_lowest(H)[0]
            assert abs(r["e0"] - E0) <= 1e-10 * abs(E0), (sec, r["e0"], E0)
            assert abs(r["e0"] - plain) <= 1e-10 * abs(plain)
            assert r1["e0"] == plain          # grouping off: the plain path itself
        else:
            assert abs(r["e0"] - plain) <= 1e-4 * abs(plain), (sec, r["e0"], plain)


def test_batch_groups_edge_shapes(edx):
    """Edge sectors through the grouped path (wide_min_dim 1 sends every job
    to it): no electron of one spin, a completely filled spin, D = 1, and a
    small ragged sector; four bath sets of each shape, FP64 energies against
    the dense oracle spectrum (a D = 1 sector breaks down at the first step)."""
    ns = 6
    ms = _models(1, ns - 1, 4, seed0=2600)
    secs = [(0, 3), (3, 0), (0, 0), (ns, ns), (ns, 2), (2, 3)]
    jobs, refs = [], []
    for sec in secs:
        for m in ms:
            jobs.append(edx.build_sector(m, *sec))
            refs.append(spectra.dense_lowest(fock.explicit_hamiltonian(m, *sec))[0][0])
    kw = dict(vtype="f64", niter=200, tol=1e-13, seed=4, check_every=2)
    tiles = {"lane_wgs": 8, "ccols": np.ones(len(jobs), np.int32),
             "rcols": np.full(len(jobs), 32, np.int32), "wide_min_dim": 1, "multi_k": 4}
    res, _ = edx.batch_ground_state(jobs, tiles=tiles, **kw)
    for S, r, E0 in zip(jobs, res, refs):
        assert r["status"] == 0, (S.dim, r)
        assert abs(r["e0"] - E0) <= 1e-10 * max(1.0, abs(E0)), (S.dim, r["e0"], E0)
