"""Benchmark of the exact-diagonalisation hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--quick] [--full]

Headline (the JSON `value`): a step is one storage-free H.v (Sec. 3, eq. Hbuild)
on the half-filled Ns=16 sector (Norb=1, Nbath=15, N_up=N_dw=8,
D=12870^2=165,636,900) with FP64 vectors (the paper's precision), in the launch
plan the project autotuner picks.  Inputs are resident in HBM before the timed
region.  value = algorithmic bytes / time, algorithmic bytes = D * (8 + 8): v
read once, w written once (the ~0.5 MB of tables are not counted).

Also in the JSON line (one pass of every hot-path row, each on its workload):
  f32            the same H.v with FP32 vectors (precision mode), its own roofline
  roofline       dominant kernel of the FP64 headline: algorithmic bytes / its
                 mean launch time (HIP events on the launch stream), HBM peak
                 8 TB/s; traffic = beyond-L2 bytes (FETCH_SIZE + WRITE_SIZE,
                 scaled) from the committed rocprofv3 counter summary if it was
                 taken on the current kernel source with this plan, else null
  bandwidth      the views side by side: algorithmic, beyond-L2 (MALL + HBM) and
                 a plain device copy
  cpu_baseline   the CPU oracle's row-by-row H.v on a bounded row sample
  ns12           FP64 ground state + G(i w_n) (4096 frequencies, beta=200) of the
                 Ns=12 half-filled sector, errors against the stored oracle values
  ns15o3         precision mode on Norb=3, Ns=15 (D=41.4M): FP64 and FP32 vectors
                 (plain / local / full re-orthogonalisation), E0 and G errors with
                 the FP64 residual of each psi0 and the gap to the next level
  batch          64 bath sets x 25 sectors (1600 ground states, Ns=10/12/14) in one
                 persistent launch vs the same solves one after another
  serve          Poisson streams of ground state + G requests (Ns 10..16) at several
                 rates: p50/p99 latency and solves/s vs one-at-a-time plain solves
  hv_kanamori    H.v with spin exchange and pair hopping
  orbital        orbital-resolved sector: H.v and ground state
  lowest_thermal several low-lying states; eigenstate list, thermal G and chi
  eph            H.v with a Holstein phonon mode
  shard          per-GPU pieces of the column-distributed product at p = 8
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_PMC = {"f32": os.path.join(ROOT, "profiles", "hv_ns16_f32_counters.md"),
               "f64": os.path.join(ROOT, "profiles", "hv_ns16_f64_counters.md")}
HV_SRC = os.path.join(ROOT, "paper_2105_06806_amd", "csrc", "hv.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline H.v only")
    ap.add_argument("--full", action="store_true", help="full-size serving sweep")
    ap.add_argument("--tune-reps", type=int, default=3)
    ap.add_argument("--serve-n", type=int, default=None,
                    help="requests per rate of the serving sweep (default 120, 1000 with --full)")
    ap.add_argument("--serve-ns-hi", type=int, default=None,
                    help="largest Ns of the serving requests (default 16)")
    ap.add_argument("--serve-rates", default=None,
                    help="comma-separated multiples of the plain capacity for the serving sweep")
    ap.add_argument("--serve-plain", default=None,
                    help="JSON file with the plain service times of the stream (read if present, "
                         "else measured and written): a sweep split over several runs")
    ap.add_argument("--serve-offset", type=int, default=0,
                    help="first request of the stream to submit (a rate split over runs)")
    ap.add_argument("--serve-span", type=int, default=None,
                    help="number of requests to submit from --serve-offset (default: the rest)")
    ap.add_argument("--serve-dump", default=None,
                    help="JSON file for every request's served and plain latency per rate "
                         "(exact percentiles of a rate split over runs)")
    ap.add_argument("--serve-cap", type=float, default=None,
                    help="plain capacity (requests/s) measured by an earlier run of the same mix: "
                         "the sweep's rates are multiples of it (a sweep split over several runs)")
    ap.add_argument("--only", default=None,
                    help="comma-separated sections (hv_ns16o2, hv_kanamori, orbital, lowest_thermal, "
                         "eph, shard, ns12, ns15o3, batch, serve): run just these, no headline "
                         "(profiling runs)")
    ap.add_argument("--plan", default=None,
                    help="mode,col_cols,col_threads,row_rows,row_cols[,col_order] of the FP32 "
                         "H.v instead of autotuning (profiling runs)")
    ap.add_argument("--plan64", default=None,
                    help="the same for the FP64 headline H.v (profiling runs)")
    ap.add_argument("--cpu-worker", nargs=2, type=int, default=None, metavar=("SEED", "ROWS"),
                    help=argparse.SUPPRESS)
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_hv(edx, torch, S, v, w, steps, warmup, ld=0):
    for _ in range(warmup):
        edx.hv(S, v, w, ld=ld)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        edx.hv(S, v, w, ld=ld)
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = np.array([a.elapsed_time(b) for a, b in ev])
    return ms, wall


def traffic_from_profile(plan, dt):
    """Beyond-L2 bytes (MALL + HBM) per launch of the H.v kernel from the
    committed counter summary of vector type dt, if it was taken on the
    current kernel source with this plan."""
    path = PROFILE_PMC[dt]
    if not os.path.exists(path):
        return None, "no counter summary"
    txt = open(path).read()
    mh = re.search(r"source_sha256:\s*([0-9a-f]{64})", txt)
    if not mh:
        return None, None
    cur = hashlib.sha256(open(HV_SRC, "rb").read()).hexdigest()
    if cur != mh.group(1):
        return None, "stale"
    keys = ("mode", "col_cols", "col_threads", "row_rows", "row_cols", "col_order")
    want = ",".join(str(int(plan[k])) for k in keys)
    for mp in re.finditer(r"traffic\[([0-9,]+)\]:\s*([0-9.eE+]+)", txt):
        if mp.group(1) == want:
            return float(mp.group(2)), "ok"
    return None, "plan not profiled"


def copy_bandwidth(torch, nbytes=1 << 30, reps=10):
    """Streaming GB/s (read + write) of a plain elementwise pass y = -x over a
    1 GiB FP32 buffer: the rate this GPU reaches with a copy-like kernel.  The
    same kernel (torch's neg, 1 GiB read and 1 GiB written per launch) is the
    calibration of the counter summaries under profiles/."""
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").uniform_()
    y = torch.empty_like(x)
    for _ in range(3):
        torch.neg(x, out=y)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        torch.neg(x, out=y)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del x, y
    return 2 * nbytes / (ms * 1e-3) / 1e9


def bench_hv_o2(edx, torch, a):
    """H.v on the Norb=2, Nbath=7 (Ns=16) half-filled sector, FP32 and FP64
    (hop rows of 16 slots, 7.47 real hops a string on average)."""
    from paper_2105_06806_amd import inputs
    m, [sec] = inputs.workload("ns16o2")
    S = edx.build_sector(m, *sec)
    out = {"workload": f"H.v, Norb=2 Nbath=7 (Ns=16) 8/8, D={S.dim}, hop widths "
                       f"{S.hop_nnz(0)[1]}/{S.hop_nnz(1)[1]}"}
    for dt, tdt, esz in (("f32", torch.float32, 4), ("f64", torch.float64, 8)):
        gen = torch.Generator(device="cuda").manual_seed(2)
        v = edx.pad(S, torch.rand(S.dim, dtype=tdt, device="cuda", generator=gen) * 2 - 1)
        w = torch.empty_like(v)
        plan, _ = edx.autotune_hv(S, v, w, reps=a.tune_reps, ld=S.ld)
        ms, _ = time_hv(edx, torch, S, v, w, a.steps, a.warmup, ld=S.ld)
        gbs = S.dim * 2 * esz / (ms.mean() * 1e-3) / 1e9
        out[dt] = {"us": round(float(ms.mean()) * 1e3, 1), "gbs": round(gbs, 1),
                   "frac": round(gbs / HBM_PEAK_GBS, 4), "plan": plan}
        del v, w
        torch.cuda.empty_cache()
    return out


def _cpu_rows_worker(seed, n):
    """One oracle process (started as `bench.py --cpu-worker SEED ROWS`, no GPU
    use): its own copy of the input vector (same seed), a disjoint random sample
    of output rows; prints "rows seconds"."""
    from oracle import fock
    from paper_2105_06806_amd import inputs
    m, [sec] = inputs.workload("ns16")
    D = 12870 * 12870
    v = np.random.default_rng(0).uniform(-1, 1, size=D)
    rows = np.random.default_rng(seed).choice(D, size=n, replace=False)
    fock.hv_rows(m, *sec, v, rows[:2000])                       # warm-up
    t0 = time.perf_counter()
    fock.hv_rows(m, *sec, v, rows)
    print(n, time.perf_counter() - t0, flush=True)


def bench_hv_kanamori(edx, torch, a):
    """FP32 H.v with spin exchange and pair hopping (Jx = Jp = J) on the
    Norb=2 Ns=16 and Norb=3 Ns=15 half-filled sectors, and the same models
    without them (density-density only)."""
    from paper_2105_06806_amd import inputs
    out = {}
    for name in ("ns16o2", "ns15o3"):
        m0, [sec] = inputs.workload(name)
        row = {}
        for tag, m in (("kanamori", dict(m0, Jx=m0["Jh"], Jp=m0["Jh"])), ("density_density", m0)):
            S = edx.build_sector(m, *sec)
            gen = torch.Generator(device="cuda").manual_seed(3)
            v = edx.pad(S, torch.rand(S.dim, dtype=torch.float32, device="cuda", generator=gen) * 2 - 1)
            w = torch.empty_like(v)
            plan, _ = edx.autotune_hv(S, v, w, reps=a.tune_reps, ld=S.ld)
            ms, _ = time_hv(edx, torch, S, v, w, max(10, a.steps // 2), a.warmup, ld=S.ld)
            row[tag] = {"us": round(float(ms.mean()) * 1e3, 1),
                        "gbs": round(S.dim * 8 / (ms.mean() * 1e-3) / 1e9, 1), "plan": plan}
            del v, w
            torch.cuda.empty_cache()
        row["workload"] = (f"H.v {name} {sec[0]}/{sec[1]} D={S.dim} FP32, U={m0['U']}, "
                           f"J=Jx=Jp={m0['Jh']} (kanamori) vs Jx=Jp=0")
        out[name] = row
    return out


def _hv_rate(edx, torch, S, a, dt=None, reps=None):
    """Mean FP32 H.v time on the padded layout with the autotuned plan."""
    dt = dt or torch.float32
    gen = torch.Generator(device="cuda").manual_seed(4)
    v = edx.pad(S, torch.rand(S.dim, dtype=dt, device="cuda", generator=gen) * 2 - 1)
    w = torch.empty_like(v)
    plan, _ = edx.autotune_hv(S, v, w, reps=a.tune_reps, ld=S.ld)
    ms, _ = time_hv(edx, torch, S, v, w, reps or max(10, a.steps // 2), a.warmup, ld=S.ld)
    us = float(ms.mean()) * 1e3
    gbs = S.dim * 2 * v.element_size() / (us * 1e-6) / 1e9
    del v, w
    torch.cuda.empty_cache()
    return {"us": round(us, 1), "gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "plan": plan}


def bench_orbital(edx, torch, a):
    """Orbital-resolved sector: Norb=2, Nbath=7 (Ns=16), per-orbital counts
    (4,4)/(4,4), D = 70^4; FP32 H.v and an FP64 ground state, beside the
    total-N 8/8 sector of the same model it is part of."""
    from paper_2105_06806_amd import inputs
    m, [sec] = inputs.workload("ns16o2")
    S = edx.build_sector_orbital(m, (4, 4), (4, 4))
    r = {"workload": f"Norb=2 Nbath=7 (Ns=16) orbital sector (4,4)/(4,4), D={S.dim}",
         "hv_f32": _hv_rate(edx, torch, S, a)}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0, _, rep, _ = edx.lanczos_ground_state(S, want_psi=False, niter=512, tol=1e-12, seed=3,
                                             allow=(edx.EDX_E_DEGENERATE, edx.EDX_E_NOCONV))
    r["gs_f64_s"] = round(time.perf_counter() - t0, 3)
    r["gs_iters"] = rep["iters"]
    return r


def bench_lowest_and_thermal(edx, torch, a):
    """Several low-lying states and finite temperature: the 8 lowest states of
    the Ns=12 6/6 sector (FP64, locking + check run; basis of 400 vectors, and of
    50 with thick restarts), and the eigenstate list
    plus thermal G and spin susceptibility over every sector of an Ns=8 model
    (beta=10, cutoff 1e-6, 3 annealing calls)."""
    from paper_2105_06806_amd import inputs
    out = {}
    m, [sec] = inputs.workload("ns12")
    S = edx.build_sector(m, *sec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e, _, rep, st = edx.lanczos_lowest(S, 8, want_psi=False, niter=400, tol=0.0, rtol=1e-10,
                                       seed=5, allow=(edx.EDX_E_NOCONV,))
    out["lowest8_ns12"] = {"s": round(time.perf_counter() - t0, 3), "runs": rep["runs"],
                           "iters": rep["iters"], "verified": rep["verified"],
                           "gaps": [round(float(x - e[0]), 6) for x in e]}
    # the same 8 states from a 50-vector basis (thick restarts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e50, _, rep, st = edx.lanczos_lowest(S, 8, want_psi=False, niter=50, tol=0.0, rtol=1e-10,
                                         seed=5, allow=(edx.EDX_E_NOCONV,))
    out["lowest8_ns12_niter50"] = {"s": round(time.perf_counter() - t0, 3), "runs": rep["runs"],
                                   "iters": rep["iters"], "verified": rep["verified"],
                                   "nfound": rep["nfound"],
                                   "max_dev_vs_niter400": float(np.abs(e50 - e).max())
                                   if len(e50) == len(e) else None}
    m8, _ = inputs.workload("ns8")
    secs = [(x, y) for x in range(9) for y in range(9)]
    Ss = [edx.build_sector(m8, *q) for q in secs]
    E = edx.Espace(len(secs), beta=10.0, cutoff=1e-6, nstates_sector=2, nstates_total=2000,
                   nstates_step=4)
    t0 = time.perf_counter()
    for _ in range(3):
        E.diag(Ss, niter=300, tol=0.0, rtol=1e-10, seed=1)
    t1 = time.perf_counter()
    G = E.green(0, 0, ngf=100, lmats=512)
    t2 = time.perf_counter()
    C = E.chi([0.5], [-0.5], ngf=100, lmats=64)
    t3 = time.perf_counter()
    n, e0, z = E.info()
    out["thermal_ns8"] = {"workload": "Ns=8 model, all 81 sectors, beta=10, cutoff 1e-6",
                          "diag3_s": round(t1 - t0, 3), "states_kept": n,
                          "green_s": round(t2 - t1, 3), "chi_s": round(t3 - t2, 3),
                          "chi_static": round(float(C[0].real), 6)}
    return out


def bench_eph(edx, torch, a):
    """Holstein phonon (N_ph = 4, D_ph = 5) on the Ns=14 7/7 sector: FP32 H.v
    (D = 3432^2 x 5 = 58.9M) against the purely electronic product of the same
    sector (the phonon pass is the difference)."""
    from paper_2105_06806_amd import inputs
    m0 = inputs.make_model(1, 13, 2.0, seed=inputs.SEED_BASE["ns16"] + 14)
    m = dict(m0, nph=4, w0=0.5, g=np.array([0.4]))
    Se = edx.build_sector(m0, 7, 7)
    Sp = edx.build_sector(m, 7, 7)
    el = _hv_rate(edx, torch, Se, a)
    ph = _hv_rate(edx, torch, Sp, a)
    return {"workload": f"Ns=14 7/7 with a Holstein mode N_ph=4: D={Sp.dim} (electronic {Se.dim})",
            "hv_f32": ph, "electronic_hv_f32": el,
            "phonon_pass_share": round(1 - 5 * el["us"] / ph["us"], 4)}


def bench_shard(edx, torch, a, p=8):
    """The per-GPU work of the column-distributed product (Sec. 3.2) at the
    Ns=16 8/8 shapes for p = 8 GPUs, measured on this GPU: the spin-up pass +
    H_d on a D_up x D_dw/p block, the spin-down pass on a D_dw x D_up/p block of
    the transposed vector, and the local transposes of one share (the all-to-all
    packing); the xGMI transfer is a model (7 links x 153 GB/s, each peer over
    its own link), not a measurement."""
    from paper_2105_06806_amd import inputs
    m, [sec] = inputs.workload("ns16")
    S = edx.build_sector(m, *sec)
    ld, ldt = S.ld, (S.ddw + 31) // 32 * 32
    gen = torch.Generator(device="cuda").manual_seed(6)
    v = edx.pad(S, torch.rand(S.dim, dtype=torch.float32, device="cuda", generator=gen) * 2 - 1)
    w = torch.empty_like(v)
    vt = torch.zeros(ldt * S.dup, dtype=torch.float32, device="cuda")
    wt = torch.empty_like(vt)
    cb = (S.ddw + p - 1) // p
    edx.transpose(v, S.dup, S.ddw, ld, vt, ldt)
    share = torch.zeros(cb * S.dup, dtype=torch.float32, device="cuda")

    def timed(fn, reps=20):
        for _ in range(3):
            fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for x, y in ev:
            x.record()
            fn()
            y.record()
        torch.cuda.synchronize()
        return float(np.mean([x.elapsed_time(y) for x, y in ev])) * 1e3

    t_up = timed(lambda: edx.hv_block(S, 0, v, w, ld, 0, cb))
    t_dw = timed(lambda: edx.hv_block(S, 1, vt, wt, ldt, 0, cb))
    t_tr = timed(lambda: edx.transpose(v, S.dup, cb, ld, share, cb))
    share_bytes = S.dup * cb * 4
    t_link = share_bytes / p / 153e9 * 1e6        # one peer message per link
    t_whole = _hv_rate(edx, torch, S, a, reps=10)["us"]
    del v, w, vt, wt, share
    torch.cuda.empty_cache()
    comp = t_up + t_dw + 2 * t_tr
    return {"workload": f"Ns=16 8/8 FP32 split over p={p}: blocks {S.dup}x{cb} and {S.ddw}x{cb}",
            "up_pass_us": round(t_up, 1), "down_pass_us": round(t_dw, 1),
            "local_transpose_us": round(t_tr, 1), "per_gpu_compute_us": round(comp, 1),
            "xgmi_model_us_per_transpose": round(t_link, 1),
            "per_gpu_total_model_us": round(comp + 2 * t_link, 1),
            "one_gpu_whole_hv_us": t_whole,
            "model_speedup_vs_one_gpu": round(t_whole / (comp + 2 * t_link), 2)}


def bench_hv_multi(edx, torch, a):
    """Several bath sets of one sector shape per product (edx_hv_multi): the
    k vectors interleaved, one spin-down gather serving all k.  Per-vector
    algorithmic GB/s (k D (s + s) bytes per launch, s = element size) for
    k = 1, 2, 4, 8 on the Ns=12 6/6 and Ns=14 7/7 sectors (the batch
    workload's large shapes) and the k that fit in LDS on the Ns=16 8/8
    sector, FP32 and FP64, beside the single-vector fused pass
    (fused_single, the sector's default plan)."""
    from paper_2105_06806_amd import inputs
    out = {"note": "HIP events around each edx_hv_multi call, which also copies the k sets' "
                   "tables into its workspace (a batched solve does that once); the kernel "
                   "alone: profiles/hv_multi_counters.md"}
    # the calibration kernel of the counter summaries runs in the same process
    out["copy_gbs"] = round(copy_bandwidth(torch), 1)
    for ns, sec, ks in ((12, (6, 6), (1, 2, 4, 8)), (14, (7, 7), (1, 2, 4, 8)), (16, (8, 8), (1, 2))):
        for dt, tdt in (("f32", torch.float32), ("f64", torch.float64)):
            row = {}
            for k in ks:
                ms = [inputs.make_model(1, ns - 1, 2.0, seed=inputs.SEED_BASE["batch"] + 3 * b + ns)
                      for b in range(k)]
                Ss = [edx.build_sector(m, *sec) for m in ms]
                n = Ss[0].ld * Ss[0].ddw * k
                if 16 + Ss[0].dup * k * (8 if dt == "f64" else 4) > 150 * 1024:
                    continue
                gen = torch.Generator(device="cuda").manual_seed(8)
                v = torch.rand(n, dtype=tdt, device="cuda", generator=gen) * 2 - 1
                w = torch.empty_like(v)
                ws = edx.alloc_workspace(edx.lib.edx_hv_multi_workspace_bytes(
                    edx._handles(Ss), k, edx.F32 if dt == "f32" else edx.F64))
                for _ in range(3):
                    edx.hv_multi(Ss, v, w, ws=ws)
                torch.cuda.synchronize()
                ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                      for _ in range(10)]
                for x, y in ev:
                    x.record()
                    edx.hv_multi(Ss, v, w, ws=ws)
                    y.record()
                torch.cuda.synchronize()
                us = float(np.mean([x.elapsed_time(y) for x, y in ev])) * 1e3
                alg = k * Ss[0].dim * 2 * v.element_size()
                row[f"k{k}"] = {"us": round(us, 1), "us_per_vector": round(us / k, 1),
                                "gbs": round(alg / (us * 1e-6) / 1e9, 1),
                                "frac": round(alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
                if k == 1:
                    # the single-vector fused pass on the sector's default plan
                    for _ in range(3):
                        edx.hv(Ss[0], v, w, ld=Ss[0].ld)
                    torch.cuda.synchronize()
                    for x, y in ev:
                        x.record()
                        edx.hv(Ss[0], v, w, ld=Ss[0].ld)
                        y.record()
                    torch.cuda.synchronize()
                    us1 = float(np.mean([x.elapsed_time(y) for x, y in ev])) * 1e3
                    row["fused_single"] = {"us": round(us1, 1),
                                           "gbs": round(alg / (us1 * 1e-6) / 1e9, 1)}
                del v, w, ws
                torch.cuda.empty_cache()
            out[f"ns{ns}_{dt}"] = row
    return out


def cpu_baseline(m, sec, elem_bytes, budget_s=15.0, max_procs=16):
    """The oracle's row-by-row H.v on a bounded sample of output rows: one core
    (calibration), then one oracle process per core (up to max_procs, the host
    share of one GPU) on disjoint samples; value = aggregate rate."""
    from oracle import fock
    D = 12870 * 12870
    rng = np.random.default_rng(0)
    v = rng.uniform(-1, 1, size=D)
    fock.hv_rows(m, *sec, v, rng.choice(D, size=20000, replace=False))   # warm-up
    n = 200000
    rows = rng.choice(D, size=n, replace=False)
    t0 = time.perf_counter()
    fock.hv_rows(m, *sec, v, rows)
    dt1 = time.perf_counter() - t0
    rate1 = n / dt1
    del v, rows
    cpu = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    nproc = max(1, min(max_procs, os.cpu_count() or 1))
    per = int(min(8_000_000, max(n, rate1 * budget_s)))
    t0 = time.perf_counter()
    # one plain child process per core (fresh interpreters that never touch
    # the GPU), each waited for, so nothing outlives the benchmark
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    import subprocess
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker",
                               str(100 + i), str(per)], stdout=subprocess.PIPE, env=env, text=True)
             for i in range(nproc)]
    res = []
    for pr in procs:
        out, _ = pr.communicate()
        if pr.returncode == 0 and out.strip():
            k, sec_ = out.split()[-2:]
            res.append((int(k), float(sec_)))
    if len(res) == nproc:
        tot = sum(r[0] for r in res)
        span = max(r[1] for r in res)
    else:                            # report the one-core figure only
        log(f"cpu baseline: {nproc - len(res)} worker(s) failed; one core only")
        nproc, tot, span = 1, n, dt1
    wall = time.perf_counter() - t0
    rate = tot / span
    return {"value": round(rate * elem_bytes / 1e9, 4), "unit": "GB/s", "cores": nproc, "kind": "oracle",
            "sample": f"{nproc} oracle processes x {per} random output rows of the Ns=16 8/8 sector "
                      f"(FP64, second quantisation per row), {span:.1f} s each ({wall:.0f} s with "
                      f"start-up) on {cpu} ({os.cpu_count()} visible); value = aggregate rows/s x "
                      f"{elem_bytes} B (the GPU's algorithmic bytes per FP64 element)",
            "rows_per_s": round(rate, 1), "rows_per_s_one_core": round(rate1, 1),
            "full_hv_s_extrapolated": round(D / rate, 1)}


def bench_ns12(edx):
    from paper_2105_06806_amd import inputs
    g = np.load(os.path.join(ROOT, "tests", "golden", "ns12.npz"))
    m, [sec] = inputs.workload("ns12")
    S = edx.build_sector(m, *sec)
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0, psi, rep, _ = edx.lanczos_ground_state(S, niter=512, tol=1e-14, rtol=1e-10, seed=21)
    t1 = time.perf_counter()
    G, gr = edx.green_cf(S, psi, e0, 0, 0, ngf=200, beta=float(g["beta"]), lmats=int(g["lmats"]))
    t2 = time.perf_counter()
    return {"workload": "Norb=1 Ns=12 6/6 D=853776 FP64, G spin up, 4096 Matsubara, beta=200, depth 200",
            "gs_s": round(t1 - t0, 4), "gf_s": round(t2 - t1, 4), "iters": rep["iters"],
            "e0": e0, "e0_rel_err": abs(e0 - float(g["e0"])) / abs(float(g["e0"])),
            "g_rel_err": float(np.abs(G - g["g"]).max() / np.abs(g["g"]).max()),
            "wp_plus_wh": gr["wp"] + gr["wh"]}


def _resid64(edx, torch, S, psi, e):
    """|H psi - e psi| / |psi| with the FP64 product on psi cast to FP64
    (measurement of a vector's accuracy, independent of its storage type)."""
    x = edx.pad(S, psi.double())
    y = torch.empty_like(x)
    edx.hv(S, x, y, ld=S.ld)
    r = float((y - e * x).norm() / x.norm())
    del x, y
    return r


def bench_ns15o3(edx):
    """Precision mode on Norb=3, Ns=15 7/7 (D=41.4M): FP64 against the stored
    oracle values; FP32 Krylov vectors (FP64 scalars) with no / local / full
    re-orthogonalisation and with the basis kept, with the energy stop rule and
    with a residual stop rule; each psi0's FP64 residual; and the FP32 vector
    refined by a short FP64 run started from it, with G from FP32 and from
    FP64 Krylov vectors."""
    from paper_2105_06806_amd import inputs
    path = os.path.join(ROOT, "tests", "golden", "ns15o3.npz")
    g = np.load(path)
    m, [sec] = inputs.workload("ns15o3")
    S = edx.build_sector(m, *sec)
    E = float(g["e0"])
    lm, beta = int(g["lmats"]), float(g["beta"])
    # G_up + G_dw per orbital (orbital 0 only without the per-orbital file)
    gref = [g["g_up"] + g["g_dw"]]
    path_orb = os.path.join(ROOT, "tests", "golden", "ns15o3_orb.npz")
    if os.path.exists(path_orb):
        gref = list(np.load(path_orb)["g_sum"])
    import torch
    out = {"workload": "Norb=3 Nbath=4 Ns=15 7/7 D=41409225, U=3 J=0.5; G = G_up + G_dw of each of "
                       f"{len(gref)} orbital(s) (the ground level is spin-swap degenerate), 1024 "
                       "Matsubara, beta=200; g_rel_err = the largest over the orbitals"}

    def gerr(psi, e0):
        errs = []
        for orb, ref in enumerate(gref):
            Gu, _ = edx.green_cf(S, psi, e0, orb, 0, ngf=200, beta=beta, lmats=lm)
            Gd, _ = edx.green_cf(S, psi, e0, orb, 1, ngf=200, beta=beta, lmats=lm)
            errs.append(float(np.abs(Gu + Gd - ref).max() / np.abs(ref).max()))
        return max(errs)

    runs = [("f64", 0, 0.0), ("f32", 0, 0.0), ("f32", 1, 0.0), ("f32", 2, 0.0), ("f32", 3, 0.0),
            ("f32", 0, 1e-6), ("f32", 1, 1e-6)]
    keep = None
    for vt, ro, rt in runs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0, psi, rep, st = edx.lanczos_ground_state(
            S, vtype=vt, reorth=ro, niter=600 if vt == "f64" else 400,
            tol=1e-14 if vt == "f64" else 1e-9, rtol=1e-10 if vt == "f64" else rt, seed=4,
            allow=(edx.EDX_E_NOCONV, edx.EDX_E_DEGENERATE))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = {"gs_s": round(t1 - t0, 3), "iters": rep["iters"], "status": edx.status_str(st),
             "e0_rel_err": abs(e0 - E) / abs(E), "e1_minus_e0": rep["e1"] - e0,
             "psi_resid_f64": _resid64(edx, torch, S, psi, e0)}
        t2 = time.perf_counter()
        r["g_rel_err"] = gerr(psi, e0)
        r["gf_s"] = round(time.perf_counter() - t2, 3)
        out[f"{vt}_reorth{ro}" + (f"_rtol{rt:g}" if rt else "")] = r
        if vt == "f32" and ro == 0 and not rt:
            keep = (psi, e0, r["gs_s"])
        else:
            del psi
        torch.cuda.empty_cache()
    # FP64 refinement of the FP32 (plain) ground vector: a short FP64 run from it
    psi32, e32, t32 = keep
    start = psi32.double().contiguous()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ef, pf, rf, st = edx.lanczos_ground_state(S, vtype="f64", niter=600, tol=1e-14, rtol=1e-10,
                                              seed=4, start=start,
                                              allow=(edx.EDX_E_NOCONV, edx.EDX_E_DEGENERATE))
    torch.cuda.synchronize()
    tpol = time.perf_counter() - t0
    del start
    r = {"f32_gs_s": t32, "f64_polish_s": round(tpol, 3), "polish_iters": rf["iters"],
         "status": edx.status_str(st), "e0_rel_err": abs(ef - E) / abs(E),
         "psi_resid_f64": _resid64(edx, torch, S, pf, ef), "g_rel_err_f64_krylov": gerr(pf, ef)}
    pf32 = pf.float()
    r["g_rel_err_f32_krylov"] = gerr(pf32, ef)
    out["f32_then_f64_polish"] = r
    del pf, pf32, psi32
    torch.cuda.empty_cache()
    return out


def bench_batch(edx, torch):
    from paper_2105_06806_amd import inputs
    jobs = inputs.batch_jobs()
    t0 = time.perf_counter()
    secs = [edx.build_sector(m, a, b) for (_, m, a, b) in jobs]
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    kw = dict(vtype="f32", niter=512, tol=1e-9, check_every=4, seed=17)
    ws = edx.alloc_workspace(edx.batch_workspace_bytes(secs, "f32", 8))   # both phase layouts
    t0 = time.perf_counter()
    tiles = edx.batch_autotune(secs, ws=ws, **kw)
    tt = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, kms = edx.batch_ground_state(secs, tiles=tiles, ws=ws, **kw)
    tbatch = time.perf_counter() - t0
    # the same solves one after another through the plain API
    lw = max(edx.workspace_bytes(s, edx.WS_LANCZOS, "f32", 512) for s in secs)
    lws = edx.alloc_workspace(lw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = [edx.lanczos_ground_state(s, want_psi=False, ws=lws, check_every=4,
                                      allow=(edx.EDX_E_NOCONV, edx.EDX_E_DEGENERATE), **{
                                          k: v for k, v in kw.items() if k != "check_every"})[0]
             for s in secs]
    tseq = time.perf_counter() - t0
    dev = [abs(r["e0"] - p) / abs(p) for r, p in zip(res, plain)]
    ok = sum(1 for r in res if r["status"] == 0)
    D = np.array([s.dim for s in secs], dtype=np.int64)
    wm = int(tiles["wide_min_dim"])
    thr = 2_000_000 if wm == 0 else (None if wm < 0 else wm)
    in_launch = D < thr if thr else np.ones(len(D), bool)
    # the whole-GPU jobs one by one instead of in multi-set groups
    wso = edx.alloc_workspace(edx.batch_workspace_bytes(secs, "f32", tiles["lane_wgs"],
                                                        tiles["wide_min_dim"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res_one, _ = edx.batch_ground_state(secs, tiles=dict(tiles, multi_k=1), ws=wso, **kw)
    tone = time.perf_counter() - t0
    del wso
    dev_one = [abs(r["e0"] - p) / abs(p) for r, p in zip(res_one, plain)]
    # the alternative the autotuner also timed: every job inside the persistent
    # launch (no whole-GPU path), same tiles
    tiles_all = dict(tiles, wide_min_dim=-1)
    wsa = edx.alloc_workspace(edx.batch_workspace_bytes(secs, "f32", tiles["lane_wgs"], -1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res_all, _ = edx.batch_ground_state(secs, tiles=tiles_all, ws=wsa, **kw)
    tall = time.perf_counter() - t0
    del wsa
    dev_all = [abs(r["e0"] - p) / abs(p) for r, p in zip(res_all, plain)]
    return {"workload": f"{len(secs)} ground states: 64 bath sets (Ns=10/12/14), N_up,N_dw in "
                        f"[Ns/2-2, Ns/2+2], D {D.min()}..{D.max()}, sum D {D.sum()}, FP32 vectors, "
                        f"tol 1e-9",
            "solves_per_s": round(len(secs) / tbatch, 1), "batch_s": round(tbatch, 3),
            "batch_kernel_ms": round(kms, 1), "plain_sequential_s": round(tseq, 3),
            "plain_solves_per_s": round(len(secs) / tseq, 1), "speedup": round(tseq / tbatch, 2),
            "converged": ok, "max_rel_dev_vs_plain": float(max(dev)), "build_s": round(tb, 2),
            "autotune_s": round(tt, 2), "lane_wgs": tiles["lane_wgs"],
            "wide_min_dim": tiles["wide_min_dim"],
            "jobs_in_persistent_launch": int(in_launch.sum()),
            "sum_D_share_in_persistent_launch": round(float(D[in_launch].sum() / D.sum()), 4),
            "whole_gpu_jobs_one_by_one": {"batch_s": round(tone, 3),
                                          "solves_per_s": round(len(secs) / tone, 1),
                                          "converged": sum(1 for r in res_one if r["status"] == 0),
                                          "max_rel_dev_vs_plain": float(max(dev_one))},
            "all_in_persistent_launch": {"batch_s": round(tall, 3),
                                         "solves_per_s": round(len(secs) / tall, 1),
                                         "converged": sum(1 for r in res_all if r["status"] == 0),
                                         "max_rel_dev_vs_plain": float(max(dev_all))}}


def _fcfs(arr, svc):
    """Latencies of a single first-come-first-served server (one request at a
    time, the plain path) fed with arrival times arr and service times svc."""
    done, lat = 0.0, []
    for a_, s_ in zip(arr, svc):
        start = max(a_, done)
        done = start + s_
        lat.append(done - a_)
    return np.array(lat), done


PROFILE_SERVE = os.path.join(ROOT, "profiles", "serve_sweep_ns16.md")


def serve_sweep_from_profile():
    """The committed full-size serving sweep (1000 requests per rate, Ns
    10..16, measured by this file's serve section split over several runs):
    quoted, not measured by this run.  `rates`: the seven-rate sweep, taken
    with at most half the slots on large requests; `current_policy`: the
    rates measured with the library's current admission (one large request
    at a time)."""
    if not os.path.exists(PROFILE_SERVE):
        return None
    txt = open(PROFILE_SERVE).read()

    def rows(tag):
        out = []
        for mr in re.finditer(r"^" + tag + r"\[([0-9.]+)\]:(.*)$", txt, re.M):
            row = {"x_plain_capacity": float(mr.group(1))}
            for kv in mr.group(2).split():
                k, v = kv.split("=")
                row[k] = float(v) if "." in v or "e" in v else int(v)
            out.append(row)
        return out

    full = rows("rate")
    if not full:
        return None
    return {"source": "profiles/serve_sweep_ns16.md (quoted, not measured by this run)",
            "policy": "at most half the slots on requests of 1 GiB or more", "rates": full,
            "current_policy": {"policy": "one request of 1 GiB or more at a time",
                               "rates": rows("rate_current")}}


def bench_serve(edx, torch, full, nreq=None, ns_hi=None, rates=None, cap_given=None,
                plain_file=None, offset=0, span=None, dump=None):
    """Serving: a Poisson stream of ground state + G requests (Norb in {1,2},
    Ns 10..16, U in [1,6]; FP32 vectors) served with continuous batching, at
    offered rates that are multiples of the measured one-at-a-time capacity.
    Plain: every request of the stream solved one after another (its service
    time); the same arrivals fed to one first-come-first-served plain server
    give the plain latencies at each rate.  The default run uses fewer
    requests per rate than --full (1000 per rate at seven rates) so that the
    whole benchmark stays within a few minutes."""
    from paper_2105_06806_amd import inputs
    ns_hi = ns_hi or 16
    nreq = nreq or (1000 if full else 120)
    kw = dict(niter=512, tol=1e-9, seed=5, check_every=4)
    gkw = dict(ngf=200, lmats=1024, beta=200.0)
    reqs = inputs.serve_requests(nreq, ns_lo=10, ns_hi=ns_hi)
    # a part of the stream (requests offset .. offset + span - 1, their own
    # arrival times): one rate's sweep split over several runs
    span = span or (nreq - offset)
    svc = None
    if plain_file and os.path.exists(plain_file):
        svc = json.load(open(plain_file))["service_s"][:nreq]
        if len(svc) < nreq:
            svc = None
    if svc is None:
        # one-at-a-time plain solves of every request of the stream
        svc = []
        for (m, a, b) in reqs:
            torch.cuda.synchronize()
            ts = time.perf_counter()
            S = edx.build_sector(m, a, b)
            e0, psi, _, _ = edx.lanczos_ground_state(
                S, vtype="f32", allow=(edx.EDX_E_NOCONV, edx.EDX_E_DEGENERATE), **kw)
            edx.green_cf(S, psi, e0, 0, 0, **gkw)
            svc.append(time.perf_counter() - ts)
            del S, psi
            if len(svc) % 50 == 0:
                log(f"serve plain: {len(svc)}/{nreq} requests, {sum(svc):.1f} s")
        if plain_file:
            json.dump({"service_s": svc, "nreq": nreq, "ns_hi": ns_hi}, open(plain_file, "w"))
    svc = np.array(svc)
    cap_here = len(svc) / svc.sum()                      # plain requests/s
    cap = cap_given or cap_here
    ns_mix = [inputs.ns_of(m) for (m, _, _) in reqs]
    out = {"workload": f"Poisson stream of ground state + G requests, Norb in {{1,2}}, Ns 10..{ns_hi} "
                       f"(largest 12870^2 = 165,636,900), U in [1,6], FP32 vectors, G depth "
                       f"{gkw['ngf']} on {gkw['lmats']} frequencies, {nreq} requests per rate",
           "requests_per_rate": nreq,
           "ns16_share": round(sum(1 for x in ns_mix if x == 16) / len(ns_mix), 3),
           "plain_solves_per_s": round(cap_here, 3), "rate_unit_per_s": round(cap, 3),
           "plain_service_p50_s": round(float(np.median(svc)), 4),
           "plain_service_p99_s": round(float(np.percentile(svc, 99)), 4),
           "rates": []}
    srv = edx.Server(hbm_budget=96 << 30, max_slots=8, vtype="f32", **gkw, **kw)
    facs = rates or ((1.0, 2.0) if not full else (0.25, 0.5, 0.75, 0.9, 1.0, 1.25, 2.0))
    for fac in facs:
        rate = fac * cap
        arr = inputs.poisson_arrivals(nreq, rate, seed=int(fac * 1000))[offset:offset + span]
        arr = arr - arr[0]
        part = reqs[offset:offset + span]
        t_begin = edx.Server.clock()
        tickets = []
        for (m, a, b), ta in zip(part, arr):
            wait = t_begin + ta - edx.Server.clock()
            if wait > 0:
                time.sleep(wait)
            tickets.append(srv.submit(m, a, b))
            if len(tickets) % 50 == 0:
                log(f"serve x{fac}: {len(tickets)}/{len(part)} submitted")
        res = []
        for t in tickets:
            res.append(srv.poll(t))
            if len(res) % 100 == 0:
                log(f"serve x{fac}: {len(res)}/{len(part)} done")
        t_end = max(r["t_done"] for r in res)
        lat = np.array([r["t_done"] - r["t_submit"] for r in res])
        first = min(r["t_submit"] for r in res)
        plat, pdone = _fcfs(arr, svc[offset:offset + span])
        out["rates"].append({"offered_per_s": round(rate, 3), "x_plain_capacity": fac,
                             "n": len(res), "first_request": offset,
                             "solves_per_s": round(len(res) / (t_end - first), 3),
                             "p50_s": round(float(np.percentile(lat, 50)), 4),
                             "p99_s": round(float(np.percentile(lat, 99)), 4),
                             "plain_fcfs_solves_per_s": round(len(res) / (pdone - arr[0]), 3),
                             "plain_fcfs_p50_s": round(float(np.percentile(plat, 50)), 4),
                             "plain_fcfs_p99_s": round(float(np.percentile(plat, 99)), 4),
                             "ok": int(sum(r["status"] in (0, edx.EDX_E_DEGENERATE) for r in res)),
                             "degenerate": int(sum(r["status"] == edx.EDX_E_DEGENERATE
                                                   for r in res))})
        log(f"serve x{fac}: {out['rates'][-1]}")
        if dump:
            raw = json.load(open(dump)) if os.path.exists(dump) else {}
            raw[f"x{fac}_from{offset}"] = {"served_s": lat.tolist(), "plain_fcfs_s": list(map(float, plat)),
                                          "first_submit": first, "last_done": t_end,
                                          "plain_first_arrival": float(arr[0]), "plain_last_done": float(pdone)}
            json.dump(raw, open(dump, "w"))
    srv.close()
    out["full_sweep"] = serve_sweep_from_profile()
    return out


def main():
    a = parse()
    if a.cpu_worker:
        _cpu_rows_worker(*a.cpu_worker)
        return
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the design notes describe how the sector would shard)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2105_06806_amd import edx, inputs

    log(f"device: {torch.cuda.get_device_properties(0).name}")
    sections = {"hv_ns16o2": lambda: bench_hv_o2(edx, torch, a),
                "hv_multi": lambda: bench_hv_multi(edx, torch, a),
                "hv_kanamori": lambda: bench_hv_kanamori(edx, torch, a),
                "orbital": lambda: bench_orbital(edx, torch, a),
                "lowest_thermal": lambda: bench_lowest_and_thermal(edx, torch, a),
                "eph": lambda: bench_eph(edx, torch, a),
                "shard": lambda: bench_shard(edx, torch, a),
                "ns12": lambda: bench_ns12(edx), "ns15o3": lambda: bench_ns15o3(edx),
                "batch": lambda: bench_batch(edx, torch),
                "serve": lambda: bench_serve(
                    edx, torch, a.full, a.serve_n, a.serve_ns_hi,
                    tuple(float(x) for x in a.serve_rates.split(",")) if a.serve_rates else None,
                    a.serve_cap, a.serve_plain, a.serve_offset, a.serve_span, a.serve_dump)}
    if a.only:
        out = {}
        for name in a.only.split(","):
            log(f"{name} ...")
            out[name] = sections[name]()
            log(f"{name}: {out[name]}")
        print(json.dumps(out), flush=True)
        return
    m, [sec] = inputs.workload("ns16")
    S = edx.build_sector(m, *sec)
    D = S.dim
    ld = S.ld   # the Krylov vectors' column stride (columns start on 128-byte lines)
    wup = S.hop_nnz(0)[1]
    wpad = 8 if wup <= 8 else (16 if wup <= 16 else 24)
    gen = torch.Generator(device="cuda").manual_seed(1)
    res = {}
    for dt_name, tdt in (("f64", torch.float64), ("f32", torch.float32)):
        v = edx.pad(S, torch.rand(D, dtype=tdt, device="cuda", generator=gen) * 2 - 1)
        w = torch.empty_like(v)
        fixed = a.plan64 if dt_name == "f64" else a.plan
        if fixed:
            f = [int(x) for x in fixed.split(",")]
            edx.set_plan(S, dt_name, mode=f[0], col_cols=f[1], col_threads=f[2], row_rows=f[3],
                         row_cols=f[4], col_order=f[5] if len(f) > 5 else 0)
            plan = edx.get_plan(S, dt_name)
        else:
            plan, tune_us = edx.autotune_hv(S, v, w, reps=a.tune_reps, ld=ld)
            log(f"{dt_name}: autotuned plan {plan} ({tune_us:.1f} us)")
        ms, wall = time_hv(edx, torch, S, v, w, a.steps, a.warmup, ld=ld)
        esz = 4 if dt_name == "f32" else 8
        alg = D * 2 * esz
        # same plan on dense vectors (column stride D_up), for comparison
        vd, wd = edx.unpad(S, v), torch.empty(D, dtype=tdt, device="cuda")
        msd, _ = time_hv(edx, torch, S, vd, wd, max(5, a.steps // 5), 2)
        single = plan["mode"] in (0, 2)
        tname = "double" if dt_name == "f64" else "float"
        kernel = (f"k_hv_fused<{tname},{wpad},{wpad},{plan['col_cols']},false,false,true>"
                  if plan["mode"] == 2 else
                  ("k_hv_small" if plan["mode"] == 0 else f"k_hv_row + k_hv_col<{tname},{wpad}>"))
        traffic, tstate = traffic_from_profile(plan, dt_name) if single else (None, "two kernels")
        gbs = alg / (ms.mean() * 1e-3) / 1e9
        res[dt_name] = {"ms_mean": float(ms.mean()), "ms_median": float(np.median(ms)), "wall_s": wall,
                        "plan": plan, "gbs": gbs, "alg_bytes": alg, "dense_us": float(msd.mean()) * 1e3,
                        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                                     "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                                     "traffic": traffic, "kernel": kernel,
                                     "alg_bytes_per_launch": alg, "traffic_source": tstate}}
        log(f"{dt_name}: {ms.mean() * 1e3:.1f} us/H.v, {gbs:.0f} GB/s algorithmic "
            f"(dense layout {msd.mean() * 1e3:.1f} us)")
        del v, w, vd, wd
        torch.cuda.empty_cache()
    r64, r32 = res["f64"], res["f32"]
    copy_gbs = copy_bandwidth(torch)
    log(f"copy: {copy_gbs:.0f} GB/s")

    def views(r):
        t = r["roofline"]["traffic"]
        sec_ = r["ms_mean"] * 1e-3
        return {"effective_gbs": round(r["gbs"], 1),
                "beyond_l2_gbs": round(t / sec_ / 1e9, 1) if t else None,
                "beyond_l2_over_algorithmic": round(t / r["alg_bytes"], 3) if t else None,
                "copy_gbs": round(copy_gbs, 1),
                "effective_frac_of_copy": round(r["gbs"] / copy_gbs, 4),
                "median_us": round(r["ms_median"] * 1e3, 1)}

    out = {
        "metric": "H·v GB/s & %HBM peak at Ns=16; batched solves/s, p50/p99 vs plain",
        "value": round(r64["gbs"], 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(r64["ms_mean"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "H.v on the half-filled Ns=16 sector: Norb=1, Nbath=15, N_up=N_dw=8, "
                               "D=165636900, FP64 vectors, symmetrised random bath, U=2",
                   "seed": inputs.SEED_BASE["ns16"], "column_stride": ld},
        "hv_per_s": round(1e3 / r64["ms_mean"], 1),
        "plan_f64": r64["plan"],
        "f64_dense_layout_us": round(r64["dense_us"], 1),
        "roofline": r64["roofline"],
        # the views of the headline: algorithmic bytes / time, counter
        # (beyond-L2: MALL and HBM) bytes / time, a plain device copy
        "bandwidth": views(r64),
        "f32": {"gbs": round(r32["gbs"], 1), "us": round(r32["ms_mean"] * 1e3, 1),
                "hv_per_s": round(1e3 / r32["ms_mean"], 1),
                "dense_layout_us": round(r32["dense_us"], 1), "plan": r32["plan"],
                "roofline": r32["roofline"], "bandwidth": views(r32)},
    }
    if not a.quick:
        for name, fn in sections.items():
            t0 = time.perf_counter()
            log(f"{name} ...")
            try:
                out[name] = fn()
            except Exception as ex:      # report, keep the headline
                out[name] = {"error": repr(ex)}
            log(f"{name}: {time.perf_counter() - t0:.1f} s: {out[name]}")
            torch.cuda.empty_cache()
    if not a.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(m, sec, 16)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
