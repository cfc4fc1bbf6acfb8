"""Benchmark: HS-field sweeps per second of the kagome DQMC hot path on one GPU.

One step = one full sweep: a pass over all L_tau slices (window decisions,
delayed rank-k flushes and FFT wraps, a QR-stabilization every n_stab
slices), on seeded synthetic fields and uniforms that are resident in device
memory before the timed region starts.  Passes alternate upward and downward
(the standard sweep order of DQMC; each pass keeps the stabilization stack
the next one needs), or are all upward with --passes up (then every pass
ends by rebuilding the left stack).  Each pass's uniforms are copied into one
fixed device buffer first, so every timed pass replays the HIP graphs
captured during the warm-up.

Prints ONE JSON line.  The headline is the L=12, U=-4, beta=8 FP64 workload
(delay k=32).  `roofline` is for the dominant kernel (largest share of the
kernel time, from HIP events recorded by the library around every launch);
`cpu_baseline` times the CPU oracle on a bounded sample of the same workload.
`extra` holds the other workloads of the metric, each with its own steps and
ms_per_step: L=24 and L=18 in FP64 and mixed precision, the batch of 64
uneven chains in both precisions, and the FFT wrap's GB/s at L=12, 18, 24.
No rate is quoted for a run whose chains drifted: every run ends with the
library's health check (the wrap error of every stabilization against the
context's tolerance), and a failed check replaces the rate by the reason.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

import numpy as np  # noqa: E402

import seeded_inputs as si  # noqa: E402

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFS = 78.6           # MI355X FP64 (vector and matrix)
F16_PEAK_TFS = 2500.0          # MI355X dense FP16/BF16 MFMA

CONFIGS = {"c1": si.C1, "c2": si.C2, "c3": si.C3, "c5": si.C5, "c4": None}
AUTOTUNED = ("c3", "c4", "c5")   # workloads whose delay rank and FFT tile come from the autotuner


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def schedule(delay_k, window, fft_tile, w, prec, n_stab, autotuned):
    """(delay_k, window, fft_tile, from_autotuner): explicit values win; for
    autotuned workloads the cached autotuner choice (same lattice, beta,
    precision and interval) is used when present, else the workload default."""
    t = None
    if autotuned and not delay_k:
        from paper_2608_03894_amd import autotune
        t = autotune.lookup(w.L, w.U, w.beta, w.dtau, prec, n_stab, any_U=True)
    k = delay_k or (t["delay_k"] if t else w.delay_k)
    window = window or (t["window"] if t else 0)
    tile = fft_tile or (t["fft_tile"] if t else 0)
    return k, window, tile, t is not None


def mixed_interval(w, prec):
    """Stabilization interval of a mixed-precision run: the autotuner's choice
    (the longest interval whose error against the FP64 path stays within
    1e-5) with its error table, or (None, None) when it has not been
    measured for this lattice."""
    from paper_2608_03894_amd import autotune
    e = autotune.lookup_interval(w.L, w.U, w.beta, w.dtau, prec)
    if e is None:
        return None, None
    return e["n_stab"], e


def cpu_baseline(w, n_slices):
    """Oracle (NumPy/SciPy FP64) on the first n_slices slices of a sweep of the
    same workload, including its stabilizations; scaled to sweeps/s."""
    from oracle import dqmc
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [os.cpu_count()])
    except Exception:
        threads = os.cpu_count()
    m = dqmc.Model.from_workload(w, mu=-1.0)
    f = si.ising_fields(w.L, m.L_tau, w.seed)
    u = si.metropolis_uniforms(w.L, m.L_tau, w.seed)[0]
    g0 = dqmc.green_scratch(m, f, 0)
    t0 = time.perf_counter()
    dqmc.sweep(m, f, g0, uniforms=u, k=w.delay_k, n_stab=w.n_stab, record=False, l_stop=n_slices)
    dt = time.perf_counter() - t0
    per_sweep = dt * m.L_tau / n_slices
    return {"value": 1.0 / per_sweep, "unit": "sweeps/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n_slices} of {m.L_tau} slices (incl. {n_slices // w.n_stab} stabilizations) "
                      f"of one sweep, {dt:.1f} s, scaled by L_tau/{n_slices}"}


CU_FP64_TFS = FP64_PEAK_TFS / 256   # one compute unit's share (4 SIMDs x 16 FP64 lanes x 2 x 2.4 GHz)


def qr_panel_flops(n, b=16):
    """Householder flops of all 16-column panels of one n x n QR
    (2 m b^2 - 2 b^3 / 3 per m x b panel)."""
    f, j = 0.0, 0
    while j < n:
        m = n - j
        bb = min(b, m)
        f += 2.0 * m * bb * bb - 2.0 * bb ** 3 / 3.0
        j += bb
    return f


def qr_panels(n, b=16):
    return (n + b - 1) // b


def kernel_rooflines(prof, N, prec, k_avg, a_avg, windows_per_launch=1):
    """{phase: roofline dict} from the profiled (HIP-event) per-phase totals.

    achieved = algorithmic bytes or flops per launch / average launch time:
      wrap_cols, wrap_rows, bmul: 2 N^2 s bytes (G read once, written once),
          against HBM;
      flush (rank-k product of k = accepted flips per flush group) and
      flush_decide (the fused window launch, rank a = the window's accepts):
          bytes 2 N^2 s + 2 N r s (G read and written, the two factors read),
          flops 2 N^2 r.  Their arithmetic intensity (about r/8 flop/B in
          FP64) lies below the FP64 ridge (78.6 TFLOP/s / 8 TB/s = 9.8 flop/B)
          for r < 80, so they are rated against HBM, with the MFMA rate
          beside it; flush_decide also carries the next window's sequential
          decisions, whose latency per accepted flip is reported separately;
      qr_panel: Householder panel flops; one workgroup per panel, so it is
          rated against one compute unit's FP64 rate (78.6 TFLOP/s / 256).
    With the persistent slice launch (windows_per_launch = the slice's
    windows) one flush_decide launch carries all of a slice's windows: its
    algorithmic work is that many window flushes (the tiles keep G in
    registers across them, so the measured HBM traffic is far lower).
    """
    out = {}
    es = 8 if prec == "fp64" else 4
    for name, (ms, n) in prof.items():
        if n == 0 or name == "stabilize":
            continue
        t = ms / n / 1000.0
        r = {"avg_us": round(1e6 * t, 3), "launches": n}
        if name in ("wrap_cols", "wrap_rows", "bmul"):
            e = 8 if name == "bmul" else es
            byt = 2.0 * N * N * e
            ach = byt / t / 1e9
            r.update(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                     algorithmic_per_launch=byt)
        elif name in ("flush", "flush_decide"):
            rank = k_avg if name == "flush" else a_avg
            nwin = windows_per_launch if name == "flush_decide" else 1
            fl = 2.0 * N * N * rank * nwin
            byt = (2.0 * N * N * es + 2.0 * N * rank * es) * nwin
            pk = FP64_PEAK_TFS if prec == "fp64" else F16_PEAK_TFS
            ach = byt / t / 1e9
            r.update(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                     algorithmic_per_launch=byt, rank=rank,
                     mfma_tflops=fl / t / 1e12, mfma_peak=pk, mfma_frac=fl / t / 1e12 / pk,
                     flops_per_launch=fl)
            if name == "flush_decide":
                r["us_per_accept"] = round(1e6 * t / max(rank * nwin, 1e-9), 4)
                r["windows_per_launch"] = nwin
                if nwin > 1:
                    r["kernel_name"] = "k_slice_persist"
                    r["note"] = ("one resident launch per slice: every 64x64 tile of G in registers for the "
                                 "slice takes each window's factors and rank-a flush, one workgroup decides "
                                 "the windows in turn; the algorithmic bytes count a G read and write per "
                                 "window (the method's flush), the tiles touch G once per slice; "
                                 "us_per_accept = launch time / accepted flips of the slice")
                else:
                    r["kernel_name"] = "k_flush_decide"
                    r["note"] = ("one launch per window: the window's factors and its rank-a flush on every "
                                 "64x64 tile, and the next window's sequential decisions on one workgroup; "
                                 "us_per_accept = launch time / accepted flips of the window")
        elif name == "qr_panel":
            fl = qr_panel_flops(N) * (n / qr_panels(N)) / n
            ach = fl / t / 1e12
            r.update(bound="alu", achieved=ach, peak=CU_FP64_TFS, unit="TFLOP/s", frac=ach / CU_FP64_TFS,
                     algorithmic_per_launch=fl, note="one workgroup per panel (sequential columns)")
        elif name == "decide":
            r.update(bound="latency", note="one wave per window (sequential sites)")
        else:
            r.update(bound=None)
        out[name] = r
    return out


def _sha1(path):
    import hashlib
    with open(path, "rb") as fh:
        return hashlib.sha1(fh.read()).hexdigest()


def pmc_traffic(phase, workload):
    """HBM bytes per launch of a phase's kernel from a committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (profiles/pmc_traffic_*.txt), or None when
    there is none or the kernel's source has changed since it was taken."""
    import glob
    for f in sorted(glob.glob(os.path.join(HERE, "profiles", "pmc_traffic_*.txt"))):
        kv = {}
        with open(f) as fh:
            for line in fh:
                if ":" in line and not line.startswith(("#", " ")):
                    a, b = line.split(":", 1)
                    kv[a.strip()] = b.strip()
        if kv.get("phase") != phase or kv.get("workload") != workload:
            continue
        src = os.path.join(HERE, kv.get("source", ""))
        if not os.path.isfile(src) or _sha1(src) != kv.get("source_sha1"):
            return None
        try:
            return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])
        except (KeyError, ValueError):
            return None
    return None


def copy_calibration(mib=1024, reps=5):
    """A plain device copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE
    counters: each dispatch reads and writes mib MiB."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        torch.neg(a, out=b)   # an elementwise kernel: one 8 B read and one 8 B write per element
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_dispatch": n * 8, "dispatches": reps}), flush=True)


def run_chain(w, prec, n_stab, k, window, tile, steps, warmup, passes="alternate", profile=False,
              label=None, slice_launch="persistent"):
    """Times `steps` sweeps of one chain after `warmup` sweeps (graphs
    captured in the warm-up, replayed in the timed region).  Returns a dict;
    with profile=True the same sweeps are run again with a HIP event around
    every launch (direct launches) and the per-phase totals are added."""
    import torch
    from paper_2608_03894_amd import kdqmc
    dev = torch.device("cuda:0")
    p = kdqmc.make_params(w.L, w.U, w.beta, w.dtau, mu=-1.0, n_stab=n_stab, delay_k=k,
                          window=window, fft_tile=tile, prec=prec)
    ch = kdqmc.Chain(p, device=dev)
    N, Lt = ch.N, ch.L_tau
    total = warmup + steps
    fields = torch.from_numpy(si.ising_fields(w.L, Lt, w.seed)).to(dev)
    uni = torch.from_numpy(si.metropolis_uniforms(w.L, Lt, w.seed, n_sweeps=total)).to(dev)
    ub = torch.empty_like(uni[0])          # the one buffer every pass reads
    acc = torch.zeros((Lt, N), dtype=torch.uint8, device=dev)
    errs = torch.zeros(Lt // n_stab, dtype=torch.float64, device=dev)
    # the library's default: one resident launch per slice where the shape allows it
    persistent = ch.set_slice_launch(slice_launch == "persistent")
    wps = -(-N // min(window or min(k, 32), N))
    log(f"{label or w.name}: prec={prec} k={k} window={window} n_stab={n_stab} N={N} L_tau={Lt} "
        f"persistent={persistent}")
    ch.set_fields(fields)
    alt = passes == "alternate"

    def one_pass(s):
        ub.copy_(uni[s])
        if alt and s % 2 == 1:
            ch.sweep_down(ub, None, acc, None, errs)
        else:
            ch.sweep(ub, None, acc, None, errs)

    for s in range(warmup):
        one_pass(s)
    torch.cuda.synchronize()
    log(f"  {warmup} warm-up sweeps done")
    t0 = time.perf_counter()
    for s in range(steps):
        one_pass(warmup + s)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    worst, ok = ch.health(raise_on_error=False)
    accepts = int(acc.sum().item())  # last sweep's accepts
    res = {"steps": steps, "warmup": warmup, "ms_per_step": 1000.0 * elapsed / steps,
           "value": steps / elapsed, "unit": "sweeps/s", "healthy": ok, "max_wrap_err": worst,
           "wrap_tolerance": 1e-5 if prec == "fp64" else 1e-4, "acceptance": accepts / (N * Lt),
           "accepts_last_sweep": accepts, "N": N, "L_tau": Lt, "persistent": persistent,
           "windows_per_slice": wps}
    log(f"  timed {steps} sweeps in {elapsed:.3f} s -> {res['value']:.4f} sweeps/s "
        f"(max wrap error {worst:.3e}, healthy={ok})")
    if not ok:
        res["refused"] = ("the chain drifted: a stabilization's wrap error was not finite or above the "
                          f"tolerance (largest {worst:.3e}); no rate is quoted")
        res["value"] = None
    if profile:
        ch.set_fields(fields)
        for s in range(warmup):
            one_pass(s)
        ch.profile_enable(True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for s in range(steps):
            one_pass(warmup + s)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        res["prof"] = ch.profile_read()
        ch.profile_enable(False)
        res["profiled_ms_per_step"] = 1000.0 * (t3 - t2) / steps
        log(f"  profiled (direct launches) {steps} sweeps in {t3 - t2:.3f} s")
        for name, (ms, n) in res["prof"].items():
            if n:
                log(f"    {name:12s} {ms:10.3f} ms  {n:7d} launches  {1000 * ms / n:9.2f} us/launch")
    ch.close()
    return res


def bench_batch(prec, steps, warmup, n_stab_override=None, passes="alternate"):
    """64 independent chains of uneven L, U, beta (grouped by shape, one
    batched context and stream per group); one step = one sweep of every
    chain.  Value: aggregate chain-sweeps per second."""
    import torch
    from paper_2608_03894_amd import kdqmc
    chains = si.batched_chains(64, 64)
    dev = torch.device("cuda:0")
    params, fields, unis, intervals = [], [], [], []
    total = warmup + steps
    n_tuned = 0
    for w in chains:
        n_stab = n_stab_override or w.n_stab
        if prec != "fp64" and not n_stab_override:
            ni, _ = mixed_interval(w, prec)
            n_stab = ni or n_stab
        intervals.append(n_stab)
        k, window, tile, tuned = schedule(0, 0, 0, w, prec, n_stab, True)
        n_tuned += tuned
        params.append(kdqmc.make_params(w.L, w.U, w.beta, w.dtau, mu=-1.0, n_stab=n_stab,
                                        delay_k=k, window=window, fft_tile=tile, prec=prec))
        Lt = si.l_tau(w.beta, w.dtau)
        fields.append(torch.from_numpy(si.ising_fields(w.L, Lt, w.seed)).to(dev))
        unis.append(torch.from_numpy(si.metropolis_uniforms(w.L, Lt, w.seed, n_sweeps=total)).to(dev))
    b = kdqmc.Batch(params, device=dev)
    log(f"batch of {b.n_chains} chains in {len(b.groups)} shape groups, prec={prec}")
    b.set_inputs(fields, unis)
    alt = passes == "alternate"
    for s in range(warmup):
        b.sweep(s, down=alt and s % 2 == 1)
    torch.cuda.synchronize()
    log(f"  {warmup} warm-up batch sweeps done")
    t0 = time.perf_counter()
    for s in range(steps):
        b.sweep(warmup + s, down=alt and (warmup + s) % 2 == 1)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    worst, ok = b.health()
    value = b.n_chains * steps / elapsed
    upd = b.field_updates_per_sweep()
    log(f"  timed {steps} batch sweeps in {elapsed:.3f} s -> {value:.2f} chain-sweeps/s "
        f"(max wrap error {worst:.3e}, healthy={ok})")
    groups = [{"L": g["chain"].p.L, "beta": g["chain"].p.beta, "chains": len(g["idx"]),
               "delay_k": g["chain"].p.delay_k, "window": g["chain"].p.window,
               "n_stab": g["chain"].p.n_stab} for g in b.groups]
    res = {"value": value if ok else None, "unit": "chain-sweeps/s", "steps": steps, "warmup": warmup,
           "ms_per_step": 1000.0 * elapsed / steps, "healthy": ok, "max_wrap_err": worst,
           "field_updates_per_s": upd * steps / elapsed if ok else None,
           "acceptance": b.accepted() / upd,
           "config": {"workload": "kagome-batch-64-chains-L6-15-U3-5-beta4-8", "chains": b.n_chains,
                      "groups": groups, "prec": prec, "autotuned_chains": n_tuned, "passes": passes}}
    if not ok:
        res["refused"] = (f"a chain drifted (largest wrap error {worst:.3e} above the tolerance or not "
                          "finite); no rate is quoted")
    b.close()
    return res


def bench_wrap(Ls=(12, 18, 24), reps=50, fft_tile=0):
    """The FFT wrap alone (both passes of kdqmc_wrap_slice) on a resident G, at
    L = 12, 18, 24 in FP64 and FP32: GB/s = 2 N^2 s bytes per pass / average
    pass time (HIP events).  'resident' is one chain (its G stays in the
    256 MB Infinity Cache between passes); 'batch' runs enough chains in one
    batched context that their G matrices exceed 256 MB, so every pass
    streams from HBM."""
    import torch
    from paper_2608_03894_amd import kdqmc
    dev = torch.device("cuda:0")
    res = []
    beta, dtau = 10.0, 0.1
    Lt = si.l_tau(beta, dtau)
    for L in Ls:
        for prec in ("fp64", "mixed_f16"):
            N = 3 * L * L
            es = 8 if prec == "fp64" else 4
            for mode in ("resident", "batch"):
                nch = 1 if mode == "resident" else max(2, int(np.ceil(320e6 / (N * N * es))))
                p = kdqmc.make_params(L, -4.0, beta, dtau, mu=-1.0, n_stab=Lt, delay_k=32,
                                      fft_tile=fft_tile, prec=prec)
                try:
                    ch = kdqmc.Chain(p, device=dev, n_chains=nch)
                except kdqmc.KdqmcError as e:
                    log(f"wrap L={L} {prec} {mode}: {e}")
                    continue
                g = torch.eye(N, dtype=torch.float64, device=dev).expand(nch, N, N).contiguous()
                g += 1e-3 * torch.rand(nch, N, N, dtype=torch.float64, device=dev)
                ch.set_fields(torch.ones((nch, Lt, N), dtype=torch.int8, device=dev))
                ch.set_G(g, 0)
                for l in range(1, 4):
                    ch.wrap_slice(l)
                ch.profile_enable(True)
                ch.set_G(g, 0)
                n_rep = max(4, min(Lt - 1, reps))
                for l in range(1, n_rep + 1):
                    ch.wrap_slice(l)
                ch.sync()
                prof = ch.profile_read()
                ch.profile_enable(False)
                byt = 2.0 * N * N * es * nch
                row = {"L": L, "N": N, "prec": prec, "mode": mode, "chains": nch}
                for ph in ("wrap_cols", "wrap_rows"):
                    ms, n = prof[ph]
                    t = ms / n / 1000.0
                    row[ph + "_us"] = round(1e6 * t, 2)
                    row[ph + "_GBs"] = round(byt / t / 1e9, 1)
                    row[ph + "_frac"] = round(byt / t / 1e9 / HBM_PEAK_GBS, 4)
                log(json.dumps(row))
                res.append(row)
                ch.close()
                del g
                torch.cuda.synchronize()
    return {"metric": "FFT wrap HBM GB/s", "unit": "GB/s", "peak": HBM_PEAK_GBS,
            "algorithmic": "2 N^2 s bytes per pass per chain (G read once, written once)",
            "results": res}


def batch_roofline(n_chains=256, L=12, beta=4.0, delay_k=128, window=32, steps=2, warmup=1):
    """The batched form as the roofline case: n_chains chains of one shape
    (L=12, U=-4, FP64) in one batched context, so every kernel launches once
    for all of them (chains along the grid's z) and their G matrices
    (n_chains x 1.5 MB) exceed the 256 MB Infinity Cache.  Delay rank 128 in
    32-site windows: the pending factors are flushed every four windows, at a
    rank near 80 (the FP64 ridge of 9.8 flop/B).  Rates from a timed run,
    per-kernel rooflines from a profiled run (HIP events per launch)."""
    import torch
    from paper_2608_03894_amd import kdqmc
    dev = torch.device("cuda:0")
    p = kdqmc.make_params(L, -4.0, beta, 0.1, mu=-1.0, n_stab=10, delay_k=delay_k, window=window)
    ch = kdqmc.Chain(p, device=dev, n_chains=n_chains)
    N, Lt = ch.N, ch.L_tau
    f = torch.from_numpy(np.stack([si.ising_fields(L, Lt, 9000 + z) for z in range(n_chains)])).to(dev)
    u = torch.from_numpy(np.stack([si.metropolis_uniforms(L, Lt, 9000 + z, n_sweeps=warmup + 2 * steps)
                                   for z in range(n_chains)], axis=1)).to(dev)   # (sweeps, chains, Lt, N)
    ub = torch.empty_like(u[0])
    acc = torch.zeros((n_chains, Lt, N), dtype=torch.uint8, device=dev)
    ch.set_fields(f)

    def one(s):
        ub.copy_(u[s])
        (ch.sweep_down if s % 2 else ch.sweep)(ub, None, acc, None, None)
    for s in range(warmup):
        one(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        one(warmup + s)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    worst, ok = ch.health(raise_on_error=False)
    accepts = float(acc.sum().item())
    ch.set_fields(f)
    ch.profile_enable(True)
    for s in range(steps):
        one(warmup + steps + s)
    prof = ch.profile_read()
    ch.profile_enable(False)
    ch.close()
    n_fl = prof["flush"][1] // steps
    k_avg = accepts / n_chains / max(1, n_fl)           # rank of one chain's flush
    kern = {}
    for name in ("wrap_cols", "wrap_rows", "flush", "decide", "extend", "prep", "bmul"):
        ms, n = prof[name]
        if not n:
            continue
        t = ms / n / 1000.0
        r = {"avg_us": round(1e6 * t, 2), "launches": n}
        if name in ("wrap_cols", "wrap_rows", "bmul"):
            byt = 2.0 * N * N * 8 * n_chains
            r.update(bound="hbm", achieved=byt / t / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
                     frac=byt / t / 1e9 / HBM_PEAK_GBS)
        elif name == "flush":
            fl = 2.0 * N * N * k_avg * n_chains
            byt = (2.0 * N * N * 8 + 2.0 * N * k_avg * 8) * n_chains
            r.update(bound="mfma", achieved=fl / t / 1e12, peak=FP64_PEAK_TFS, unit="TFLOP/s",
                     frac=fl / t / 1e12 / FP64_PEAK_TFS, rank=k_avg, hbm_gbs=byt / t / 1e9,
                     hbm_frac=byt / t / 1e9 / HBM_PEAK_GBS)
        kern[name] = r
    res = {"workload": f"kagome-batch-{n_chains}x-L{L}-U-4-beta{beta:g}-fp64-k{delay_k}",
           "chains": n_chains, "N": N, "L_tau": Lt, "G_bytes_total": N * N * 8 * n_chains,
           "value": n_chains * steps / el if ok else None, "unit": "chain-sweeps/s", "steps": steps,
           "warmup": warmup, "ms_per_step": 1000.0 * el / steps, "healthy": ok, "max_wrap_err": worst,
           "field_updates_per_s": n_chains * N * Lt * steps / el if ok else None,
           "phases_ms_per_sweep": {k: round(v[0] / steps, 3) for k, v in prof.items() if v[1]},
           "kernels": kern}
    log("batch roofline", json.dumps(res))
    return res


def _loglog_slope(xs, ys):
    x, y = np.log(np.asarray(xs, float)), np.log(np.asarray(ys, float))
    return float(np.polyfit(x, y, 1)[0])


def fig1_multiply(Ls=(3, 6, 9, 12, 15, 18, 24), reps=20):
    """The paper's Fig. 1 on this GPU: time of one propagator product
    e^{-dtau K} M (N x N, FP64) by the FFT path of Eqs. (5)-(6)
    (kdqmc_expK_f64: per column 2D FFTs, 3x3 Bloch blocks, inverse FFTs)
    against a dense multiply by the N x N matrix e^{-dtau K}: this library's
    FP64 MFMA GEMM and the vendor DGEMM (torch.matmul, FP64).  Log-log slopes
    of time against L as the paper's linear fits."""
    import torch
    from paper_2608_03894_amd import kdqmc
    dev = torch.device("cuda:0")
    rows = []
    for L in Ls:
        p = kdqmc.make_params(L, -4.0, 1.0, 0.1, mu=-1.0, n_stab=10, delay_k=1 if L == 3 else 32)
        ch = kdqmc.Chain(p, device=dev)
        N = ch.N
        g = torch.Generator(device="cpu").manual_seed(L)
        M = torch.rand((N, N), dtype=torch.float64, generator=g).to(dev)
        A = M.clone()
        E = torch.eye(N, dtype=torch.float64, device=dev)
        ch.expK_f64(E)                         # the dense e^{-dtau K}, built by the FFT path
        C = torch.empty_like(M)
        ch.expK_f64(A)
        ref = E @ M
        err = float(((A - ref).abs().max() / ref.abs().max()).item())
        timing = {}
        for name, fn in (("fft", lambda: ch.expK_f64(A)),
                         ("gemm_mfma", lambda: ch.gemm_f64(False, False, N, N, N, 1.0, E, N, M, N, 0.0, C, N)),
                         ("gemm_vendor", lambda: torch.matmul(E, M, out=C))):
            for _ in range(3):
                fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            timing[name] = e0.elapsed_time(e1) * 1000.0 / reps   # us per product
        row = {"L": L, "N": N, "fft_us": round(timing["fft"], 2), "gemm_mfma_us": round(timing["gemm_mfma"], 2),
               "gemm_vendor_us": round(timing["gemm_vendor"], 2),
               "speedup_vs_vendor": round(timing["gemm_vendor"] / timing["fft"], 2),
               "fft_vs_dense_rel_err": err}
        log("fig1", json.dumps(row))
        rows.append(row)
        ch.close()
    big = [r for r in rows if r["L"] >= 9]
    fits = {k: _loglog_slope([r["L"] for r in big], [r[k] for r in big])
            for k in ("fft_us", "gemm_mfma_us", "gemm_vendor_us")}
    return {"what": "time per product e^{-dtau K} M (N x N, FP64): FFT path vs dense GEMM",
            "rows": rows, "loglog_slope_vs_L_for_L_ge_9": fits,
            "expected_slopes": "FFT N^2 log N ~ L^4 (x log); dense N^3 ~ L^6"}


def fig2_runtime(Ls=(6, 9, 12, 15, 18, 24), U=-5.0, beta=10.0, passes=2, window=5):
    """The paper's Fig. 2 on this GPU: the projector workload of Sec. III
    (U = -5, rho = 2/3: n_occ = L^2 trial orbitals, projection length
    beta = 10, delay k = 32, stabilization every 10 slices).  One step = an
    upward and a downward pass (a sweep), with the estimators measured after
    every slice within `window` slices of the middle of the projection.
    Time per sweep (wall clock, synchronized), the share of the GPU time per
    process from HIP events around every launch (FFT multiplication: wrap and
    stack products; delay update: decisions, factors and flushes;
    measurement; the rest of the stabilization: QR, GEMM, solves), and the
    fitted exponent of time against L over 12 <= L <= 24."""
    import torch
    from paper_2608_03894_amd import kdqmc
    dev = torch.device("cuda:0")
    rows = []
    for L in Ls:
        n_occ = L * L
        p = kdqmc.make_params(L, U, beta, 0.1, mu=-1.0, n_stab=10, delay_k=32, n_occ=n_occ)
        ch = kdqmc.Chain(p, device=dev)
        N, Lt = ch.N, ch.L_tau
        ch.set_trial(torch.from_numpy(kdqmc.trial_orbitals(L, n_occ)).to(dev))
        f = torch.from_numpy(si.ising_fields(L, Lt, 7000 + L)).to(dev)
        u = torch.from_numpy(si.metropolis_uniforms(L, Lt, 7000 + L, n_sweeps=2 + 2 * passes)).to(dev)
        obs = torch.zeros(8, dtype=torch.float64, device=dev)
        ch.set_fields(f)
        ub = torch.empty_like(u[0])
        for s in range(2):                      # warm-up: one sweep from captured graphs
            ub.copy_(u[s])
            (ch.sweep_down if s % 2 else ch.sweep)(ub)
        mid = Lt // 2

        def one_sweep(s0):
            for l in range(1, Lt + 1):
                ch.sweep_slice(l, u[s0][l - 1])
                if l % 10 == 0:
                    ch.stabilize()
                if abs(l - mid) <= window:
                    ch.measure(obs)
            for l in range(Lt, 0, -1):
                ch.sweep_slice_down(l, u[s0 + 1][l - 1])
                if (l - 1) % 10 == 0:
                    ch.stabilize()
                if abs(l - 1 - mid) <= window:
                    ch.measure(obs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(passes // 2 or 1):
            one_sweep(2 + 2 * k)
        torch.cuda.synchronize()
        sweeps = passes // 2 or 1
        t_sweep = (time.perf_counter() - t0) / sweeps
        ch.set_fields(f)
        ch.profile_enable(True)
        for k in range(sweeps):
            one_sweep(2 + 2 * k)
        prof = ch.profile_read()
        ch.profile_enable(False)
        ms = {k: v[0] / sweeps for k, v in prof.items()}
        fft = ms["wrap_cols"] + ms["wrap_rows"] + ms["bmul"]
        delay = ms["decide"] + ms["extend"] + ms["prep"] + ms["flush"] + ms["flush_decide"]
        meas = ms["measure"]
        stab_rest = ms["stabilize"] - ms["bmul"]
        tot = fft + delay + meas + stab_rest
        row = {"L": L, "N": N, "L_tau": Lt, "n_occ": n_occ, "s_per_sweep": round(t_sweep, 5),
               "gpu_ms_per_sweep": round(tot, 3),
               "share": {"fft_multiply": round(fft / tot, 4), "delay_update": round(delay / tot, 4),
                         "measurement": round(meas / tot, 4), "stabilization_qr_gemm": round(stab_rest / tot, 4)}}
        log("fig2", json.dumps(row))
        rows.append(row)
        ch.close()
    big = [r for r in rows if r["L"] >= 12]
    a = _loglog_slope([r["L"] for r in big], [r["s_per_sweep"] for r in big])
    return {"what": "projector workload of Sec. III (U=-5, rho=2/3, beta=10): time per sweep and GPU-time "
                    "shares per process vs L", "rows": rows,
            "fit_12_le_L_le_24": {"time_vs_L_exponent": a, "time_vs_N_exponent": a / 2.0},
            "paper_context": "Time ~ L^4.98 ~ N^2.49 over 12 <= L <= 27 on 20-30 Xeon E5-2678 v3 cores"}


def workload_record(w, prec, n_stab, k, window, tile, res, tuned, table=None):
    rec = {"metric": "HS-field sweeps/sec", "value": res["value"], "unit": "sweeps/s",
           "steps": res["steps"], "warmup": res["warmup"], "ms_per_step": res["ms_per_step"],
           "dtype": "f64" if prec == "fp64" else f"f32+{prec.split('_')[1]}",
           "config": {"workload": w.name, "L": w.L, "N": res["N"], "U": w.U, "beta": w.beta,
                      "L_tau": res["L_tau"], "delay_k": k, "window": window, "fft_tile": tile,
                      "autotuned": tuned, "prec": prec, "n_stab": n_stab},
           "healthy": res["healthy"], "max_wrap_err": res["max_wrap_err"],
           "acceptance": res["acceptance"]}
    if res["value"] is not None:
        rec["field_updates_per_s"] = res["value"] * res["N"] * res["L_tau"]
    if "refused" in res:
        rec["refused"] = res["refused"]
    if table is not None:
        rec["error_vs_fp64"] = {"at_n_stab": table["n_stab"], "max_dG": table["table"][str(table["n_stab"])]
                                ["max_dG"], "ratio_rel_err": table["table"][str(table["n_stab"])]["ratio_err"],
                                "target": table["target"], "measured_on": table["measured_on"],
                                "table": table["table"]}
    return rec


def extras(args):
    """The metric's other workloads, each timed on its own (few steps)."""
    out = {}
    big = [("c5", si.C5, args.extra_steps_big, 1), ("c3", si.C3, args.extra_steps, 1)]
    for key, w, steps, warm in big:
        for prec in ("fp64", "mixed_f16"):
            if prec == "fp64":
                n_stab, table = w.n_stab, None
            else:
                n_stab, table = mixed_interval(w, prec)
                if n_stab is None:
                    out[f"{key}_{prec}"] = {"value": None, "refused": "no measured interval for this lattice"}
                    continue
            k, window, tile, tuned = schedule(0, 0, 0, w, prec, n_stab, True)
            try:
                res = run_chain(w, prec, n_stab, k, window, tile, steps, warm, label=f"{key} {prec}")
                out[f"{key}_{prec}"] = workload_record(w, prec, n_stab, k, window, tile, res, tuned, table)
            except Exception as e:  # a failed extra must not hide the headline
                out[f"{key}_{prec}"] = {"value": None, "error": str(e)}
        if key == "c5" and not args.no_mixed_at_config_interval:
            # the workload's own interval (every 10 slices) in mixed precision:
            # shown to be refused (drifting), never quoted as a rate
            prec = "mixed_f16"
            k, window, tile, tuned = schedule(0, 0, 0, w, prec, w.n_stab, True)
            try:
                res = run_chain(w, prec, w.n_stab, k, window, tile, 1, 1, label=f"{key} {prec} n_stab=10")
                out[f"{key}_{prec}_n_stab10"] = workload_record(w, prec, w.n_stab, k, window, tile, res, tuned)
            except Exception as e:
                out[f"{key}_{prec}_n_stab10"] = {"value": None, "error": str(e)}
    for prec in ("fp64", "mixed_f16"):
        try:
            out[f"c4_batch_{prec}"] = bench_batch(prec, args.extra_steps_batch, 2)
        except Exception as e:
            out[f"c4_batch_{prec}"] = {"value": None, "error": str(e)}
    try:
        out["wrap"] = bench_wrap()
    except Exception as e:
        out["wrap"] = {"error": str(e)}
    for key, fn in (("batch_roofline", batch_roofline), ("fig1_multiply", fig1_multiply),
                    ("fig2_runtime", fig2_runtime)):
        try:
            out[key] = fn()
        except Exception as e:
            out[key] = {"error": str(e)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2", choices=sorted(CONFIGS))
    ap.add_argument("--prec", default=None, help="fp64 | mixed_f16 | mixed_bf16 (default: workload's)")
    ap.add_argument("--delay-k", type=int, default=None)
    ap.add_argument("--window", type=int, default=0)
    ap.add_argument("--fft-tile", type=int, default=0)
    ap.add_argument("--n-stab", type=int, default=None, help="slices between stabilizations")
    ap.add_argument("--passes", default="alternate", choices=["alternate", "up"],
                    help="sweep directions: alternating upward/downward passes, or upward only")
    ap.add_argument("--slice-launch", default="persistent", choices=["persistent", "per-window"],
                    help="FP64 site updates: one resident launch per slice (where it fits) "
                         "or one launch per window")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-slices", type=int, default=20)
    ap.add_argument("--no-extras", action="store_true", help="only the headline workload")
    ap.add_argument("--no-profile", action="store_true", help="skip the HIP-event profiled repeat")
    ap.add_argument("--no-mixed-at-config-interval", action="store_true")
    ap.add_argument("--extra-steps", type=int, default=3)
    ap.add_argument("--extra-steps-big", type=int, default=2)
    ap.add_argument("--extra-steps-batch", type=int, default=4)
    ap.add_argument("--wrap-only", action="store_true",
                    help="only time the FFT wrap passes at L = 12, 18, 24 and exit")
    ap.add_argument("--fig", choices=["1", "2"], default=None,
                    help="only run the paper's Fig. 1 (multiply) or Fig. 2 (runtime) experiment and exit")
    ap.add_argument("--batch-roofline", action="store_true",
                    help="only run the 256-chain batched roofline case and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(independent chains shard across GPUs without collectives; "
                                   "see the design notes)"}))
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return
    if args.batch_roofline:
        print(json.dumps(batch_roofline(steps=args.steps, warmup=args.warmup)), flush=True)
        return
    if args.fig:
        print(json.dumps(fig1_multiply() if args.fig == "1" else fig2_runtime()), flush=True)
        return
    if args.wrap_only:
        print(json.dumps(bench_wrap(fft_tile=args.fft_tile)), flush=True)
        return
    if args.config == "c4":
        prec = args.prec or "mixed_f16"
        r = bench_batch(prec, args.steps, args.warmup, args.n_stab, args.passes)
        r.update({"metric": "HS-field sweeps/sec (batched, aggregate over chains)", "n_gpus": 1,
                  "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                  "dtype": "f64" if prec == "fp64" else f"f32+{prec.split('_')[1]}",
                  "data": "synthetic", "roofline": None, "cpu_baseline": None})
        print(json.dumps(r), flush=True)
        return

    w = CONFIGS[args.config]
    prec = args.prec or ("fp64" if w.prec == "fp64" else w.prec)
    table = None
    if args.n_stab:
        n_stab = args.n_stab
    elif prec != "fp64":
        n_stab, table = mixed_interval(w, prec)
        n_stab = n_stab or w.n_stab
    else:
        n_stab = w.n_stab
    k, window, tile, tuned = schedule(args.delay_k, args.window, args.fft_tile, w, prec, n_stab,
                                      args.config in AUTOTUNED)
    res = run_chain(w, prec, n_stab, k, window, tile, args.steps, args.warmup, args.passes,
                    profile=not args.no_profile, slice_launch=args.slice_launch)
    N, Lt = res["N"], res["L_tau"]
    win = min(window or min(k, 32), N)   # the library's default window: min(delay_k, 32)

    roof, kernels = None, None
    if "prof" in res:
        prof = res["prof"]
        steps = args.steps
        accepts = res["accepts_last_sweep"]
        # rank of a flush: accepts per flush launch (three-kernel schedule), or
        # per window launch (fused schedule: each window launch flushes one
        # window's accepts)
        n_fl = prof["flush"][1] // steps
        n_fd = prof.get("flush_decide", (0, 0))[1] // steps
        nwin = res["windows_per_slice"] if res.get("persistent") else 1
        k_avg = accepts / n_fl if n_fl else 0.0
        a_avg = accepts / (n_fd * nwin) if n_fd else 0.0
        kernels = kernel_rooflines(prof, N, prec, k_avg, a_avg, nwin)
        cand = {n: v for n, v in prof.items() if n != "stabilize" and v[1] > 0}
        dom = max(cand, key=lambda n: cand[n][0])
        roof = dict(kernels.get(dom, {"bound": None, "achieved": None, "peak": None, "unit": None,
                                      "frac": None}))
        roof["kernel"] = dom
        roof["traffic"] = pmc_traffic(dom, w.name)
    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle on {args.cpu_slices} slices ...")
        cpu = cpu_baseline(w, min(args.cpu_slices, Lt))
        log(f"cpu baseline {cpu['value']:.4f} sweeps/s")

    out = {
        "metric": "HS-field sweeps/sec",
        "value": res["value"],
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else f"f32+{prec.split('_')[1]}",
        "data": "synthetic",
        "config": {"workload": w.name, "L": w.L, "N": N, "U": w.U, "beta": w.beta, "L_tau": Lt,
                   "delay_k": k, "window": win, "fft_tile": tile, "autotuned": tuned,
                   "prec": prec, "n_stab": n_stab, "passes": args.passes,
                   "field_updates_per_s": (res["value"] or 0.0) * N * Lt},
        "roofline": roof,
        "kernels": kernels,
        "cpu_baseline": cpu,
        "healthy": res["healthy"],
        "max_wrap_err": res["max_wrap_err"],
        "acceptance": res["acceptance"],
        "parity_note": ("FP64 G agrees with the oracle within 1e-10 right after every stabilization; "
                        "between stabilizations both drift from the exact G (the wrap amplifies "
                        "rounding about 2.5x per slice at this workload: 2e-10 at slice 10), and the "
                        "per-slice parity bound is max(1e-10, 2x the oracle's own drift)"),
    }
    if "refused" in res:
        out["refused"] = res["refused"]
    if "prof" in res:
        out["profiled_ms_per_step"] = res["profiled_ms_per_step"]
        out["phases_ms_per_sweep"] = {n: round(v[0] / args.steps, 4) for n, v in res["prof"].items() if v[1]}
        out["launches_per_sweep"] = {n: v[1] // args.steps for n, v in res["prof"].items() if v[1]}
    if table is not None:
        out["error_vs_fp64"] = table
    if not args.no_extras and args.config == "c2":
        out["extra"] = extras(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
