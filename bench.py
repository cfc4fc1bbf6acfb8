"""Benchmark: HS-field sweeps per second of the kagome DQMC hot path on one GPU.

One step = one full sweep: a pass over all L_tau slices (window decisions,
delayed rank-k flushes and FFT wraps, a QR-stabilization every n_stab
slices), on seeded synthetic fields and uniforms that are resident in device
memory before the timed region starts.  Passes alternate upward and downward
(the standard sweep order of DQMC; each pass keeps the stabilization stack
the next one needs), or are all upward with --passes up (then every pass
ends by rebuilding the left stack).

Prints ONE JSON line.  `roofline` is for the dominant kernel (largest share
of the timed region's kernel time, from HIP events recorded by the library
around every launch); `cpu_baseline` times the CPU oracle on a bounded
sample of the same workload.
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


def schedule(args, w, prec, n_stab, autotuned):
    """(delay_k, window, fft_tile, from_autotuner): command-line values win;
    for autotuned workloads the cached autotuner choice (same lattice, beta,
    precision and interval) is used when present, else the workload default."""
    t = None
    if autotuned and not args.delay_k:
        from paper_2608_03894_amd import autotune
        t = autotune.lookup(w.L, w.U, w.beta, w.dtau, prec, n_stab, any_U=True)
    k = args.delay_k or (t["delay_k"] if t else w.delay_k)
    window = args.window or (t["window"] if t else 0)
    tile = args.fft_tile or (t["fft_tile"] if t else 0)
    return k, window, tile, t is not None


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


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


def panel_width(m):
    """The library's QR panel width (16 columns for every panel height m)."""
    return 16


def qr_panel_flops(n):
    """Householder flops of all panels of one n x n QR (2 m b^2 - 2 b^3 / 3 per
    m x b panel)."""
    f, j = 0.0, 0
    while j < n:
        m = n - j
        b = min(panel_width(m), m)
        f += 2.0 * m * b * b - 2.0 * b ** 3 / 3.0
        j += b
    return f


def qr_panels(n):
    cnt, j = 0, 0
    while j < n:
        j += min(panel_width(n - j), n - j)
        cnt += 1
    return cnt


def kernel_rooflines(prof, N, Lt, prec, k_avg, n_stab):
    """{phase: roofline dict} from the profiled (HIP-event) per-phase totals.

    achieved = algorithmic bytes or flops per launch / average launch time:
      wrap_cols, wrap_rows, bmul: 2 N^2 s bytes (G read once, written once)
      flush: 2 N^2 k flops (k = accepted flips per flush), HBM bytes 2 N^2 s + 2 N k s
      qr_panel: Householder panel flops; one workgroup, so the peak is one
                compute unit's FP64 rate (the chip's 78.6 TFLOP/s / 256)
      decide: sequential per-site decisions on one workgroup; 2 w^2 flops per
              accepted flip (the rank-one update of the window block), against
              one compute unit's FP64 rate
      flush_decide: the fused window launch (factors, flush, next window's
              decisions); its duration is set by the decisions on one compute
              unit, so it is rated like decide, with the flush's MFMA rate
              (2 N^2 k flops per launch) beside it
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
        elif name == "flush":
            fl = 2.0 * N * N * k_avg
            pk = FP64_PEAK_TFS if prec == "fp64" else F16_PEAK_TFS
            ach = fl / t / 1e12
            byt = 2.0 * N * N * es + 2.0 * N * k_avg * es
            r.update(bound="mfma", achieved=ach, peak=pk, unit="TFLOP/s", frac=ach / pk,
                     algorithmic_per_launch=fl, hbm_gbs=byt / t / 1e9,
                     hbm_frac=byt / t / 1e9 / HBM_PEAK_GBS, k_avg=k_avg)
        elif name == "qr_panel":
            per_sweep_qr = n  # launches
            fl_qr = qr_panel_flops(N)
            n_qr = per_sweep_qr / qr_panels(N)
            fl = fl_qr * n_qr / n
            ach = fl / t / 1e12
            r.update(bound="alu", achieved=ach, peak=CU_FP64_TFS, unit="TFLOP/s", frac=ach / CU_FP64_TFS,
                     algorithmic_per_launch=fl, note="one workgroup per panel (sequential columns)")
        elif name in ("decide", "flush_decide"):
            r.update(bound="alu", unit="TFLOP/s", peak=CU_FP64_TFS,
                     note="one workgroup per window (sequential sites)")
            if name == "flush_decide":
                fl = 2.0 * N * N * k_avg
                r.update(mfma_achieved=fl / t / 1e12, mfma_peak=FP64_PEAK_TFS,
                         mfma_frac=fl / t / 1e12 / FP64_PEAK_TFS, k_avg=k_avg,
                         note="one launch per window: factors and flush on every tile, the "
                              "next window's sequential decisions on one workgroup")
            out[name] = r
            continue
        else:
            r.update(bound=None)
        out[name] = r
    return out


def decide_roofline(kern, prof, accepts_per_sweep, steps, window):
    """Fills the decide and flush_decide entries: 2 w^2 flops per accepted flip,
    the accepts spread evenly over the launches that make decisions."""
    names = [x for x in ("decide", "flush_decide") if x in kern]
    launches = sum(prof[x][1] for x in names)
    if not launches:
        return
    fl = 2.0 * window * window * accepts_per_sweep * steps / launches
    for x in names:
        ms, n = prof[x]
        t = ms / n / 1000.0
        ach = fl / t / 1e12
        kern[x].update(achieved=ach, frac=ach / CU_FP64_TFS, algorithmic_per_launch=fl)


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


def bench_batch(args):
    """64 independent chains of uneven L, U, beta (grouped by shape, one
    batched context and stream per group); one step = one sweep of every
    chain.  Value: aggregate chain-sweeps per second."""
    import torch
    from paper_2608_03894_amd import kdqmc
    chains = si.batched_chains(64, 64)
    prec = args.prec or "mixed_f16"
    dev = torch.device("cuda:0")
    params, fields, unis = [], [], []
    total = args.warmup + args.steps
    n_tuned = 0
    for w in chains:
        n_stab = args.n_stab or w.n_stab
        k, window, tile, tuned = schedule(args, w, prec, n_stab, True)
        n_tuned += tuned
        params.append(kdqmc.make_params(w.L, w.U, w.beta, w.dtau, mu=-1.0, n_stab=n_stab,
                                        delay_k=k, window=window, fft_tile=tile, prec=prec))
        Lt = si.l_tau(w.beta, w.dtau)
        fields.append(torch.from_numpy(si.ising_fields(w.L, Lt, w.seed)).to(dev))
        unis.append(torch.from_numpy(si.metropolis_uniforms(w.L, Lt, w.seed, n_sweeps=total)).to(dev))
    b = kdqmc.Batch(params, device=dev)
    log(f"batch of {b.n_chains} chains in {len(b.groups)} shape groups, prec={prec}")
    b.set_inputs(fields, unis)
    alt = args.passes == "alternate"
    for s in range(args.warmup):
        b.sweep(s, down=alt and s % 2 == 1)
        log(f"warmup sweep {s + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        b.sweep(args.warmup + s, down=alt and (args.warmup + s) % 2 == 1)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = b.n_chains * args.steps / elapsed
    upd = b.field_updates_per_sweep()
    log(f"timed {args.steps} batch sweeps in {elapsed:.3f} s -> {value:.2f} chain-sweeps/s")
    groups = [{"L": g["chain"].p.L, "beta": g["chain"].p.beta, "chains": len(g["idx"]),
               "delay_k": g["chain"].p.delay_k, "window": g["chain"].p.window} for g in b.groups]
    out = {
        "metric": "HS-field sweeps/sec (batched, aggregate over chains)",
        "value": value,
        "unit": "chain-sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else f"f32+{prec.split('_')[1]}",
        "data": "synthetic",
        "config": {"workload": "kagome-batch-64-chains-L6-15-U3-5-beta4-8", "chains": b.n_chains,
                   "groups": groups, "prec": prec, "autotuned_chains": n_tuned, "passes": args.passes,
                   "field_updates_per_s": upd * args.steps / elapsed},
        "roofline": None,
        "cpu_baseline": None,
        "acceptance": b.accepted() / upd,
        "max_wrap_err": b.max_wrap_err(),
    }
    b.close()
    print(json.dumps(out), flush=True)


def bench_wrap(args):
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
    for L in (int(x) for x in args.wrap_L.split(",")):
        for prec in ("fp64", "mixed_f16"):
            N = 3 * L * L
            es = 8 if prec == "fp64" else 4
            for mode in ("resident", "batch"):
                nch = 1 if mode == "resident" else max(2, int(np.ceil(320e6 / (N * N * es))))
                p = kdqmc.make_params(L, -4.0, beta, dtau, mu=-1.0, n_stab=Lt, delay_k=32,
                                      fft_tile=args.fft_tile, prec=prec)
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
                prof = None
                reps = max(4, min(Lt - 1, args.wrap_reps))
                for l in range(1, reps + 1):
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
    print(json.dumps({"metric": "FFT wrap HBM GB/s", "unit": "GB/s", "peak": HBM_PEAK_GBS,
                      "algorithmic": "2 N^2 s bytes per pass per chain (G read once, written once)",
                      "results": res}), flush=True)


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
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-slices", type=int, default=20)
    ap.add_argument("--wrap-only", action="store_true",
                    help="only time the FFT wrap passes at the lattice sizes of --wrap-L and exit")
    ap.add_argument("--wrap-L", default="12,18,24")
    ap.add_argument("--wrap-reps", type=int, default=50)
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
    if args.config == "c4":
        bench_batch(args)
        return
    if args.wrap_only:
        bench_wrap(args)
        return

    import torch
    from paper_2608_03894_amd import kdqmc

    w = CONFIGS[args.config]
    prec = args.prec or ("fp64" if w.prec == "fp64" else w.prec)
    n_stab = args.n_stab or w.n_stab
    k, window, tile, tuned = schedule(args, w, prec, n_stab, args.config in AUTOTUNED)
    dev = torch.device("cuda:0")
    p = kdqmc.make_params(w.L, w.U, w.beta, w.dtau, mu=-1.0, n_stab=n_stab, delay_k=k,
                          window=window, fft_tile=tile, prec=prec)
    ch = kdqmc.Chain(p, device=dev)
    N, Lt = ch.N, ch.L_tau
    total = args.warmup + args.steps
    fields = torch.from_numpy(si.ising_fields(w.L, Lt, w.seed)).to(dev)
    uni = torch.from_numpy(si.metropolis_uniforms(w.L, Lt, w.seed, n_sweeps=total)).to(dev)
    acc = torch.zeros((Lt, N), dtype=torch.uint8, device=dev)
    errs = torch.zeros(Lt // n_stab, dtype=torch.float64, device=dev)
    log(f"workload {w.name} prec={prec} k={k} N={N} L_tau={Lt}")
    ch.set_fields(fields)
    alt = args.passes == "alternate"

    def one_pass(s):
        if alt and s % 2 == 1:
            ch.sweep_down(uni[s], None, acc, None, errs)
        else:
            ch.sweep(uni[s], None, acc, None, errs)

    for s in range(args.warmup):
        one_pass(s)
        log(f"warmup sweep {s + 1}/{args.warmup} done")
    torch.cuda.synchronize()

    # timed region: K sweeps replayed from the captured HIP graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        one_pass(args.warmup + s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    accepts = int(acc.sum().item())  # last sweep's accepts
    wrap_err = float(errs.max().item())
    elapsed = t1 - t0
    value = args.steps / elapsed
    log(f"timed {args.steps} sweeps in {elapsed:.3f} s -> {value:.3f} sweeps/s")

    # the same K sweeps again with a HIP event around every kernel launch
    # (direct launches: events inside a graph are not timed)
    ch.set_fields(fields)
    for s in range(args.warmup):
        one_pass(s)
    ch.profile_enable(True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for s in range(args.steps):
        one_pass(args.warmup + s)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    prof = ch.profile_read()
    ch.profile_enable(False)
    log(f"profiled (direct launches) {args.steps} sweeps in {t3 - t2:.3f} s")
    for name, (ms, n) in prof.items():
        if n:
            log(f"  {name:10s} {ms:10.3f} ms  {n:7d} launches  {1000 * ms / n:9.2f} us/launch")

    # per-kernel rooflines from the HIP-event durations; the dominant kernel
    # (stabilize is a composite of bmul / qr_panel / gemm and is skipped)
    flushes = max(1, (prof["flush"][1] + prof.get("flush_decide", (0, 0))[1]) // args.steps)
    k_avg = accepts / flushes
    kernels = kernel_rooflines(prof, N, Lt, prec, k_avg, n_stab)
    win = min(window or min(k, 32), N)   # the library's default window: min(delay_k, 32)
    decide_roofline(kernels, prof, accepts, args.steps, win)
    cand = {n: v for n, v in prof.items() if n != "stabilize" and v[1] > 0}
    dom = max(cand, key=lambda n: cand[n][0])
    roof = dict(kernels.get(dom, {"bound": "alu", "achieved": None, "peak": None, "unit": None,
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
        "value": value,
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else f"f32+{prec.split('_')[1]}",
        "data": "synthetic",
        "config": {"workload": w.name, "L": w.L, "N": N, "U": w.U, "beta": w.beta, "L_tau": Lt,
                   "delay_k": k, "window": win, "fft_tile": tile, "autotuned": tuned,
                   "prec": prec, "n_stab": n_stab, "passes": args.passes,
                   "field_updates_per_s": value * N * Lt},
        "roofline": roof,
        "kernels": kernels,
        "cpu_baseline": cpu,
        "profiled_ms_per_step": 1000.0 * (t3 - t2) / args.steps,
        "phases_ms_per_sweep": {n: round(v[0] / args.steps, 4) for n, v in prof.items() if v[1]},
        "launches_per_sweep": {n: v[1] // args.steps for n, v in prof.items() if v[1]},
        "acceptance": accepts / (N * Lt),
        "max_wrap_err": wrap_err,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
