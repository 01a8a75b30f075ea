"""Throughput benchmark: particle-steps/s of the full simulation step on one MI355X.

A step is one pass of the whole hot path (radial sort, harmonic moments,
prefix/suffix carry scans, boundary response + drive, field + leapfrog push)
over all particles.  Default workload: the largest single-GPU run of the
scale sweep, 1.6e7 electrons, l_max = 16, uniform shell 1 < r < 5, T_e = 3 eV,
n_e = 1e15 m^-3, +-1 V Gaussian pulse, in the FP32-compensated mode, with the
plain FP64 run of the same state timed beside it.

Prints ONE JSON line.  `roofline` reports the dominant kernel (field_push)
against the vector peak of its precision; `cpu_baseline` times the CPU oracle
on a bounded sample of the same state (all threads and one thread) and also
gives the field error of the GPU against it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/s at l_max vs FP64 oracle error; p50/p99 sim latency (served)"
FP64_VECTOR_PEAK_TFLOPS = 78.6
FP32_VECTOR_PEAK_TFLOPS = 157.3


def algorithmic_flops_per_particle(l_max: int) -> float:
    """Floor of the method per particle-step: one harmonic evaluation, two
    scans and the 3-component gradient contraction over 2C coefficients,
    about 20 (l_max + 1)^2 flops."""
    return 20.0 * (l_max + 1) ** 2


def _code_hash(text: str) -> str:
    """Hash of HIP/C++ source with comments and whitespace removed (so an edit
    of a comment does not retire a profile taken on the same code)."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    text = re.sub(r"\s+", " ", text).strip()
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def _kernel_source_hash() -> str:
    p = os.path.join(ROOT, "paper_2111_13072_amd", "csrc", "mrpsim.hip")
    return _code_hash(open(p).read())


def _traffic_from_profiles(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when it is missing or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_sha256_16") != _kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(wl, st, prm, u_now, q_s, budget_s: float, gpu_fields: dict):
    """The oracle (plain FP64 pair sums + leapfrog push) on a bounded random
    sample of particles of the same state, timed on the host cores with all
    threads and with one; returns the baseline record and, for each GPU field
    given, its error on the sample (max |dE| / RMS |E| of the oracle)."""
    import oracle as O

    op = O.Params(d=prm.d, eps_r=prm.eps_r, r_out=prm.r_out, dt=prm.dt, ntilde=prm.ntilde,
                  ion_density=prm.ion_density, l_max=prm.l_max, m_mode=prm.m_mode,
                  probe_bc=prm.probe_bc, wall_bc=prm.wall_bc, seed=prm.seed)
    from concurrent.futures import ThreadPoolExecutor

    rng = np.random.default_rng(12345)
    threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or (os.cpu_count() or 1)
    order = rng.permutation(wl.n)
    ids = np.arange(wl.n, dtype=np.uint32)

    def one_target(k):
        E, _ = O.field(op, st.pos, ids=ids, q_surface=q_s, u_asy=u_now, targets=[k])
        return E[0]

    def timed(targets, nthreads):
        """Oracle field + push of the targets, one target per call on
        nthreads host threads (each call single-threaded)."""
        t0 = time.perf_counter()
        with ThreadPoolExecutor(nthreads, initializer=O.set_threads, initargs=(1,)) as ex:
            E = np.array(list(ex.map(one_target, targets))).reshape(-1, 3)
        v = st.vel[targets] - E * prm.dt          # the push of the sampled particles
        _ = st.pos[targets] + v * prm.dt
        return E, time.perf_counter() - t0

    # all threads: a first probe, then as many targets as fit the budget
    first = np.sort(order[:threads])
    E0, t_first = timed(first, threads)
    per = t_first / len(first)
    extra = int(max(0, (0.75 * budget_s - t_first) / per))
    rest = np.sort(order[len(first):len(first) + min(extra, wl.n // 2)])
    E1, t_rest = timed(rest, threads) if len(rest) else (np.zeros((0, 3)), 0.0)
    targets = np.concatenate([first, rest])
    Eo = np.concatenate([E0, E1])
    rate_all = len(targets) / (t_first + t_rest)
    # one thread: about a quarter of the budget
    n1 = max(1, int(0.25 * budget_s / (per * threads)))
    one = order[len(targets):len(targets) + n1]
    _, t_one = timed(np.sort(one), 1)
    rate_one = len(one) / t_one
    rms = float(np.sqrt(np.mean(np.sum(Eo * Eo, axis=1))))
    errs = {k: float(np.max(np.abs(E[targets] - Eo)) / rms) for k, E in gpu_fields.items()}
    rec = {"value": rate_all, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
           "value_1_thread": rate_one,
           "sample": f"pair-sum field + leapfrog push of {len(targets)} random particles of the "
                     f"{wl.n}-particle, l_max={wl.l_max} state (one step) on {threads} threads in "
                     f"{t_first + t_rest:.1f} s, and of {len(one)} others on 1 thread in "
                     f"{t_one:.1f} s"}
    return rec, errs, len(targets)


# ---------------------------------------------------------------------------
# rocprofv3 summaries (profiles/)
# ---------------------------------------------------------------------------

def _read_csv(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def _find(dirpath, suffix):
    for root, _, files in os.walk(dirpath):
        for fn in files:
            if fn.endswith(suffix):
                return os.path.join(root, fn)
    raise FileNotFoundError(f"no *{suffix} under {dirpath}")


def summarize_trace(trace_dir: str, out_md: str, command: str):
    """Kernel-time table from `rocprofv3 --kernel-trace --stats` CSV output."""
    rows = _read_csv(_find(trace_dir, "kernel_stats.csv"))
    lines = ["# rocprofv3 kernel statistics", "", "Command:", "", "```", command, "```", "",
             "| kernel | calls | average us | total % |", "|---|---|---|---|"]
    for r in rows:
        name = r["Name"]
        short = name.replace("void ", "").replace("(anonymous namespace)::", "").split("(")[0]
        lines.append(f"| {short[:60]} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['Percentage']):.2f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")
    print(f"wrote {out_md}")


def _counter_by_kernel(pmc_dir, counter):
    rows = _read_csv(_find(pmc_dir, "counter_collection.csv"))
    acc = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        k = r["Kernel_Name"]
        acc.setdefault(k, []).append(float(r["Counter_Value"]))
    return acc


def _copy_scales(cf, cw, copy_bytes: int):
    """Scales of FETCH_SIZE and WRITE_SIZE from the plain copy's readings (KiB)
    of copy_bytes in and out; 1 where the run holds no copy kernel.  A copy
    without its size would scale every figure to zero, so it is an error."""
    if (cf or cw) and copy_bytes <= 0:
        raise ValueError("the counters hold the calibration copy: give its size "
                         "(--calibrate-copy-mib)")
    sf = copy_bytes / (cf * 1024.0) if cf else 1.0
    sw = copy_bytes / (cw * 1024.0) if cw else 1.0
    return sf, sw


def summarize_traffic(fetch_dir: str, write_dir: str, out_json: str, workload: str,
                      kernel: str, copy_bytes: int, commands: list):
    """HBM bytes per launch of `kernel` from FETCH_SIZE / WRITE_SIZE (KiB per
    dispatch), each scaled by what the counter reads for a plain copy kernel
    that moves copy_bytes in and copy_bytes out."""
    f = _counter_by_kernel(fetch_dir, "FETCH_SIZE")
    w = _counter_by_kernel(write_dir, "WRITE_SIZE")

    def pick(d, key):
        c = [v for k, v in d.items() if key in k]
        if not c:
            raise KeyError(key)
        return float(np.mean(c[0]))

    def pick_copy(d):
        c = [v for k, v in d.items() if "UnaryFunctor" in k or "MulFunctor" in k]
        return float(np.median(c[0])) if c else None

    kf, kw = pick(f, kernel), pick(w, kernel)
    cf, cw = pick_copy(f), pick_copy(w)
    sf, sw = _copy_scales(cf, cw, copy_bytes)
    d = {"kernel": kernel, "workload": workload, "fetch_kib_per_launch": kf,
         "write_kib_per_launch": kw, "copy_fetch_kib": cf, "copy_write_kib": cw,
         "copy_bytes": copy_bytes, "fetch_scale": sf, "write_scale": sw,
         "hbm_bytes_per_launch": kf * 1024.0 * sf + kw * 1024.0 * sw,
         "source_sha256_16": _kernel_source_hash(), "commands": commands}
    json.dump(d, open(out_json, "w"), indent=1)
    print(f"wrote {out_json}: {d['hbm_bytes_per_launch'] / 1e6:.1f} MB per launch")
    # all kernels, as a table beside it
    md = out_json.replace("_traffic.json", "_traffic.md")
    lines = ["# HBM traffic per dispatch (rocprofv3 FETCH_SIZE / WRITE_SIZE)", "",
             f"Workload {workload}.  Counters are scaled by a plain copy of {copy_bytes} B in and "
             f"out: fetch x{sf:.3f}, write x{sw:.3f}.", "", "Commands:", ""]
    lines += ["```"] + commands + ["```", "",
                                   "| kernel | fetch MB | write MB |", "|---|---|---|"]
    for k in sorted(set(f) | set(w)):
        if "at::native" in k or "rocclr" in k:
            continue
        fk = np.median(f.get(k, [0.0])) * 1024.0 * sf / 1e6
        wk = np.median(w.get(k, [0.0])) * 1024.0 * sw / 1e6
        short = k.replace("void ", "").replace("(anonymous namespace)::", "").split("(")[0]
        lines.append(f"| {short} | {fk:.1f} | {wk:.1f} |")
    open(md, "w").write("\n".join(lines) + "\n")
    print(f"wrote {md}")


HBM_PEAK_GBS = 8000.0
N_SIMD = 1024             # 256 compute units x 4 SIMDs
CLOCK_GHZ = 2.4           # peak engine clock
VALU_CYCLES = 4           # a wave64 VALU instruction on a 16-lane SIMD


def _short_kernel(name: str) -> str:
    return name.replace("void ", "").replace("(anonymous namespace)::", "").split("(")[0]


def summarize_util(trace_dir: str, valu_dir: str, fetch_dir: str, write_dir: str, out_md: str,
                   copy_bytes: int, commands: list):
    """Per kernel, against the MI355X peaks: achieved HBM GB/s (FETCH_SIZE and
    WRITE_SIZE scaled by a plain copy of copy_bytes in and out, over the
    kernel's average duration in the trace), VALU busy (rocprof's VALUBusy
    definition, one quad-cycle per VALU instruction: SQ_INSTS_VALU x 4 cycles
    over 1024 SIMDs x duration x 2.4 GHz) and executed FP64/FP32 vector flop
    rates (SQ_INSTS_VALU_FLOPS_* adds each VALU instruction's flops per lane,
    so x 64 lanes)."""
    dur = {}
    for r in _read_csv(_find(trace_dir, "kernel_stats.csv")):
        dur[_short_kernel(r["Name"])] = float(r["AverageNs"]) * 1e-9

    def by_short(d):   # the counters of one kernel under its short name
        out = {}
        for k, v in d.items():
            out.setdefault(_short_kernel(k), []).extend(v)
        return out

    f = by_short(_counter_by_kernel(fetch_dir, "FETCH_SIZE"))
    w = by_short(_counter_by_kernel(write_dir, "WRITE_SIZE"))

    def copy_kib(d):
        c = [v for k, v in d.items() if "UnaryFunctor" in k or "MulFunctor" in k]
        return float(np.median(c[0])) if c else None

    cf, cw = copy_kib(f), copy_kib(w)
    sf, sw = _copy_scales(cf, cw, copy_bytes)
    cnt = {c: by_short(_counter_by_kernel(valu_dir, c)) for c in
           ("SQ_INSTS_VALU", "SQ_WAVES", "SQ_INSTS_VALU_FLOPS_FP64", "SQ_INSTS_VALU_FLOPS_FP32")}

    def med(d, k):
        v = d.get(k)
        return float(np.median(v)) if v else None

    lines = ["# Kernels against the MI355X peaks (HBM 8 TB/s, FP64 vector 78.6 TFLOP/s, "
             "FP32 vector 157.3 TFLOP/s)", "",
             f"Trace durations; FETCH_SIZE / WRITE_SIZE scaled by a plain copy of {copy_bytes} B "
             f"in and out (fetch x{sf:.3f}, write x{sw:.3f}); VALU busy = SQ_INSTS_VALU x "
             f"{VALU_CYCLES} cycles / ({N_SIMD} SIMDs x duration x {CLOCK_GHZ} GHz), rocprof's "
             "VALUBusy at the peak clock (one quad-cycle per instruction: FP32 operations issue "
             "faster on gfx950, so FP32 work can read above 100%); executed flops = 64 x "
             "SQ_INSTS_VALU_FLOPS_FP64 (or _FP32) per dispatch over the duration.",
             "", "Commands:", "", "```"] + commands + ["```", "",
             "| kernel | us | HBM MB | GB/s | % of HBM peak | VALU instr / wave | VALU busy % "
             "| FP64 TFLOP/s | % of FP64 peak | FP32 TFLOP/s |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    names = sorted(set(cnt["SQ_INSTS_VALU"]) | set(f) | set(w))
    rows = []
    for k in names:
        if "at::native" in k or "rocclr" in k:
            continue
        s = k
        t = dur.get(s)
        if not t:
            continue
        hbm = ((med(f, k) or 0.0) * sf + (med(w, k) or 0.0) * sw) * 1024.0
        gbs = hbm / t / 1e9
        vi, wv = med(cnt["SQ_INSTS_VALU"], k), med(cnt["SQ_WAVES"], k)
        f64, f32 = med(cnt["SQ_INSTS_VALU_FLOPS_FP64"], k), med(cnt["SQ_INSTS_VALU_FLOPS_FP32"], k)
        issue = vi * VALU_CYCLES / (N_SIMD * t * CLOCK_GHZ * 1e9) if vi else None
        tf64 = 64.0 * f64 / t / 1e12 if f64 else 0.0
        tf32 = 64.0 * f32 / t / 1e12 if f32 else 0.0
        rows.append((t, s, hbm, gbs, vi, wv, issue, tf64, tf32))
    for t, s, hbm, gbs, vi, wv, issue, tf64, tf32 in sorted(rows, reverse=True):
        per_wave = f"{vi / wv:.0f}" if vi and wv else "-"
        lines.append(f"| {s} | {t * 1e6:.2f} | {hbm / 1e6:.1f} | {gbs:.0f} | "
                     f"{100 * gbs / HBM_PEAK_GBS:.1f} | {per_wave} | "
                     f"{'-' if issue is None else f'{100 * issue:.1f}'} | {tf64:.2f} | "
                     f"{100 * tf64 / FP64_VECTOR_PEAK_TFLOPS:.1f} | {tf32:.2f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")
    print(f"wrote {out_md}")


def summarize_clock(pmc_dir: str, out_md: str, commands: list, n_xcd: int = 8):
    """Engine clock and VALU occupancy per kernel from one counter run of
    GRBM_GUI_ACTIVE (cycles, summed over the XCDs), SQ_INSTS_VALU,
    SQ_ACTIVE_INST_VALU (quad-cycles) and SQ_WAVES, over each dispatch's own
    start and end timestamps (first dispatch of each kernel)."""
    first = {}
    for r in _read_csv(_find(pmc_dir, "counter_collection.csv")):
        k = _short_kernel(r["Kernel_Name"])
        if "at::native" in k or "rocclr" in k:
            continue
        d = int(r["Dispatch_Id"])
        if k in first and first[k][0] != d:
            continue
        rec = first.setdefault(k, (d, {}))[1]
        rec[r["Counter_Name"]] = float(r["Counter_Value"])
        rec["dur"] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    lines = ["# Engine clock and VALU occupancy per kernel", "",
             f"GRBM_GUI_ACTIVE / {n_xcd} XCDs over the dispatch's duration gives the clock; VALU "
             f"busy = SQ_INSTS_VALU x {VALU_CYCLES} cycles / ({N_SIMD} SIMDs x those cycles); "
             "SQ_ACTIVE_INST_VALU / SQ_INSTS_VALU > 1 where instructions take more than one "
             "quad-cycle.  Kernels shorter than 100 us are left out: the counter window around a "
             "dispatch adds several microseconds of cycles to it.", "", "Command:", "", "```"
             ] + commands + ["```", "",
             "| kernel | us | GHz | VALU busy % | ACTIVE_INST_VALU / INSTS_VALU | VALU pipe busy % |",
             "|---|---|---|---|---|---|"]
    rows = []
    for k, (_, c) in first.items():
        t = c.get("dur", 0.0)
        cyc = c.get("GRBM_GUI_ACTIVE", 0.0) / n_xcd
        vi = c.get("SQ_INSTS_VALU", 0.0)
        if t < 100e-6 or cyc <= 0 or vi <= 0:
            continue
        busy = vi * VALU_CYCLES / (N_SIMD * cyc)
        ratio = c.get("SQ_ACTIVE_INST_VALU", vi) / vi
        rows.append((t, k, cyc / t / 1e9, busy, ratio))
    for t, k, ghz, busy, ratio in sorted(rows, reverse=True):
        lines.append(f"| {k} | {t * 1e6:.1f} | {ghz:.2f} | {100 * busy:.1f} | {ratio:.3f} | "
                     f"{100 * busy * ratio:.1f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")
    print(f"wrote {out_md}")


def calibrate_copy(nbytes: int, reps: int = 3):
    """A plain elementwise copy of known size, for counter calibration."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()


def _alive(b, k):
    return int(b.read_state(k)["alive"].sum())


def bench_batch(args):
    """64 independent runs of a parameter scan (N from 1e4 to 1e6, T_e 1-5 eV,
    n_e 1e14-1e16), l_max = 16, in one batch: aggregate particle-steps/s of
    the batched launch, and of the same runs one after another (in the same
    precision and as plain FP64 runs)."""
    from dataclasses import replace

    import torch

    from paper_2111_13072_amd import sim as S
    from paper_2111_13072_amd import workload as W

    wls = W.batch_workloads()
    fp32 = args.precision == "fp32c"
    cp = S.SimParams(l_max=wls[0].l_max, precision=S.SIM_FP32_COMP if fp32 else S.SIM_FP64)
    n_steps = max(wls[0].n_steps, args.warmup + args.steps + args.profile_steps + 1)
    members = []
    for wl in wls:
        st = wl.particles()
        members.append(S.Member(pos=st.pos, vel=st.vel, u_asy=wl.drive(n_steps), ntilde=wl.ntilde,
                                r_out=wl.r_out, dt=wl.dt))
    n_all = sum(wl.n for wl in wls)
    print(f"[bench] batch of {len(wls)} runs, {n_all} particles, l_max={cp.l_max} "
          f"{args.precision}", file=sys.stderr, flush=True)
    tuning = None
    if args.autotune:
        from paper_2111_13072_amd import tune as T
        tuned = T.autotune(T.batch_builder(members), cp, n_all, steps=5, warmup=2)
        cp = tuned.apply(cp)
        tuning = {"sort_bucket": tuned.sort_bucket, "carry_chunk": tuned.carry_chunk,
                  "near_split": tuned.near_split,
                  "trial_ms_per_step": round(tuned.ms_per_step, 4),
                  "default_trial_ms_per_step": round(tuned.default_ms_per_step, 4)}
        print(f"[bench] autotune: {tuning}", file=sys.stderr, flush=True)
    b = S.Batch(cp, members)
    b.step(args.warmup)
    b.sync()
    alive0 = [_alive(b, k) for k in range(len(wls))]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(args.steps)
    b.sync()
    t1 = time.perf_counter()
    alive1 = [_alive(b, k) for k in range(len(wls))]
    elapsed = t1 - t0
    live = 0.5 * (sum(alive0) + sum(alive1))
    value = live * args.steps / elapsed
    print(f"[bench] batch: {args.steps} steps in {elapsed:.3f} s: {value:.4e} particle-steps/s",
          file=sys.stderr, flush=True)
    kms = b.profile(args.profile_steps)
    b.close()

    # the same runs one after another (each its own handle and graph), in the
    # batch's precision and, for FP32c, also as plain FP64 runs
    def sequential(params, label):
        total = 0.0
        for k, mb in enumerate(members):
            with S.Batch(params, [mb]) as one:
                one.step(args.warmup)
                one.sync()
                ta = time.perf_counter()
                one.step(args.seq_steps)
                one.sync()
                total += (time.perf_counter() - ta) / args.seq_steps
            if k % 16 == 15:
                print(f"[bench] sequential {label}: {k + 1} runs timed", file=sys.stderr,
                      flush=True)
        return live / total

    seq_value = sequential(cp, args.precision)
    seq_fp64 = sequential(replace(cp, precision=S.SIM_FP64), "fp64") if fp32 else seq_value
    dom = "field_push"
    flops = algorithmic_flops_per_particle(cp.l_max) * live
    achieved = flops / (kms[dom] * 1e-3) / 1e12
    peak = FP32_VECTOR_PEAK_TFLOPS if fp32 else FP64_VECTOR_PEAK_TFLOPS
    line = {"metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32+f64" if fp32 else "f64", "data": "synthetic",
            "config": {"workload": f"batch{len(wls)}-L{cp.l_max}", "members": len(wls),
                       "n_particles": n_all, "l_max": cp.l_max, "precision": args.precision,
                       "parallelism": "single-gpu"},
            "sequential_value": seq_value, "batch_speedup": value / seq_value,
            "sequential_fp64_value": seq_fp64, "speedup_vs_fp64_runs": value / seq_fp64,
            "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                         "frac": achieved / peak, "traffic": None, "kernel": dom,
                         "kernel_ms": kms[dom],
                         "per_kernel_ms": {k: round(v, 5) for k, v in kms.items()}}}
    if tuning is not None:
        line["tuning"] = tuning
    print(json.dumps(line), flush=True)
    return 0


def bench_serve(args):
    """Continuous batching of Poisson arrivals (N log-uniform in [1e4, 4e6],
    l_max in {8, 16, 32}, 2e3-2e4 steps, T_e 1-5 eV, n_e 1e14-1e16) at 80%
    offered device load, with resident pools holding 80% of the GPU's HBM:
    latency percentiles from arrival to completion, and the aggregate
    particle-steps/s over the whole service."""
    from paper_2111_13072_amd import serve as SV
    from paper_2111_13072_amd import sim as S

    import torch

    fp32 = args.precision == "fp32c"
    steps_range = tuple(int(float(v)) for v in args.serve_steps.split(","))
    reqs = SV.request_stream(seed=5, duration_s=args.serve_seconds, load=0.8,
                             steps_range=steps_range)
    free_b, total_b = torch.cuda.mem_get_info()
    budget = (int(args.serve_budget_gib * 2**30) if args.serve_budget_gib > 0
              else int(args.serve_hbm_fraction * total_b))
    print(f"[bench] serving {len(reqs)} requests over {args.serve_seconds:.0f} s, steps "
          f"{steps_range}, pools of {budget / 2**30:.1f} GiB ({budget / total_b:.0%} of "
          f"{total_b / 2**30:.0f} GiB HBM)", file=sys.stderr, flush=True)
    srv = SV.Server(budget, precision=S.SIM_FP32_COMP if fp32 else S.SIM_FP64,
                    tick_steps=args.serve_tick_steps, tick_seconds=args.serve_tick_seconds,
                    small_max=args.serve_small_max, max_steps=steps_range[1])
    held = torch.cuda.memory_reserved()
    t0 = time.perf_counter()
    try:
        done = srv.run(reqs, log=lambda m: print(f"[serve] {m}", file=sys.stderr, flush=True))
    finally:
        srv.close()
    wall = time.perf_counter() - t0
    work = sum(d.n * d.n_steps for d in done)
    # time-averaged fraction of the pools' particle slots holding a request
    occupancy = sum(d.n * (d.finished - d.admitted) for d in done) / (wall * sum(srv.slots.values()))
    lat = SV.latency_summary(done)
    isolated = _isolated_fp64(done, reqs, args)
    line = {"metric": METRIC, "value": work / wall, "unit": "particle-steps/s", "n_gpus": 1,
            "steps": None, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64" if fp32 else "f64",
            "data": "synthetic",
            "config": {"workload": "served-poisson", "requests": len(reqs),
                       "arrival_window_s": args.serve_seconds, "offered_load": 0.8,
                       "l_max": [8, 16, 32], "n_range": [1e4, 4e6],
                       "steps_range": list(steps_range),
                       "pools_gib": budget / 2**30, "hbm_gib": total_b / 2**30,
                       "pools_fraction_of_hbm": held / total_b,
                       "tick_steps": args.serve_tick_steps,
                       "tick_seconds": args.serve_tick_seconds,
                       "small_max": args.serve_small_max,
                       "precision": args.precision, "parallelism": "single-gpu"},
            "latency_s": lat, "rejected": len(srv.rejected), "wall_s": wall,
            "slot_occupancy": occupancy,
            "isolated_fp64": isolated}
    print(json.dumps(line), flush=True)
    return 0


def _isolated_fp64(done, reqs, args, sample: int = 8, steps: int = 40):
    """Plain per-request FP64 baseline on a sample of the served requests
    (spread over the size range): each run alone as one simulation, `steps`
    timed steps scaled to its step count; the served latency over that time."""
    import torch

    from paper_2111_13072_amd import sim as S

    if not done:
        return None
    by_id = {r.rid: r for r in reqs}
    ordered = sorted(done, key=lambda d: d.n * d.n_steps)
    pick = [ordered[round(i * (len(ordered) - 1) / max(sample - 1, 1))] for i in range(sample)]
    pick = list({d.rid: d for d in pick}.values())
    ratios, iso_work, iso_time = [], 0.0, 0.0
    for d in pick:
        wl = by_id[d.rid].workload()
        st = wl.particles()
        prm = S.SimParams(ntilde=wl.ntilde, l_max=wl.l_max, r_out=wl.r_out, dt=wl.dt,
                          precision=S.SIM_FP64)
        with S.Sim(prm, st.pos, st.vel, wl.drive(steps + 5)) as sim:
            sim.step(5)
            sim.sync()
            torch.cuda.synchronize()
            ta = time.perf_counter()
            sim.step(steps)
            sim.sync()
            per_step = (time.perf_counter() - ta) / steps
        t_iso = per_step * d.n_steps
        ratios.append(d.latency / t_iso)
        iso_work += d.n * d.n_steps
        iso_time += t_iso
    print(f"[bench] isolated FP64 baseline on {len(pick)} requests", file=sys.stderr, flush=True)
    return {"requests": len(pick), "steps_timed": steps,
            "particle_steps_per_s": iso_work / iso_time,
            "served_latency_over_isolated_p50": float(np.median(ratios)),
            "served_latency_over_isolated_max": float(np.max(ratios))}


def bench_spectrum(args):
    """The single large run as specified: 2e6 electrons, l_max 16, 20,000
    steps, FP64 and FP32-compensated, each as a driven run (the paper's
    impulse, u_asy = 1 at the first step) and an undriven twin from the same
    state.  Reports, per precision, the damped-sine fit of the twin
    difference on t <= 20 (resonance c, full width 2b; Sec. 4), the peak and
    half-width of Re Y of that fit's transform, and of Re Y from the Fourier
    transform of the record up to t = 40 (after that the twins' chaotic
    divergence, not the response, dominates the difference), and their FP32c /
    FP64 ratios; plus the throughput of the runs."""
    import torch

    from paper_2111_13072_amd import analysis as A
    from paper_2111_13072_amd import sim as S
    from paper_2111_13072_amd import workload as W

    wl = W.LARGE
    steps = args.spectrum_steps
    st = wl.particles()
    t = np.arange(steps) * wl.dt
    out = {}
    for name, prec in (("fp64", S.SIM_FP64), ("fp32c", S.SIM_FP32_COMP)):
        qs = []
        elapsed = 0.0
        for drive in (True, False):
            u = W.impulse_drive(steps, 1.0) if drive else np.zeros(steps)
            prm = S.SimParams(ntilde=wl.ntilde, l_max=wl.l_max, precision=prec)
            with S.Sim(prm, st.pos, st.vel, u) as sim:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sim.step(steps)
                sim.sync()
                elapsed += time.perf_counter() - t0
                qs.append(sim.read_response(0, steps))
            print(f"[bench] spectrum {name} {'driven' if drive else 'undriven'}: {steps} steps",
                  file=sys.stderr, flush=True)
        diff = A.twin_difference(*qs)
        m = t <= 20.0
        fit = A.fit_damped_sine(t[m], diff[m], 1.0)
        omega = np.linspace(0.01, 1.5, 3000)
        fit_peak, fit_fwhm = A.admittance_from_fit(fit, omega).peak()
        early = t <= 40.0
        spec = A.admittance(diff[early], W.impulse_drive(int(early.sum()), 1.0), wl.dt,
                            pad=16, w_max=1.5)
        w_peak, fwhm = spec.peak()
        out[name] = {"fit_c": fit.frequency, "fit_2b": fit.fwhm, "fit_re_y_peak": fit_peak,
                     "fit_re_y_fwhm": fit_fwhm, "fft40_re_y_peak": w_peak,
                     "fft40_re_y_fwhm": fwhm, "particle_steps_per_s": 2 * wl.n * steps / elapsed,
                     "fit_points": int(m.sum())}
    f64, f32 = out["fp64"], out["fp32c"]
    line = {"metric": METRIC, "value": f32["particle_steps_per_s"], "unit": "particle-steps/s",
            "n_gpus": 1, "steps": steps, "warmup": 0, "ms_per_step": None,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": f"{wl.name}-spectrum", "n_particles": wl.n, "l_max": wl.l_max,
                       "steps": steps, "drive": "impulse 1 at step 0", "parallelism": "single-gpu"},
            "spectra": out,
            "fp32c_over_fp64": {k: f32[k] / f64[k] for k in (
                "fit_c", "fit_2b", "fit_re_y_peak", "fit_re_y_fwhm", "fft40_re_y_peak",
                "fft40_re_y_fwhm")}}
    print(json.dumps(line), flush=True)
    return 0


def bench_sweep(args):
    """Scale and accuracy sweep: 1.6e7 particles at l_max 8, 16, 32 for
    n_e in {1e15, 1e16} m^-3 and T_e in {1, 3, 5} eV (FP64, or
    FP32-compensated with --precision fp32c): one JSON line per run with its
    particle-steps/s and kernel times, each timed over --steps steps after
    --warmup."""
    from paper_2111_13072_amd import sim as S
    from paper_2111_13072_amd import workload as W

    fp32 = args.precision == "fp32c"
    ls = tuple(int(v) for v in args.sweep_l.split(","))
    plasmas = [(n_e, te) for n_e in (1e15, 1e16) for te in (1.0, 3.0, 5.0)]
    if args.sweep_one_plasma:
        plasmas = [(1e15, 3.0)]
    for L in ls:
        for n_e, te in plasmas:
            if True:
                wl = W.sweep_workload(L, n_e, te)
                st = wl.particles()
                n_total = args.warmup + args.steps + args.profile_steps + 1
                prm = S.SimParams(d=wl.d, eps_r=wl.eps_r, r_out=wl.r_out, dt=wl.dt,
                                  ntilde=wl.ntilde, l_max=L,
                                  precision=S.SIM_FP32_COMP if fp32 else S.SIM_FP64)
                with S.Sim(prm, st.pos, st.vel, wl.drive(n_total)) as sim:
                    sim.step(args.warmup)
                    sim.sync()
                    t0 = time.perf_counter()
                    sim.step(args.steps)
                    sim.sync()
                    el = time.perf_counter() - t0
                    kms = sim.profile(args.profile_steps)
                flops = algorithmic_flops_per_particle(L) * wl.n / (kms["field_push"] * 1e-3) / 1e12
                peak = FP32_VECTOR_PEAK_TFLOPS if fp32 else FP64_VECTOR_PEAK_TFLOPS
                print(json.dumps({"workload": wl.name, "precision": args.precision,
                                  "value": wl.n * args.steps / el, "unit": "particle-steps/s",
                                  "ms_per_step": 1e3 * el / args.steps,
                                  "field_push_frac": flops / peak,
                                  "per_kernel_ms": {k: round(v, 4) for k, v in kms.items()}}),
                      flush=True)
                del st
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--workload", default="scale",
                    choices=["scale", "large", "small", "batch64", "serve", "sweep", "spectrum"],
                    help="scale: 1.6e7 electrons, l_max 16, T_e 3 eV, n_e 1e15 (the largest "
                         "single-GPU run; FP32-compensated with the FP64 run beside it); large: "
                         "2e6, l_max 16; small: 1e4, l_max 8")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="serve: length of the Poisson arrival window")
    ap.add_argument("--serve-budget-gib", type=float, default=0.0,
                    help="serve: device memory of the pools (0: --serve-hbm-fraction of HBM)")
    ap.add_argument("--serve-hbm-fraction", type=float, default=0.8)
    ap.add_argument("--serve-tick-steps", type=int, default=500,
                    help="serve: most steps per tick of a pool")
    ap.add_argument("--serve-tick-seconds", type=float, default=0.025,
                    help="serve: a pool's tick is about this long (0: always --serve-tick-steps)")
    ap.add_argument("--spectrum-steps", type=int, default=20000,
                    help="spectrum: steps of each run (driven and undriven, both precisions)")
    ap.add_argument("--serve-steps", default="2000,20000",
                    help="serve: range of the requests' step counts")
    ap.add_argument("--serve-small-max", type=int, default=200000,
                    help="serve: requests of at most this many particles get pools of their own "
                         "(0: one pool per l_max)")
    ap.add_argument("--sweep-l", default="8,16,32", help="sweep: the l_max values")
    ap.add_argument("--sweep-one-plasma", action="store_true",
                    help="sweep: only n_e 1e15 m^-3, T_e 3 eV")
    ap.add_argument("--seq-steps", type=int, default=20,
                    help="batch64: timed steps of each member run alone, for comparison")
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32c"],
                    help="default: fp32c for the scale workload, fp64 otherwise")
    ap.add_argument("--no-fp64-leg", action="store_true",
                    help="fp32c single runs: skip the FP64 run of the same state")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="single runs and batch64: choose sort bucket and carry chunk sizes by "
                         "short timed trials first (outside the timed region)")
    ap.add_argument("--cpu-budget-s", type=float, default=15.0)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="after the run, launch a plain copy of this size (counter calibration)")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("TRACE_DIR", "OUT_MD"))
    ap.add_argument("--summarize-traffic", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT_JSON"))
    ap.add_argument("--summarize-util", nargs=5,
                    metavar=("TRACE_DIR", "VALU_DIR", "FETCH_DIR", "WRITE_DIR", "OUT_MD"))
    ap.add_argument("--summarize-clock", nargs=2, metavar=("PMC_DIR", "OUT_MD"))
    ap.add_argument("--command", default="", help="command recorded in a summary")
    args = ap.parse_args(argv)

    if args.summarize_trace:
        summarize_trace(args.summarize_trace[0], args.summarize_trace[1], args.command)
        return 0
    if args.summarize_traffic:
        from paper_2111_13072_amd import workload as W
        wl_name = {"scale": W.SCALE, "large": W.LARGE, "small": W.SMALL_FP64}[args.workload].name
        if (args.precision or ("fp32c" if args.workload == "scale" else "fp64")) == "fp32c":
            wl_name += "-fp32c"
        summarize_traffic(args.summarize_traffic[0], args.summarize_traffic[1],
                          args.summarize_traffic[2], wl_name, "field_push",
                          args.calibrate_copy_mib * 2**20, args.command.split(" ;; "))
        return 0
    if args.summarize_clock:
        summarize_clock(args.summarize_clock[0], args.summarize_clock[1], args.command.split(" ;; "))
        return 0
    if args.summarize_util:
        summarize_util(*args.summarize_util, args.calibrate_copy_mib * 2**20,
                       args.command.split(" ;; "))
        return 0

    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported: this "
              "build steps one simulation (or one batch) on one GPU and has no multi-GPU path",
              file=sys.stderr)
        return 2

    import torch

    from paper_2111_13072_amd import workload as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "batch64":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "sweep":
        return bench_sweep(args)
    if args.workload == "spectrum":
        return bench_spectrum(args)
    wl = {"scale": W.SCALE, "large": W.LARGE, "small": W.SMALL_FP64}[args.workload]
    precision = args.precision or ("fp32c" if args.workload == "scale" else "fp64")
    return bench_single(args, wl, precision)


def _leg(wl, st, precision: str, args, u, field: bool):
    """One handle of the workload in one precision: W warmup steps, then K
    timed steps (HIP graph replays on torch's stream, bracketed by device
    synchronisation), then per-kernel times from HIP events over a few more
    steps.  Particle-steps count the particles alive at the start and the end
    of the timed window (their mean)."""
    import torch

    from paper_2111_13072_amd import sim as S

    prm = S.SimParams(d=wl.d, eps_r=wl.eps_r, r_out=wl.r_out, dt=wl.dt, ntilde=wl.ntilde,
                      ion_density=1.0, l_max=wl.l_max,
                      precision=S.SIM_FP32_COMP if precision == "fp32c" else S.SIM_FP64)
    out = {"params": prm}
    if args.autotune:
        from paper_2111_13072_amd import tune as T
        tuned = T.autotune(T.sim_builder(st.pos, st.vel), prm, wl.n)
        prm = tuned.apply(prm)
        out["tuning"] = {"sort_bucket": tuned.sort_bucket, "carry_chunk": tuned.carry_chunk,
                         "near_split": tuned.near_split,
                         "trial_ms_per_step": round(tuned.ms_per_step, 4),
                         "default_trial_ms_per_step": round(tuned.default_ms_per_step, 4)}
        print(f"[bench] autotune: {out['tuning']}", file=sys.stderr, flush=True)
    print(f"[bench] {wl.name} {precision}: create", file=sys.stderr, flush=True)
    with S.Sim(prm, st.pos, st.vel, u) as sim:
        out["E"] = sim.eval_field() if field else None
        sim.step(args.warmup)
        n_before = sim.counts()["alive"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(args.steps)
        sim.sync()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        n_after = sim.counts()["alive"]
        out["kms"] = sim.profile(args.profile_steps)
    out["elapsed"] = t1 - t0
    out["live"] = 0.5 * (n_before + n_after)
    out["value"] = out["live"] * args.steps / out["elapsed"]
    out["ms_per_step"] = 1e3 * out["elapsed"] / args.steps
    print(f"[bench] {wl.name} {precision}: {args.steps} steps in {out['elapsed']:.3f} s, "
          f"{out['value']:.4e} particle-steps/s", file=sys.stderr, flush=True)
    return out


def bench_single(args, wl, precision: str):
    """One simulation of the workload: the timed leg in `precision`, and for
    the FP32-compensated mode the plain FP64 run of the same state beside it
    (the per-run FP64 baseline on the same GPU).  The roofline is the field
    kernel's; the CPU baseline times the oracle on a sample of the same state
    and gives the field error of each leg on that sample."""
    import torch

    torch.cuda.set_device(0)
    st = wl.particles()
    n_total = args.warmup + args.steps + args.profile_steps + 1
    u = wl.drive(max(n_total, 64))
    fp32 = precision == "fp32c"
    print(f"[bench] workload {wl.name}: n={wl.n} l_max={wl.l_max} {precision}, "
          f"warmup={args.warmup} steps={args.steps}", file=sys.stderr, flush=True)
    want_field = not args.no_cpu_baseline
    main_leg = _leg(wl, st, precision, args, u, want_field)
    fp64_leg = None
    if fp32 and not args.no_fp64_leg:
        fp64_leg = _leg(wl, st, "fp64", args, u, want_field)
    prm = main_leg["params"]
    kms = main_leg["kms"]
    dom = "field_push"
    flops = algorithmic_flops_per_particle(wl.l_max) * main_leg["live"]
    achieved = flops / (kms[dom] * 1e-3) / 1e12
    traffic = _traffic_from_profiles(dom, wl.name + ("-fp32c" if fp32 else ""))
    peak = FP32_VECTOR_PEAK_TFLOPS if fp32 else FP64_VECTOR_PEAK_TFLOPS
    roof = {"bound": "alu", "achieved": achieved, "peak": peak,
            "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
            "kernel": dom, "kernel_ms": kms[dom],
            "flops_per_launch": flops,
            "per_kernel_ms": {k: round(v, 5) for k, v in kms.items()}}
    line = {"metric": METRIC, "value": main_leg["value"], "unit": "particle-steps/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": main_leg["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None,
            "dtype": "f32+f64" if fp32 else "f64", "data": "synthetic",
            "config": {"workload": wl.name, "n_particles": wl.n, "seed": wl.seed,
                       "l_max": wl.l_max, "m_mode": "full", "precision": precision, "tile": 64,
                       "n_e_m3": wl.n_e, "T_e_eV": wl.t_e_ev, "r_out": wl.r_out, "dt": wl.dt,
                       "parallelism": "single-gpu"},
            "roofline": roof}
    if "tuning" in main_leg:
        line["tuning"] = main_leg["tuning"]
    if fp64_leg is not None:
        line["fp64_run"] = {"value": fp64_leg["value"], "ms_per_step": fp64_leg["ms_per_step"],
                            "speedup_of_fp32c": main_leg["value"] / fp64_leg["value"],
                            "per_kernel_ms": {k: round(v, 5) for k, v in fp64_leg["kms"].items()}}
    if not args.no_cpu_baseline:
        fields = {precision: main_leg["E"]}
        if fp64_leg is not None:
            fields["fp64"] = fp64_leg["E"]
        rec, errs, ns = cpu_baseline(wl, st, prm, float(u[0]), prm.q_surface0,
                                     args.cpu_budget_s, fields)
        line["cpu_baseline"] = rec
        line["field_rel_err_vs_oracle"] = errs[precision]
        if fp64_leg is not None:
            line["fp64_run"]["field_rel_err_vs_oracle"] = errs["fp64"]
        line["field_err_sample"] = ns
    print(json.dumps(line), flush=True)
    if args.calibrate_copy_mib:
        calibrate_copy(args.calibrate_copy_mib * 2**20)
    return 0


if __name__ == "__main__":
    sys.exit(main())
