"""Throughput benchmark: particle-steps/s of the full simulation step on one MI355X.

A step is one pass of the whole hot path (radial sort, harmonic moments,
prefix/suffix carry scans, boundary response + drive, field + leapfrog push)
over all particles.  Default workload: 2e6 electrons, l_max = 16, uniform
shell 1 < r < 5, T_e = 2 eV, n_e = 1e15 m^-3, +-1 V Gaussian pulse.

Prints ONE JSON line.  `roofline` reports the dominant kernel (field_push)
against the FP64 vector peak; `cpu_baseline` times the CPU oracle on a
bounded sample of the same workload and also gives the field error of the
GPU against it.
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


def _kernel_source_hash() -> str:
    p = os.path.join(ROOT, "paper_2111_13072_amd", "csrc", "mrpsim.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


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


def cpu_baseline(wl, st, prm, E_gpu, u_now, q_s, budget_s: float):
    """Oracle field + push at a bounded random sample of particles of the same
    state; returns the baseline record and the GPU field error on the sample."""
    import oracle as O

    op = O.Params(d=prm.d, eps_r=prm.eps_r, r_out=prm.r_out, dt=prm.dt, ntilde=prm.ntilde,
                  ion_density=prm.ion_density, l_max=prm.l_max, m_mode=prm.m_mode,
                  probe_bc=prm.probe_bc, wall_bc=prm.wall_bc, seed=prm.seed)
    rng = np.random.default_rng(12345)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    first = np.sort(rng.choice(wl.n, 8 * threads, replace=False))
    t0 = time.perf_counter()
    E0, _ = O.field(op, st.pos, q_surface=q_s, u_asy=u_now, targets=first)
    t_first = time.perf_counter() - t0
    per = t_first / len(first)
    extra = int(max(0, (budget_s - t_first) / per))
    rest = np.setdiff1d(np.sort(rng.choice(wl.n, min(extra, wl.n // 2), replace=False)), first)
    t1 = time.perf_counter()
    E1, _ = O.field(op, st.pos, q_surface=q_s, u_asy=u_now, targets=rest)
    t_rest = time.perf_counter() - t1
    targets = np.concatenate([first, rest])
    Eo = np.concatenate([E0, E1])
    # the push of the sampled particles (part of a particle-step)
    t2 = time.perf_counter()
    v = st.vel[targets] - Eo * prm.dt
    _ = st.pos[targets] + v * prm.dt
    t_push = time.perf_counter() - t2
    total = t_first + t_rest + t_push
    rms = float(np.sqrt(np.mean(np.sum(Eo * Eo, axis=1))))
    err = float(np.max(np.abs(E_gpu[targets] - Eo)) / rms)
    rec = {"value": len(targets) / total, "unit": "particle-steps/s", "cores": threads,
           "kind": "oracle",
           "sample": f"pair-sum field + leapfrog push of {len(targets)} random particles of the "
                     f"{wl.n}-particle, l_max={wl.l_max} state (one step), {total:.1f} s"}
    return rec, err, len(targets)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--workload", default="large", choices=["large", "small"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget-s", type=float, default=15.0)
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(one simulation is one GPU's work; see DESIGN.md for how it would shard)",
              file=sys.stderr)
        return 2

    import torch

    from paper_2111_13072_amd import sim as S
    from paper_2111_13072_amd import workload as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    wl = W.LARGE if args.workload == "large" else W.SMALL_FP64
    st = wl.particles()
    n_total = args.warmup + args.steps + args.profile_steps + 1
    u = wl.drive(max(n_total, 64))
    prm = S.SimParams(d=wl.d, eps_r=wl.eps_r, r_out=wl.r_out, dt=wl.dt, ntilde=wl.ntilde,
                      ion_density=1.0, l_max=wl.l_max, precision=S.SIM_FP64)
    print(f"[bench] workload {wl.name}: n={wl.n} l_max={wl.l_max} fp64, "
          f"warmup={args.warmup} steps={args.steps}", file=sys.stderr, flush=True)

    sim = S.Sim(prm, st.pos, st.vel, u)
    E_gpu = sim.eval_field() if not args.no_cpu_baseline else None
    s0 = sim.read_state()
    u_now, q_s0 = float(u[0]), s0["q_surface"]

    sim.step(args.warmup)
    torch.cuda.synchronize()
    n_before = int(sim.read_state()["alive"].sum())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n_after = int(sim.read_state()["alive"].sum())
    elapsed = t1 - t0
    particle_steps = 0.5 * (n_before + n_after) * args.steps
    value = particle_steps / elapsed
    print(f"[bench] timed {args.steps} steps in {elapsed:.3f} s: {value:.4e} particle-steps/s",
          file=sys.stderr, flush=True)

    kms = sim.profile(args.profile_steps)
    sim.close()
    dom = "field_push"
    t_dom = kms[dom] * 1e-3
    flops = algorithmic_flops_per_particle(wl.l_max) * 0.5 * (n_before + n_after)
    achieved = flops / t_dom / 1e12
    traffic = _traffic_from_profiles(dom, wl.name)
    roof = {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": traffic,
            "kernel": dom, "kernel_ms": kms[dom],
            "per_kernel_ms": {k: round(v, 5) for k, v in kms.items()}}

    line = {"metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": wl.name, "n_particles": wl.n, "l_max": wl.l_max,
                       "m_mode": "full", "precision": "fp64", "tile": 64,
                       "n_e_m3": wl.n_e, "T_e_eV": wl.t_e_ev, "r_out": wl.r_out, "dt": wl.dt,
                       "parallelism": "single-gpu"},
            "roofline": roof}
    if not args.no_cpu_baseline:
        rec, err, ns = cpu_baseline(wl, st, prm, E_gpu, u_now, q_s0, args.cpu_budget_s)
        line["cpu_baseline"] = rec
        line["field_rel_err_vs_oracle"] = err
        line["field_err_sample"] = ns
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
