"""Autotuner for the launch sizes that leave the results unchanged.

Three sizes of the step are free: the mean number of particles per radial
sort bucket (sim_params.sort_bucket: fewer per bucket means a longer
histogram scan and fewer key comparisons in the rank kernel), the groups of
256 particle slots per carry chunk (sim_params.carry_chunk: shorter chunks
mean more parallel carry work and a longer scan over chunks) and, in FP64,
the near field's block (sim_params.near_split: half tiles of 32 particles,
the built-in where the precision allows it, halve the pair sums and double
the tile sums the field kernel reads; whole tiles of 64 the opposite, which
pays at large l_max, where those sums' bytes grow as l_max^2).  The tile is
the wavefront (64) and the moment kernel's channel batch is fixed by its LDS
layout.  None changes the physics: the bucket size only changes the order in
which the sort finds the exact radial order, the chunk length only the
rounding order of the FP64 carries, the near-field block only how the same
pair sum is split between the pairwise and the scan form (≤ 1e-13 of the RMS
field in FP64; in FP32 whole tiles are never less accurate than half tiles,
so the search is safe in both precisions).

The search is coordinate-wise: the bucket size over BUCKETS with the built-in
chunk, then the chunk over CHUNKS with the best bucket, then the
near-field block over SPLITS; each candidate is timed on the caller's own
workload (a runner built from the candidate parameters), median of `reps`
timings of `steps` steps after `warmup`.
Results are cached per shape class (particles to the nearest power of two,
l_max, m mode, precision), in memory and optionally in a JSON file.
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import asdict, dataclass, field, replace
from typing import Callable, Dict, List, Optional

from . import sim as S

BUCKETS = (4, 8, 16, 32, 64)
CHUNKS = (0, 8, 16, 32, 64, 128)   # 0: the built-in choice by member size
SPLITS = (0, -1)                   # near-field block: 0 built-in, -1 whole tiles

# A runner for one candidate: runner(k) advances k steps and waits for them.
Runner = Callable[[int], None]
Build = Callable[[S.SimParams], "RunnerHandle"]


class RunnerHandle:
    """What a build function returns: run(k) and close()."""

    def __init__(self, run: Runner, close: Callable[[], None]):
        self.run = run
        self.close = close


@dataclass
class Trial:
    sort_bucket: int
    carry_chunk: int
    ms_per_step: float
    near_split: int = 0


@dataclass
class Tuned:
    sort_bucket: int
    carry_chunk: int
    ms_per_step: float        # of the chosen candidate
    default_ms_per_step: float  # of the built-in choice (8, automatic, built-in block)
    trials: List[Trial] = field(default_factory=list)
    near_split: int = 0

    def apply(self, params: S.SimParams) -> S.SimParams:
        return replace(params, sort_bucket=self.sort_bucket, carry_chunk=self.carry_chunk,
                       near_split=self.near_split)


def shape_key(params: S.SimParams, n: int) -> str:
    return (f"n{1 << max(0, round(math.log2(max(n, 1))))}-L{params.l_max}-m{params.m_mode}"
            f"-p{params.precision}")


def time_steps(handle: RunnerHandle, steps: int, warmup: int, reps: int) -> float:
    """Median wall time per step (ms) of `reps` runs of `steps` steps."""
    handle.run(warmup)
    out = []
    for _ in range(reps):
        t0 = time.perf_counter()
        handle.run(steps)
        out.append((time.perf_counter() - t0) * 1e3 / steps)
    out.sort()
    return out[len(out) // 2]


class Cache:
    """Tuned sizes per shape class; persisted to `path` when given."""

    def __init__(self, path: Optional[str] = None):
        self.path = path
        self.entries: Dict[str, dict] = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.entries = json.load(f)

    def get(self, key: str) -> Optional[Tuned]:
        e = self.entries.get(key)
        if e is None:
            return None
        return Tuned(e["sort_bucket"], e["carry_chunk"], e["ms_per_step"],
                     e["default_ms_per_step"], [Trial(**t) for t in e.get("trials", [])],
                     e.get("near_split", 0))

    def put(self, key: str, t: Tuned):
        self.entries[key] = asdict(t)
        if self.path:
            d = os.path.dirname(self.path)
            if d:
                os.makedirs(d, exist_ok=True)
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.entries, f, indent=1)
            os.replace(tmp, self.path)


def autotune(build: Build, params: S.SimParams, n: int, *, steps: int = 10, warmup: int = 3,
             reps: int = 3, cache: Optional[Cache] = None,
             buckets=BUCKETS, chunks=CHUNKS, splits=SPLITS,
             measure: Callable[[RunnerHandle, int, int, int], float] = time_steps) -> Tuned:
    """Tune sort_bucket, carry_chunk and near_split for a workload of
    n particles with these parameters.  build(params) must return a
    RunnerHandle over the caller's workload built with `params`."""
    key = shape_key(params, n)
    if cache is not None:
        hit = cache.get(key)
        if hit is not None:
            return hit
    timed: Dict[tuple, float] = {}

    def trial(b: int, c: int, s: int = 0) -> float:
        if (b, c, s) not in timed:
            h = build(replace(params, sort_bucket=b, carry_chunk=c, near_split=s))
            try:
                timed[(b, c, s)] = measure(h, steps, warmup, reps)
            finally:
                h.close()
        return timed[(b, c, s)]

    best_b = min(buckets, key=lambda b: (trial(b, 0), b))
    best_c = min(chunks, key=lambda c: (trial(best_b, c), c))
    best_s = min(splits, key=lambda s: (trial(best_b, best_c, s), abs(s)))
    default = trial(8, 0) if 8 in buckets else timed[(best_b, 0, 0)]
    result = Tuned(best_b, best_c, timed[(best_b, best_c, best_s)], default,
                   [Trial(b, c, ms, s) for (b, c, s), ms in sorted(timed.items())], best_s)
    if cache is not None:
        cache.put(key, result)
    return result


def sim_builder(pos, vel, n_steps: int = 1000) -> Build:
    """Builds single simulations of this state with a zero drive of n_steps
    (enough for the warmup and timed steps of a search)."""
    import numpy as np

    def build(p: S.SimParams) -> RunnerHandle:
        s = S.Sim(p, pos, vel, np.zeros(n_steps))

        def run(k: int):
            s.step(k)
            s.sync()

        return RunnerHandle(run, s.close)

    return build


def batch_builder(members, slot_capacity: int = 0) -> Build:
    """Builds batches of these members (sim.Member)."""

    def build(p: S.SimParams) -> RunnerHandle:
        b = S.Batch(p, members, slot_capacity=slot_capacity)

        def run(k: int):
            b.step(k)
            b.sync()

        return RunnerHandle(run, b.close)

    return build
