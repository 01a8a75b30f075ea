"""Continuous-batching service of independent simulations.

Requests (a plasma, a particle count, an l_max and a number of steps) arrive
over time.  The server keeps resident batches ("pools") per l_max class, and
optionally per size class, each on its own HIP stream.  Whenever a pool's
tick (a fixed number of steps of all its members) has completed, the server
retires the members that reached their length after reading their response,
admits waiting requests when its slots, chunks, buckets and memory allow
(first come, first served within the pool), and launches the next tick; it
never waits on one pool to tend another.  A request's response equals, bit
for bit, that of the same request run alone (members never interact).

The particles of newly arrived requests are generated on worker threads
while the device steps the pools.
"""
from __future__ import annotations

import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import sim as S
from . import workload as W


@dataclass
class Request:
    rid: int
    arrival: float      # seconds after the start of the service
    n: int
    l_max: int
    n_steps: int
    t_e_ev: float
    n_e: float
    seed: int

    def workload(self) -> W.Workload:
        return W.Workload(f"req{self.rid}", n=self.n, seed=self.seed, l_max=self.l_max,
                          n_steps=self.n_steps, n_e=self.n_e, t_e_ev=self.t_e_ev)

    def member(self) -> S.Member:
        wl = self.workload()
        st = wl.particles()
        return S.Member(pos=st.pos, vel=st.vel, u_asy=wl.drive(self.n_steps), ntilde=wl.ntilde,
                        r_out=wl.r_out, dt=wl.dt)


def gpu_seconds_estimate(n: int, l_max: int, n_steps: int,
                         s_per_particle_step: float = 1.8e-10,
                         s_per_particle_step_per_channel: float = 1.3e-12) -> float:
    """Device time of a request at the measured cost of the step: a part per
    particle-step that does not depend on l_max (sort, push) plus a part
    proportional to (l_max + 1)^2 (moments, carries, field); the two
    constants fit the FP64 step times at 1.6e7 particles, l_max 8 and 32."""
    return n * n_steps * (s_per_particle_step + (l_max + 1) ** 2 * s_per_particle_step_per_channel)


def request_stream(seed: int = 5, duration_s: float = 60.0, load: float = 0.8,
                   n_range=(1e4, 4e6), l_choices=(8, 16, 32), steps_range=(2000, 20000)) -> list:
    """Poisson arrivals over duration_s.  N is log-uniform in n_range, l_max
    uniform over l_choices, steps uniform in steps_range, T_e ~ U(1, 5) eV,
    log10 n_e ~ U(14, 16).  The rate is set so that the offered device work
    is `load` times one GPU (Little's law with the mean work per request)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    # mean device seconds per request, by sampling the same distributions
    m = rng.uniform(np.log10(n_range[0]), np.log10(n_range[1]), 4096)
    ls = rng.choice(l_choices, 4096)
    ss = rng.integers(steps_range[0], steps_range[1] + 1, 4096)
    mean_work = float(np.mean([gpu_seconds_estimate(10 ** a, b, c) for a, b, c in zip(m, ls, ss)]))
    rate = load / mean_work
    out = []
    t = 0.0
    rid = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration_s:
            break
        n = int(round(10 ** rng.uniform(np.log10(n_range[0]), np.log10(n_range[1]))))
        out.append(Request(rid, t, n, int(rng.choice(l_choices)),
                           int(rng.integers(steps_range[0], steps_range[1] + 1)),
                           float(rng.uniform(1.0, 5.0)), float(10 ** rng.uniform(14.0, 16.0)),
                           5000 + rid))
        rid += 1
    return out


@dataclass
class Done:
    rid: int
    arrival: float
    admitted: float
    finished: float
    n: int
    l_max: int
    n_steps: int
    q_diff: np.ndarray = field(repr=False)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class Pool:
    """One resident batch: the requests it runs (member index -> [request,
    admission time, steps done]), whether a tick is in flight and how many
    steps it has."""
    key: tuple                      # (l_max, size class)
    batch: S.Batch
    running: dict = field(default_factory=dict)
    busy: bool = False
    tick: int = 0


class Server:
    """Pools per l_max class and, with small_max > 0, per size class: requests
    of at most small_max particles go to the class's small pool (small_share
    of its memory), larger ones to its large pool, so that a small request
    does not advance at the pace of a pool holding multi-million-particle
    runs.  budget_bytes of device memory is split over the l_max classes in
    proportion to their per-particle footprint (equal particle capacity per
    class).  Each pool steps on its own stream and is tended as soon as its
    tick completes, whatever the other pools are doing."""

    def __init__(self, budget_bytes: int, l_classes=(8, 16, 32), precision: int = S.SIM_FP64,
                 tick_steps: int = 50, max_members: int = 256, small_max: int = 0,
                 small_share: float = 0.25, max_steps: int = 20000, allocator="torch",
                 tick_seconds: float = 0.0):
        """tick_steps: steps per tick; with tick_seconds > 0 a pool's tick is
        instead as many steps as take about tick_seconds at the estimated cost
        of a step of its members (at most tick_steps), so that a pool of large
        requests does not hold the device queue it may share with a small
        pool for long."""
        self.tick = tick_steps
        self.tick_seconds = tick_seconds
        self.small_max = small_max
        self.pools = {}
        self.slots = {}   # particle slots of each pool
        # every member slot can hold a request of up to max_steps steps: the
        # members' drive and response arrays come from each pool's data pool
        mdata = max_members * S.member_data_bytes(max_steps)
        per_particle = {}
        for L in l_classes:
            cp = S.SimParams(l_max=L, precision=precision)
            probe = 1 << 20
            per_particle[L] = S.batch_footprint_bytes(cp, probe, max_members) / probe
        total = sum(per_particle.values())
        for L in l_classes:
            cp = S.SimParams(l_max=L, precision=precision)
            # equal particle capacity per class: bytes in proportion to footprint
            slots = int(budget_bytes / total) // S.SLOT_GROUP * S.SLOT_GROUP
            if small_max > 0:
                small = int(slots * small_share) // S.SLOT_GROUP * S.SLOT_GROUP
                shares = {0: small, 1: slots - small}
            else:
                shares = {0: slots}
            for cls, n in shares.items():
                self.slots[(L, cls)] = max(n, S.SLOT_GROUP)
                self.pools[(L, cls)] = Pool((L, cls), S.Batch(
                    cp, [], slot_capacity=max(n, S.SLOT_GROUP), max_members=max_members,
                    member_data=mdata, use_torch_stream=False, allocator=allocator))
        self.rejected = []   # requests larger than their pool

    def pool_key(self, req: Request) -> tuple:
        """The request's pool: its l_max class, and the small pool when it has
        at most small_max particles and fits that pool's slots (a request too
        big for the small pool goes to the large one)."""
        if (req.l_max, 0) not in self.pools:
            raise ValueError(f"no pool for l_max {req.l_max}")
        if self.small_max <= 0:
            return (req.l_max, 0)
        slots = -(-req.n // S.SLOT_GROUP) * S.SLOT_GROUP
        small = req.n <= self.small_max and slots <= self.slots[(req.l_max, 0)]
        return (req.l_max, 0 if small else 1)

    def close(self):
        for p in self.pools.values():
            p.batch.close()

    @staticmethod
    def _admit(pool: Pool, req, member, now) -> bool:
        try:
            idx = pool.batch.add(member)
        except S.SimError as e:
            if e.code == S.SIM_ENOMEM:
                return False
            raise
        pool.running[idx] = [req, now, 0]
        return True

    def tick_for(self, pool: Pool) -> int:
        """Steps of the pool's next tick."""
        if self.tick_seconds <= 0 or not pool.running:
            return self.tick
        L = pool.key[0]
        n = sum(rec[0].n for rec in pool.running.values())
        step_s = gpu_seconds_estimate(n, L, 1) + 1e-4   # plus ~10 launches
        return int(max(1, min(self.tick, round(self.tick_seconds / step_s))))

    def _retire(self, pool: Pool, now, done, log):
        """After a tick: the members whose step count reached their length
        (counted on the host, confirmed by the library) answer and leave."""
        for idx, rec in list(pool.running.items()):
            r, adm, steps = rec
            rec[2] = steps = min(steps + pool.tick, r.n_steps)
            if steps < r.n_steps:
                continue
            info = pool.batch.info(idx)
            if info["step"] < info["n_steps"]:
                raise RuntimeError(f"request {r.rid}: host and device step counts disagree")
            q = pool.batch.read_response(idx, 0, info["n_steps"])
            pool.batch.remove(idx)
            del pool.running[idx]
            done.append(Done(r.rid, r.arrival, adm, now, r.n, r.l_max, r.n_steps, q))
            if log:
                log(f"done {r.rid} L{r.l_max} n={r.n} steps={r.n_steps} "
                    f"latency {now - r.arrival:.2f} s")

    def run(self, requests, clock=time.perf_counter, log=None, workers: int = 4,
            poll_s: float = 2e-4) -> list:
        """Serve the requests (sorted by arrival) in real time; returns Done
        records in completion order."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        waiting = {k: deque() for k in self.pools}   # (request, future of its member)
        done = []
        pools = list(self.pools.values())
        with ThreadPoolExecutor(max_workers=workers) as ex:
            t0 = clock()
            while pending or any(waiting.values()) or any(p.running for p in pools):
                progressed = False
                now = clock() - t0
                while pending and pending[0].arrival <= now:
                    r = pending.popleft()
                    waiting[self.pool_key(r)].append((r, ex.submit(r.member)))
                    progressed = True
                for pool in pools:
                    if pool.busy:
                        if not pool.batch.query():
                            continue
                        pool.busy = False
                        self._retire(pool, clock() - t0, done, log)
                        progressed = True
                    # admissions, first come first served within the pool; a
                    # request that does not fit an empty pool never will
                    wq = waiting[pool.key]
                    while wq and wq[0][1].done():
                        r, fut = wq[0]
                        if not self._admit(pool, r, fut.result(), clock() - t0):
                            if pool.running:
                                break
                            self.rejected.append(r)
                        wq.popleft()
                        progressed = True
                    if pool.running:
                        pool.tick = self.tick_for(pool)
                        pool.batch.step(pool.tick)
                        pool.busy = True
                        progressed = True
                if not progressed:
                    idle = not any(p.busy for p in pools) and not any(waiting.values())
                    if idle and pending:
                        time.sleep(max(0.0, pending[0].arrival - (clock() - t0)))
                    else:
                        time.sleep(poll_s)
        return done


def latency_summary(done) -> dict:
    lat = np.array([d.latency for d in done])
    return {"requests": len(done), "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
            "max_s": float(lat.max())}
