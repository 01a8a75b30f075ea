"""Continuous batching: requests arriving over time, admitted into resident
pools between steps, each answered exactly as if it had run alone, and as the
CPU oracle answers it."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle as O
from paper_2111_13072_amd import serve as SV
from paper_2111_13072_amd import sim as S

pytestmark = pytest.mark.gpu

_ORACLE = {}


def oracle_response(r: SV.Request) -> np.ndarray:
    """Q_diff of the request's simulation from the CPU oracle (same seeded
    member: particles, drive, ntilde, walls), cached across the tests."""
    if r.rid not in _ORACLE:
        wl = r.workload()
        st = wl.particles()
        op = O.Params(d=wl.d, eps_r=wl.eps_r, r_out=wl.r_out, dt=wl.dt, ntilde=wl.ntilde,
                      ion_density=1.0, l_max=r.l_max)
        _ORACLE[r.rid] = O.run(op, st.pos, st.vel, wl.drive(r.n_steps), r.n_steps).qdiff
    return _ORACLE[r.rid]


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def small_requests():
    rng = np.random.default_rng(17)
    reqs = []
    t = 0.0
    for rid in range(10):
        t += float(rng.exponential(0.05))
        reqs.append(SV.Request(rid, t, int(rng.integers(300, 3000)), int(rng.choice([4, 6])),
                               int(rng.integers(20, 80)), float(rng.uniform(1, 5)),
                               float(10 ** rng.uniform(14, 16)), 900 + rid))
    return reqs


@pytest.mark.parametrize("small_max", [0, 1500])
def test_served_results_equal_runs_alone(small_max):
    reqs = small_requests()
    # room for about two requests per class at a time: admission has to wait;
    # with small_max, requests of up to 1500 particles have pools of their own
    cp = S.SimParams(l_max=6)
    per = S.batch_footprint_bytes(cp, 1 << 16, 16) / (1 << 16)
    srv = SV.Server(int(2 * 6000 * per), l_classes=(4, 6), tick_steps=8, max_members=16,
                    small_max=small_max)
    assert len(srv.pools) == (4 if small_max else 2)
    _say(f"[gpu] serving {len(reqs)} requests, small_max {small_max}")
    try:
        done = srv.run(reqs)
    finally:
        srv.close()
    assert not srv.rejected
    assert sorted(d.rid for d in done) == list(range(len(reqs)))
    waited = [d for d in done if d.admitted > d.arrival + 1e-3]
    _say(f"[gpu] {len(waited)} requests waited for admission")
    worst = 0.0
    for d in done:
        r = reqs[d.rid]
        assert d.q_diff.shape == (r.n_steps,)
        assert d.finished >= d.admitted >= d.arrival - 1e-9
        with S.Batch(S.SimParams(l_max=r.l_max), [r.member()]) as b:
            b.step(r.n_steps)
            q = b.read_response(0, 0, r.n_steps)
        assert np.array_equal(q, d.q_diff), d.rid
        # and the served response is the method's: the oracle's run of the
        # same request, relative to the response's scale
        qo = oracle_response(r)
        dev = float(np.max(np.abs(d.q_diff - qo)) / np.max(np.abs(qo)))
        worst = max(worst, dev)
        assert dev <= 1e-12, (d.rid, dev)
    _say(f"[gpu] served responses vs oracle: worst relative deviation {worst:.2e}")
    s = SV.latency_summary(done)
    assert s["requests"] == len(reqs) and 0 < s["p50_s"] <= s["p99_s"] <= s["max_s"]


def test_oversized_request_is_rejected_not_stuck():
    srv = SV.Server(1, l_classes=(4,), tick_steps=4, max_members=4)   # one tile of capacity
    reqs = [SV.Request(0, 0.0, 5000, 4, 10, 2.0, 1e15, 1),
            SV.Request(1, 0.0, 50, 4, 10, 2.0, 1e15, 2)]
    try:
        done = srv.run(reqs)
    finally:
        srv.close()
    assert [r.rid for r in srv.rejected] == [0]
    assert [d.rid for d in done] == [1]
