"""Batches: many independent simulations in the same kernel launches.

Each member's fields, responses and states must equal, bit for bit, those of
the same member run alone (its arithmetic does not depend on the others); one
member is also checked against the oracle.  Members are admitted and retired
between steps.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle as O
from paper_2111_13072_amd import sim as S
from paper_2111_13072_amd import workload as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def make_member(n, gen_seed, n_steps, r_out=5.0, v_th=0.08311, **kw):
    st = W.uniform_shell(n, gen_seed, r_out, v_th)
    rng = np.random.default_rng(gen_seed + 1000)
    u = 0.05 * rng.standard_normal(n_steps)
    return S.Member(pos=st.pos, vel=st.vel, u_asy=u, ntilde=W.ntilde_for(n, r_out),
                    r_out=r_out, **kw)


def common(L=8, precision=S.SIM_FP64, m_mode=S.SIM_M_FULL, **kw):
    return S.SimParams(l_max=L, precision=precision, m_mode=m_mode, **kw)


def run_alone(cp, mb, steps):
    """The member alone: (responses, state, field after the steps)."""
    with S.Batch(cp, [mb]) as b:
        b.step(steps)
        st = b.info(0)["step"]
        q = b.read_response(0, mb.start_step, st - mb.start_step)
        return q, b.read_state(0), b.eval_field(0)


MIXED = [
    # n, seed, n_steps, extra
    (1000, 41, 12, {}),
    (64, 42, 12, {"r_out": 4.0, "dt": 0.04}),
    (777, 43, 7, {"probe_bc": S.SIM_BC_SPECULAR, "wall_bc": S.SIM_BC_DIFFUSE, "seed": 9}),
    (1, 44, 12, {}),
    (3000, 45, 10, {"ion_density": 0.5, "q_surface0": -3.0}),
    # mobile ions: the upper half of the ids carry the ion marker
    (900, 46, 9, {"ion_density": 0.0, "ion_mass": 100.0,
                  "ids": np.arange(900, dtype=np.uint32) | np.where(np.arange(900) % 2 == 1,
                                                                     np.uint32(0x80000000),
                                                                     np.uint32(0))}),
]


@pytest.mark.parametrize("precision", [S.SIM_FP64, S.SIM_FP32_COMP], ids=["fp64", "fp32c"])
def test_members_equal_runs_alone(precision):
    cp = common(L=8, precision=precision)
    members = [make_member(n, seed, ns, **kw) for n, seed, ns, kw in MIXED]
    _say(f"[gpu] batch of {len(members)} members, precision {precision}")
    with S.Batch(cp, members) as b:
        E0 = [b.eval_field(i) for i in range(len(members))]
        b.step(12)                                  # members with 7 or 10 steps stop there
        outs = []
        for i, mb in enumerate(members):
            info = b.info(i)
            assert info["step"] == mb.u_asy.shape[0]
            outs.append((b.read_response(i, 0, info["step"]), b.read_state(i), b.eval_field(i)))
    for i, mb in enumerate(members):
        _say(f"[gpu]   member {i} alone: n={mb.pos.shape[0]}")
        with S.Batch(cp, [mb]) as a:
            assert np.array_equal(a.eval_field(0), E0[i])
        q, st, E = run_alone(cp, mb, 12)
        bq, bst, bE = outs[i]
        assert np.array_equal(q, bq)
        for k in ("pos", "vel", "alive"):
            assert np.array_equal(st[k], bst[k]), k
        assert st["q_surface"] == bst["q_surface"] and st["step"] == bst["step"]
        assert np.array_equal(E, bE)


def test_field_evaluations_mid_run_change_no_member():
    """Field evaluations between batch steps, some while members are still
    running and some after a member has finished, leave every member's run
    bit for bit equal to the member run alone."""
    cp = common(L=6, sort_keys=1)
    picks = [MIXED[0], MIXED[2], MIXED[4]]            # 12, 7 and 10 steps
    members = [make_member(n, seed, ns, **kw) for n, seed, ns, kw in picks]
    _say(f"[gpu] batch field evaluations mid-run, {len(members)} members")
    with S.Batch(cp, members) as b:
        b.step(5)
        E_mid = b.eval_field(0)
        b.step(3)                                     # the 7-step member finishes here
        b.eval_field(1)
        b.eval_field(2)
        b.step(4)
        outs = [(b.read_response(i, 0, b.info(i)["step"]), b.read_state(i))
                for i in range(len(members))]
    with S.Batch(cp, [members[0]]) as a:
        a.step(5)
        assert np.array_equal(a.eval_field(0), E_mid)
    for i, mb in enumerate(members):
        q, st, _ = run_alone(cp, mb, 12)
        bq, bst = outs[i]
        assert np.array_equal(q, bq), i
        for k in ("pos", "vel", "alive"):
            assert np.array_equal(st[k], bst[k]), (i, k)


def test_batch_member_matches_oracle():
    cp = common(L=6)
    members = [make_member(900, 51, 4), make_member(500, 52, 4, r_out=3.0)]
    with S.Batch(cp, members) as b:
        for i, mb in enumerate(members):
            _say(f"[gpu] batch member {i} vs oracle: n={mb.pos.shape[0]}")
            E = b.eval_field(i)
            op = O.Params(d=cp.d, eps_r=cp.eps_r, r_out=mb.r_out, dt=mb.dt, ntilde=mb.ntilde,
                          ion_density=mb.ion_density, l_max=cp.l_max)
            Eo, _ = O.field(op, mb.pos, u_asy=mb.u_asy[0])
            rms = np.sqrt(np.mean(np.sum(Eo * Eo, axis=1)))
            assert np.max(np.abs(E - Eo)) / rms < 1e-12


def test_admit_and_retire_between_steps():
    # sort keys from the push, so that a member retired while running leaves
    # counts in its buckets for the next member to find cleared
    cp = common(L=4, sort_keys=1)
    a = make_member(700, 61, 20)
    bm = make_member(300, 62, 8)
    c = make_member(650, 63, 5)
    _say("[gpu] pool: admit/retire")
    with S.Batch(cp, [], slot_capacity=1600, max_members=3,
                 member_data=3 * S.member_data_bytes(20)) as pool:
        ia = pool.add(a)
        pool.step(5)
        ib = pool.add(bm)
        pool.step(5)
        qa_mid = pool.read_response(ia, 0, 10)
        pool.remove(ia)                              # frees 768 slots (3 groups)
        ic = pool.add(c)                             # reuses them
        pool.step(10)
        qb = pool.read_response(ib, 0, 8)
        qc = pool.read_response(ic, 0, 5)
        stc = pool.read_state(ic)
    qa, _, _ = run_alone(cp, a, 10)
    assert np.array_equal(qa[:10], qa_mid)
    q, _, _ = run_alone(cp, bm, 8)
    assert np.array_equal(q, qb)
    q, st, _ = run_alone(cp, c, 5)
    assert np.array_equal(q, qc)
    assert np.array_equal(st["pos"], stc["pos"])


def test_admission_limits_leave_the_pool_working():
    cp = common(L=3)
    a = make_member(500, 71, 6)
    with S.Batch(cp, [a], slot_capacity=600, max_members=2,
                 member_data=2 * S.member_data_bytes(6)) as pool:
        with pytest.raises(S.SimError) as ei:
            pool.add(make_member(300, 72, 6))      # 512 + 512 slots > 768
        assert ei.value.code == S.SIM_ENOMEM
        with pytest.raises(S.SimError) as ei:
            pool.add(make_member(50, 74, 40))      # its drive does not fit the data pool
        assert ei.value.code == S.SIM_ENOMEM
        with pytest.raises(S.SimError) as ei:
            pool.add(make_member(10, 73, 6, r_out=0.5))
        assert ei.value.code == S.SIM_EINVAL
        with pytest.raises(S.SimError) as ei:
            pool.remove(1)
        assert ei.value.code == S.SIM_ERANGE
        pool.step(6)
        q = pool.read_response(0, 0, 6)
    qa, _, _ = run_alone(cp, a, 6)
    assert np.array_equal(q, qa)


def test_strict_step_and_lenient_batch_step():
    cp = common(L=2)
    with S.Batch(cp, [make_member(100, 81, 3), make_member(100, 82, 5)]) as b:
        with pytest.raises(S.SimError) as ei:
            b.step_strict(4)
        assert ei.value.code == S.SIM_ERANGE
        b.step(100)
        assert b.info(0)["step"] == 3 and b.info(1)["step"] == 5
        assert b.read_state(0)["step"] == 3 and b.read_state(1)["step"] == 5


def test_query_reports_completion():
    """sim_query answers without waiting: busy or done, and done after a sync."""
    import time

    _say("[gpu] sim_query on a stepping handle")
    mb = make_member(30000, 7, 60)
    with S.Batch(common(L=8), [mb], use_torch_stream=False) as b:
        b.sync()
        assert b.query()                  # nothing enqueued
        b.step(40)
        seen_done = False
        t_end = time.perf_counter() + 60.0
        while time.perf_counter() < t_end:
            if b.query():
                seen_done = True
                break
            time.sleep(1e-3)
        assert seen_done
        b.sync()
        assert b.query()
        assert b.info(0)["step"] == 40


def test_torch_allocated_run_equals_hipmalloc_run():
    """Device memory from torch's caching allocator (one block of the
    footprint, visible in torch's accounting while the handle lives) or from
    hipMalloc inside the library: the same run bit for bit, on torch's stream
    and on a stream of the handle's own."""
    import torch

    n, L, steps = 3000, 6, 6
    _say(f"[gpu] allocator: torch vs hipMalloc n={n} L={L} steps={steps}")
    st = W.uniform_shell(n, 91, 5.0, 0.3)
    sp = S.SimParams(ntilde=W.ntilde_for(n, 5.0), l_max=L, q_surface0=-3.0)
    u = W.gaussian_drive(steps, sp.dt, 20.0, 289.52, t_center=0.1)
    outs = []
    for alloc, own in (("hip", False), ("torch", False), ("torch", True)):
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        with S.Sim(sp, st.pos, st.vel, u, allocator=alloc, use_torch_stream=not own) as sim:
            held = torch.cuda.memory_allocated() - before
            if alloc == "torch":
                assert held >= S.footprint_bytes(sp, n, steps)
            else:
                assert held == 0
            sim.step(steps)
            outs.append((sim.read_state(), sim.read_response(0, steps), sim.eval_field()))
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
    (a, qa, Ea) = outs[0]
    for (b, qb, Eb) in outs[1:]:
        for key in ("pos", "vel", "alive"):
            np.testing.assert_array_equal(a[key], b[key])
        np.testing.assert_array_equal(qa, qb)
        np.testing.assert_array_equal(Ea, Eb)
