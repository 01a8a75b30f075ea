"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and its host logic (defaults, validation, footprint, error strings)
behaves as documented.  No compute call is made here."""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2111_13072_amd import sim as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "mrpsim.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sim_[a-z_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert _declared_functions() == sorted(S.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = S.lib()
    for name in _declared_functions():
        assert hasattr(L, name), name


def test_params_layout_matches_header():
    p = S.sim_params()
    S.lib().sim_params_default(C.byref(p))
    assert p.struct_size == C.sizeof(S.sim_params) == 120
    assert (p.d, p.eps_r, p.r_out, p.dt, p.l_max) == (0.25, 4.0, 5.0, 0.05, 8)
    assert (p.sort_bucket, p.carry_chunk, p.sort_keys, p.near_split) == (0, 0, 0, 0)


def test_strerror_covers_codes():
    L = S.lib()
    for code in (0, -1, -2, -3, -4, -5, S.SIM_BUSY):
        assert L.sim_strerror(code).decode() not in ("", "unknown status")


def test_query_rejects_a_null_handle():
    assert S.lib().sim_query(None) == S.SIM_ESTATE


def test_footprint_grows_with_size_and_rejects_bad_params():
    a = S.footprint_bytes(S.SimParams(l_max=8), 10_000, 1000)
    b = S.footprint_bytes(S.SimParams(l_max=16), 10_000, 1000)
    c = S.footprint_bytes(S.SimParams(l_max=8), 20_000, 1000)
    assert 0 < a < b and a < c
    # finer sort buckets and shorter carry chunks take more histogram and carry memory
    d = S.footprint_bytes(S.SimParams(l_max=8, sort_bucket=1, carry_chunk=8), 10_000, 1000)
    e = S.footprint_bytes(S.SimParams(l_max=8, sort_bucket=64, carry_chunk=256), 10_000, 1000)
    assert d > a > e
    for bad in (dict(l_max=65), dict(l_max=-1), dict(d=0.0), dict(eps_r=0.0), dict(r_out=1.0),
                dict(m_mode=3), dict(wall_bc=0), dict(tile=48), dict(sort_bucket=-1),
                dict(sort_bucket=257), dict(carry_chunk=4), dict(carry_chunk=2048),
                dict(sort_keys=2), dict(sort_keys=-2), dict(near_split=2), dict(near_split=-2)):
        with pytest.raises(S.SimError) as ei:
            S.footprint_bytes(S.SimParams(**bad), 1000, 10)
        assert ei.value.code == S.SIM_EINVAL


@pytest.mark.parametrize("case", ["outside", "nan", "dup_ids", "start"])
def test_create_rejects_invalid_state_before_touching_the_device(case):
    pos = np.array([[2.0, 0, 0], [0, 3.0, 0]])
    vel = np.zeros((2, 3))
    ids = None
    u = np.zeros(4)
    start = 0
    if case == "outside":
        pos[1] = [0, 0, 0.5]
    elif case == "nan":
        vel[0, 1] = np.nan
    elif case == "dup_ids":
        ids = np.array([3, 3], dtype=np.uint32)
    elif case == "start":
        start = 5
    with pytest.raises(S.SimError) as ei:
        S.Sim(S.SimParams(), pos, vel, u, ids=ids, start_step=start, use_torch_stream=False)
    assert ei.value.code == S.SIM_EINVAL


def test_memory_limit_is_enforced_before_allocation():
    pos = np.array([[2.0, 0, 0], [0, 3.0, 0]])
    with pytest.raises(S.SimError) as ei:
        S.Sim(S.SimParams(mem_limit_bytes=1024), pos, np.zeros((2, 3)), np.zeros(4),
              use_torch_stream=False)
    assert ei.value.code == S.SIM_ENOMEM


def test_member_data_bytes_and_batch_footprint():
    """A member takes 16 B per step (drive and response, each 256-byte
    aligned) plus 16 B per ion-profile node of the batch's data pool, and the
    pool is part of the batch's one allocation."""
    assert S.member_data_bytes(1000) == 2 * 8192
    assert S.member_data_bytes(1000, 100) == 2 * 8192 + 1792
    assert S.member_data_bytes(0) == 2 * 256
    cp = S.SimParams(l_max=8)
    a = S.batch_footprint_bytes(cp, 1 << 14, 8)
    b = S.batch_footprint_bytes(cp, 1 << 14, 8, member_data=1 << 20)
    assert b - a == (1 << 20) - 256
    with pytest.raises(S.SimError):
        S.batch_footprint_bytes(cp, 1 << 14, 8, member_data=-1)


def test_caller_allocator_is_asked_once_for_the_footprint():
    """sim_create asks the caller's allocator for one block of exactly
    sim_footprint_bytes before any other device call; when it returns NULL
    the call fails with SIM_ENOMEM and nothing is freed."""
    calls = []

    def alloc(nbytes, stream):
        calls.append(("alloc", nbytes, stream))
        return 0

    def free(ptr, nbytes, stream):
        calls.append(("free", ptr, nbytes))

    pos = np.array([[2.0, 0, 0], [0, 3.0, 0]])
    prm = S.SimParams(l_max=4)
    with pytest.raises(S.SimError) as ei:
        S.Sim(prm, pos, np.zeros((2, 3)), np.zeros(7), use_torch_stream=False,
              allocator=S.Allocator(alloc, free))
    assert ei.value.code == S.SIM_ENOMEM
    assert calls == [("alloc", S.footprint_bytes(prm, 2, 7), 0)]
