"""Host logic of the server: which pool a request goes to (no device)."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_2111_13072_amd import serve as SV  # noqa: E402


def _shell(small_max, small_slots=1536, large_slots=4608, classes=(4, 8)):
    """A server's routing state without its device pools."""
    srv = SV.Server.__new__(SV.Server)
    srv.small_max = small_max
    srv.pools = {}
    srv.slots = {}
    for L in classes:
        for cls, n in ((0, small_slots), (1, large_slots)) if small_max > 0 else ((0, large_slots),):
            srv.pools[(L, cls)] = None
            srv.slots[(L, cls)] = n
    return srv


def _req(n, L=4):
    return SV.Request(0, 0.0, n, L, 10, 2.0, 1e15, 1)


def test_small_requests_go_to_the_small_pool_when_they_fit():
    srv = _shell(1600)
    assert srv.pool_key(_req(300)) == (4, 0)
    assert srv.pool_key(_req(1536)) == (4, 0)       # 6 whole groups of 256: fits 1536 slots
    assert srv.pool_key(_req(1537)) == (4, 1)       # 7 groups: too big for the small pool
    assert srv.pool_key(_req(1601)) == (4, 1)       # above small_max
    assert srv.pool_key(_req(300, L=8)) == (8, 0)


def test_one_pool_per_class_without_a_split():
    srv = _shell(0)
    assert srv.pool_key(_req(10)) == (4, 0)
    assert srv.pool_key(_req(10 ** 6)) == (4, 0)


def test_unknown_l_max_is_refused():
    with pytest.raises(ValueError):
        _shell(1500).pool_key(_req(100, L=6))


def test_time_bounded_ticks_shrink_for_large_pools():
    """With tick_seconds, a pool of large requests ticks in fewer steps than a
    pool of small ones (each tick ~tick_seconds at the estimated step cost),
    within [1, tick_steps]."""
    srv = _shell(0)
    srv.tick, srv.tick_seconds = 500, 0.025
    small = SV.Pool((8, 0), None, running={0: [_req(20_000, L=8), 0.0, 0]})
    large = SV.Pool((8, 0), None, running={0: [_req(4_000_000, L=8), 0.0, 0]})
    assert 100 < srv.tick_for(small) <= 500
    assert 1 <= srv.tick_for(large) < 100
    srv.tick_seconds = 0.0
    assert srv.tick_for(large) == 500
