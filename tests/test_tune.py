"""The launch-size autotuner (sort bucket, carry chunk, near-field
block): its search and cache on the CPU with a synthetic timing model; on the
GPU, that tuned sizes give the field of the default sizes."""
import json

import numpy as np
import pytest

from paper_2111_13072_amd import sim as S
from paper_2111_13072_amd import tune as T


class _Fake:
    """A build function whose 'timing' is a known function of the sizes."""

    def __init__(self, cost):
        self.cost = cost
        self.built = []

    def __call__(self, p):
        self.built.append((p.sort_bucket, p.carry_chunk, p.near_split))
        h = T.RunnerHandle(lambda k: None, lambda: None)
        h.cost = self.cost(p.sort_bucket, p.carry_chunk) + (0.25 if p.near_split < 0 else 0.0)
        return h


def _measure(h, steps, warmup, reps):
    return h.cost


def test_coordinate_search_finds_the_minimum_along_its_path():
    # separable cost: best bucket 16, best chunk 32
    cost = lambda b, c: abs(np.log2(b) - 4) + (0.5 if c == 0 else abs(np.log2(c) - 5))
    f = _Fake(cost)
    t = T.autotune(f, S.SimParams(l_max=8), 100_000, measure=_measure)
    assert (t.sort_bucket, t.carry_chunk) == (16, 32)
    assert t.ms_per_step == cost(16, 32) and t.default_ms_per_step == cost(8, 0)
    # every candidate built at most once, each one closed; the near-field
    # block is a third coordinate (whole tiles cost more here)
    assert len(f.built) == len(set(f.built)) == len(T.BUCKETS) + len(T.CHUNKS) - 1 + 1
    assert t.near_split == 0
    assert t.apply(S.SimParams(l_max=8)).sort_bucket == 16


def test_near_field_block_is_searched_never_forcing_half_tiles():
    f = _Fake(lambda b, c: 1.0)
    t = T.autotune(f, S.SimParams(precision=S.SIM_FP32_COMP), 1000, measure=_measure)
    assert all(s in (0, -1) for _, _, s in f.built) and t.near_split == 0
    g = _Fake(lambda b, c: 1.0)

    def cheaper_whole_tiles(p):
        h = g(p)
        h.cost = 0.5 if p.near_split < 0 else 1.0
        return h

    t = T.autotune(cheaper_whole_tiles, S.SimParams(), 1000, measure=_measure)
    assert t.near_split == -1 and t.apply(S.SimParams()).near_split == -1


def test_ties_keep_the_smaller_size_and_default_is_a_candidate():
    f = _Fake(lambda b, c: 1.0)
    t = T.autotune(f, S.SimParams(), 1000, measure=_measure)
    assert (t.sort_bucket, t.carry_chunk) == (min(T.BUCKETS), 0)
    assert 8 in T.BUCKETS and 0 in T.CHUNKS


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    f = _Fake(lambda b, c: b + (c or 100))
    c1 = T.Cache(path)
    t1 = T.autotune(f, S.SimParams(l_max=16), 2_000_000, measure=_measure, cache=c1)
    n_built = len(f.built)
    # a second search of the same shape class is served from the file
    c2 = T.Cache(path)
    t2 = T.autotune(f, S.SimParams(l_max=16), 2_100_000, measure=_measure, cache=c2)
    assert len(f.built) == n_built
    assert (t2.sort_bucket, t2.carry_chunk, t2.ms_per_step) == (t1.sort_bucket, t1.carry_chunk,
                                                                t1.ms_per_step)
    assert json.load(open(path))[T.shape_key(S.SimParams(l_max=16), 2_000_000)]
    # a different l_max is a different shape class
    T.autotune(f, S.SimParams(l_max=8), 2_000_000, measure=_measure, cache=c2)
    assert len(f.built) > n_built


def test_candidates_are_valid_parameters():
    for b in T.BUCKETS:
        for c in T.CHUNKS:
            assert S.footprint_bytes(S.SimParams(sort_bucket=b, carry_chunk=c), 50_000, 10) > 0


@pytest.mark.gpu
def test_tuned_sizes_keep_the_field():
    """Autotune a 3e4-particle, l_max 8 workload; the field with the chosen
    sizes equals the field with the built-in ones to the rounding order of the
    carries, and every candidate's field does."""
    from paper_2111_13072_amd import workload as W
    import sys

    n = 30_000
    st = W.uniform_shell(n, 5, 5.0, 0.0831)
    prm = S.SimParams(ntilde=W.ntilde_for(n, 5.0), l_max=8)
    print(f"[gpu] autotune n={n} L=8", file=sys.stderr, flush=True)
    t = T.autotune(T.sim_builder(st.pos, st.vel), prm, n, steps=3, warmup=1, reps=1)
    assert t.sort_bucket in T.BUCKETS and t.carry_chunk in T.CHUNKS
    assert len(t.trials) == len(T.BUCKETS) + len(T.CHUNKS) - 1 + 1
    u = np.zeros(4)
    with S.Sim(prm, st.pos, st.vel, u) as s:
        E0 = s.eval_field()
    rms = np.sqrt(np.mean(np.sum(E0 * E0, axis=1)))
    for b, c, sp in ((t.sort_bucket, t.carry_chunk, t.near_split), (4, 8, 0), (64, 128, -1)):
        with S.Sim(S.SimParams(ntilde=prm.ntilde, l_max=8, sort_bucket=b, carry_chunk=c,
                               near_split=sp), st.pos, st.vel, u) as s:
            E = s.eval_field()
        assert np.max(np.abs(E - E0)) <= 1e-13 * rms, (b, c, sp)
