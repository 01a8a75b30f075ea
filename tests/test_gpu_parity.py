"""GPU (HIP) against the CPU oracle on identical seeded inputs.

Field metric: max_k |E_gpu - E_oracle| / RMS_k |E_oracle|; bar 1e-12 in FP64,
1e-5 in the FP32-compensated mode at every l_max.
Every case prints its name, size and seed before touching the GPU.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle as O
from paper_2111_13072_amd import sim as S
from paper_2111_13072_amd import workload as W

pytestmark = pytest.mark.gpu

FP64_FIELD_TOL = 1e-12


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _rel_err(E, Eo, mask=None):
    if mask is not None:
        E, Eo = E[mask], Eo[mask]
    rms = np.sqrt(np.mean(np.sum(Eo * Eo, axis=1)))
    return float(np.max(np.abs(E - Eo)) / rms)


def _params(n, L, mode=S.SIM_M_FULL, r_out=5.0, **kw):
    nt = W.ntilde_for(n, r_out)
    sp = S.SimParams(ntilde=nt, l_max=L, m_mode=mode, r_out=r_out, **kw)
    op = O.Params(d=sp.d, eps_r=sp.eps_r, r_out=r_out, dt=sp.dt, ntilde=nt,
                  ion_density=sp.ion_density, l_max=L, m_mode=mode, probe_bc=sp.probe_bc,
                  wall_bc=sp.wall_bc, seed=sp.seed)
    return sp, op


FIELD_CASES = [
    # name, n, l_max, m_mode, seed
    ("shell-3000-L8", 3000, 8, S.SIM_M_FULL, 21),
    ("ragged-777-L5", 777, 5, S.SIM_M_FULL, 22),
    ("monopole-500-L0", 500, 0, S.SIM_M_FULL, 23),
    ("dipole-axisym-1000-L1", 1000, 1, S.SIM_M_AXISYM, 24),
    ("axisym-640-L6", 640, 6, S.SIM_M_AXISYM, 25),
    ("shell-2000-L16", 2000, 16, S.SIM_M_FULL, 26),
    ("single-particle-L4", 1, 4, S.SIM_M_FULL, 27),
    ("one-tile-64-L3", 64, 3, S.SIM_M_FULL, 28),
    ("two-tiles-65-L3", 65, 3, S.SIM_M_FULL, 29),
    ("shell-1000-L32", 1000, 32, S.SIM_M_FULL, 30),
    # the largest l_max: the tile coefficients pass through LDS in nine windows
    ("shell-700-L64", 700, 64, S.SIM_M_FULL, 31),
]


@pytest.mark.parametrize("name,n,L,mode,seed", FIELD_CASES, ids=[c[0] for c in FIELD_CASES])
def test_field_matches_oracle(name, n, L, mode, seed):
    _say(f"[gpu] field parity {name}: n={n} L={L} mode={mode} seed={seed}")
    sp, op = _params(n, L, mode, q_surface0=-7.0)
    st = W.uniform_shell(n, seed, 5.0, 0.0831)
    u = np.array([0.0, 0.0, 0.3, 0.0])
    with S.Sim(sp, st.pos, st.vel, u, start_step=2) as sim:
        E = sim.eval_field()
    Eo, _ = O.field(op, st.pos, q_surface=-7.0, u_asy=0.3)
    err = _rel_err(E, Eo)
    _say(f"[gpu]   rel err {err:.3e}")
    assert err <= FP64_FIELD_TOL


WHOLE_TILE_CASES = [c for c in FIELD_CASES if c[0] in
                    ("shell-3000-L8", "ragged-777-L5", "axisym-640-L6", "shell-2000-L16",
                     "two-tiles-65-L3", "shell-700-L64")]


@pytest.mark.parametrize("name,n,L,mode,seed", WHOLE_TILE_CASES,
                         ids=[c[0] for c in WHOLE_TILE_CASES])
def test_field_matches_oracle_with_whole_tile_near_field(name, n, L, mode, seed):
    """The near field's pair sums over whole tiles of 64 (the FP64 default
    is half tiles of 32): the same sum split differently, the same bar."""
    _say(f"[gpu] field parity, near field per tile, {name}: n={n} L={L} mode={mode} seed={seed}")
    sp, op = _params(n, L, mode, q_surface0=-7.0, near_split=-1)
    st = W.uniform_shell(n, seed, 5.0, 0.0831)
    u = np.array([0.0, 0.0, 0.3, 0.0])
    with S.Sim(sp, st.pos, st.vel, u, start_step=2) as sim:
        E = sim.eval_field()
    Eo, _ = O.field(op, st.pos, q_surface=-7.0, u_asy=0.3)
    err = _rel_err(E, Eo)
    _say(f"[gpu]   rel err {err:.3e}")
    assert err <= FP64_FIELD_TOL


def test_field_radius_tie_broken_by_id():
    """Two particles at exactly equal r^2 (coordinates swapped): the order,
    and so the gradient branch of r_< / r_>, follows the id."""
    _say("[gpu] field parity with an exact radius tie")
    st = W.uniform_shell(300, 31, 5.0, 0.08)
    pos = st.pos.copy()
    pos[7] = [pos[3, 1], pos[3, 0], pos[3, 2]]
    assert np.dot(pos[7], pos[7]) == np.dot(pos[3], pos[3])
    ids = np.arange(300, dtype=np.uint32)[::-1].copy()
    sp, op = _params(300, 6)
    with S.Sim(sp, pos, st.vel, np.zeros(2), ids=ids) as sim:
        E = sim.eval_field()
    Eo, _ = O.field(op, pos, ids=ids)
    assert _rel_err(E, Eo) <= FP64_FIELD_TOL


@pytest.mark.parametrize("sort_keys", [1, -1], ids=["keys-in-push", "key-pass"])
def test_steps_match_oracle_with_absorption(sort_keys):
    """Five steps with a strong drive: Q_diff, positions, velocities,
    absorbed set and Q_S against the oracle's leapfrog, with the sort keys
    taken in the push or in a pass of their own."""
    n, L, steps = 2000, 8, 5
    _say(f"[gpu] stepping parity n={n} L={L} steps={steps} sort_keys={sort_keys}")
    sp, op = _params(n, L, q_surface0=-2.0, sort_keys=sort_keys)
    st = W.uniform_shell(n, 41, 5.0, 0.3)  # hot, so some reach the probe
    u = W.gaussian_drive(steps, sp.dt, 50.0, 289.52, t_center=0.1)
    with S.Sim(sp, st.pos, st.vel, u) as sim:
        sim.step(steps)
        qd = sim.read_response(0, steps)
        out = sim.read_state()
    ref = O.run(op, st.pos, st.vel, u, steps, q_surface=-2.0)
    _say(f"[gpu]   absorbed gpu={int((out['alive'] == 0).sum())} oracle={ref.absorbed}")
    np.testing.assert_array_equal(out["alive"], ref.alive)
    assert out["q_surface"] == ref.q_surface
    assert out["step"] == steps
    scale = np.max(np.abs(ref.qdiff))
    assert np.max(np.abs(qd - ref.qdiff)) <= 1e-12 * scale
    assert np.max(np.abs(out["pos"] - ref.pos)) <= 1e-12
    assert np.max(np.abs(out["vel"] - ref.vel)) <= 1e-12


@pytest.mark.parametrize("precision", [S.SIM_FP64, S.SIM_FP32_COMP], ids=["fp64", "fp32c"])
def test_sort_key_paths_agree_bitwise(precision):
    """Sort keys taken in the push and in a pass of their own give the same
    run bit for bit (absorbing probe, diffuse outer wall, fast particles)."""
    n, L, steps = 2500, 6, 6
    _say(f"[gpu] sort-key paths n={n} L={L} steps={steps} precision={precision}")
    st = W.uniform_shell(n, 57, 2.5, 0.6)
    u = W.gaussian_drive(steps, 0.05, 30.0, 289.52, t_center=0.1)
    outs = []
    for keys in (1, -1):
        sp, _ = _params(n, L, sort_keys=keys, precision=precision, wall_bc=S.SIM_BC_DIFFUSE,
                        seed=77)
        with S.Sim(sp, st.pos, st.vel, u) as sim:
            sim.step(steps)
            outs.append((sim.read_state(), sim.read_response(0, steps), sim.eval_field()))
    (a, qa, Ea), (b, qb, Eb) = outs
    assert (a["alive"] == 0).any()
    for key in ("pos", "vel", "alive"):
        np.testing.assert_array_equal(a[key], b[key])
    assert a["q_surface"] == b["q_surface"]
    np.testing.assert_array_equal(qa, qb)
    np.testing.assert_array_equal(Ea, Eb)


def test_concentrated_shell_ranks_past_the_lds_window():
    """2000 of 3000 particles inside one sort bucket's shell (r in [2, 2.004];
    the 375 buckets are 0.028 wide there): 250 times the mean occupancy, more
    records than the rank kernel stages in LDS, so it ranks them from global
    memory.  The field and three steps still match the oracle."""
    n, L, steps, k = 3000, 6, 3, 2000
    _say(f"[gpu] concentrated shell n={n} (k={k} in one bucket) L={L} steps={steps}")
    sp, op = _params(n, L)
    st = W.uniform_shell(n, 61, 5.0, 0.05)
    g = np.random.Generator(np.random.PCG64(62))
    pos = st.pos.copy()
    r = 2.0 + 0.004 * g.random(k)
    pos[:k] *= (r / np.sqrt(np.sum(pos[:k] ** 2, axis=1)))[:, None]
    u = W.gaussian_drive(steps, sp.dt, 20.0, 289.52, t_center=0.1)
    with S.Sim(sp, pos, st.vel, u) as sim:
        E = sim.eval_field()
        sim.step(steps)
        qd = sim.read_response(0, steps)
        out = sim.read_state()
    Eo, _ = O.field(op, pos, u_asy=u[0])
    assert _rel_err(E, Eo) <= FP64_FIELD_TOL
    ref = O.run(op, pos, st.vel, u, steps)
    np.testing.assert_array_equal(out["alive"], ref.alive)
    scale = np.max(np.abs(ref.qdiff))
    assert np.max(np.abs(qd - ref.qdiff)) <= 1e-12 * scale
    assert np.max(np.abs(out["pos"] - ref.pos)) <= 1e-12
    assert np.max(np.abs(out["vel"] - ref.vel)) <= 1e-12


@pytest.mark.parametrize("probe_bc,wall_bc", [(S.SIM_BC_SPECULAR, S.SIM_BC_SPECULAR),
                                              (S.SIM_BC_DIFFUSE, S.SIM_BC_DIFFUSE)])
def test_reflecting_walls_match_oracle(probe_bc, wall_bc):
    n, L, steps = 1500, 4, 6
    _say(f"[gpu] wall parity probe_bc={probe_bc} wall_bc={wall_bc} n={n}")
    sp, op = _params(n, L, probe_bc=probe_bc, wall_bc=wall_bc, seed=12345)
    st = W.uniform_shell(n, 43, 5.0, 0.5)
    u = np.zeros(steps)
    with S.Sim(sp, st.pos, st.vel, u) as sim:
        sim.step(steps)
        out = sim.read_state()
    ref = O.run(op, st.pos, st.vel, u, steps)
    assert np.all(out["alive"] == 1) and np.all(ref.alive == 1)
    assert np.max(np.abs(out["pos"] - ref.pos)) <= 1e-11
    assert np.max(np.abs(out["vel"] - ref.vel)) <= 1e-11


def test_trajectory_small_workload():
    """The 1e4-particle, l_max = 8 workload: 10 steps of the Gaussian pulse
    against the oracle."""
    wl = W.SMALL_FP64
    steps = 10
    _say(f"[gpu] trajectory {wl.name} steps={steps}")
    st = wl.particles()
    u = wl.drive()
    sp, op = _params(wl.n, wl.l_max)
    with S.Sim(sp, st.pos, st.vel, u) as sim:
        sim.step(steps)
        qd = sim.read_response(0, steps)
        out = sim.read_state()
    ref = O.run(op, st.pos, st.vel, u, steps)
    np.testing.assert_array_equal(out["alive"], ref.alive)
    assert np.max(np.abs(qd - ref.qdiff)) <= 1e-10
    assert np.max(np.abs(out["pos"] - ref.pos)) <= 1e-11


def test_large_workload_sampled_field():
    """2e6 particles, l_max = 16 (the benchmark shape): the full GPU field
    against the oracle's pair sums at 48 sampled particles."""
    wl = W.LARGE
    _say(f"[gpu] sampled field parity {wl.name}")
    st = wl.particles()
    sp, op = _params(wl.n, wl.l_max, q_surface0=-40.0)
    u = wl.drive(30)
    with S.Sim(sp, st.pos, st.vel, u, start_step=20) as sim:
        E = sim.eval_field()
    rng = np.random.default_rng(5)
    targets = np.sort(rng.choice(wl.n, 48, replace=False))
    Eo, _ = O.field(op, st.pos, q_surface=-40.0, u_asy=u[20], targets=targets)
    rms = np.sqrt(np.mean(np.sum(Eo * Eo, axis=1)))
    err = float(np.max(np.abs(E[targets] - Eo)) / rms)
    _say(f"[gpu]   rel err {err:.3e}")
    assert err <= FP64_FIELD_TOL


def test_large_workload_steps_with_keys_from_the_push():
    """2e6 particles, l_max = 16, in the benchmark's launch configuration
    (sort keys taken in the push at this size): ten steps equal bit for bit
    the same steps with the keys taken in a pass of their own, and the field
    of the stepped state matches the oracle at 48 sampled alive particles."""
    wl = W.LARGE
    steps = 10
    _say(f"[gpu] stepped {wl.name}, {steps} steps, push-keyed vs key pass")
    st = wl.particles()
    u = wl.drive(steps + 1)
    outs = []
    for keys in (0, -1):
        sp, op = _params(wl.n, wl.l_max, sort_keys=keys)
        with S.Sim(sp, st.pos, st.vel, u) as sim:
            sim.step(steps)
            outs.append((sim.read_state(), sim.read_response(0, steps),
                         sim.eval_field() if keys == 0 else None))
    (a, qa, E), (b, qb, _) = outs
    for key in ("pos", "vel", "alive"):
        np.testing.assert_array_equal(a[key], b[key])
    assert a["q_surface"] == b["q_surface"]
    np.testing.assert_array_equal(qa, qb)
    alive = a["alive"] == 1
    rng = np.random.default_rng(6)
    targets = np.sort(rng.choice(np.nonzero(alive)[0], 48, replace=False))
    Eo, _ = O.field(op, a["pos"], alive=alive, q_surface=a["q_surface"], u_asy=u[steps],
                    targets=targets)
    rms = np.sqrt(np.mean(np.sum(Eo * Eo, axis=1)))
    err = float(np.max(np.abs(E[targets] - Eo)) / rms)
    _say(f"[gpu]   rel err {err:.3e}, absorbed {int((~alive).sum())}")
    assert err <= FP64_FIELD_TOL


@pytest.mark.parametrize("sort_keys", [1, -1], ids=["keys-in-push", "key-pass"])
def test_deterministic_and_resumable(sort_keys):
    """Same inputs give bitwise-equal states; k + k steps with a dump and a
    re-creation in between equal 2k uninterrupted steps bitwise."""
    n, L, k = 3000, 6, 4
    _say(f"[gpu] determinism/resume n={n} L={L} k={k} sort_keys={sort_keys}")
    sp, _ = _params(n, L, sort_keys=sort_keys)
    st = W.uniform_shell(n, 51, 5.0, 0.3)
    u = W.gaussian_drive(2 * k, sp.dt, 20.0, 289.52, t_center=0.1)
    outs = []
    for _ in range(2):
        with S.Sim(sp, st.pos, st.vel, u) as sim:
            sim.step(2 * k)
            outs.append((sim.read_state(), sim.read_response(0, 2 * k)))
    np.testing.assert_array_equal(outs[0][0]["pos"], outs[1][0]["pos"])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
    with S.Sim(sp, st.pos, st.vel, u) as sim:
        sim.step(k)
        mid = sim.read_state()
        q_first = sim.read_response(0, k)
    keep = mid["alive"] == 1
    ids = np.nonzero(keep)[0].astype(np.uint32)
    sp2 = S.SimParams(**{**sp.__dict__, "q_surface0": mid["q_surface"]})
    with S.Sim(sp2, mid["pos"][keep], mid["vel"][keep], u, ids=ids, start_step=k) as sim:
        sim.step(k)
        end = sim.read_state()
        q_second = sim.read_response(k, k)
    full = outs[0][0]
    np.testing.assert_array_equal(end["pos"], full["pos"][keep])
    np.testing.assert_array_equal(end["vel"], full["vel"][keep])
    np.testing.assert_array_equal(np.concatenate([q_first, q_second]), outs[0][1])
    assert end["q_surface"] == full["q_surface"]


def test_field_evaluation_between_steps_changes_nothing():
    """A field evaluation between steps sorts on its own; the run stays
    bitwise equal to an uninterrupted one (absorbing probe, fast particles so
    that some are absorbed), repeated evaluations agree, and the field of a
    finished run can still be evaluated."""
    n, L, k = 3000, 6, 4
    _say(f"[gpu] field evaluation between steps n={n} L={L} k={k}")
    sp, _ = _params(n, L, sort_keys=1)
    st = W.uniform_shell(n, 53, 1.6, 0.8)
    u = W.gaussian_drive(3 * k, sp.dt, 20.0, 289.52, t_center=0.1)
    with S.Sim(sp, st.pos, st.vel, u) as sim:
        sim.step(3 * k)
        ref = sim.read_state()
        q_ref = sim.read_response(0, 3 * k)
        E_end = sim.eval_field()
    assert (ref["alive"] == 0).any()
    with S.Sim(sp, st.pos, st.vel, u) as sim:
        sim.step(k)
        E1 = sim.eval_field()
        E1b = sim.eval_field()
        sim.step(k)
        sim.eval_field()
        sim.step(k)
        got = sim.read_state()
        q_got = sim.read_response(0, 3 * k)
        E_end_b = sim.eval_field()
    np.testing.assert_array_equal(E1, E1b)
    np.testing.assert_array_equal(got["pos"], ref["pos"])
    np.testing.assert_array_equal(got["vel"], ref["vel"])
    np.testing.assert_array_equal(got["alive"], ref["alive"])
    np.testing.assert_array_equal(q_got, q_ref)
    np.testing.assert_array_equal(E_end_b, E_end)


# --------------------------------------------------------------------------
# FP32-compensated mode: same oracle, bar 1e-5 on the field
# --------------------------------------------------------------------------

FP32_FIELD_TOL = 1e-5

FP32_CASES = [
    # name, n, l_max, m_mode, seed, r_out
    ("shell-3000-L8", 3000, 8, S.SIM_M_FULL, 61, 5.0),
    ("ragged-777-L5", 777, 5, S.SIM_M_FULL, 62, 5.0),
    ("shell-2000-L16", 2000, 16, S.SIM_M_FULL, 63, 5.0),
    ("shell-1500-L20", 1500, 20, S.SIM_M_FULL, 70, 5.0),
    ("shell-1500-L24", 1500, 24, S.SIM_M_FULL, 71, 5.0),
    ("shell-1000-L32", 1000, 32, S.SIM_M_FULL, 64, 5.0),
    ("shell-700-L48", 700, 48, S.SIM_M_FULL, 72, 5.0),
    ("shell-700-L64", 700, 64, S.SIM_M_FULL, 73, 5.0),
    ("axisym-640-L6", 640, 6, S.SIM_M_AXISYM, 65, 5.0),
    ("monopole-500-L0", 500, 0, S.SIM_M_FULL, 66, 5.0),
    # the worst cases of an earlier search over random shells
    ("shell-2109-L13-rout10", 2109, 13, S.SIM_M_FULL, 890459, 10.0),
    ("shell-1390-L13", 1390, 13, S.SIM_M_FULL, 890459, 5.0),
]


def _random_fp32_cases(count=34):
    """Seeded random shells: n in [200, 3000), l_max in [1, 16], outer wall at
    2, 5 or 10 probe radii (denser and sparser than the workloads)."""
    out = []
    for i in range(count):
        g = np.random.default_rng(20211126 + i)
        n = int(g.integers(200, 3000))
        L = int(g.integers(1, 17))
        r_out = (2.0, 5.0, 10.0)[i % 3]
        out.append((f"random{i}-{n}-L{L}-rout{r_out:g}", n, L, S.SIM_M_FULL, 7000 + i, r_out))
    return out


FP32_CASES += _random_fp32_cases()


@pytest.mark.parametrize("name,n,L,mode,seed,r_out", FP32_CASES, ids=[c[0] for c in FP32_CASES])
def test_fp32_field_matches_oracle(name, n, L, mode, seed, r_out):
    _say(f"[gpu] fp32 field parity {name}: n={n} L={L} mode={mode} seed={seed} r_out={r_out}")
    sp, op = _params(n, L, mode, r_out=r_out, q_surface0=-7.0, precision=S.SIM_FP32_COMP)
    st = W.uniform_shell(n, seed, r_out, 0.0831)
    u = np.array([0.0, 0.0, 0.3, 0.0])
    with S.Sim(sp, st.pos, st.vel, u, start_step=2) as sim:
        E = sim.eval_field()
    Eo, _ = O.field(op, st.pos, q_surface=-7.0, u_asy=0.3)
    err = _rel_err(E, Eo)
    _say(f"[gpu]   rel err {err:.3e}")
    assert err <= FP32_FIELD_TOL


@pytest.mark.parametrize("precision,tol", [(S.SIM_FP64, FP64_FIELD_TOL),
                                           (S.SIM_FP32_COMP, FP32_FIELD_TOL)])
def test_near_probe_stress(precision, tol):
    """A fifth of the particles in 1 < r < 1.05, where the direct exterior
    term and the image term of the dielectric oppose each other."""
    n, L = 2500, 16
    _say(f"[gpu] near-probe stress precision={precision} n={n} L={L}")
    st = W.uniform_shell(n, 71, 5.0, 0.0831)
    pos = st.pos.copy()
    rng = np.random.default_rng(71)
    k = rng.choice(n, n // 5, replace=False)
    rr = np.linalg.norm(pos[k], axis=1)
    pos[k] *= ((1.0 + 0.05 * rng.random(k.size)) / rr)[:, None]
    sp, op = _params(n, L, q_surface0=-30.0, precision=precision)
    with S.Sim(sp, pos, st.vel, np.zeros(2)) as sim:
        E = sim.eval_field()
    Eo, _ = O.field(op, pos, q_surface=-30.0)
    err = _rel_err(E, Eo)
    near = _rel_err(E, Eo, mask=np.isin(np.arange(n), k))
    _say(f"[gpu]   rel err {err:.3e} (near-probe subset {near:.3e})")
    assert err <= tol


@pytest.mark.parametrize("n,L,seed,n_t", [(40_000, 8, 91, 200), (40_000, 14, 92, 200),
                                           (60_000, 4, 93, 200), (1_200_000, 32, 94, 64)],
                         ids=["40k-L8", "40k-L14", "60k-L4", "1.2M-L32"])
def test_fp32_dense_sampled(n, L, seed, n_t):
    """FP32 where l_max^2 <= sqrt(n) (the near field per half tile by
    default), at sampled particles against the oracle."""
    _say(f"[gpu] fp32 dense n={n} L={L} seed={seed}")
    sp, op = _params(n, L, q_surface0=-9.0, precision=S.SIM_FP32_COMP)
    st = W.uniform_shell(n, seed, 5.0, 0.0831)
    u = np.array([0.0, 0.0, 0.3, 0.0])
    with S.Sim(sp, st.pos, st.vel, u, start_step=2) as sim:
        E = sim.eval_field()
    targets = np.sort(np.random.default_rng(seed).choice(n, n_t, replace=False))
    Eo, _ = O.field(op, st.pos, q_surface=-9.0, u_asy=0.3, targets=targets)
    rms = np.sqrt(np.mean(np.sum(Eo * Eo, axis=1)))
    err = float(np.max(np.abs(E[targets] - Eo)) / rms)
    _say(f"[gpu]   rel err {err:.3e}")
    assert err <= FP32_FIELD_TOL


def test_fp32_large_workload_sampled_field():
    wl = W.LARGE
    _say(f"[gpu] fp32 sampled field parity {wl.name}")
    st = wl.particles()
    sp, op = _params(wl.n, wl.l_max, q_surface0=-40.0, precision=S.SIM_FP32_COMP)
    u = wl.drive(30)
    with S.Sim(sp, st.pos, st.vel, u, start_step=20) as sim:
        E = sim.eval_field()
    rng = np.random.default_rng(5)
    targets = np.sort(rng.choice(wl.n, 48, replace=False))
    Eo, _ = O.field(op, st.pos, q_surface=-40.0, u_asy=u[20], targets=targets)
    rms = np.sqrt(np.mean(np.sum(Eo * Eo, axis=1)))
    err = float(np.max(np.abs(E[targets] - Eo)) / rms)
    _say(f"[gpu]   rel err {err:.3e}")
    assert err <= FP32_FIELD_TOL


@pytest.mark.parametrize("L", [8, 20, 34], ids=["L8", "L20", "L34-fp64-near"])
def test_fp32_steps_track_oracle(L):
    n, steps = 2000, 5
    _say(f"[gpu] fp32 stepping n={n} L={L} steps={steps}")
    sp, op = _params(n, L, q_surface0=-2.0, precision=S.SIM_FP32_COMP)
    st = W.uniform_shell(n, 41, 5.0, 0.3)
    u = W.gaussian_drive(steps, sp.dt, 50.0, 289.52, t_center=0.1)
    with S.Sim(sp, st.pos, st.vel, u) as sim:
        sim.step(steps)
        qd = sim.read_response(0, steps)
        out = sim.read_state()
    ref = O.run(op, st.pos, st.vel, u, steps, q_surface=-2.0)
    np.testing.assert_array_equal(out["alive"], ref.alive)
    # a relative field error e moves a particle by < e |E| dt^2 per step
    assert np.max(np.abs(out["pos"] - ref.pos)) <= 1e-2 * FP32_FIELD_TOL
    assert np.max(np.abs(qd - ref.qdiff)) <= 0.1 * FP32_FIELD_TOL * np.max(np.abs(ref.qdiff))
