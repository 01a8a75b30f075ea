"""The allocation-free field evaluation (sim_eval_field_static) against the
handle's sim_eval_field: the same kernels on the same state, so the same
field bit for bit, on consecutive calls (the second smaller, so the static
buffer holds the first call's contents), in FP64 and FP32-compensated; and
the FP64 field against the CPU oracle."""
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


def _handle_field(sp, pos, q_surface, u_asy):
    u = np.array([0.0, 0.0, u_asy, 0.0])
    with S.Sim(sp, pos, np.zeros_like(pos), u, start_step=2) as sim:
        return sim.eval_field()


@pytest.mark.parametrize("precision", [S.SIM_FP64, S.SIM_FP32_COMP], ids=["fp64", "fp32c"])
def test_static_field_equals_handle_field_on_consecutive_calls(precision):
    import torch

    for n, L, seed, qs, ua in ((5000, 8, 81, -7.0, 0.3), (1200, 6, 82, -3.0, -0.2)):
        _say(f"[gpu] static field n={n} L={L} seed={seed} precision={precision}")
        st = W.uniform_shell(n, seed, 5.0, 0.08)
        sp = S.SimParams(ntilde=W.ntilde_for(n, 5.0), l_max=L, q_surface0=qs,
                         precision=precision)
        assert S.eval_field_static_bytes(sp, n) <= 64 << 20
        pos_d = torch.from_numpy(st.pos).to("cuda")
        E_d = torch.full((n, 3), float("nan"), dtype=torch.float64, device="cuda")
        S.eval_field_static(sp, pos_d, E_d, q_surface=qs, u_asy=ua)
        E = E_d.cpu().numpy()
        Eh = _handle_field(sp, st.pos, qs, ua)
        np.testing.assert_array_equal(E, Eh)
        if precision == S.SIM_FP64:
            op = O.Params(ntilde=sp.ntilde, l_max=L)
            Eo, _ = O.field(op, st.pos, q_surface=qs, u_asy=ua)
            rms = np.sqrt(np.mean(np.sum(Eo * Eo, axis=1)))
            err = float(np.max(np.abs(E - Eo)) / rms)
            _say(f"[gpu]   vs oracle {err:.2e}")
            assert err <= 1e-12


def test_static_field_rejects_what_does_not_fit():
    import torch

    sp = S.SimParams(ntilde=1.0, l_max=32)
    n = 400_000
    assert S.eval_field_static_bytes(sp, n) > 64 << 20
    pos_d = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    E_d = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(S.SimError) as ei:
        S.eval_field_static(sp, pos_d, E_d)
    assert ei.value.code == S.SIM_ENOMEM
