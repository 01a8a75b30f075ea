"""Write the stored oracle references used by the GPU tests.

Calls only oracle/ and the seeded input generators; nothing from the HIP
path.  Run:  OMP_NUM_THREADS=<cores> python tests/golden/make_golden.py [impulse|gaussian]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2111_13072_amd import workload as W  # noqa: E402

IMPULSE_STEPS = 400
IMPULSE_FILE = os.path.join(HERE, "shell-1e4-L8_impulse_qdiff.txt")
PERTURBATION = 1e-12


def impulse_twins_small():
    """The 1e4-particle, l_max = 8 workload driven by the impulse of Sec. 4
    (u_asy = 1 at the first step only), its undriven twin, and the driven run
    again from positions perturbed by a relative 1e-12 (the chaotic divergence
    envelope of the trajectory)."""
    wl = W.SMALL_FP64
    st = wl.particles()
    p = O.Params(d=wl.d, eps_r=wl.eps_r, r_out=wl.r_out, dt=wl.dt, ntilde=wl.ntilde,
                 ion_density=1.0, l_max=wl.l_max)
    kick = W.impulse_drive(IMPULSE_STEPS, 1.0)
    jitter = np.random.default_rng(99).standard_normal(st.pos.shape)
    runs = [("driven", st.pos, kick),
            ("undriven", st.pos, np.zeros(IMPULSE_STEPS)),
            ("driven, perturbed", st.pos * (1.0 + PERTURBATION * jitter), kick)]
    cols = []
    for name, pos, u in runs:
        t0 = time.time()
        r = O.run(p, pos, st.vel, u, IMPULSE_STEPS)
        print(f"oracle {name}: {time.time() - t0:.0f} s, absorbed {r.absorbed}",
              flush=True)
        cols.append(r.qdiff)
    header = ("Q_diff(t_n), n = 0..%d, from the oracle.  Workload shell-1e4-L8: N = 1e4 uniform "
              "shell, seed 1, T_e = 2 eV, n_e = 1e15 m^-3, l_max 8 FULL, dt 0.05, absorb/specular.  "
              "Drive: u_asy = 1 at n = 0 only (impulse, Sec. 4).  Columns: driven; undriven twin; "
              "driven from positions scaled by 1 + %g * N(0,1) (numpy default_rng(99))."
              % (IMPULSE_STEPS - 1, PERTURBATION))
    np.savetxt(IMPULSE_FILE, np.stack(cols, axis=1), header=header, fmt="%.17e")
    print("wrote", IMPULSE_FILE)


GAUSS_STEPS = 1000
GAUSS_FILE = os.path.join(HERE, "shell-1e4-L8_gaussian_qdiff.txt")


def gaussian_twins_small():
    """The 1e4-particle, l_max = 8 workload as specified for the plain FP64
    run: the +-1 V Gaussian pulse on the two hemispheres (sigma 0.2, centre
    1.0 in 1/omega_pe), 1000 steps; its undriven twin; and the driven run from
    positions perturbed by a relative 1e-12 (the divergence envelope)."""
    wl = W.SMALL_FP64
    st = wl.particles()
    p = O.Params(d=wl.d, eps_r=wl.eps_r, r_out=wl.r_out, dt=wl.dt, ntilde=wl.ntilde,
                 ion_density=1.0, l_max=wl.l_max)
    u = wl.drive(GAUSS_STEPS)
    jitter = np.random.default_rng(99).standard_normal(st.pos.shape)
    runs = [("driven", st.pos, u),
            ("undriven", st.pos, np.zeros(GAUSS_STEPS)),
            ("driven, perturbed", st.pos * (1.0 + PERTURBATION * jitter), u)]
    cols = []
    for name, pos, drive in runs:
        t0 = time.time()
        r = O.run(p, pos, st.vel, drive, GAUSS_STEPS)
        print(f"oracle {name}: {time.time() - t0:.0f} s, absorbed {r.absorbed}", flush=True)
        cols.append(r.qdiff)
    header = ("Q_diff(t_n), n = 0..%d, from the oracle.  Workload shell-1e4-L8: N = 1e4 uniform "
              "shell, seed 1, T_e = 2 eV, n_e = 1e15 m^-3, l_max 8 FULL, dt 0.05, absorb/specular.  "
              "Drive: +-1 V Gaussian pulse, u_asy = 2 V g(t) / U0, sigma 0.2, centre 1.0, U0 = "
              "%.6g V.  Columns: driven; undriven twin; driven from positions scaled by "
              "1 + %g * N(0,1) (numpy default_rng(99))."
              % (GAUSS_STEPS - 1, wl.scales.u0_volts, PERTURBATION))
    np.savetxt(GAUSS_FILE, np.stack(cols, axis=1), header=header, fmt="%.17e")
    print("wrote", GAUSS_FILE)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    if which in ("all", "impulse"):
        impulse_twins_small()
    if which in ("all", "gaussian"):
        gaussian_twins_small()
