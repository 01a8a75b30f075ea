"""Seeded synthetic inputs for the probe simulation.

This module holds no arithmetic of the simulation method itself: it only
draws particle states and drive waveforms, and converts physical plasma
parameters into the dimensionless units the method works in (lengths in
units of the probe radius R, times in 1/omega_pe, charges in e, masses in
m_e, densities in n_inf; Sec. 4 of the paper).  Both the HIP path and the
CPU oracle receive exactly the arrays produced here.

Recipe for the uniform shell (the stand-in for the paper's Poisson-Boltzmann
equilibrium of App. D, whose profile values the paper does not print):
numpy Generator(PCG64(seed)); draw U_r, U_c, U_phi of shape [N], in that
order, then a standard normal of shape [N, 3].  Then
r = (1 + U_r (r_out^3 - 1))^(1/3), cos(theta) = 2 U_c - 1, phi = 2 pi U_phi,
v = v_th * normal with v_th = lambda_D / R (thermal speed sqrt(T_e/m_e) in
units of R omega_pe).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# CODATA 2018 values (SI).
E_CHARGE = 1.602176634e-19
EPS0 = 8.8541878128e-12
M_E = 9.1093837015e-31


@dataclass(frozen=True)
class PlasmaScales:
    """Physical scales of a plasma of density n_e [m^-3] and temperature T_e [eV]."""

    n_e: float
    t_e_ev: float
    probe_radius_m: float

    @property
    def omega_pe(self) -> float:
        return math.sqrt(self.n_e * E_CHARGE**2 / (EPS0 * M_E))

    @property
    def debye_length_m(self) -> float:
        return math.sqrt(EPS0 * self.t_e_ev / (self.n_e * E_CHARGE))

    @property
    def v_th(self) -> float:
        """Thermal speed sqrt(T_e/m_e) in units of R*omega_pe, i.e. lambda_D/R."""
        return self.debye_length_m / self.probe_radius_m

    @property
    def u0_volts(self) -> float:
        """Potential unit e n_e R^2 / eps0 of the dimensionless Poisson equation."""
        return E_CHARGE * self.n_e * self.probe_radius_m**2 / EPS0


def shell_volume(r_out: float) -> float:
    """Volume of the shell 1 < r < r_out in units of R^3."""
    return 4.0 * math.pi / 3.0 * (r_out**3 - 1.0)


def ntilde_for(n_particles: int, r_out: float) -> float:
    """Super-particles per unit volume R^3 when n_particles fill the shell at density n_e."""
    return n_particles / shell_volume(r_out)


@dataclass
class ParticleState:
    pos: np.ndarray  # float64 [N, 3]
    vel: np.ndarray  # float64 [N, 3], velocity at t = -dt/2
    ids: np.ndarray  # uint32 [N]


def uniform_shell(n: int, seed: int, r_out: float, v_th: float) -> ParticleState:
    """Uniform density in 1 < r < r_out, isotropic angles, Maxwellian velocities."""
    g = np.random.Generator(np.random.PCG64(seed))
    u_r = g.random(n)
    u_c = g.random(n)
    u_p = g.random(n)
    normal = g.standard_normal((n, 3))
    r = np.cbrt(1.0 + u_r * (r_out**3 - 1.0))
    ct = 2.0 * u_c - 1.0
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    ph = 2.0 * math.pi * u_p
    pos = np.empty((n, 3))
    pos[:, 0] = r * st * np.cos(ph)
    pos[:, 1] = r * st * np.sin(ph)
    pos[:, 2] = r * ct
    vel = v_th * normal
    ids = np.arange(n, dtype=np.uint32)
    return ParticleState(np.ascontiguousarray(pos), np.ascontiguousarray(vel), ids)


def quantile_shell(n: int, seed: int, r_out: float, ntilde: float,
                   amplitude: float = 0.01) -> ParticleState:
    """Cold shell with particle k at the radius that encloses k + 1/2 super-particles
    of a unit-density background, then displaced radially by
    amplitude * sin(pi (r - 1) / (r_out - 1)).  Angles are isotropic (seeded);
    velocities are zero.  Used for the bulk plasma-oscillation check."""
    g = np.random.Generator(np.random.PCG64(seed))
    u_c = g.random(n)
    u_p = g.random(n)
    k = np.arange(n, dtype=np.float64)
    vol = (k + 0.5) / ntilde
    r0 = np.cbrt(1.0 + vol * 3.0 / (4.0 * math.pi))
    r = r0 + amplitude * np.sin(math.pi * (r0 - 1.0) / (r_out - 1.0))
    ct = 2.0 * u_c - 1.0
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    ph = 2.0 * math.pi * u_p
    pos = np.stack([r * st * np.cos(ph), r * st * np.sin(ph), r * ct], axis=1)
    return ParticleState(np.ascontiguousarray(pos), np.zeros((n, 3)),
                         np.arange(n, dtype=np.uint32))


def gaussian_drive(n_steps: int, dt: float, volts: float, u0_volts: float,
                   sigma: float = 0.2, t_center: float = 1.0) -> np.ndarray:
    """u_asy[n] = u_1 - u_2 for a +volts / -volts Gaussian pulse on the two
    hemispheres, in units of u0_volts, sampled at t_n = n dt."""
    t = np.arange(n_steps, dtype=np.float64) * dt
    return 2.0 * volts * np.exp(-((t - t_center) ** 2) / (2.0 * sigma**2)) / u0_volts


def impulse_drive(n_steps: int, amplitude: float = 1.0) -> np.ndarray:
    """u_asy = amplitude at the first step only, zero afterwards (Sec. 4)."""
    u = np.zeros(n_steps)
    if n_steps:
        u[0] = amplitude
    return u


@dataclass(frozen=True)
class Workload:
    """One of the standard workloads (geometry d = 0.25, eps_r = 4, r_out = 5,
    dt = 0.05, immobile unit-density ion background, +-1 V Gaussian pulse)."""

    name: str
    n: int
    seed: int
    l_max: int
    n_steps: int
    n_e: float = 1e15
    t_e_ev: float = 2.0
    probe_radius_m: float = 4e-3
    d: float = 0.25
    eps_r: float = 4.0
    r_out: float = 5.0
    dt: float = 0.05
    volts: float = 1.0

    @property
    def scales(self) -> PlasmaScales:
        return PlasmaScales(self.n_e, self.t_e_ev, self.probe_radius_m)

    @property
    def ntilde(self) -> float:
        return ntilde_for(self.n, self.r_out)

    def particles(self) -> ParticleState:
        return uniform_shell(self.n, self.seed, self.r_out, self.scales.v_th)

    def drive(self, n_steps: int | None = None) -> np.ndarray:
        return gaussian_drive(self.n_steps if n_steps is None else n_steps, self.dt,
                              self.volts, self.scales.u0_volts)


SMALL_FP64 = Workload("shell-1e4-L8", n=10_000, seed=1, l_max=8, n_steps=1000)
LARGE = Workload("shell-2e6-L16", n=2_000_000, seed=2, l_max=16, n_steps=20_000)


def sweep_workload(l_max: int, n_e: float, t_e_ev: float) -> Workload:
    return Workload(f"shell-1.6e7-L{l_max}-n{n_e:.0e}-T{t_e_ev:g}", n=16_000_000, seed=3,
                    l_max=l_max, n_steps=10_000, n_e=n_e, t_e_ev=t_e_ev)


# The largest single-GPU run: the scale sweep at l_max 16, n_e 1e15 m^-3,
# T_e 3 eV (the benchmark's default workload).
SCALE = sweep_workload(16, 1e15, 3.0)


def batch_workloads(count: int = 64, seed: int = 4, l_max: int = 16,
                    n_steps: int = 5000) -> list[Workload]:
    """Independent runs of a parameter scan, drawn in this order from one
    generator: log10 N ~ U(4, 6), T_e ~ U(1, 5) eV, log10 n_e ~ U(14, 16)
    m^-3.  Member k's particles come from seed 1000 * seed + k."""
    rng = np.random.Generator(np.random.PCG64(seed))
    log_n = rng.uniform(4.0, 6.0, count)
    t_e = rng.uniform(1.0, 5.0, count)
    log_ne = rng.uniform(14.0, 16.0, count)
    return [Workload(f"batch{seed}-{k}", n=int(round(10.0 ** log_n[k])), seed=1000 * seed + k,
                     l_max=l_max, n_steps=n_steps, n_e=float(10.0 ** log_ne[k]),
                     t_e_ev=float(t_e[k]))
            for k in range(count)]
