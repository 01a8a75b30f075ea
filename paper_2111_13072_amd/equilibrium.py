"""Initial condition: the floating probe-plasma equilibrium of App. D.

Spherically symmetric, in units of R and of the potential T_e / e
(psi = e Phi / T_e, psi -> 0 far away), with Lambda = lambda_D / R:

  Poisson:    -Lambda^2 (1/r^2) d/dr (r^2 dpsi/dr) = n_i - n_e
  electrons:  n_e = exp(psi)                                 (Boltzmann)
  ions:       n_i = (R^2 / r^2) / sqrt(-2 psi)  (cold radial inflow with the
              constant flux 4 pi R^2 n_inf sqrt(T_e/m_i), energy conservation)
  floating:   R^2 sqrt(T_e/m_i) = sqrt(T_e/(2 pi m_e)) exp(psi(1))
              (Hertz-Langmuir: ion and electron fluxes to the probe equal)

where R stands for the unknown flux radius R^ of App. D.  For a trial R^ the
Poisson equation is integrated inward from far away, where the plasma is
quasi-neutral (n_i = n_e fixes psi(r)), to the probe surface; the floating
condition is then one equation for R^, solved by bracketing (shooting).

The probe's static charge follows from Gauss's law at r = 1:
Q_S = -4 pi Lambda^2 psi'(1) in units of e n_inf R^3 (negative).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .workload import ParticleState, PlasmaScales

# Electron masses per ion mass unit (CODATA 2018) and argon's atomic mass
# (the paper does not name the gas; argon is taken).
AMU_IN_ME = 1822.888486
ARGON_AMU = 39.948


@dataclass
class Equilibrium:
    debye: float          # Lambda = lambda_D / R
    mass_ratio: float     # m_i / m_e
    r_hat: float          # flux radius R^ (units of R)
    psi_probe: float      # psi(1)
    dpsi_probe: float     # psi'(1)
    _sol: object          # dense solution of the inward integration
    r_start: float        # where the integration started (quasi-neutral)

    def psi(self, r):
        """Potential e Phi / T_e at radii r >= 1."""
        r = np.asarray(r, dtype=np.float64)
        out = np.empty_like(r)
        inner = r <= self.r_start
        out[inner] = self._sol.sol(r[inner])[0]
        out[~inner] = [quasi_neutral_psi(x, self.r_hat) for x in np.atleast_1d(r[~inner])]
        return out

    def n_e(self, r):
        return np.exp(self.psi(r))

    def n_i(self, r):
        r = np.asarray(r, dtype=np.float64)
        return self.r_hat ** 2 / r ** 2 / np.sqrt(-2.0 * self.psi(r))

    @property
    def surface_charge(self) -> float:
        """Q_S in units of e n_inf R^3."""
        return -4.0 * math.pi * self.debye ** 2 * self.dpsi_probe

    def ion_profile(self, r_out: float, nodes: int = 4097) -> np.ndarray:
        """Ion density at `nodes` equally spaced radii from 1 to r_out."""
        return self.n_i(np.linspace(1.0, r_out, nodes))


def quasi_neutral_psi(r: float, r_hat: float) -> float:
    """psi with n_i = n_e: exp(psi) sqrt(-2 psi) = R^2 / r^2, on the branch
    -1/2 < psi < 0 (ions slower than the Bohm speed)."""
    from scipy.optimize import brentq

    t = r_hat ** 2 / r ** 2
    if t >= math.exp(-0.5):
        raise ValueError("no quasi-neutral solution inside the sonic radius")
    return brentq(lambda p: math.exp(p) * math.sqrt(-2.0 * p) - t, -0.5, -1e-300, xtol=1e-300)


def _integrate_inward(debye: float, r_hat: float, r_start: float, rtol: float = 1e-11):
    from scipy.integrate import solve_ivp

    p0 = quasi_neutral_psi(r_start, r_hat)
    dp0 = -2.0 / (r_start * (1.0 + 1.0 / (2.0 * p0)))   # derivative of the quasi-neutral psi
    inv_l2 = 1.0 / debye ** 2

    def rhs(r, y):
        p = min(y[0], -1e-300)
        return [y[1], -2.0 * y[1] / r + inv_l2 * (math.exp(p) - r_hat ** 2 / r ** 2 / math.sqrt(-2.0 * p))]

    return solve_ivp(rhs, [r_start, 1.0], [p0, dp0], method="LSODA", rtol=rtol, atol=1e-14,
                     dense_output=True)


def solve_floating_equilibrium(debye: float, mass_ratio: float = ARGON_AMU * AMU_IN_ME,
                               r_start: float | None = None) -> Equilibrium:
    """Shoot for R^ such that the floating condition holds at r = 1."""
    from scipy.optimize import brentq

    c = math.sqrt(mass_ratio / (2.0 * math.pi))

    def start(rh):
        # where the quasi-neutral |psi| is 1e-4 (-2 psi ~ (R^/r)^4): further out
        # the Poisson correction to quasi-neutrality is ~ Lambda^2 psi^2 / r^2
        # (below 1e-11), while the ion term makes the equation ever stiffer
        return r_start if r_start is not None else max(2.0, rh * (2e-4) ** -0.25)

    def mismatch(rh):
        sol = _integrate_inward(debye, rh, start(rh))
        if sol.status != 0:
            raise RuntimeError(f"inward integration failed for R^ = {rh}: {sol.message}")
        return sol.y[0, -1] - math.log(rh * rh / c)

    # bracket: small R^ keeps the probe in the quasi-neutral region (psi(1) >
    # -1/2 while the floating potential is far below); grow until the sign flips
    lo, hi = 0.3, 0.45
    f_lo = mismatch(lo)
    while True:
        f_hi = mismatch(hi)
        if f_lo > 0 > f_hi:
            break
        lo, f_lo, hi = hi, f_hi, hi * 1.5
        if hi > 1e3:
            raise RuntimeError("no floating equilibrium found")
    rh = brentq(mismatch, lo, hi, xtol=1e-14)
    sol = _integrate_inward(debye, rh, start(rh))
    return Equilibrium(debye, mass_ratio, rh, float(sol.y[0, -1]), float(sol.y[1, -1]), sol,
                       start(rh))


def sample_electrons(eq: Equilibrium, n: int, seed: int, r_out: float, v_th: float,
                     grid: int = 200001) -> ParticleState:
    """n electrons with radial density n_e(r) 4 pi r^2 on (1, r_out) (inverse
    CDF on a fine grid), isotropic directions and Maxwellian velocities of
    thermal speed v_th per component.  Draw order: U_r, U_c, U_phi [n], then
    a standard normal [n, 3]."""
    rg = np.linspace(1.0, r_out, grid)
    w = eq.n_e(rg) * rg ** 2
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (w[1:] + w[:-1]) * np.diff(rg))])
    cdf /= cdf[-1]
    rng = np.random.Generator(np.random.PCG64(seed))
    ur, uc, uphi = rng.random(n), rng.random(n), rng.random(n)
    vel = v_th * rng.standard_normal((n, 3))
    r = np.interp(ur, cdf, rg)
    r = np.clip(r, np.nextafter(1.0, 2.0), np.nextafter(r_out, 0.0))
    ct = 2.0 * uc - 1.0
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    ph = 2.0 * np.pi * uphi
    pos = np.stack([r * st * np.cos(ph), r * st * np.sin(ph), r * ct], axis=1)
    return ParticleState(pos=pos, vel=vel, ids=np.arange(n, dtype=np.uint32))


def _radial_cdf(density, r_out: float, grid: int):
    rg = np.linspace(1.0, r_out, grid)
    w = density(rg) * rg ** 2
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (w[1:] + w[:-1]) * np.diff(rg))])
    return rg, cdf


def electron_count_density(eq: Equilibrium, r_out: float, grid: int = 200001) -> float:
    """4 pi int_1^r_out n_e r^2 dr: electrons (in n_inf R^3) between the walls."""
    _, cdf = _radial_cdf(eq.n_e, r_out, grid)
    return float(4.0 * np.pi * cdf[-1])


def ion_count_density(eq: Equilibrium, r_out: float, grid: int = 200001) -> float:
    """4 pi int_1^r_out n_i r^2 dr: ions (in n_inf R^3) between the walls."""
    _, cdf = _radial_cdf(eq.n_i, r_out, grid)
    return float(4.0 * np.pi * cdf[-1])


ION_ID_BIT = np.uint32(0x80000000)


def sample_ions(eq: Equilibrium, n: int, seed: int, r_out: float, id_offset: int = 0,
                grid: int = 200001) -> ParticleState:
    """n ions with radial density n_i(r) 4 pi r^2 on (1, r_out), isotropic
    directions and the cold radial inflow of App. D: speed
    sqrt(-2 psi) c_s toward the probe, c_s = Lambda sqrt(m_e/m_i) in units of
    R omega_pe.  Ids id_offset.. with bit 31 set (the ion marker).  Draw
    order: U_r, U_c, U_phi [n]."""
    rg, cdf = _radial_cdf(eq.n_i, r_out, grid)
    cdf /= cdf[-1]
    rng = np.random.Generator(np.random.PCG64(seed))
    ur, uc, uphi = rng.random(n), rng.random(n), rng.random(n)
    r = np.clip(np.interp(ur, cdf, rg), np.nextafter(1.0, 2.0), np.nextafter(r_out, 0.0))
    ct = 2.0 * uc - 1.0
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    ph = 2.0 * np.pi * uphi
    rhat = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)
    c_s = eq.debye / math.sqrt(eq.mass_ratio)
    speed = np.sqrt(-2.0 * eq.psi(r)) * c_s
    ids = (np.arange(n, dtype=np.uint32) + np.uint32(id_offset)) | ION_ID_BIT
    return ParticleState(pos=r[:, None] * rhat, vel=-speed[:, None] * rhat, ids=ids)


@dataclass
class PaperSetup:
    """The paper's own workload (Sec. 4 with App. D): the floating
    equilibrium between the probe and r_out = 10 at n_inf = 1e15 m^-3,
    T_e = 3 eV, diffuse walls, dt = 0.01, impulse drive; n super-particles
    in total, electrons and mobile ions in the equilibrium's proportion
    (or, with mobile_ions False, n electrons over an immobile ion profile)."""
    n: int = 1_000_000
    seed: int = 6
    n_e: float = 1e15
    t_e_ev: float = 3.0
    r_out: float = 10.0
    dt: float = 0.01
    probe_radius_m: float = 4e-3
    mobile_ions: bool = True

    def build(self):
        """(equilibrium, particles, ntilde, q_surface0 in super-particle units,
        ion profile or None)."""
        sc = PlasmaScales(self.n_e, self.t_e_ev, self.probe_radius_m)
        eq = solve_floating_equilibrium(sc.v_th)
        ne = electron_count_density(eq, self.r_out)
        if not self.mobile_ions:
            st = sample_electrons(eq, self.n, self.seed, self.r_out, sc.v_th)
            ntilde = self.n / ne
            return eq, st, ntilde, eq.surface_charge * ntilde, eq.ion_profile(self.r_out)
        ni = ion_count_density(eq, self.r_out)
        ntilde = self.n / (ne + ni)
        n_el = int(round(ntilde * ne))
        el = sample_electrons(eq, n_el, self.seed, self.r_out, sc.v_th)
        io = sample_ions(eq, self.n - n_el, self.seed + 1, self.r_out, id_offset=n_el)
        st = ParticleState(pos=np.concatenate([el.pos, io.pos]),
                           vel=np.concatenate([el.vel, io.vel]),
                           ids=np.concatenate([el.ids, io.ids]))
        return eq, st, ntilde, eq.surface_charge * ntilde, None
