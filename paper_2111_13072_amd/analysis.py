"""Response analysis of the probe (host side): Q_diff(t) -> spectrum.

The probe signal is u_asy(t) and its response the electrode charge
difference Q_diff(t) (Sec. 4).  The static part of Q_diff is thermal noise of
the finite particle number, so the response is taken as the difference of a
driven run and an undriven twin started from the same state.

* damped-sine fit (Sec. 4): f(t) = a exp(-b (t - t0)) sin(c (t - t0) + phi) + d
  for t > t0; the resonance is at c and its half-width (full width at half
  maximum of the Lorentzian) is 2b.
* admittance: with the current I = dQ_diff/dt, Y(omega) = I^(omega) / u^(omega)
  = i omega Q^(omega) / u^(omega) (Sec. 4, the admittance from the Fourier
  transform of Q_diff); Re Y peaks at the resonance.  Zero padding refines the
  frequency grid.
"""
from __future__ import annotations

import warnings
from dataclasses import dataclass

import numpy as np


@dataclass
class DampedSine:
    amplitude: float
    damping: float      # b
    frequency: float    # c  (resonance, units of omega_pe)
    phase: float
    offset: float
    t0: float

    @property
    def fwhm(self) -> float:
        """Full width at half maximum of the Lorentzian |response|^2 peak: 2b."""
        return 2.0 * self.damping

    def __call__(self, t):
        t = np.asarray(t, dtype=np.float64) - self.t0
        return self.amplitude * np.exp(-self.damping * t) * np.sin(self.frequency * t + self.phase) \
            + self.offset


def twin_difference(q_driven, q_undriven) -> np.ndarray:
    return np.asarray(q_driven, dtype=np.float64) - np.asarray(q_undriven, dtype=np.float64)


def _dominant_frequency(tt, qq) -> float:
    n = 16 * len(qq)
    spec = np.abs(np.fft.rfft((qq - qq.mean()) * np.hanning(len(qq)), n))
    w = 2 * np.pi * np.fft.rfftfreq(n, tt[1] - tt[0])
    return float(w[1 + np.argmax(spec[1:])])


def _normalise(a, b, c, ph, t0) -> DampedSine:
    if a < 0:
        a, ph = -a, ph + np.pi
    if c < 0:
        c, ph = -c, np.pi - ph
    return DampedSine(float(a), float(b), float(c), float(np.mod(ph, 2 * np.pi)), 0.0, t0)


def fit_damped_sines(t, q, t0: float, w_guesses, b_guess: float = 0.05) -> tuple[list[DampedSine], float]:
    """Least-squares fit of a sum of damped sines (the mode expansion of the
    fit function in Sec. 4), f(t) = sum_s a_s exp(-b_s (t - t0)) sin(c_s (t - t0) + phi_s) + d,
    to q(t) for t >= t0, one mode per entry of w_guesses.  Returns the modes
    sorted by frequency and the offset d."""
    from scipy.optimize import OptimizeWarning, curve_fit

    t = np.asarray(t, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    m = t >= t0
    tt, qq = t[m] - t0, q[m]
    ns = len(w_guesses)
    a0 = float(np.max(np.abs(qq - qq.mean()))) / ns

    def f(t, *p):
        out = np.full_like(t, p[-1])
        with np.errstate(over="ignore", invalid="ignore"):
            for s in range(ns):
                a, b, c, ph = p[4 * s:4 * s + 4]
                out += a * np.exp(-b * t) * np.sin(c * t + ph)
        return out

    best = None
    for ph0 in (0.0, np.pi / 2, np.pi, 3 * np.pi / 2):
        p0 = []
        for w in w_guesses:
            p0 += [a0, b_guess, float(w), ph0]
        p0.append(float(qq.mean()))
        try:
            with warnings.catch_warnings():
                warnings.simplefilter("ignore", OptimizeWarning)
                popt, _ = curve_fit(f, tt, qq, p0=p0, maxfev=40000)
        except RuntimeError:
            continue
        res = float(np.sum((f(tt, *popt) - qq) ** 2))
        if not np.isfinite(res):
            continue
        if best is None or res < best[0]:
            best = (res, popt)
    if best is None:
        raise RuntimeError("damped-sine fit did not converge")
    popt = best[1]
    modes = [_normalise(*popt[4 * s:4 * s + 4], t0) for s in range(ns)]
    d = float(popt[-1])
    for md in modes:
        md.offset = d
    return sorted(modes, key=lambda md: md.frequency), d


def fit_damped_sine(t, q, t0: float, w_guess: float | None = None) -> DampedSine:
    """Single-mode fit (s = 1 in the mode expansion of Sec. 4): the resonance
    is c and the half-width 2b."""
    t = np.asarray(t, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    if w_guess is None:
        m = t >= t0
        w_guess = _dominant_frequency(t[m] - t0, q[m])
    modes, _ = fit_damped_sines(t, q, t0, [w_guess])
    return modes[0]


@dataclass
class Spectrum:
    omega: np.ndarray
    admittance: np.ndarray   # complex Y(omega)

    def peak(self) -> tuple[float, float]:
        """(omega at max Re Y by parabolic interpolation, FWHM of Re Y by linear
        interpolation of the half-maximum crossings)."""
        re = self.admittance.real
        i = int(np.argmax(re))
        if 0 < i < len(re) - 1:
            y0, y1, y2 = re[i - 1], re[i], re[i + 1]
            den = y0 - 2 * y1 + y2
            shift = 0.5 * (y0 - y2) / den if den != 0 else 0.0
        else:
            shift = 0.0
        dw = self.omega[1] - self.omega[0]
        w_peak = float(self.omega[i] + shift * dw)
        half = 0.5 * re[i]
        lo = i
        while lo > 0 and re[lo] > half:
            lo -= 1
        hi = i
        while hi < len(re) - 1 and re[hi] > half:
            hi += 1

        def cross(a, b):
            ya, yb = re[a], re[b]
            if yb == ya:
                return float(self.omega[a])
            return float(self.omega[a] + (half - ya) / (yb - ya) * (self.omega[b] - self.omega[a]))

        return w_peak, cross(hi - 1, hi) - cross(lo, lo + 1)


def admittance(q_response, u_asy, dt: float, pad: int = 16, w_max: float = 2.0) -> Spectrum:
    """Y(omega) = i omega Q^(omega) / u^(omega): the current is dQ/dt, so its
    transform is i omega times that of Q (Sec. 4, admittance from the Fourier
    transform of Q_diff).  Transforming Q rather than a differenced current
    avoids the half-sample error at the kink of an impulse response; both
    transforms use the same zero padding."""
    q = np.asarray(q_response, dtype=np.float64)
    u = np.asarray(u_asy, dtype=np.float64)[:len(q)]
    n = pad * len(q)
    Qh = np.fft.rfft(q, n) * dt
    Uh = np.fft.rfft(u, n) * dt
    w = 2 * np.pi * np.fft.rfftfreq(n, dt)
    keep = (w > 0) & (w <= w_max)
    with np.errstate(divide="ignore", invalid="ignore"):
        Y = 1j * w[keep] * Qh[keep] / Uh[keep]
    return Spectrum(w[keep], Y)


def admittance_from_fit(fit: DampedSine, omega, u_area: float = 1.0) -> Spectrum:
    """Admittance of the fitted response (Sec. 4 takes the Fourier transform
    of the fit).  The fit, a exp(-b (t - t0)) sin(c (t - t0) + phi) for
    t >= t0, is continued back to the impulse at t = 0 as
    a' exp(-b t) sin(c t + phi') with a' = a exp(b t0), phi' = phi - c t0;
    its transform is Q^(w) = a' [c cos phi' + (b + i w) sin phi'] /
    ((b + i w)^2 + c^2), and Y = i w Q^ / u^ with u^ = u_area for an impulse.
    The fit's constant offset, a static shift, is left out."""
    w = np.asarray(omega, dtype=np.float64)
    amp = fit.amplitude * np.exp(fit.damping * fit.t0)
    ph = fit.phase - fit.frequency * fit.t0
    s = fit.damping + 1j * w
    qh = amp * (fit.frequency * np.cos(ph) + s * np.sin(ph)) / (s * s + fit.frequency ** 2)
    return Spectrum(w, 1j * w * qh / u_area)


def lorentzian_from_fit(fit: DampedSine, omega) -> np.ndarray:
    """Spectrum of the fitted damped sine (Sec. 4: the transform of the fit)."""
    w = np.asarray(omega, dtype=np.float64)
    return fit.amplitude / ((fit.frequency - w) ** 2 + fit.damping ** 2)


# ---------------------------------------------------------------------------
# Drude (cold fluid) model of the ideal probe and the temperature formula
# (Sec. 4: admittance as vacuum coupling plus series resonance circuits, the
# least-squares match of the kinetic admittance, nu_eff = K v_th / R).
#
# Geometry (units of R): electrodes of radius a = 1 - d at potentials
# +-u/2 (hemispheres), dielectric eps_r on (a, 1), vacuum sheath on
# (1, 1 + delta), plasma of permittivity eps_p = 1 - 1/(omega (omega - i nu))
# on (1 + delta, r_out), vacuum beyond r_out (r_out = inf: unbounded plasma).
# The electrode potential (u/2) sign(cos theta) has Legendre coefficients
# u c_l (odd l); each mode l is an independent radial problem.
# ---------------------------------------------------------------------------

def plasma_permittivity(omega, nu: float = 0.0):
    """Cold plasma with collision rate nu (units of omega_pe)."""
    w = np.asarray(omega, dtype=np.complex128)
    return 1.0 - 1.0 / (w * (w - 1j * nu))


def drive_coefficients(l_max: int) -> np.ndarray:
    """c_l, l = 0..l_max: Legendre coefficients of (1/2) sign(cos theta),
    (1/2)[P_{l-1}(0) - P_{l+1}(0)] for odd l, zero for even l."""
    p0 = np.zeros(l_max + 3)          # P_l(0)
    p0[0] = 1.0
    for l in range(1, l_max + 2):
        p0[l + 1] = -l * p0[l - 1] / (l + 1)
    c = np.zeros(l_max + 1)
    for l in range(1, l_max + 1, 2):
        c[l] = 0.5 * (p0[l - 1] - p0[l + 1])
    return c


def mode_surface_charge(l: int, eps_p, d: float = 0.25, eps_r: float = 4.0,
                        delta: float = 0.0, r_out: float = np.inf) -> np.ndarray:
    """Surface-charge amplitude on the electrode, sigma_l = eps_r E_r(a), of
    the mode l for unit electrode potential P_l(cos theta), as a function of
    the plasma permittivity (array).  Potential and eps dPhi/dr are
    continuous at every interface; the outermost region decays."""
    a = 1.0 - d
    eps_p = np.atleast_1d(np.asarray(eps_p, dtype=np.complex128))
    radii = [1.0] + ([1.0 + delta] if delta > 0 else [])
    if np.isfinite(r_out):
        radii.append(r_out)
    out = np.empty(eps_p.shape, dtype=np.complex128)
    for k, ep in enumerate(eps_p):
        eps = [eps_r] + ([1.0] if delta > 0 else []) + [ep] + ([1.0] if np.isfinite(r_out) else [])
        nreg = len(eps)
        nunk = 2 * nreg - 1          # (r^l, r^-(l+1)) per region, decaying only outside
        M = np.zeros((nunk, nunk), dtype=np.complex128)
        rhs = np.zeros(nunk, dtype=np.complex128)
        M[0, 0], M[0, 1], rhs[0] = a ** l, a ** (-l - 1), 1.0

        def cols(reg):
            return [2 * reg, 2 * reg + 1] if reg < nreg - 1 else [2 * reg]

        def basis(reg, r):
            v = [r ** l, r ** (-l - 1)]
            return v if reg < nreg - 1 else v[1:]

        def dbasis(reg, r):
            v = [l * r ** (l - 1), -(l + 1) * r ** (-l - 2)]
            return v if reg < nreg - 1 else v[1:]

        row = 1
        for i, r in enumerate(radii):
            for c, v in zip(cols(i), basis(i, r)):
                M[row, c] += v
            for c, v in zip(cols(i + 1), basis(i + 1, r)):
                M[row, c] -= v
            for c, v in zip(cols(i), dbasis(i, r)):
                M[row + 1, c] += eps[i] * v
            for c, v in zip(cols(i + 1), dbasis(i + 1, r)):
                M[row + 1, c] -= eps[i + 1] * v
            row += 2
        x = np.linalg.solve(M, rhs)
        out[k] = -eps_r * (l * a ** (l - 1) * x[0] - (l + 1) * a ** (-l - 2) * x[1])
    return out


def _mode_weight(l: int, d: float, c_l: float) -> float:
    """Q_diff = (Q_1 - Q_2)/2 per unit sigma_l for electrode potential
    u c_l P_l: the hemisphere integral of P_l is 2 pi a^2 (2 c_l / (2l+1))."""
    a = 1.0 - d
    return 4.0 * np.pi * a * a * c_l * c_l / (2 * l + 1)


def drude_admittance(omega, delta: float, nu: float, d: float = 0.25, eps_r: float = 4.0,
                     l_max: int = 15, r_out: float = np.inf, vacuum: bool = False) -> np.ndarray:
    """Y(omega) = i omega Q_diff / u of the probe in a cold plasma, by direct
    solution of each radial problem.  vacuum=False leaves out the vacuum
    coupling i omega C_vac (the plasma replaced by vacuum), which the kinetic
    readout of Q_diff does not contain."""
    w = np.asarray(omega, dtype=np.float64)
    c = drive_coefficients(l_max)
    eps_p = plasma_permittivity(w, nu)
    y = np.zeros(w.shape, dtype=np.complex128)
    for l in range(1, l_max + 1, 2):
        s = mode_surface_charge(l, eps_p, d, eps_r, delta, r_out)
        if not vacuum:
            s = s - mode_surface_charge(l, 1.0, d, eps_r, delta, r_out)[0]
        y += 1j * w * _mode_weight(l, d, c[l]) * s.reshape(w.shape)
    return y


@dataclass
class DrudeCircuit:
    """One series resonance circuit of the Drude admittance (Sec. 4): mode l,
    capacitance C_l and resonance eta_l omega_pe."""
    l: int
    capacitance: float
    eta: float


def drude_circuits(delta: float, d: float = 0.25, eps_r: float = 4.0,
                   l_max: int = 15) -> tuple[float, list[DrudeCircuit]]:
    """(C_vac, circuits) of the unbounded-plasma probe.  Each mode's electrode
    charge is a Moebius function (A eps + B)/(eps + P) of the plasma
    permittivity; with eps = 1 - 1/(omega (omega - i nu)) its plasma part is
    the series circuit C_l (1/(i omega) + (i omega + nu)/eta_l^2)^-1 with
    eta_l^2 = 1/(1 + P) and C_l = (A P - B)/(1 + P)."""
    c = drive_coefficients(l_max)
    c_vac = 0.0
    circuits = []
    probe = np.array([0.0, 1.0, 2.0])
    for l in range(1, l_max + 1, 2):
        wgt = _mode_weight(l, d, c[l])
        q0, q1, q2 = (wgt * mode_surface_charge(l, probe, d, eps_r, delta)).real
        # B - P q0 = 0; A + B - P q1 = q1; 2A + B - P q2 = 2 q2
        A_, B_, P_ = np.linalg.solve(np.array([[0.0, 1.0, -q0], [1.0, 1.0, -q1], [2.0, 1.0, -q2]]),
                                     np.array([0.0, q1, 2.0 * q2]))
        c_vac += q1
        circuits.append(DrudeCircuit(l, float((A_ * P_ - B_) / (1.0 + P_)),
                                     float(np.sqrt(1.0 / (1.0 + P_)))))
    return c_vac, circuits


def drude_admittance_circuits(omega, delta: float, nu: float, d: float = 0.25,
                              eps_r: float = 4.0, l_max: int = 15,
                              vacuum: bool = False) -> np.ndarray:
    """The series-circuit form of the Drude admittance (Sec. 4)."""
    w = np.asarray(omega, dtype=np.float64).astype(np.complex128)
    c_vac, circuits = drude_circuits(delta, d, eps_r, l_max)
    y = 1j * w * c_vac if vacuum else np.zeros_like(w)
    for ck in circuits:
        y = y + ck.capacitance / (1.0 / (1j * w) + (1j * w + nu) / ck.eta ** 2)
    return y


@dataclass
class DrudeMatch:
    delta: float
    nu: float
    residual: float


def match_drude(omega, y_kin, d: float = 0.25, eps_r: float = 4.0, l_max: int = 15,
                r_out: float = np.inf, w_max: float = 1.0,
                start: tuple[float, float] = (0.3, 0.1)) -> DrudeMatch:
    """Least-squares match of the Drude admittance to a kinetic one (Sec. 4):
    minimise the integral over 0 < omega < w_max of (Re Y_Drude(delta, nu) -
    Re Y_kin)^2 over the sheath thickness delta and the collision rate nu."""
    from scipy.optimize import least_squares

    w = np.asarray(omega, dtype=np.float64)
    y = np.asarray(y_kin)
    m = (w > 0) & (w <= w_max)
    w, y = w[m], y[m].real
    dw = np.gradient(w)

    def res(p):
        return (drude_admittance(w, p[0], p[1], d, eps_r, l_max, r_out).real - y) * np.sqrt(dw)

    sol = least_squares(res, np.array(start, dtype=np.float64), bounds=([0.0, 0.0], [5.0, 2.0]),
                        x_scale=[0.1, 0.05])
    return DrudeMatch(float(sol.x[0]), float(sol.x[1]), float(2.0 * sol.cost))


def k_coefficient(nu_eff: float, debye_over_r: float) -> float:
    """K of nu_eff = K v_th / R = K lambda_D omega_pe / R (Sec. 4), with nu_eff
    in units of omega_pe."""
    return nu_eff / debye_over_r
