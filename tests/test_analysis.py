"""Response analysis (host side): damped-sine fits and the admittance
estimator, pinned against closed-form transforms."""
import numpy as np
import pytest

from paper_2111_13072_amd import analysis as A


def damped(t, a, b, c, ph, t0=0.0):
    tt = np.asarray(t) - t0
    return np.where(tt >= 0, a * np.exp(-b * tt) * np.sin(c * tt + ph), 0.0)


def test_twin_difference():
    assert np.array_equal(A.twin_difference([3.0, 2.0], [1.0, 5.0]), [2.0, -3.0])


def test_single_mode_fit_recovers_parameters():
    t = np.arange(0, 40, 0.05)
    rng = np.random.default_rng(0)
    q = damped(t, 0.3, 0.07, 0.58, 1.1, t0=1.0) + 0.02 + 1e-4 * rng.standard_normal(t.size)
    f = A.fit_damped_sine(t, q, t0=1.0)
    assert f.frequency == pytest.approx(0.58, rel=1e-3)
    assert f.damping == pytest.approx(0.07, rel=1e-2)
    assert f.amplitude == pytest.approx(0.3, rel=1e-2)
    assert f.offset == pytest.approx(0.02, abs=1e-3)
    assert f.fwhm == pytest.approx(0.14, rel=1e-2)
    # the fitted function reproduces the signal
    m = t >= 1.0
    assert np.max(np.abs(f(t[m]) - q[m])) < 1e-3


def test_fit_without_frequency_guess_and_negative_amplitude():
    t = np.arange(0, 60, 0.05)
    q = -damped(t, 1.0, 0.02, 0.36, 0.0)
    f = A.fit_damped_sine(t, q, t0=0.0)
    assert f.amplitude > 0
    assert f.frequency == pytest.approx(0.36, rel=1e-4)
    assert np.max(np.abs(f(t) - q)) < 1e-6


def test_two_mode_fit():
    """The mode expansion of Sec. 4 with two modes (as for l = 1 and l = 3)."""
    t = np.arange(0, 80, 0.05)
    q = damped(t, 0.4, 0.01, 0.362, 0.3) + damped(t, 0.1, 0.03, 0.444, 2.0)
    modes, d = A.fit_damped_sines(t, q, 0.0, [0.35, 0.45])
    assert [m.frequency for m in modes] == pytest.approx([0.362, 0.444], rel=1e-5)
    assert [m.damping for m in modes] == pytest.approx([0.01, 0.03], rel=1e-4)
    assert abs(d) < 1e-8


def exact_re_admittance(w, a, b, c):
    """Closed-form Re Y for q(t) = a e^{-bt} sin(ct) (t >= 0) answering a unit
    impulse: Q^(w) = a c / ((b + i w)^2 + c^2) and Y = i w Q^(w) / u^(w) with
    u^ = 1 (unit area)."""
    return np.real(1j * w * a * c / ((b + 1j * w) ** 2 + c ** 2))


def test_admittance_matches_closed_form_transform():
    dt = 0.05
    a, b, c = 0.4, 0.06, 0.55
    t = np.arange(0, 600, dt)
    q = damped(t, a, b, c, 0.0)
    u = A.np.zeros_like(t)
    u[0] = 1.0 / dt                     # unit-area impulse
    sp = A.admittance(q, u, dt, pad=4, w_max=1.5)
    ref = exact_re_admittance(sp.omega, a, b, c)
    assert np.max(np.abs(sp.admittance.real - ref)) < 2e-3 * np.max(ref)
    # peak and full width at half maximum of the exact curve, on a fine grid
    wf = np.linspace(0.3, 0.8, 200001)
    rf = exact_re_admittance(wf, a, b, c)
    i = np.argmax(rf)
    above = wf[rf >= rf[i] / 2]
    w_pk, fwhm = sp.peak()
    assert w_pk == pytest.approx(wf[i], rel=2e-3)
    assert fwhm == pytest.approx(above[-1] - above[0], rel=1e-2)
    # for b << c the Lorentzian half-width is 2b (the fit's reading)
    assert above[-1] - above[0] == pytest.approx(2 * b, rel=2e-2)


def test_lorentzian_from_fit_half_width():
    f = A.DampedSine(1.0, 0.05, 0.6, 0.0, 0.0, 0.0)
    w = np.array([0.6, 0.55, 0.65])
    s = A.lorentzian_from_fit(f, w)
    assert s[1] == pytest.approx(s[0] / 2) and s[2] == pytest.approx(s[0] / 2)


# --- Drude model of the ideal probe and the temperature formula (Sec. 4) ---

def test_drive_coefficients_match_sign_function_expansion():
    c = A.drive_coefficients(9)
    assert c[[1, 3, 5, 7, 9]] == pytest.approx([0.75, -0.4375, 0.34375, -0.29296875, 0.259765625],
                                               abs=1e-15)
    assert np.all(c[::2] == 0)
    # projection of (1/2) sign(x) on P_l by Gauss-Legendre quadrature on (0, 1)
    from numpy.polynomial import legendre
    xg, wg = legendre.leggauss(64)
    x, wq = 0.5 * (xg + 1), 0.5 * wg
    c = A.drive_coefficients(31)
    for l in range(32):
        pl = legendre.legval(x, np.eye(32)[l])
        proj = (2 * l + 1) / 2 * (1 - (-1) ** l) * 0.5 * np.sum(wq * pl)
        assert c[l] == pytest.approx(proj, abs=1e-13)


@pytest.mark.parametrize("delta", [0.0, 0.3])
def test_series_circuit_form_equals_direct_solution(delta):
    """The paper's circuit form (vacuum coupling + series circuits) is an
    exact rewriting of the cold-fluid electrostatics, for any nu."""
    w = np.linspace(0.01, 1.5, 37)
    for nu in (0.0, 0.05, 0.3):
        for vac in (False, True):
            y1 = A.drude_admittance(w, delta, nu, vacuum=vac)
            y2 = A.drude_admittance_circuits(w, delta, nu, vacuum=vac)
            # nu = 0 puts undamped poles on the grid: conditioning, not error
            assert np.max(np.abs(y1 - y2)) < 1e-10 * np.max(np.abs(y1))


def test_vacuum_sheath_resonances_closed_form():
    """No dielectric (eps_r = 1): a grounded sphere of radius a, vacuum to
    rho = 1 + delta, plasma beyond.  Potential A (r^l - a^{2l+1} r^{-l-1})
    inside, B r^{-l-1} outside; the interface conditions give
    eta_l^2 = (l+1)/(2l+1) (1 - (a/rho)^{2l+1})."""
    a, delta = 0.75, 0.1
    _, circuits = A.drude_circuits(delta, d=1 - a, eps_r=1.0, l_max=9)
    for ck in circuits:
        l = ck.l
        assert ck.eta ** 2 == pytest.approx((l + 1) / (2 * l + 1) * (1 - (a / (1 + delta)) ** (2 * l + 1)),
                                            rel=1e-12)
        assert ck.capacitance > 0


def test_vacuum_capacitance_of_a_bare_sphere():
    """eps_r = 1: the electrode in vacuum carries sigma_l = (l+1) V / a."""
    a = 0.75
    c = A.drive_coefficients(15)
    c_vac, _ = A.drude_circuits(0.2, d=1 - a, eps_r=1.0, l_max=15)
    expect = sum(4 * np.pi * a * a * c[l] ** 2 / (2 * l + 1) * (l + 1) / a for l in range(1, 16, 2))
    assert c_vac == pytest.approx(expect, rel=1e-12)


def test_finite_plasma_shell_resonance_and_unbounded_limit():
    """delta = 0, plasma (1, 5), nu -> 0: Re Y peaks at the inner dipole
    mode of the layered sphere; the unbounded plasma's eta_1 is its
    r_out -> infinity limit."""
    w = np.linspace(0.30, 0.42, 12001)
    y = A.drude_admittance(w, 0.0, 1e-3, r_out=5.0, l_max=1)
    assert w[np.argmax(y.real)] == pytest.approx(0.36193, abs=2e-5)
    _, circuits = A.drude_circuits(0.0, l_max=1)
    assert circuits[0].eta == pytest.approx(0.368146, abs=2e-6)


def test_drude_half_width_is_the_collision_rate():
    """A single series circuit has a Lorentzian Re Y with FWHM = nu."""
    w = np.linspace(0.3, 0.9, 60001)
    y = A.drude_admittance(w, 0.2, 0.02, l_max=1)
    re = y.real
    above = w[re >= re.max() / 2]
    assert above[-1] - above[0] == pytest.approx(0.02, rel=2e-2)


def test_match_recovers_drude_parameters():
    w = np.linspace(0.005, 1.0, 400)
    y = A.drude_admittance(w, 0.45, 0.08)
    m = A.match_drude(w, y, start=(0.2, 0.2))
    assert m.delta == pytest.approx(0.45, rel=1e-4)
    assert m.nu == pytest.approx(0.08, rel=1e-4)


def test_k_coefficient_reproduces_paper_value():
    """Sec. 4 prints nu_eff for T_e = 2, 3, 5 eV at n_e = 1e15 m^-3, R = 4 mm
    and K = 1.264; with lambda_D = sqrt(eps0 T_e / (n_e e^2)) the three K
    average to that value."""
    import os
    from paper_2111_13072_amd import workload as W
    rows = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "paper_nu_eff.txt"))
    ks = [A.k_coefficient(nu, W.PlasmaScales(1e15, te, 0.004).v_th) for te, nu in rows]
    assert np.mean(ks) == pytest.approx(1.264, abs=1e-3)
    assert max(ks) - min(ks) < 0.02


def test_admittance_from_fit_matches_transform_of_the_fit():
    """Closed-form transform of the fitted damped sine against the FFT
    estimator applied to the same function sampled finely."""
    f = A.DampedSine(0.7, 0.05, 0.55, 0.8, 0.0, 0.0)
    dt = 0.01
    t = np.arange(0, 800, dt)
    q = f(t)
    u = np.zeros_like(t)
    u[0] = 1.0 / dt
    num = A.admittance(q, u, dt, pad=2, w_max=1.2)
    ana = A.admittance_from_fit(f, num.omega)
    # the sampled signal starts at q(0) = a sin(phi) != 0: the FFT of samples
    # is the integral to first order in dt
    assert np.max(np.abs(num.admittance - ana.admittance)) < 2e-3 * np.max(np.abs(ana.admittance))


def test_admittance_from_fit_is_independent_of_the_fit_origin():
    """The same function fitted from a later start t0 gives the same Y."""
    t = np.arange(0, 200, 0.02)
    q = damped(t, 0.5, 0.04, 0.6, 0.3)
    w = np.linspace(0.05, 1.2, 50)
    f0 = A.fit_damped_sine(t, q, 0.0, 0.6)
    f1 = A.fit_damped_sine(t, q, 2.5, 0.6)
    y0 = A.admittance_from_fit(f0, w).admittance
    y1 = A.admittance_from_fit(f1, w).admittance
    assert np.max(np.abs(y0 - y1)) < 1e-6 * np.max(np.abs(y0))
