"""The floating probe-plasma equilibrium of App. D (initial condition), and
the oracle's ion field for a radial ion profile."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2111_13072_amd import equilibrium as EQ

LAM_3EV = 0.10179   # lambda_D / R at 3 eV, 1e15 m^-3, R = 4 mm


@pytest.fixture(scope="module")
def eq():
    return EQ.solve_floating_equilibrium(LAM_3EV)


def test_floating_condition(eq):
    """Hertz-Langmuir: R^2 sqrt(T_e/m_i) = sqrt(T_e/(2 pi m_e)) exp(psi(1))."""
    c = math.sqrt(eq.mass_ratio / (2 * math.pi))
    assert eq.psi_probe == pytest.approx(math.log(eq.r_hat ** 2 / c), abs=1e-8)
    assert eq.psi_probe < -3.0 and eq.surface_charge < 0


def test_poisson_equation_holds(eq):
    """Finite differences of the solution satisfy
    -Lambda^2 (psi'' + 2 psi'/r) = n_i - n_e."""
    r = np.linspace(1.05, eq.r_start - 0.05, 60)
    h = 1e-3
    p0, pp, pm = eq.psi(r), eq.psi(r + h), eq.psi(r - h)
    lap = (pp - 2 * p0 + pm) / h ** 2 + (pp - pm) / (h * r)
    res = -eq.debye ** 2 * lap - (eq.n_i(r) - eq.n_e(r))
    assert np.max(np.abs(res)) < 2e-5


def test_gauss_law_balances_the_probe_charge(eq):
    """Q_S + 4 pi int_1^R (n_i - n_e) r^2 dr = -4 pi Lambda^2 R^2 psi'(R)."""
    for R in (1.5, 3.0, eq.r_start - 1e-9):
        r = np.linspace(1.0, R, 200001)
        q = eq.surface_charge + 4 * np.pi * np.trapezoid((eq.n_i(r) - eq.n_e(r)) * r * r, r)
        h = 1e-4
        dpsi = (eq.psi(R) - eq.psi(R - h)) / h
        flux = -4 * np.pi * eq.debye ** 2 * R ** 2 * dpsi
        assert q == pytest.approx(flux, abs=2e-4 * abs(eq.surface_charge))


def test_quasi_neutral_far_away(eq):
    """Beyond the sheath the plasma is neutral to the Poisson correction."""
    r = np.array([4.0, 6.0, 8.0, eq.r_start * 0.999])
    ni, ne = eq.n_i(r), eq.n_e(r)
    assert np.max(np.abs(ni - ne)) < 1e-3
    qn = np.array([EQ.quasi_neutral_psi(x, eq.r_hat) for x in r])
    assert np.max(np.abs(eq.psi(r) - qn)) < 1e-4 * np.max(np.abs(qn)) + 1e-9
    # sheath: electron-depleted at the probe, ions at most at the Bohm-limited density
    assert eq.n_e(np.array([1.0]))[0] < 0.05 < eq.n_i(np.array([1.0]))[0] < 1.0


def test_thin_sheath_limit():
    """Lambda -> 0: the sheath is thin and planar, the ion flux at the probe
    is the Bohm flux n_inf exp(-1/2) c_s, so R^ -> exp(-1/4) from above and
    psi(1) -> -1/2 - ln sqrt(m_i / (2 pi m_e))."""
    rh = [EQ.solve_floating_equilibrium(lam).r_hat for lam in (0.05, 0.02)]
    lim = math.exp(-0.25)
    assert rh[0] > rh[1] > lim
    assert (rh[1] - lim) < 0.6 * (rh[0] - lim)


def test_sampled_electrons_follow_the_density(eq):
    st = EQ.sample_electrons(eq, 200_000, 3, 10.0, 0.1)
    r = np.linalg.norm(st.pos, axis=1)
    assert np.all((r > 1.0) & (r < 10.0))
    edges = np.linspace(1.0, 10.0, 19)
    hist, _ = np.histogram(r, edges)
    rg = np.linspace(1.0, 10.0, 90001)
    w = eq.n_e(rg) * rg ** 2
    expect = np.array([np.trapezoid(w[(rg >= a) & (rg <= b)], rg[(rg >= a) & (rg <= b)])
                       for a, b in zip(edges[:-1], edges[1:])])
    expect *= len(r) / expect.sum()
    assert np.all(np.abs(hist - expect) < 5 * np.sqrt(expect) + 5)
    assert np.std(st.vel) == pytest.approx(0.1, rel=0.01)
    assert abs(np.mean(st.pos[:, 2] / r)) < 0.01


def test_oracle_ion_field_of_a_profile(eq):
    """Gauss's law and E = -dPhi/dr for the piecewise-linear profile, against
    a fine trapezoid of the linear interpolant; a constant profile gives the
    uniform background's closed form."""
    r_out = 10.0
    prof = eq.ion_profile(r_out, 257)
    p = O.Params(r_out=r_out, ion_profile=prof)
    nodes = np.linspace(1.0, r_out, prof.size)
    for r in (1.0, 1.2345, 3.3, 7.77, 9.999):
        s = np.linspace(1.0, r, 400001)
        q = np.trapezoid(np.interp(s, nodes, prof) * s * s, s)
        e, _ = O.ion_field(p, r)
        assert e * r * r == pytest.approx(q, rel=1e-8, abs=1e-14)
        h = 1e-5
        if 1.0 + h < r < r_out - h:
            dphi = (O.ion_field(p, r + h)[1] - O.ion_field(p, r - h)[1]) / (2 * h)
            assert -dphi == pytest.approx(e, rel=1e-6)
    u = O.Params(r_out=r_out, ion_density=0.7)
    c = O.Params(r_out=r_out, ion_profile=np.full(33, 0.7))
    for r in (1.5, 4.0, 9.0):
        assert O.ion_field(c, r)[0] == pytest.approx(O.ion_field(u, r)[0], rel=1e-14)
        assert O.ion_field(c, r)[1] == pytest.approx(O.ion_field(u, r)[1], rel=1e-14)


def test_sampled_ions_follow_the_density_and_inflow(eq):
    st = EQ.sample_ions(eq, 100_000, 4, 10.0, id_offset=7)
    r = np.linalg.norm(st.pos, axis=1)
    assert np.all((r > 1.0) & (r < 10.0))
    assert np.all(st.ids & np.uint32(0x80000000)) and st.ids[0] & np.uint32(0x7fffffff) == 7
    # radial inflow at sqrt(-2 psi) c_s: energy conservation of App. D
    vr = np.sum(st.vel * st.pos, axis=1) / r
    c_s = eq.debye / math.sqrt(eq.mass_ratio)
    assert np.allclose(0.5 * vr ** 2 / c_s ** 2 + eq.psi(r), 0.0, atol=1e-12)
    assert np.all(vr < 0)
    tang = st.vel - vr[:, None] * st.pos / r[:, None]
    assert np.max(np.abs(tang)) < 1e-12 * np.max(np.abs(st.vel))
    edges = np.linspace(1.0, 10.0, 10)
    hist, _ = np.histogram(r, edges)
    rg = np.linspace(1.0, 10.0, 90001)
    w = eq.n_i(rg) * rg ** 2
    expect = np.array([np.trapezoid(w[(rg >= a) & (rg <= b)], rg[(rg >= a) & (rg <= b)])
                       for a, b in zip(edges[:-1], edges[1:])])
    expect *= len(r) / expect.sum()
    assert np.all(np.abs(hist - expect) < 5 * np.sqrt(expect) + 5)


def test_paper_setup_counts_both_species():
    ps = EQ.PaperSetup(n=20_000)
    eq, st, nt, qs, prof = ps.build()
    ions = (st.ids & np.uint32(0x80000000)) != 0
    assert prof is None and st.pos.shape == (20_000, 3)
    ne, ni = EQ.electron_count_density(eq, 10.0), EQ.ion_count_density(eq, 10.0)
    assert ions.sum() == pytest.approx(20_000 * ni / (ne + ni), abs=1)
    assert nt == pytest.approx(20_000 / (ne + ni))
    assert len(np.unique(st.ids)) == 20_000
    # net charge of the probe plus the plasma between the walls ~ 0 (the
    # quasi-neutral tail beyond r_out carries the rest)
    assert abs(qs + (ions.sum() - (~ions).sum())) < 0.01 * ions.sum()
