"""Pins of the oracle against closed-form physics and the paper's printed
numbers: shear-wave viscosity (Sec. 4.1, Table 1), acoustic damping
(Sec. 4.3), isentropic sound speed (Sec. 2.5 and 5.1), thermal diffusion
(Sec. 2.1 entropy equation), the viscous heat (energy balance), the convected
isentropic vortex (Sec. 4.2), the Sod shock tube (Sec. 5.2) and the
Rankine-Hugoniot states of a normal shock."""
import json
import math
import os

import numpy as np
import pytest

import hlbm_inputs as hi
import oracle
import riemann_exact

CS2 = 1.0 / 3.0
HERE = os.path.dirname(os.path.abspath(__file__))


def mode_amp_phase(field, axis):
    """Amplitude and phase of the first Fourier mode of a quasi-1D field."""
    prof = field.mean(axis=1) if axis == "y" else field.mean(axis=0)
    n = prof.size
    z = np.sum(prof * np.exp(-2j * np.pi * np.arange(n) / n)) * 2 / n
    return abs(z), np.angle(z)


def fit_decay(ts, amps, skip=2):
    ts = np.asarray(ts, dtype=np.float64)
    la = np.log(np.asarray(amps))
    return -np.polyfit(ts[skip:], la[skip:], 1)[0]


def run_series(S, nsteps, every, fn):
    ts, vals = [], []
    for _ in range(nsteps // every + 1):
        ts.append(S.steps)
        vals.append(fn(S.moments()))
        S.step(every)
    return ts, vals


# ---------------------------------------------------------------- shear wave
with open(os.path.join(HERE, "golden", "table1_shear_viscosity.json")) as fh:
    TABLE1 = json.load(fh)["entries"]


@pytest.mark.parametrize("entry", TABLE1, ids=lambda e: f"nu{e['nu_phys']}-Ma{e['mach']}")
def test_shear_wave_viscosity_table1(entry):
    """Decay rate of max u_x gives nu (Eq. Shearwave); the fitted relative
    error reproduces the paper's Table 1 (present model) within 10 %, and the
    measured nu is within 0.2 % of the input.  The amplitude is 1 % of the
    sound speed (linear regime); the paper's fit window is not stated and at
    its 20 m/s amplitude the fitted error drifts by ~10 % with the window."""
    n, theta, nu = 200, 0.375, entry["nu_lat"]
    c = hi.sound_speed(1.4, theta)
    r, u, v, t = hi.shear_wave(n, 0.01 * c, entry["mach"] * c, theta)
    S = oracle.OracleSolver(oracle.OracleParams(2, n, mu=nu, sigma=0.0), r, u, v, theta=t)
    ts, amps = run_series(S, 2000, 50, lambda m: mode_amp_phase(m["ux"], "y")[0])
    k = 2 * np.pi / n
    rel = fit_decay(ts, amps) / k ** 2 / nu - 1.0
    assert abs(rel) < 2e-3
    assert rel == pytest.approx(entry["rel_err"], rel=0.10)


def test_shear_wave_second_order_convergence():
    """The viscosity error falls ~4x when the resolution doubles."""
    errs = []
    for n in (32, 64):
        theta, nu = 0.375, 0.02
        r, u, v, t = hi.shear_wave(n, 0.004, 0.2, theta)
        S = oracle.OracleSolver(oracle.OracleParams(2, n, mu=nu), r, u, v, theta=t)
        ts, amps = run_series(S, int(300 * (n / 32) ** 2), 20,
                              lambda m: mode_amp_phase(m["ux"], "y")[0])
        errs.append(abs(fit_decay(ts, amps) / (2 * np.pi / n) ** 2 / nu - 1))
    assert 3.0 < errs[0] / errs[1] < 5.0


# ----------------------------------------------------------- acoustic damping
def acoustic_rate(gamma, n=128, steps=12000, every=200, **kw):
    theta, nu, pr = hi.THETA_PAPER, 0.0150654, 0.71
    r, u, v, t = hi.acoustic_wave(n, 5e-5, gamma, theta)
    P = oracle.OracleParams(n, 2, gamma=gamma, mu=nu, sigma=0.95, prandtl=pr, **kw)
    S = oracle.OracleSolver(P, r, u, v, theta=t)
    ts, amps = run_series(S, steps, every,
                          lambda m: mode_amp_phase(m["rho"] * CS2 * m["theta"], "x")[0])
    k = 2 * np.pi / n
    alpha_th = 0.5 * nu + 0.5 * (gamma - 1) * nu / pr   # Eq. (coef acoustic wave decay)
    return fit_decay(ts, amps) / k ** 2, alpha_th, nu


@pytest.mark.parametrize("gamma", [1.4, 2.0])
def test_acoustic_damping_rate(gamma):
    """Pressure amplitude decays at alpha k^2 with
    alpha = (D-1)/D nu + (gamma-1)/2 nu/Pr: zero bulk viscosity thanks to E2,
    and lambda = mu c_p / Pr (Sec. 4.3).  128 points per wavelength."""
    alpha, alpha_th, _ = acoustic_rate(gamma)
    assert alpha / alpha_th == pytest.approx(1.0, abs=0.04)


def test_acoustic_damping_without_e2_has_bulk_viscosity():
    """Dropping E2 (original model) adds the spurious bulk viscosity
    mu (2 - gamma) of a monatomic lattice at gamma = 1.4 (Sec. 3.2, 4.3)."""
    a_on, _, nu = acoustic_rate(1.4)
    a_off, _, _ = acoustic_rate(1.4, e2_off=True)
    excess = (a_off - a_on) / nu
    assert excess == pytest.approx((2.0 - 1.4) / 2.0, rel=0.15)


# ------------------------------------------------------------ speed of sound
@pytest.mark.parametrize("gamma,theta", [(1.1, 0.2), (1.4, hi.THETA_PAPER), (1.7, 0.15),
                                         (2.0, 0.1), (1.4, 0.08)])
def test_speed_of_sound(gamma, theta):
    """A right-running sound wave travels at c = sqrt(gamma c_s^2 theta)
    (Eq. speed of sound), for several gamma and temperatures (Sec. 5.1)."""
    n = 200
    r, u, v, t = hi.acoustic_wave(n, 1e-5, gamma, theta)
    S = oracle.OracleSolver(oracle.OracleParams(n, 2, gamma=gamma, mu=2e-3, sigma=0.95),
                            r, u, v, theta=t)
    ts, ph = run_series(S, 1200, 100, lambda m: mode_amp_phase(m["rho"], "x")[1])
    ph = np.unwrap(ph)
    speed = -np.polyfit(ts, ph, 1)[0] / (2 * np.pi / n)
    assert speed == pytest.approx(hi.sound_speed(gamma, theta), rel=5e-3)


# ---------------------------------------------------------- thermal diffusion
def test_isobaric_entropy_wave_diffusion():
    """An isobaric temperature wave decays at kappa k^2 with
    kappa = lambda / (rho c_p) = nu / Pr (Fourier term of the entropy
    equation with lambda = mu c_p / Pr)."""
    n, nu, pr = 64, 0.05, 0.71
    r, u, v, t = hi.entropy_wave(n, 1e-3, 0.2)
    S = oracle.OracleSolver(oracle.OracleParams(n, 2, mu=nu, prandtl=pr, sigma=0.5),
                            r, u, v, theta=t)
    ts, amps = run_series(S, 1500, 50, lambda m: mode_amp_phase(m["theta"], "x")[0])
    kappa = fit_decay(ts, amps, skip=4) / (2 * np.pi / n) ** 2
    assert kappa == pytest.approx(nu / pr, rel=0.02)


def test_entropy_wave_advection_speed_and_bounds():
    """An isobaric entropy spot advected by a uniform stream moves at the
    stream speed (MUSCL upwinding) and creates no new extrema (van Albada)."""
    n = 80
    X = np.arange(n)
    theta = 0.2 * (1 + 0.05 * ((X > 20) & (X < 40)))[None, :].repeat(2, 0)
    rho = 0.2 / theta
    u = np.full_like(rho, 0.1)
    S = oracle.OracleSolver(oracle.OracleParams(n, 2, mu=1e-6, sigma=0.0), rho, u,
                            np.zeros_like(rho), theta=theta)
    s0 = S.moments()["s"]
    S.step(200)
    s1 = S.moments()["s"]
    span = s0.max() - s0.min()
    assert s1.max() <= s0.max() + 1e-3 * span
    assert s1.min() >= s0.min() - 1e-3 * span
    w0 = s0.mean(0) - s0.min()
    w1 = s1.mean(0) - s0.min()
    c0 = (w0 * X).sum() / w0.sum()
    c1 = (w1 * X).sum() / w1.sum()
    assert c1 - c0 == pytest.approx(0.1 * 200, abs=0.5)


# ----------------------------------------------------------------- viscous heat
@pytest.mark.parametrize("sigma,phi_mode", [(0.0, "lbm"), (0.9, "lbm"), (0.9, "fd")])
def test_viscous_heat_balances_kinetic_energy(sigma, phi_mode):
    """In a decaying periodic shear wave the kinetic energy lost equals the
    internal energy gained: total energy sum(rho c_v theta + rho u^2/2) stays
    constant to a few percent of the dissipated amount only if Phi is right
    (Eq. viscous heat / viscous heat discret)."""
    n, theta, nu = 64, 0.3, 0.02
    r, u, v, t = hi.shear_wave(n, 0.05, 0.0, theta)
    S = oracle.OracleSolver(oracle.OracleParams(2, n, mu=nu, sigma=sigma, phi_mode=phi_mode),
                            r, u, v, theta=t)
    e0 = S.totals()[3]
    m0 = S.moments()
    ke0 = 0.5 * (m0["rho"] * (m0["ux"] ** 2 + m0["uy"] ** 2)).sum()
    S.step(800)
    m1 = S.moments()
    ke1 = 0.5 * (m1["rho"] * (m1["ux"] ** 2 + m1["uy"] ** 2)).sum()
    e1 = S.totals()[3]
    dissipated = ke0 - ke1
    assert dissipated > 0.2 * ke0
    assert abs(e1 - e0) < 0.03 * dissipated


# ----------------------------------------------------------- isentropic vortex
def vortex_centre(rho, rho_inf):
    w = np.clip(rho_inf - rho, 0, None)
    ny, nx = rho.shape
    ys, xs = np.mgrid[0:ny, 0:nx]
    # centroid in a window around the minimum
    j, i = np.unravel_index(np.argmin(rho), rho.shape)
    win = (np.abs(xs - i) <= 12) & (np.abs(ys - j) <= 12)
    return (w * xs * win).sum() / (w * win).sum(), (w * ys * win).sum() / (w * win).sum()


@pytest.mark.parametrize("mach", [0.5, 1.3])
def test_isentropic_vortex_convects(mach):
    """The isentropic vortex is an exact Euler solution that translates at
    u_inf (Sec. 4.2): centre drift within 0.3 cell of u_inf t, and the density
    dip keeps its depth within 8 % (viscous spreading and numerical
    dissipation at R = 8 cells); the present model is stable at Ma 1.3."""
    n, R, steps, x0 = 96, 8.0, 100, 24.0
    r, u, v, t = hi.vortex(n, n, x0, 48, R, mach, 0.1 * mach if mach > 1 else 0.25)
    S = oracle.OracleSolver(oracle.OracleParams(n, n, mu=1e-3, sigma=0.0), r, u, v, theta=t)
    c0 = vortex_centre(r, 1.0)
    dip0 = 1.0 - r.min()
    S.step(steps)
    m = S.moments()
    assert np.isfinite(m["rho"]).all()
    c1 = vortex_centre(m["rho"], 1.0)
    u_inf = mach * hi.sound_speed(1.4, hi.THETA_PAPER)
    assert c1[0] - c0[0] == pytest.approx(u_inf * steps, abs=0.3)
    assert c1[1] - c0[1] == pytest.approx(0.0, abs=0.3)
    assert (1.0 - m["rho"].min()) == pytest.approx(dip0, rel=0.08)


# ---------------------------------------------------------------- shock tube
def test_sod_shock_tube_matches_exact_riemann():
    """Sod (rho, u, p) = (1, 0, 1) | (0.125, 0, 0.1): plateau pressure and
    velocity within 2 %, shock and contact positions within 3 % of the
    distance travelled (Sec. 5.2; the paper notes a small temperature deficit
    between contact and shock from the non-conservative energy equation)."""
    nx, steps, ts = 600, 500, 0.2
    r, u, v, t = hi.sod(nx, 2, theta_scale=ts)
    S = oracle.OracleSolver(oracle.OracleParams(nx, 2, mu=1e-3, sigma=0.4, phi_mode="fd",
                                                bc_x="extrapolate"), r, u, v, theta=t)
    S.step(steps)
    m = S.moments()
    vs = math.sqrt(ts * CS2)             # lattice units of normalised velocity
    rho = m["rho"].mean(0)
    uu = m["ux"].mean(0) / vs
    p = (m["rho"] * m["theta"]).mean(0) / ts   # normalised p = rho T
    tn = steps * vs                           # normalised time (cells)
    xi = (np.arange(nx) + 0.0 - nx // 2) / tn
    L, R_ = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    gamma = 1.4
    pstar, ustar = riemann_exact.star_state(L, R_, gamma)
    head, contact, shock = riemann_exact.wave_speeds(L, R_, gamma)
    # plateau between the rarefaction tail and the shock (away from the fronts)
    sel = (xi > 0.2 * contact) & (xi < 0.85 * shock)
    assert np.median(p[sel]) == pytest.approx(pstar, rel=0.02)
    assert np.median(uu[sel]) == pytest.approx(ustar, rel=0.02)
    # shock: where density crosses halfway between post-shock and right state
    rs, _, _ = riemann_exact.sample(L, R_, gamma, np.array([0.5 * (contact + shock)]))
    mid = 0.5 * (rs[0] + 0.125)
    x_shock = np.where(rho > mid)[0].max() - nx // 2
    assert x_shock / tn == pytest.approx(shock, rel=0.03)
    exact = riemann_exact.sample(L, R_, gamma, xi)
    far = np.abs(xi - contact) > 0.15  # away from the smeared contact
    l1 = np.abs(rho - exact[0])[far].mean()
    assert l1 < 0.02


def test_normal_shock_jump_conditions():
    """A Mach-2 normal shock started from Rankine-Hugoniot states (extrapolation
    inflow/outflow in x).  Mass and momentum are conserved by the lattice
    part, so in the frame of the (slowly drifting) shock the mass and momentum
    fluxes match across it within 1.5 %.  The entropy equation is not in
    conservation form, so the post-shock temperature is low (the defect the
    paper reports for its shock tube, Sec. 5.2); at Mach 2 the oracle gives a
    deficit of about 9 % (density about 8 % high), asserted below 13 %."""
    nx, ny = 240, 2
    r, u, v, t = hi.normal_shock(nx, ny, mach=2.0, theta1=0.1, perturb=0.0)
    S = oracle.OracleSolver(oracle.OracleParams(nx, ny, mu=1e-3, sigma=0.0, phi_mode="fd",
                                                bc_x="extrapolate"), r, u, v, theta=t)

    def front(m):
        """Sub-cell position of the first crossing of the mid density."""
        rho = m["rho"].mean(0)
        mid = 0.5 * (1.0 + 8.0 / 3.0)
        j = int(np.argmax(rho > mid))
        return j - 1 + (mid - rho[j - 1]) / (rho[j] - rho[j - 1])

    S.step(200)
    m0 = S.moments()
    x0 = front(m0)
    S.step(600)
    m = S.moments()
    assert np.isfinite(m["rho"]).all()
    speed = (front(m) - x0) / 600.0
    xs = int(front(m))
    up = slice(5, xs - 40)
    down = slice(xs + 15, nx - 10)
    rho1, rho2 = m["rho"][:, up].mean(), m["rho"][:, down].mean()
    u1, u2 = m["ux"][:, up].mean(), m["ux"][:, down].mean()
    p = m["rho"] * CS2 * m["theta"]
    p1, p2 = p[:, up].mean(), p[:, down].mean()
    w1, w2 = u1 - speed, u2 - speed
    assert rho2 * w2 == pytest.approx(rho1 * w1, rel=0.015)
    assert rho2 * w2 * w2 + p2 == pytest.approx(rho1 * w1 * w1 + p1, rel=0.015)
    ex = hi.rankine_hugoniot(2.0)
    t_ratio = m["theta"][:, down].mean() / m["theta"][:, up].mean()
    assert 0.87 * ex[3] < t_ratio < ex[3]


@pytest.mark.parametrize("mach", [1.0, 1.5])
def test_original_model_diverges_present_model_stable(mach):
    """Table 1: the original model (centred E1) diverges for Ma >= 1 in the
    shear-wave case while the present model (upwind E1) stays stable."""
    n, theta, nu = 200, 0.375, 0.0240918
    c = hi.sound_speed(1.4, theta)
    fields = hi.shear_wave(n, 0.0240918, mach * c, theta)

    def survives(**kw):
        S = oracle.OracleSolver(oracle.OracleParams(2, n, mu=nu, sigma=0.0, **kw), *fields[:3],
                                theta=fields[3])
        for _ in range(8):
            S.step(200)
            m = S.moments()
            if not np.isfinite(m["rho"]).all() or np.abs(m["ux"]).max() > 1.0:
                return False
        return True

    assert survives()
    assert not survives(e1_centred=True, e2_off=True, feq_order=3)


def test_acoustic_pulse_reference_closed_form_checks():
    """The 2-D pulse reference: at t = 0 it is the Gaussian itself; for
    large t the front travels at c (peak of r^(1/2) p' near r = c t); its
    space integral (the monopole) stays eps pi / alpha."""
    from acoustics_exact import pulse_pressure
    alpha, c = 1.0 / (2 * 6.0 ** 2), 0.3
    r = np.linspace(0, 60, 301)
    np.testing.assert_allclose(pulse_pressure(r, 0.0, c, alpha), np.exp(-alpha * r * r), atol=1e-6)
    t = 150.0
    p = pulse_pressure(r, t, c, alpha)
    rp = r[np.argmax(np.sqrt(r) * np.abs(p))]
    assert abs(rp - c * t) < 6.0
    rr = np.linspace(0, 200, 4001)
    integral = np.trapezoid(2 * np.pi * rr * pulse_pressure(rr, 60.0, c, alpha), rr)
    assert integral == pytest.approx(np.pi / alpha, rel=1e-3)


def test_paper_shock_tube_3to1():
    """The shock tube of Sec. 5.2: (3 rho, 0, 3 p) | (rho, 0, p) at one
    temperature, 401 x 2 points over 1 m, mu = 1e-5 kg/(m s) (3.03e-6 in
    lattice units), sigma 0.4, T_r = 1460 K, extrapolated ends.  The paper
    plots the profiles at an unstated time; here 400 steps (0.89 ms), before
    any wave reaches an end.  Against the exact Riemann solution: pressure
    and velocity of the star region within 1 %, shock within 2 cells of its
    exact position.  Between the contact and the shock the temperature is
    slightly low, as the paper reports and attributes to the non-conservative
    entropy equation: the oracle's deficit there is about 0.5 %, asserted to
    be a deficit (below the exact value) of less than 2 %."""
    nx, ny, steps = 401, 2, 400
    r, u, v, t = hi.paper_shock_tube(nx, ny)
    mu = hi.paper_tube_mu(nx)
    assert mu == pytest.approx(3.0324e-6, rel=1e-4)
    S = oracle.OracleSolver(oracle.OracleParams(nx, ny, mu=mu, sigma=0.4, phi_mode="fd",
                                                bc_x="extrapolate"), r, u, v, theta=t)
    S.step(steps)
    m = S.moments()
    assert np.isfinite(m["rho"]).all()
    p_inf = CS2 * t[0, 0]
    L, R_ = (3.0, 0.0, 3.0 * p_inf), (1.0, 0.0, p_inf)
    gamma = 1.4
    pstar, ustar = riemann_exact.star_state(L, R_, gamma)
    head, contact, shock = riemann_exact.wave_speeds(L, R_, gamma)
    # the split lies half-way between nodes 199 and 200
    xi = (np.arange(nx) - 199.5) / steps
    rho = m["rho"].mean(0)
    p = (m["rho"] * CS2 * m["theta"]).mean(0)
    ux = m["ux"].mean(0)
    th = m["theta"].mean(0)
    # the star region between the rarefaction tail and the shock
    rho_l, u_l, p_l = riemann_exact.sample(L, R_, gamma, np.array([0.5 * contact]))
    tail = ustar - math.sqrt(gamma * pstar / rho_l[0])
    star = (xi > tail + 0.2 * (contact - tail)) & (xi < shock - 0.2 * (shock - contact))
    assert np.median(p[star]) == pytest.approx(pstar, rel=0.01)
    assert np.median(ux[star]) == pytest.approx(ustar, rel=0.01)
    # shock position: last node above the mid density of the jump
    rs, _, _ = riemann_exact.sample(L, R_, gamma, np.array([0.5 * (contact + shock)]))
    mid = 0.5 * (rs[0] + 1.0)
    x_shock = np.where(rho > mid)[0].max() + 0.5 - 199.5
    assert x_shock == pytest.approx(shock * steps, abs=2.0)
    # temperature between contact and shock
    band = (xi > contact + 0.2 * (shock - contact)) & (xi < shock - 0.2 * (shock - contact))
    t_exact = pstar / (rs[0] * CS2)   # theta = p / (rho c_s^2)
    deficit = float(np.median(th[band]) / t_exact - 1.0)
    print(f"paper shock tube: p*/exact {np.median(p[star]) / pstar:.4f}, "
          f"u*/exact {np.median(ux[star]) / ustar:.4f}, T deficit {deficit:+.4f}")
    assert -0.02 < deficit < 0.0
