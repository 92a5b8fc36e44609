"""Walls of the oracle pinned by the thermal Couette flow (Sec. 4.4).

Between two walls at the same temperature T_w, one at rest and one moving
along x at U = Ma c_w, the steady flow has the linear velocity U y / H and
the closed-form temperature the paper gives,
    (T - T_w) / T_w = (y/H) Pr Ma^2 (gamma - 1) / 2 (1 - y/H),
the balance of viscous heating mu (U/H)^2 and conduction lambda T'' with
lambda = mu c_p / Pr.  The profile depends on the viscous heat production,
the heat conductivity (so on Pr and on c_p, so on gamma) and on the walls'
velocity and temperature; a dropped or mis-signed term in any of them moves
it.  Each case starts from the steady velocity at uniform T_w on a 2 x 32
channel and runs until the slowest thermal mode has decayed.
"""
import numpy as np
import pytest

import hlbm_inputs as hi
import oracle


def closed_form_rise(eta, ma, pr, gamma):
    return eta * pr * ma * ma * (gamma - 1.0) / 2.0 * (1.0 - eta)


def run_couette(ny=32, nu=0.1, steps=8000, gamma=1.4, pr=0.71, ma=0.8, thw=0.2, sigma=0.9,
                phi="lbm", u_lo=0.0):
    H = ny - 1
    U = ma * hi.sound_speed(gamma, thw)
    eta = np.arange(ny) / H
    ones = np.ones((ny, 2))
    p = oracle.OracleParams(2, ny, gamma=gamma, prandtl=pr, mu=nu, sigma=sigma, bc_y="wall",
                            wall_ux_lo=u_lo, wall_ux_hi=u_lo + U, wall_theta=thw, phi_mode=phi)
    S = oracle.OracleSolver(p, ones, (u_lo + U * eta)[:, None] * ones, 0 * ones,
                            theta=thw * ones)
    S.step(steps)
    m = S.moments()
    rise = closed_form_rise(eta, ma, pr, gamma)
    t_err = np.abs(m["theta"][:, 0] - thw * (1 + rise)).max() / (thw * rise.max())
    u_err = np.abs(m["ux"][:, 0] - (u_lo + U * eta)).max() / U
    return t_err, u_err, m


@pytest.mark.parametrize("case", [
    dict(),                                   # Ma 0.8, Pr 0.71, gamma 1.4, sigma 0.9
    dict(ma=0.3), dict(ma=1.2),               # rise ~ Ma^2
    dict(pr=2.0, steps=16000),                # rise ~ Pr, slower conduction
    dict(gamma=5.0 / 3.0), dict(gamma=1.1),   # rise ~ gamma - 1
    dict(sigma=0.0), dict(phi="fd"),          # stress from FD only; Phi by FD
])
def test_couette_closed_form(case):
    t_err, u_err, m = run_couette(**case)
    assert t_err < 1e-4, t_err
    assert u_err < 1e-5, u_err
    assert np.abs(m["uy"]).max() < 1e-7


def test_couette_galilean_wall_speeds():
    """Both walls shifted by the same speed: the same temperature rise."""
    t_err, u_err, _ = run_couette(u_lo=-0.1, ma=0.6)
    assert t_err < 1e-4, t_err
    assert u_err < 1e-5, u_err


def test_walls_hold_their_values():
    """After any step the wall rows carry exactly the wall velocity and
    temperature, and a fluid at rest at T_w between walls at rest stays so."""
    ny, thw = 12, 0.25
    rng = np.random.default_rng(3)
    r = 1.0 + 0.01 * rng.standard_normal((ny, 6))
    u = 0.02 * rng.standard_normal((ny, 6))
    v = 0.02 * rng.standard_normal((ny, 6))
    p = oracle.OracleParams(6, ny, mu=0.05, sigma=0.5, bc_y="wall", wall_ux_lo=0.03,
                            wall_ux_hi=-0.07, wall_theta=thw)
    S = oracle.OracleSolver(p, r, u, v, theta=thw * np.ones((ny, 6)))
    S.step(7)
    m = S.moments()
    np.testing.assert_allclose(m["ux"][0], 0.03, rtol=0, atol=1e-14)
    np.testing.assert_allclose(m["ux"][-1], -0.07, rtol=0, atol=1e-14)
    np.testing.assert_allclose(m["uy"][[0, -1]], 0.0, rtol=0, atol=1e-14)
    np.testing.assert_allclose(m["theta"][[0, -1]], thw, rtol=1e-13)

    ones = np.ones((ny, 6))
    p0 = oracle.OracleParams(6, ny, mu=0.05, sigma=0.5, bc_y="wall", wall_theta=thw)
    R = oracle.OracleSolver(p0, ones, 0 * ones, 0 * ones, theta=thw * ones)
    R.step(20)
    m = R.moments()
    np.testing.assert_allclose(m["rho"], 1.0, rtol=1e-14)
    np.testing.assert_allclose(m["theta"], thw, rtol=1e-14)
    assert np.abs(m["ux"]).max() < 1e-15 and np.abs(m["uy"]).max() < 1e-15


def test_wall_parameters_validated():
    for bad in (dict(ny=3), dict(wall_theta=0.0)):
        kw = dict(nx=2, ny=8, bc_y="wall", wall_theta=0.2)
        kw.update(bad)
        with pytest.raises(ValueError):
            oracle.OracleSolver(oracle.OracleParams(**kw), np.ones((kw["ny"], 2)),
                                np.zeros((kw["ny"], 2)), np.zeros((kw["ny"], 2)),
                                theta=0.2 * np.ones((kw["ny"], 2)))


def test_walls_pass_no_mass():
    """A closed channel keeps its mass: an acoustic pulse started next to the
    lower wall reflects between the walls for 300 steps while the total mass
    stays within 1e-5 of its initial value (8 % of the pulse's excess mass;
    the wet-node rebuild is not exactly conservative, the drift oscillates)
    and the wall-normal velocity on the wall rows stays exactly zero.  Taking
    the wall density from the populations that did not come from the
    interior loses about a fifth of the pulse's mass instead."""
    nx, ny, thw = 24, 40, 0.2
    y = np.arange(ny)[:, None]
    rho = 1.0 + 1e-3 * np.exp(-((y - 6) ** 2) / 8.0) * np.ones((1, nx))
    zero = np.zeros((ny, nx))
    p = oracle.OracleParams(nx, ny, mu=0.02, sigma=0.9, bc_y="wall", wall_theta=thw)
    S = oracle.OracleSolver(p, rho, zero, zero, theta=thw * np.ones((ny, nx)))
    m0 = S.totals()[0]
    for n in (30, 150, 300):
        S.step(n - S.steps)
        assert abs(S.totals()[0] / m0 - 1.0) < 1e-5, n
        assert np.all(S.moments()["uy"][[0, -1]] == 0.0)
