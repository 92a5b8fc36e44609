"""Pins of the exact Riemann solver in tests/riemann_exact.py, which the
oracle's shock-tube tests rely on.

* Sod's problem (rho, u, p) = (1, 0, 1) | (0.125, 0, 0.1), gamma 1.4: the
  star state and wave speeds published in the textbook treatment of the exact
  solver (Toro, Riemann Solvers and Numerical Methods for Fluid Dynamics,
  Ch. 4): p* = 0.30313, u* = 0.92745, rho*_L = 0.42632, rho*_R = 0.26557,
  rarefaction head -1.18322, tail -0.07027, shock 1.75216.
* For any problem: the sampled solution satisfies the Rankine-Hugoniot
  conditions across each shock (mass, momentum and energy fluxes equal in
  the shock frame), is isentropic with a constant Riemann invariant through
  each rarefaction fan, and has continuous pressure and velocity across the
  contact.  These follow from the Euler equations alone, so a mistake in any
  branch of the solver fails one of them.
"""
import math

import numpy as np
import pytest

import riemann_exact as rx

G = 1.4


def test_sod_star_state_and_waves():
    L, R = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    ps, us = rx.star_state(L, R, G)
    assert ps == pytest.approx(0.30313, abs=1e-5)
    assert us == pytest.approx(0.92745, abs=1e-5)
    head, contact, shock = rx.wave_speeds(L, R, G)
    assert head == pytest.approx(-1.18322, abs=1e-5)
    assert contact == pytest.approx(0.92745, abs=1e-5)
    assert shock == pytest.approx(1.75216, abs=1e-5)
    rho, u, p = rx.sample(L, R, G, np.array([0.5, 1.2]))
    assert rho[0] == pytest.approx(0.42632, abs=1e-5)   # left star (between tail and contact)
    assert rho[1] == pytest.approx(0.26557, abs=1e-5)   # right star (contact to shock)
    cs = math.sqrt(G * ps / rho[0])
    assert us - cs == pytest.approx(-0.07027, abs=1e-5)  # rarefaction tail


def _flux(rho, u, p, s):
    """Mass, momentum and energy fluxes in a frame moving at speed s."""
    w = u - s
    e = p / (G - 1.0) + 0.5 * rho * w * w
    return np.array([rho * w, rho * w * w + p, (e + p) * w])


PROBLEMS = [
    ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1)),      # rarefaction | shock
    ((3.0, 0.0, 3.0), (1.0, 0.0, 1.0)),        # the 3:1 tube of Sec. 5.2 (normalised)
    ((1.0, -2.0, 0.4), (1.0, 2.0, 0.4)),       # two rarefactions
    ((1.0, 1.0, 1.0), (1.0, -1.0, 1.0)),       # two shocks
    ((0.5, 0.3, 0.2), (2.0, -0.1, 1.5)),       # shock | rarefaction
]


@pytest.mark.parametrize("L,R", PROBLEMS)
def test_solution_satisfies_the_euler_jump_and_fan_conditions(L, R):
    ps, us = rx.star_state(L, R, G)
    eps = 1e-9
    for side, (rk, uk, pk), sgn in (("L", L, -1.0), ("R", R, 1.0)):
        ck = math.sqrt(G * pk / rk)
        # star density on this side, read just inside the contact
        rho_s, u_s, p_s = rx.sample(L, R, G, np.array([us + sgn * 1e-7]))
        assert u_s[0] == pytest.approx(us, rel=1e-12, abs=1e-12)
        assert p_s[0] == pytest.approx(ps, rel=1e-12)
        if ps > pk:
            # shock: speed from mass conservation, then all three fluxes match
            s = (rho_s[0] * us - rk * uk) / (rho_s[0] - rk)
            f_out = _flux(rk, uk, pk, s)
            f_in = _flux(rho_s[0], us, ps, s)
            np.testing.assert_allclose(f_in, f_out, rtol=1e-10, atol=1e-12)
            # the sampled profile jumps there
            before = rx.sample(L, R, G, np.array([s + sgn * eps]))
            assert before[0][0] == pytest.approx(rk, rel=1e-12)
        else:
            # rarefaction: isentropic, Riemann invariant constant through the fan
            head = uk + sgn * ck
            cs = math.sqrt(G * ps / rho_s[0])
            tail = us + sgn * cs
            assert ps / rho_s[0] ** G == pytest.approx(pk / rk ** G, rel=1e-10)
            inv = lambda r_, u_, p_: u_ - sgn * 2.0 * math.sqrt(G * p_ / r_) / (G - 1.0)  # noqa
            xi = np.linspace(min(head, tail), max(head, tail), 7)[1:-1]
            rr, uu, pp = rx.sample(L, R, G, xi)
            for a, b, c in zip(rr, uu, pp):
                assert inv(a, b, c) == pytest.approx(inv(rk, uk, pk), rel=1e-10, abs=1e-12)
                assert c / a ** G == pytest.approx(pk / rk ** G, rel=1e-10)
            # inside the fan the characteristic through the origin: u + sgn c = xi
            np.testing.assert_allclose(uu + sgn * np.sqrt(G * pp / rr), xi, rtol=1e-10, atol=1e-12)
    # contact: pressure and velocity continuous, the density may jump
    a = rx.sample(L, R, G, np.array([us - 1e-9, us + 1e-9]))
    assert a[1][0] == pytest.approx(a[1][1], rel=1e-12, abs=1e-12)
    assert a[2][0] == pytest.approx(a[2][1], rel=1e-12)
