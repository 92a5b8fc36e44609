"""The rounding band of the upwind E1 sign (Sec. 3.2).

The E1 scheme upwinds by sgn(u_alpha) at the node.  The oracle and the
library take sgn(u) = 0 (the centred difference) inside |u| <= sgn_eps, 1e-12
by default, because the literal sign turns rounding-level velocities of
opposite signs into O(dGamma) differences.  The band must be inert wherever
|u| stays above it: on flows whose velocity components never come within
1e-12 of zero at a node, the oracle at sgn_eps = 0 (the literal sign) and at
1e-12 must agree bitwise.  Two such flows: the supersonic isentropic vortex
of Sec. 4.2 (Ma 1.3) convected obliquely, so both components of the stream
exceed the vortex's own velocity everywhere, and the shear wave of Table 1
at Ma 1.0 with the zeros of its sine half-way between nodes.
"""
import numpy as np
import pytest

import hlbm_inputs as hi
import oracle


def run(params_kw, fields, steps, checkpoints):
    r, u, v, t = fields
    out = {}
    for eps in (0.0, 1e-12):
        S = oracle.OracleSolver(oracle.OracleParams(sgn_eps=eps, **params_kw), r, u, v, theta=t)
        snaps = []
        done = 0
        for c in checkpoints:
            S.step(c - done)
            done = c
            snaps.append(S.state())
        out[eps] = snaps
    return out


def min_speed(F):
    """Smallest |u_x| and |u_y| over the nodes of a population state."""
    cx = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], float)
    cy = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], float)
    rho = F.sum(0)
    ux = np.tensordot(cx, F, 1) / rho
    uy = np.tensordot(cy, F, 1) / rho
    return np.abs(ux).min(), np.abs(uy).min()


def test_literal_sign_equals_band_on_supersonic_vortex():
    n = 96
    f = hi.vortex(n, n, 30, 48, 8, 1.3, 0.13, angle=0.6, periodic_images=True)
    res = run(dict(nx=n, ny=n, mu=1e-3, sigma=0.0), f, 120, [1, 40, 120])
    for k, ((F0, s0), (F1, s1)) in enumerate(zip(res[0.0], res[1e-12])):
        assert min(min_speed(F0)) > 1e-9, k   # far from the band at every checkpoint
        assert np.array_equal(F0, F1) and np.array_equal(s0, s1), k


@pytest.mark.parametrize("axis", ["y", "x"])
def test_literal_sign_equals_band_on_table1_shear_wave(axis):
    n, theta, nu, a0 = 200, 0.375, 0.0240918, 0.0240918
    c = hi.sound_speed(1.4, theta)
    f = hi.shear_wave(n, a0, 1.0 * c, theta, axis=axis, shift=0.5)
    nx, ny = (2, n) if axis == "y" else (n, 2)
    res = run(dict(nx=nx, ny=ny, mu=nu, sigma=0.0), f, 300, [1, 100, 300])
    for k, ((F0, s0), (F1, s1)) in enumerate(zip(res[0.0], res[1e-12])):
        assert max(min_speed(F0)) > 1e-9, k   # the convecting component never nears zero
        assert np.array_equal(F0, F1) and np.array_equal(s0, s1), k


def test_band_decides_at_an_exact_zero():
    """Where a velocity component is exactly zero both settings take the
    centred difference (sgn(0) = 0), so a quasi-1D flow along x, whose u_y
    is exactly zero everywhere, gives the same result too; a velocity of 1e-13
    inside the band is centred at 1e-12 but upwinded at 0, and the results
    then differ."""
    nx = 64
    r, u, v, t = hi.random_smooth(nx, 2, seed=4, amp=0.02, u0=(0.3, 0.0))
    v = np.zeros_like(v)
    r = np.repeat(r[:1], 2, 0)
    u = np.repeat(u[:1], 2, 0)
    t = np.repeat(t[:1], 2, 0)
    kw = dict(nx=nx, ny=2, mu=1e-3, sigma=0.0)
    res = run(kw, (r, u, v, t), 20, [20])
    assert np.array_equal(res[0.0][0][0], res[1e-12][0][0])
    # velocities of 1e-13 with a density gradient: the band changes E1
    u2 = np.full_like(u, 1e-13)
    res = run(kw, (r, u2, v, t), 1, [1])
    assert not np.array_equal(res[0.0][0][0], res[1e-12][0][0])
