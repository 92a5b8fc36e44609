"""Walls (bc_y = wall) on the GPU, through the C ABI.

FP64: parity with the oracle within 1e-12 per field on flows that touch the
walls, over several tiles with ragged tails and strips that end next to a
wall.  FP32: relative L2 distance to the FP64 GPU path within frozen
tolerances.  The thermal Couette flow of Sec. 4.4 on the paper's 2 x 100
channel reaches the closed-form temperature profile."""
import numpy as np
import pytest

import hlbm_inputs as hi
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2002_03644_amd import Params, Solver  # noqa: E402
from paper_2002_03644_amd.studies import thermal_couette  # noqa: E402

FIELDS = ("rho", "ux", "uy", "s")


def channel_fields(nx, ny, thw, u_lo, u_hi, seed=0):
    """Vortex in a sheared channel whose wall rows carry the wall state."""
    r, u, v, t = hi.vortex(nx, ny, nx / 2, ny / 2, ny / 6, 0.4, 0.1, theta_inf=thw,
                           noise=1e-3, seed=seed)
    eta = np.arange(ny)[:, None] / (ny - 1)
    u = u + u_lo + (u_hi - u_lo) * eta
    u[0], u[-1] = u_lo, u_hi
    v[0], v[-1] = 0.0, 0.0
    t[0], t[-1] = thw, thw
    return r, u, v, t


def pair(nx, ny, steps, sigma=0.5, tile=(0, 0), bc_x="periodic", phi="lbm", **kw):
    thw, u_lo, u_hi = 0.2, -0.05, 0.1
    r, u, v, t = channel_fields(nx, ny, thw, u_lo, u_hi)
    s = oracle.entropy_from_theta(r, t, 1.4)
    wall = dict(bc_y="wall", wall_ux_lo=u_lo, wall_ux_hi=u_hi, wall_theta=thw)
    O = oracle.OracleSolver(oracle.OracleParams(nx, ny, mu=0.02, sigma=sigma, bc_x=bc_x,
                                                phi_mode=phi, **wall), r, u, v, s=s)
    G = Solver(Params(nx, ny, dtype="f64", mu=0.02, sigma=sigma, bc_x=bc_x, phi_mode=phi,
                      tile_w=tile[0], tile_h=tile[1], **wall, **kw), r, u, v, s=s)
    O.step(steps)
    G.step(steps)
    return O.moments(), {k: x.double().cpu().numpy() for k, x in G.moments().items()}


def assert_parity(mo, mg, tol=1e-12):
    vscale = max(np.abs(mo["ux"]).max(), np.abs(mo["uy"]).max())
    for k in FIELDS:
        scale = vscale if k in ("ux", "uy") else np.abs(mo[k]).max()
        err = float(np.abs(mg[k] - mo[k]).max() / scale)
        assert err < tol, (k, err)


@pytest.mark.parametrize("sigma", [0.0, 0.9])
def test_f64_walls_parity_several_tiles(sigma):
    """70 x 37 with 64 x 8 tiles: two tiles in x (ragged), five strips with a
    ragged last one, strips ending on both wall rows."""
    mo, mg = pair(70, 37, 25, sigma=sigma, tile=(64, 8))
    assert_parity(mo, mg)


@pytest.mark.parametrize("opts", [dict(tile=(128, 0)), dict(bc_x="extrapolate"),
                                  dict(phi="fd"), dict(tile=(64, 1))])
def test_f64_walls_parity_options(opts):
    mo, mg = pair(50, 20, 15, **opts)
    assert_parity(mo, mg)


def test_f64_walls_smallest_channel():
    """ny = 4: each wall reads the two interior rows, which the other wall
    also reads."""
    mo, mg = pair(9, 4, 10)
    assert_parity(mo, mg)


def test_f32_walls_tolerance():
    thw, u_lo, u_hi = 0.2, -0.05, 0.1
    r, u, v, t = channel_fields(96, 48, thw, u_lo, u_hi, seed=1)
    s = oracle.entropy_from_theta(r, t, 1.4)
    wall = dict(bc_y="wall", wall_ux_lo=u_lo, wall_ux_hi=u_hi, wall_theta=thw)
    out = {}
    for dt in ("f64", "f32"):
        G = Solver(Params(96, 48, dtype=dt, mu=0.02, sigma=0.9, theta_ref=thw, **wall),
                   r, u, v, s=s)
        G.step(200)
        out[dt] = {k: x.double().cpu().numpy() for k, x in G.moments().items()}
    # measured: rho 2.6e-3 (centred), u_x 3.5e-5, u_y 3.9e-4, s 2.8e-6
    for k, tol in (("rho", 5e-3), ("ux", 1e-4), ("uy", 1e-3), ("s", 1e-5)):
        a, b = out["f32"][k], out["f64"][k]
        ref = b - b.mean() if k != "s" else b
        err = np.linalg.norm(a - b) / np.linalg.norm(ref)
        assert err < tol, (k, err)


@pytest.mark.parametrize("dtype,precise,tol,utol", [("f64", True, 1e-9, 1e-9),
                                                     ("f32", True, 6e-4, 3e-4),
                                                     ("f32", False, 6e-3, 3e-4)])
def test_couette_paper_channel(dtype, precise, tol, utol):
    """2 x 100, sigma 0.9, Ma 0.8, Pr 0.71, gamma 1.4, T_w / T_r = 0.2.
    Measured: FP64 1.7e-11 of the temperature rise and 6.3e-13 of U in u_x;
    FP32 1.9e-4 and 1.4e-4 with precise theta, 3.1e-3 without.  Without it
    the temperature Laplacian (about 1e-6) is formed from FP32 temperatures
    rounded to 1.5e-8 through a fast exp; with it from deviations accurate
    relative to themselves."""
    res = thermal_couette(ny=100, dtype=dtype, precise_theta=precise)
    assert res["error"] < tol, res["error"]
    assert res["ux_error"] < utol, res["ux_error"]


def test_couette_mach_and_prandtl():
    for ma, pr in ((0.4, 0.71), (1.2, 0.71), (0.8, 2.0)):
        res = thermal_couette(ny=40, ma=ma, pr=pr)
        assert res["error"] < 1e-8, (ma, pr, res["error"])  # measured <= 2.7e-10
