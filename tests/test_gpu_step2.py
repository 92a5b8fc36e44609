"""The two-step sweep (two time steps per kernel launch, periodic domains).

Each step's per-node arithmetic is the one-step kernel's in the same order, so
FP64 runs (built without contraction) must be bitwise equal to one step per
launch, for every tile shape, ragged tiles and grids thinner than the sweep's
radius-4 halo, and match the oracle within 1e-12; FP32 (fused multiply-adds
placed per compiled kernel) within a few units in the last place."""
import numpy as np
import pytest

import hlbm_inputs as hi
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2002_03644_amd import HLBM_EDIVERGED, HLBM_OK, Params, Solver, launch_plan  # noqa: E402


def state(S):
    return torch.cat([S.populations().flatten(), S.moments()["s"].flatten()])


def run(p, f, steps):
    r, u, v, t = f
    s = oracle.entropy_from_theta(r, t, p.gamma)
    S = Solver(p, r, u, v, s=s)
    S.step(steps)
    return S


@pytest.mark.parametrize("shape", [(130, 70), (301, 97), (64, 64), (1, 1), (2, 3), (5, 2),
                                   (3, 200), (61, 2), (200, 7)])
def test_f64_two_steps_bitwise_equal_one_step(shape):
    nx, ny = shape
    f = hi.random_smooth(nx, ny, seed=nx + ny, amp=0.04, u0=(0.15, -0.1))
    base = dict(dtype="f64", mu=2e-3, sigma=0.4)
    one = run(Params(nx, ny, steps_per_launch=1, **base), f, 9)
    for tw, th in ((64, 8), (128, 32), (128, 5), (64, 1)):
        p = Params(nx, ny, steps_per_launch=2, tile_w=tw, tile_h=th, **base)
        assert launch_plan(p)[0] == 2
        two = run(p, f, 9)              # four two-step launches and one single step
        assert torch.equal(state(two), state(one)), (shape, tw, th)


@pytest.mark.parametrize("opts", [dict(e1_centred=True, e2_off=True, feq_order=3),
                                  dict(phi_mode="fd", sigma=0.0), dict(precise_theta=True),
                                  dict(sgn_eps=0.0, sigma=0.9), dict(gamma=5.0 / 3.0,
                                                                     prandtl=2.0)])
def test_f64_two_steps_options_bitwise(opts):
    nx, ny = 150, 90
    f = hi.random_smooth(nx, ny, seed=33, amp=0.05, u0=(0.2, 0.1))
    kw = dict(dtype="f64", mu=3e-3, sigma=0.3)
    kw.update(opts)
    one = run(Params(nx, ny, steps_per_launch=1, **kw), f, 12)
    two = run(Params(nx, ny, steps_per_launch=2, **kw), f, 12)
    assert torch.equal(state(two), state(one)), opts


@pytest.mark.parametrize("sigma", [0.0, 0.5])
def test_f64_two_steps_vortex_matches_oracle(sigma):
    """The isentropic vortex of the FP64 parity case (128^2, Ma 0.5, 500
    steps) with two steps per launch, against the oracle."""
    n = 128
    r, u, v, t = hi.vortex(n, n, 64, 64, 10, 0.5, 0.25, noise=1e-6, seed=0)
    s = oracle.entropy_from_theta(r, t, 1.4)
    O = oracle.OracleSolver(oracle.OracleParams(n, n, mu=1e-3, sigma=sigma), r, u, v, s=s)
    G = Solver(Params(n, n, dtype="f64", mu=1e-3, sigma=sigma, steps_per_launch=2), r, u, v, s=s)
    O.step(500)
    G.step(500)
    mo = O.moments()
    mg = {k: x.double().cpu().numpy() for k, x in G.moments().items()}
    vscale = max(np.abs(mo["ux"]).max(), np.abs(mo["uy"]).max())
    for k in ("rho", "ux", "uy", "s"):
        scale = vscale if k in ("ux", "uy") else np.abs(mo[k]).max()
        err = float(np.abs(mg[k] - mo[k]).max() / scale)
        assert err < 1e-12, (k, err)


@pytest.mark.parametrize("nx,ny", [(1031, 300), (8192, 40), (700, 130)])
def test_f32_two_steps_follow_one_step(nx, ny):
    """FP32 two steps per launch (the default from 900,000 nodes; these
    grids ask for it) against one step per launch: a few units in the last
    place after 20 steps."""
    f = hi.turbulence(nx, 0.5, hi.THETA_PAPER, seed=3, ny=ny)
    two = run(Params(nx, ny, dtype="f32", mu=1e-3, sigma=0.0, steps_per_launch=2), f, 20)
    # 184-column tiles from 1024 columns, 120 below (ragged last tile columns)
    assert launch_plan(two.p)[:2] == (2, 184 if nx >= 1024 else 120)
    one = run(Params(nx, ny, dtype="f32", mu=1e-3, sigma=0.0, steps_per_launch=1), f, 20)
    a, b = state(two), state(one)
    scale = b.abs().max().item()
    assert (a - b).abs().max().item() < 2e-6 * scale


def test_f32_two_step_tile_invariance():
    nx, ny = 301, 97
    r, u, v, t = hi.vortex(nx, ny, 150, 48, 9, 0.9, 0.3, noise=1e-4, seed=1)
    outs = []
    for tw, th in ((64, 8), (128, 32), (192, 16), (256, 5), (192, 97), (128, 1)):
        S = run(Params(nx, ny, dtype="f32", mu=1e-3, sigma=0.3, tile_w=tw, tile_h=th,
                       steps_per_launch=2), (r, u, v, t), 24)
        outs.append(state(S))
    for o in outs[1:]:
        assert (o - outs[0]).abs().max().item() < 2e-6


def test_two_step_flags_divergence():
    n = 64
    r, u, v, t = hi.random_smooth(n, n, seed=2)
    u = u.copy()
    u[20:24, 30:34] += 3.0          # CFL far above 1 in a patch
    G = Solver(Params(n, n, dtype="f32", mu=1e-3, steps_per_launch=2), r, u, v, theta=t)
    G.step(10)
    assert G.status()[0] == HLBM_EDIVERGED


def test_two_step_conserves_mass_and_momentum():
    n = 96
    r, u, v, t = hi.random_smooth(n, n, seed=9, amp=0.05)
    G = Solver(Params(n, n, dtype="f64", mu=2e-3, sigma=0.5, steps_per_launch=2), r, u, v,
               theta=t)
    t0 = G.totals()
    G.step(200)
    t1 = G.totals()
    assert G.status()[0] == HLBM_OK
    for k in range(3):
        assert abs(t1[k] - t0[k]) / t0[0] < 1e-13
