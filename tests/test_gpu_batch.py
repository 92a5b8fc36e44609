"""Batched engine: one persistent launch per step (two steps per launch when
every domain is periodic and FP32) over many uneven domains.

Per-node arithmetic is the single-domain kernel's, so a batched run must be
bitwise identical to running each domain alone with the same tile shape and
the same steps per launch."""
import dataclasses
import json
import os

import numpy as np
import pytest

import hlbm_inputs as hi

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2002_03644_amd import BatchSolver, Params, Solver  # noqa: E402

SHAPES = [(64, 64), (100, 77), (130, 130), (257, 63), (33, 200), (5, 3), (300, 41)]


def domain_set(dtype, poison=None, spl=1, periodic=False):
    params, fields = [], []
    for k, (nx, ny) in enumerate(SHAPES):
        mach = 0.2 + 0.15 * k
        th = hi.theta_for_cfl(1.2 * mach)
        if k % 2 == 0:
            f = hi.vortex(nx, ny, nx / 2, ny / 2, max(2.0, min(nx, ny) / 8), mach, 0.1 * mach,
                          theta_inf=th, angle=0.3 * k)
        else:
            f = hi.random_smooth(nx, ny, seed=k, amp=0.03, theta0=th, u0=(0.1, -0.05))
        if poison == k:
            f = (f[0], f[1] + 3.0, f[2], f[3])   # CFL far above 1: diverges
        bc = "extrapolate" if k == 3 and not periodic else "periodic"
        params.append(Params(nx, ny, dtype=dtype, mu=1e-3 * (1 + k), sigma=0.1 * k,
                             bc_x=bc, theta_ref=th, tile_w=128, tile_h=32,
                             steps_per_launch=spl))
        fields.append(f)
    return params, fields


def singles(params, fields, steps):
    out = []
    for p, f in zip(params, fields):
        S = Solver(p, *f[:3], theta=f[3])
        S.step(steps)
        out.append({k: v.clone() for k, v in S.moments().items()})
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("graph,tile", [(False, (128, 32)), (True, (128, 32)),
                                        (True, (192, 16))])
def test_batch_bitwise_equals_single_domains(dtype, graph, tile):
    params, fields = domain_set(dtype)
    B = BatchSolver(params, fields)
    B.set_tile(*tile)
    B.step(23, graph=graph)
    mb = B.moments()
    # FP32 FMA placement may differ between kernels compiled for different
    # widths, so the single-domain reference uses the batch's tile
    ms = singles([dataclasses.replace(p, tile_w=tile[0], tile_h=tile[1]) for p in params],
                 fields, 23)
    for k in range(len(params)):
        for key in ("rho", "ux", "uy", "s"):
            assert torch.equal(mb[k][key], ms[k][key]), (k, key)
    assert B.status()[0] == 0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("graph,tile,steps", [(False, (128, 32), 23), (True, (128, 16), 37),
                                              (True, (64, 8), 23), (True, (184, 16), 23),
                                              (False, (184, 8), 9), (True, (120, 8), 23)])
def test_two_step_batch_bitwise_equals_single_domains(dtype, graph, tile, steps):
    """All domains periodic, two steps per launch (an odd count ends with a
    one-step launch, on 120- and 184-column strips the one-step kernel of
    that width): each domain equals its single run with the same tile and
    plan, bit for bit.  Those two widths are FP32 only."""
    if dtype == "f64" and tile[0] in (120, 184):
        pytest.skip("120- and 184-column strips take FP32 domains only")
    params, fields = domain_set(dtype, spl=2, periodic=True)
    B = BatchSolver(params, fields)
    B.set_tile(*tile)
    B.step(steps, graph=graph)
    mb = B.moments()
    ms = singles([dataclasses.replace(p, tile_w=tile[0], tile_h=tile[1]) for p in params],
                 fields, steps)
    for k in range(len(params)):
        for key in ("rho", "ux", "uy", "s"):
            assert torch.equal(mb[k][key], ms[k][key]), (k, key)
    assert B.status()[0] == 0 and B.steps == steps


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_with_mixed_options_equals_single_domains(dtype):
    """Every per-domain option travels in the batch's parameter table: domains
    with precise theta, the original-model ablation (centred E1, no E2),
    Phi by finite differences, extrapolated x boundaries and their own
    gamma and Prandtl number each match their single run bitwise."""
    opts = [dict(precise_theta=True), dict(e1_centred=True, e2_off=True),
            dict(phi_mode="fd", bc_x="extrapolate"), dict(gamma=5.0 / 3.0, prandtl=2.0),
            dict()]
    params, fields = [], []
    for k, o in enumerate(opts):
        nx, ny = 96 + 17 * k, 70 + 9 * k
        th = hi.theta_for_cfl(0.5)
        fields.append(hi.vortex(nx, ny, nx / 2, ny / 2, 7, 0.4, 0.04, theta_inf=th,
                                gamma=o.get("gamma", 1.4), angle=0.4 * k))
        params.append(Params(nx, ny, dtype=dtype, mu=1e-3, sigma=0.25, theta_ref=th,
                             tile_w=128, tile_h=16, steps_per_launch=1, **o))
    B = BatchSolver(params, fields)
    B.set_tile(128, 16)
    B.step(19, graph=True)
    mb = B.moments()
    ms = singles(params, fields, 19)
    for k in range(len(params)):
        for key in ("rho", "ux", "uy", "s"):
            assert torch.equal(mb[k][key], ms[k][key]), (k, key)
    assert B.status()[0] == 0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_with_padded_planes_equals_single_domains(dtype):
    """A domain large enough for the padded plane stride (over 4 MiB per
    plane) between two small ones: the batch's per-domain offsets follow the
    padded size, and every domain still matches its single run bitwise."""
    shapes = [(64, 64), (1100, 1031), (130, 70)]
    params, fields = [], []
    for k, (nx, ny) in enumerate(shapes):
        th = hi.theta_for_cfl(0.6)
        fields.append(hi.vortex(nx, ny, nx / 2, ny / 2, max(2.0, min(nx, ny) / 8), 0.4, 0.04,
                                theta_inf=th, angle=0.5 * k))
        params.append(Params(nx, ny, dtype=dtype, mu=1e-3, sigma=0.3, theta_ref=th,
                             tile_w=192, tile_h=16))
    B = BatchSolver(params, fields)
    B.set_tile(192, 16)
    B.step(6, graph=True)
    mb = B.moments()
    ms = singles(params, fields, 6)
    for k in range(len(params)):
        for key in ("rho", "ux", "uy", "s"):
            assert torch.equal(mb[k][key], ms[k][key]), (k, key)
    assert B.status()[0] == 0


def test_graph_replays_match_eager_between_eager_work():
    """Replays of the captured graphs (two-step and sixteen-step, and an odd
    count that ends eagerly and moves the state to the other buffer, so the
    graphs are captured again), interleaved with unrelated eager work and
    synchronisations, equal an eager run after every call."""
    params, fields = domain_set("f32")
    A = BatchSolver(params, fields)
    E = BatchSolver(params, fields)
    x = torch.randn(512, 512, device="cuda")
    counts = (6, 22, 6, 35, 16, 6)
    for rep, n in enumerate(counts):
        A.step(n, graph=True)
        E.step(n, graph=False)
        y = (x @ x).sum()          # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(y)
        ma, me = A.moments(), E.moments()
        for k in range(len(params)):
            assert torch.equal(ma[k]["rho"], me[k]["rho"]), (rep, k)
            assert torch.equal(ma[k]["s"], me[k]["s"]), (rep, k)
    assert A.steps == E.steps == sum(counts)


def test_diverged_domain_is_isolated():
    params, fields = domain_set("f32", poison=2)
    B = BatchSolver(params, fields)
    B.set_tile(128, 32)
    B.step(40)
    bad, flags = B.status()
    assert bad == 1 and flags[2] == 1 and flags.sum() == 1
    mb = B.moments()
    keep = [k for k in range(len(params)) if k != 2]
    ms = singles([params[k] for k in keep], [fields[k] for k in keep], 40)
    for j, k in enumerate(keep):
        assert torch.equal(mb[k]["rho"], ms[j]["rho"]), k


def test_autotune_restores_state_and_caches(tmp_path):
    params, fields = domain_set("f32")
    B = BatchSolver(params, fields)
    B.step(4)
    before = [m["rho"].clone() for m in B.moments()]
    cache = str(tmp_path / "tune.json")
    kern, w, h = B.autotune(steps=2, cache_path=cache)
    if kern == "strips":
        assert w in (64, 120, 128, 184, 192, 256) and h in (4, 8, 16, 32, 64, 128)
    else:
        assert kern == "tiles" and (w, h) in ((32, 8), (32, 16), (64, 8), (32, 32), (64, 16))
    assert B.plan()[1:] == (kern, w, h)
    after = [m["rho"] for m in B.moments()]
    assert B.steps == 4 and B.status()[0] == 0
    for a, b in zip(before, after):
        assert torch.equal(a, b)
    with open(cache) as fh:
        assert json.load(fh)[B.signature()] == [kern, w, h]
    assert B.autotune(cache_path=cache) == (kern, w, h)   # served from the cache


def test_batch_256_domains_seed0():
    """The 256-domain batch (log-uniform sizes 64..1016, vortex or turbulence,
    Mach 0.1-2.0, seed 0): 20 graph-replayed steps; domains that stay finite
    are bitwise equal to their single-domain runs (checked on a sample), and
    the divergence flags agree with a finite-value scan."""
    specs = hi.batch_specs(256, seed=0)
    params, fields = [], []
    for sp in specs:
        f = hi.batch_domain_fields(sp)
        params.append(Params(sp.n, sp.n, dtype="f32", mu=1e-3, sigma=0.0, theta_ref=sp.theta,
                             tile_w=128, tile_h=32))
        fields.append(f)
    assert sum(p.nx * p.ny for p in params) == 58630144
    B = BatchSolver(params, fields)
    B.set_tile(128, 32)
    B.step(20, graph=True)
    bad, flags = B.status()
    mb = B.moments()
    for k in range(256):
        finite = bool(torch.isfinite(mb[k]["rho"]).all())
        if flags[k] == 0:
            assert finite, k
    print(f"256-domain batch: {bad} domains diverged within 20 steps")
    for k in (0, 5, 17, 100, 255):
        if flags[k]:
            continue
        S = Solver(params[k], *fields[k][:3], theta=fields[k][3])
        S.step(20)
        assert torch.equal(S.moments()["rho"], mb[k]["rho"]), k


def test_divergence_mid_launch_leaves_healthy_domains_bitwise():
    """Domains that diverge while the same launch is sweeping large healthy
    domains: a large one whose CFL is far above 1 in a patch (it diverges
    within the first steps, while its own tiles are still being swept by
    other workgroups) and a small one that diverges at once.  The skip of a
    frozen domain's items is decided per workgroup, so no tile of a healthy
    domain may change: every healthy domain is bitwise equal to its single
    run, at several tile shapes."""
    shapes = [(700, 520), (640, 610), (512, 480), (900, 300), (96, 80), (450, 470)]
    poisoned = {1: "patch", 4: "all"}
    params, fields = [], []
    for k, (nx, ny) in enumerate(shapes):
        th = hi.theta_for_cfl(0.6)
        f = hi.vortex(nx, ny, nx / 2, ny / 2, 12, 0.4, 0.05, theta_inf=th, angle=0.7 * k)
        if poisoned.get(k) == "patch":
            ux = f[1].copy()
            ux[ny // 3: ny // 3 + 20, nx // 2: nx // 2 + 20] += 3.0
            f = (f[0], ux, f[2], f[3])
        elif poisoned.get(k) == "all":
            f = (f[0], f[1] + 3.0, f[2], f[3])
        fields.append(f)
        params.append(Params(nx, ny, dtype="f32", mu=1e-3, sigma=0.2, theta_ref=th))
    healthy = [k for k in range(len(shapes)) if k not in poisoned]
    for tw, th_ in ((128, 16), (192, 8), (64, 4)):
        ps = [dataclasses.replace(p, tile_w=tw, tile_h=th_) for p in params]
        B = BatchSolver(ps, fields)
        B.set_tile(tw, th_)
        B.step(12, graph=True)
        bad, flags = B.status()
        assert set(np.nonzero(flags)[0]) == set(poisoned), (tw, th_, flags)
        mb = B.moments()
        ms = singles([ps[k] for k in healthy], [fields[k] for k in healthy], 12)
        for j, k in enumerate(healthy):
            for key in ("rho", "ux", "uy", "s"):
                assert torch.equal(mb[k][key], ms[j][key]), (tw, th_, k, key)
        del B
