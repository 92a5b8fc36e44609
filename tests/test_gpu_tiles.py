"""Batched step on two-dimensional tiles (kernel "tiles"): one step per
launch, each tile's radius-2 halo loaded at once.

FP64 results must match the CPU oracle within 1e-12 per field and equal the
single-domain one-step kernel bit for bit (the per-node arithmetic is the
same, compiled without contraction); FP32 results must stay within a few
rounding steps of the single-domain run.  The domain sets include domains
smaller than one tile, sizes that leave ragged tiles on both axes, and
extrapolated boundaries."""
import dataclasses

import numpy as np
import pytest

import hlbm_inputs as hi
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2002_03644_amd import BatchSolver, HlbmError, Params, Solver  # noqa: E402

SHAPES = [(64, 64), (100, 77), (130, 130), (257, 63), (33, 200), (5, 3), (300, 41)]
TILES_F64 = [(32, 8), (32, 16), (64, 8)]
TILES_F32 = TILES_F64 + [(32, 32), (64, 16)]
FIELDS = ("rho", "ux", "uy", "s")


def domain_set(dtype, poison=None):
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
        bc_x = "extrapolate" if k == 3 else "periodic"
        bc_y = "extrapolate" if k == 4 else "periodic"
        params.append(Params(nx, ny, dtype=dtype, mu=1e-3 * (1 + k), sigma=0.1 * k,
                             bc_x=bc_x, bc_y=bc_y, theta_ref=th, steps_per_launch=1))
        fields.append(f)
    return params, fields


def singles(params, fields, steps):
    out = []
    for p, f in zip(params, fields):
        S = Solver(dataclasses.replace(p, steps_per_launch=1), *f[:3], theta=f[3])
        S.step(steps)
        out.append({k: v.clone() for k, v in S.moments().items()})
    return out


def scaled_err(a, b):
    """Per field max |a - b| over max |b|, velocities over the largest speed."""
    a = {k: v.double().cpu().numpy() if torch.is_tensor(v) else v for k, v in a.items()}
    b = {k: v.double().cpu().numpy() if torch.is_tensor(v) else v for k, v in b.items()}
    vs = max(np.abs(b["ux"]).max(), np.abs(b["uy"]).max(), 1e-300)
    return {k: float(np.abs(a[k] - b[k]).max() / (vs if k in ("ux", "uy") else
                                                  max(np.abs(b[k]).max(), 1e-300)))
            for k in FIELDS}


@pytest.mark.parametrize("tile", TILES_F64)
def test_f64_tiles_match_oracle(tile):
    """Every domain after 12 steps against the FP64 oracle started from the
    same stored entropy."""
    params, fields = domain_set("f64")
    B = BatchSolver(params, fields)
    B.set_tile(*tile, kernel="tiles")
    assert B.plan() == (1, "tiles") + tile
    s0 = [m["s"].cpu().numpy() for m in B.moments()]
    B.step(12, graph=True)
    mb = B.moments()
    for k, (p, f) in enumerate(zip(params, fields)):
        O = oracle.OracleSolver(oracle.OracleParams(p.nx, p.ny, mu=p.mu, sigma=p.sigma,
                                                    bc_x=p.bc_x, bc_y=p.bc_y),
                                f[0], f[1], f[2], s=s0[k])
        O.step(12)
        err = scaled_err(mb[k], O.moments())
        assert max(err.values()) < 1e-12, (k, err)
    assert B.status()[0] == 0


@pytest.mark.parametrize("tile", TILES_F64)
def test_f64_tiles_bitwise_equal_one_step_kernel(tile):
    params, fields = domain_set("f64")
    B = BatchSolver(params, fields)
    B.set_tile(*tile, kernel="tiles")
    B.step(23, graph=True)
    mb = B.moments()
    ms = singles(params, fields, 23)
    for k in range(len(params)):
        for key in FIELDS:
            assert torch.equal(mb[k][key], ms[k][key]), (tile, k, key)


@pytest.mark.parametrize("tile", TILES_F32)
def test_f32_tiles_close_to_one_step_kernel(tile):
    """FP32: the same arithmetic, but the compiler may place fused
    multiply-adds differently in the two kernels, so the runs may part by
    rounding; after 23 steps they stay within 2e-5 of each field's scale
    (the FP32 unit roundoff is 6e-8)."""
    params, fields = domain_set("f32")
    B = BatchSolver(params, fields)
    B.set_tile(*tile, kernel="tiles")
    B.step(23, graph=True)
    mb = B.moments()
    ms = singles(params, fields, 23)
    same = 0
    for k in range(len(params)):
        err = scaled_err(mb[k], ms[k])
        assert max(err.values()) < 2e-5, (tile, k, err)
        same += all(torch.equal(mb[k][key], ms[k][key]) for key in FIELDS)
    print(f"tiles {tile}: {same} of {len(params)} domains bitwise equal to the one-step kernel")
    assert B.status()[0] == 0


def test_tiles_options_bitwise_in_f64():
    """Per-domain options (precise theta, the original-model ablation with
    third-order equilibria, Phi by finite differences with extrapolated x,
    another gamma and Prandtl number) through the tile kernel."""
    opts = [dict(precise_theta=True), dict(e1_centred=True, e2_off=True, feq_order=3),
            dict(phi_mode="fd", bc_x="extrapolate"), dict(gamma=5.0 / 3.0, prandtl=2.0),
            dict(sgn_eps=0.0)]
    params, fields = [], []
    for k, o in enumerate(opts):
        nx, ny = 96 + 17 * k, 70 + 9 * k
        th = hi.theta_for_cfl(0.5)
        fields.append(hi.vortex(nx, ny, nx / 2, ny / 2, 7, 0.4, 0.04, theta_inf=th,
                                gamma=o.get("gamma", 1.4), angle=0.4 * k))
        params.append(Params(nx, ny, dtype="f64", mu=1e-3, sigma=0.25, theta_ref=th,
                             steps_per_launch=1, **o))
    B = BatchSolver(params, fields)
    B.set_tile(32, 16, kernel="tiles")
    B.step(19, graph=True)
    mb = B.moments()
    ms = singles(params, fields, 19)
    for k in range(len(params)):
        for key in FIELDS:
            assert torch.equal(mb[k][key], ms[k][key]), (k, key)


def test_tiles_diverged_domain_is_isolated():
    """A domain that diverges at once is frozen; every other domain equals
    its single run bit for bit (FP64)."""
    params, fields = domain_set("f64", poison=2)
    B = BatchSolver(params, fields)
    B.set_tile(32, 8, kernel="tiles")
    B.step(30, graph=True)
    bad, flags = B.status()
    assert bad == 1 and flags[2] == 1 and flags.sum() == 1
    mb = B.moments()
    keep = [k for k in range(len(params)) if k != 2]
    ms = singles([params[k] for k in keep], [fields[k] for k in keep], 30)
    for j, k in enumerate(keep):
        for key in FIELDS:
            assert torch.equal(mb[k][key], ms[j][key]), (k, key)


def test_tiles_graph_replays_match_eager():
    """Sixteen- and two-step graphs of the tile kernel, replayed between
    unrelated eager work, equal an eager run after every call."""
    params, fields = domain_set("f32")
    A = BatchSolver(params, fields)
    E = BatchSolver(params, fields)
    for S in (A, E):
        S.set_tile(32, 16, kernel="tiles")
    x = torch.randn(512, 512, device="cuda")
    counts = (16, 3, 34, 2, 17)
    for rep, n in enumerate(counts):
        A.step(n, graph=True)
        E.step(n, graph=False)
        y = (x @ x).sum()
        torch.cuda.synchronize()
        assert torch.isfinite(y)
        ma, me = A.moments(), E.moments()
        for k in range(len(params)):
            for key in FIELDS:
                assert torch.equal(ma[k][key], me[k][key]), (rep, k, key)
    assert A.steps == E.steps == sum(counts)


def test_switching_kernels_keeps_the_state():
    """Strips (two steps per launch) for 6 steps, tiles for 5, strips again
    for 5: in FP64 equal to 16 single-domain steps bit for bit."""
    params, fields = [], []
    for k, (nx, ny) in enumerate([(96, 80), (64, 64), (150, 33)]):
        th = hi.theta_for_cfl(0.6)
        fields.append(hi.vortex(nx, ny, nx / 2, ny / 2, 8, 0.4, 0.04, theta_inf=th,
                                angle=0.5 * k))
        params.append(Params(nx, ny, dtype="f64", mu=1e-3, sigma=0.3, theta_ref=th,
                             tile_w=64, tile_h=16, steps_per_launch=2))
    B = BatchSolver(params, fields)
    assert B.plan()[:2] == (2, "strips")
    B.set_tile(64, 16)
    B.step(6, graph=True)
    B.set_tile(64, 8, kernel="tiles")
    assert B.plan() == (1, "tiles", 64, 8)
    B.step(5, graph=True)
    B.set_tile(64, 16)
    assert B.plan() == (2, "strips", 64, 16)
    B.step(5, graph=True)
    mb = B.moments()
    # the two-step strip kernel is bitwise the one-step kernel in FP64
    ms = singles(params, fields, 16)
    for k in range(len(params)):
        for key in FIELDS:
            assert torch.equal(mb[k][key], ms[k][key]), (k, key)


@pytest.mark.parametrize("kernel,w,h", [("tiles", 48, 8), ("tiles", 32, 4), ("tiles", 128, 8),
                                        ("strips", 32, 8), ("bricks", 32, 8)])
def test_set_tile_rejects_shapes_the_kernels_lack(kernel, w, h):
    params, fields = domain_set("f32")
    B = BatchSolver(params[:2], fields[:2])
    with pytest.raises((HlbmError, ValueError)):
        B.set_tile(w, h, kernel=kernel)
    assert B.plan()[1] == "strips"   # unchanged


def test_f64_rejects_the_large_tiles():
    params, fields = domain_set("f64")
    B = BatchSolver(params[:2], fields[:2])
    for w, h in ((32, 32), (64, 16)):
        with pytest.raises(HlbmError):
            B.set_tile(w, h, kernel="tiles")


def test_tiles_256_domain_batch_sample():
    """The 256-domain batch (log-uniform sizes 64..1016, seed 0) on 32 x 16
    tiles for 20 steps: divergence flags agree with a finite-value scan, and
    sampled healthy domains stay within FP32 rounding of their single runs."""
    specs = hi.batch_specs(256, seed=0)
    params = [Params(sp.n, sp.n, dtype="f32", mu=1e-3, sigma=0.0, theta_ref=sp.theta,
                     steps_per_launch=1) for sp in specs]
    fields = [hi.batch_domain_fields(sp) for sp in specs]
    B = BatchSolver(params, fields)
    B.set_tile(32, 16, kernel="tiles")
    B.step(20, graph=True)
    bad, flags = B.status()
    mb = B.moments()
    for k in range(256):
        if flags[k] == 0:
            assert bool(torch.isfinite(mb[k]["rho"]).all()), k
    for k in (0, 5, 17, 100, 255):
        if flags[k]:
            continue
        ms = singles([params[k]], [fields[k]], 20)[0]
        err = scaled_err(mb[k], ms)
        assert max(err.values()) < 2e-5, (k, err)


# ------------------------------------------------ two steps per launch (FP32)
def periodic_set(poison=None, spl=0):
    params, fields = domain_set("f32", poison=poison)
    params = [dataclasses.replace(p, bc_x="periodic", bc_y="periodic", steps_per_launch=spl)
              for p in params]
    return params, fields


@pytest.mark.parametrize("tile,steps", [((32, 16), 22), ((32, 16), 23), ((64, 8), 23)])
def test_two_step_tiles_close_to_one_step_kernel(tile, steps):
    """All domains periodic: 32 x 16 and 64 x 8 tiles take two steps per
    launch (an odd count ends with a one-step tile launch).  Each domain
    stays within FP32 rounding of its single-domain run, and of the same
    batch on one-step tiles."""
    params, fields = periodic_set()
    B = BatchSolver(params, fields)
    B.set_tile(*tile, kernel="tiles")
    assert B.plan() == (2, "tiles") + tile
    B.step(steps, graph=True)
    assert B.status()[0] == 0 and B.steps == steps
    mb = B.moments()
    p1, _ = periodic_set(spl=1)
    C = BatchSolver(p1, fields)
    C.set_tile(*tile, kernel="tiles")
    assert C.plan() == (1, "tiles") + tile
    C.step(steps, graph=True)
    mc = C.moments()
    ms = singles(params, fields, steps)
    same = 0
    for k in range(len(params)):
        for ref in (ms[k], mc[k]):
            err = scaled_err(mb[k], ref)
            assert max(err.values()) < 2e-5, (k, err)
        same += all(torch.equal(mb[k][key], mc[k][key]) for key in FIELDS)
    print(f"two-step tiles: {same} of {len(params)} domains bitwise equal to one-step tiles")


def test_two_step_tiles_divergence_and_graph_replays():
    """A domain that diverges at once is frozen by the two-step tile kernel;
    graph replays equal an eager run after every call on every healthy
    domain (a frozen domain keeps whatever its tiles held when each
    workgroup saw the flag, which depends on timing)."""
    params, fields = periodic_set(poison=2)
    keep = [k for k in range(len(params)) if k != 2]
    A = BatchSolver(params, fields)
    E = BatchSolver(params, fields)
    for S in (A, E):
        S.set_tile(32, 16, kernel="tiles")
    for rep, n in enumerate((16, 3, 34, 2, 17)):
        A.step(n, graph=True)
        E.step(n, graph=False)
        torch.cuda.synchronize()
        ma, me = A.moments(), E.moments()
        for k in keep:
            for key in FIELDS:
                assert torch.equal(ma[k][key], me[k][key]), (rep, k, key)
    bad, flags = A.status()
    assert bad == 1 and flags[2] == 1 and flags.sum() == 1
    mb = A.moments()
    ms = singles([params[k] for k in keep], [fields[k] for k in keep], A.steps)
    for j, k in enumerate(keep):
        err = scaled_err(mb[k], ms[j])
        assert max(err.values()) < 5e-5, (k, err)
