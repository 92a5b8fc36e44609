"""Guard canaries: every workspace the library is given sits between two
4 KiB zones filled with a byte pattern, and the zones must be unchanged
after the library has run on it (initialisation, steps, graph replays, the
batch autotuner's trial tilings, moments, checkpoints, network training and
inference).  Output buffers of the field calls get the same guards.  A write
past the end (or before the start) of any region the library owns shows up
here, independently of whether the results look right."""
import ctypes

import numpy as np
import pytest

import hlbm_inputs as hi

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2002_03644_amd import CNN, BatchSolver, Params, Solver  # noqa: E402
from paper_2002_03644_amd import _lib  # noqa: E402
from paper_2002_03644_amd._lib import _ptr, _stream, lib  # noqa: E402

G = 4096
PATTERN = 0xA5


def guarded(nbytes):
    """(whole buffer, the nbytes-long view between the two guard zones)"""
    buf = torch.full((nbytes + 2 * G,), PATTERN, dtype=torch.uint8, device="cuda")
    return buf, buf[G:G + nbytes]


def assert_intact(buf, nbytes, what):
    torch.cuda.synchronize()
    head = bool((buf[:G] == PATTERN).all())
    tail = bool((buf[G + nbytes:] == PATTERN).all())
    assert head and tail, (what, head, tail)


@pytest.mark.parametrize("dtype,tile,walls", [("f32", (0, 0), False), ("f64", (64, 5), False),
                                              ("f32", (192, 7), True), ("f64", (0, 0), True)])
def test_single_domain_workspace_and_outputs(dtype, tile, walls):
    nx, ny = 131, 77
    r, u, v, t = hi.vortex(nx, ny, 60, 40, 8, 0.5, 0.2, noise=1e-4, seed=2)
    kw = dict(bc_y="wall", wall_ux_lo=0.0, wall_ux_hi=0.05, wall_theta=float(t.mean())) \
        if walls else {}
    if walls:
        u[0], u[-1], v[0], v[-1] = 0.0, 0.05, 0.0, 0.0
    p = Params(nx, ny, dtype=dtype, mu=2e-3, sigma=0.5, tile_w=tile[0], tile_h=tile[1], **kw)
    nbytes = lib().hlbm_workspace_bytes(ctypes.byref(p.c()))
    buf, ws = guarded(nbytes)
    S = Solver(p, r, u, v, theta=t, workspace=ws)
    S.step(9)
    snap = S.save_state()
    S.step(4)
    S.load_state(snap)
    S.totals()
    S.status()
    # field outputs written into guarded buffers through the ABI
    es = 8 if dtype == "f64" else 4
    n = nx * ny
    outs = [guarded(n * es) for _ in range(5)]
    code = lib().hlbm_moments(S.h, *[_ptr(o[1]) for o in outs], _stream())
    assert code == 0
    fb, fv = guarded(9 * n * es)
    assert lib().hlbm_populations(S.h, _ptr(fv), _stream()) == 0
    assert_intact(buf, nbytes, "workspace")
    for k, (b, _) in enumerate(outs):
        assert_intact(b, n * es, f"moments output {k}")
    assert_intact(fb, 9 * n * es, "populations output")


def test_batch_workspace_through_autotune_and_graphs():
    shapes = [(64, 64), (130, 70), (200, 33), (96, 96)]
    params, fields = [], []
    for k, (nx, ny) in enumerate(shapes):
        th = hi.theta_for_cfl(0.5)
        fields.append(hi.vortex(nx, ny, nx / 2, ny / 2, max(2.0, min(nx, ny) / 8), 0.3, 0.05,
                                theta_inf=th))
        params.append(Params(nx, ny, dtype="f32", mu=1e-3, sigma=0.2, theta_ref=th))
    arr = (_lib.CParams * len(params))(*[p.c() for p in params])
    nbytes = lib().hlbm_batch_workspace_bytes(arr, len(params))
    buf, ws = guarded(nbytes)
    B = BatchSolver(params, fields, workspace=ws)
    B.step(3, graph=False)
    B.step(6, graph=True)
    B.autotune(steps=2)          # every tile shape, largest item list included
    B.step(4, graph=True)
    B.moments_cat()
    B.status()
    assert_intact(buf, nbytes, "batch workspace")


def test_network_workspace_training_and_inference():
    from oracle import cnn_oracle
    H, W, mb = 8, 64, 3
    params = cnn_oracle.flatten(cnn_oracle.init_params(4)).astype(np.float32)
    nbytes = lib().hlbm_cnn_workspace_bytes(mb, H, W)
    buf, ws = guarded(nbytes)
    net = CNN(mb, H, W, params, workspace=ws)
    rng = np.random.default_rng(5)
    x = torch.from_numpy(rng.normal(size=(mb, 4, H, W)).astype(np.float32)).cuda()
    tgt = torch.from_numpy(rng.normal(size=(mb, 4, H, W)).astype(np.float32)).cuda()
    for _ in range(3):
        net.train_step(x, tgt, 1e-3)
    net.forward(x)
    net.set_fused(False)
    net.forward(x)
    idx = torch.tensor([2, 0], dtype=torch.int32, device="cuda")
    net.loss_grad(x, tgt, idx=idx)
    assert_intact(buf, nbytes, "network workspace")
