"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol the headers under include/ declare, and its host-only functions
validate parameters and size workspaces."""
import glob
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"\b(hlbm_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_core_entry_points():
    names = declared_functions()
    for n in ("hlbm_init", "hlbm_step", "hlbm_moments", "hlbm_totals", "hlbm_status",
              "hlbm_destroy", "hlbm_workspace_bytes"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2002_03644_amd import _lib
    L = _lib.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def _params(**kw):
    from paper_2002_03644_amd import Params
    base = dict(nx=64, ny=32, dtype="f32")
    base.update(kw)
    return Params(**base)


def test_validate_accepts_defaults():
    from paper_2002_03644_amd import HLBM_OK, validate
    assert validate(_params()) == HLBM_OK
    assert validate(_params(dtype="f64", bc_x="extrapolate", phi_mode="fd")) == HLBM_OK


@pytest.mark.parametrize("bad", [dict(nx=0), dict(ny=-3), dict(gamma=1.0), dict(prandtl=0.0),
                                 dict(mu=-1e-3), dict(sigma=1.5), dict(rho_ref=0.0),
                                 dict(theta_ref=-1.0), dict(tile_w=96), dict(tile_h=-1),
                                 dict(nx=20000, ny=20000), dict(mu=float("nan"))])
def test_validate_rejects(bad):
    from paper_2002_03644_amd import HLBM_EINVAL, validate, workspace_bytes
    p = _params(**bad)
    assert validate(p) == HLBM_EINVAL
    assert workspace_bytes(p) == 0


def test_validate_bounds_padded_plane_offsets():
    """The step addresses a plane with (y pitch + x) in 32-bit int and its
    byte offset in 32 bits, with pitch = nx rounded up to 64.  Narrow, tall
    grids pass the 9 nx ny < 2^31 element bound but not this one: at nx = 1
    the pitch is 64, so FP64 allows ny < 2^23 and FP32 ny < 2^24."""
    from paper_2002_03644_amd import HLBM_EINVAL, HLBM_OK, validate
    assert validate(_params(nx=1, ny=(1 << 23) - 1, dtype="f64")) == HLBM_OK
    assert validate(_params(nx=1, ny=1 << 23, dtype="f64")) == HLBM_EINVAL
    assert validate(_params(nx=1, ny=(1 << 24) - 1, dtype="f32")) == HLBM_OK
    assert validate(_params(nx=1, ny=1 << 24, dtype="f32")) == HLBM_EINVAL
    # 16 x 10M in FP64: 9 nx ny < 2^31 holds, the padded plane is 4.8 GiB
    assert 9 * 16 * 10_000_000 < 2 ** 31
    assert validate(_params(nx=16, ny=10_000_000, dtype="f64")) == HLBM_EINVAL
    # a wide grid near the element bound is accepted
    assert validate(_params(nx=8192, ny=29000)) == HLBM_OK


@pytest.mark.parametrize("order,ok", [(0, True), (3, True), (4, True), (2, False), (5, False)])
def test_validate_feq_order(order, ok):
    from paper_2002_03644_amd import HLBM_EINVAL, HLBM_OK, validate
    assert validate(_params(feq_order=order)) == (HLBM_OK if ok else HLBM_EINVAL)


def test_launch_plan_and_steps_per_launch():
    from paper_2002_03644_amd import HLBM_EINVAL, launch_plan, validate
    assert launch_plan(_params(nx=8192, ny=8192))[0] == 2               # FP32 periodic
    assert launch_plan(_params(nx=1000, ny=1000))[0] == 2               # from 900,000 nodes
    assert launch_plan(_params(nx=768, ny=768))[0] == 1                 # smaller: one step
    assert launch_plan(_params(nx=4096, ny=256))[0] == 2                # nodes, not width
    assert launch_plan(_params(nx=8192, ny=8192, dtype="f64"))[0] == 1  # FP64 default
    assert launch_plan(_params(bc_x="extrapolate"))[0] == 1
    assert launch_plan(_params(bc_y="wall", wall_theta=0.2))[0] == 1
    assert launch_plan(_params(steps_per_launch=1))[0] == 1
    spl, tw, th = launch_plan(_params(nx=8192, ny=8192))
    assert (tw, th) == (184, 64)
    assert launch_plan(_params(nx=100, ny=100, dtype="f64", steps_per_launch=2))[0] == 2
    for bad in (dict(steps_per_launch=3), dict(steps_per_launch=-1),
                dict(steps_per_launch=2, bc_x="extrapolate"),
                dict(steps_per_launch=2, bc_y="wall", wall_theta=0.2),
                dict(steps_per_launch=2, dtype="f64", tile_w=192)):
        assert validate(_params(**bad)) == HLBM_EINVAL, bad


def test_wall_parameters_validated_on_the_host():
    from paper_2002_03644_amd import HLBM_EINVAL, HLBM_OK, validate
    ok = dict(bc_y="wall", wall_theta=0.2, wall_ux_hi=0.1)
    assert validate(_params(**ok)) == HLBM_OK
    assert validate(_params(ny=4, **ok)) == HLBM_OK
    for bad in (dict(ny=3), dict(wall_theta=0.0), dict(wall_theta=float("inf")),
                dict(wall_ux_lo=float("nan"))):
        kw = dict(ok)
        kw.update(bad)
        assert validate(_params(**kw)) == HLBM_EINVAL, bad
    assert validate(_params(bc_x="wall", wall_theta=0.2)) == HLBM_EINVAL  # walls along y only


def test_batches_reject_walls():
    import ctypes
    from paper_2002_03644_amd import _lib
    ps = [_params(), _params(bc_y="wall", wall_theta=0.2)]
    arr = (_lib.CParams * 2)(*[p.c() for p in ps])
    assert _lib.lib().hlbm_batch_workspace_bytes(arr, 1) > 0
    assert _lib.lib().hlbm_batch_workspace_bytes(arr, 2) == 0


def test_workspace_size_covers_two_state_buffers():
    from paper_2002_03644_amd import workspace_bytes
    for dt, es in (("f32", 4), ("f64", 8)):
        for nx, ny in ((8192, 8192), (4096, 4), (1, 1), (131, 77)):
            ws = workspace_bytes(_params(nx=nx, ny=ny, dtype=dt))
            assert ws >= 2 * 10 * nx * ny * es
            # rows padded to 64 elements, plus at most 192 KiB + 256 B of
            # stride padding per plane
            pitch = -(-nx // 64) * 64
            assert ws < 2 * 10 * ((pitch * ny + 64) * es + 192 * 1024 + 256) + 2 * 2 ** 20


@pytest.mark.parametrize("dt,es", [("f32", 4), ("f64", 8)])
def test_large_planes_get_a_stride_off_the_power_of_two(dt, es):
    """Rows are padded to 64 elements (256-byte aligned FP32 rows); planes of
    4 MiB or more sit 64 KiB + 256 B past a multiple of 128 KiB apart, so
    that a node's ten values do not share HBM channels and banks; smaller
    planes keep a 64-element stride."""
    from paper_2002_03644_amd import Params
    from paper_2002_03644_amd._lib import lib
    for nx, ny in ((8192, 8192), (4096, 4096), (6000, 6000), (1024, 1024), (131, 77), (1, 1)):
        plane = lib().hlbm_state_bytes(ctypes.byref(Params(nx, ny, dtype=dt).c())) // 10
        pitch = -(-nx // 64) * 64
        base = -(-pitch * ny // 64) * 64 * es
        if base < 4 * 2 ** 20:
            assert plane == base, (nx, ny)
        else:
            assert plane % (128 * 1024) == 64 * 1024 + 256, (nx, ny)
            assert base < plane <= base + 192 * 1024 + 256, (nx, ny)


@pytest.mark.parametrize("nx,ny,dt,shape", [
    (8192, 8192, "f32", (192, 16)),   # the bench grid
    (8192, 8192, "f64", (192, 32)),
    (15446, 15446, "f32", (192, 16)),
    (1500, 1500, "f32", (192, 8)),    # halved until about 768 workgroups
    (1024, 1024, "f32", (192, 8)),
    (1024, 1024, "f64", (192, 8)),    # about 512 in FP64
    (1023, 1023, "f32", (128, 8)),
    (768, 768, "f32", (128, 4)),
    (64, 64, "f32", (64, 4)),
    (2, 100, "f64", (64, 4)),         # the Couette channel
    (1, 1, "f64", (64, 1)),           # never more rows than ny
    (300, 3, "f32", (128, 3)),
])
def test_default_launch_shape(nx, ny, dt, shape):
    """Defaults of the one-step sweep."""
    from paper_2002_03644_amd import launch_shape
    assert launch_shape(_params(nx=nx, ny=ny, dtype=dt, steps_per_launch=1)) == shape


@pytest.mark.parametrize("nx,ny,dt,shape", [
    (8192, 8192, "f32", (184, 64)),   # the bench grid
    (6000, 6000, "f32", (184, 64)),   # 3102 workgroups: four rounds of 1024, 76 % full
    (4096, 4096, "f32", (184, 32)),   # 64 rows: 1472 workgroups fill two rounds to 72 %
    (3000, 3000, "f32", (184, 64)),   # 799 workgroups
    (2048, 2048, "f32", (184, 32)),   # halved until 768 workgroups
    (1500, 1500, "f32", (184, 16)),
    (1024, 1024, "f32", (184, 8)),
    (1000, 1000, "f32", (120, 8)),    # 640 .. 1023 columns: 120, halved until 768 workgroups
    (768, 768, "f32", (120, 8)),
    (600, 600, "f32", (128, 8)),      # narrower grids: 128 columns, about 384 workgroups
    (256, 256, "f32", (128, 8)),
    (64, 64, "f32", (64, 8)),
    (1, 1, "f32", (64, 1)),           # never more rows than ny
    (1024, 1024, "f64", (128, 16)),   # FP64 keeps 128-column tiles
])
def test_default_two_step_shape(nx, ny, dt, shape):
    from paper_2002_03644_amd import launch_plan
    assert launch_plan(_params(nx=nx, ny=ny, dtype=dt, steps_per_launch=2)) == (2,) + shape


def test_launch_shape_takes_given_tiles_and_rejects_bad_input():
    import ctypes as C

    from paper_2002_03644_amd import launch_shape
    from paper_2002_03644_amd._lib import lib
    assert launch_shape(_params(nx=100, ny=100, tile_w=256, tile_h=7)) == (256, 7)
    assert launch_shape(_params(nx=100, ny=5, tile_w=64, tile_h=40)) == (64, 5)
    w = C.c_int32()
    p = _params(nx=100, ny=100).c()
    assert lib().hlbm_launch_shape(C.byref(p), C.byref(w), None) != 0
    bad = _params(nx=100, ny=100, tile_w=100).c()
    assert lib().hlbm_launch_shape(C.byref(bad), C.byref(w), C.byref(w)) != 0


def test_largest_grid_accepted():
    from paper_2002_03644_amd import HLBM_OK, validate
    assert validate(_params(nx=15446, ny=15446)) == HLBM_OK  # 9 n^2 < 2^31
    assert validate(_params(nx=15447, ny=15447)) != HLBM_OK


def test_init_rejects_null_and_small_workspace():
    from paper_2002_03644_amd import _lib
    L = _lib.lib()
    cp = _params().c()
    h = ctypes.c_void_p()
    code = L.hlbm_init(ctypes.byref(h), ctypes.byref(cp), None, 0, None, None, None, None, None)
    assert code == _lib.HLBM_EINVAL
    fake = ctypes.c_void_p(256)  # never dereferenced: rejected before any launch
    code = L.hlbm_init(ctypes.byref(h), ctypes.byref(cp), fake, 16, fake, fake, fake, fake, None)
    assert code == _lib.HLBM_EWORKSPACE
    assert not h.value


def test_strerror_covers_codes():
    from paper_2002_03644_amd import strerror
    for c in (0, 1, -1, -2, -3, -4, -5):
        assert strerror(c) and "unknown" not in strerror(c)


def test_nn_header_declares_the_closure_entry_points():
    names = declared_functions()
    for n in ("hlbm_cnn_init", "hlbm_cnn_forward", "hlbm_cnn_loss_grad", "hlbm_cnn_adam",
              "hlbm_restrict", "hlbm_batch_correct", "hlbm_closure_step"):
        assert n in names


@pytest.mark.parametrize("dims,ok", [((8, 256, 256), True), ((1, 4, 32), True),
                                     ((0, 256, 256), False), ((8, 250, 256), False),
                                     ((8, 256, 48), False), ((8, 2, 32), False),
                                     ((40000, 256, 256), False)])
def test_cnn_workspace_validates_dims(dims, ok):
    from paper_2002_03644_amd import _lib
    n = _lib.lib().hlbm_cnn_workspace_bytes(*dims)
    assert (n > 0) == ok
    if ok:   # at least the activations: 4 + 32 + 32 (+ gradients) BF16 channels per pixel
        b, h, w = dims
        assert n >= b * h * w * 2 * (4 + 32 + 32 + 4 + 32 + 32)


def test_nn_entry_points_validate_on_the_host():
    """Invalid arguments are rejected before any device work (no GPU needed)."""
    import ctypes

    from paper_2002_03644_amd import _lib
    L = _lib.lib()
    EINVAL, EWS = _lib.HLBM_EINVAL, _lib.HLBM_EWORKSPACE
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)
    # bad sizes, missing parameters, missing or short workspace
    assert L.hlbm_cnn_init(ctypes.byref(h), 0, 256, 256, fake, 1 << 30, fake, None) == EINVAL
    assert L.hlbm_cnn_init(ctypes.byref(h), 1, 256, 250, fake, 1 << 30, fake, None) == EINVAL
    assert L.hlbm_cnn_init(ctypes.byref(h), 1, 256, 256, fake, 1 << 30, None, None) == EINVAL
    assert L.hlbm_cnn_init(ctypes.byref(h), 1, 32, 64, None, 0, fake, None) == EWS
    need = L.hlbm_cnn_workspace_bytes(1, 32, 64)
    assert L.hlbm_cnn_init(ctypes.byref(h), 1, 32, 64, fake, need - 1, fake, None) == EWS
    assert h.value is None
    # null handles
    assert L.hlbm_cnn_set_norm(None, (ctypes.c_float * 16)()) == EINVAL
    assert L.hlbm_cnn_set_output_clip(None, 1.0) == EINVAL
    assert L.hlbm_cnn_set_fused(None, 1) == EINVAL
    assert L.hlbm_cnn_adam(None, 1e-3, None) == EINVAL
    assert L.hlbm_cnn_forward(None, fake, 4, 1, None, 1, fake, 4, 1, None) == EINVAL
    assert L.hlbm_cnn_loss_grad(None, fake, 4, 1, fake, 4, 1, None, 1, None, None) == EINVAL
    assert L.hlbm_batch_correct(None, fake, fake, 1, None) == EINVAL
    assert L.hlbm_closure_step(None, None, 1, 1, 1, 1, None) == EINVAL
    # restriction: sizes must divide, pointers and strides must be given
    assert L.hlbm_restrict(fake, fake, fake, fake, 1, 10, 12, 4, fake, 16, 4, None) == EINVAL
    assert L.hlbm_restrict(fake, fake, fake, None, 1, 16, 16, 4, fake, 64, 16, None) == EINVAL
    assert L.hlbm_restrict(fake, fake, fake, fake, 1, 16, 16, 4, fake, 0, 16, None) == EINVAL
    assert L.hlbm_restrict(fake, fake, fake, fake, 0, 16, 16, 4, fake, 64, 16, None) == EINVAL


def test_binding_rejects_buffers_the_abi_cannot_check():
    """The ABI takes raw pointers, so the binding checks a caller's buffer
    (type, device, contiguity, dtype, size) before passing it on."""
    import numpy as np
    import torch
    from paper_2002_03644_amd._lib import _dev_buf
    ok = torch.zeros(16, dtype=torch.float32)
    assert _dev_buf(ok, "cpu", 64, torch.float32) is ok
    with pytest.raises(TypeError):
        _dev_buf(np.zeros(16, dtype=np.float32), "cpu", 64)
    with pytest.raises(ValueError):
        _dev_buf(ok, "cpu", 65)                                   # too short
    with pytest.raises(ValueError):
        _dev_buf(ok, "cpu", 64, torch.float64)                    # wrong dtype
    with pytest.raises(ValueError):
        _dev_buf(torch.zeros(8, 4)[:, ::2], "cpu", 16)            # not contiguous


def test_network_binding_checks_field_extents_and_idx():
    import torch
    from paper_2002_03644_amd._nn import _check_extent, _check_idx
    x = torch.zeros(3, 4, 8, 32)
    _check_extent(x, 4 * 8 * 32, 8 * 32, 3, 8, 32, "x")
    _check_extent(x[1:], 4 * 8 * 32, 8 * 32, 2, 8, 32, "x")       # a view: offset counted
    with pytest.raises(ValueError):
        _check_extent(x, 4 * 8 * 32, 8 * 32, 4, 8, 32, "x")       # one sample too many
    with pytest.raises(ValueError):
        _check_extent(x[1:], 4 * 8 * 32, 8 * 32, 3, 8, 32, "x")
    with pytest.raises(ValueError):
        _check_extent(x.double(), 4 * 8 * 32, 8 * 32, 1, 8, 32, "x")
    _check_idx(None, 5, "cpu")
    _check_idx(torch.zeros(5, dtype=torch.int32), 5, "cpu")
    with pytest.raises(ValueError):
        _check_idx(torch.zeros(4, dtype=torch.int32), 5, "cpu")    # too few entries
    with pytest.raises(ValueError):
        _check_idx(torch.zeros(5, dtype=torch.int64), 5, "cpu")    # wrong dtype


def test_default_plans_are_built_shapes():
    """Over grids from 1 x 1 to 15446^2 (periodic and extrapolated, FP32 and
    FP64), the default plan names a tile width the kernels are built for
    with that plan and a strip height of at least 1 and at most ny."""
    from paper_2002_03644_amd import launch_plan
    sizes = [1, 2, 5, 31, 64, 65, 100, 200, 511, 512, 640, 700, 767, 768, 1000, 1023, 1024,
             1031, 1500, 2048, 3000, 4096, 6000, 8192, 12288, 15446]
    for dt in ("f32", "f64"):
        for bc in ("periodic", "extrapolate"):
            for nx in sizes:
                for ny in (1, 3, 64, 300, nx):
                    if 9 * nx * ny >= 2 ** 31:
                        continue
                    spl, tw, th = launch_plan(_params(nx=nx, ny=ny, dtype=dt, bc_x=bc))
                    if spl == 2:
                        built = (64, 120, 128, 184) if dt == "f32" else (64, 128)
                    else:
                        built = (64, 128, 192, 256)
                    assert tw in built, (dt, bc, nx, ny, spl, tw)
                    assert 1 <= th <= ny, (dt, bc, nx, ny, spl, th)
                    assert spl == 1 or (bc == "periodic" and dt == "f32"), (dt, bc, nx, ny)
