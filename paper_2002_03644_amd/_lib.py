"""ctypes binding of libhlbm.so (declared in include/hlbm.h).

Argument marshalling only: PyTorch provides device memory and the stream;
every step of the method runs in the library's HIP kernels.  There is no CPU
fallback -- if the library is missing or no GPU is present, calls fail.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhlbm.so")

HLBM_OK, HLBM_WARN_CFL = 0, 1
HLBM_EINVAL, HLBM_EWORKSPACE, HLBM_EHIP, HLBM_EDIVERGED, HLBM_ENOMEM = -1, -2, -3, -4, -5
F64, F32 = 0, 1
BC = {"periodic": 0, "extrapolate": 1, "wall": 2}
PHI = {"lbm": 0, "fd": 1}
BATCH_KERNELS = {"strips": 0, "tiles": 1}   # hlbm_batch_kernel
BATCH_KERNEL_NAMES = {v: k for k, v in BATCH_KERNELS.items()}


class HlbmError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} (code {code})")


class CParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("phi_mode", ctypes.c_int32),
                ("e1_centred", ctypes.c_int32), ("e2_off", ctypes.c_int32),
                ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("prandtl", ctypes.c_double),
                ("mu", ctypes.c_double), ("sigma", ctypes.c_double),
                ("rho_ref", ctypes.c_double), ("theta_ref", ctypes.c_double),
                ("sgn_eps", ctypes.c_double), ("wall_ux_lo", ctypes.c_double),
                ("wall_ux_hi", ctypes.c_double), ("wall_theta", ctypes.c_double),
                ("precise_theta", ctypes.c_int32), ("feq_order", ctypes.c_int32),
                ("steps_per_launch", ctypes.c_int32)]


_lib = None


def lib():
    """Load libhlbm.so (built by paper_2002_03644_amd.build); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2002_03644_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        PP = ctypes.POINTER(CParams)
        dp = ctypes.POINTER(ctypes.c_double)
        sig = {
            "hlbm_workspace_bytes": (sz, [PP]),
            "hlbm_state_bytes": (sz, [PP]),
            "hlbm_launch_shape": (ctypes.c_int, [PP, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
            "hlbm_launch_plan": (ctypes.c_int, [PP, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                                ctypes.POINTER(i32)]),
            "hlbm_validate": (ctypes.c_int, [PP]),
            "hlbm_init": (ctypes.c_int, [ctypes.POINTER(vp), PP, vp, sz, vp, vp, vp, vp, vp]),
            "hlbm_step": (ctypes.c_int, [vp, i32, vp]),
            "hlbm_moments": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp]),
            "hlbm_populations": (ctypes.c_int, [vp, vp, vp]),
            "hlbm_set_populations": (ctypes.c_int, [vp, vp, vp, vp]),
            "hlbm_totals": (ctypes.c_int, [vp, dp, vp]),
            "hlbm_status": (ctypes.c_int, [vp, dp, vp]),
            "hlbm_save_state": (ctypes.c_int, [vp, vp, vp]),
            "hlbm_load_state": (ctypes.c_int, [vp, vp, vp]),
            "hlbm_steps_done": (i64, [vp]),
            "hlbm_destroy": (None, [vp]),
            "hlbm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
            "hlbm_entropy_from_theta": (ctypes.c_int, [i32, ctypes.c_double, vp, vp, vp, i64, vp]),
            "hlbm_state_totals": (ctypes.c_int, [PP, vp, dp, vp]),
            "hlbm_batch_workspace_bytes": (sz, [PP, i32]),
            "hlbm_batch_init": (ctypes.c_int, [ctypes.POINTER(vp), PP, i32, vp, sz, vp, vp, vp, vp,
                                               vp]),
            "hlbm_batch_step": (ctypes.c_int, [vp, i32, i32, vp]),
            "hlbm_batch_moments": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp]),
            "hlbm_batch_status": (ctypes.c_int, [vp, ctypes.POINTER(i32), vp]),
            "hlbm_batch_set_tile": (ctypes.c_int, [vp, i32, i32, vp]),
            "hlbm_batch_set_shape": (ctypes.c_int, [vp, i32, i32, i32, vp]),
            "hlbm_batch_autotune": (ctypes.c_int, [vp, i32, vp, ctypes.POINTER(i32),
                                                   ctypes.POINTER(i32), ctypes.POINTER(i32), vp]),
            "hlbm_batch_state_bytes": (sz, [vp]),
            "hlbm_batch_save_state": (ctypes.c_int, [vp, vp, vp]),
            "hlbm_batch_load_state": (ctypes.c_int, [vp, vp, vp]),
            "hlbm_batch_nodes": (i64, [vp]),
            "hlbm_batch_plan": (ctypes.c_int, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                               ctypes.POINTER(i32), ctypes.POINTER(i32)]),
            "hlbm_batch_steps_done": (i64, [vp]),
            "hlbm_batch_destroy": (None, [vp]),
            # learned closure (include/hlbm_nn.h)
            "hlbm_cnn_workspace_bytes": (sz, [i32, i32, i32]),
            "hlbm_cnn_init": (ctypes.c_int, [ctypes.POINTER(vp), i32, i32, i32, vp, sz, vp, vp]),
            "hlbm_cnn_set_params": (ctypes.c_int, [vp, vp, vp]),
            "hlbm_cnn_get_params": (ctypes.c_int, [vp, vp, vp]),
            "hlbm_cnn_get_grads": (ctypes.c_int, [vp, vp, vp]),
            "hlbm_cnn_set_norm": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_float)]),
            "hlbm_cnn_set_output_clip": (ctypes.c_int, [vp, ctypes.c_float]),
            "hlbm_cnn_set_fused": (ctypes.c_int, [vp, i32]),
            "hlbm_cnn_forward": (ctypes.c_int, [vp, vp, i64, i64, vp, i32, vp, i64, i64, vp]),
            "hlbm_cnn_loss_grad": (ctypes.c_int, [vp, vp, i64, i64, vp, i64, i64, vp, i32, vp,
                                                  vp]),
            "hlbm_cnn_adam": (ctypes.c_int, [vp, ctypes.c_float, vp]),
            "hlbm_cnn_train_step": (ctypes.c_int, [vp, vp, i64, i64, vp, i64, i64, vp, i32,
                                                   ctypes.c_float, vp, vp]),
            "hlbm_cnn_destroy": (None, [vp]),
            "hlbm_restrict": (ctypes.c_int, [vp, vp, vp, vp, i32, i32, i32, i32, vp, i64, i64,
                                             vp]),
            "hlbm_batch_correct": (ctypes.c_int, [vp, vp, vp, i32, vp]),
            "hlbm_closure_step": (ctypes.c_int, [vp, vp, i32, i32, i32, i32, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().hlbm_strerror(int(code)).decode()
    except ImportError:
        return f"status {code}"


def _check(code, what):
    if code < 0:
        raise HlbmError(code, what)
    return code


@dataclass
class Params:
    """Parameters of one domain (mirror of hlbm_params)."""
    nx: int
    ny: int
    dtype: str = "f64"
    gamma: float = 1.4
    prandtl: float = 0.71
    mu: float = 1e-3
    sigma: float = 0.0
    bc_x: str = "periodic"
    bc_y: str = "periodic"
    phi_mode: str = "lbm"
    e1_centred: bool = False
    e2_off: bool = False
    rho_ref: float = 1.0
    theta_ref: float = 240.0 / 1183.0
    tile_w: int = 0
    tile_h: int = 0
    sgn_eps: float = 1e-12
    # bc_y = "wall": x velocities of the walls y = 0 and y = ny - 1, their temperature
    wall_ux_lo: float = 0.0
    wall_ux_hi: float = 0.0
    wall_theta: float = 1.0
    # theta - theta_ref computed accurately relative to the deviation (slow
    # diffusive flows; about 1 % slower)
    precise_theta: bool = False
    # 4: fourth-order Hermite expansion (present model); 3: truncated at third
    # order (the original model, with e1_centred and e2_off)
    feq_order: int = 4
    # 0: automatic (two steps per kernel launch for FP32 domains periodic in
    # both axes), 1 or 2 steps per launch
    steps_per_launch: int = 0

    def c(self) -> CParams:
        return CParams(self.nx, self.ny, BC[self.bc_x], BC[self.bc_y],
                       F64 if self.dtype == "f64" else F32, PHI[self.phi_mode],
                       int(self.e1_centred), int(self.e2_off), int(self.tile_w), int(self.tile_h),
                       self.gamma, self.prandtl, self.mu, self.sigma, self.rho_ref, self.theta_ref,
                       self.sgn_eps, self.wall_ux_lo, self.wall_ux_hi, self.wall_theta,
                       int(self.precise_theta), int(self.feq_order), int(self.steps_per_launch))

    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.dtype == "f64" else torch.float32


def validate(p: Params) -> int:
    cp = p.c()
    return lib().hlbm_validate(ctypes.byref(cp))


def workspace_bytes(p: Params) -> int:
    cp = p.c()
    return int(lib().hlbm_workspace_bytes(ctypes.byref(cp)))


def launch_shape(p: Params):
    """(tile_w, tile_h) that the single-domain step launches for p."""
    cp = p.c()
    w, h = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().hlbm_launch_shape(ctypes.byref(cp), ctypes.byref(w), ctypes.byref(h)),
           "hlbm_launch_shape")
    return int(w.value), int(h.value)


def launch_plan(p: Params):
    """(steps_per_launch, tile_w, tile_h) of hlbm_step for p."""
    cp = p.c()
    n, w, h = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().hlbm_launch_plan(ctypes.byref(cp), ctypes.byref(n), ctypes.byref(w),
                                  ctypes.byref(h)), "hlbm_launch_plan")
    return int(n.value), int(w.value), int(h.value)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dev_buf(t, device, nbytes, dtype=None, what="buffer"):
    """Check that a caller's tensor can back a raw device pointer of at least
    nbytes bytes: a contiguous torch tensor on `device` (of `dtype` if given).
    The ABI cannot check sizes itself, so a short buffer would be read or
    written out of bounds."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor")
    def norm(d):
        d = torch.device(d)
        if d.type == "cuda" and d.index is None:
            d = torch.device("cuda", torch.cuda.current_device())
        return d
    if norm(t.device) != norm(device):
        raise ValueError(f"{what}: on {t.device}, expected {device}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{what}: dtype {t.dtype}, expected {dtype}")
    if t.numel() * t.element_size() < nbytes:
        raise ValueError(f"{what}: {t.numel() * t.element_size()} bytes, need {nbytes}")
    return t


def _workspace(ws, nbytes, device):
    """A caller-given workspace (uint8 tensor of at least nbytes bytes,
    256-byte aligned) or a new one."""
    import torch
    if ws is None:
        return torch.empty(nbytes, dtype=torch.uint8, device=device)
    _dev_buf(ws, device, nbytes, torch.uint8, "workspace")
    if ws.data_ptr() % 256:
        raise ValueError("workspace: must be 256-byte aligned")
    return ws


def _dev_field(a, p: Params, device):
    import torch
    t = torch.as_tensor(a)
    t = t.to(device=device, dtype=p.torch_dtype).contiguous()
    if t.numel() != p.nx * p.ny:
        raise ValueError("field size does not match nx * ny")
    return t.reshape(p.ny, p.nx)


def entropy_from_theta(rho, theta, gamma, dtype="f64", device="cuda"):
    """s = c_v ln(theta / rho^(gamma - 1)) on the GPU."""
    import torch
    td = torch.float64 if dtype == "f64" else torch.float32
    r = torch.as_tensor(rho).to(device=device, dtype=td).contiguous()
    th = torch.as_tensor(theta).to(device=device, dtype=td).contiguous()
    if th.numel() != r.numel():
        raise ValueError("entropy_from_theta: rho and theta differ in size")
    s = torch.empty_like(r)
    _check(lib().hlbm_entropy_from_theta(F64 if dtype == "f64" else F32, float(gamma), _ptr(r),
                                         _ptr(th), _ptr(s), r.numel(), _stream()),
           "hlbm_entropy_from_theta")
    return s


def state_totals(p: Params, state, stream=None):
    """hlbm_state_totals: conservation totals of a raw state buffer (a
    device uint8 tensor of hlbm_state_bytes(p) bytes, e.g. from
    Solver.save_state), with the library's static scratch (no allocation)."""
    cp = p.c()
    _dev_buf(state, state.device, lib().hlbm_state_bytes(ctypes.byref(cp)), what="state")
    out = (ctypes.c_double * 4)()
    _check(lib().hlbm_state_totals(ctypes.byref(cp), _ptr(state), out, _stream(stream)),
           "hlbm_state_totals")
    return np.array(out[:])


class Solver:
    """One HLBM domain on the GPU.  Fields are torch tensors (or numpy arrays,
    copied to the device); either s or theta is given."""

    def __init__(self, params: Params, rho, ux, uy, s=None, theta=None, device="cuda",
                 workspace=None):
        import torch
        self.p = params
        self.device = torch.device(device)
        rho = _dev_field(rho, params, self.device)
        ux = _dev_field(ux, params, self.device)
        uy = _dev_field(uy, params, self.device)
        if s is None:
            th = _dev_field(theta, params, self.device)
            s = entropy_from_theta(rho, th, params.gamma, params.dtype, self.device)
        s = _dev_field(s, params, self.device)
        self._cp = params.c()
        nbytes = lib().hlbm_workspace_bytes(ctypes.byref(self._cp))
        if nbytes == 0:
            raise HlbmError(HLBM_EINVAL, "hlbm_workspace_bytes")
        self.workspace = _workspace(workspace, nbytes, self.device)
        h = ctypes.c_void_p()
        code = lib().hlbm_init(ctypes.byref(h), ctypes.byref(self._cp), _ptr(self.workspace),
                               nbytes, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(s), _stream())
        _check(code, "hlbm_init")
        self.init_code = code
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            lib().hlbm_destroy(h)
            self.h = None

    @property
    def steps(self) -> int:
        return int(lib().hlbm_steps_done(self.h))

    def step(self, n=1, stream=None):
        _check(lib().hlbm_step(self.h, int(n), _stream(stream)), "hlbm_step")
        return self

    def _empty(self, *shape):
        import torch
        return torch.empty(*shape, dtype=self.p.torch_dtype, device=self.device)

    def moments(self):
        out = {k: self._empty(self.p.ny, self.p.nx) for k in ("rho", "ux", "uy", "s", "theta")}
        _check(lib().hlbm_moments(self.h, _ptr(out["rho"]), _ptr(out["ux"]), _ptr(out["uy"]),
                                  _ptr(out["s"]), _ptr(out["theta"]), _stream()), "hlbm_moments")
        return out

    def populations(self):
        F = self._empty(9, self.p.ny, self.p.nx)
        _check(lib().hlbm_populations(self.h, _ptr(F), _stream()), "hlbm_populations")
        return F

    def set_populations(self, F, s):
        import torch
        F = torch.as_tensor(F).to(self.device, self.p.torch_dtype).contiguous()
        s = torch.as_tensor(s).to(self.device, self.p.torch_dtype).contiguous()
        n = self.p.nx * self.p.ny
        if F.numel() != 9 * n or s.numel() != n:
            raise ValueError("set_populations: F must hold 9 nx ny values and s nx ny")
        _check(lib().hlbm_set_populations(self.h, _ptr(F), _ptr(s), _stream()),
               "hlbm_set_populations")

    def totals(self):
        out = (ctypes.c_double * 4)()
        _check(lib().hlbm_totals(self.h, out, _stream()), "hlbm_totals")
        return np.array(out[:])

    def status(self):
        cfl = ctypes.c_double(0.0)
        code = lib().hlbm_status(self.h, ctypes.byref(cfl), _stream())
        if code not in (HLBM_OK, HLBM_EDIVERGED):
            raise HlbmError(code, "hlbm_status")
        return code, cfl.value

    def save_state(self):
        import torch
        n = lib().hlbm_state_bytes(ctypes.byref(self._cp))
        buf = torch.empty(n, dtype=torch.uint8, device=self.device)
        _check(lib().hlbm_save_state(self.h, _ptr(buf), _stream()), "hlbm_save_state")
        return buf

    def load_state(self, buf):
        _dev_buf(buf, self.device, lib().hlbm_state_bytes(ctypes.byref(self._cp)),
                 what="load_state")
        _check(lib().hlbm_load_state(self.h, _ptr(buf), _stream()), "hlbm_load_state")


class BatchSolver:
    """Many independent domains advanced by one persistent launch per step.

    ``params``: list of Params (one dtype); ``fields``: list of (rho, ux, uy,
    theta) per domain (host or device arrays).  Graph replay needs a
    non-default stream, so the solver owns one and orders it after the
    caller's current stream."""

    def __init__(self, params, fields, device="cuda", workspace=None):
        import torch
        if len(params) != len(fields) or not params:
            raise ValueError("one field tuple per parameter set")
        self.params = list(params)
        self.device = torch.device(device)
        td = self.params[0].torch_dtype
        self.sizes = [p.nx * p.ny for p in self.params]
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        n = int(self.offsets[-1])
        cat = [torch.empty(n, dtype=td, device=self.device) for _ in range(3)]
        s_all = torch.empty(n, dtype=td, device=self.device)
        for k, (p, f) in enumerate(zip(self.params, fields)):
            a, b = int(self.offsets[k]), int(self.offsets[k + 1])
            rho = _dev_field(f[0], p, self.device).reshape(-1)
            cat[0][a:b] = rho
            cat[1][a:b] = _dev_field(f[1], p, self.device).reshape(-1)
            cat[2][a:b] = _dev_field(f[2], p, self.device).reshape(-1)
            th = _dev_field(f[3], p, self.device).reshape(-1)
            s_all[a:b] = entropy_from_theta(rho, th, p.gamma, p.dtype, self.device)
        arr = (CParams * len(self.params))(*[p.c() for p in self.params])
        self._carr = arr
        nbytes = lib().hlbm_batch_workspace_bytes(arr, len(self.params))
        if nbytes == 0:
            raise HlbmError(HLBM_EINVAL, "hlbm_batch_workspace_bytes")
        self.workspace = _workspace(workspace, nbytes, self.device)
        self.stream = torch.cuda.Stream(device=self.device)  # default priority
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        h = ctypes.c_void_p()
        _check(lib().hlbm_batch_init(ctypes.byref(h), arr, len(self.params), _ptr(self.workspace),
                                     nbytes, _ptr(cat[0]), _ptr(cat[1]), _ptr(cat[2]),
                                     _ptr(s_all), _stream(self.stream)), "hlbm_batch_init")
        self.h = h
        self.nodes = int(lib().hlbm_batch_nodes(h))

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            lib().hlbm_batch_destroy(h)
            self.h = None

    @property
    def steps(self):
        return int(lib().hlbm_batch_steps_done(self.h))

    def plan(self):
        """(steps_per_launch, kernel, tile_w, tile_h) of the batch kernel;
        kernel is "strips" or "tiles" (see set_tile)."""
        n, k, w, h = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().hlbm_batch_plan(self.h, ctypes.byref(n), ctypes.byref(k), ctypes.byref(w),
                                     ctypes.byref(h)), "hlbm_batch_plan")
        return int(n.value), BATCH_KERNEL_NAMES[k.value], int(w.value), int(h.value)

    def _enter(self):
        import torch
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        import torch
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def step(self, n=1, graph=True):
        self._enter()
        _check(lib().hlbm_batch_step(self.h, int(n), int(bool(graph)), _stream(self.stream)),
               "hlbm_batch_step")
        self._leave()
        return self

    def moments_cat(self, out=None, keys=("rho", "ux", "uy", "s", "theta")):
        """Concatenated fields of all domains: dict of 1-D tensors.  With
        ``out`` (a [len(keys)][nodes] tensor) the fields are written there."""
        import torch
        td = self.params[0].torch_dtype
        n = int(self.offsets[-1])
        if out is None:
            out = torch.empty(len(keys), n, dtype=td, device=self.device)
        elif tuple(out.shape) != (len(keys), n):
            raise ValueError(f"moments_cat: out must be [{len(keys)}][{n}]")
        _dev_buf(out, self.device, 0, td, "moments_cat out")
        cat = {k: out[j] for j, k in enumerate(keys)}
        self._enter()
        _check(lib().hlbm_batch_moments(self.h, _ptr(cat.get("rho")), _ptr(cat.get("ux")),
                                        _ptr(cat.get("uy")), _ptr(cat.get("s")),
                                        _ptr(cat.get("theta")), _stream(self.stream)),
               "hlbm_batch_moments")
        self._leave()
        return cat

    def moments(self):
        """List of per-domain dicts of [ny][nx] tensors (views of one buffer)."""
        cat = self.moments_cat()
        out = []
        for k, p in enumerate(self.params):
            a, b = int(self.offsets[k]), int(self.offsets[k + 1])
            out.append({key: v[a:b].view(p.ny, p.nx) for key, v in cat.items()})
        return out

    def status(self):
        flags = (ctypes.c_int32 * len(self.params))()
        self._enter()
        bad = _check(lib().hlbm_batch_status(self.h, flags, _stream(self.stream)),
                     "hlbm_batch_status")
        return bad, np.array(flags[:], dtype=np.int32)

    def set_tile(self, tile_w, tile_h, kernel="strips"):
        """Kernel of the batched step and its tile shape: "strips" (row
        strips of tile_w columns, tile_h rows) or "tiles" (tile_w x tile_h
        tiles, one step per launch)."""
        if kernel not in BATCH_KERNELS:
            raise ValueError(f"batch kernel {kernel!r}: expected one of {sorted(BATCH_KERNELS)}")
        self._enter()
        _check(lib().hlbm_batch_set_shape(self.h, BATCH_KERNELS[kernel], int(tile_w), int(tile_h),
                                          _stream(self.stream)), "hlbm_batch_set_shape")

    def save_state(self):
        import torch
        buf = torch.empty(lib().hlbm_batch_state_bytes(self.h), dtype=torch.uint8,
                          device=self.device)
        self._enter()
        _check(lib().hlbm_batch_save_state(self.h, _ptr(buf), _stream(self.stream)),
               "hlbm_batch_save_state")
        self._leave()
        return buf

    def load_state(self, buf):
        _dev_buf(buf, self.device, lib().hlbm_batch_state_bytes(self.h), what="load_state")
        self._enter()
        _check(lib().hlbm_batch_load_state(self.h, _ptr(buf), _stream(self.stream)),
               "hlbm_batch_load_state")
        self._leave()

    def correct(self, x, delta, conserve=True):
        """Apply increments ``delta`` to moments ``x`` (both [4][count][ny nx]
        float32 device tensors) of an FP32 batch of equal-size domains."""
        import torch
        for t, what in ((x, "correct x"), (delta, "correct delta")):
            _dev_buf(t, self.device, 4 * self.nodes * 4, torch.float32, what)
        self._enter()
        _check(lib().hlbm_batch_correct(self.h, _ptr(x), _ptr(delta), int(bool(conserve)),
                                        _stream(self.stream)), "hlbm_batch_correct")
        self._leave()

    def closure_step(self, net, n=1, every=1, conserve=True, graph=True):
        """n cycles of `every` steps, each cycle followed by the network's
        correction."""
        self._enter()
        _check(lib().hlbm_closure_step(self.h, net.h, int(n), int(every), int(bool(conserve)),
                                       int(bool(graph)), _stream(self.stream)),
               "hlbm_closure_step")
        self._leave()
        return self

    def signature(self):
        import hashlib
        key = ";".join(f"{p.nx}x{p.ny}:{p.dtype}" for p in self.params)
        return hashlib.sha256(key.encode()).hexdigest()[:20]

    def autotune(self, steps=10, cache_path=None):
        """Pick the fastest kernel and tile shape by timing and return
        (kernel, tile_w, tile_h); every shape is timed from the same state,
        which is restored afterwards (flags and step count too).  With
        ``cache_path`` the choice is read from / written to a JSON file keyed
        by the batch's domain sizes and dtype."""
        import json
        sig = self.signature()
        cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as fh:
                cache = json.load(fh)
            if sig in cache and len(cache[sig]) == 3:
                k, w, h = cache[sig]
                self.set_tile(w, h, k)
                return k, int(w), int(h)
        import torch
        scratch = torch.empty(lib().hlbm_batch_state_bytes(self.h), dtype=torch.uint8,
                              device=self.device)
        bk, bw, bh = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        self._enter()
        _check(lib().hlbm_batch_autotune(self.h, int(steps), _ptr(scratch), ctypes.byref(bk),
                                         ctypes.byref(bw),
                                         ctypes.byref(bh), _stream(self.stream)),
               "hlbm_batch_autotune")
        self._leave()
        del scratch
        kernel = BATCH_KERNEL_NAMES[bk.value]
        if cache_path:
            cache[sig] = [kernel, bw.value, bh.value]
            os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
            with open(cache_path, "w") as fh:
                json.dump(cache, fh, indent=1)
        return kernel, bw.value, bh.value
