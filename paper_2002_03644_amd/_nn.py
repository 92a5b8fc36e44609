"""Binding of the learned closure (include/hlbm_nn.h): argument marshalling
only -- the network's forward and backward passes, Adam and the restriction
run in the library's HIP kernels."""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import HLBM_EINVAL, HlbmError, _check, _ptr, _stream, _workspace, lib

N_PARAMS = 11588


def _field_strides(t, ny, nx, what):
    """(sample, channel) strides of a [S][4][ny][nx] float32 tensor whose
    [ny][nx] planes are contiguous (any sample / channel strides)."""
    import torch
    if t.dtype != torch.float32 or t.dim() != 4 or t.shape[1] != 4 or t.shape[2:] != (ny, nx):
        raise ValueError(f"{what}: expected a float32 [S][4][{ny}][{nx}] tensor")
    if t.stride(3) != 1 or t.stride(2) != nx:
        raise ValueError(f"{what}: [ny][nx] planes must be contiguous")
    return t.stride(0), t.stride(1)


def _check_extent(t, sb, sc, nsamp, ny, nx, what):
    """The kernels read or write element s sb + c sc + i (s < nsamp, c < 4,
    i < ny nx) from t's first element on; all of it must lie in t's storage."""
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32:
        raise ValueError(f"{what}: expected a float32 torch tensor")
    avail = t.untyped_storage().nbytes() // t.element_size() - t.storage_offset()
    need = (nsamp - 1) * sb + 3 * sc + ny * nx
    if nsamp < 1 or sb < 0 or sc < 0 or need > avail:
        raise ValueError(f"{what}: {nsamp} samples with strides ({sb}, {sc}) need {need} "
                         f"elements, the tensor has {avail}")


def _check_idx(idx, batch, device):
    """idx: int32 device tensor of at least `batch` entries.  Its values must
    be sample indices of x (and target); they are not read back here, which
    would synchronise the stream on every training step."""
    import torch
    if idx is None:
        return
    if not isinstance(idx, torch.Tensor) or idx.dtype != torch.int32 or not idx.is_contiguous():
        raise ValueError("idx: expected a contiguous int32 torch tensor")
    if idx.device.type != torch.device(device).type or idx.numel() < batch:
        raise ValueError(f"idx: needs {batch} entries on the network's device")


def _f32(t, device):
    import torch
    return torch.as_tensor(t).to(device=device, dtype=torch.float32).contiguous()


class CNN:
    """The 4 -> 32 -> 32 -> 4 closure network for batches of up to
    ``max_batch`` fields of ny x nx.  Field batches are float32 device tensors
    addressed as x[s * sstride + c * cstride + i]; a [S][4][ny][nx] tensor
    has sstride 4 ny nx and cstride ny nx (the defaults)."""

    def __init__(self, max_batch, ny, nx, params, device="cuda", workspace=None):
        import torch
        self.device = torch.device(device)
        self.max_batch, self.ny, self.nx = int(max_batch), int(ny), int(nx)
        nbytes = lib().hlbm_cnn_workspace_bytes(self.max_batch, self.ny, self.nx)
        if nbytes == 0:
            raise HlbmError(HLBM_EINVAL, "hlbm_cnn_workspace_bytes")
        self.workspace = _workspace(workspace, nbytes, self.device)
        p = _f32(params, self.device).reshape(-1)
        if p.numel() != N_PARAMS:
            raise ValueError(f"expected {N_PARAMS} parameters")
        h = ctypes.c_void_p()
        _check(lib().hlbm_cnn_init(ctypes.byref(h), self.max_batch, self.ny, self.nx,
                                   _ptr(self.workspace), nbytes, _ptr(p), _stream()),
               "hlbm_cnn_init")
        self.h = h
        self.norm = np.array([0, 0, 0, 0, 1, 1, 1, 1, 0, 0, 0, 0, 1, 1, 1, 1], np.float32)
        self.clip = 0.0

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            lib().hlbm_cnn_destroy(h)
            self.h = None

    def set_params(self, params):
        p = _f32(params, self.device).reshape(-1)
        _check(lib().hlbm_cnn_set_params(self.h, _ptr(p), _stream()), "hlbm_cnn_set_params")

    def params(self):
        import torch
        out = torch.empty(N_PARAMS, dtype=torch.float32, device=self.device)
        _check(lib().hlbm_cnn_get_params(self.h, _ptr(out), _stream()), "hlbm_cnn_get_params")
        return out

    def grads(self):
        import torch
        out = torch.empty(N_PARAMS, dtype=torch.float32, device=self.device)
        _check(lib().hlbm_cnn_get_grads(self.h, _ptr(out), _stream()), "hlbm_cnn_get_grads")
        return out

    def set_norm(self, in_mean, in_std, out_mean, out_std):
        norm = np.concatenate([in_mean, in_std, out_mean, out_std]).astype(np.float32)
        arr = (ctypes.c_float * 16)(*norm.tolist())
        _check(lib().hlbm_cnn_set_norm(self.h, arr), "hlbm_cnn_set_norm")
        self.norm = norm

    def set_output_clip(self, clip):
        """Clamp the standardised inference output to [-clip, clip] (0: off)."""
        _check(lib().hlbm_cnn_set_output_clip(self.h, float(clip)), "hlbm_cnn_set_output_clip")
        self.clip = float(clip)

    def set_fused(self, enable):
        """Inference in one fused kernel (True, the default) or per layer."""
        _check(lib().hlbm_cnn_set_fused(self.h, int(bool(enable))), "hlbm_cnn_set_fused")

    def _strides(self, t, sstride, cstride, what="x"):
        """Explicit strides, or those of a [S][4][ny][nx] tensor."""
        if sstride is not None and cstride is not None:
            return int(sstride), int(cstride)
        return _field_strides(t, self.ny, self.nx, what)

    def _check_pair(self, x, sb, sc, target, tsb, tsc, batch, idx):
        _check_idx(idx, batch, self.device)
        if idx is None:
            _check_extent(x, sb, sc, batch, self.ny, self.nx, "x")
            _check_extent(target, tsb, tsc, batch, self.ny, self.nx, "target")

    def forward(self, x, batch=None, idx=None, sstride=None, cstride=None, out=None):
        """Raw increments [batch][4][ny][nx] for the fields x."""
        import torch
        sb, sc = self._strides(x, sstride, cstride)
        batch = int(batch if batch is not None else (len(idx) if idx is not None else x.shape[0]))
        if out is None:
            out = torch.empty(batch, 4, self.ny, self.nx, dtype=torch.float32, device=self.device)
        osb, osc = _field_strides(out, self.ny, self.nx, "out")
        _check_idx(idx, batch, self.device)
        if idx is None:
            _check_extent(x, sb, sc, batch, self.ny, self.nx, "x")
        _check_extent(out, osb, osc, batch, self.ny, self.nx, "out")
        _check(lib().hlbm_cnn_forward(self.h, _ptr(x), sb, sc, _ptr(idx), batch, _ptr(out),
                                      osb, osc, _stream()), "hlbm_cnn_forward")
        return out

    def loss_grad(self, x, target, batch=None, idx=None, sstride=None, cstride=None,
                  t_sstride=None, t_cstride=None, loss=None):
        import torch
        sb, sc = self._strides(x, sstride, cstride)
        tsb, tsc = self._strides(target, t_sstride, t_cstride, "target")
        batch = int(batch if batch is not None else (len(idx) if idx is not None else x.shape[0]))
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=self.device)
        self._check_pair(x, sb, sc, target, tsb, tsc, batch, idx)
        _check(lib().hlbm_cnn_loss_grad(self.h, _ptr(x), sb, sc, _ptr(target), tsb, tsc,
                                        _ptr(idx), batch, _ptr(loss), _stream()),
               "hlbm_cnn_loss_grad")
        return loss

    def adam(self, lr):
        return _check(lib().hlbm_cnn_adam(self.h, float(lr), _stream()), "hlbm_cnn_adam")

    def train_step(self, x, target, lr, batch=None, idx=None, sstride=None, cstride=None,
                   t_sstride=None, t_cstride=None, loss=None):
        import torch
        sb, sc = self._strides(x, sstride, cstride)
        tsb, tsc = self._strides(target, t_sstride, t_cstride, "target")
        batch = int(batch if batch is not None else (len(idx) if idx is not None else x.shape[0]))
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=self.device)
        self._check_pair(x, sb, sc, target, tsb, tsc, batch, idx)
        _check(lib().hlbm_cnn_train_step(self.h, _ptr(x), sb, sc, _ptr(target), tsb, tsc,
                                         _ptr(idx), batch, float(lr), _ptr(loss), _stream()),
               "hlbm_cnn_train_step")
        return loss


def restrict(rho, ux, uy, theta, factor, batch=1, out=None):
    """Conservative block-mean restriction of [batch][ny][nx] float32 fields
    to [batch][4][ny/f][nx/f] (rho, u_x, u_y, theta)."""
    import torch
    ny, nx = rho.shape[-2], rho.shape[-1]
    nyc, nxc = ny // factor, nx // factor
    for a in (rho, ux, uy, theta):
        if a.dtype != torch.float32 or not a.is_contiguous() or a.numel() != batch * ny * nx:
            raise ValueError("fine fields: contiguous float32 [batch][ny][nx]")
    if out is None:
        out = torch.empty(batch, 4, nyc, nxc, dtype=torch.float32, device=rho.device)
    if out.shape[0] != batch:
        raise ValueError("out: one entry per batch member")
    osb, osc = _field_strides(out, nyc, nxc, "out")
    _check(lib().hlbm_restrict(_ptr(rho), _ptr(ux), _ptr(uy), _ptr(theta), int(batch), int(ny),
                               int(nx), int(factor), _ptr(out), osb, osc, _stream()),
           "hlbm_restrict")
    return out
