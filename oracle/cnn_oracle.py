"""FP64 numpy oracle of the learned closure -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may use
it.  It defines what the GPU's BF16-MFMA kernels compute:

* restriction R of a fine field onto a grid coarser by a factor f: block
  means rho_c = <rho>, u_c = <rho u> / <rho>, theta_c = <rho theta> / <rho>
  (mass, momentum and rho*theta -- i.e. pressure -- of each block conserved);
* a 3-layer 3x3 convolutional network on the 4 channels (rho, u_x, u_y,
  theta), periodic padding, channels 4 -> 32 -> 32 -> 4, ReLU after the first
  two layers (cross-correlation: out[y, x] = sum_{dy, dx, ci}
  in[y + dy - 1, x + dx - 1, ci] w[dy, dx, ci, co] + b[co]);
* mean-squared-error loss and its exact gradient (reverse mode written out
  layer by layer);
* the Adam update (Kingma & Ba) with bias correction;
* a storage-precision variant of the forward and backward passes
  (``loss_and_grads_stored``) in which every tensor the GPU path keeps in
  BF16 -- the standardised input, the weights, the hidden activations and the
  back-propagated gradients -- is rounded to BF16 (round to nearest, ties to
  even) where it is stored, all arithmetic staying FP64.  Parity of the BF16
  kernels is checked against it.

Arrays are NHWC: [batch, y, x, channel]; weights [3, 3, c_in, c_out].
"""
from __future__ import annotations

import numpy as np

CHANNELS = (4, 32, 32, 4)


def conv3x3(x, w, b):
    """Periodic 3x3 cross-correlation, NHWC."""
    B, H, W, ci = x.shape
    co = w.shape[3]
    out = np.zeros((B, H, W, co))
    for dy in range(3):
        for dx in range(3):
            shifted = np.roll(np.roll(x, -(dy - 1), axis=1), -(dx - 1), axis=2)
            out += shifted @ w[dy, dx]
    return out + b


def conv3x3_grad(x, w, gout):
    """Gradients of sum(gout * conv3x3(x, w, b)) w.r.t. x, w and b."""
    gx = np.zeros_like(x)
    gw = np.zeros_like(w)
    for dy in range(3):
        for dx in range(3):
            shifted = np.roll(np.roll(x, -(dy - 1), axis=1), -(dx - 1), axis=2)
            gw[dy, dx] = np.einsum("byxi,byxo->io", shifted, gout)
            back = gout @ w[dy, dx].T
            gx += np.roll(np.roll(back, dy - 1, axis=1), dx - 1, axis=2)
    gb = gout.sum(axis=(0, 1, 2))
    return gx, gw, gb


def bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64:
    the float32 bit pattern with its low 16 bits rounded away."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(seed=0):
    """He-uniform weights, zero biases; the last layer scaled down so the
    initial correction is small."""
    rng = np.random.default_rng(seed)
    params = []
    for k in range(3):
        ci, co = CHANNELS[k], CHANNELS[k + 1]
        bound = np.sqrt(6.0 / (9 * ci))
        w = rng.uniform(-bound, bound, size=(3, 3, ci, co))
        if k == 2:
            w *= 0.1
        params.append((w, np.zeros(co)))
    return params


def forward(params, x):
    """Returns the output and the per-layer inputs/pre-activations."""
    acts = [x]
    zs = []
    h = x
    for k, (w, b) in enumerate(params):
        z = conv3x3(h, w, b)
        zs.append(z)
        h = np.maximum(z, 0.0) if k < 2 else z
        acts.append(h)
    return h, acts, zs


def loss_and_grads(params, x, target):
    """Mean-squared error over all output elements and its gradients."""
    y, acts, zs = forward(params, x)
    n = y.size
    diff = y - target
    loss = float((diff * diff).sum() / n)
    g = 2.0 * diff / n
    grads = [None] * 3
    for k in (2, 1, 0):
        if k < 2:
            g = g * (zs[k] > 0)
        gx, gw, gb = conv3x3_grad(acts[k], params[k][0], g)
        grads[k] = (gw, gb)
        g = gx
    return loss, grads


class Adam:
    """Adam with bias correction: m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
    p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)."""

    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.t = 0
        self.m = [[np.zeros_like(p) for p in layer] for layer in params]
        self.v = [[np.zeros_like(p) for p in layer] for layer in params]

    def step(self, params, grads):
        self.t += 1
        out = []
        for k, layer in enumerate(params):
            new = []
            for j, p in enumerate(layer):
                g = grads[k][j]
                self.m[k][j] = self.b1 * self.m[k][j] + (1 - self.b1) * g
                self.v[k][j] = self.b2 * self.v[k][j] + (1 - self.b2) * g * g
                mh = self.m[k][j] / (1 - self.b1 ** self.t)
                vh = self.v[k][j] / (1 - self.b2 ** self.t)
                new.append(p - self.lr * mh / (np.sqrt(vh) + self.eps))
            out.append(tuple(new))
        return out


def restrict(rho, ux, uy, theta, factor):
    """Block means of mass, momentum and rho*theta over factor x factor blocks."""
    ny, nx = rho.shape
    shp = (ny // factor, factor, nx // factor, factor)

    def bmean(a):
        return a.reshape(shp).mean(axis=(1, 3))

    rc = bmean(rho)
    return rc, bmean(rho * ux) / rc, bmean(rho * uy) / rc, bmean(rho * theta) / rc


def forward_stored(params, x):
    """Forward pass with BF16 storage of input, weights and hidden
    activations (biases and the output stay unrounded)."""
    h = bf16(x)
    acts = [h]
    for k, (w, b) in enumerate(params):
        z = conv3x3(h, bf16(w), b)
        if k < 2:
            h = bf16(np.maximum(z, 0.0))
            acts.append(h)
        else:
            h = z
    return h, acts


def loss_and_grads_stored(params, x, target):
    """MSE loss and parameter gradients with BF16 storage of the output
    gradient and of the gradients passed back through each hidden layer; the
    ReLU mask is taken from the stored activation (a > 0)."""
    y, acts = forward_stored(params, x)
    n = y.size
    diff = y - target
    loss = float((diff * diff).sum() / n)
    g = bf16(2.0 * diff / n)
    grads = [None] * 3
    for k in (2, 1, 0):
        gx, gw, gb = conv3x3_grad(acts[k], bf16(params[k][0]), g)
        grads[k] = (gw, gb)
        if k > 0:
            g = bf16(gx * (acts[k] > 0))
    return loss, grads


def flatten(params):
    """Canonical parameter vector: per layer the weights [3][3][c_in][c_out]
    then the biases."""
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])


def unflatten(vec):
    out, o = [], 0
    for k in range(3):
        ci, co = CHANNELS[k], CHANNELS[k + 1]
        nw = 9 * ci * co
        out.append((np.asarray(vec[o:o + nw], dtype=np.float64).reshape(3, 3, ci, co),
                    np.asarray(vec[o + nw:o + nw + co], dtype=np.float64)))
        o += nw + co
    return out


def apply_correction(rho, ux, uy, theta, d, conserve=True):
    """Corrected moments of one domain: rho' = rho + d_rho - a,
    rho' u' = rho' (u + d_u) - b, theta' = theta + d_theta, where a = <d_rho>
    and b = <(rho + d_rho)(u + d_u) - rho u> - a <u + d_u> keep the total mass
    and momentum (a = b = 0 without conservation)."""
    dr, du, dv, dt = d
    a = dr.mean() if conserve else 0.0
    bx = ((rho + dr) * (ux + du) - rho * ux).mean() - a * (ux + du).mean() if conserve else 0.0
    by = ((rho + dr) * (uy + dv) - rho * uy).mean() - a * (uy + dv).mean() if conserve else 0.0
    r2 = rho + dr - a
    return r2, (ux + du) - bx / r2, (uy + dv) - by / r2, theta + dt
