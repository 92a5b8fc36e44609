"""Learned closure for coarse HLBM runs: data generation, training and
evaluation, all on the GPU through the library (include/hlbm.h,
include/hlbm_nn.h).

Setup (the method's own data; the paper has no learned component):
* fine runs: decaying compressible turbulence on a periodic fine_n^2 grid
  (random-phase solenoidal velocity, E(k) ~ k^4 exp(-2 (k/8)^2), uniform
  rho = 1 and theta), turbulent Mach number drawn per seed in mach_range,
  theta from the CFL rule with M_max = 3 Ma_t, dynamic viscosity mu_fine;
* coarse runs: the same flow on a grid coarser by `factor`, in acoustic
  scaling (one coarse step = factor fine steps, mu_coarse = mu_fine /
  factor), initialised from the conservative block-mean restriction R of
  the fine state;
* training pairs, per coarse step n: input Y_n = moments after `every`
  plain coarse steps from R(fine_{factor n}), target
  D_n = R(fine_{factor (n+every)}) - Y_n, on (rho, u_x, u_y, theta),
  per-channel standardised;
* inference: after every `every` coarse steps X <- X + CNN(X) with the mass
  and momentum of each domain kept (hlbm_closure_step);
* reference: the fine run restricted to the coarse grid; density error
  e = ||rho - rho_fine||_2 / ||rho_fine - <rho_fine>||_2 averaged over the
  held-out seeds and the checkpoints;
* plain ladder: plain runs at intermediate resolutions N (initialised from
  the Fourier-truncated fine initial field, mu = mu_fine N / fine_n,
  N / coarse_n steps per coarse step), restricted to the coarse grid by
  area-weighted averaging, give e(N) and their wall time t(N).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

import hlbm_inputs as hi

from ._lib import BatchSolver, HlbmError, Params
from ._nn import CNN, restrict


@dataclass
class ClosureSetup:
    fine_n: int = 1024
    factor: int = 4
    mu_fine: float = 4e-3
    coarse_steps: int = 250
    mach_range: tuple = (0.25, 0.45)   # turbulent Mach numbers the plain runs survive
    gamma: float = 1.4
    train_seeds: tuple = tuple(range(1000, 1064))
    eval_seeds: tuple = tuple(range(2000, 2008))
    checkpoints: tuple = (50, 100, 150, 200, 250)
    ladder: tuple = (384, 512, 768)
    chunk: int = 16            # fine domains per batched run
    every: int = 10            # coarse steps per correction

    @property
    def coarse_n(self):
        return self.fine_n // self.factor

    @property
    def mu_coarse(self):
        return self.mu_fine / self.factor


def seed_flow(seed, setup: ClosureSetup):
    """Turbulent Mach number and temperature of one seed's flow."""
    rng = np.random.default_rng(seed + 7919)
    mach = float(rng.uniform(*setup.mach_range))
    return mach, hi.theta_for_cfl(3.0 * mach, setup.gamma)


def fine_initial(seed, setup: ClosureSetup):
    mach, theta = seed_flow(seed, setup)
    return hi.turbulence(setup.fine_n, mach, theta, seed, gamma=setup.gamma)


def _params(n, mu, theta, setup):
    return Params(n, n, dtype="f32", gamma=setup.gamma, mu=mu, sigma=0.0, theta_ref=theta)


def restricted_trajectories(seeds, setup: ClosureSetup, steps=None, device="cuda"):
    """R(fine_{factor n}) for n = 0..steps of every seed: a float32 device
    tensor [len(seeds)][steps + 1][4][nc][nc], and the per-seed divergence
    flags of the fine runs."""
    import torch
    steps = setup.coarse_steps if steps is None else steps
    nc, nf = setup.coarse_n, setup.fine_n
    out = torch.empty(len(seeds), steps + 1, 4, nc, nc, dtype=torch.float32, device=device)
    flags = np.zeros(len(seeds), np.int32)
    for c0 in range(0, len(seeds), setup.chunk):
        chunk = list(seeds[c0:c0 + setup.chunk])
        params = [_params(nf, setup.mu_fine, seed_flow(s, setup)[1], setup) for s in chunk]
        B = BatchSolver(params, [fine_initial(s, setup) for s in chunk], device=device)
        buf = torch.empty(4, len(chunk) * nf * nf, dtype=torch.float32, device=device)
        for n in range(steps + 1):
            cat = B.moments_cat(out=buf, keys=("rho", "ux", "uy", "theta"))
            B.stream.synchronize()
            f = [cat[k].view(len(chunk), nf, nf) for k in ("rho", "ux", "uy", "theta")]
            restrict(*f, setup.factor, batch=len(chunk), out=out[c0:c0 + len(chunk), n])
            if n < steps:
                B.step(setup.factor, graph=True)
        flags[c0:c0 + len(chunk)] = B.status()[1]
        del B
    torch.cuda.synchronize()
    return out, flags


def coarse_one_step(X, thetas, setup: ClosureSetup, chunk=256, steps=1):
    """Moments after `steps` plain coarse steps from each state X[m] (float32
    [M][4][nc][nc]); thetas[m] is the storage reference of sample m."""
    import torch
    nc = setup.coarse_n
    Y = torch.empty_like(X)
    for c0 in range(0, X.shape[0], chunk):
        m = min(chunk, X.shape[0] - c0)
        params = [_params(nc, setup.mu_coarse, float(thetas[c0 + j]), setup) for j in range(m)]
        fields = [(X[c0 + j, 0], X[c0 + j, 1], X[c0 + j, 2], X[c0 + j, 3]) for j in range(m)]
        B = BatchSolver(params, fields, device=X.device)
        B.step(steps, graph=False)
        buf = torch.empty(4, m * nc * nc, dtype=torch.float32, device=X.device)
        B.moments_cat(out=buf, keys=("rho", "ux", "uy", "theta"))
        B.stream.synchronize()
        Y[c0:c0 + m] = buf.view(4, m, nc, nc).permute(1, 0, 2, 3)
        del B
    return Y


def training_pairs(traj, seeds, setup: ClosureSetup):
    """Inputs Y_n and targets D_n = X_{n+every} - Y_n of every seed and
    start n, flattened to [S][4][nc][nc] each."""
    k = setup.every
    S, T1 = traj.shape[0], traj.shape[1]
    X = traj[:, :-k].reshape(S * (T1 - k), 4, setup.coarse_n, setup.coarse_n)
    thetas = np.repeat([seed_flow(s, setup)[1] for s in seeds], T1 - k)
    Y = coarse_one_step(X, thetas, setup, steps=k)
    D = traj[:, k:].reshape_as(Y) - Y
    return Y, D


def channel_stats(A):
    """Per-channel mean and standard deviation of [S][4][..] (FP64 sums)."""
    a = A.transpose(0, 1).reshape(4, -1).double()
    mean = a.mean(dim=1)
    std = a.std(dim=1).clamp_min(1e-12)
    return mean.float().cpu().numpy(), std.float().cpu().numpy()


def train(net: CNN, Y, D, steps, batch=32, lr=2e-3, seed=0, log_every=500, lr_final=None):
    """Adam on random minibatches of the pairs (Y, D); cosine learning-rate
    decay from lr to lr_final.  Returns the logged (step, loss) pairs."""
    import torch
    g = torch.Generator(device=Y.device)
    g.manual_seed(seed)
    S = Y.shape[0]
    lr_final = lr * 0.05 if lr_final is None else lr_final
    log = []
    loss = torch.zeros(1, dtype=torch.float32, device=Y.device)
    for k in range(steps):
        idx = torch.randint(0, S, (batch,), generator=g, device=Y.device, dtype=torch.int32)
        lr_k = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * k / max(1, steps)))
        net.train_step(Y, D, lr_k, idx=idx, loss=loss)
        if log_every and (k % log_every == 0 or k == steps - 1):
            log.append((k, float(loss.item())))
    return log


def area_matrix(n_from, n_to, device):
    """Averaging matrix [n_to][n_from]: overlap of target cell i (width
    n_from / n_to) with source cell k, divided by the target width."""
    import torch
    r = n_from / n_to
    A = np.zeros((n_to, n_from))
    for i in range(n_to):
        a, b = i * r, (i + 1) * r
        for k in range(int(math.floor(a)), int(math.ceil(b))):
            A[i, k] = (min(b, k + 1) - max(a, k)) / r
    return torch.from_numpy(A).to(device)


def to_coarse(rho, ux, uy, n_to):
    """Density-weighted area average of [B][N][N] fields to n_to^2 (FP64):
    rho_c = A rho A^T, u_c = A (rho u) A^T / rho_c."""
    A = area_matrix(rho.shape[-1], n_to, rho.device)
    r = rho.double()
    rc = A @ r @ A.T
    return rc, (A @ (r * ux.double()) @ A.T) / rc, (A @ (r * uy.double()) @ A.T) / rc


def fourier_resample(a, n):
    """Samples on an n x n grid (n <= N) of the Fourier series of a periodic
    [N][N] field truncated to |k_x|, |k_y| < n / 2."""
    N = a.shape[0]
    if n == N:
        return np.array(a, dtype=np.float64)
    if n > N:
        raise ValueError("resampling to a finer grid is not needed here")
    F = np.fft.rfft2(a)
    k = n // 2
    G = np.zeros((n, n // 2 + 1), complex)
    G[:k, :k] = F[:k, :k]
    G[n - k + 1:, :k] = F[N - k + 1:, :k]
    return np.fft.irfft2(G, s=(n, n)) * (n * n) / (N * N)


def density_error(rho, fine_ref):
    """||rho - fine_ref||_2 / ||fine_ref - <fine_ref>||_2 per sample."""
    d = (rho.double() - fine_ref.double()).flatten(1)
    j = fine_ref.double().flatten(1)
    j = j - j.mean(dim=1, keepdim=True)
    return (d.norm(dim=1) / j.norm(dim=1)).cpu().numpy()


def _time(fn, stream):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3


@dataclass
class Evaluation:
    e_learned: float
    e_plain: dict          # N -> error (coarse N included, fine_n -> 0)
    t_learned: float       # seconds for coarse_steps corrected steps, all seeds batched
    t_plain: dict          # N -> seconds for the same physical time
    e_learned_curve: list = field(default_factory=list)
    e_plain_curve: dict = field(default_factory=dict)
    diverged: dict = field(default_factory=dict)

    def n_equal_error(self):
        """Resolution N* of the plain ladder with the learned error
        (log-log interpolation; None outside the ladder)."""
        ns = sorted(n for n in self.e_plain if self.e_plain[n] > 0)
        for a, b in zip(ns, ns[1:]):
            ea, eb = self.e_plain[a], self.e_plain[b]
            if (ea - self.e_learned) * (eb - self.e_learned) <= 0 and ea != eb:
                w = (math.log(self.e_learned) - math.log(ea)) / (math.log(eb) - math.log(ea))
                return math.exp(math.log(a) + w * (math.log(b) - math.log(a)))
        return None

    def time_at_equal_error(self):
        """t_plain(N*) / t_learned, t_plain interpolated log-log in N."""
        ns = self.n_equal_error()
        if ns is None:
            return None
        pts = sorted(self.t_plain)
        for a, b in zip(pts, pts[1:]):
            if a <= ns <= b:
                w = (math.log(ns) - math.log(a)) / (math.log(b) - math.log(a))
                t = math.exp(math.log(self.t_plain[a]) + w * (math.log(self.t_plain[b]) -
                                                              math.log(self.t_plain[a])))
                return t / self.t_learned
        return None


def initial_params(seed=0):
    """Canonical parameter vector (float32, 11588): He-uniform weights
    U(-b, b), b = sqrt(6 / (9 c_in)), the last layer scaled by 0.1 so the
    initial correction is small; zero biases."""
    rng = np.random.default_rng(seed)
    chans = (4, 32, 32, 4)
    parts = []
    for k in range(3):
        ci, co = chans[k], chans[k + 1]
        b = math.sqrt(6.0 / (9 * ci))
        w = rng.uniform(-b, b, size=9 * ci * co) * (0.1 if k == 2 else 1.0)
        parts += [w, np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


def build_network(Y, D, setup: ClosureSetup, max_batch=16, seed=0):
    """Network for coarse_n^2 fields with the standardisation of the pairs."""
    net = CNN(max_batch, setup.coarse_n, setup.coarse_n, initial_params(seed), device=Y.device)
    im, istd = channel_stats(Y)
    om, ostd = channel_stats(D)
    net.set_norm(im, istd, om, ostd)
    return net


def fit(setup: ClosureSetup, steps=20000, batch=32, lr=2e-3, clip=4.0, seed=0, log=print):
    """Train the closure network for `setup`: restricted fine trajectories of
    the training seeds, the (input, target) pairs, `steps` Adam steps.
    Returns the network (output clamp `clip` set) and a record of the run."""
    import torch
    t0 = time.perf_counter()
    traj, flags = restricted_trajectories(setup.train_seeds, setup)
    Y, D = training_pairs(traj, setup.train_seeds, setup)
    del traj
    rec = {"fine_diverged": int(flags.sum()), "pairs": int(Y.shape[0]),
           "data_s": time.perf_counter() - t0}
    log(f"[closure] {Y.shape[0]} pairs ({setup.every}-step targets) in {rec['data_s']:.1f} s")
    net = build_network(Y, D, setup, max_batch=batch, seed=seed)
    t0 = time.perf_counter()
    rec["loss"] = train(net, Y, D, steps, batch=batch, lr=lr, seed=seed)
    torch.cuda.synchronize()
    rec["train_s"] = time.perf_counter() - t0
    log(f"[closure] {steps} Adam steps (batch {batch}) in {rec['train_s']:.1f} s, "
        f"loss {rec['loss'][-1][1]:.4f}")
    del Y, D
    if clip:
        net.set_output_clip(clip)
    return net, rec


def _arm(make, advance, targets, n_res, nc, fine_ref, nseeds):
    """Run one arm to each checkpoint's step count; density errors [cp][seed]."""
    B = make()
    errs, done = [], 0
    for cp, target in targets:
        advance(B, target - done)
        done = target
        m = B.moments_cat(keys=("rho", "ux", "uy"))
        rho = m["rho"].view(nseeds, n_res, n_res)
        if n_res != nc:
            rho, _, _ = to_coarse(rho, m["ux"].view_as(rho), m["uy"].view_as(rho), nc)
        errs.append(density_error(rho, fine_ref[:, cp, 0]))
    bad = int(B.status()[0])
    del B
    return np.array(errs), bad


def _ladder_fields(seeds, N, setup, fine0):
    out = []
    for s in seeds:
        _, u, v, t = fine0[s]
        out.append((np.ones((N, N)), fourier_resample(u, N), fourier_resample(v, N),
                    np.full((N, N), float(t[0, 0]))))
    return out


def evaluate(net: CNN, setup: ClosureSetup, seeds=None, ladder=None, fine_ref=None, timing=True,
             device="cuda"):
    """Learned and plain coarse runs of the held-out seeds against the
    restricted fine runs (see the module docstring).  Timings are for
    coarse_steps coarse steps (the same physical time on every grid), all
    seeds batched, graph-replayed, after a few warm-up steps."""
    seeds = list(setup.eval_seeds if seeds is None else seeds)
    ladder = list(setup.ladder if ladder is None else ladder)
    nc, nf = setup.coarse_n, setup.fine_n
    steps, cps = setup.coarse_steps, list(setup.checkpoints)
    for N in ladder + [nf]:
        for cp in cps + [steps]:
            if (cp * N) % nc:
                raise ValueError(f"checkpoint {cp} is not a whole number of steps at {N}")
    if fine_ref is None:
        fine_ref, _ = restricted_trajectories(seeds, setup, steps=steps, device=device)
    thetas = [seed_flow(s, setup)[1] for s in seeds]
    x0 = fine_ref[:, 0]
    cparams = [_params(nc, setup.mu_coarse, th, setup) for th in thetas]
    cfields = [(x0[j, 0], x0[j, 1], x0[j, 2], x0[j, 3]) for j in range(len(seeds))]
    make_c = lambda: BatchSolver(cparams, cfields, device=device)  # noqa: E731
    if net.max_batch < len(seeds):
        inf = CNN(len(seeds), nc, nc, net.params(), device=device)
        inf.set_norm(*np.split(net.norm, 4))
        inf.set_output_clip(getattr(net, "clip", 0.0))
        net = inf
    k = setup.every
    if any(c % k for c in cps) or steps % k:
        raise ValueError("checkpoints must be whole correction cycles")
    learned = lambda B, n: B.closure_step(net, n // k, every=k, conserve=True,  # noqa: E731
                                          graph=True)
    plain = lambda B, n: B.step(n, graph=True)  # noqa: E731
    ns = len(seeds)
    diverged = {}
    el, diverged["learned"] = _arm(make_c, learned, [(c, c) for c in cps], nc, nc, fine_ref, ns)
    ep, diverged[nc] = _arm(make_c, plain, [(c, c) for c in cps], nc, nc, fine_ref, ns)
    e_plain, curves = {nc: float(ep.mean()), nf: 0.0}, {nc: ep.mean(axis=1).tolist()}
    fine0 = {s: fine_initial(s, setup) for s in seeds}
    for N in ladder:
        pm = [_params(N, setup.mu_fine * N / nf, th, setup) for th in thetas]
        fl = _ladder_fields(seeds, N, setup, fine0)
        make = lambda pm=pm, fl=fl: BatchSolver(pm, fl, device=device)  # noqa: E731
        e, diverged[N] = _arm(make, plain, [(c, c * N // nc) for c in cps], N, nc, fine_ref, ns)
        e_plain[N] = float(e.mean())
        curves[N] = e.mean(axis=1).tolist()

    t_learned, t_plain = float("nan"), {}
    if timing:
        # every arm on its fastest tile shape (the autotuner restores the
        # state); the autotuner times plain steps, so the learned arm also
        # tries the two-step tiles, whose correction cost differs by shape
        B = make_c()
        shapes = [B.autotune(steps=10)]
        del B
        shapes += [s for s in (("tiles", 32, 16), ("tiles", 64, 8)) if s not in shapes]
        times = []
        for kern, w, h in shapes:
            B = make_c()
            try:
                B.set_tile(w, h, kernel=kern)
            except (HlbmError, ValueError):
                continue
            learned(B, 4)
            times.append(_time(lambda: learned(B, steps), B.stream))
            del B
        t_learned = min(times)
        B = make_c()
        B.autotune(steps=10)
        plain(B, 4)
        t_plain[nc] = _time(lambda: plain(B, steps), B.stream)
        del B
        for N in ladder + [nf]:
            pm = [_params(N, setup.mu_fine * N / nf, th, setup) for th in thetas]
            fl = [fine0[s] for s in seeds] if N == nf else _ladder_fields(seeds, N, setup, fine0)
            B = BatchSolver(pm, fl, device=device)
            B.autotune(steps=10)
            plain(B, 4)
            t_plain[N] = _time(lambda: plain(B, steps * N // nc), B.stream)
            del B
    return Evaluation(float(el.mean()), e_plain, t_learned, t_plain,
                      el.mean(axis=1).tolist(), curves, diverged)
