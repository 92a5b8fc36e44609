"""Parameter studies of the method, run on the batched engine.

sigma_mach_map: the convected isentropic vortex of Sec. 4.2 on a periodic
n x n box (R = n / 10 points per radius, vortex intensity Ma_v = 0.1 Ma),
one temperature for every Mach number (theta = 240/1183, the paper's
T/T_r = 300 / 1478.75), advected along x for 50 convective times L / u_inf
-- after which the exact solution is the initial field again -- for a grid
of HRR blends sigma and Mach numbers, and, at sigma = 0, the original model
(equilibrium truncated at third order, centred E1, no E2).  Per run: the L2 error of the pressure relative to the
vortex's pressure perturbation, ||p - p_0||_2 / ||p_0 - p_inf||_2, a
divergence flag (non-finite or non-physical state), and an energy flag set
when the largest total-energy density p / (gamma - 1) + rho |u|^2 / 2 grew
above the initial one by more than 1e-4 of it (the paper marks runs that
diverged or whose total-energy maximum grew as failed).  All sigma values of one Mach number (and the
original model) advance together as one batch.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

import hlbm_inputs as hi

from ._lib import BatchSolver, Params


@dataclass
class MapResult:
    machs: list
    sigmas: list
    n: int
    conv_times: float
    steps: dict = field(default_factory=dict)        # mach -> steps run
    error: dict = field(default_factory=dict)        # (model, mach, sigma) -> e_p (None if diverged)
    diverged: dict = field(default_factory=dict)     # (model, mach, sigma) -> bool
    energy_grew: dict = field(default_factory=dict)  # (model, mach, sigma) -> bool
    seconds: float = 0.0
    node_updates: float = 0.0

    def failed(self, model, mach, sigma):
        return self.diverged[(model, mach, sigma)] or self.energy_grew[(model, mach, sigma)]


def _pressure(rho, theta):
    return rho * hi.CS2 * theta


def sigma_mach_map(machs=None, sigmas=None, n=200, conv_times=50.0, beta=0.1, mu=1.5e-6,
                   gamma=1.4, theta=hi.THETA_PAPER, dtype="f32", original=True,
                   device="cuda", log=None):
    """Run the map (see the module docstring).  mu defaults to the paper's
    air viscosity (1e-5 kg/(m s) at 300 K, 1 atm) in the lattice units of its
    200-point, 1 m box with T_r = 1478.75 K."""
    import torch
    machs = [round(0.3 + 0.1 * k, 10) for k in range(11)] if machs is None else list(machs)
    sigmas = [round(0.1 * k, 10) for k in range(11)] if sigmas is None else list(sigmas)
    R = n / 10.0
    c = hi.sound_speed(gamma, theta)
    res = MapResult(machs, sigmas, n, conv_times)
    t0 = time.perf_counter()
    for mach in machs:
        steps = int(round(conv_times * n / (mach * c)))
        mach_eff = conv_times * n / (steps * c)      # whole number of box crossings
        f = hi.vortex(n, n, n / 2, n / 2, R, mach_eff, beta * mach_eff, gamma=gamma,
                      theta_inf=theta, periodic_images=True)
        models = [("present", s) for s in sigmas] + ([("original", 0.0)] if original else [])
        params = [Params(n, n, dtype=dtype, gamma=gamma, mu=mu, sigma=s, theta_ref=theta,
                         e1_centred=(m == "original"), e2_off=(m == "original"),
                         feq_order=3 if m == "original" else 4)
                  for m, s in models]
        B = BatchSolver(params, [f] * len(models), device=device)
        B.autotune(steps=10)
        B.step(steps, graph=True)
        _, flags = B.status()
        mom = B.moments()
        p0 = _pressure(f[0], f[3])
        p_inf = _pressure(1.0, theta)
        e0 = p0 / (gamma - 1.0) + 0.5 * f[0] * (f[1] ** 2 + f[2] ** 2)
        den = np.linalg.norm(p0 - p_inf)
        for k, (m, s) in enumerate(models):
            d = {key: v.double().cpu().numpy() for key, v in mom[k].items()}
            p = _pressure(d["rho"], d["theta"])
            ok = bool(flags[k] == 0 and np.isfinite(p).all())
            res.error[(m, mach, s)] = float(np.linalg.norm(p - p0) / den) if ok else None
            res.diverged[(m, mach, s)] = not ok
            grew = False
            if ok:
                et = p / (gamma - 1.0) + 0.5 * d["rho"] * (d["ux"] ** 2 + d["uy"] ** 2)
                grew = bool(et.max() > e0.max() * (1.0 + 1e-4))
            res.energy_grew[(m, mach, s)] = grew
        res.steps[mach] = steps
        res.node_updates += float(steps) * n * n * len(models)
        if log:
            def cell(m, s):
                if res.diverged[(m, mach, s)]:
                    return "x"
                return f"{res.error[(m, mach, s)]:.3g}" + ("*" if res.energy_grew[(m, mach, s)] else "")
            log(f"[map] Ma {mach:.1f}: {steps} steps, e_p(sigma) = "
                + " ".join(cell("present", s) for s in sigmas)
                + (f", original {cell('original', 0.0)}" if original else ""))
        del B
    torch.cuda.synchronize()
    res.seconds = time.perf_counter() - t0
    return res


def map_summary(res: MapResult):
    """JSON-friendly form of a map."""
    def key(m, s):
        return f"{m:.1f}/{s:.1f}"
    out = {"machs": res.machs, "sigmas": res.sigmas, "n": res.n, "conv_times": res.conv_times,
           "steps": {f"{m:.1f}": v for m, v in res.steps.items()},
           "present": {key(m, s): res.error[("present", m, s)] for m in res.machs
                       for s in res.sigmas},
           "present_diverged": [key(m, s) for m in res.machs for s in res.sigmas
                                if res.diverged[("present", m, s)]],
           "present_energy_grew": [key(m, s) for m in res.machs for s in res.sigmas
                                   if res.energy_grew[("present", m, s)]],
           "seconds": round(res.seconds, 2),
           "glups": round(res.node_updates / max(res.seconds, 1e-9) / 1e9, 2)}
    if ("original", res.machs[0], 0.0) in res.error:
        out["original_sigma0"] = {f"{m:.1f}": res.error[("original", m, 0.0)] for m in res.machs}
        out["original_diverged"] = [f"{m:.1f}" for m in res.machs
                                    if res.diverged[("original", m, 0.0)]]
    return out



def acoustic_pulse_cases(n=201, R=6.0, amp_pa=10.0, p_inf_pa=101323.0, t_frac=0.4, gamma=1.4,
                         theta=hi.THETA_PAPER, mu=1.5e-6):
    """Set-up of the Gaussian acoustic pulse of Sec. 5.1 at Ma = 0 (sigma
    0.95, centred) and Ma = 1 (sigma 0, started at x = n / 10 so both end at
    the centre) on a periodic n x n box: p = p_inf (1 + A exp(-r^2 / (2
    R^2))) with A = amp_pa / p_inf_pa, isentropic rho and theta, u_x = Ma c.
    Returns (steps, cases); steps = round(t_frac n / c); each case is a dict
    with mach, sigma, x0, y0, the parameter keywords of the domain (mu,
    sigma, gamma) and its host fields (rho, ux, uy, theta)."""
    c = hi.sound_speed(gamma, theta)
    steps = int(round(t_frac * n / c))
    p_inf = hi.CS2 * theta
    X, Y = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64))
    cases = []
    for mach, sigma, xc in ((0.0, 0.95, n // 2), (1.0, 0.0, n // 10)):
        dx = (X - xc + n / 2) % n - n / 2
        dy = (Y - n // 2 + n / 2) % n - n / 2
        p = p_inf * (1.0 + amp_pa / p_inf_pa * np.exp(-(dx * dx + dy * dy) / (2.0 * R * R)))
        rho = (p / p_inf) ** (1.0 / gamma)
        cases.append({"mach": mach, "sigma": sigma, "x0": float(xc), "y0": float(n // 2),
                      "kw": dict(gamma=gamma, mu=mu, sigma=sigma),
                      "fields": (rho, np.full((n, n), mach * c), np.zeros((n, n)),
                                 p / (rho * hi.CS2)),
                      "u": mach * c, "amp": p_inf * amp_pa / p_inf_pa, "c": c, "R": R,
                      "p_inf": p_inf})
    return steps, cases


def acoustic_pulse(n=201, dtype="f64", device="cuda", **kw):
    """Both pulses of acoustic_pulse_cases as one batch of two domains,
    advanced on the GPU.  Returns, per Mach number, the pressure perturbation
    p - p_inf [n][n] (FP64 numpy), the final fields (rho, ux, uy, s, theta),
    the initial centre (x0, y0) in cells, the mean velocity and the steps."""
    theta = kw.get("theta", hi.THETA_PAPER)
    steps, cases = acoustic_pulse_cases(n, **kw)
    params = [Params(n, n, dtype=dtype, theta_ref=theta, **cs["kw"]) for cs in cases]
    B = BatchSolver(params, [cs["fields"] for cs in cases], device=device)
    B.step(steps, graph=True)
    mom = B.moments()
    out = {}
    for k, cs in enumerate(cases):
        d = {key: v.double().cpu().numpy() for key, v in mom[k].items()}
        out[cs["mach"]] = {"p_prime": _pressure(d["rho"], d["theta"]) - cs["p_inf"],
                           "fields": d, "x0": cs["x0"], "y0": cs["y0"], "u": cs["u"],
                           "steps": steps, "sigma": cs["sigma"], "amp": cs["amp"],
                           "c": cs["c"], "R": cs["R"]}
    return out


def couette_exact(eta, ma, pr, gamma):
    """Steady temperature of the thermal Couette flow between walls at one
    temperature T_w (Sec. 4.4): (T - T_w) / T_w = eta Pr Ma^2 (gamma - 1) / 2
    (1 - eta), eta = y / H, Ma = U / c at T_w."""
    eta = np.asarray(eta, dtype=np.float64)
    return eta * pr * ma * ma * (gamma - 1.0) / 2.0 * (1.0 - eta)


def thermal_couette(ny=100, nx=2, ma=0.8, pr=0.71, gamma=1.4, sigma=0.9, theta_w=300.0 / 1500.0,
                    nu=0.1, steps=None, dtype="f64", phi_mode="lbm", precise_theta=True,
                    device="cuda"):
    """The thermal Couette flow of Sec. 4.4 on an nx x ny channel (the paper
    uses 2 x 100, T_r = 1500 K, T_w = 300 K, sigma 0.9): periodic in x, walls
    at the rows y = 0 (at rest) and y = ny - 1 (moving at U = Ma c_w, c_w the
    sound speed at theta_w), both at theta_w.  Starts from the steady velocity
    U y / H at uniform theta_w and density 1 and runs `steps` steps (default:
    enough for the slowest thermal mode, decaying as exp(-pi^2 nu t / (Pr
    H^2)), to fall below 1e-7).  Returns the theta and u_x profiles (FP64
    numpy, averaged over x), the closed-form profiles, and the largest
    temperature error relative to the largest temperature rise.
    precise_theta (the default here) takes the Fourier term's Laplacian of
    temperature deviations computed accurately, which this slow,
    well-resolved flow needs in FP32."""
    import torch
    from ._lib import Solver
    H = ny - 1
    c = hi.sound_speed(gamma, theta_w)
    U = ma * c
    if steps is None:
        steps = int(np.ceil(1.7 * H * H * max(pr, 1.0) / nu))
    eta = np.arange(ny, dtype=np.float64) / H
    ones = np.ones((ny, nx))
    p = Params(nx, ny, dtype=dtype, gamma=gamma, prandtl=pr, mu=nu, sigma=sigma, bc_y="wall",
               wall_ux_lo=0.0, wall_ux_hi=U, wall_theta=theta_w, theta_ref=theta_w,
               phi_mode=phi_mode, precise_theta=precise_theta)
    S = Solver(p, ones, U * eta[:, None] * ones, 0.0 * ones, theta=theta_w * ones, device=device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.step(steps)
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    m = {k: v.double().cpu().numpy() for k, v in S.moments().items()}
    theta = m["theta"].mean(axis=1)
    ux = m["ux"].mean(axis=1)
    rise = couette_exact(eta, ma, pr, gamma)
    exact = theta_w * (1.0 + rise)
    err = float(np.abs(theta - exact).max() / (theta_w * rise.max()))
    return {"theta": theta, "theta_exact": exact, "ux": ux, "ux_exact": U * eta, "error": err,
            "ux_error": float(np.abs(ux - U * eta).max() / U), "steps": steps,
            "seconds": seconds, "U": U, "nx": nx, "ny": ny}
