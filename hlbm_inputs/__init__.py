"""Seeded synthetic initial fields for the D2Q9 hybrid LBM.

This module is shared by the CPU oracle and the GPU path so both receive the
same bytes.  It holds only case set-up (analytic initial conditions in lattice
units, Dx = Dt = 1, c_s^2 = 1/3): every function returns host float64 arrays
``rho, ux, uy, theta`` shaped ``[ny][nx]`` (x fastest).  Conversion of theta to
the entropy variable, and everything the method computes, lives on each side
separately.

Conventions (all in lattice units):

* theta is the temperature scaled by the reference temperature T_r (Sec. 2.1);
  the sound speed of the set-up is c = sqrt(gamma * c_s^2 * theta) (Sec. 2.5).
* ``THETA_PAPER = 240/1183`` is T_inf / T_r for T_inf = 300 K and the paper's
  T_r = 1478.75 K (Sec. 4.2), which makes c_inf = 4/13 exactly at gamma = 1.4.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

CS2 = 1.0 / 3.0
THETA_PAPER = 240.0 / 1183.0


def sound_speed(gamma: float, theta: float) -> float:
    """Isentropic sound speed c = sqrt(gamma c_s^2 theta) (Sec. 2.5)."""
    return math.sqrt(gamma * CS2 * theta)


def theta_for_cfl(mach_max: float, gamma: float = 1.4, cfl: float = 0.7,
                  cap: float = THETA_PAPER) -> float:
    """Largest theta with CFL = (Ma + 1) sqrt(gamma c_s^2 theta) <= cfl
    (Sec. 3.5, CFL relation), capped at ``cap``."""
    return min(cap, (cfl / (1.0 + mach_max)) ** 2 / (gamma * CS2))


def _grid(nx, ny):
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    return np.meshgrid(x, y, indexing="xy")  # X[j, i] = i, Y[j, i] = j


def uniform(nx, ny, rho=1.0, ux=0.0, uy=0.0, theta=THETA_PAPER):
    shape = (ny, nx)
    return (np.full(shape, rho), np.full(shape, ux), np.full(shape, uy),
            np.full(shape, theta))


def random_smooth(nx, ny, seed, amp=0.02, rho0=1.0, theta0=THETA_PAPER, u0=(0.05, -0.03)):
    """Smooth random periodic perturbation of every field (a few Fourier modes
    with seeded amplitudes/phases); used for invariance and parity tests."""
    rng = np.random.default_rng(seed)
    X, Y = _grid(nx, ny)
    out = []
    base = [rho0, u0[0], u0[1], theta0]
    scale = [amp, amp, amp, amp * theta0]
    for b, sc in zip(base, scale):
        f = np.full((ny, nx), b, dtype=np.float64)
        for _ in range(3):
            kx, ky = rng.integers(1, 3), rng.integers(1, 3)
            ph = rng.uniform(0, 2 * np.pi)
            a = rng.uniform(-1, 1) * sc
            f = f + a * np.sin(2 * np.pi * (kx * X / nx + ky * Y / ny) + ph)
        out.append(f)
    return tuple(out)


def vortex(nx, ny, xc, yc, R, mach_inf, mach_v, angle=0.0, gamma=1.4,
           theta_inf=THETA_PAPER, rho_inf=1.0, noise=0.0, seed=0, periodic_images=False):
    """Isentropic vortex convected by a uniform stream (Sec. 4.2).

    u_theta = c_inf Ma_v r exp((1 - r^2)/2), r = distance / R, anticlockwise.
    Temperature T/T_inf = 1 - (gamma-1)/2 Ma_v^2 exp(1 - r^2) and
    rho = rho_inf (T/T_inf)^(1/(gamma-1)) -- the radial-equilibrium form of the
    printed density (the stray factor r is dropped; see the design notes).
    Optional density noise: rho <- rho (1 + noise xi), xi ~ U[-1, 1) (seeded),
    theta unchanged.
    """
    X, Y = _grid(nx, ny)
    dx = X - xc
    dy = Y - yc
    if periodic_images:
        dx = (dx + nx / 2) % nx - nx / 2
        dy = (dy + ny / 2) % ny - ny / 2
    r2 = (dx * dx + dy * dy) / (R * R)
    c_inf = sound_speed(gamma, theta_inf)
    amp = c_inf * mach_v * np.exp((1.0 - r2) / 2.0) / R  # u_theta / (r R)
    u_inf = mach_inf * c_inf
    ux = u_inf * math.cos(angle) - amp * dy
    uy = u_inf * math.sin(angle) + amp * dx
    t_ratio = 1.0 - 0.5 * (gamma - 1.0) * mach_v ** 2 * np.exp(1.0 - r2)
    rho = rho_inf * t_ratio ** (1.0 / (gamma - 1.0))
    theta = theta_inf * t_ratio
    if noise:
        rng = np.random.default_rng(seed)
        xi = rng.uniform(-1.0, 1.0, size=(ny, nx))
        rho = rho * (1.0 + noise * xi)
    return rho, ux, uy, theta


def shear_wave(n, a0, u_inf, theta, rho=1.0, width=2, axis="y", shift=0.0):
    """u_x = a0 sin(2 pi (y + shift) / L), u_y = u_inf, uniform p and T
    (Sec. 4.1).  Quasi-1D: ``width`` columns across, ``n`` points per
    wavelength.  shift = 0.5 puts the zeros of u_x half-way between nodes."""
    if axis == "y":
        nx, ny = width, n
        _, Y = _grid(nx, ny)
        ux = a0 * np.sin(2 * np.pi * (Y + shift) / n)
        uy = np.full((ny, nx), u_inf)
    else:  # transposed: u_y = a0 sin(2 pi (x + shift) / L), u_x = u_inf
        nx, ny = n, width
        X, _ = _grid(nx, ny)
        uy = a0 * np.sin(2 * np.pi * (X + shift) / n)
        ux = np.full((ny, nx), u_inf)
    return np.full((ny, nx), rho), ux, uy, np.full((ny, nx), theta)


def acoustic_wave(n, amp, gamma, theta_inf, rho_inf=1.0, width=2, u_mean=0.0):
    """Right-running isentropic sine wave along x (Sec. 4.3):
    p' = amp p_inf sin(2 pi x / L), u' = p'/(rho c), isentropic T and rho."""
    nx, ny = n, width
    X, _ = _grid(nx, ny)
    p_inf = rho_inf * CS2 * theta_inf
    c_inf = sound_speed(gamma, theta_inf)
    pt = amp * p_inf * np.sin(2 * np.pi * X / n)
    p = p_inf + pt
    rho = rho_inf * (p / p_inf) ** (1.0 / gamma)
    theta = p / (rho * CS2)
    ux = u_mean + pt / (rho_inf * c_inf)
    return rho, ux, np.zeros_like(ux), theta


def gaussian_pulse_1d(n, amp, gamma, theta_inf, sigma_pts, x0=None, rho_inf=1.0, width=2,
                      travelling=True):
    """Gaussian pressure pulse along x, isentropic, optionally with the velocity
    u = p'/(rho c) of a right-running wave (Sec. 5.1, speed-of-sound case)."""
    nx, ny = n, width
    X, _ = _grid(nx, ny)
    if x0 is None:
        x0 = n / 2
    d = (X - x0 + n / 2) % n - n / 2
    p_inf = rho_inf * CS2 * theta_inf
    c_inf = sound_speed(gamma, theta_inf)
    pt = amp * p_inf * np.exp(-0.5 * (d / sigma_pts) ** 2)
    p = p_inf + pt
    rho = rho_inf * (p / p_inf) ** (1.0 / gamma)
    theta = p / (rho * CS2)
    ux = pt / (rho_inf * c_inf) if travelling else np.zeros_like(pt)
    return rho, ux, np.zeros_like(ux), theta


def entropy_wave(n, amp, theta_inf, rho_inf=1.0, width=2, u_mean=0.0):
    """Isobaric temperature wave along x: theta = theta_inf (1 + amp sin),
    rho theta = const, uniform velocity u_mean."""
    nx, ny = n, width
    X, _ = _grid(nx, ny)
    theta = theta_inf * (1.0 + amp * np.sin(2 * np.pi * X / n))
    rho = rho_inf * theta_inf / theta
    return rho, np.full_like(rho, u_mean), np.zeros_like(rho), theta


def riemann(nx, ny, left, right, x_split=None, theta_scale=0.2):
    """Riemann problem along x with normalised (rho, u, p) states; theta is
    mapped as theta = theta_scale * p / rho (normalised T = p / rho)."""
    if x_split is None:
        x_split = nx // 2
    X, _ = _grid(nx, ny)
    mask = X < x_split
    def fld(i):
        return np.where(mask, left[i], right[i]).astype(np.float64)
    rho = fld(0)
    u_scale = math.sqrt(theta_scale * CS2)  # velocity unit sqrt(p/rho) -> lattice
    ux = fld(1) * u_scale
    theta = theta_scale * fld(2) / rho
    return rho, ux, np.zeros_like(ux), theta


def sod(nx, ny, theta_scale=0.2):
    """Standard Sod states (rho, u, p) = (1, 0, 1) | (0.125, 0, 0.1)."""
    return riemann(nx, ny, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), theta_scale=theta_scale)


# The shock tube of Sec. 5.2 in lattice units.  Air, r = 287.15 J/(kg K) (the
# paper's value), T_inf = 300 K on both sides, T_r = 1460 K, p_inf = 101325
# Pa, a 1 m tube of 401 points (dx = 1/400 m), mu = 1e-5 kg/(m s).  The
# velocity unit is C_0 = sqrt(r T_r / c_s^2) and the density unit rho_inf, so
# mu_lattice = mu / (rho_inf dx C_0).
PAPER_TUBE = dict(r=287.15, T_inf=300.0, T_r=1460.0, p_inf=101325.0, length=1.0, nx=401,
                  mu=1e-5)


def paper_tube_mu(nx=PAPER_TUBE["nx"]):
    """Lattice dynamic viscosity of the Sec. 5.2 tube on nx points."""
    c = PAPER_TUBE
    dx = c["length"] / (nx - 1)
    c0 = math.sqrt(c["r"] * c["T_r"] / CS2)
    rho_inf = c["p_inf"] / (c["r"] * c["T_inf"])
    return c["mu"] / (rho_inf * dx * c0)


def paper_shock_tube(nx=PAPER_TUBE["nx"], ny=2):
    """Sec. 5.2: (rho, u, p) = (3 rho_inf, 0, 3 p_inf) for x < 0.5 m and
    (rho_inf, 0, p_inf) beyond, one temperature T_inf throughout, so theta =
    T_inf / T_r on both sides and rho = 3 | 1 in units of rho_inf.  The split
    falls between node (nx - 1) / 2 - 1 and (nx - 1) / 2 (x_i = i dx)."""
    c = PAPER_TUBE
    theta = c["T_inf"] / c["T_r"]
    X, _ = _grid(nx, ny)
    dx = c["length"] / (nx - 1)
    rho = np.where(X * dx < 0.5 * c["length"], 3.0, 1.0)
    return rho, np.zeros_like(rho), np.zeros_like(rho), np.full_like(rho, theta)


def rankine_hugoniot(mach, gamma=1.4):
    """Normal-shock jump ratios (rho2/rho1, u2/u1, p2/p1, T2/T1, M2)."""
    m2 = mach * mach
    r = (gamma + 1) * m2 / ((gamma - 1) * m2 + 2)
    pr = 1 + 2 * gamma / (gamma + 1) * (m2 - 1)
    t = pr / r
    mdown = math.sqrt(((gamma - 1) * m2 + 2) / (2 * gamma * m2 - (gamma - 1)))
    return r, 1.0 / r, pr, t, mdown


def normal_shock(nx, ny, mach=2.0, theta1=0.1, gamma=1.4, rho1=1.0, x_split=None,
                 perturb=1e-3, seed=0, transverse=False):
    """Stationary normal shock from Rankine-Hugoniot states; the upstream
    velocity gets a seeded perturbation perturb * u1 * N(0, 1).  By default
    the perturbation varies along x only (one draw per column, u_x only), so
    the flow stays quasi-one-dimensional; ``transverse=True`` draws it per
    node on both components (grid-scale 2-D noise)."""
    if x_split is None:
        x_split = nx // 2
    r, ur, pr, tr, _ = rankine_hugoniot(mach, gamma)
    c1 = sound_speed(gamma, theta1)
    u1 = mach * c1
    X, _ = _grid(nx, ny)
    up = X < x_split
    rho = np.where(up, rho1, rho1 * r)
    theta = np.where(up, theta1, theta1 * tr)
    ux = np.where(up, u1, u1 * ur)
    uy = np.zeros_like(ux)
    if perturb:
        rng = np.random.default_rng(seed)
        if transverse:
            nxp = rng.standard_normal((ny, nx))
            nyp = rng.standard_normal((ny, nx))
            uy = uy + np.where(up, perturb * u1 * nyp, 0.0)
        else:
            nxp = np.repeat(rng.standard_normal((1, nx)), ny, axis=0)
        ux = ux + np.where(up, perturb * u1 * nxp, 0.0)
    return rho, ux, uy, theta


def turbulence(n, mach_t, theta, seed, kpeak=8.0, rho=1.0, gamma=1.4, ny=None):
    """Random-phase solenoidal velocity from a stream function with
    |psi_hat(k)|^2 ~ E(k)/(pi k^3), E(k) = k^4 exp(-2 (k/kpeak)^2) (k in units
    of 2 pi / L), k = 0 removed, scaled so sqrt(<|u|^2>) = mach_t * c.
    Uniform rho and theta."""
    nx = n
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    kx = np.fft.rfftfreq(nx, d=1.0 / nx)           # integer wavenumbers
    ky = np.fft.fftfreq(ny, d=1.0 / ny)
    KX, KY = np.meshgrid(kx, ky, indexing="xy")
    K = np.sqrt(KX * KX + KY * KY)
    K[0, 0] = 1.0
    E = K ** 4 * np.exp(-2.0 * (K / kpeak) ** 2)
    amp = np.sqrt(E / (np.pi * K ** 3))
    amp[0, 0] = 0.0
    phase = rng.uniform(0.0, 2 * np.pi, size=K.shape)
    psi_hat = amp * np.exp(1j * phase)
    del E, amp, phase, K
    # u = d psi / dy, v = -d psi / dx (spectral derivatives, 2 pi / L units)
    ux = np.fft.irfft2(1j * (2 * np.pi / ny) * KY * psi_hat, s=(ny, nx))
    uy = np.fft.irfft2(-1j * (2 * np.pi / nx) * KX * psi_hat, s=(ny, nx))
    del psi_hat, KX, KY
    rms = math.sqrt(float(np.mean(ux * ux + uy * uy)))
    target = mach_t * sound_speed(gamma, theta)
    scale = target / rms if rms > 0 else 0.0
    ux *= scale
    uy *= scale
    return np.full((ny, nx), rho), ux, uy, np.full((ny, nx), theta)


@dataclass
class DomainSpec:
    n: int
    kind: int          # 0 vortex, 1 turbulence
    mach: float
    theta: float
    seed: int
    angle: float = 0.0


def batch_specs(count=256, seed=0, nmin=64, nmax=1024, gamma=1.4):
    """Sizes (log-uniform), kinds and Mach numbers for a batch of independent
    periodic square domains, drawn in that order from one seeded generator.
    Theta per domain from the CFL rule with M_max = 1.1 Ma (vortex) or
    3 Ma_t (turbulence).  Per-domain field seed = 1000 + d."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), count))).astype(int)
    kinds = rng.integers(0, 2, count)
    machs = rng.uniform(0.1, 2.0, count)
    angles = rng.uniform(0.0, 2 * np.pi, count)
    specs = []
    for d in range(count):
        mm = 1.1 * machs[d] if kinds[d] == 0 else 3.0 * machs[d]
        specs.append(DomainSpec(int(sizes[d]), int(kinds[d]), float(machs[d]),
                                theta_for_cfl(mm, gamma), 1000 + d, float(angles[d])))
    return specs


def batch_domain_fields(spec: DomainSpec, gamma=1.4):
    n = spec.n
    if spec.kind == 0:
        return vortex(n, n, n / 2, n / 2, n / 12.8, spec.mach, 0.1 * spec.mach,
                      angle=spec.angle, gamma=gamma, theta_inf=spec.theta)
    return turbulence(n, spec.mach, spec.theta, spec.seed, gamma=gamma)
