"""Linear-acoustics solution of a Gaussian pressure pulse in 2-D (test
reference for the acoustic-pulse case of Sec. 5.1).

Initial state: p' = eps exp(-alpha r^2), u' = 0, uniform medium at rest
(a mean flow only translates the solution).  The pressure obeys the wave
equation p_tt = c^2 lap p with p_t(0) = 0, so in Hankel space
P(k, t) = P(k, 0) cos(c k t) with P(k, 0) = (eps / (2 alpha))
exp(-k^2 / (4 alpha)), and
    p'(r, t) = (eps / (2 alpha)) int_0^inf exp(-k^2 / (4 alpha)) cos(c k t)
               J0(k r) k dk.
"""
import numpy as np
from scipy.special import j0


def pulse_pressure(r, t, c, alpha, eps=1.0, nk=4000):
    """p'(r, t) on an array of radii, by the trapezoid rule in k up to where
    the Gaussian factor falls below 1e-16."""
    kmax = np.sqrt(4.0 * alpha * 37.0)
    k = np.linspace(0.0, kmax, nk)
    w = np.exp(-k * k / (4.0 * alpha)) * np.cos(c * k * t) * k
    r = np.asarray(r, dtype=np.float64)
    integrand = w[None, :] * j0(np.outer(r.ravel(), k))
    vals = np.trapezoid(integrand, k, axis=1) if hasattr(np, "trapezoid") else np.trapz(integrand, k, axis=1)
    return (eps / (2.0 * alpha) * vals).reshape(r.shape)
