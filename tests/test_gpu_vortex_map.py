"""The sigma x Mach vortex study (Sec. 4.2) on the batched engine: one cell
against the oracle, and a reduced map."""
import numpy as np
import pytest

import hlbm_inputs as hi
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2002_03644_amd import BatchSolver, Params  # noqa: E402
from paper_2002_03644_amd import studies  # noqa: E402


@pytest.mark.parametrize("original", [False, True])
def test_map_cell_matches_oracle(original):
    """Ma 1.3, sigma 0.5 (or the original model at sigma 0), the map's
    near-inviscid viscosity, FP64 batch vs the oracle after 40 steps."""
    n, mach = 64, 1.3
    sigma = 0.0 if original else 0.5
    f = hi.vortex(n, n, n / 2, n / 2, n / 10, mach, 0.1 * mach, periodic_images=True)
    p = Params(n, n, dtype="f64", mu=1.5e-6, sigma=sigma, e1_centred=original, e2_off=original)
    B = BatchSolver([p, p], [f, f])
    B.step(40, graph=True)
    m = B.moments()[1]
    s = oracle.entropy_from_theta(f[0], f[3], 1.4)
    O = oracle.OracleSolver(oracle.OracleParams(n, n, mu=1.5e-6, sigma=sigma, e1_centred=original,
                                                e2_off=original), *f[:3], s=s)
    O.step(40)
    mo = O.moments()
    for k in ("rho", "ux", "uy", "s"):
        g = m[k].cpu().numpy()
        scale = np.abs(mo[k]).max() if k in ("rho", "s") else np.hypot(mo["ux"], mo["uy"]).max()
        assert np.abs(g - mo[k]).max() / scale < 1e-12, k


def test_reduced_sigma_mach_map():
    res = studies.sigma_mach_map(machs=[0.5, 1.3], sigmas=[0.0, 1.0], n=64, conv_times=2.0,
                                 log=print)
    for mach in (0.5, 1.3):
        assert not res.diverged[("present", mach, 0.0)], mach
        e = res.error[("present", mach, 0.0)]
        assert np.isfinite(e) and e < 1.0, (mach, e)
    print(studies.map_summary(res))
