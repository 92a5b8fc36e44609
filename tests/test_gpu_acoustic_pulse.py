"""Gaussian acoustic pulse (Sec. 5.1) at Ma 0 and 1 against linear
acoustics (tests/acoustics_exact.py): 201^2 periodic box, 6 points per pulse
radius, 0.4 acoustic crossing times."""
import numpy as np
import pytest

from acoustics_exact import pulse_pressure

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2002_03644_amd import studies  # noqa: E402


def test_acoustic_pulse_matches_linear_acoustics():
    res = studies.acoustic_pulse()
    n = 201
    X, Y = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64))
    errs = {}
    for mach, r in res.items():
        t = r["steps"]
        xc = r["x0"] + r["u"] * t
        dx = (X - xc + n / 2) % n - n / 2
        dy = (Y - r["y0"] + n / 2) % n - n / 2
        exact = r["amp"] * pulse_pressure(np.hypot(dx, dy), t, r["c"], 1.0 / (2 * r["R"] ** 2))
        num = r["p_prime"]
        e2 = np.linalg.norm(num - exact) / np.linalg.norm(exact)
        row = int(r["y0"])
        eline = np.abs(num[row] - exact[row]).max() / np.abs(exact[row]).max()
        errs[mach] = (e2, eline)
        print(f"Ma {mach}: relative L2 error {e2:.3f}, worst on y = 0.5 line {eline:.3f}")
    assert errs[0.0][0] < 0.1 and errs[0.0][1] < 0.1
    assert errs[1.0][0] < 0.25 and errs[1.0][1] < 0.25
    # isotropy of the Ma = 0 pulse: the ring's radial profile along the four
    # axis directions and the four diagonals agree
    p = res[0.0]["p_prime"]
    c0 = n // 2
    axes = [p[c0, c0:], p[c0, c0::-1], p[c0:, c0], p[c0::-1, c0]]
    spread = np.max(np.std(np.stack([a[:90] for a in axes]), axis=0)) / np.abs(p).max()
    print(f"axis spread {spread:.4f}")
    assert spread < 1e-6   # the four axes are symmetric images of each other
    diag = np.array([p[c0 + k, c0 + k] for k in range(64)])
    rad = np.interp(np.arange(64) * np.sqrt(2.0), np.arange(90), axes[0][:90])
    aniso = np.abs(diag - rad).max() / np.abs(p).max()
    print(f"diagonal vs axis {aniso:.3f}")
    assert aniso < 0.1
