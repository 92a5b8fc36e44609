"""The learned closure gains over the method without it.

Reduced protocol (same recipe as the full one, fewer seeds and steps): 32
training seeds of 1024^2 decaying turbulence (Ma_t 0.25-0.45) restricted 4x
to 256^2, 100 coarse steps each, one correction per 10 coarse steps; the
network trained on the GPU by the library's kernels; two held-out seeds
measured against their restricted fine runs.  The corrected 256^2 runs must have a lower density error than the
plain 256^2 runs, at every checkpoint, and stay finite."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2002_03644_amd import learned as L  # noqa: E402


def test_learned_closure_beats_plain_coarse_run():
    setup = L.ClosureSetup(train_seeds=tuple(range(1000, 1032)), eval_seeds=(2000, 2001),
                           coarse_steps=100, checkpoints=(50, 100), ladder=())
    net, rec = L.fit(setup, steps=6000, batch=32, lr=2e-3, clip=4.0, log=print)
    ev = L.evaluate(net, setup, ladder=[], timing=False)
    nc = setup.coarse_n
    print(f"density error: learned {ev.e_learned:.4f}, plain {ev.e_plain[nc]:.4f}; "
          f"curves {np.round(ev.e_learned_curve, 4)} vs {np.round(ev.e_plain_curve[nc], 4)}")
    assert rec["fine_diverged"] == 0
    assert ev.diverged["learned"] == 0 and ev.diverged[nc] == 0
    assert np.isfinite(ev.e_learned)
    assert ev.e_learned < 0.9 * ev.e_plain[nc]
    for a, b in zip(ev.e_learned_curve, ev.e_plain_curve[nc]):
        assert a < b
