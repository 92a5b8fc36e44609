"""hlbm_state_totals, the allocation-free entry point: conservation totals
of a raw state buffer with the library's static device scratch, against
hlbm_totals of the handle that state came from (same kernels, same fixed
reduction order: the same bits), on two calls in a row, the second with a
smaller domain; FP64 and FP32."""
import ctypes

import numpy as np
import pytest

import hlbm_inputs as hi

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2002_03644_amd import HLBM_EINVAL, Params, Solver, _lib, state_totals  # noqa: E402


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_state_totals_match_handle_totals(dtype):
    runs = []
    for nx, ny in ((700, 530), (96, 40)):        # second call: a smaller domain
        r, u, v, t = hi.random_smooth(nx, ny, seed=nx, amp=0.05)
        p = Params(nx, ny, dtype=dtype, mu=2e-3, sigma=0.5)
        S = Solver(p, r, u, v, theta=t)
        S.step(7)
        runs.append((p, S, S.save_state()))
    for p, S, snap in runs:
        want = S.totals()
        got = state_totals(p, snap)
        assert np.array_equal(got, want), (p.nx, p.ny, got, want)
        assert got[0] > 0
    # the first domain again, after the smaller one used the scratch
    p, S, snap = runs[0]
    assert np.array_equal(state_totals(p, snap), S.totals())


def test_state_totals_rejects_invalid_arguments():
    p = Params(64, 64, dtype="f64")
    cp = p.c()
    buf = torch.zeros(_lib.lib().hlbm_state_bytes(ctypes.byref(cp)), dtype=torch.uint8,
                      device="cuda")
    out = (ctypes.c_double * 4)()
    L = _lib.lib()
    assert L.hlbm_state_totals(ctypes.byref(cp), None, out, None) == HLBM_EINVAL
    assert L.hlbm_state_totals(ctypes.byref(cp), ctypes.c_void_p(buf.data_ptr()), None,
                               None) == HLBM_EINVAL
    bad = Params(0, 64, dtype="f64").c()
    assert L.hlbm_state_totals(ctypes.byref(bad), ctypes.c_void_p(buf.data_ptr()), out,
                               None) == HLBM_EINVAL
