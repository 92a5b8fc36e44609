"""Pins of the learned-closure oracle: convolution against its definition by
explicit loops, gradients against central finite differences, Adam's first
step against its closed form, and the restriction's conservation."""
import itertools

import numpy as np
import pytest

from oracle import cnn_oracle as C


def test_conv3x3_matches_explicit_loops():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 4, 5, 3))
    w = rng.normal(size=(3, 3, 3, 2))
    b = rng.normal(size=2)
    out = C.conv3x3(x, w, b)
    B, H, W, _ = x.shape
    for n, y, xx, co in itertools.product(range(B), range(H), range(W), range(2)):
        s = b[co]
        for dy, dx, ci in itertools.product(range(3), range(3), range(3)):
            s += x[n, (y + dy - 1) % H, (xx + dx - 1) % W, ci] * w[dy, dx, ci, co]
        assert out[n, y, xx, co] == pytest.approx(s, abs=1e-12)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    params = C.init_params(seed=2)
    params = [(w * 3.0, rng.normal(size=b.shape) * 0.1) for w, b in params]
    x = rng.normal(size=(2, 4, 4, 4))
    t = rng.normal(size=(2, 4, 4, 4))
    loss, grads = C.loss_and_grads(params, x, t)
    h = 1e-6
    for k in range(3):
        for j in range(2):
            p = params[k][j]
            flat_idx = rng.choice(p.size, size=min(6, p.size), replace=False)
            for fi in flat_idx:
                idx = np.unravel_index(fi, p.shape)
                def perturbed(delta):
                    q = [list(l) for l in params]
                    arr = q[k][j].copy()
                    arr[idx] += delta
                    q[k][j] = arr
                    return C.loss_and_grads([tuple(l) for l in q], x, t)[0]
                fd = (perturbed(h) - perturbed(-h)) / (2 * h)
                an = grads[k][j][idx]
                assert an == pytest.approx(fd, rel=1e-5, abs=1e-9), (k, j, idx)


def test_adam_first_step_closed_form():
    """After one step from zero moments, m_hat = g and v_hat = g^2, so the
    update is -lr g / (|g| + eps)."""
    rng = np.random.default_rng(3)
    params = [(rng.normal(size=(2, 3)), rng.normal(size=3))]
    grads = [(rng.normal(size=(2, 3)), rng.normal(size=3))]
    opt = C.Adam(params, lr=0.01)
    new = opt.step(params, grads)
    for (p, g), q in zip(zip(params[0], grads[0]), new[0]):
        np.testing.assert_allclose(q - p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # with a constant gradient the bias-corrected moments stay g and g^2,
    # so the second step equals the first
    new2 = opt.step(new, grads)
    for p1, p2, g in zip(new[0], new2[0], grads[0]):
        np.testing.assert_allclose(p2 - p1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9)


def test_restriction_conserves_block_totals():
    rng = np.random.default_rng(4)
    rho = rng.uniform(0.5, 1.5, size=(16, 24))
    ux, uy = rng.normal(size=(2, 16, 24))
    th = rng.uniform(0.1, 0.3, size=(16, 24))
    rc, uc, vc, tc = C.restrict(rho, ux, uy, th, 4)
    assert rc.shape == (4, 6)
    assert (rc * 16).sum() == pytest.approx(rho.sum(), rel=1e-14)
    assert (rc * uc * 16).sum() == pytest.approx((rho * ux).sum(), rel=1e-12, abs=1e-12)
    assert (rc * vc * 16).sum() == pytest.approx((rho * uy).sum(), rel=1e-12, abs=1e-12)
    assert (rc * tc * 16).sum() == pytest.approx((rho * th).sum(), rel=1e-14)
    one = C.restrict(np.full((8, 8), 1.2), np.full((8, 8), 0.1), np.zeros((8, 8)),
                     np.full((8, 8), 0.2), 4)
    for a, v in zip(one, (1.2, 0.1, 0.0, 0.2)):
        np.testing.assert_allclose(a, v, rtol=1e-15)


def test_parameter_count():
    params = C.init_params()
    assert sum(w.size + b.size for w, b in params) == 11588


def test_bf16_rounding_ties_to_even_and_matches_torch():
    one = np.float64(1.0)
    assert C.bf16(np.array([one + 2.0 ** -8]))[0] == 1.0            # tie -> even (1)
    assert C.bf16(np.array([one + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6   # tie -> even
    assert C.bf16(np.array([one + 2.0 ** -8 + 2.0 ** -20]))[0] == 1.0 + 2.0 ** -7
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(5).normal(size=10000) * 10.0 ** np.random.default_rng(6).integers(-20, 20, 10000)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(C.bf16(x), ref)


def test_stored_precision_variant_is_close_and_exact_on_representable_data():
    """With inputs and weights already BF16-representable and activations
    that stay representable (small-integer data), the stored-precision
    passes equal the FP64 ones exactly."""
    rng = np.random.default_rng(7)
    w1 = rng.integers(-1, 2, size=(3, 3, 4, 32)) / 4.0          # |z1| <= 9, step 1/4
    w2 = np.zeros((3, 3, 32, 32))
    w2[1, 1] = np.eye(32)                                        # z2 = a1 + b2
    w3 = rng.integers(0, 2, size=(3, 3, 32, 4)) / 2.0
    params = [(w1, rng.integers(-2, 3, 32) / 4.0), (w2, rng.integers(-2, 3, 32) / 4.0),
              (w3, rng.integers(-2, 3, 4) / 4.0)]
    x = rng.integers(-1, 2, size=(1, 4, 32, 4)).astype(float)
    y, _, _ = C.forward(params, x)
    ys, _ = C.forward_stored(params, x)
    np.testing.assert_array_equal(y, ys)
    # generic data: stored variant within BF16 rounding of the FP64 passes
    params = C.init_params(1)
    x = rng.normal(size=(2, 8, 32, 4))
    t = rng.normal(size=(2, 8, 32, 4)) * 0.1
    l, g = C.loss_and_grads(params, x, t)
    ls, gs = C.loss_and_grads_stored(params, x, t)
    assert ls == pytest.approx(l, rel=2e-2)
    for (gw, gb), (sw, sb) in zip(g, gs):
        assert np.linalg.norm(sw - gw) < 3e-2 * np.linalg.norm(gw)
        assert np.linalg.norm(sb - gb) < 3e-2 * np.linalg.norm(gb) + 1e-12


def test_flatten_layout_and_round_trip():
    params = C.init_params(3)
    v = C.flatten(params)
    assert v.size == 11588
    # W1[dy=1][dx=2][ci=3][co=5] sits at ((1*3+2)*4+3)*32+5
    assert v[((1 * 3 + 2) * 4 + 3) * 32 + 5] == params[0][0][1, 2, 3, 5]
    assert v[1152 + 7] == params[0][1][7]
    back = C.unflatten(v)
    for (w, b), (w2, b2) in zip(params, back):
        np.testing.assert_array_equal(w, w2)
        np.testing.assert_array_equal(b, b2)


def test_correction_conserves_mass_and_momentum():
    rng = np.random.default_rng(8)
    rho = rng.uniform(0.8, 1.2, size=(16, 16))
    ux, uy = rng.normal(size=(2, 16, 16)) * 0.1
    th = rng.uniform(0.2, 0.3, size=(16, 16))
    d = rng.normal(size=(4, 16, 16)) * 0.01
    r2, u2, v2, t2 = C.apply_correction(rho, ux, uy, th, d)
    assert r2.sum() == pytest.approx(rho.sum(), rel=1e-14)
    assert (r2 * u2).sum() == pytest.approx((rho * ux).sum(), abs=1e-12)
    assert (r2 * v2).sum() == pytest.approx((rho * uy).sum(), abs=1e-12)
    np.testing.assert_allclose(t2, th + d[3])
    # zero increment: unchanged state
    z = C.apply_correction(rho, ux, uy, th, np.zeros((4, 16, 16)))
    for a, b in zip(z, (rho, ux, uy, th)):
        np.testing.assert_allclose(a, b, rtol=1e-15, atol=1e-17)
    # without conservation: plain increments
    r3, u3, v3, _ = C.apply_correction(rho, ux, uy, th, d, conserve=False)
    np.testing.assert_allclose(r3, rho + d[0])
    np.testing.assert_allclose(u3, ux + d[1])
