"""Learned closure on the GPU: BF16-MFMA network kernels, Adam, restriction
and the batch coupling against the FP64 oracle (oracle/cnn_oracle.py).

The oracle's stored-precision passes round to BF16 exactly where the GPU
stores BF16 (standardised input, weights, hidden activations, propagated
gradients).  What remains is FP32 accumulation against FP64 and the rare
BF16 rounding decision that the two accumulations place on opposite sides
of a boundary (a tie flip, one BF16 spacing of a stored value).  The network
outputs and the parameter gradients are therefore compared element by
element: each element must lie within one BF16 spacing of the oracle's value
(2^(e - 7) for a value in [2^e, 2^(e + 1))), except for a counted set of
outliers -- elements whose value is small against the terms it sums, where
a tie flip or the accumulation order moves it by more than its own spacing
-- which must be at most 1 % of the elements and each within one BF16 spacing
of the absolute sum of the terms (sum |w h| + |b| for an output, sum over
pixels of |activation| |gradient| for a weight gradient)."""
import numpy as np
import pytest

import hlbm_inputs as hi
import oracle
from oracle import cnn_oracle as C

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2002_03644_amd import CNN, BatchSolver, Params, restrict  # noqa: E402

NORM = (np.array([1.0, 0.01, -0.02, 0.2], np.float32), np.array([0.05, 0.1, 0.1, 0.02], np.float32),
        np.array([1e-4, -2e-4, 3e-4, 1e-5], np.float32),
        np.array([2e-3, 3e-3, 1e-3, 5e-4], np.float32))


def rand_params(seed):
    rng = np.random.default_rng(seed)
    params = C.init_params(seed)
    params = [(w * (3.0 if k == 2 else 1.0), rng.normal(size=b.shape) * 0.05)
              for k, (w, b) in enumerate(params)]
    return params


def fields(B, H, W, seed):
    rng = np.random.default_rng(seed)
    x = np.empty((B, 4, H, W), np.float32)
    for c in range(4):
        x[:, c] = NORM[0][c] + NORM[1][c] * rng.normal(size=(B, H, W))
    t = np.empty((B, 4, H, W), np.float32)
    for c in range(4):
        t[:, c] = NORM[2][c] + NORM[3][c] * rng.normal(size=(B, H, W))
    return x, t


def standardise(a, mean, std):
    """As the kernels do it, in FP32: (a - mean) * (1 / std); NHWC out."""
    inv = (np.float32(1.0) / std).astype(np.float32)
    s = (a - mean[None, :, None, None]) * inv[None, :, None, None]
    return np.ascontiguousarray(s.astype(np.float32).transpose(0, 2, 3, 1)).astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def bf16_spacing(a):
    """Spacing of BF16 numbers at |a|: 2^(e - 7) for |a| in [2^e, 2^(e + 1))."""
    a = np.abs(np.asarray(a, dtype=np.float64))
    e = np.floor(np.log2(np.maximum(a, 1e-300)))
    return np.where(a > 0, 2.0 ** (e - 7), 0.0)


def check_elementwise(got, want, abs_sum, what, max_outlier_frac=0.01):
    """Every element within one BF16 spacing of the oracle value, or a
    counted outlier within one BF16 spacing of its absolute sum."""
    err = np.abs(got - want)
    inside = err <= bf16_spacing(want)
    out = ~inside
    n_out = int(out.sum())
    frac = n_out / err.size
    worst = float((err[out] / bf16_spacing(abs_sum[out])).max()) if n_out else 0.0
    ratio = float((err / np.maximum(bf16_spacing(want), 1e-300)).max())
    print(f"{what}: {err.size} elements, {n_out} beyond one spacing of the value "
          f"({100 * frac:.3f} %), worst outlier {worst:.3f} spacings of its absolute sum, "
          f"largest error {ratio:.3g} spacings of the value")
    assert frac <= max_outlier_frac, (what, n_out, err.size)
    assert (err[out] <= bf16_spacing(abs_sum[out])).all(), (what, worst)


def make_net(B, H, W, params):
    net = CNN(B, H, W, C.flatten(params).astype(np.float32))
    net.set_norm(*NORM)
    return net


@pytest.mark.parametrize("B,H,W", [(3, 12, 64), (2, 36, 32), (2, 256, 256)])
def test_forward_matches_oracle(B, H, W):
    params = rand_params(1)
    x, _ = fields(B, H, W, 2)
    net = make_net(B, H, W, params)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    xs = standardise(x, NORM[0], NORM[1])
    ys, acts = C.forward_stored([(w, b) for w, b in params], xs)
    # absolute sum of the last layer's terms, per output element
    w3, b3 = params[2]
    s3 = C.conv3x3(np.abs(acts[2]), np.abs(C.bf16(w3)), np.abs(b3))
    # compare in standardised units (the de-standardisation is one FP32 FMA)
    std = NORM[3][None, :, None, None].astype(np.float64)
    mean = NORM[2][None, :, None, None].astype(np.float64)
    y_std = ((y - mean) / std).transpose(0, 2, 3, 1)
    check_elementwise(y_std, ys, s3, f"forward {B}x{H}x{W}")
    # and, in raw units, a relative L2 summary
    yo = ys.transpose(0, 3, 1, 2) * std + mean
    for c in range(4):
        assert rel(y[:, c] - NORM[2][c], yo[:, c] - NORM[2][c]) < 1e-3


@pytest.mark.parametrize("B,H,W", [(3, 12, 64), (2, 36, 32), (1, 256, 256)])
def test_gradients_match_oracle(B, H, W):
    params = rand_params(3)
    x, t = fields(B, H, W, 4)
    net = make_net(B, H, W, params)
    loss = net.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    g = C.unflatten(net.grads().cpu().numpy().astype(np.float64))
    xs = standardise(x, NORM[0], NORM[1])
    ts = standardise(t, NORM[2], NORM[3])
    lo, go = C.loss_and_grads_stored(params, xs, ts)
    assert float(loss.item()) == pytest.approx(lo, rel=1e-3)
    # absolute sums of the gradient sums over the pixels: the oracle's stored
    # activations and stored back-propagated gradients, in absolute value
    y, acts = C.forward_stored(params, xs)
    gk = C.bf16(2.0 * (y - ts) / y.size)
    for k in (2, 1, 0):
        wb = C.bf16(params[k][0])
        _, sw, sb = C.conv3x3_grad(np.abs(acts[k]), np.abs(wb), np.abs(gk))
        check_elementwise(g[k][0], go[k][0], sw, f"dW{k + 1} {B}x{H}x{W}")
        check_elementwise(g[k][1], go[k][1], sb, f"db{k + 1} {B}x{H}x{W}")
        ew, eb = rel(g[k][0], go[k][0]), rel(g[k][1], go[k][1])
        print(f"layer {k + 1}: dW rel L2 {ew:.2e}, db rel L2 {eb:.2e}")
        if k > 0:
            gx, _, _ = C.conv3x3_grad(acts[k], wb, gk)
            gk = C.bf16(gx * (acts[k] > 0))


def test_batch_index_selects_samples():
    """idx gathers samples out of a larger pool, for inputs and targets."""
    H, W = 8, 32
    params = rand_params(5)
    x, t = fields(5, H, W, 6)
    net = make_net(3, H, W, params)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    idx = torch.tensor([4, 0, 2], dtype=torch.int32, device="cuda")
    y_idx = net.forward(xd, idx=idx)
    y_dir = net.forward(xd[[4, 0, 2]].contiguous())
    assert torch.equal(y_idx, y_dir)
    l1 = net.loss_grad(xd, td, idx=idx).clone()
    g1 = net.grads().clone()
    l2 = net.loss_grad(xd[[4, 0, 2]].contiguous(), td[[4, 0, 2]].contiguous())
    assert torch.equal(l1, l2) and torch.equal(g1, net.grads())


def test_adam_steps_match_oracle_and_repack():
    B, H, W = 2, 16, 64
    params = rand_params(7)
    x, t = fields(B, H, W, 8)
    net = make_net(B, H, W, params)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    opt = C.Adam(params, lr=1e-3)
    cur = [(w.copy(), b.copy()) for w, b in params]
    for step in range(2):
        net.loss_grad(xd, td)
        g = C.unflatten(net.grads().cpu().numpy().astype(np.float64))
        assert net.adam(1e-3) == step + 1
        cur = opt.step(cur, g)
        got = net.params().cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(got, C.flatten(cur), rtol=0, atol=2e-6)
    # the packed BF16 weights follow the update: the forward pass equals a
    # fresh network built from the updated parameters
    fresh = make_net(B, H, W, C.unflatten(net.params().cpu().numpy()))
    assert torch.equal(net.forward(xd), fresh.forward(xd))


def test_training_reduces_loss():
    """A few hundred Adam steps on a fixed smooth target map."""
    B, H, W = 4, 32, 32
    x, _ = fields(B, H, W, 10)
    xs = standardise(x, NORM[0], NORM[1])
    teacher = rand_params(11)
    yt, _, _ = C.forward(teacher, xs)
    t = np.ascontiguousarray((yt.transpose(0, 3, 1, 2) * NORM[3][None, :, None, None]
                              + NORM[2][None, :, None, None]).astype(np.float32))
    net = make_net(B, H, W, C.init_params(12))
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    first = float(net.loss_grad(xd, td).item())
    for _ in range(300):
        loss = net.train_step(xd, td, 3e-3)
    last = float(loss.item())
    print(f"loss {first:.4f} -> {last:.4f}")
    assert last < 0.2 * first


def test_restriction_matches_oracle():
    B, ny, nx, f = 2, 48, 64, 4
    rng = np.random.default_rng(13)
    r = rng.uniform(0.5, 1.5, size=(B, ny, nx)).astype(np.float32)
    u, v = (rng.normal(size=(2, B, ny, nx)) * 0.1).astype(np.float32)
    th = rng.uniform(0.1, 0.3, size=(B, ny, nx)).astype(np.float32)
    out = restrict(*[torch.from_numpy(a).cuda() for a in (r, u, v, th)], f, batch=B)
    out = out.cpu().numpy().astype(np.float64)
    for b in range(B):
        ref = C.restrict(r[b].astype(np.float64), u[b].astype(np.float64),
                         v[b].astype(np.float64), th[b].astype(np.float64), f)
        for c in range(4):
            np.testing.assert_allclose(out[b, c], ref[c], rtol=2e-6, atol=2e-7)


def closure_batch(count=3, n=64, seed=14):
    params, flds = [], []
    for k in range(count):
        f = hi.random_smooth(n, n, seed=seed + k, amp=0.03, theta0=hi.THETA_PAPER)
        params.append(Params(n, n, dtype="f32", mu=1e-3, theta_ref=hi.THETA_PAPER))
        flds.append(f)
    return params, flds


def moments_cat(B):
    m = B.moments()
    return torch.stack([torch.stack([d[k].reshape(-1) for d in m]) for k in
                        ("rho", "ux", "uy", "theta")])


@pytest.mark.parametrize("conserve", [True, False])
def test_batch_correction_matches_oracle(conserve):
    params, flds = closure_batch()
    B = BatchSolver(params, flds)
    B.step(3, graph=False)
    x = moments_cat(B).contiguous()                   # [4][count][n]
    rng = np.random.default_rng(15)
    scale = np.array([1e-3, 2e-3, 2e-3, 1e-4])[:, None, None]
    d = torch.from_numpy((rng.normal(size=tuple(x.shape)) * scale).astype(np.float32)).cuda()
    B.correct(x, d, conserve=conserve)
    x2 = moments_cat(B).double().cpu().numpy()
    xc = x.double().cpu().numpy()
    dc = d.double().cpu().numpy()
    for k in range(len(params)):
        want = C.apply_correction(xc[0, k], xc[1, k], xc[2, k], xc[3, k], dc[:, k],
                                  conserve=conserve)
        for c in range(4):
            err = np.abs(x2[c, k] - want[c]).max()
            assert err < 5e-6, (k, c, err)
        if conserve:
            assert x2[0, k].sum() == pytest.approx(xc[0, k].sum(), rel=1e-6)
            mom0 = (xc[0, k] * xc[1, k]).sum()
            assert abs((x2[0, k] * x2[1, k]).sum() - mom0) < 1e-5 * x2[0, k].sum() * 0.05


def test_correction_moves_only_the_equilibrium():
    """F' - F = f^eq(X') - f^eq(X) (HLBM oracle's equilibrium), checked on a
    single-domain batch through its populations."""
    params, flds = closure_batch(count=1, n=32, seed=20)
    B = BatchSolver(params, flds)
    B.step(2, graph=False)
    snap = B.save_state()
    x = moments_cat(B).contiguous()
    rng = np.random.default_rng(21)
    d = torch.from_numpy((rng.normal(size=tuple(x.shape)) *
                          np.array([1e-3, 1e-3, 1e-3, 1e-4])[:, None, None]).astype(np.float32)).cuda()
    B.correct(x, d, conserve=False)
    after = B.save_state()
    nx = ny = 32
    n = nx * ny
    # a saved state is the current buffer: ten planes of FP32 deviations,
    # rows padded to 64 elements, planes to a multiple of 64
    pitch = -(-nx // 64) * 64
    plane = -(-(pitch * ny) // 64) * 64

    def dense(buf):
        a = buf.view(torch.float32)[: 10 * plane].reshape(10, plane)[:, : pitch * ny]
        return a.reshape(10, ny, pitch)[:, :, :nx].reshape(10, n).double().cpu().numpy()
    s0, s1 = dense(snap), dense(after)
    xc = x.double().cpu().numpy()[:, 0]
    dc = d.double().cpu().numpy()[:, 0]
    r2, u2, v2, t2 = C.apply_correction(xc[0], xc[1], xc[2], xc[3], dc, conserve=False)
    dfe = np.stack([oracle.feq(r2[i], u2[i], v2[i], t2[i]) - oracle.feq(xc[0][i], xc[1][i],
                                                                       xc[2][i], xc[3][i])
                    for i in range(n)], axis=1)
    np.testing.assert_allclose(s1[:9] - s0[:9], dfe, rtol=0, atol=2e-7)
    ds = oracle.entropy_from_theta(r2, t2, 1.4) - oracle.entropy_from_theta(xc[0], xc[3], 1.4)
    np.testing.assert_allclose(s1[9] - s0[9], ds, rtol=0, atol=2e-6)


@pytest.mark.parametrize("kernel", ["strips", "tiles"])
@pytest.mark.parametrize("every", [1, 2, 3])
def test_closure_step_graph_equals_eager_and_manual_sequence(every, kernel):
    """Corrected cycles (`every` plain steps, then the correction): graph
    replay, eager launches and a manual step / moments / forward / correct
    sequence agree bit for bit.  With the tile kernels the cycle's last step
    writes the network's input moments itself; they must equal the separate
    moments pass of the manual sequence."""
    params, flds = closure_batch(count=3, n=64, seed=30)
    net_params = rand_params(31)
    net_params[2] = (net_params[2][0] * 0.01, net_params[2][1] * 0.0)
    A = BatchSolver(params, flds)
    E = BatchSolver(params, flds)
    M = BatchSolver(params, flds)
    if kernel == "tiles":
        for S in (A, E, M):
            S.set_tile(32, 16, kernel="tiles")
        assert A.plan()[:2] == (2, "tiles")
    na, ne, nm = (make_net(3, 64, 64, net_params) for _ in range(3))
    for nt in (na, ne, nm):
        nt.set_norm(np.array([1.0, 0, 0, 0.2], np.float32), np.array([0.03, 0.05, 0.05, 0.01], np.float32),
                    np.zeros(4, np.float32), np.array([1e-4, 1e-4, 1e-4, 1e-5], np.float32))
    x = torch.empty(4, 3, 64 * 64, device="cuda")
    for rep in range(3):
        A.closure_step(na, 4, every=every, graph=True)
        E.closure_step(ne, 4, every=every, graph=False)
        for _ in range(4):
            M.step(every, graph=False)
            x.copy_(moments_cat(M))
            dl = nm.forward(x, batch=3, sstride=64 * 64, cstride=3 * 64 * 64)
            d = dl.permute(1, 0, 2, 3).reshape(4, 3, -1).contiguous()
            M.correct(x, d, conserve=True)
        torch.cuda.synchronize()
        ma, me, mm = moments_cat(A), moments_cat(E), moments_cat(M)
        assert torch.equal(ma, me), rep
        assert torch.equal(ma, mm), rep
        assert torch.isfinite(ma).all()
    assert A.steps == E.steps == M.steps == 12 * every


@pytest.mark.parametrize("B,H,W", [(3, 12, 64), (2, 256, 256), (1, 36, 128), (5, 8, 192)])
def test_fused_inference_equals_layer_kernels(B, H, W):
    """The one-kernel inference (activations in LDS) and the per-layer
    kernels share every rounding point, so they agree bit for bit; the
    clamp bounds the standardised output."""
    params = rand_params(21)
    x, _ = fields(B, H, W, 22)
    xd = torch.from_numpy(x).cuda()
    net = make_net(B, H, W, params)
    y_fused = net.forward(xd).clone()
    net.set_fused(False)
    y_layer = net.forward(xd)
    assert torch.equal(y_fused, y_layer)
    ys, acts = C.forward_stored(params, standardise(x, NORM[0], NORM[1]))
    s3 = C.conv3x3(np.abs(acts[2]), np.abs(C.bf16(params[2][0])), np.abs(params[2][1]))
    std = NORM[3][None, :, None, None].astype(np.float64)
    mean = NORM[2][None, :, None, None].astype(np.float64)
    for clip in (0.5, 2.0):
        net.set_output_clip(clip)
        for fused in (True, False):
            net.set_fused(fused)
            y = net.forward(xd).cpu().numpy().astype(np.float64)
            y_std = ((y - mean) / std).transpose(0, 2, 3, 1)
            assert np.abs(y_std).max() <= clip * (1 + 2 ** -20)
            check_elementwise(y_std, np.clip(ys, -clip, clip), s3,
                              f"clip {clip} fused {fused} {B}x{H}x{W}")


@pytest.mark.parametrize("kernel", ["tiles", "strips"])
def test_closure_step_mixed_call_lengths(kernel):
    """Calls of 2, 4, 1, 3, 2, 11 and 9 cycles (two-cycle graphs and
    eight-cycle ones, captured with and without a pending correction at
    their start; with the tile kernels the correction is applied by the next
    cycle's first step and the last one of each call before it returns)
    equal the same calls run eagerly, bit for bit, and the state after every
    call is the corrected one (a plain moments pass of it equals the one of
    the eager run)."""
    params, flds = closure_batch(count=3, n=64, seed=40)
    net_params = rand_params(41)
    net_params[2] = (net_params[2][0] * 0.01, net_params[2][1] * 0.0)
    A = BatchSolver(params, flds)
    E = BatchSolver(params, flds)
    for S in (A, E):
        if kernel == "tiles":
            S.set_tile(32, 16, kernel="tiles")
        else:
            S.set_tile(64, 8)
    na, ne = (make_net(3, 64, 64, net_params) for _ in range(2))
    for nt in (na, ne):
        nt.set_norm(np.array([1.0, 0, 0, 0.2], np.float32), np.array([0.03, 0.05, 0.05, 0.01], np.float32),
                    np.zeros(4, np.float32), np.array([1e-4, 1e-4, 1e-4, 1e-5], np.float32))
    for rep, n in enumerate((2, 4, 1, 3, 2, 11, 9)):
        A.closure_step(na, n, every=4, graph=True)
        E.closure_step(ne, n, every=4, graph=False)
        torch.cuda.synchronize()
        assert torch.equal(moments_cat(A), moments_cat(E)), rep
    assert A.steps == E.steps == 4 * 32


def test_closure_step_one_step_tiles_equal_manual_sequence():
    """Domains extrapolated along x take one step per launch: the one-step
    tile kernel then applies the pending correction in the cycle's first
    launch (three launches per cycle); the result equals a manual
    step/moments/forward/correct sequence bit for bit."""
    import dataclasses
    params, flds = closure_batch(count=3, n=64, seed=50)
    params = [dataclasses.replace(p, bc_x="extrapolate") for p in params]
    net_params = rand_params(51)
    net_params[2] = (net_params[2][0] * 0.01, net_params[2][1] * 0.0)
    A = BatchSolver(params, flds)
    M = BatchSolver(params, flds)
    for S in (A, M):
        S.set_tile(32, 16, kernel="tiles")
    assert A.plan() == (1, "tiles", 32, 16)
    na, nm = (make_net(3, 64, 64, net_params) for _ in range(2))
    for nt in (na, nm):
        nt.set_norm(np.array([1.0, 0, 0, 0.2], np.float32), np.array([0.03, 0.05, 0.05, 0.01], np.float32),
                    np.zeros(4, np.float32), np.array([1e-4, 1e-4, 1e-4, 1e-5], np.float32))
    x = torch.empty(4, 3, 64 * 64, device="cuda")
    for rep in range(2):
        A.closure_step(na, 3, every=3, graph=True)
        for _ in range(3):
            M.step(3, graph=False)
            x.copy_(moments_cat(M))
            dl = nm.forward(x, batch=3, sstride=64 * 64, cstride=3 * 64 * 64)
            d = dl.permute(1, 0, 2, 3).reshape(4, 3, -1).contiguous()
            M.correct(x, d, conserve=True)
        torch.cuda.synchronize()
        assert torch.equal(moments_cat(A), moments_cat(M)), rep
    assert A.steps == M.steps == 18
