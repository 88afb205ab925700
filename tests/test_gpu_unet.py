"""GPU parity of the learned warm start's network (twg_unet_* through the C
ABI) against the FP64 reference in oracle/unet.py.

Both sides use the same bf16-representable weights and inputs, round every
stored activation to bf16, and (for gradients) store every layer's
activation gradient in bf16 too; the GPU accumulates in FP32.  Values are
compared with a relative tolerance: 2e-2 of the largest magnitude for
outputs, 1e-2 in norm for gradients (FP32 accumulation, plus the few ReLU
decisions and bf16 roundings that an FP32 value takes differently from an
FP64 one).
"""
import numpy as np
import pytest

import oracle.unet as ou

pytestmark = pytest.mark.gpu


def flat(p):
    return np.concatenate([np.concatenate([p[n + ".w"].ravel(), p[n + ".b"]]) for n, *_ in ou.LAYERS])


def unflat(v):
    p, o = {}, 0
    for n, cin, cout, k in ou.LAYERS:
        nw = cout * cin * k * k
        p[n + ".w"] = v[o:o + nw].reshape(cout, cin, k, k)
        o += nw
        p[n + ".b"] = v[o:o + cout].copy()
        o += cout
    return p


def bf16_params(seed, bias=0.1):
    rng = np.random.default_rng(seed + 100)
    p = ou.init_params(seed)
    for n, *_ in ou.LAYERS:
        p[n + ".w"] = ou.bf16_round(p[n + ".w"])
        p[n + ".b"] = ou.bf16_round(rng.uniform(-bias, bias, p[n + ".b"].shape))
    return p


def inputs(seed, B, H, W):
    rng = np.random.default_rng(seed)
    occ = (rng.uniform(size=(B, H, W)) < 0.2).astype(np.float64)
    gd = rng.uniform(0, 1, size=(B, H, W))
    rt = rng.integers(0, 9, size=(B, H, W)) / 8.0
    return ou.bf16_round(np.stack([occ, gd, rt], axis=-1))  # [B, H, W, 3]


def gpu_net(ctx, p):
    import torch
    from paper_1903_07441_amd import twg
    net = twg.UNet(ctx)
    net.set_params(torch.as_tensor(flat(p), dtype=torch.float32))
    return net


def test_params_round_trip(ctx):
    import torch
    from paper_1903_07441_amd import twg
    net = twg.UNet(ctx)
    v = np.random.default_rng(0).standard_normal(net.n_params).astype(np.float32)
    net.set_params(torch.as_tensor(v))
    back = net.get_params().cpu().numpy()
    assert np.array_equal(back, v)
    net.close()


@pytest.mark.parametrize("B,H,W", [(2, 32, 32), (1, 40, 24), (1, 64, 48)])
def test_forward_matches_oracle(ctx, B, H, W):
    import torch
    p = bf16_params(1)
    x = inputs(2, B, H, W)
    net = gpu_net(ctx, p)
    y = net.forward(torch.as_tensor(x, dtype=torch.float32).cuda()).cpu().numpy()
    for b in range(B):
        want, _ = ou.forward(p, x[b].transpose(2, 0, 1), bf16_acts=True)
        scale = np.max(np.abs(want))
        assert scale > 1e-3
        err = np.max(np.abs(y[b] - want))
        assert err <= 2e-2 * scale, (b, err, scale)
        # most outputs agree far better than the worst one
        assert np.median(np.abs(y[b] - want)) <= 2e-3 * scale
    net.close()


def _grad_parity(ctx, B, H, W, seed, rel_tol, cos_tol):
    import torch
    p = bf16_params(seed)
    x = inputs(seed + 1, B, H, W)
    rng = np.random.default_rng(seed + 2)
    target = rng.uniform(0, 1, size=(B, H, W))
    cls = np.where(rng.uniform(size=(B, H, W)) < 0.7, 0, 1).astype(np.uint8)
    net = gpu_net(ctx, p)
    grads = torch.empty(net.n_params, dtype=torch.float32, device="cuda")
    loss = net.loss_grad(torch.as_tensor(x, dtype=torch.float32).cuda(),
                         torch.as_tensor(target, dtype=torch.float32).cuda(),
                         torch.as_tensor(cls).cuda(), grads=grads)
    torch.cuda.synchronize()
    # the oracle stores activations and activation gradients in bf16 as the
    # GPU does; only the FP32 accumulation (and ReLU decisions an FP32
    # pre-activation takes differently) separate the two
    want_loss, want = ou.loss_and_grads(p, [x[b].transpose(2, 0, 1) for b in range(B)], list(target),
                                        [cls[b] == 0 for b in range(B)], bf16_acts=True, bf16_grads=True)
    assert abs(float(loss.item()) - want_loss) <= 1e-3 * want_loss
    g = unflat(grads.cpu().numpy().astype(np.float64))
    worst = 0.0
    for n, *_ in ou.LAYERS:
        for part in (".w", ".b"):
            a, b = g[n + part], want[n + part]
            nb = np.linalg.norm(b)
            assert nb > 0, n + part
            rel = np.linalg.norm(a - b) / nb
            cos = float(np.sum(a * b) / (np.linalg.norm(a) * nb))
            worst = max(worst, rel)
            print(f"B={B} {H}x{W} {n + part}: rel {rel:.2e} cos {cos:.7f}", flush=True)
            assert rel <= rel_tol and cos >= cos_tol, (n + part, rel, cos)
    net.close()
    return worst


def test_gradients_match_oracle(ctx):
    # P13: GPU gradients within ~1e-2 of the FP64 reference on the same bf16
    # operands (FP32 accumulation)
    _grad_parity(ctx, 2, 32, 32, 3, 1e-2, 0.9999)


def _splits_summing_several_tiles(B, H, W):
    """Layers whose weight-gradient kernel sums more than one 16 x 16 pixel
    tile per split of the pixel reduction: the kernel splits the reduction of
    a layer with CIN input channels into max(1, 256 / (CIN / 32)) parts (at
    most one per tile) over B * ceil(h / 16) * ceil(w / 16) tiles at the
    layer's resolution h x w."""
    layers = {"e0": (32, 1), "e1": (32, 2), "e2": (64, 4), "e3": (128, 8),
              "d2": (256, 4), "d1": (128, 2), "d0": (64, 1)}
    out = set()
    for name, (cin, down) in layers.items():
        h, w = H // down, W // down
        ntile = B * ((h + 15) // 16) * ((w + 15) // 16)
        if ntile > max(1, 256 // (cin // 32)):
            out.add(name)
    return out


def test_gradients_match_oracle_multi_tile_splits(ctx):
    # the training batch (16 x 256 x 256) makes every split of the weight
    # gradient's pixel reduction sum several tiles in layers e0, e1, e2, d2,
    # d1 and d0; this batch does the same, so the accumulation over tiles
    # within a split is compared with the oracle too
    train = _splits_summing_several_tiles(16, 256, 256)
    here = _splits_summing_several_tiles(9, 256, 256)
    print(f"multi-tile splits: training {sorted(train)}, test {sorted(here)}", flush=True)
    assert train <= here and len(train) == 6
    _grad_parity(ctx, 9, 256, 256, 21, 1e-2, 0.9999)


def test_gradients_deterministic(ctx):
    import torch
    B, H, W = 2, 48, 32
    p = bf16_params(6)
    x = torch.as_tensor(inputs(7, B, H, W), dtype=torch.float32).cuda()
    rng = np.random.default_rng(8)
    t = torch.as_tensor(rng.uniform(0, 1, size=(B, H, W)), dtype=torch.float32).cuda()
    c = torch.as_tensor(np.where(rng.uniform(size=(B, H, W)) < 0.7, 0, 1).astype(np.uint8)).cuda()
    net = gpu_net(ctx, p)
    g1 = torch.empty(net.n_params, dtype=torch.float32, device="cuda")
    g2 = torch.empty_like(g1)
    net.loss_grad(x, t, c, grads=g1)
    net.loss_grad(x, t, c, grads=g2)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)
    net.close()


def test_adam_steps_match_oracle(ctx):
    """Two Adam steps.  The first step of Adam moves every parameter by lr
    times the sign of its gradient, so after it GPU and oracle agree wherever
    the two gradients have the same sign (they may differ only where a
    gradient is near zero).  The second step depends on the ratio of the two
    steps' gradients, so it agrees to the gradients' relative accuracy."""
    import torch
    B, H, W = 1, 32, 32
    p = bf16_params(9)
    x = inputs(10, B, H, W)
    rng = np.random.default_rng(11)
    target = rng.uniform(0, 1, size=(B, H, W))
    cls = np.zeros((B, H, W), dtype=np.uint8)
    lr = 1e-3
    net = gpu_net(ctx, p)
    xt = torch.as_tensor(x, dtype=torch.float32).cuda()
    tt = torch.as_tensor(target, dtype=torch.float32).cuda()
    ct = torch.as_tensor(cls).cuda()
    po = {k: v.copy() for k, v in p.items()}
    state = {}
    for step in range(2):
        net.train_step(xt, tt, ct, lr)
        _, g = ou.loss_and_grads(po, [x[0].transpose(2, 0, 1)], [target[0]], [cls[0] == 0], bf16_acts=True)
        po = ou.adam_step(po, g, state, lr)
        got = net.get_params().cpu().numpy().astype(np.float64)
        d = np.abs(got - flat(po))
        if step == 0:
            assert np.max(d) <= 2 * lr + 1e-6
            assert np.mean(d > 1e-6) <= 0.02, np.mean(d > 1e-6)
        else:
            assert np.max(d) <= 4 * lr + 1e-6
            assert np.median(d) <= 0.05 * lr, np.median(d)
    net.close()


def test_features_definition(ctx, orc):
    import torch
    from paper_1903_07441_amd import scenarios, twg
    from conftest import scenario_tensors
    sc = scenarios.scenario("warped512", 1, side=100)
    pos, vel, rad = scenario_tensors(sc)
    cls, ring = ctx.rasterize(sc["nx"], sc["ny"], sc["robot"], sc["goal"], pos, vel, rad, W=sc["W"],
                              robot_speed=sc["vr"])
    net = twg.UNet(ctx)
    f = net.features(cls, ring, sc["goal"]).cpu().numpy()
    assert f.shape == (104, 104, 3)
    oc, orr = orc.rasterize(sc)
    occ = np.ones((104, 104), np.float32)
    occ[:100, :100] = np.isin(oc, (orc.OBST, orc.WALL)).astype(np.float32)
    assert np.array_equal(f[..., 0], occ)
    yy, xx = np.mgrid[0:104, 0:104]
    gx, gy = sc["goal"]
    d2 = ((xx - gx) ** 2 + (yy - gy) ** 2).astype(np.float32)
    inv = np.float32(1.0 / (100 * np.sqrt(2.0)))
    assert np.allclose(f[..., 1], np.sqrt(d2) * inv, rtol=0, atol=2e-7)
    rt = np.zeros((104, 104), np.float32)
    rt[:100, :100] = orr.astype(np.float32) * (np.float32(1.0) / np.float32(orr.max()))
    assert np.array_equal(f[..., 2], rt)
    net.close()


def test_warm_start_field(ctx):
    import torch
    from paper_1903_07441_amd import scenarios, twg
    from conftest import scenario_tensors
    sc = scenarios.scenario("warped512", 2, side=90)
    pos, vel, rad = scenario_tensors(sc)
    nx, ny = sc["nx"], sc["ny"]
    cls = torch.empty((ny, 96), dtype=torch.uint8, device="cuda")[:, :nx]
    ring = torch.empty((ny, 96), dtype=torch.uint16, device="cuda")[:, :nx]
    ctx.rasterize(nx, ny, sc["robot"], sc["goal"], pos, vel, rad, W=sc["W"], robot_speed=sc["vr"], cls=cls,
                  ring=ring)
    net = gpu_net(ctx, bf16_params(12))
    x = net.features(cls, ring, sc["goal"])
    y = net.forward(x[None].contiguous())[0, :ny, :nx].cpu().numpy()
    psi = torch.full((ny, 96), -7.0, dtype=torch.float32, device="cuda")[:, :nx]
    net.warm_start(cls, ring, sc["goal"], psi)
    got = psi.cpu().numpy()
    c = cls.cpu().numpy()
    free = c == twg.FREE
    assert np.array_equal(got[free], np.clip(y[free], 0, 1))
    assert np.all(got[(c == twg.OBST) | (c == twg.WALL)] == 0)
    assert np.all(got[c == twg.GOAL] == 1)
    net.close()


@pytest.mark.parametrize("where,value", [("conv", float("nan")), ("head_bias", float("inf"))])
def test_warm_start_falls_back_on_non_finite_network(ctx, where, value):
    # a network whose output is not finite (NaN parameters, an infinite
    # bias) is rejected: every FREE cell holds the plain start 0.5, the
    # status word reads NET_FALLBACK, and the relaxation converges from that
    # field as from the plain start; the same call with finite parameters
    # reports OK
    import torch
    from paper_1903_07441_amd import scenarios, twg
    from conftest import scenario_tensors
    sc = scenarios.scenario("warped512", 4, side=128)
    pos, vel, rad = scenario_tensors(sc)
    nx, ny = sc["nx"], sc["ny"]
    cls, ring = ctx.rasterize(nx, ny, sc["robot"], sc["goal"], pos, vel, rad, W=sc["W"], robot_speed=sc["vr"])
    params = flat(bf16_params(5)).astype(np.float32)
    net = twg.UNet(ctx)
    net.set_params(torch.as_tensor(params))
    status = torch.full((1,), -99, dtype=torch.int32, device="cuda")
    psi = torch.full((ny, nx), -7.0, dtype=torch.float32, device="cuda")
    net.warm_start(cls, ring, sc["goal"], psi, status=status)
    assert int(status.item()) == twg.OK
    bad = params.copy()
    if where == "conv":
        bad[100] = np.float32(value)      # a weight of the first conv
    else:
        bad[-1] = np.float32(value)       # the head's bias
    net.set_params(torch.as_tensor(bad))
    psi.fill_(-7.0)
    net.warm_start(cls, ring, sc["goal"], psi, status=status)
    print(f"fallback {where}={value}: status {int(status.item())}", flush=True)
    assert int(status.item()) == twg.NET_FALLBACK
    got = psi.cpu().numpy()
    c = cls.cpu().numpy()
    assert np.all(got[c == twg.FREE] == 0.5)
    assert np.all(got[(c == twg.OBST) | (c == twg.WALL)] == 0)
    assert np.all(got[c == twg.GOAL] == 1)
    st = ctx.relax(cls, psi, None, tol=1e-6, init=twg.INIT_KEEP)
    ref = torch.empty_like(psi)
    st_ref = ctx.relax(cls, ref, None, tol=1e-6, init=twg.INIT_HALF)
    assert st["status"] == twg.OK and st["sweeps"] == st_ref["sweeps"] and torch.equal(psi, ref)
    net.close()


def test_training_lowers_loss(ctx, orc):
    """A few Adam steps on relaxed 64x64 fields lower the masked MSE."""
    import torch
    from paper_1903_07441_amd import scenarios, twg
    from conftest import scenario_tensors
    B = 4
    xs, ts, cs = [], [], []
    net = twg.UNet(ctx)
    p = ou.init_params(0)
    net.set_params(torch.as_tensor(flat(p), dtype=torch.float32))
    for i in range(B):
        sc = scenarios.scenario("static64", 10 + i)
        oc, orr = orc.rasterize(sc)
        field, _ = orc.relax(oc, tol=1e-9)
        cls = torch.as_tensor(oc).cuda().contiguous()
        ring = torch.as_tensor(orr.astype(np.uint16)).cuda().contiguous()
        xs.append(net.features(cls, ring, sc["goal"]))
        ts.append(torch.as_tensor(field, dtype=torch.float32).cuda())
        cs.append(cls)
    x, t, c = torch.stack(xs), torch.stack(ts), torch.stack(cs)
    first = float(net.loss_grad(x, t, c).item())
    for _ in range(40):
        loss = net.train_step(x, t, c, 2e-3)
    last = float(net.loss_grad(x, t, c).item())
    assert np.isfinite(last) and last < 0.5 * first, (first, last)
    net.close()


def test_rejects_bad_arguments(ctx):
    import torch
    from paper_1903_07441_amd import twg
    net = twg.UNet(ctx)
    x = torch.zeros((1, 12, 16, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(twg.TwgError):
        net.forward(x)  # H not a multiple of 8
    with pytest.raises(twg.TwgError):
        net.adam_step(0.0)
    net.close()


@pytest.mark.parametrize("factor", [4, 8])
def test_coarse_features_and_target_match_oracle(ctx, orc, factor):
    # the coarse inputs, the training mask and the coarse target of a ragged
    # grid against the oracle's definitions (FP32 on the GPU)
    import torch
    from paper_1903_07441_amd import scenarios, twg
    from conftest import scenario_tensors
    sc = scenarios.custom(100, 70, 30, rad=(2.0, 6.0), seed=5)
    pos, vel, rad = scenario_tensors(sc)
    nx, ny = sc["nx"], sc["ny"]
    cls, ring = ctx.rasterize(nx, ny, sc["robot"], sc["goal"], pos, vel, rad, W=sc["W"], robot_speed=sc["vr"])
    net = twg.UNet(ctx)
    x, ccls = net.features_coarse(cls, ring, sc["goal"], factor)
    c, r = cls.cpu().numpy(), ring.cpu().numpy()
    wx, wmask = ou.coarse_features(c, r, sc["goal"], factor)
    print(f"coarse features factor {factor}: frame {tuple(x.shape[:2])}", flush=True)
    assert x.shape == wx.shape
    xg = x.cpu().numpy()
    assert np.array_equal(xg[..., 0], wx[..., 0].astype(np.float32))
    assert np.allclose(xg[..., 1], wx[..., 1], rtol=0, atol=2e-7)
    assert np.allclose(xg[..., 2], wx[..., 2], rtol=0, atol=2e-7)
    assert np.array_equal(ccls.cpu().numpy(), wmask)
    psi = torch.rand((ny, nx), generator=torch.Generator().manual_seed(factor)).cuda()
    t = net.coarse_target(cls, psi, factor).cpu().numpy()
    want = ou.coarse_target(psi.cpu().numpy().astype(np.float64), c, factor)
    assert np.allclose(t, want, rtol=0, atol=1e-6)
    net.close()


def test_coarse_warm_start_is_the_network_output_interpolated(ctx, orc):
    # warm_start_coarse = the oracle's interpolation of the network's own
    # coarse output (the forward pass is checked against the FP64 reference
    # elsewhere)
    import torch
    from paper_1903_07441_amd import scenarios, twg
    from conftest import scenario_tensors
    sc = scenarios.scenario("warped512", 6, side=120)
    pos, vel, rad = scenario_tensors(sc)
    nx, ny = sc["nx"], sc["ny"]
    cls, ring = ctx.rasterize(nx, ny, sc["robot"], sc["goal"], pos, vel, rad, W=sc["W"], robot_speed=sc["vr"])
    net = gpu_net(ctx, bf16_params(21))
    f = 4
    x, _ = net.features_coarse(cls, ring, sc["goal"], f)
    yc = net.forward(x[None].contiguous())[0].cpu().numpy().astype(np.float64)
    psi = torch.full((ny, nx), -3.0, dtype=torch.float32, device="cuda")
    status = torch.full((1,), -9, dtype=torch.int32, device="cuda")
    net.warm_start_coarse(cls, ring, sc["goal"], psi, f, status=status)
    want = ou.upsample_field_f(yc, cls.cpu().numpy(), f)
    got = psi.cpu().numpy()
    print(f"coarse warm start: max |gpu - oracle| {np.max(np.abs(got - want)):.2e}", flush=True)
    assert int(status.item()) == twg.OK
    assert np.allclose(got, want, rtol=0, atol=1e-6)
    net.close()
