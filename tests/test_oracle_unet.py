"""Pins of the FP64 reference network: library correlation, central finite
differences, adjoint identities, bfloat16 rounding against torch's cast, the
parameter count, and the first Adam step's closed form."""
import numpy as np
import pytest
import scipy.signal
import torch

from oracle import unet


def test_conv_is_cross_correlation_with_zero_padding():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(3, 9, 7))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    got = unet.conv(x, w, b)
    for o in range(4):
        want = b[o] + sum(scipy.signal.correlate2d(x[c], w[o, c], mode="same") for c in range(3))
        np.testing.assert_allclose(got[o], want, rtol=1e-12, atol=1e-12)
    w1 = rng.normal(size=(2, 3, 1, 1))
    np.testing.assert_allclose(unet.conv(x, w1, np.zeros(2)),
                               np.einsum("oc,chw->ohw", w1[:, :, 0, 0], x), rtol=1e-12)


def test_pool_and_up_adjoints():
    rng = np.random.default_rng(1)
    a = rng.normal(size=(3, 4, 6))
    b = rng.normal(size=(3, 8, 12))
    assert np.isclose((unet.up(a) * b).sum(), (a * unet.up_backward(b)).sum())
    assert np.isclose((unet.pool(b) * a).sum(), (b * unet.pool_backward(a)).sum())
    np.testing.assert_allclose(unet.pool(unet.up(a)), a)


def test_conv_backward_adjoint():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(5, 6, 8))
    w = rng.normal(size=(3, 5, 3, 3))
    d = rng.normal(size=(3, 6, 8))
    dx, dw, db = unet.conv_backward(x, w, d)
    # <conv(x) - b, d> is bilinear in (x, w)
    lin = (unet.conv(x, w, np.zeros(3)) * d).sum()
    assert np.isclose(lin, (dx * x).sum())
    assert np.isclose(lin, (dw * w).sum())
    np.testing.assert_allclose(db, d.sum(axis=(1, 2)))


def test_parameter_count():
    assert unet.n_params() == 443745
    p = unet.init_params(0)
    assert sum(v.size for v in p.values()) == 443745


@pytest.mark.parametrize("val,want", [(1.0, 1.0), (1.0 + 2**-8, 1.0), (1.0 + 3 * 2**-8, 1.0 + 2**-6),
                                      (-(1.0 + 2**-8 + 2**-20), -(1.0 + 2**-7))])
def test_bf16_round_known_values(val, want):
    # bfloat16 keeps 7 mantissa bits: ties go to the even mantissa
    assert float(unet.bf16_round(np.array([val]))[0]) == want


def test_bf16_round_matches_torch_cast():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(size=20000) * 10.0 ** rng.integers(-30, 30, size=20000),
                        [0.0, -0.0, np.inf, -np.inf]]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = unet.bf16_round(x)
    np.testing.assert_array_equal(got, want)
    assert np.isnan(unet.bf16_round(np.array([np.nan]))[0])


def test_gradients_central_differences():
    rng = np.random.default_rng(4)
    p = unet.init_params(5)
    for k in p:
        if k.endswith(".b"):
            p[k] = rng.normal(size=p[k].shape) * 0.1
    x = rng.uniform(size=(3, 16, 16))
    t = rng.uniform(size=(16, 16))
    m = rng.uniform(size=(16, 16)) < 0.8

    def loss(pp, xx):
        y, _ = unet.forward(pp, xx)
        return unet.masked_mse(y, t, m)[0]

    y, c = unet.forward(p, x)
    _, dy = unet.masked_mse(y, t, m)
    g = unet.backward(p, c, dy)
    h = 1e-6
    for k in p:
        idxs = [tuple(rng.integers(0, s) for s in p[k].shape) for _ in range(3)]
        for idx in idxs:
            pp = {kk: vv.copy() for kk, vv in p.items()}
            pp[k][idx] += h
            lp = loss(pp, x)
            pp[k][idx] -= 2 * h
            lm = loss(pp, x)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k][idx]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (k, idx, fd, g[k][idx])
    for _ in range(5):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (loss(p, xp) - loss(p, xm)) / (2 * h)
        assert abs(fd - g["x"][idx]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9


def test_first_adam_step_closed_form():
    # after one step m_hat = g and v_hat = g^2, so the update is lr * g / (|g| + eps)
    p = {"a": np.array([1.0, -2.0, 3.0])}
    g = {"a": np.array([0.5, -4.0, 1e-3])}
    st = {}
    q = unet.adam_step({"a": p["a"].copy()}, g, st, lr=0.01)
    np.testing.assert_allclose(q["a"], p["a"] - 0.01 * g["a"] / (np.abs(g["a"]) + 1e-8), rtol=1e-12)


def test_training_decreases_loss():
    rng = np.random.default_rng(6)
    p = unet.init_params(7)
    xs = [rng.uniform(size=(3, 16, 16)) for _ in range(2)]
    ts = [0.3 + 0.1 * x[0] for x in xs]
    ms = [np.ones((16, 16), bool)] * 2
    st = {}
    l0, g = unet.loss_and_grads(p, xs, ts, ms)
    for _ in range(10):
        p = unet.adam_step(p, g, st, lr=2e-3)
        l, g = unet.loss_and_grads(p, xs, ts, ms)
    assert l < 0.5 * l0


def test_bf16_gradient_storage_option():
    # bf16_grads rounds each layer's masked pre-activation gradient to bf16:
    # the gradients then differ from the FP64 ones by about one 2^-9 rounding
    # (not by zero, not by more); the loss does not change
    rng = np.random.default_rng(8)
    p = unet.init_params(9)
    for k in p:
        if k.endswith(".b"):
            p[k] = rng.normal(size=p[k].shape) * 0.1
    xs = [unet.bf16_round(rng.uniform(size=(3, 16, 16))) for _ in range(2)]
    ts = [rng.uniform(size=(16, 16)) for _ in range(2)]
    ms = [rng.uniform(size=(16, 16)) < 0.8 for _ in range(2)]
    l0, g0 = unet.loss_and_grads(p, xs, ts, ms, bf16_acts=True)
    l1, g1 = unet.loss_and_grads(p, xs, ts, ms, bf16_acts=True, bf16_grads=True)
    assert l0 == l1
    for k in g0:
        rel = np.linalg.norm(g1[k] - g0[k]) / np.linalg.norm(g0[k])
        # the head's own gradients come before any rounding
        if k.startswith("head"):
            assert rel == 0.0, k
        else:
            assert 0.0 < rel < 2.0 ** -7, (k, rel)
    # one rounding of the head's masked gradient, checked elementwise
    y, c = unet.forward(p, xs[0], bf16_acts=True)
    _, dy = unet.masked_mse(y, ts[0], ms[0])
    want = unet.bf16_round(p["head.w"][0, :, 0, 0][:, None, None] * dy[None] * (c["d0"] > 0))
    dd0, _, _ = unet.conv_backward(c["d0"], p["head.w"], dy[None])
    np.testing.assert_array_equal(unet.bf16_round(dd0 * (c["d0"] > 0)), want)


# ---- coarse-scale warm start ------------------------------------------------

def _fine_features(cls, ring, goal):
    """The fine-scale input channels written out from their definition."""
    ny, nx = cls.shape
    yy, xx = np.mgrid[0:ny, 0:nx]
    occ = np.isin(cls, (unet.OBST, unet.WALL)).astype(np.float64)
    gd = np.hypot(xx - goal[0], yy - goal[1]) / (max(nx, ny) * np.sqrt(2.0))
    rt = ring / ring.max()
    return np.stack([occ, gd, rt], -1)


def test_coarse_features_at_factor_one_are_the_fine_features():
    rng = np.random.default_rng(3)
    ny, nx = 16, 24  # multiples of 8: the frame is the grid
    cls = rng.choice([0, 0, 0, 1, 2, 3], size=(ny, nx)).astype(np.uint8)
    ring = rng.integers(0, 9, size=(ny, nx))
    ring[0, 0] = 8
    x, mask = unet.coarse_features(cls, ring, (5, 7), 1)
    assert np.allclose(x, _fine_features(cls, ring, (5, 7)), rtol=0, atol=1e-15)
    assert np.array_equal(mask == unet.FREE, cls == unet.FREE)


def test_coarse_features_counts_and_outside_cells():
    # a 10 x 6 grid at f = 4: the frame is 8 x 8 blocks; block (2, 1) holds
    # fine columns 8..11 (10, 11 outside) and rows 4..7 (6, 7 outside)
    cls = np.zeros((6, 10), np.uint8)
    cls[4, 8] = unet.OBST
    cls[5, 9] = unet.GOAL
    x, mask = unet.coarse_features(cls, None, (0, 0), 4)
    assert x.shape == (8, 8, 3)
    outside = 16 - 4  # 4 cells inside the grid
    assert x[1, 2, 0] == (outside + 1) / 16.0
    assert mask[1, 2] == unet.FREE  # (9, 4) is FREE
    assert x[5, 5, 0] == 1.0 and mask[5, 5] == unet.OBST  # wholly outside
    assert x[0, 0, 0] == 0.0 and np.all(x[..., 2] == 0.0)
    # block centre (1.5, 1.5) for block (0, 0): distance to the goal (0, 0)
    assert np.isclose(x[0, 0, 1], np.hypot(1.5, 1.5) / (10 * np.sqrt(2.0)))


def test_coarse_target_of_a_linear_field_is_its_value_at_block_centres():
    # the mean of a linear function over a full block is its value at the
    # block's centre; blocks without FREE cells read 0
    f, ny, nx = 4, 16, 16
    cls = np.zeros((ny, nx), np.uint8)
    cls[12:, 12:] = unet.OBST
    yy, xx = np.mgrid[0:ny, 0:nx]
    psi = 0.25 + 0.01 * xx - 0.02 * yy
    t = unet.coarse_target(psi, cls, f)
    for Y in range(3):
        for X in range(3):
            cx, cy = X * f + 1.5, Y * f + 1.5
            assert np.isclose(t[Y, X], 0.25 + 0.01 * cx - 0.02 * cy, rtol=0, atol=1e-14)
    assert t[3, 3] == 0.0


def test_upsample_reproduces_linear_fields_and_the_round_trip():
    # bilinear interpolation is exact on linear functions, so a linear field
    # pooled to block centres and interpolated back is the field itself away
    # from the clamped border; fixed cells take their Dirichlet values
    f, ny, nx = 4, 32, 32
    cls = np.zeros((ny, nx), np.uint8)
    cls[0, :] = unet.WALL
    cls[20, 20] = unet.GOAL
    yy, xx = np.mgrid[0:ny, 0:nx]
    psi = 0.2 + 0.005 * xx + 0.01 * yy
    t = unet.coarse_target(psi, np.zeros_like(cls), f)
    back = unet.upsample_field_f(t, cls, f)
    inner = (slice(2, ny - 2), slice(2, nx - 2))
    free = cls[inner] == unet.FREE
    assert np.allclose(back[inner][free], psi[inner][free], rtol=0, atol=1e-13)
    assert np.all(back[0, :] == 0.0) and back[20, 20] == 1.0
    # clamping to [0, 1] and to the frame
    yc = np.full((8, 8), 3.0)
    assert np.all(unet.upsample_field_f(yc, np.zeros((32, 32), np.uint8), 4) == 1.0)
