"""FP64 reference of the learned warm start's encoder-decoder network.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy, float64,
written from the layer definitions below; a matrix product over channels is
the only library step.  It shares no code with the HIP kernels.

The warm start is not in the paper (its only mention of learning is future
work on predicting obstacle motion); the network maps occupancy, goal and
ring-time channels to an initial potential psi0, which the relaxation then
corrects.  Architecture (4 levels, 32 base channels):

    e0 = relu(conv3(x,  3 -> 32))            H
    e1 = relu(conv3(pool(e0), 32 -> 64))     H/2
    e2 = relu(conv3(pool(e1), 64 -> 128))    H/4
    e3 = relu(conv3(pool(e2), 128 -> 128))   H/8
    d2 = relu(conv3(cat(up(e3), e2), 256 -> 64))   H/4
    d1 = relu(conv3(cat(up(d2), e1), 128 -> 32))   H/2
    d0 = relu(conv3(cat(up(d1), e0), 64 -> 32))    H
    y  = conv1(d0, 32 -> 1)                  H

conv3: 3x3 cross-correlation with zero padding 1 and a bias; pool: 2x2
average; up: 2x2 nearest-neighbour copy; cat: channel concatenation.
Activations are [C, H, W] per sample.  With ``bf16_acts`` every stored
activation and the input are rounded to bfloat16 (round to nearest even),
which is the storage precision of the GPU kernels; arithmetic stays FP64.
"""
from __future__ import annotations

import numpy as np

LAYERS = [  # name, cin, cout, k
    ("e0", 3, 32, 3), ("e1", 32, 64, 3), ("e2", 64, 128, 3), ("e3", 128, 128, 3),
    ("d2", 256, 64, 3), ("d1", 128, 32, 3), ("d0", 64, 32, 3), ("head", 32, 1, 1),
]


def bf16_round(a):
    """Round float values to bfloat16 (RNE) from the float32 bit pattern;
    NaN stays NaN.  Returns float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def init_params(seed=0):
    """He-uniform weights, zero biases (FP64 master copy)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, cin, cout, k in LAYERS:
        fan_in = cin * k * k
        lim = np.sqrt(6.0 / fan_in)
        p[name + ".w"] = rng.uniform(-lim, lim, size=(cout, cin, k, k))
        p[name + ".b"] = np.zeros(cout)
    p["head.w"] *= 0.1
    return p


def n_params():
    return sum(cout * cin * k * k + cout for _, cin, cout, k in LAYERS)


# ---- layer definitions -----------------------------------------------------

def conv(x, w, b):
    """out[o, y, x] = b[o] + sum_{c, dy, dx} w[o, c, dy, dx] x[c, y + dy - r, x + dx - r]
    with zero padding r = (k - 1) / 2."""
    C, H, W = x.shape
    O, C2, k, _ = w.shape
    assert C == C2
    r = (k - 1) // 2
    xp = np.zeros((C, H + 2 * r, W + 2 * r))
    xp[:, r:r + H, r:r + W] = x
    out = np.broadcast_to(b[:, None, None], (O, H, W)).copy()
    for dy in range(k):
        for dx in range(k):
            patch = xp[:, dy:dy + H, dx:dx + W].reshape(C, H * W)
            # a contiguous tap matrix lets NumPy hand the product to BLAS
            out += (np.ascontiguousarray(w[:, :, dy, dx]) @ patch).reshape(O, H, W)
    return out


def conv_backward(x, w, dout):
    """Gradients of conv with respect to x, w and b."""
    C, H, W = x.shape
    O, _, k, _ = w.shape
    r = (k - 1) // 2
    xp = np.zeros((C, H + 2 * r, W + 2 * r))
    xp[:, r:r + H, r:r + W] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    g = dout.reshape(O, H * W)
    for dy in range(k):
        for dx in range(k):
            patch = xp[:, dy:dy + H, dx:dx + W].reshape(C, H * W)
            dw[:, :, dy, dx] = g @ patch.T
            wt = np.ascontiguousarray(w[:, :, dy, dx].T)
            dxp[:, dy:dy + H, dx:dx + W] += (wt @ g).reshape(C, H, W)
    db = dout.sum(axis=(1, 2))
    return dxp[:, r:r + H, r:r + W], dw, db


def pool(x):
    C, H, W = x.shape
    return x.reshape(C, H // 2, 2, W // 2, 2).mean(axis=(2, 4))


def pool_backward(d):
    return np.repeat(np.repeat(d, 2, axis=1), 2, axis=2) * 0.25


def up(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up_backward(d):
    C, H, W = d.shape
    return d.reshape(C, H // 2, 2, W // 2, 2).sum(axis=(2, 4))


def relu(x):
    return np.maximum(x, 0.0)


# ---- network -------------------------------------------------------------

def forward(p, x, bf16_acts=False):
    """x: [3, H, W] (H, W divisible by 8).  Returns (y [H, W], cache)."""
    q = bf16_round if bf16_acts else (lambda a: a)
    c = {}
    c["x"] = q(x)
    c["e0"] = q(relu(conv(c["x"], p["e0.w"], p["e0.b"])))
    c["p0"] = q(pool(c["e0"]))
    c["e1"] = q(relu(conv(c["p0"], p["e1.w"], p["e1.b"])))
    c["p1"] = q(pool(c["e1"]))
    c["e2"] = q(relu(conv(c["p1"], p["e2.w"], p["e2.b"])))
    c["p2"] = q(pool(c["e2"]))
    c["e3"] = q(relu(conv(c["p2"], p["e3.w"], p["e3.b"])))
    c["c2"] = np.concatenate([up(c["e3"]), c["e2"]])
    c["d2"] = q(relu(conv(c["c2"], p["d2.w"], p["d2.b"])))
    c["c1"] = np.concatenate([up(c["d2"]), c["e1"]])
    c["d1"] = q(relu(conv(c["c1"], p["d1.w"], p["d1.b"])))
    c["c0"] = np.concatenate([up(c["d1"]), c["e0"]])
    c["d0"] = q(relu(conv(c["c0"], p["d0.w"], p["d0.b"])))
    y = conv(c["d0"], p["head.w"], p["head.b"])[0]
    return y, c


def backward(p, c, dy, bf16_grads=False):
    """Gradients of a scalar loss with d loss / d y = dy, for every parameter
    and for the input x.  With ``bf16_grads`` the gradient with respect to
    each layer's pre-activation (after the ReLU mask) is rounded to bfloat16,
    the storage precision of the GPU's backward pass; the parameter and
    input gradients themselves stay FP64."""
    q = bf16_round if bf16_grads else (lambda a: a)
    g = {}
    dd0, g["head.w"], g["head.b"] = conv_backward(c["d0"], p["head.w"], dy[None])
    dd0 = q(dd0 * (c["d0"] > 0))
    dc0, g["d0.w"], g["d0.b"] = conv_backward(c["c0"], p["d0.w"], dd0)
    n1 = c["d1"].shape[0]
    dd1 = up_backward(dc0[:n1])
    de0 = dc0[n1:].copy()
    dd1 = q(dd1 * (c["d1"] > 0))
    dc1, g["d1.w"], g["d1.b"] = conv_backward(c["c1"], p["d1.w"], dd1)
    n2 = c["d2"].shape[0]
    dd2 = up_backward(dc1[:n2])
    de1 = dc1[n2:].copy()
    dd2 = q(dd2 * (c["d2"] > 0))
    dc2, g["d2.w"], g["d2.b"] = conv_backward(c["c2"], p["d2.w"], dd2)
    n3 = c["e3"].shape[0]
    de3 = up_backward(dc2[:n3])
    de2 = dc2[n3:].copy()
    de3 = q(de3 * (c["e3"] > 0))
    dp2, g["e3.w"], g["e3.b"] = conv_backward(c["p2"], p["e3.w"], de3)
    de2 = q((de2 + pool_backward(dp2)) * (c["e2"] > 0))
    dp1, g["e2.w"], g["e2.b"] = conv_backward(c["p1"], p["e2.w"], de2)
    de1 = q((de1 + pool_backward(dp1)) * (c["e1"] > 0))
    dp0, g["e1.w"], g["e1.b"] = conv_backward(c["p0"], p["e1.w"], de1)
    de0 = q((de0 + pool_backward(dp0)) * (c["e0"] > 0))
    dx, g["e0.w"], g["e0.b"] = conv_backward(c["x"], p["e0.w"], de0)
    g["x"] = dx
    return g


def masked_mse(y, target, mask):
    """Mean over masked cells of (y - target)^2 and its gradient."""
    n = max(1, int(mask.sum()))
    diff = np.where(mask, y - target, 0.0)
    return float((diff * diff).sum() / n), 2.0 * diff / n


def loss_and_grads(p, xs, targets, masks, bf16_acts=False, bf16_grads=False):
    """Batch loss (mean of per-sample losses) and summed parameter gradients
    (``bf16_acts``, ``bf16_grads``: see ``forward`` and ``backward``)."""
    total = 0.0
    grads = {k: np.zeros_like(v) for k, v in p.items()}
    B = len(xs)
    for x, t, m in zip(xs, targets, masks):
        y, c = forward(p, x, bf16_acts)
        l, dy = masked_mse(y, t, m)
        total += l / B
        g = backward(p, c, dy / B, bf16_grads)
        for k in grads:
            grads[k] += g[k]
    return total, grads


def adam_step(p, g, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) on FP64 masters; state holds m, v, t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m." + k, np.zeros_like(p[k]))
        v = state.setdefault("v." + k, np.zeros_like(p[k]))
        m[:] = b1 * m + (1 - b1) * g[k]
        v[:] = b2 * v + (1 - b2) * g[k] * g[k]
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p


# ---------------------------------------------------------------------------
# Coarse-scale warm start: the grid seen at 1/f of its resolution, and the
# network's coarse output interpolated back to the grid.  Plain loops over
# blocks and cells (small grids only), float64.
# ---------------------------------------------------------------------------

FREE, OBST, WALL, GOAL, FIXED = 0, 1, 2, 3, 4


def coarse_frame(nx, ny, f):
    """(Hc, Wc): the coarse sides ceil(n / f) rounded up to multiples of 8
    (at least 8)."""
    hc = max(8, (-(-ny // f) + 7) // 8 * 8)
    wc = max(8, (-(-nx // f) + 7) // 8 * 8)
    return hc, wc


def coarse_features(cls, ring, goal, f):
    """Input channels [Hc, Wc, 3] and training mask [Hc, Wc] of the grid
    `cls` [ny, nx] seen at 1/f.  Block (X, Y) covers fine cells
    [fX, fX + f) x [fY, fY + f); cells outside the grid count as walls.
    Occupancy = share of OBST / WALL / outside cells in the block; goal
    distance of the block's centre (fX + (f - 1)/2, fY + (f - 1)/2) over
    max(nx, ny) sqrt 2; ring of the fine cell (fX + f // 2, fY + f // 2)
    clamped into the grid, over the largest ring (0 without a ring map, and
    for blocks wholly outside the grid).  Mask: FREE where the block holds a
    FREE cell, else OBST."""
    ny, nx = cls.shape
    hc, wc = coarse_frame(nx, ny, f)
    x = np.zeros((hc, wc, 3))
    mask = np.full((hc, wc), OBST, np.uint8)
    diag = max(nx, ny) * np.sqrt(2.0)
    jmax = float(ring.max()) if ring is not None and ring.size else 0.0
    gx, gy = goal
    for Y in range(hc):
        for X in range(wc):
            blocked = 0
            free = 0
            for y in range(Y * f, Y * f + f):
                for xx in range(X * f, X * f + f):
                    if xx >= nx or y >= ny:
                        blocked += 1
                        continue
                    c = cls[y, xx]
                    blocked += c in (OBST, WALL)
                    free += c == FREE
            x[Y, X, 0] = blocked / (f * f)
            cx, cy = X * f + (f - 1) / 2.0, Y * f + (f - 1) / 2.0
            x[Y, X, 1] = np.hypot(cx - gx, cy - gy) / diag
            if ring is not None and jmax > 0 and X * f < nx and Y * f < ny:
                rx, ry = min(X * f + f // 2, nx - 1), min(Y * f + f // 2, ny - 1)
                x[Y, X, 2] = ring[ry, rx] / jmax
            if free:
                mask[Y, X] = FREE
    return x, mask


def coarse_target(psi, cls, f):
    """[Hc, Wc]: the mean of psi over the FREE cells of each block (0 when the
    block has none)."""
    ny, nx = cls.shape
    hc, wc = coarse_frame(nx, ny, f)
    out = np.zeros((hc, wc))
    for Y in range(hc):
        for X in range(wc):
            blk_c = cls[Y * f:Y * f + f, X * f:X * f + f]
            blk_p = psi[Y * f:Y * f + f, X * f:X * f + f]
            sel = blk_c == FREE
            if sel.any():
                out[Y, X] = blk_p[sel].mean()
    return out


def upsample_field_f(yc, cls, f, psi_in=None):
    """FREE cell (x, y) takes the bilinear interpolation of yc at
    ((x + 1/2)/f - 1/2, (y + 1/2)/f - 1/2), each coordinate clamped to the
    frame, the value then clamped to [0, 1]; OBST and WALL 0, GOAL 1, FIXED
    keep psi_in's value."""
    ny, nx = cls.shape
    hc, wc = yc.shape
    out = np.zeros((ny, nx)) if psi_in is None else np.array(psi_in, dtype=np.float64)
    for y in range(ny):
        for x in range(nx):
            c = cls[y, x]
            if c == FREE:
                u = min(max((x + 0.5) / f - 0.5, 0.0), wc - 1.0)
                v = min(max((y + 0.5) / f - 0.5, 0.0), hc - 1.0)
                x0, y0 = int(np.floor(u)), int(np.floor(v))
                x1, y1 = min(x0 + 1, wc - 1), min(y0 + 1, hc - 1)
                a, b = u - x0, v - y0
                top = (1 - a) * yc[y0, x0] + a * yc[y0, x1]
                bot = (1 - a) * yc[y1, x0] + a * yc[y1, x1]
                out[y, x] = min(max((1 - b) * top + b * bot, 0.0), 1.0)
            elif c in (OBST, WALL):
                out[y, x] = 0.0
            elif c == GOAL:
                out[y, x] = 1.0
    return out
