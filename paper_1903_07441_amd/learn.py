"""Train and evaluate the learned warm start on the GPU.

The training set is made by the library itself: seeded 256 x 256 scenarios
are rasterised (twg_rasterize), their fields relaxed (hpf_relax_batched), and
the network input channels computed (twg_unet_features); the network is then
trained with twg_unet_loss_grad / twg_unet_adam_step (masked MSE over FREE
cells, Adam).  Evaluation relaxes held-out scenarios to residual 1e-6 from the
plain initial fields and from the network's field and reports sweeps and time.

    python -m paper_1903_07441_amd.learn --train 4096 --eval 64 --epochs 4 \\
        --out paper_1903_07441_amd/weights/unet_learn256.npz

With --coarse F the network is trained at 1/F of full-size replanning maps
(2048 x 2048, 500 moving discs): inputs and targets are the maps' block-level
views (twg_unet_features_coarse, twg_unet_coarse_target of fields the library
relaxed), and the warm start interpolates the coarse output back
(twg_unet_warm_start_coarse):

    python -m paper_1903_07441_amd.learn --coarse 8 --train 2048 --eval 8 \\
        --epochs 10 --out paper_1903_07441_amd/weights/unet_coarse8_replan2048.npz

Weights are stored as an .npz with one FP32 array ``params`` (the C ABI's
parameter order) and a text array ``meta`` (JSON); load with
``np.load(path)`` (no pickles).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import scenarios, twg

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "unet_learn256.npz")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def he_init(seed=0):
    """He-uniform conv weights, zero biases, head scaled by 0.1 (parameter
    order of the C ABI)."""
    rng = np.random.default_rng(seed)
    spec = [(3, 32, 3), (32, 64, 3), (64, 128, 3), (128, 128, 3), (256, 64, 3), (128, 32, 3), (64, 32, 3),
            (32, 1, 1)]
    parts = []
    for i, (cin, cout, k) in enumerate(spec):
        lim = math.sqrt(6.0 / (cin * k * k))
        w = rng.uniform(-lim, lim, size=cout * cin * k * k)
        if i == len(spec) - 1:
            w *= 0.1
        parts += [w, np.zeros(cout)]
    return np.concatenate(parts).astype(np.float32)


def save_weights(path, params, meta):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, params=np.asarray(params, dtype=np.float32), meta=np.array(json.dumps(meta)))


def load_weights(path=DEFAULT_WEIGHTS):
    with np.load(path, allow_pickle=False) as z:
        return z["params"].astype(np.float32), json.loads(str(z["meta"]))


def make_dataset(ctx, net, first, n, name="learn256", side=None):
    """Rasterise scenarios first .. first + n - 1 of recipe `name`, compute the
    network inputs, and keep class map, ring map and goal of each."""
    dev = torch.device("cuda", ctx.device)
    sc0 = scenarios.scenario(name, first, side=side)
    H, W = sc0["ny"], sc0["nx"]
    x = torch.empty((n, H, W, 3), dtype=torch.float32, device=dev)
    cls = torch.empty((n, H, W), dtype=torch.uint8, device=dev)
    ring = torch.empty((n, H, W), dtype=torch.uint16, device=dev)
    goals = []
    for k in range(n):
        sc = scenarios.scenario(name, first + k, side=side)
        pos = torch.as_tensor(sc["pos"], dtype=torch.float64).reshape(-1, 2).to(dev)
        vel = torch.as_tensor(sc["vel"], dtype=torch.float64).reshape(-1, 2).to(dev)
        rad = torch.as_tensor(sc["rad"], dtype=torch.float64).to(dev)
        ctx.rasterize(W, H, sc["robot"], sc["goal"], pos, vel, rad, W=sc["W"], robot_speed=sc["vr"],
                      cls=cls[k], ring=ring[k])
        net.features(cls[k], ring[k], sc["goal"], H=H, W=W, out=x[k])
        goals.append((int(sc["goal"][0]), int(sc["goal"][1])))
        if (k + 1) % 512 == 0 or k + 1 == n:
            log(f"  rasterised {k + 1}/{n}")
    return dict(x=x, cls=cls, ring=ring, goals=goals, H=H, W=W, first=first, name=name)


def relax_targets(ctx, data, tol=3e-7, chunk=256, max_sweeps=20000):
    """Converged FP32 fields of every scenario (batched relaxation; the
    tolerance sits just above FP32's rounding floor next to the goal)."""
    n, H, W = data["cls"].shape
    psi = torch.empty((n, H, W), dtype=torch.float32, device=data["cls"].device)
    cls_flat = data["cls"].view(-1)
    psi_flat = psi.view(-1)
    sweeps = []
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        descs = [(W, H, W, (k - s) * H * W) for k in range(s, e)]
        st = ctx.relax_batched(cls_flat[s * H * W:e * H * W], psi_flat[s * H * W:e * H * W], descs, tol=tol,
                               max_sweeps=max_sweeps)
        sweeps += [d["sweeps"] for d in st]
        log(f"  relaxed {e}/{n} (median sweeps {int(np.median(sweeps))}, "
            f"{sum(d['status'] == twg.OK for d in st)}/{len(st)} at tol)")
    data["target"] = psi
    return psi


def make_coarse_dataset(ctx, net, first, n, factor, name="replan2048", tol=3e-7):
    """Scenarios first .. first + n - 1 of recipe `name` seen at 1/factor:
    each is rasterised and relaxed at full resolution by the library (FP32,
    from psi = 0, to residual `tol`), and its coarse inputs, coarse training
    mask and coarse target (the relaxed field's mean over each block's FREE
    cells) are kept.  Returns dict(x, cls, target, H, W, factor, ...)."""
    dev = torch.device("cuda", ctx.device)
    sc0 = scenarios.scenario(name, first)
    ny, nx = sc0["ny"], sc0["nx"]
    Hc, Wc = twg.UNet.coarse_frame(nx, ny, factor)
    x = torch.empty((n, Hc, Wc, 3), dtype=torch.float32, device=dev)
    ccls = torch.empty((n, Hc, Wc), dtype=torch.uint8, device=dev)
    target = torch.empty((n, Hc, Wc), dtype=torch.float32, device=dev)
    cls = torch.empty((ny, nx), dtype=torch.uint8, device=dev)
    ring = torch.empty((ny, nx), dtype=torch.uint16, device=dev)
    psi = torch.empty((ny, nx), dtype=torch.float32, device=dev)
    sweeps = []
    for k in range(n):
        sc = scenarios.scenario(name, first + k)
        pos = torch.as_tensor(sc["pos"], dtype=torch.float64).reshape(-1, 2).to(dev)
        vel = torch.as_tensor(sc["vel"], dtype=torch.float64).reshape(-1, 2).to(dev)
        rad = torch.as_tensor(sc["rad"], dtype=torch.float64).to(dev)
        ctx.rasterize(nx, ny, sc["robot"], sc["goal"], pos, vel, rad, W=sc["W"], robot_speed=sc["vr"],
                      cls=cls, ring=ring)
        st = ctx.relax(cls, psi, None, tol=tol, init=twg.INIT_ZERO)
        sweeps.append(st["sweeps"])
        net.features_coarse(cls, ring, sc["goal"], factor, x=x[k], ccls=ccls[k])
        net.coarse_target(cls, psi, factor, out=target[k])
        if (k + 1) % 256 == 0 or k + 1 == n:
            log(f"  coarse data {k + 1}/{n} (median sweeps {int(np.median(sweeps))})")
    return dict(x=x, cls=ccls, target=target, H=Hc, W=Wc, factor=factor, first=first, name=name)


def evaluate_coarse(ctx, net, first, n, factor, name="replan2048", omegas=(0.0, 1.95, 1.98), tol=1e-6):
    """Held-out scenarios at full resolution: time (and sweeps) to residual
    `tol` from the plain start psi = 0 and from the coarse network's field
    (its forward pass and interpolation counted), each with its best factor
    of `omegas` (0 = tuned), median over the scenarios."""
    dev = torch.device("cuda", ctx.device)
    sc0 = scenarios.scenario(name, first)
    ny, nx = sc0["ny"], sc0["nx"]
    cls = torch.empty((ny, nx), dtype=torch.uint8, device=dev)
    ring = torch.empty((ny, nx), dtype=torch.uint16, device=dev)
    psi = torch.empty((ny, nx), dtype=torch.float32, device=dev)
    ev0, ev1, ev2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    rows = {"zero": [], "coarse_net": []}
    net_ms = []
    for k in range(n):
        sc = scenarios.scenario(name, first + k)
        pos = torch.as_tensor(sc["pos"], dtype=torch.float64).reshape(-1, 2).to(dev)
        vel = torch.as_tensor(sc["vel"], dtype=torch.float64).reshape(-1, 2).to(dev)
        rad = torch.as_tensor(sc["rad"], dtype=torch.float64).to(dev)
        ctx.rasterize(nx, ny, sc["robot"], sc["goal"], pos, vel, rad, W=sc["W"], robot_speed=sc["vr"],
                      cls=cls, ring=ring)
        for kind in rows:
            best = None
            for w in omegas:
                torch.cuda.synchronize()
                ev0.record()
                if kind == "coarse_net":
                    net.warm_start_coarse(cls, ring, sc["goal"], psi, factor)
                ev1.record()
                st = ctx.relax(cls, psi, None, tol=tol, init=twg.INIT_KEEP if kind == "coarse_net" else twg.INIT_ZERO,
                               omega=w)
                ev2.record()
                torch.cuda.synchronize()
                r = (ev0.elapsed_time(ev2), st["sweeps"], w)
                if kind == "coarse_net":
                    net_ms.append(ev0.elapsed_time(ev1))
                if best is None or r[0] < best[0]:
                    best = r
            rows[kind].append(best)
    out = {"scenarios": [first, first + n], "factor": factor, "net_median_ms": float(np.median(net_ms))}
    for kind, v in rows.items():
        a = np.array([(t, s) for t, s, _ in v])
        out[kind] = {"median_ms": float(np.median(a[:, 0])), "median_sweeps": float(np.median(a[:, 1])),
                     "omegas": [w for _, _, w in v]}
    out["time_ratio_zero_over_net"] = out["zero"]["median_ms"] / out["coarse_net"]["median_ms"]
    return out


def train(net, data, epochs=4, batch=16, lr=1e-3, lr_min=2e-5, log_every=100):
    """Adam over contiguous batches of the (already random) scenarios with a
    cosine learning-rate decay.  Returns the loss history (per logged step)."""
    n = data["x"].shape[0]
    steps_per_epoch = n // batch
    total = epochs * steps_per_epoch
    loss = torch.empty(1, dtype=torch.float32, device=data["x"].device)
    hist = []
    t0 = time.perf_counter()
    step = 0
    for ep in range(epochs):
        for b in range(steps_per_epoch):
            s, e = b * batch, (b + 1) * batch
            a = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * step / max(1, total)))
            net.loss_grad(data["x"][s:e], data["target"][s:e], data["cls"][s:e], loss)
            net.adam_step(a)
            step += 1
            if step % log_every == 0 or step == total:
                v = float(loss.item())
                hist.append((step, v))
                log(f"  step {step}/{total} epoch {ep + 1} loss {v:.3e} lr {a:.2e} "
                    f"({(time.perf_counter() - t0) / step * 1e3:.2f} ms/step)")
    torch.cuda.synchronize()
    return hist, (time.perf_counter() - t0) / max(1, total)


OMEGAS = (1.6, 1.8, 1.9, 1.95, 0.0)  # 0 = the open-rectangle optimum of the grid


def evaluate(ctx, net, data, tol=1e-6, omegas=OMEGAS):
    """Relax every scenario of `data` to `tol` from the plain initial fields
    (half, zero, linear ramp) and from the network's field, each with every SOR factor of
    `omegas`; per-mode median sweeps and times (the learned time includes
    features and network).  Both paths are credited with their best factor:
    obstacles shrink the domain, so the best factor is below the open-grid
    optimum, and a warm start's error is mostly short-wavelength, which
    smaller factors damp fastest."""
    n, H, W = data["cls"].shape
    dev = data["cls"].device
    psi = torch.empty((H, W), dtype=torch.float32, device=dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    kinds = ("half", "zero", "linear", "learned")
    out = {(kd, w): [] for kd in kinds for w in omegas}
    net_ms, net_err = [], []
    for k in range(n):
        cls, ring, goal = data["cls"][k], data["ring"][k], data["goals"][k]
        ev0.record()
        net.warm_start(cls, ring, goal, psi)
        ev1.record()
        torch.cuda.synchronize()
        net_ms.append(ev0.elapsed_time(ev1))
        if "target" in data:
            free = cls == twg.FREE
            net_err.append(float((psi - data["target"][k]).abs()[free].max().item()))
        for w in omegas:
            for kd, init in (("half", twg.INIT_HALF), ("zero", twg.INIT_ZERO), ("linear", twg.INIT_LINEAR),
                             ("learned", twg.INIT_KEEP)):
                ev0.record()
                if kd == "learned":
                    net.warm_start(cls, ring, goal, psi)
                st = ctx.relax(cls, psi, None, tol=tol, init=init, omega=w, goal=goal)
                ev1.record()
                torch.cuda.synchronize()
                out[(kd, w)].append((st["sweeps"], ev0.elapsed_time(ev1), st["residual"]))
    summ = {"omegas": list(omegas)}
    for kd in kinds:
        rows = {}
        for w in omegas:
            a = np.array(out[(kd, w)])
            rows[f"{w:g}"] = {"median_sweeps": float(np.median(a[:, 0])), "median_ms": float(np.median(a[:, 1])),
                             "max_residual": float(np.max(a[:, 2]))}
        best = min(rows, key=lambda r: rows[r]["median_ms"])
        summ[kd] = {"by_omega": rows, "best_omega": float(best), **rows[best]}
    summ["net_median_ms"] = float(np.median(net_ms))
    if net_err:
        summ["net_median_max_err"] = float(np.median(net_err))
    plain_kd = min(("half", "zero", "linear"), key=lambda kd: summ[kd]["median_ms"])
    plain = summ[plain_kd]
    summ["plain_best"] = {"init": plain_kd, "omega": plain["best_omega"],
                          "median_ms": plain["median_ms"], "median_sweeps": plain["median_sweeps"]}
    summ["time_ratio_plain_over_learned"] = plain["median_ms"] / max(1e-9, summ["learned"]["median_ms"])
    summ["sweep_ratio_plain_over_learned"] = plain["median_sweeps"] / max(1.0, summ["learned"]["median_sweeps"])
    return summ


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=4096)
    ap.add_argument("--eval", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--init", default=None, help="start from these weights instead of He init")
    ap.add_argument("--coarse", type=int, default=0,
                    help="train the coarse-scale warm start at 1/COARSE of the replan2048 grids instead")
    args = ap.parse_args()
    if args.coarse:
        return main_coarse(args)

    torch.cuda.set_device(0)
    ctx = twg.Context(0)
    net = twg.UNet(ctx)
    params = load_weights(args.init)[0] if args.init else he_init(args.seed)
    net.set_params(torch.as_tensor(params))
    t0 = time.perf_counter()
    log(f"dataset: {args.train} training + {args.eval} held-out 256x256 scenarios")
    tr = make_dataset(ctx, net, 0, args.train)
    relax_targets(ctx, tr)
    ev = make_dataset(ctx, net, 100000, args.eval)
    relax_targets(ctx, ev)
    t_data = time.perf_counter() - t0
    log(f"dataset ready in {t_data:.1f} s")
    before = evaluate(ctx, net, ev) if args.init is None else None
    hist, ms_step = train(net, tr, epochs=args.epochs, batch=args.batch, lr=args.lr)
    after = evaluate(ctx, net, ev)
    meta = {"train_scenarios": [0, args.train], "eval_scenarios": [100000, 100000 + args.eval],
            "recipe": "learn256", "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
            "ms_per_step": ms_step, "loss_history": hist, "eval": after}
    save_weights(args.out, net.get_params().cpu().numpy(), meta)
    print(json.dumps({"data_s": round(t_data, 1), "ms_per_train_step": round(ms_step * 1e3, 3),
                      "final_loss": hist[-1][1] if hist else None, "eval_untrained": before,
                      "eval_trained": after}), flush=True)
    net.close()
    ctx.close()


def main_coarse(args):
    """Coarse-scale training on full-size replanning maps (2048 x 2048, 500
    moving discs): the network learns the field's mean over factor x factor
    blocks from block-level inputs; the warm start interpolates it back."""
    torch.cuda.set_device(0)
    ctx = twg.Context(0)
    net = twg.UNet(ctx)
    params = load_weights(args.init)[0] if args.init else he_init(args.seed)
    net.set_params(torch.as_tensor(params))
    f = args.coarse
    t0 = time.perf_counter()
    # the relaxation's tiling and factors for this size, tuned on one map
    sc = scenarios.scenario("replan2048", 2)
    dev = torch.device("cuda", 0)
    cls, _ = ctx.rasterize(sc["nx"], sc["ny"], sc["robot"], sc["goal"],
                           torch.as_tensor(sc["pos"], dtype=torch.float64, device=dev).contiguous(),
                           torch.as_tensor(sc["vel"], dtype=torch.float64, device=dev).contiguous(),
                           torch.as_tensor(sc["rad"], dtype=torch.float64, device=dev).contiguous(),
                           W=sc["W"], robot_speed=sc["vr"], want_ring=False)
    ctx.autotune(cls)
    log(f"coarse dataset: {args.train} training scenarios of replan2048 at 1/{f}")
    tr = make_coarse_dataset(ctx, net, 1000, args.train, f)
    t_data = time.perf_counter() - t0
    before = evaluate_coarse(ctx, net, 100, args.eval, f) if args.init is None else None
    hist, ms_step = train(net, tr, epochs=args.epochs, batch=args.batch, lr=args.lr)
    after = evaluate_coarse(ctx, net, 100, args.eval, f)
    meta = {"train_scenarios": ["replan2048", 1000, 1000 + args.train], "eval_scenarios": ["replan2048", 100,
                                                                                          100 + args.eval],
            "recipe": "replan2048", "coarse_factor": f, "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
            "ms_per_step": ms_step, "loss_history": hist, "eval": after}
    save_weights(args.out, net.get_params().cpu().numpy(), meta)
    print(json.dumps({"data_s": round(t_data, 1), "ms_per_train_step": round(ms_step * 1e3, 3),
                      "final_loss": hist[-1][1] if hist else None, "eval_untrained": before,
                      "eval_trained": after}), flush=True)
    net.close()
    ctx.close()


if __name__ == "__main__":
    main()
