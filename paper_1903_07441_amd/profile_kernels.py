"""Drive the relaxation kernel (default) or the network kernels (--net)
alone, for profilers.

Rasterises a 2048 x 2048 replanning scenario, tunes the tiling, then runs
`--passes` passes of the streamed SOR kernel (with --rhs as many passes with
a source term, with --fp64 as many FP64 passes), followed by one device copy of
`--copy-mib` MiB (a kernel of known traffic: it reads and writes exactly that
many bytes) so that hardware byte counters can be calibrated against it.

    rocprofv3 --kernel-trace --stats -d OUT -- python -m paper_1903_07441_amd.profile_kernels
    rocprofv3 --pmc FETCH_SIZE -d OUT -- python -m paper_1903_07441_amd.profile_kernels

With --net: `--passes` warm starts (features + forward + head) of the
network on the rasterised grid, then `--passes` training steps (forward,
backward, Adam) on a batch of 16 random 256 x 256 inputs.

With --step: after autotuning, `--passes` whole replanning steps as bench.py
times them (rasterise, FP32 relaxation from psi = 0 to residual 1e-6, FP64
defect correction to a certified 5e-7, descent from the robot).
"""
from __future__ import annotations

import argparse
import sys

import torch

from . import scenarios, twg


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--scenario", default="replan2048")
    ap.add_argument("--index", type=int, default=1)
    ap.add_argument("--passes", type=int, default=50)
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--net", action="store_true", help="profile the network kernels instead")
    ap.add_argument("--step", action="store_true", help="profile whole replanning steps instead")
    ap.add_argument("--S", type=int, default=0, help="sweeps per tile load (with --RH: skip the autotuner)")
    ap.add_argument("--RH", type=int, default=0, help="output rows per tile")
    ap.add_argument("--fp64", action="store_true", help="also run the FP64 sweeps")
    ap.add_argument("--rhs", action="store_true",
                    help="also run FP32 sweeps with a source term (the defect-correction solves' kernel)")
    ap.add_argument("--S64", type=int, default=0, help="FP64 sweeps per tile load (with --RH64)")
    ap.add_argument("--RH64", type=int, default=0, help="FP64 output rows per tile")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    sc = scenarios.scenario(args.scenario, args.index)
    nx, ny = sc["nx"], sc["ny"]
    ctx = twg.Context(0)
    pos = torch.as_tensor(sc["pos"], dtype=torch.float64, device=dev).contiguous()
    vel = torch.as_tensor(sc["vel"], dtype=torch.float64, device=dev).contiguous()
    rad = torch.as_tensor(sc["rad"], dtype=torch.float64, device=dev).contiguous()
    cls, _ = ctx.rasterize(nx, ny, sc["robot"], sc["goal"], pos, vel, rad, W=sc["W"],
                           robot_speed=sc["vr"], want_ring=False)
    if args.net:
        import numpy as np
        from . import learn
        net = twg.UNet(ctx, torch.as_tensor(learn.he_init(0)))
        ring = torch.empty((ny, nx), dtype=torch.uint16, device=dev)
        ctx.rasterize(nx, ny, sc["robot"], sc["goal"], pos, vel, rad, W=sc["W"], robot_speed=sc["vr"],
                      cls=cls, ring=ring)
        psi = torch.empty((ny, nx), dtype=torch.float32, device=dev)
        for _ in range(args.passes):
            net.warm_start(cls, ring, sc["goal"], psi)
        rng = np.random.default_rng(0)
        B, H = 16, 256
        x = torch.as_tensor(rng.uniform(0, 1, (B, H, H, 3)), dtype=torch.float32, device=dev)
        t = torch.as_tensor(rng.uniform(0, 1, (B, H, H)), dtype=torch.float32, device=dev)
        c = torch.zeros((B, H, H), dtype=torch.uint8, device=dev)
        for _ in range(args.passes):
            net.train_step(x, t, c, 1e-4)
        torch.cuda.synchronize()
        print(f"profiled {args.passes} warm starts on {nx}x{ny} and {args.passes} training steps "
              f"(batch {B}, {H}x{H})", flush=True)
        net.close()
        ctx.close()
        return 0
    if args.step:
        from . import replan
        ctx.autotune(cls)
        pl = replan.Planner(ctx, sc)
        robot = [int(sc["robot"][0]), int(sc["robot"][1])]
        for _ in range(args.passes):
            pl.rasterize(robot, pos, vel)
            pl.solve(robot)
        torch.cuda.synchronize()
        info = pl.info
        print(f"profiled {args.passes} replanning steps on {nx}x{ny} (each opens with k_raster_base; the "
              f"autotuner before them rasterises nothing); last descent {info.tolist()}", flush=True)
        ctx.close()
        return 0
    if args.S and args.RH:
        ctx.set_tiling(nx, ny, args.S, args.RH, S64=args.S64, RH64=args.RH64)
        tune = {"S": args.S, "RH": args.RH, "omega": 1.99, "S64": args.S64 or 4}
    else:
        tune = ctx.autotune(cls)
    psi = torch.full((ny, nx), 0.5, dtype=torch.float32, device=dev)
    ctx.sweeps(cls, psi, tune["omega"], 2 * tune["S"] * args.passes, sweeps_per_pass=tune["S"])
    if args.rhs:
        src = torch.zeros_like(psi)
        ctx.sweeps(cls, psi, tune["omega"], 2 * tune["S"] * args.passes, sweeps_per_pass=tune["S"], f=src)
    if args.fp64:
        psi64 = torch.full((ny, nx), 0.5, dtype=torch.float64, device=dev)
        s64 = int(tune.get("S64") or tune["S"])
        ctx.sweeps64(cls, psi64, tune["omega"], 2 * s64 * args.passes, sweeps_per_pass=s64)
    n = args.copy_mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"profiled {2 * args.passes} passes of S={tune['S']} RH={tune['RH']} on {nx}x{ny}"
          + (" and as many with a source term" if args.rhs else "")
          + (f" and as many FP64 passes (S={tune['S64']})" if args.fp64 else "")
          + f"; copy of {args.copy_mib} MiB", flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
