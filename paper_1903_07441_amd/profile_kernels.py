"""Drive the relaxation kernel alone, for profilers.

Rasterises a 2048 x 2048 replanning scenario, tunes the tiling, then runs
`--passes` passes of the streamed SOR kernel, followed by one device copy of
`--copy-mib` MiB (a kernel of known traffic: it reads and writes exactly that
many bytes) so that hardware byte counters can be calibrated against it.

    rocprofv3 --kernel-trace --stats -d OUT -- python -m paper_1903_07441_amd.profile_kernels
    rocprofv3 --pmc FETCH_SIZE -d OUT -- python -m paper_1903_07441_amd.profile_kernels
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
    tune = ctx.autotune(cls)
    psi = torch.full((ny, nx), 0.5, dtype=torch.float32, device=dev)
    ctx.sweeps(cls, psi, tune["omega"], 2 * tune["S"] * args.passes, sweeps_per_pass=tune["S"])
    n = args.copy_mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"profiled {2 * args.passes} passes of S={tune['S']} RH={tune['RH']} on {nx}x{ny}; "
          f"copy of {args.copy_mib} MiB", flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
