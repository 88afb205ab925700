"""What the trained warm-start network gains over the method without it.

The committed weights (paper_1903_07441_amd/weights/unet_learn256.npz, trained
on the GPU on relaxed 256 x 256 fields) are evaluated on held-out scenarios
of the same recipe.  Every start is relaxed with the same SOR factor to the
same residual; the relaxation always has the last word, so every field meets
the tolerance.  The trained network must need fewer sweeps than the paper's
initial field (free cells at 0.5) and than the same network untrained.  The
all-zero field (psi = 0, phi = 1) is reported too: it is a strong plain start
on these maps, and the network does not beat it by much.
"""
import os

import numpy as np
import pytest
import torch

from conftest import scenario_tensors
from paper_1903_07441_amd import learn, scenarios, twg

pytestmark = pytest.mark.gpu

WEIGHTS = learn.DEFAULT_WEIGHTS


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained weights")
def test_trained_network_gain(ctx):
    params, meta = learn.load_weights(WEIGHTS)
    trained = twg.UNet(ctx, torch.as_tensor(params))
    untrained = twg.UNet(ctx, torch.as_tensor(learn.he_init(0)))
    omega, tol = 1.95, 1e-6
    sweeps = {"half": [], "zero": [], "trained": [], "untrained": []}
    for i in range(16):
        sc = scenarios.scenario("learn256", 200000 + i)
        pos, vel, rad = scenario_tensors(sc)
        cls, ring = ctx.rasterize(sc["nx"], sc["ny"], sc["robot"], sc["goal"], pos, vel, rad, W=sc["W"],
                                  robot_speed=sc["vr"])
        psi = torch.empty((sc["ny"], sc["nx"]), dtype=torch.float32, device="cuda")
        for name, init in (("half", twg.INIT_HALF), ("zero", twg.INIT_ZERO)):
            st = ctx.relax(cls, psi, None, tol=tol, init=init, omega=omega)
            assert st["status"] == twg.OK and st["residual"] <= tol
            sweeps[name].append(st["sweeps"])
        for name, net in (("trained", trained), ("untrained", untrained)):
            net.warm_start(cls, ring, sc["goal"], psi)
            st = ctx.relax(cls, psi, None, tol=tol, init=twg.INIT_KEEP, omega=omega)
            assert st["status"] == twg.OK and st["residual"] <= tol
            sweeps[name].append(st["sweeps"])
    med = {k: float(np.median(v)) for k, v in sweeps.items()}
    print(f"median sweeps to residual {tol} at omega {omega}: {med}", flush=True)
    assert med["trained"] < med["half"]
    assert med["trained"] < med["untrained"]
    trained.close()
    untrained.close()
