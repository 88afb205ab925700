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


COARSE_WEIGHTS = os.path.join(os.path.dirname(WEIGHTS), "unet_coarse8_replan2048.npz")


@pytest.mark.skipif(not os.path.exists(COARSE_WEIGHTS), reason="no trained coarse weights")
def test_trained_coarse_network_gain(ctx):
    """The coarse-scale network (trained at 1/8 of full-size replanning
    maps) on held-out 2048 x 2048 maps: from its interpolated field the
    relaxation reaches residual 1e-6 in fewer sweeps than from psi = 0, the
    best plain start, each with its best factor of a fixed family; the same
    network untrained does not."""
    params, meta = learn.load_weights(COARSE_WEIGHTS)
    assert meta["coarse_factor"] == 8
    trained = twg.UNet(ctx, torch.as_tensor(params))
    untrained = twg.UNet(ctx, torch.as_tensor(learn.he_init(0)))
    omegas, tol = (1.95, 1.98, 1.99), 1e-6
    best = {"zero": [], "trained": [], "untrained": []}
    for i in range(3):
        sc = scenarios.scenario("replan2048", 100 + i)
        pos, vel, rad = scenario_tensors(sc)
        cls, ring = ctx.rasterize(sc["nx"], sc["ny"], sc["robot"], sc["goal"], pos, vel, rad, W=sc["W"],
                                  robot_speed=sc["vr"])
        psi = torch.empty((sc["ny"], sc["nx"]), dtype=torch.float32, device="cuda")
        for name, net in (("zero", None), ("trained", trained), ("untrained", untrained)):
            counts = []
            for w in omegas:
                if net is None:
                    st = ctx.relax(cls, psi, None, tol=tol, init=twg.INIT_ZERO, omega=w)
                else:
                    net.warm_start_coarse(cls, ring, sc["goal"], psi, 8)
                    st = ctx.relax(cls, psi, None, tol=tol, init=twg.INIT_KEEP, omega=w)
                assert st["status"] == twg.OK and st["residual"] <= tol
                counts.append(st["sweeps"])
            best[name].append(min(counts))
    med = {k: float(np.median(v)) for k, v in best.items()}
    print(f"held-out 2048x2048, best sweeps to residual {tol}: {med}", flush=True)
    assert med["trained"] < med["zero"]
    assert med["trained"] < med["untrained"]
    trained.close()
    untrained.close()
