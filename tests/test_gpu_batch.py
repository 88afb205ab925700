"""GPU parity of the batched relaxation: every grid of an uneven batch meets the
tolerance (residual recomputed by the oracle) and equals, bit for bit, the same
number of sweeps run on that grid alone."""
import numpy as np
import pytest
import torch

from paper_1903_07441_amd import scenarios

pytestmark = pytest.mark.gpu


def pack(classes, pad=0):
    descs, off = [], 0
    for c in classes:
        ny, nx = c.shape
        pitch = nx + pad
        descs.append((nx, ny, pitch, off))
        off += pitch * ny + 64
    flat_c = np.full(off, 2, np.uint8)
    for (nx, ny, pitch, o), c in zip(descs, classes):
        flat_c[o:o + pitch * ny].reshape(ny, pitch)[:, :nx] = c
    return flat_c, descs


def unpack(flat, descs):
    return [flat[o:o + p * ny].reshape(ny, p)[:, :nx] for nx, ny, p, o in descs]


@pytest.mark.parametrize("pad", [0, 3])
def test_batch_matches_solo_and_converges(ctx, orc, pad):
    sides = [64, 128, 256, 512, 64, 128, 96, 200, 130, 64, 256, 1024]
    classes = []
    for k, n in enumerate(sides):
        sc = scenarios.scenario("batch", seed=3000 + k, side=n)
        classes.append(orc.rasterize(sc)[0])
    flat_c, descs = pack(classes, pad)
    cls = torch.as_tensor(flat_c).cuda()
    psi = torch.zeros(len(flat_c), dtype=torch.float32, device="cuda")
    print(f"batch of {len(sides)} grids, pad={pad}", flush=True)
    stats = ctx.relax_batched(cls, psi, descs, tol=1e-6, sweeps_per_pass=4)
    torch.cuda.synchronize()
    got = unpack(psi.cpu().numpy(), descs)
    for k, (c, st, g) in enumerate(zip(classes, stats, got)):
        assert st["status"] == 0, (k, st)
        r = orc.residual(c, g.astype(np.float64))
        assert r <= 1e-6 and abs(r - st["residual"]) <= 1e-12, (k, r, st)
    # bit-exact against the same sweeps run on the grid alone
    for k in (0, 5, 11):
        c = torch.as_tensor(classes[k]).cuda()
        solo = torch.where(c == 3, 1.0, torch.where(c == 0, 0.5, 0.0)).float()
        st = stats[k]
        assert st["sweeps"] % 4 == 0
        ctx.sweeps(c, solo, st["omega"], st["sweeps"], sweeps_per_pass=4)
        torch.cuda.synchronize()
        assert np.array_equal(solo.cpu().numpy(), got[k]), k


def test_batch_graphs_equal_eager(ctx, orc):
    """The batched relaxation gives identical fields and statistics with its
    passes replayed from a captured graph and launched one by one."""
    sides = [64, 256, 128, 512, 96]
    classes = [orc.rasterize(scenarios.scenario("batch", seed=3100 + k, side=n))[0] for k, n in enumerate(sides)]
    flat_c, descs = pack(classes, 0)
    cls = torch.as_tensor(flat_c).cuda()
    out = []
    try:
        for graphs in (False, True, True):
            ctx.set_graphs(graphs)
            psi = torch.zeros(len(flat_c), dtype=torch.float32, device="cuda")
            st = ctx.relax_batched(cls, psi, descs, tol=1e-6, sweeps_per_pass=2)
            torch.cuda.synchronize()
            out.append((psi.cpu().numpy(), [(s["sweeps"], s["residual"], s["status"]) for s in st]))
    finally:
        ctx.set_graphs(True)
    for psi, st in out[1:]:
        assert np.array_equal(psi, out[0][0])
        assert st == out[0][1]


def test_batch_checked_often_converges(ctx, orc):
    """With residual checks as often as the batch allows (every 8 passes),
    every grid still runs to the tolerance: the noisy early residuals of a
    large grid are not taken for its rounding floor."""
    sides = [64, 256, 1024, 512]
    classes = [orc.rasterize(scenarios.scenario("batch", seed=3200 + k, side=n))[0] for k, n in enumerate(sides)]
    flat_c, descs = pack(classes, 0)
    cls = torch.as_tensor(flat_c).cuda()
    psi = torch.zeros(len(flat_c), dtype=torch.float32, device="cuda")
    stats = ctx.relax_batched(cls, psi, descs, tol=1e-6, sweeps_per_pass=4, check_passes=1)
    torch.cuda.synchronize()
    got = unpack(psi.cpu().numpy(), descs)
    for k, (c, st, g) in enumerate(zip(classes, stats, got)):
        assert st["status"] == 0, (k, st)
        r = orc.residual(c, g.astype(np.float64))
        assert r <= 1e-6 and abs(r - st["residual"]) <= 1e-12, (k, r, st)


def test_batch_rejects_bad_arguments(ctx):
    from paper_1903_07441_amd import twg
    cls = torch.zeros(100, dtype=torch.uint8, device="cuda")
    psi = torch.zeros(100, dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        ctx.relax_batched(cls, psi, [(10, 20, 10, 0)])
    with pytest.raises(twg.TwgError):
        ctx.relax_batched(cls, psi, [(10, 5, 9, 0)])
