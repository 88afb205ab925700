"""GPU parity of the batched relaxation: every grid of an uneven batch meets the
tolerance (residual recomputed by the oracle) and equals, bit for bit, the same
number of sweeps run on that grid alone, whether the tiled passes or the
LDS-resident worker (small grids) solved it; the asynchronous and
graph-captured batch equal the blocking one."""
import ctypes

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


def test_batch_full_workload_as_benchmarked(orc):
    # the benchmark's batch at full size: 256 grids of sides {64, ..., 1024}
    # (seed 3000), factors per size and the batch tiling from the library's
    # autotuners, tolerance 1e-6; every grid's residual recomputed by the
    # oracle, and one grid of each size equal, bit for bit, to the same
    # sweeps run on it alone
    from paper_1903_07441_amd import twg
    scs = scenarios.batch(256, seed=3000)
    classes = [orc.rasterize(sc)[0] for sc in scs]
    flat_c, descs = pack(classes)
    ctx = twg.Context(0)
    try:
        cls = torch.as_tensor(flat_c).cuda()
        psi = torch.zeros(len(flat_c), dtype=torch.float32, device="cuda")
        first = {}
        for k, (nx, ny, p, o) in enumerate(descs):
            if (nx, ny) not in first:
                first[(nx, ny)] = k
                ctx.autotune(cls[o:o + p * ny].view(ny, p)[:, :nx])
        bt = ctx.autotune_batched(cls, descs)
        print(f"batch of {len(descs)} grids, {len(flat_c)} cells, tiling {bt}", flush=True)
        stats = ctx.relax_batched(cls, psi, descs, tol=1e-6)
        torch.cuda.synchronize()
        got = unpack(psi.cpu().numpy(), descs)
        for k, (c, st, g) in enumerate(zip(classes, stats, got)):
            assert st["status"] == 0, (k, st)
            r = orc.residual(c, g.astype(np.float64))
            assert r <= 1e-6 and abs(r - st["residual"]) <= 1e-12, (k, r, st)
        for (nx, ny), k in sorted(first.items()):
            c = torch.as_tensor(classes[k]).cuda()
            solo = torch.where(c == 3, 1.0, torch.where(c == 0, 0.5, 0.0)).float()
            st = stats[k]
            assert st["sweeps"] % bt["S"] == 0
            ctx.sweeps(c, solo, st["omega"], st["sweeps"], sweeps_per_pass=bt["S"])
            torch.cuda.synchronize()
            assert np.array_equal(solo.cpu().numpy(), got[k]), (nx, ny, k)
    finally:
        ctx.close()


def test_batch_async_and_graph_equal_blocking(ctx, orc):
    """The asynchronous batch (fixed slot count, device-side stop) gives the
    fields and statistics of the blocking call, and so does the same call
    captured into a graph and replayed, on every replay, with eager work
    between the replays."""
    from paper_1903_07441_amd import twg
    sides = [64, 256, 128, 512, 96]
    classes = [orc.rasterize(scenarios.scenario("batch", seed=3100 + k, side=n))[0] for k, n in enumerate(sides)]
    flat_c, descs = pack(classes, 0)
    cls = torch.as_tensor(flat_c).cuda()
    n = len(sides)
    psi = torch.zeros(len(flat_c), dtype=torch.float32, device="cuda")
    want = ctx.relax_batched(cls, psi, descs, tol=1e-6, sweeps_per_pass=2)
    torch.cuda.synchronize()
    want_psi = psi.clone()
    slots = max(s["sweeps"] for s in want) // 2 + 16
    print(f"async batch of {n} grids: {slots} slots", flush=True)
    psi_a = torch.zeros_like(psi)
    stats = ctx.relax_batched(cls, psi_a, descs, tol=1e-6, sweeps_per_pass=2, slots=slots)
    got = twg.batch_stats_from_device(stats, n)
    assert torch.equal(psi_a, want_psi)
    assert [(s["sweeps"], s["residual"], s["status"]) for s in got] == \
        [(s["sweeps"], s["residual"], s["status"]) for s in want]
    # the same enqueue captured once and replayed
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        g.capture_begin()
        ctx.relax_batched(cls, psi_a, descs, tol=1e-6, sweeps_per_pass=2, slots=slots, stats=stats)
        g.capture_end()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    scratch = torch.zeros_like(psi)
    for rep in range(3):
        psi_a.fill_(-1.0)
        stats.zero_()
        g.replay()
        torch.cuda.synchronize()
        # eager work between replays (the same context scratch)
        ctx.relax_batched(cls, scratch, descs, tol=1e-3, sweeps_per_pass=2)
        got = twg.batch_stats_from_device(stats, n)
        print(f"replay {rep}: sweeps {[s['sweeps'] for s in got]}", flush=True)
        # every grid cell rewritten (the padding between grids is not part
        # of any grid)
        for a_k, w_k in zip(unpack(psi_a.cpu().numpy(), descs), unpack(want_psi.cpu().numpy(), descs)):
            assert np.array_equal(a_k, w_k)
        assert [s["sweeps"] for s in got] == [s["sweeps"] for s in want]


def test_batch_async_budget_ends_grids(ctx, orc):
    """Too few slots: the final launch ends the grids still running with
    status NOT_CONVERGED and their fields as their last pass left them (the
    same sweeps run alone), while grids that finished keep their result."""
    from paper_1903_07441_amd import twg
    sides = [64, 512]
    classes = [orc.rasterize(scenarios.scenario("batch", seed=3300 + k, side=n))[0] for k, n in enumerate(sides)]
    flat_c, descs = pack(classes, 0)
    cls = torch.as_tensor(flat_c).cuda()
    psi = torch.zeros(len(flat_c), dtype=torch.float32, device="cuda")
    full = ctx.relax_batched(cls, psi, descs, tol=1e-6, sweeps_per_pass=2)
    slots = full[0]["sweeps"] // 2 + 10  # the small grid finishes, the large one does not
    assert slots * 2 < full[1]["sweeps"]
    psi.zero_()
    stats = ctx.relax_batched(cls, psi, descs, tol=1e-6, sweeps_per_pass=2, slots=slots)
    st = twg.batch_stats_from_device(stats, 2)
    print(f"budget {slots} slots: {[(s['status'], s['sweeps']) for s in st]}", flush=True)
    assert st[0]["status"] == twg.OK and st[0]["sweeps"] == full[0]["sweeps"]
    assert st[1]["status"] == twg.NOT_CONVERGED and st[1]["sweeps"] == 2 * slots
    got = unpack(psi.cpu().numpy(), descs)
    for k in (0, 1):
        c = torch.as_tensor(classes[k]).cuda()
        solo = torch.where(c == 3, 1.0, torch.where(c == 0, 0.5, 0.0)).float()
        ctx.sweeps(c, solo, st[k]["omega"], st[k]["sweeps"], sweeps_per_pass=2)
        torch.cuda.synchronize()
        assert np.array_equal(solo.cpu().numpy(), got[k]), k


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


def test_batch_autotune_picks_a_tiling_the_batch_then_uses(ctx, orc):
    """hpf_autotune_batched remembers the fastest of its candidate tilings;
    a later batch call without a tiling of its own runs with it, bit for bit
    as the same call with that tiling given."""
    sides = [64, 256, 128, 512]
    classes = [orc.rasterize(scenarios.scenario("batch", seed=3400 + k, side=n))[0] for k, n in enumerate(sides)]
    flat_c, descs = pack(classes, 0)
    cls = torch.as_tensor(flat_c).cuda()
    bt = ctx.autotune_batched(cls, descs)
    print(f"batch tiling {bt}", flush=True)
    assert (bt["S"], bt["RH"]) in {(4, 32), (6, 64), (8, 64), (6, 128), (8, 128)} and bt["ms"] > 0
    a = torch.zeros(len(flat_c), dtype=torch.float32, device="cuda")
    b = torch.zeros_like(a)
    sa = ctx.relax_batched(cls, a, descs, tol=1e-6)
    sb = ctx.relax_batched(cls, b, descs, tol=1e-6, sweeps_per_pass=bt["S"], rows_per_tile=bt["RH"])
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert [s["sweeps"] for s in sa] == [s["sweeps"] for s in sb]
    assert all(s["sweeps"] % bt["S"] == 0 for s in sa)


def test_batch_rejects_bad_arguments(ctx):
    from paper_1903_07441_amd import twg
    cls = torch.zeros(100, dtype=torch.uint8, device="cuda")
    psi = torch.zeros(100, dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        ctx.relax_batched(cls, psi, [(10, 20, 10, 0)])
    with pytest.raises(twg.TwgError):
        ctx.relax_batched(cls, psi, [(10, 5, 9, 0)])


@pytest.mark.parametrize("lds", [True, False])
def test_batch_small_grids_in_lds(ctx, orc, lds):
    """Small grids solved whole in one workgroup's LDS (TWG_GRID_LDS) and the
    same grids through the tiled passes (the default): both meet the
    tolerance (oracle residual), and every field equals, bit for bit, its own
    sweep count run on the grid alone.  The LDS worker checks every S sweeps,
    so its check count is sweeps / S + 1; the tiled passes check far less
    often."""
    sides = [64, 96, 128, 130, 176, 64, 256]
    S = 4
    classes = [orc.rasterize(scenarios.scenario("batch", seed=3500 + k, side=n))[0] for k, n in enumerate(sides)]
    flat_c, descs = pack(classes, 0)
    cls = torch.as_tensor(flat_c).cuda()
    psi = torch.zeros(len(flat_c), dtype=torch.float32, device="cuda")
    stats = ctx.relax_batched(cls, psi, descs, tol=1e-6, sweeps_per_pass=S, lds=lds)
    torch.cuda.synchronize()
    got = unpack(psi.cpu().numpy(), descs)
    in_lds = [st["checks"] == st["sweeps"] // S + 1 for st in stats]
    print(f"lds={lds}: sweeps {[st['sweeps'] for st in stats]} checks {[st['checks'] for st in stats]} "
          f"LDS-solved {in_lds}", flush=True)
    for k, (c, st, g) in enumerate(zip(classes, stats, got)):
        assert st["status"] == 0, (k, st)
        assert st["sweeps"] % S == 0
        r = orc.residual(c, g.astype(np.float64))
        assert r <= 1e-6 and abs(r - st["residual"]) <= 1e-12, (k, r, st)
        cd = torch.as_tensor(c).cuda()
        solo = torch.where(cd == 3, 1.0, torch.where(cd == 0, 0.5, 0.0)).float()
        ctx.sweeps(cd, solo, st["omega"], st["sweeps"], tiled=False)
        torch.cuda.synchronize()
        assert np.array_equal(solo.cpu().numpy(), g), k
    if lds:
        # 64 x 64 needs 20 KiB: it fits in any workgroup's LDS
        assert in_lds[0] and in_lds[5]
    else:
        assert not in_lds[0] and not in_lds[5]


@pytest.mark.parametrize("lds", [True, False])
def test_batch_non_finite_field_is_rejected(ctx, orc, lds):
    """A NaN in a kept field: the grid's check finds it, on either path, and
    the call reports TWG_EINVAL."""
    from paper_1903_07441_amd import twg
    classes = [orc.rasterize(scenarios.scenario("batch", seed=3600 + k, side=n))[0] for k, n in enumerate([64, 128])]
    flat_c, descs = pack(classes, 0)
    cls = torch.as_tensor(flat_c).cuda()
    psi = torch.zeros(len(flat_c), dtype=torch.float32, device="cuda")
    free = np.flatnonzero(flat_c[:64 * 64] == 0)
    psi[int(free[len(free) // 2])] = float("nan")
    with pytest.raises(twg.TwgError) as e:
        ctx.relax_batched(cls, psi, descs, tol=1e-6, init=twg.INIT_KEEP, sweeps_per_pass=4, lds=lds)
    assert e.value.code == twg.EINVAL


def test_batch_rejects_unknown_grid_flags(ctx):
    from paper_1903_07441_amd import twg
    cls = torch.zeros(100, dtype=torch.uint8, device="cuda")
    psi = torch.zeros(100, dtype=torch.float32, device="cuda")
    arr = (twg.GridDesc * 1)(twg.GridDesc(10, 10, 10, 2, 0))
    prm = twg.HpfParams(1e-6, 0.0, 0, 0.0, twg.INIT_HALF, 0, 0, 0, 0, -1, -1)
    rc = twg.lib.hpf_relax_batched(ctx.h, 1, arr, twg._ptr(cls), twg._ptr(psi), ctypes.byref(prm), None,
                                   twg._stream())
    assert rc == twg.EINVAL
