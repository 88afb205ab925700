"""The device-driven relaxation: asynchronous launches equal the blocking
call bit for bit, a captured graph replays to the same bits, the budget and
non-finite outcomes reach the device stats, and the linear-ramp start equals
the oracle's."""
import numpy as np
import pytest
import torch

from paper_1903_07441_amd import scenarios
from test_gpu_relax import gpu_relax, random_classes, to_dev

pytestmark = pytest.mark.gpu


def _scenario_cls(orc, name, idx, side=None):
    sc = scenarios.scenario(name, idx, side=side)
    cls, _ = orc.rasterize(sc)
    return sc, cls


def _fields(cls):
    ny, nx = cls.shape
    psi = to_dev(np.zeros((ny, nx), np.float32))
    psi64 = to_dev(np.zeros((ny, nx)), dtype=torch.float64)
    return psi, psi64


KEYS = ("sweeps", "polish_sweeps", "residual", "residual32", "status", "polish_rounds", "checks", "omega")


@pytest.mark.parametrize("polish", [0, 1])
def test_async_equals_blocking(ctx, orc, polish):
    from paper_1903_07441_amd import twg
    sc, cls = _scenario_cls(orc, "warped512", 0)
    c = to_dev(cls)
    kw = dict(tol=1e-6, polish=polish, tol_cert=5e-7 if polish else 0.0)
    pb, pb64 = _fields(cls)
    sb = ctx.relax(c, pb, pb64 if polish else None, **kw)
    pa, pa64 = _fields(cls)
    stats = ctx.relax_async(c, pa, pa64 if polish else None, slots=4000, **kw)
    sa = twg.stats_from_device(stats)
    print(f"polish={polish} blocking {sb}\nasync {sa}", flush=True)
    assert sb["status"] == twg.OK
    for k in KEYS:
        assert sa[k] == sb[k], k
    assert torch.equal(pa, pb)
    if polish:
        assert torch.equal(pa64, pb64)
        assert orc.residual(cls, pa64.cpu().numpy()) <= sa["residual"] * (1 + 1e-9) + 1e-300


def test_async_graph_replays_equal_eager(ctx, orc):
    """The asynchronous relaxation (FP32 solve and defect correction)
    captured once into a graph: every replay, with eager work and
    synchronisations between replays, gives the eager call's bits and
    stats."""
    from paper_1903_07441_amd import twg
    sc, cls = _scenario_cls(orc, "warped512", 1, side=256)
    c = to_dev(cls)
    kw = dict(tol=1e-6, polish=1, tol_cert=5e-7)
    pe, pe64 = _fields(cls)
    se = twg.stats_from_device(ctx.relax_async(c, pe, pe64, slots=1500, **kw))
    assert se["status"] == twg.OK
    psi, psi64 = _fields(cls)
    stats = torch.zeros(twg.STATS_BYTES, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.relax_async(c, psi, psi64, slots=1500, stats=stats, **kw)
    for rep in range(3):
        psi.fill_(-3.0)
        psi64.fill_(-3.0)
        stats.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        sr = twg.stats_from_device(stats)
        print(f"replay {rep}: {sr}", flush=True)
        for k in KEYS:
            assert sr[k] == se[k], (rep, k)
        assert torch.equal(psi, pe) and torch.equal(psi64, pe64)
        # eager work between replays
        junk, _ = _fields(cls)
        ctx.relax(c, junk, None, tol=1e-4)
        torch.cuda.synchronize()
    del g


@pytest.mark.parametrize("polish", [0, 1])
def test_async_budget_ends_the_solve(ctx, orc, polish):
    # too few slots: the final launch ends the solve as NOT_CONVERGED with
    # the latest field in psi (and psi64 when polishing), finite
    from paper_1903_07441_amd import twg
    sc, cls = _scenario_cls(orc, "warped512", 2)
    c = to_dev(cls)
    psi, psi64 = _fields(cls)
    stats = ctx.relax_async(c, psi, psi64 if polish else None, slots=12, tol=1e-6, polish=polish,
                            tol_cert=5e-7 if polish else 0.0, sweeps_per_pass=4)
    st = twg.stats_from_device(stats)
    print(f"budget-limited: {st}", flush=True)
    assert st["status"] == twg.NOT_CONVERGED
    f = psi.cpu().numpy()
    assert np.all(np.isfinite(f)) and not np.all(f[cls == 0] == 0.5)
    if polish:
        np.testing.assert_array_equal(psi64.cpu().numpy(), f.astype(np.float64))
    # a blocking call with a one-pass budget stops after that pass
    pb, _ = _fields(cls)
    sb = ctx.relax(c, pb, None, tol=1e-6, max_sweeps=4, sweeps_per_pass=4)
    assert sb["status"] == twg.NOT_CONVERGED and sb["sweeps"] == 4


def test_kept_field_polish_cut_short_by_the_budget(ctx, orc):
    # a converged FP32 field kept for the polish, with three slots: the first
    # defect finds the field converged (no FP32 sweep), two correction passes
    # run, the final launch ends the solve; the kept field is untouched and
    # the FP64 field is its widened copy (no update ran)
    from paper_1903_07441_amd import twg
    sc, cls = _scenario_cls(orc, "warped512", 1)
    c = to_dev(cls)
    psi, psi64 = _fields(cls)
    ctx.relax(c, psi, None, tol=1e-6)
    torch.cuda.synchronize()
    kept = psi.cpu().numpy().copy()
    r32 = ctx.residual(c, psi=psi)
    stats = ctx.relax_async(c, psi, psi64, slots=3, tol=1e-6, init=twg.INIT_KEEP, polish=1, tol_cert=5e-7)
    st = twg.stats_from_device(stats)
    print(f"kept, budget-limited: {st}", flush=True)
    assert st["status"] == twg.NOT_CONVERGED and st["sweeps"] == 0 and st["polish_rounds"] == 0
    assert st["residual32"] == r32
    f = psi.cpu().numpy()
    assert np.array_equal(f, kept)
    np.testing.assert_array_equal(psi64.cpu().numpy(), f.astype(np.float64))


def test_non_finite_field_is_reported(ctx):
    from paper_1903_07441_amd import twg
    rng = np.random.default_rng(4)
    cls = random_classes(rng, 128, 96)
    c = to_dev(cls)
    psi0 = np.full((96, 128), 0.5, np.float32)
    fy, fx = np.argwhere(cls == 0)[17]
    psi0[fy, fx] = np.nan
    psi = to_dev(psi0)
    with pytest.raises(twg.TwgError) as e:
        ctx.relax(c, psi, None, tol=1e-6, init=twg.INIT_KEEP)
    assert e.value.code == twg.EINVAL
    psi = to_dev(psi0)
    st = twg.stats_from_device(ctx.relax_async(c, psi, None, slots=50, tol=1e-6, init=twg.INIT_KEEP))
    assert st["status"] == twg.EINVAL


def test_linear_init_matches_oracle(ctx, orc):
    from paper_1903_07441_amd import twg
    sc, cls = _scenario_cls(orc, "warped512", 3, side=301)
    ny, nx = cls.shape
    c = to_dev(cls, 320)
    psi = to_dev(np.full((ny, nx), 7.0, np.float32), 320)
    ctx.init_field(c, psi, twg.INIT_LINEAR, goal=sc["goal"])
    want = orc.field_init(cls, np.full((ny, nx), 7.0), orc.INIT_LINEAR, goal=sc["goal"]).astype(np.float32)
    np.testing.assert_array_equal(psi.cpu().numpy(), want)
    # and the relaxation from it reaches the tolerance
    st = ctx.relax(c, psi, None, tol=1e-6, init=twg.INIT_LINEAR, goal=sc["goal"])
    assert st["status"] == twg.OK
    assert orc.residual(cls, psi.cpu().numpy().astype(np.float64)) <= 1e-6


def test_paper_mode_100_sweeps_match_oracle(ctx, orc):
    # the paper's own mode (Algorithm 1 iterates a fixed 100 times): 100
    # Gauss-Seidel sweeps (omega = 1) from the half field, on the 2048 x 2048
    # replanning map; the FP32 field stays within FP32 rounding of the
    # oracle's 100 FP64 sweeps, and FP64 sweeps match it bit for bit
    sc = scenarios.scenario("replan2048", 1)
    cls, _ = orc.rasterize(sc)
    ny, nx = cls.shape
    want = orc.field_init(cls, None, orc.INIT_HALF)
    for _ in range(100):
        want = orc.sor_sweep(cls, want, 1.0)
    c = to_dev(cls)
    from paper_1903_07441_amd import twg
    psi = to_dev(np.zeros((ny, nx), np.float32))
    ctx.init_field(c, psi, twg.INIT_HALF)
    ctx.sweeps(c, psi, 1.0, 100)
    p64 = to_dev(orc.field_init(cls, None, orc.INIT_HALF), dtype=torch.float64)
    ctx.sweeps64(c, p64, 1.0, 100)
    torch.cuda.synchronize()
    err = float(np.max(np.abs(psi.cpu().numpy() - want)))
    print(f"paper mode: max|fp32 - oracle| = {err:.3e}", flush=True)
    assert err <= 1e-5
    np.testing.assert_array_equal(p64.cpu().numpy(), want)
