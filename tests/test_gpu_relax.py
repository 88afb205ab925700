"""GPU parity of the relaxation: tiled sweeps vs untiled sweeps (bit-exact), FP32
sweeps vs the oracle's FP64 sweep, converged fields vs the oracle's certified
field, and the certificate at full size."""
import numpy as np
import pytest
import torch

from conftest import reachable_scenario, scenario_tensors
from paper_1903_07441_amd import scenarios

pytestmark = pytest.mark.gpu


def random_classes(rng, nx, ny, p=0.2, walls=True, fixed=0.0):
    cls = np.where(rng.uniform(size=(ny, nx)) < p, 1, 0).astype(np.uint8)
    if fixed:
        cls[(rng.uniform(size=(ny, nx)) < fixed) & (cls == 0)] = 4
    if walls:
        cls[0, :] = cls[-1, :] = cls[:, 0] = cls[:, -1] = 2
        cls[rng.integers(1, ny - 1), rng.integers(1, nx - 1)] = 3
    else:
        cls[rng.integers(0, ny), rng.integers(0, nx)] = 3
    return cls


def to_dev(a, pitch=None, dtype=None):
    t = torch.as_tensor(a)
    if dtype is not None:
        t = t.to(dtype)
    ny, nx = t.shape
    pitch = pitch or nx
    buf = torch.zeros((ny, pitch), dtype=t.dtype, device="cuda")
    buf[:, :nx] = t.to("cuda")
    return buf[:, :nx]


@pytest.mark.parametrize("nx,ny,pitch", [(64, 64, 64), (300, 211, 320), (129, 1000, 130),
                                         (1, 7, 1), (7, 1, 8), (2047, 33, 2048)])
@pytest.mark.parametrize("S", [1, 2, 3, 4, 5, 6, 7, 8])
def test_tiled_equals_untiled(ctx, nx, ny, pitch, S):
    # P12: S sweeps per tile load give the same bits as one launch per colour.
    rng = np.random.default_rng(nx * 7 + ny + S)
    cls = random_classes(rng, nx, ny, walls=nx > 2 and ny > 2, fixed=0.02)
    psi0 = rng.uniform(size=(ny, nx)).astype(np.float32)
    c = to_dev(cls, pitch)
    a = to_dev(psi0, pitch)
    b = to_dev(psi0, pitch)
    sweeps = 2 * S + 1
    print(f"tiled-vs-untiled nx={nx} ny={ny} pitch={pitch} S={S}", flush=True)
    ctx.sweeps(c, a, 1.83, sweeps, tiled=False)
    ctx.sweeps(c, b, 1.83, sweeps, tiled=True, sweeps_per_pass=S)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert not torch.equal(a, to_dev(psi0, pitch))


@pytest.mark.parametrize("S", [1, 4, 5, 8])
@pytest.mark.parametrize("nx", [257, 256])  # odd: per-column access; even: paired columns
def test_tiled_equals_untiled_with_source(ctx, S, nx):
    rng = np.random.default_rng(S)
    ny = 190
    cls = random_classes(rng, nx, ny)
    f = (rng.normal(size=(ny, nx)) * 1e-3).astype(np.float32)
    c, fd = to_dev(cls), to_dev(f)
    a = to_dev(np.zeros((ny, nx), np.float32))
    b = a.clone()
    ctx.sweeps(c, a, 1.9, 3 * S, tiled=False, f=fd)
    ctx.sweeps(c, b, 1.9, 3 * S, tiled=True, sweeps_per_pass=S, f=fd)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_resume_is_bit_exact(ctx):
    # k + m sweeps equal k sweeps, stop, then m sweeps
    rng = np.random.default_rng(3)
    cls = random_classes(rng, 200, 150)
    c = to_dev(cls)
    a = to_dev(rng.uniform(size=(150, 200)).astype(np.float32))
    b = a.clone()
    ctx.sweeps(c, a, 1.8, 20, sweeps_per_pass=4)
    ctx.sweeps(c, b, 1.8, 12, sweeps_per_pass=4)
    ctx.sweeps(c, b, 1.8, 8, sweeps_per_pass=4)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_fp32_sweep_tracks_fp64_oracle_sweep(ctx, orc):
    rng = np.random.default_rng(5)
    cls = random_classes(rng, 96, 80)
    psi = orc.field_init(cls, None, orc.INIT_HALF)
    c = to_dev(cls)
    g = to_dev(psi.astype(np.float32))
    for k in range(6):
        psi = orc.sor_sweep(cls, psi, 1.7)
    ctx.sweeps(c, g, 1.7, 6, sweeps_per_pass=2)
    torch.cuda.synchronize()
    assert np.max(np.abs(g.cpu().numpy() - psi)) < 2e-6


def gpu_relax(ctx, cls, **kw):
    ny, nx = cls.shape
    c = to_dev(cls)
    psi = to_dev(np.zeros((ny, nx), np.float32))
    psi64 = to_dev(np.zeros((ny, nx)), dtype=torch.float64)
    st = ctx.relax(c, psi, psi64 if kw.get("polish") else None, **kw)
    torch.cuda.synchronize()
    return st, psi.cpu().numpy(), psi64.cpu().numpy(), c


@pytest.mark.parametrize("idx", [0, 1, 2, 3])
def test_relax_parity_static64(ctx, orc, idx):
    sc = scenarios.scenario("static64", idx)
    cls, _ = orc.rasterize(sc)
    ref, info = orc.relax(cls, tol=1e-13, tol_cert=1e-10)
    assert info["status"] == orc.OK
    st, psi, psi64, _ = gpu_relax(ctx, cls, tol=1e-6, polish=True, tol_cert=1e-9)
    print(f"static64[{idx}] stats={st}", flush=True)
    assert st["status"] == 0
    assert np.max(np.abs(psi64 - ref)) <= 1e-6
    assert np.max(np.abs(psi - ref)) <= 1e-6
    # the GPU's own certificate is honest: recomputed by the oracle
    assert orc.residual(cls, psi64) <= st["residual"] * (1 + 1e-9) + 1e-300


@pytest.mark.parametrize("nx,ny,pitch", [(201, 151, 201), (200, 151, 203)])
@pytest.mark.parametrize("tuned", [False, True])
def test_relax_parity_unpaired_polish(orc, nx, ny, pitch, tuned):
    # an odd width or an odd pitch: every pass loads each lane's two columns
    # separately, also the correction passes that read the defect's products
    # with the correction factors; tuned: the autotuner's plan, which may add
    # a start phase (and its own product plane)
    from paper_1903_07441_amd import twg
    rng = np.random.default_rng(nx * 1000 + pitch)
    cls = random_classes(rng, nx, ny, p=0.15)
    ref, info = orc.relax(cls, tol=1e-13, tol_cert=1e-10)
    assert info["status"] == orc.OK
    ctx = twg.Context(0)
    try:
        c = to_dev(cls, pitch)
        if tuned:
            tune = ctx.autotune(c)
            print(f"{nx}x{ny}/{pitch} tuned {tune}", flush=True)
        psi = to_dev(np.zeros((ny, nx), np.float32), pitch)
        psi64 = to_dev(np.zeros((ny, nx)), pitch, dtype=torch.float64)
        st = ctx.relax(c, psi, psi64, tol=1e-6, polish=True, tol_cert=1e-9)
        torch.cuda.synchronize()
        print(f"{nx}x{ny}/{pitch} tuned={tuned} stats={st}", flush=True)
        assert st["status"] == 0 and st["cert_bound"] <= 1e-9
        f64 = psi64.cpu().numpy()
        assert np.max(np.abs(f64 - ref)) <= 1e-6
        assert orc.residual(cls, f64) * orc.wbound(nx, ny) <= 1e-9 * (1 + 1e-9)
    finally:
        ctx.close()


def _degenerate_grids():
    cases = []
    cases.append(("goal_only_1x1", np.array([[3]], np.uint8), None))
    c = np.full((2, 3), 2, np.uint8)
    c[1, 1] = 3
    cases.append(("no_free_cell_3x2", c, None))
    c = np.zeros((1, 9), np.uint8)
    c[0, 0] = c[0, -1] = 2
    c[0, 4] = 3
    cases.append(("one_row_9x1", c, None))
    c = np.zeros((13, 1), np.uint8)
    c[6, 0] = 3
    cases.append(("one_column_1x13", c, None))
    c = np.zeros((2, 8), np.uint8)
    c[1, 5] = 3
    cases.append(("two_rows_open_8x2", c, None))
    c = np.zeros((5, 6), np.uint8)
    c[2, 3] = 3
    cases.append(("open_no_walls_6x5", c, None))
    cases.append(("all_free_no_goal_7x7", np.zeros((7, 7), np.uint8), None))
    c = np.zeros((17, 33), np.uint8)
    c[0, :] = c[-1, :] = c[:, 0] = c[:, -1] = 2
    c[8, 5] = c[3, 20] = 4
    c[12, 28] = 3
    v = np.zeros((17, 33))
    v[8, 5], v[3, 20] = 0.75, 0.25
    cases.append(("fixed_values_33x17", c, v))
    return cases


@pytest.mark.parametrize("name,cls,vals", _degenerate_grids(), ids=[g[0] for g in _degenerate_grids()])
def test_relax_degenerate_grids(ctx, orc, name, cls, vals):
    # the device-driven solve and its polish on grids a tile barely covers or
    # that hold no FREE cell, no wall or no goal (cells outside the grid act
    # as fixed zeros), and FIXED cells keeping the caller's values
    from paper_1903_07441_amd import twg
    ny, nx = cls.shape
    v0 = np.zeros((ny, nx)) if vals is None else vals
    ref, info = orc.relax(cls, psi=v0, init=orc.INIT_ZERO, tol=1e-12, tol_cert=1e-10)
    assert info["status"] == orc.OK
    c = to_dev(cls)
    psi = to_dev(v0.astype(np.float32))
    psi64 = to_dev(v0, dtype=torch.float64)
    st = ctx.relax(c, psi, psi64, tol=1e-6, init=twg.INIT_ZERO, polish=1, tol_cert=1e-7)
    torch.cuda.synchronize()
    print(f"{name} stats={st}", flush=True)
    assert st["status"] == twg.OK and st["cert_bound"] <= 1e-7
    f64 = psi64.cpu().numpy()
    assert np.max(np.abs(f64 - ref)) <= 1e-6
    assert orc.residual(cls, f64) * orc.wbound(nx, ny) <= 1e-7 * (1 + 1e-9)
    fixed = cls != 0
    assert np.array_equal(f64[fixed], ref[fixed])


def test_relax_parity_warped512(ctx, orc):
    sc = scenarios.scenario("warped512", 0)
    cls, _ = orc.rasterize(sc)
    ref, info = orc.relax(cls, tol=1e-9, tol_cert=1e-8)
    assert info["status"] == orc.OK
    st, psi, psi64, c = gpu_relax(ctx, cls, tol=1e-6, polish=True, tol_cert=5e-7)
    print(f"warped512 stats={st}", flush=True)
    assert st["status"] == 0
    err = np.max(np.abs(psi64 - ref))
    print(f"warped512 max|gpu-oracle|={err:.3e}", flush=True)
    assert err <= 1e-6
    r = orc.residual(cls, psi64)
    assert r * orc.wbound(512, 512) <= 5e-7


def test_relax_fp32_only_reaches_tolerance(ctx, orc):
    sc = scenarios.scenario("warped512", 1)
    cls, _ = orc.rasterize(sc)
    st, psi, _, c = gpu_relax(ctx, cls, tol=1e-6)
    print(f"fp32-only stats={st}", flush=True)
    assert st["status"] == 0
    # FP64 residual of the returned FP32 field, recomputed by the oracle
    r = orc.residual(cls, psi.astype(np.float64))
    assert r <= 1e-6 and abs(r - st["residual"]) <= 1e-12


def test_kept_field_polish_starts_from_its_fp64_defect(ctx, orc):
    """A kept field already at tol, then the defect correction: the FP32
    stage sweeps nothing and reports the residual the standalone FP32
    residual kernel gives for that field, bit for bit (the first pass's
    fused check evaluates the same FP64 expression), and the correction
    still certifies the result."""
    from paper_1903_07441_amd import twg
    sc = scenarios.scenario("warped512", 0)
    cls, _ = orc.rasterize(sc)
    ny, nx = cls.shape
    c = to_dev(cls)
    psi = to_dev(np.zeros((ny, nx), np.float32))
    psi64 = to_dev(np.zeros((ny, nx)), dtype=torch.float64)
    ctx.relax(c, psi, None, tol=1e-6)
    r32 = ctx.residual(c, psi=psi)
    kept = psi.cpu().numpy()
    st = ctx.relax(c, psi, psi64, tol=1e-6, init=twg.INIT_KEEP, polish=1, tol_cert=5e-7)
    torch.cuda.synchronize()
    print(f"kept-field polish stats={st}", flush=True)
    assert st["sweeps"] == 0 and st["residual32"] == r32 and st["residual_rel"] > 0
    # the same residual recomputed by the oracle from the kept FP32 field
    assert abs(orc.residual(cls, kept.astype(np.float64)) - r32) <= 1e-12 * r32
    assert st["status"] == 0 and st["polish_sweeps"] > 0
    assert orc.residual(cls, psi64.cpu().numpy()) * orc.wbound(nx, ny) <= 5e-7


def test_kept_unconverged_field_polish_runs_the_fp32_stage(ctx, orc):
    """A kept field above tol: the polish's first defect finds it unconverged,
    the FP32 solve runs from its own initial check and the first defect comes
    again, so the result equals, bit for bit, the same solve started from the
    same field by HPF_INIT_ZERO (one check more for the first defect)."""
    from paper_1903_07441_amd import twg
    sc = scenarios.scenario("warped512", 2)
    cls, _ = orc.rasterize(sc)
    ny, nx = cls.shape
    c = to_dev(cls)
    out = {}
    for init in (twg.INIT_KEEP, twg.INIT_ZERO):
        psi = to_dev(np.where(cls == 3, 1.0, 0.0).astype(np.float32))
        psi64 = to_dev(np.zeros((ny, nx)), dtype=torch.float64)
        st = ctx.relax(c, psi, psi64, tol=1e-6, init=init, polish=1, tol_cert=5e-7)
        torch.cuda.synchronize()
        print(f"init={init} stats={st}", flush=True)
        assert st["status"] == twg.OK and st["sweeps"] > 0 and st["residual32"] <= 1e-6
        out[init] = (st, psi.cpu().numpy(), psi64.cpu().numpy())
    (sk, pk, qk), (sz, pz, qz) = out[twg.INIT_KEEP], out[twg.INIT_ZERO]
    assert np.array_equal(pk, pz) and np.array_equal(qk, qz)
    for key in ("sweeps", "polish_sweeps", "residual", "residual32", "residual_rel", "polish_rounds"):
        assert sk[key] == sz[key], key
    assert sk["checks"] == sz["checks"] + 1
    assert orc.residual(cls, qk) * orc.wbound(nx, ny) <= 5e-7


def test_relax_full_size_2048_certified(ctx, orc):
    # 2048 x 2048 time-warped field with a goal reachable from the start: the
    # certificate |psi - psi*| <= r * wbound (maximum principle, any size)
    # with r recomputed in FP64 by the oracle, and a field that is not
    # trivially zero
    sc = reachable_scenario("replan2048", 0)
    cls, _ = orc.rasterize(sc)
    st, psi, psi64, c = gpu_relax(ctx, cls, tol=1e-6, polish=True, tol_cert=5e-7)
    print(f"replan2048 goal draw {sc['goal_draw']} stats={st}", flush=True)
    assert st["status"] == 0
    r = orc.residual(cls, psi64)
    bound = r * orc.wbound(2048, 2048)
    print(f"replan2048 oracle residual={r:.3e} certified error bound={bound:.3e}", flush=True)
    assert bound <= 1e-6
    # the goal's component carries a potential well above the bound near the
    # goal (far from it the harmonic potential decays below any absolute
    # bound between the obstacles, so the robot's cell itself may hold
    # ~1e-11), and the robot's cell is strictly positive
    rx, ry = sc["robot"]
    above = int(np.count_nonzero(psi64[cls == 0] > 100 * bound))
    print(f"replan2048 cells above 100 x bound: {above}; psi64 at the robot {psi64[ry, rx]:.3e}", flush=True)
    assert above >= 1000 and psi64[ry, rx] > 0.0
    # the FP32 copy of the field is within FP32 rounding of the FP64 one
    assert np.max(np.abs(psi - psi64)) <= 6e-8


def test_relax_2048_enclosed_goal_is_zero_field(ctx, orc):
    # the unredrawn goal of replan2048[0] is enclosed by a predicted disc:
    # no FREE cell sees the goal's value, every other Dirichlet value is 0,
    # so the exact field is psi = 0 and the result lies within its own
    # certified bound of it
    sc = scenarios.scenario("replan2048", 0)
    cls, _ = orc.rasterize(sc)
    assert not orc.goal_reachable(cls, sc["robot"])
    st, psi, psi64, c = gpu_relax(ctx, cls, tol=1e-6, polish=True, tol_cert=5e-7)
    assert st["status"] == 0
    gx, gy = sc["goal"]
    nb = [cls[gy + dy, gx + dx] for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1))]
    assert all(v != 0 for v in nb)
    assert np.max(np.abs(psi64[cls == 0])) <= st["cert_bound"] <= 5e-7


def test_relax_closed_form_linear(ctx):
    # FIXED border at a linear ramp: the exact field is the ramp
    nx, ny = 150, 90
    cls = np.zeros((ny, nx), np.uint8)
    cls[0, :] = cls[-1, :] = cls[:, 0] = cls[:, -1] = 4
    xx = np.tile(np.arange(nx) / (nx - 1.0), (ny, 1))
    c = to_dev(cls)
    psi = to_dev(np.where(cls == 4, xx, 0.0).astype(np.float32))
    psi64 = to_dev(np.zeros((ny, nx)), dtype=torch.float64)
    st = ctx.relax(c, psi, psi64, tol=1e-7, polish=True, tol_cert=1e-8, init=0)
    torch.cuda.synchronize()
    # boundary values are the FP32-rounded ramp (|perturbation| <= 3e-8), so by
    # the maximum principle the field is within that of the ramp, plus the
    # certified 1e-8
    err = np.max(np.abs(psi64.cpu().numpy() - xx))
    assert st["status"] == 0 and err < 5e-8


def test_relax_not_converged_and_errors(ctx):
    from paper_1903_07441_amd import twg
    rng = np.random.default_rng(9)
    cls = random_classes(rng, 300, 300, p=0.05)
    st, _, _, c = gpu_relax(ctx, cls, tol=1e-9, max_sweeps=40)
    assert st["status"] == twg.NOT_CONVERGED and st["sweeps"] == 40
    psi = to_dev(np.zeros((300, 300), np.float32))
    with pytest.raises(twg.TwgError) as e:
        ctx.relax(c, psi, None, tol=1e-6, polish=True)
    assert e.value.code == twg.EINVAL
    with pytest.raises(twg.TwgError) as e:
        ctx.relax(c, psi, None, tol=-1.0)
    assert e.value.code == twg.EINVAL
    with pytest.raises(twg.TwgError) as e:
        ctx.relax(c, psi, None, omega=2.5)
    assert e.value.code == twg.EINVAL
    with pytest.raises(twg.TwgError) as e:
        ctx.relax(c, psi, None, sweeps_per_pass=9)
    assert e.value.code == twg.EINVAL


def test_relax_stops_at_the_fp32_rounding_floor(ctx, orc):
    # a tolerance FP32 cannot reach: the solve stops once the residual stops
    # improving, long before its (default, 10^7) sweep budget, and reports it
    from paper_1903_07441_amd import twg
    sc = scenarios.scenario("warped512", 2)
    cls, _ = orc.rasterize(sc)
    st, psi, _, _ = gpu_relax(ctx, cls, tol=1e-13)
    print(f"floor stats={st}", flush=True)
    assert st["status"] == twg.NOT_CONVERGED
    assert st["sweeps"] < 40 * 512
    assert 1e-13 < st["residual"] < 1e-5
    assert abs(orc.residual(cls, psi.astype(np.float64)) - st["residual"]) <= 1e-12


def test_relax_checked_every_pass_stops_at_the_first_converged_pass(ctx, orc):
    # a residual check after every pass: the solve runs to the first pass
    # whose residual meets the tolerance.  Not earlier (the max-norm residual
    # is not monotone from check to check, which must not read as a stall)
    # and not later (one pass fewer is still above it).
    from paper_1903_07441_amd import twg
    sc = scenarios.scenario("warped512", 2)
    cls, _ = orc.rasterize(sc)
    S = 4
    st, psi, _, _ = gpu_relax(ctx, cls, tol=1e-6, check_passes=1, sweeps_per_pass=S)
    print(f"checked every pass: stats={st}", flush=True)
    assert st["status"] == twg.OK and st["residual"] <= 1e-6
    assert st["sweeps"] % S == 0 and st["checks"] >= st["sweeps"] // S
    assert abs(orc.residual(cls, psi.astype(np.float64)) - st["residual"]) <= 1e-12
    st2, _, _, _ = gpu_relax(ctx, cls, tol=1e-6, check_passes=1, sweeps_per_pass=S, max_sweeps=st["sweeps"] - S)
    assert st2["status"] == twg.NOT_CONVERGED and st2["residual"] > 1e-6


@pytest.mark.parametrize("nx,ny,pitch", [(96, 80, 96), (301, 129, 320), (3, 40, 4)])
@pytest.mark.parametrize("S", [1, 3, 4, 5, 7])
def test_fp64_sweep_bit_exact_vs_oracle(ctx, orc, nx, ny, pitch, S):
    # P11: the GPU's FP64 red-black sweep equals the oracle's FP64 sweep bit for bit
    rng = np.random.default_rng(nx + S)
    cls = random_classes(rng, nx, ny, walls=nx > 2, fixed=0.02)
    psi0 = orc.field_init(cls, rng.uniform(size=(ny, nx)), orc.INIT_KEEP)
    want = psi0.copy()
    for _ in range(2 * S):
        want = orc.sor_sweep(cls, want, 1.87)
    c = to_dev(cls, pitch)
    a = to_dev(psi0, pitch, dtype=torch.float64)
    b = to_dev(psi0, pitch, dtype=torch.float64)
    ctx.sweeps64(c, a, 1.87, 2 * S, tiled=False)
    ctx.sweeps64(c, b, 1.87, 2 * S, tiled=True, sweeps_per_pass=S)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(a.cpu().numpy(), want)
    np.testing.assert_array_equal(b.cpu().numpy(), want)


@pytest.mark.parametrize("S", [2, 4, 8])
def test_graph_replay_equals_eager(ctx, S):
    """Runs of 64 passes replayed from a captured graph give the bits of one
    launch per colour; the cached graph is replayed again after eager work."""
    rng = np.random.default_rng(100 + S)
    nx, ny, pitch = 300, 211, 320
    cls = random_classes(rng, nx, ny, walls=True, fixed=0.02)
    psi0 = rng.uniform(size=(ny, nx)).astype(np.float32)
    c = to_dev(cls, pitch)
    sweeps = 3 * 64 * S + 5
    print(f"graph-vs-eager S={S} sweeps={sweeps}", flush=True)
    ref = to_dev(psi0, pitch)
    ctx.sweeps(c, ref, 1.9, sweeps, tiled=False)
    torch.cuda.synchronize()
    results = []
    try:
        for graphs in (True, False, True, True):
            ctx.set_graphs(graphs)
            a = to_dev(psi0, pitch)
            ctx.sweeps(c, a, 1.9, sweeps, tiled=True, sweeps_per_pass=S)
            torch.cuda.synchronize()
            results.append(a)
            # eager work between replays
            junk = to_dev(psi0, pitch)
            ctx.sweeps(c, junk, 1.5, 3, tiled=False)
            torch.cuda.synchronize()
    finally:
        ctx.set_graphs(True)
    for a in results:
        assert torch.equal(a, ref)


def test_autotune_factors_converge(orc):
    # the autotuner's tiling and factors, then the tuned relaxation and
    # defect-correction polish on the same 2048 x 2048 field; certificate
    # recomputed by the oracle
    from paper_1903_07441_amd import twg
    ctx = twg.Context(0)
    try:
        sc = scenarios.scenario("replan2048", 1)
        cls, _ = orc.rasterize(sc)
        c = to_dev(cls)
        tune = ctx.autotune(c)
        print(f"autotune {tune}", flush=True)
        assert 1 <= tune["S"] <= 8 and 2 <= tune["S64"] <= 8
        assert tune["RH"] >= 2 and tune["RH"] % 2 == 0
        assert 1.9 < tune["omega"] < 2.0 and 1.9 < tune["omega_dc"] < 2.0
        ny, nx = cls.shape
        # the correction solves' start phase, when kept, uses a smaller
        # factor for at most about n / 20 sweeps
        k = tune["lead_dc_sweeps"]
        assert k >= 0
        if k:
            assert 1.0 < tune["lead_dc_omega"] < tune["omega_dc"] and k <= max(nx, ny) // 20 + 4 * tune["S"]
        psi = to_dev(np.zeros((ny, nx), np.float32))
        psi64 = to_dev(np.zeros((ny, nx)), dtype=torch.float64)
        plain = ctx.relax(c, psi, None, tol=1e-6)
        pol = ctx.relax(c, psi, psi64, tol=1e-6, init=twg.INIT_KEEP, polish=1, tol_cert=1e-7)
        torch.cuda.synchronize()
        print(f"plain {plain['sweeps']} sweeps, polish {pol['polish_sweeps']} correction sweeps "
              f"in {pol['polish_rounds']} rounds", flush=True)
        assert plain["status"] == 0 and pol["status"] == 0
        assert abs(plain["omega"] - tune["omega"]) < 1e-6
        # the tuned factors keep both solves within a few thousand sweeps
        assert plain["sweeps"] < 4 * max(nx, ny) and pol["polish_sweeps"] < 4 * max(nx, ny)
        r = orc.residual(cls, psi64.cpu().numpy())
        assert r * orc.wbound(nx, ny) <= 1e-7
    finally:
        ctx.close()


def test_correction_start_phase_keeps_the_certified_field(orc):
    # the correction solves' start phase (tuned) changes only how the polish
    # gets there: with and without it (a caller's factor turns it off) the
    # polish reaches the certificate, both fields lie within their certified
    # bounds of each other, and the oracle's residual confirms each bound
    from paper_1903_07441_amd import twg
    ctx = twg.Context(0)
    try:
        sc = scenarios.scenario("warped512", 3)
        cls, _ = orc.rasterize(sc)
        c = to_dev(cls)
        tune = ctx.autotune(c)
        ny, nx = cls.shape
        out = []
        for omega in (0.0, tune["omega_dc"]):
            psi = to_dev(np.zeros((ny, nx), np.float32))
            psi64 = to_dev(np.zeros((ny, nx)), dtype=torch.float64)
            ctx.relax(c, psi, None, tol=1e-6)
            st = ctx.relax(c, psi, psi64, tol=1e-6, init=twg.INIT_KEEP, polish=1, tol_cert=1e-7, omega=omega)
            torch.cuda.synchronize()
            print(f"omega={omega}: lead {tune['lead_dc_omega']:.5f}/{tune['lead_dc_sweeps']} stats={st}", flush=True)
            assert st["status"] == twg.OK and st["cert_bound"] <= 1e-7
            f64 = psi64.cpu().numpy()
            assert orc.residual(cls, f64) * orc.wbound(nx, ny) <= 1e-7
            out.append((f64, st["cert_bound"]))
        (a, ca), (b, cb) = out
        assert np.max(np.abs(a - b)) <= ca + cb
    finally:
        ctx.close()
