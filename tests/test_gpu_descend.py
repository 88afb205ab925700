"""GPU parity of the index matrix (Eq. 3) and the descent walk."""
import numpy as np
import pytest
import torch

from conftest import reachable_scenario
from paper_1903_07441_amd import scenarios
from test_gpu_relax import gpu_relax, random_classes, to_dev

pytestmark = pytest.mark.gpu


def gpu_descend(ctx, c, psi_t, start, cap=None, use64=False):
    if use64:
        path, info = ctx.descend(c, psi64=psi_t, start=start, cap=cap)
    else:
        path, info = ctx.descend(c, psi=psi_t, start=start, cap=cap)
    torch.cuda.synchronize()
    n, status = info.cpu().tolist()
    return status, path[:n].cpu().numpy()


@pytest.mark.parametrize("name,idx", [("static64", 0), ("static64", 5), ("warped512", 0)])
def test_index_and_path_parity(ctx, orc, name, idx):
    sc = scenarios.scenario(name, idx)
    cls, _ = orc.rasterize(sc)
    st, psi, psi64, c = gpu_relax(ctx, cls, tol=1e-6, polish=True, tol_cert=1e-7)
    for use64, field in ((False, psi), (True, psi64)):
        t = to_dev(field) if not use64 else to_dev(field, dtype=torch.float64)
        kw = dict(psi64=t) if use64 else dict(psi=t)
        idx_gpu = ctx.index_matrix(c, **kw)
        torch.cuda.synchronize()
        want = orc.index_matrix(cls, field.astype(np.float64))
        np.testing.assert_array_equal(idx_gpu.cpu().numpy(), want)
        s_gpu, p_gpu = gpu_descend(ctx, c, t, sc["robot"], use64=use64)
        s_orc, p_orc = orc.descend(cls, field.astype(np.float64), sc["robot"])
        assert s_gpu == s_orc
        np.testing.assert_array_equal(p_gpu, p_orc)
        if orc.goal_reachable(cls, sc["robot"]):
            assert s_gpu == 0 and cls[p_gpu[-1][1], p_gpu[-1][0]] == 3


@pytest.mark.parametrize("pitch_pad", [0, 4, 3])
def test_descent_2048_reaches_goal(ctx, orc, pitch_pad):
    # a path of thousands of cells to a reachable goal: the walk re-stages
    # its window many times, with 128-bit staging loads (pitch a multiple of
    # 16), 32-bit ones (multiple of 4) or byte loads
    sc = reachable_scenario("replan2048", 0)
    cls, _ = orc.rasterize(sc)
    st, psi, psi64, _ = gpu_relax(ctx, cls, tol=1e-6, polish=True, tol_cert=5e-7)
    pitch = cls.shape[1] + pitch_pad
    c = to_dev(cls, pitch)
    t = to_dev(psi64, pitch, dtype=torch.float64)
    s_gpu, p_gpu = gpu_descend(ctx, c, t, sc["robot"], use64=True)
    s_orc, p_orc = orc.descend(cls, psi64, sc["robot"])
    assert s_gpu == s_orc
    np.testing.assert_array_equal(p_gpu, p_orc)
    print(f"2048 descent status={s_gpu} length={len(p_gpu)}", flush=True)
    assert s_gpu == 0 and len(p_gpu) > 500
    # buffers that fill on either side of the walk's 64-cell store groups, or
    # exactly at the goal: a truncated path is the full path's prefix
    n = len(p_gpu)
    for cap in (63, 64, 65, 128, n - 1, n):
        s_cap, p_cap = gpu_descend(ctx, c, t, sc["robot"], cap=cap, use64=True)
        np.testing.assert_array_equal(p_cap, p_gpu[:cap])
        assert s_cap == (s_gpu if cap >= n else 5)


def test_descent_outcomes(ctx, orc):
    rng = np.random.default_rng(0)
    cls = random_classes(rng, 80, 60, p=0.1)
    gy, gx = np.argwhere(cls == 3)[0]
    # enclose the goal: NO_PATH from outside
    enc = cls.copy()
    enc[gy - 1:gy + 2, gx - 1:gx + 2] = np.where(enc[gy - 1:gy + 2, gx - 1:gx + 2] == 3, 3, 1)
    st, psi, psi64, c = gpu_relax(ctx, enc, tol=1e-6)
    free = np.argwhere(enc == 0)
    y0, x0 = free[len(free) // 2]
    s, p = gpu_descend(ctx, c, to_dev(psi), (x0, y0))
    assert s == 2 and len(p) >= 1
    # start on an obstacle
    oy, ox = np.argwhere(enc == 1)[0]
    s, p = gpu_descend(ctx, c, to_dev(psi), (ox, oy))
    assert s == 3 and len(p) == 0
    # start on the goal
    s, p = gpu_descend(ctx, c, to_dev(psi), (gx, gy))
    assert s == 0 and len(p) == 1
    # truncated
    st, psi, _, c = gpu_relax(ctx, cls, tol=1e-7)
    far = np.argwhere(cls == 0)
    dist = np.abs(far[:, 0] - gy) + np.abs(far[:, 1] - gx)
    y1, x1 = far[np.argmax(dist)]
    s_full, p_full = gpu_descend(ctx, c, to_dev(psi), (x1, y1))
    s_orc, p_orc = orc.descend(cls, psi.astype(np.float64), (x1, y1))
    assert s_full == s_orc and np.array_equal(p_full, p_orc)
    if s_full == 0 and len(p_full) > 3:
        s, p = gpu_descend(ctx, c, to_dev(psi), (x1, y1), cap=3)
        assert s == 5 and len(p) == 3
        np.testing.assert_array_equal(p, p_full[:3])


def test_descend_rejects_bad_arguments(ctx):
    from paper_1903_07441_amd import twg
    c = to_dev(np.zeros((10, 10), np.uint8))
    psi = to_dev(np.zeros((10, 10), np.float32))
    with pytest.raises(twg.TwgError):
        ctx.descend(c, psi=psi, start=(10, 0))
    with pytest.raises(twg.TwgError):
        ctx.descend(c, psi=psi, start=(0, 0), cap=0)


def test_descent_grade_field_reaches_goal_2048(ctx, orc):
    # scenario 1: the goal is reachable, but psi at the robot is ~1e-13; the
    # FP64 polish plus FP64 sweeps until the descent resolves (twg.plan) gives
    # a path, identical to the oracle's walk on the same field
    from paper_1903_07441_amd import twg
    sc = scenarios.scenario("replan2048", 1)
    cls, _ = orc.rasterize(sc)
    assert orc.goal_reachable(cls, sc["robot"])
    c = to_dev(cls)
    psi = torch.zeros((2048, 2048), dtype=torch.float32, device="cuda")
    psi64 = torch.zeros((2048, 2048), dtype=torch.float64, device="cuda")
    plain, pol, path, info, rounds = twg.plan(ctx, c, psi, psi64, sc["robot"])
    torch.cuda.synchronize()
    n, status = info.cpu().tolist()
    print(f"plan: plain={plain['sweeps']} polish={pol['polish_sweeps']} rounds={rounds} status={status} "
          f"length={n}", flush=True)
    assert pol["status"] == 0 and pol["cert_bound"] <= 5e-7
    f64 = psi64.cpu().numpy()
    assert orc.residual(cls, f64) * orc.wbound(2048, 2048) <= 5e-7
    s_orc, p_orc = orc.descend(cls, f64, sc["robot"])
    assert status == s_orc == 0
    p_gpu = path[:n].cpu().numpy()
    np.testing.assert_array_equal(p_gpu, p_orc)
    steps = np.abs(np.diff(p_gpu, axis=0)).sum(axis=1)
    assert np.all(steps == 1) and cls[p_gpu[-1][1], p_gpu[-1][0]] == 3


@pytest.mark.parametrize("name,idx,k", [("static64", 1, 1.0), ("static64", 6, 0.3), ("warped512", 3, 2.0)])
def test_rubber_band_parity(ctx, orc, name, idx, k):
    """The GPU rubber band equals the oracle's on the oracle's field and path
    (bit-exact: same FP64 arithmetic, same candidate order and colours)."""
    sc = scenarios.scenario(name, idx, side=128 if name == "warped512" else None)
    cls_o, _ = orc.rasterize(sc)
    psi, _ = orc.relax(cls_o, tol=1e-11)
    st, path = orc.descend(cls_o, psi, sc["robot"])
    if len(path) < 3:
        pytest.skip("path too short for a band")
    print(f"rubber band {name}[{idx}] k={k} n={len(path)}", flush=True)
    want = orc.rubber_band(cls_o, psi, path, k=k, iters=24)
    cls = torch.as_tensor(cls_o).cuda()
    cap = len(path) + 7
    for fp64 in (True, False):
        field = psi if fp64 else psi.astype(np.float32)
        dev_path = torch.zeros((cap, 2), dtype=torch.int32, device="cuda")
        dev_path[:len(path)] = torch.as_tensor(path).cuda()
        info = torch.tensor([len(path), st], dtype=torch.int32, device="cuda")
        f = torch.as_tensor(field).cuda()
        if fp64:
            ctx.rubber_band(cls, dev_path, info, psi64=f, k=k, iters=24)
            ref = want
        else:
            ctx.rubber_band(cls, dev_path, info, psi=f, k=k, iters=24)
            ref = orc.rubber_band(cls_o, field.astype(np.float64), path, k=k, iters=24)
        torch.cuda.synchronize()
        got = dev_path.cpu().numpy()
        assert np.array_equal(got[:len(path)], ref), (name, idx, fp64)
        assert np.all(got[len(path):] == 0)


@pytest.mark.parametrize("name,idx,side,pitch_pad", [("static64", 2, None, 0), ("warped512", 4, 120, 5)])
def test_descent_from_every_cell(ctx, orc, name, idx, side, pitch_pad):
    """Pointer-jumping descent from every cell equals the oracle's walk from
    each cell (length to the goal, or -1), on the oracle's field."""
    sc = scenarios.scenario(name, idx, side=side)
    cls_o, _ = orc.rasterize(sc)
    psi, _ = orc.relax(cls_o, tol=1e-12)
    ny, nx = cls_o.shape
    want = np.full((ny, nx), -1, np.int64)
    for y in range(ny):
        for x in range(nx):
            if cls_o[y, x] in (orc.FREE, orc.GOAL):
                st, p = orc.descend(cls_o, psi, (x, y))
                if st == orc.OK:
                    want[y, x] = len(p) - 1
    pitch = nx + pitch_pad
    c = torch.zeros((ny, pitch), dtype=torch.uint8, device="cuda")[:, :nx]
    c.copy_(torch.as_tensor(cls_o))
    f = torch.zeros((ny, pitch), dtype=torch.float64, device="cuda")[:, :nx]
    f.copy_(torch.as_tensor(psi))
    print(f"descent from every cell {name}[{idx}] {nx}x{ny}", flush=True)
    steps = ctx.descent_all(c, psi64=f)
    torch.cuda.synchronize()
    got = steps.cpu().numpy()
    assert np.array_equal(got, want)
    # discrete maximum principle: every FREE cell that can reach the goal does
    reach = (want >= 0) | (cls_o != orc.FREE)
    assert reach.mean() > 0.5
