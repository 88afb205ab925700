"""Pins of the oracle's time rings, Kalman prediction and rasterisation.

Brute force in plain Python integers, special cases whose answer is known
without the method (static obstacles, a single ring, exact tangency, a
rounding tie), and two independent routes inside the oracle itself.
"""
import math

import numpy as np
import pytest

from paper_1903_07441_amd import scenarios


def test_isqrt_exact(orc):
    rng = np.random.default_rng(0)
    vals = [0, 1, 2, 3, 4, 15, 16, 17, 2**32 - 1, 2**32, 2**52 + 1, 2**62, 2**64 - 1]
    vals += [int(v) for v in rng.integers(0, 2**63 - 1, size=2000, dtype=np.int64)]
    vals += [k * k + d for k in (7, 4096, 3037000499) for d in (-1, 0, 1)]
    for v in vals:
        assert orc.isqrt(v) == math.isqrt(v), v


def test_ring_brute_force(orc):
    # P8: j is the unique integer with (jW)^2 <= d^2 < ((j+1)W)^2.
    rng = np.random.default_rng(1)
    for _ in range(3000):
        dx, dy = (int(v) for v in rng.integers(-5000, 5000, size=2))
        W = int(rng.integers(1, 40))
        d2 = dx * dx + dy * dy
        j = 0
        while ((j + 1) * W) ** 2 <= d2:
            j += 1
        assert orc.ring_of(dx, dy, W) == j


def test_ring_map_and_count(orc):
    nx, ny, robot, W = 37, 29, (5, 20), 6
    rm = orc.ring_map(nx, ny, robot, W)
    for y in range(ny):
        for x in range(nx):
            d = math.sqrt((x - robot[0]) ** 2 + (y - robot[1]) ** 2)
            assert rm[y, x] == math.isqrt((x - robot[0]) ** 2 + (y - robot[1]) ** 2) // W
            assert rm[y, x] == int(d // W) or abs(d / W - round(d / W)) < 1e-12
    assert orc.num_rings(nx, ny, robot, W) == rm.max() + 1
    # lattice-point count of each annulus equals the ring's cell count
    for j in range(rm.max() + 1):
        cnt = sum(1 for y in range(ny) for x in range(nx)
                  if (j * W) ** 2 <= (x - robot[0]) ** 2 + (y - robot[1]) ** 2 < ((j + 1) * W) ** 2)
        assert cnt == int((rm == j).sum())


def test_ring_time(orc):
    assert orc.ring_time(0, 8, 1.0) == 0.0
    assert orc.ring_time(5, 8, 1.0) == 40.0
    assert orc.ring_time(3, 8, 2.0) == 12.0
    assert orc.ring_time(1, 1, 3.0) == 1.0 / 3.0


def test_kalman_closed_form_matches_iteration(orc):
    # P10: h steps of Eqs. (9)-(10) with dt = 1 equal one step with dt = h.
    rng = np.random.default_rng(3)
    for _ in range(50):
        p = rng.uniform(0, 500, size=2)
        v = rng.normal(0, 0.5, size=2)
        h = int(rng.integers(0, 300))
        x0 = np.array([p[0], p[1], v[0], v[1]])
        P0 = 0.25 * np.eye(4)
        x, P = orc.kalman_predict_steps(x0, P0, 1.0, h)
        mu = orc.predict_mean(p, v, float(h))
        np.testing.assert_allclose(x[:2], mu, rtol=1e-12, atol=1e-9)
        np.testing.assert_array_equal(x[2:], v)
        # covariance: A(h) P0 A(h)^T has position block 0.25 (1 + h^2) I
        np.testing.assert_allclose(P[0, 0], 0.25 * (1 + h * h), rtol=1e-12)
        np.testing.assert_allclose(P[0, 2], 0.25 * h, rtol=1e-12)
        assert P[0, 1] == 0.0 and P[2, 2] == 0.25
    # process noise accumulates: Q added at every step
    Q = np.diag([0.0, 0.0, 0.01, 0.01])
    x, P = orc.kalman_predict_steps(np.zeros(4), np.zeros((4, 4)), 1.0, 3, Q)
    # velocity variance 3 * 0.01; position variance sum_k k^2 * 0.01 for k = 0..2
    np.testing.assert_allclose(P[2, 2], 0.03, rtol=1e-12)
    np.testing.assert_allclose(P[0, 0], 0.01 * (0 + 1 + 4), rtol=1e-12)


def test_kalman_update_special_cases(orc):
    # Diagonal case reduces to the scalar textbook gain p / (p + r).
    x = np.array([1.0, 2.0, 0.5, -0.5])
    P = np.diag([4.0, 9.0, 1.0, 1.0])
    z = np.array([3.0, -1.0])
    R = np.diag([1.0, 3.0])
    x1, P1 = orc.kalman_update(x, P, z, R)
    np.testing.assert_allclose(x1[:2], [1 + 4 / 5 * 2, 2 + 9 / 12 * (-3)], rtol=1e-14)
    np.testing.assert_allclose(np.diag(P1)[:2], [4 * 1 / 5, 9 * 3 / 12], rtol=1e-14)
    np.testing.assert_array_equal(x1[2:], x[2:])  # no position-velocity correlation
    # a nearly perfect sensor moves the estimate onto the measurement
    x2, _ = orc.kalman_update(x, P, z, np.eye(2) * 1e-14)
    np.testing.assert_allclose(x2[:2], z, atol=1e-12)
    # correlation: velocity is corrected through P[0, 2]
    Pc = 0.25 * np.eye(4)
    Pc[0, 2] = Pc[2, 0] = 0.2
    x3, _ = orc.kalman_update(np.zeros(4), Pc, np.array([1.0, 0.0]), np.eye(2) * 0.25)
    np.testing.assert_allclose(x3[2], 0.2 / 0.5, rtol=1e-14)


def _python_rasterize(sc, border=True, static=None):
    """The rasterisation definition with Python integers and floats."""
    nx, ny = sc["nx"], sc["ny"]
    xr, yr = int(sc["robot"][0]), int(sc["robot"][1])
    xg, yg = int(sc["goal"][0]), int(sc["goal"][1])
    W, vr = sc["W"], sc["vr"]
    cls = np.zeros((ny, nx), np.uint8)
    for y in range(ny):
        for x in range(nx):
            if border and (x in (0, nx - 1) or y in (0, ny - 1)):
                cls[y, x] = 2
                continue
            if (x, y) == (xg, yg):
                cls[y, x] = 3
                continue
            if static is not None and static[y, x]:
                cls[y, x] = 1
                continue
            j = math.isqrt((x - xr) ** 2 + (y - yr) ** 2) // W
            t = (j * W) / vr
            for (px, py), (vx, vy), r in zip(sc["pos"], sc["vel"], sc["rad"]):
                cx = round(256.0 * (float(px) + t * float(vx)))  # Python round: half to even
                cy = round(256.0 * (float(py) + t * float(vy)))
                R = round(256.0 * float(r))
                if (256 * x - cx) ** 2 + (256 * y - cy) ** 2 <= R * R:
                    cls[y, x] = 1
                    break
    return cls


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rasterize_brute_force(orc, seed):
    # P9: the oracle's two routes and a plain-Python brute force agree bit for bit.
    sc = scenarios.custom(31, 26, 9, rad=(1.5, 4.0), vel_sigma=0.7, seed=seed, W=4)
    want = _python_rasterize(sc)
    a, ring_a = orc.rasterize(sc, "allpairs")
    b, ring_b = orc.rasterize(sc, "perobs")
    np.testing.assert_array_equal(a, want)
    np.testing.assert_array_equal(b, want)
    np.testing.assert_array_equal(ring_a, ring_b)
    assert (want == 1).sum() > 10


def test_rasterize_static_occupancy_and_precedence(orc):
    sc = scenarios.custom(24, 20, 4, seed=5, W=3)
    static = np.zeros((20, 24), np.uint8)
    static[5:9, 3:12] = 1
    static[sc["goal"][1], sc["goal"][0]] = 1  # the goal stays the goal
    static[0, :] = 1                          # walls stay walls
    want = _python_rasterize(sc, static=static)
    got, _ = orc.rasterize(sc, "perobs", static_occ=static)
    np.testing.assert_array_equal(got, want)
    assert got[sc["goal"][1], sc["goal"][0]] == 3
    assert np.all(got[0, :] == 2)
    got2, _ = orc.rasterize(sc, "allpairs", static_occ=static, border_walls=False)
    assert np.all(got2[0, 1:-1] == 1)


@pytest.mark.parametrize("seed", [10, 11, 12, 13])
def test_rasterize_routes_agree_on_scenarios(orc, seed):
    sc = scenarios.custom(200, 150, 60, rad=(3.0, 12.0), vel_sigma=0.5, seed=seed)
    a, _ = orc.rasterize(sc, "allpairs")
    b, _ = orc.rasterize(sc, "perobs")
    np.testing.assert_array_equal(a, b)


def test_static_obstacles_ignore_rings(orc):
    # v = 0: every ring predicts the current pose, so W does not matter.
    sc = scenarios.scenario("static64", index=3)
    a, _ = orc.rasterize(dict(sc, W=8), "perobs")
    b, _ = orc.rasterize(dict(sc, W=1), "perobs")
    c, _ = orc.rasterize(dict(sc, W=1000), "perobs")
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(a, c)


def test_single_ring_uses_current_poses(orc):
    # W wider than the diagonal: one ring (j = 0, horizon 0) = current poses.
    sc = scenarios.custom(40, 30, 8, vel_sigma=2.0, seed=9)
    one, ring = orc.rasterize(dict(sc, W=100), "allpairs")
    assert ring.max() == 0
    still, _ = orc.rasterize(dict(sc, W=100, vel=np.zeros_like(sc["vel"])), "allpairs")
    np.testing.assert_array_equal(one, still)
    moving, _ = orc.rasterize(dict(sc, W=4), "allpairs")
    assert not np.array_equal(one, moving)


def _one_obstacle(nx, ny, robot, goal, p, v, r, W=8, vr=1.0):
    return dict(nx=nx, ny=ny, robot=np.array(robot), goal=np.array(goal), W=W, vr=vr,
                pos=np.array([p], float), vel=np.array([v], float), rad=np.array([r], float))


def test_tangent_disc_is_inclusive(orc):
    sc = _one_obstacle(30, 30, (1, 1), (28, 28), (10.0, 10.0), (0.0, 0.0), 3.0)
    cls, _ = orc.rasterize(sc, "perobs")
    assert cls[10, 13] == 1 and cls[10, 7] == 1 and cls[13, 10] == 1  # distance exactly 3
    assert cls[10, 14] == 0 and cls[7, 10] == 1                        # 4 > 3; 3 on the axis
    assert cls[12, 12] == 1 and cls[12, 13] == 0                       # sqrt(8) < 3 < sqrt(13)
    assert (cls == 1).sum() == 29                                      # lattice points with d <= 3


def test_rounding_tie_goes_to_even(orc):
    # 256 * (10 + 1/512) = 2560.5 -> 2560 (even): centre at x = 10 exactly, so a
    # radius-2 disc reaches x = 8 but not 12 + 1/256 ... checked at both sides.
    for frac, want_q in ((1 / 512, 2560), (3 / 512, 2562)):
        sc = _one_obstacle(30, 30, (1, 1), (28, 28), (10.0 + frac, 15.0), (0.0, 0.0), 2.0)
        cls, _ = orc.rasterize(sc, "allpairs")
        # covered x range on row 15 is [ceil((q - 512)/256), floor((q + 512)/256)]
        xs = np.flatnonzero(cls[15] == 1)
        assert xs.min() == -((512 - want_q) // 256) and xs.max() == (want_q + 512) // 256


def test_occupancy_follows_ring_time(orc):
    # One obstacle moving at 1 cell/step straight at a robot 60 cells away: the
    # ring holding its predicted pose is the one whose horizon matches.
    sc = _one_obstacle(128, 32, (10, 16), (120, 16), (70.0, 16.0), (-1.0, 0.0), 5.0, W=8)
    cls, ring = orc.rasterize(sc, "allpairs")
    occ = np.argwhere(cls == 1)
    assert len(occ) > 0
    for y, x in occ:
        j = ring[y, x]
        mu = 70.0 - 8.0 * j  # position at the ring's horizon
        assert (x - mu) ** 2 + (y - 16) ** 2 <= 25.0
    # meeting point: the obstacle at 70 - t and the ring at 10 + t meet at
    # x = 40; with 8-cell rings the drawn pieces sit at rings 3 and 4
    assert set(ring[cls == 1].tolist()) <= {3, 4}
    assert abs(occ[:, 1].mean() - 42) < 3
    # nothing is drawn at the obstacle's current position
    assert cls[16, 70] == 0
