"""Pins of the paper-literal time-warp modes of the oracle: the elliptical
warp metric (Eqs. 14-15), the per-object horizon of Algorithm 1 and the
covariance inflation of the predicted discs."""
import math

import numpy as np
import pytest

from paper_1903_07441_amd import scenarios


def rx_closed(dx, dy, hc, hs):
    u = hc * dx + hs * dy
    v = hs * dx - hc * dy
    return (-1.8 * u + math.sqrt(4 * u * u + 12.16 * v * v)) / 0.38


def test_ellipse_root_solves_eq15():
    # Eq. (15) with the centre 0.9 r_x ahead: r^2 = (u - 0.9 r)^2 + 16 v^2
    rng = np.random.default_rng(0)
    for _ in range(200):
        dx, dy = rng.integers(-300, 300, size=2)
        th = rng.uniform(0, 2 * math.pi)
        hc, hs = math.cos(th), math.sin(th)
        r = rx_closed(dx, dy, hc, hs)
        u = hc * dx + hs * dy
        v = hs * dx - hc * dy
        assert abs(r * r - ((u - 0.9 * r) ** 2 + 16 * v * v)) <= 1e-9 * max(1.0, r * r)
        # and the point lies on the ellipse of Eq. (14) with r_y = r_x / 4
        if r > 0:
            uc, vc = u - 0.9 * r, v
            assert abs(uc * uc / (r * r) + vc * vc / (r * r / 16) - 1) <= 1e-9


@pytest.mark.parametrize("W", [1, 3, 8])
def test_ellipse_ring_brackets_the_root(orc, W):
    # j W <= r_x < (j + 1) W wherever r_x is not within rounding of a ring edge
    rng = np.random.default_rng(W)
    for _ in range(2000):
        dx, dy = (int(v) for v in rng.integers(-200, 200, size=2))
        th = rng.uniform(0, 2 * math.pi)
        hc, hs = math.cos(th), math.sin(th)
        r = rx_closed(dx, dy, hc, hs)
        j = orc.ring_ellipse(dx, dy, hc, hs, W)
        edge = min(abs(r - j * W), abs(r - (j + 1) * W))
        if edge > 1e-9 * max(1.0, r):
            assert j * W <= r < (j + 1) * W, (dx, dy, th, r, j)


def test_ellipse_ring_special_directions(orc):
    # ahead r_x = d / 1.9, behind 10 d, to the side sqrt(12.16) / 0.38 d
    for d in (5, 19, 38, 101):
        assert orc.ring_ellipse(d, 0, 1.0, 0.0, 1) == math.floor(d / 1.9 + 1e-12)
        assert orc.ring_ellipse(-d, 0, 1.0, 0.0, 1) == 10 * d
        assert orc.ring_ellipse(0, d, 1.0, 0.0, 1) == math.floor(math.sqrt(12.16) / 0.38 * d)
    assert orc.ring_ellipse(0, 0, 1.0, 0.0, 8) == 0


def test_ellipse_ring_rotates_with_the_heading(orc):
    # a quarter turn of the scene and of the heading (exact unit vectors)
    for dx, dy in [(7, -3), (-20, 11), (0, 15), (33, 33)]:
        a = orc.ring_ellipse(dx, dy, 1.0, 0.0, 4)
        assert orc.ring_ellipse(-dy, dx, 0.0, 1.0, 4) == a
        assert orc.ring_ellipse(-dx, -dy, -1.0, 0.0, 4) == a


def test_modes_reduce_to_the_circular_per_cell_map(orc):
    sc = scenarios.scenario("warped512", 4, side=96)
    want_c, want_r = orc.rasterize(sc)
    got_c, got_r = orc.rasterize_modes(sc, ring_mode=0, per_object=False, kappa=0.0)
    assert np.array_equal(got_c, want_c) and np.array_equal(got_r, want_r)


def test_per_object_equals_per_cell_when_nothing_moves(orc):
    sc = scenarios.scenario("warped512", 5, side=96)
    sc["vel"] = np.zeros_like(sc["vel"])
    for mode in (0, 1):
        a, ra = orc.rasterize_modes(sc, ring_mode=mode, heading=(0.6, 0.8), per_object=False)
        b, rb = orc.rasterize_modes(sc, ring_mode=mode, heading=(0.6, 0.8), per_object=True)
        assert np.array_equal(a, b) and np.array_equal(ra, rb)


def test_per_object_disc_at_the_obstacles_own_horizon(orc):
    # one obstacle: its disc is predicted to the horizon of the ring of its
    # current cell and marked on every ring
    sc = dict(nx=80, ny=80, robot=np.array([40, 40]), goal=np.array([2, 2]), W=8, vr=1.0,
              pos=np.array([[60.3, 40.2]]), vel=np.array([[-0.5, 0.25]]), rad=np.array([3.0]))
    cls, ring = orc.rasterize_modes(sc, ring_mode=0, per_object=True)
    j = orc.ring_of(60 - 40, 40 - 40, 8)
    t = j * 8 / 1.0
    mu = sc["pos"][0] + t * sc["vel"][0]
    yy, xx = np.mgrid[0:80, 0:80]
    inside = (256 * xx - np.rint(256 * mu[0])) ** 2 + (256 * yy - np.rint(256 * mu[1])) ** 2 <= (256 * 3) ** 2
    border = (xx == 0) | (yy == 0) | (xx == 79) | (yy == 79)
    want = np.where(inside & ~border, 1, 0)
    got = (cls == orc.OBST).astype(int)
    assert np.array_equal(got, want)


def test_position_covariance_closed_form(orc):
    # the 2x2 position block of A(t) P A(t)^T, A(t) = [[I, tI], [0, I]]
    rng = np.random.default_rng(3)
    for _ in range(20):
        M = rng.standard_normal((4, 4))
        P = M @ M.T
        t = rng.uniform(0, 50)
        A = np.block([[np.eye(2), t * np.eye(2)], [np.zeros((2, 2)), np.eye(2)]])
        Q = A @ P @ A.T
        a, b, d = orc.pos_cov(P, t)
        assert np.allclose([a, b, d], [Q[0, 0], Q[0, 1], Q[1, 1]], rtol=1e-12, atol=1e-12)


def test_inflated_radius(orc):
    P = 0.25 * np.eye(4)
    for t in (0.0, 8.0, 40.0):
        # P(t) = 0.25 (1 + t^2) I: sigma = 0.5 sqrt(1 + t^2), capped at W
        want = 3.0 + min(8.0, 1.5 * 0.5 * math.sqrt(1 + t * t))
        assert orc.inflated_radius(3.0, P, t, 1.5, 8) == pytest.approx(want, rel=1e-15)
    assert orc.inflated_radius(3.0, P, 10.0, 0.0, 8) == 3.0
    assert orc.inflated_radius(3.0, np.zeros((4, 4)), 10.0, 2.0, 8) == 3.0


def test_inflation_grows_the_marked_discs(orc):
    sc = scenarios.scenario("warped512", 6, side=96)
    cov = np.tile(0.25 * np.eye(4), (len(sc["rad"]), 1, 1))
    a, _ = orc.rasterize_modes(sc, kappa=0.0, cov=cov)
    b, _ = orc.rasterize_modes(sc, kappa=1.0, cov=cov)
    assert np.all(b[a == orc.OBST] == orc.OBST)
    assert (b == orc.OBST).sum() > (a == orc.OBST).sum()
