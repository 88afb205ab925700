"""Seeded synthetic scenarios for the time-warped harmonic-field path.

This module only draws random numbers (NumPy PCG64); it holds none of the
method's arithmetic (no rings, no prediction, no rasterisation, no field).
Both the HIP path and the CPU oracle take their inputs from here.

Units: cells for lengths, steps for time.  Scenario recipes:

* ``static64``    64x64, 10 discs, radius U[2,5], velocity 0.
* ``warped512``   512x512, 50 discs, radius U[3,8], velocity N(0, 0.5^2)
                  per axis, covariance 0.25 I4, ring width 8, robot speed 1.
* ``batch``       one grid of a batch: side uniform over {64,...,1024},
                  obstacle count U{10..200}, radius U[2,5], velocity as above.
* ``learn256``    256x256 training field: count U{10..200}, radius U[2,5]
                  with a 25 % share U[3,12], velocity as above.
* ``replan2048``  2048x2048, 500 discs, radius U[3,12], velocity as above.

Obstacle centres are uniform over the grid; the robot start and the goal are
uniform over the interior (one cell inside the border).  Discs whose current
position would cover the start are redrawn, so that the robot does not start
inside an obstacle.  ``reachable`` redraws the goal, from a stream of its
own, until a caller-supplied test (which rasterises the map) finds it
4-connected to the start; the number of redraws is recorded.
"""
from __future__ import annotations

import numpy as np

RECIPES = {
    "static64": dict(n=64, n_obs=(10, 10), rad=((2.0, 5.0), 0.0, None), vel_sigma=0.0),
    "warped512": dict(n=512, n_obs=(50, 50), rad=((3.0, 8.0), 0.0, None), vel_sigma=0.5),
    "learn256": dict(n=256, n_obs=(10, 200), rad=((2.0, 5.0), 0.25, (3.0, 12.0)), vel_sigma=0.5),
    "replan2048": dict(n=2048, n_obs=(500, 500), rad=((3.0, 12.0), 0.0, None), vel_sigma=0.5),
}
BATCH_SIDES = (64, 128, 256, 512, 1024)
SEED_BASE = {"static64": 1000, "warped512": 2000, "batch": 3000, "learn256": 4000,
             "replan2048": 5000}


def _cell(rng, n):
    """A coordinate one cell inside the border, or anywhere on grids too
    narrow to have an inside."""
    return int(rng.integers(1, n - 1)) if n >= 3 else int(rng.integers(0, n))


def _draw(rng, nx, ny, n_obs, rad_spec, vel_sigma, W=8, vr=1.0):
    (lo, hi), share, alt = rad_spec
    robot = np.array([_cell(rng, nx), _cell(rng, ny)], dtype=np.int32)
    goal = np.array([_cell(rng, nx), _cell(rng, ny)], dtype=np.int32)
    for _ in range(64):  # tiny grids may have a single candidate cell
        if goal[0] != robot[0] or goal[1] != robot[1]:
            break
        goal = np.array([_cell(rng, nx), _cell(rng, ny)], dtype=np.int32)
    pos = np.empty((n_obs, 2))
    rad = np.empty(n_obs)
    for i in range(n_obs):
        for _ in range(100):  # bounded: on tiny grids the start may end up covered
            p = np.array([rng.uniform(0, nx), rng.uniform(0, ny)])
            if alt is not None and rng.uniform() < share:
                r = rng.uniform(*alt)
            else:
                r = rng.uniform(lo, hi)
            if np.hypot(p[0] - robot[0], p[1] - robot[1]) > r + 1.5:
                break
        pos[i], rad[i] = p, r
    vel = rng.normal(0.0, vel_sigma, size=(n_obs, 2)) if vel_sigma > 0 else np.zeros((n_obs, 2))
    cov = np.tile(0.25 * np.eye(4), (n_obs, 1, 1))
    return dict(nx=int(nx), ny=int(ny), robot=robot, goal=goal, W=int(W), vr=float(vr),
                pos=pos, vel=vel, rad=rad, cov=cov)


def _goal_draw(seed, k, nx, ny, robot):
    """The k-th redrawn goal (k >= 1) of a scenario: uniform over the
    interior, never the robot cell, from a stream keyed by the scenario
    seed alone (so redraws never change the obstacles)."""
    rng = np.random.default_rng([int(seed), 0x60A1])
    goal = None
    for _ in range(k):
        for _ in range(64):
            goal = np.array([_cell(rng, nx), _cell(rng, ny)], dtype=np.int32)
            if goal[0] != robot[0] or goal[1] != robot[1]:
                break
    return goal


def scenario(name: str, index: int = 0, seed: int | None = None, side: int | None = None,
             goal_draw: int = 0):
    """One scenario dict: nx, ny, robot[2], goal[2], W, vr, pos[n,2],
    vel[n,2], rad[n], cov[n,4,4], seed, name, goal_draw.  goal_draw = k > 0
    replaces the goal by the k-th redraw."""
    if seed is None:
        seed = SEED_BASE[name] + index
    rng = np.random.default_rng(seed)
    if name == "batch":
        n = int(side) if side is not None else int(rng.choice(BATCH_SIDES))
        n_obs = int(rng.integers(10, 201))
        sc = _draw(rng, n, n, n_obs, ((2.0, 5.0), 0.0, None), 0.5)
    else:
        rec = RECIPES[name]
        n = int(side) if side is not None else rec["n"]
        lo, hi = rec["n_obs"]
        n_obs = lo if lo == hi else int(rng.integers(lo, hi + 1))
        sc = _draw(rng, n, n, n_obs, rec["rad"], rec["vel_sigma"])
    if goal_draw:
        sc["goal"] = _goal_draw(seed, goal_draw, sc["nx"], sc["ny"], sc["robot"])
    sc["seed"] = int(seed)
    sc["name"] = name
    sc["goal_draw"] = int(goal_draw)
    return sc


def reachable(name: str, index: int = 0, is_reachable=None, seed: int | None = None,
              side: int | None = None, max_draws: int = 256):
    """The scenario with its goal redrawn until ``is_reachable(sc)`` holds
    (the caller rasterises the map and tests 4-connectivity of start and
    goal); sc["goal_draw"] counts the redraws.  Raises RuntimeError after
    max_draws."""
    for k in range(max_draws + 1):
        sc = scenario(name, index, seed=seed, side=side, goal_draw=k)
        if is_reachable(sc):
            return sc
    raise RuntimeError(f"no reachable goal in {max_draws} draws for {name}[{index}]")


def batch(n_grids: int = 256, seed: int = 3000, is_reachable=None):
    """The uneven batch: grid k uses seed + k; with is_reachable, each goal
    is redrawn until reachable (see ``reachable``)."""
    if is_reachable is None:
        return [scenario("batch", seed=seed + k) for k in range(n_grids)]
    return [reachable("batch", seed=seed + k, is_reachable=is_reachable) for k in range(n_grids)]


def custom(nx, ny, n_obs, rad=(2.0, 5.0), vel_sigma=0.5, seed=0, W=8, vr=1.0):
    rng = np.random.default_rng(seed)
    sc = _draw(rng, nx, ny, n_obs, (rad, 0.0, None), vel_sigma, W=W, vr=vr)
    sc["seed"] = int(seed)
    sc["name"] = "custom"
    return sc
