"""Pins of the oracle's harmonic-field solver against what the mathematics fixes.

Each test would fail for a plausible mistake in the oracle: a dropped
neighbour, a wrong sign, a transposed index, a wrong boundary value, a stop
rule that stops early.  None of them re-types the oracle's own update.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _fixed_border_problem(nx, ny, fn):
    """Border cells FIXED at fn(x, y); interior FREE."""
    cls = np.zeros((ny, nx), np.uint8)
    cls[0, :] = cls[-1, :] = cls[:, 0] = cls[:, -1] = 4
    yy, xx = np.mgrid[0:ny, 0:nx].astype(np.float64)
    exact = fn(xx, yy)
    psi = np.where(cls == 4, exact, 0.3)
    return cls, psi, exact


@pytest.mark.parametrize("name,fn", [
    ("linear", lambda x, y: (x - 0.0) / 40.0),
    ("xy", lambda x, y: (x - 20.0) * (y - 11.0) / 400.0),
    ("x2-y2", lambda x, y: ((x - 20.0) ** 2 - (y - 11.0) ** 2) / 400.0),
])
def test_discrete_harmonic_closed_forms(orc, name, fn):
    # P1: the 5-point average reproduces linear functions, xy and x^2 - y^2
    # exactly, so the converged field equals them up to rounding.
    cls, psi0, exact = _fixed_border_problem(41, 23, fn)
    psi, info = orc.relax(cls, psi0, init=orc.INIT_KEEP, tol=1e-14, check_every=5)
    assert info["status"] == orc.OK
    assert np.max(np.abs(psi - exact)) < 1e-11


def test_corridor_golden(orc):
    # Hand-derived fractions for one-cell-wide corridors (tests/golden/corridor.txt).
    with open(os.path.join(GOLDEN, "corridor.txt")) as fh:
        rows = [ln for ln in fh if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 5
    for ln in rows:
        L, vals = ln.split("|")
        L = int(L)
        want = [float(Fraction(v)) for v in vals.split()]
        nx, ny = L + 2, 3
        cls = np.full((ny, nx), 2, np.uint8)
        cls[1, 1:L + 1] = 0
        cls[1, L + 1] = 3
        psi, info = orc.relax(cls, init=orc.INIT_HALF, tol=1e-15, omega=1.0, check_every=1)
        assert info["status"] == orc.OK
        np.testing.assert_allclose(psi[1, 1:L + 1], want, rtol=0, atol=1e-14)


def _dense_solve(cls, psi_fixed, f=None):
    """Solve (I - J) psi = f on FREE cells with the fixed values elsewhere,
    as a dense linear system assembled from the stencil definition."""
    ny, nx = cls.shape
    free = np.argwhere(cls == 0)
    index = -np.ones((ny, nx), np.int64)
    for k, (y, x) in enumerate(free):
        index[y, x] = k
    n = len(free)
    A = np.zeros((n, n))
    b = np.zeros(n) if f is None else f[cls == 0].astype(np.float64).copy()
    for k, (y, x) in enumerate(free):
        A[k, k] = 1.0
        for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
            yy, xx = y + dy, x + dx
            if not (0 <= yy < ny and 0 <= xx < nx):
                continue  # outside the grid: psi = 0
            if cls[yy, xx] == 0:
                A[k, index[yy, xx]] -= 0.25
            else:
                b[k] += 0.25 * psi_fixed[yy, xx]
    sol = np.linalg.solve(A, b)
    out = psi_fixed.astype(np.float64).copy()
    out[cls == 0] = sol
    return out


def _random_classes(rng, nx, ny, p_obst=0.2, walls=True):
    cls = np.where(rng.uniform(size=(ny, nx)) < p_obst, 1, 0).astype(np.uint8)
    if walls:
        cls[0, :] = cls[-1, :] = cls[:, 0] = cls[:, -1] = 2
    gy, gx = rng.integers(1, ny - 1), rng.integers(1, nx - 1)
    cls[gy, gx] = 3
    return cls


@pytest.mark.parametrize("seed,nx,ny,walls", [(0, 40, 40, True), (1, 23, 37, True),
                                              (2, 17, 9, False), (3, 31, 31, True)])
def test_dense_lu_tiny_grids(orc, seed, nx, ny, walls):
    # P4: dense LAPACK solve of the same linear system.
    rng = np.random.default_rng(seed)
    cls = _random_classes(rng, nx, ny, walls=walls)
    # FIXED cells with arbitrary values exercise the keep-the-input rule
    fixed = (rng.uniform(size=cls.shape) < 0.03) & (cls == 0)
    cls[fixed] = 4
    psi0 = np.where(cls == 4, rng.uniform(size=cls.shape), 0.0)
    psi, info = orc.relax(cls, psi0, init=orc.INIT_HALF, tol=1e-15, max_sweeps=200000)
    assert info["status"] == orc.OK
    ref = _dense_solve(cls, orc.field_init(cls, psi0, orc.INIT_KEEP))
    assert np.max(np.abs(psi - ref)) <= 1e-12


def test_dense_lu_with_source(orc):
    # Source term f (the defect-correction equation): (I - J) e = f on FREE
    # cells with e = 0 on every fixed cell (all fixed cells given as FIXED 0).
    rng = np.random.default_rng(7)
    cls = _random_classes(rng, 25, 19)
    cls0 = np.where(cls == 0, 0, 4).astype(np.uint8)
    f = rng.normal(size=cls.shape) * 1e-3
    zero = np.zeros(cls.shape)
    e, info = orc.relax(cls0, zero, init=orc.INIT_KEEP, f=f, tol=1e-17, max_sweeps=200000)
    assert info["status"] == orc.OK
    ref = _dense_solve(cls0, zero, f=f)
    assert np.max(np.abs(e - ref)) <= 1e-12
    assert np.max(np.abs(ref)) > 1e-3


def test_jacobi_gs_sor_same_fixed_point(orc):
    # Eq. (1) (Jacobi), Eq. (2) (lexicographic Gauss-Seidel) and red-black SOR
    # share the fixed point; only the route differs.
    rng = np.random.default_rng(11)
    cls = _random_classes(rng, 20, 16)
    psi_sor, _ = orc.relax(cls, tol=1e-15)
    a = orc.field_init(cls, None, orc.INIT_HALF)
    b = a.copy()
    for _ in range(6000):
        a = orc.jacobi_step(cls, a)
    for _ in range(3000):
        b = orc.gs_lex_step(cls, b)
    assert np.max(np.abs(a - psi_sor)) < 1e-12
    assert np.max(np.abs(b - psi_sor)) < 1e-12


def test_one_gs_step_is_not_one_jacobi_step(orc):
    # Eq. (2) uses the updated left/upper neighbours: after one step the two
    # forms differ (the "slight distortion" before convergence).
    rng = np.random.default_rng(12)
    cls = _random_classes(rng, 12, 12)
    a = orc.field_init(cls, None, orc.INIT_HALF)
    assert not np.allclose(orc.jacobi_step(cls, a), orc.gs_lex_step(cls, a))


@pytest.mark.parametrize("n", [16, 32, 48])
def test_certificate_bound(orc, n):
    # P3: w = (I - J)^-1 1 on an open square is bounded by the supersolution
    # bound, and |psi - psi*| <= ||r|| * ||w|| holds for partially relaxed fields.
    cls = np.zeros((n, n), np.uint8)
    cls[0, :] = cls[-1, :] = cls[:, 0] = cls[:, -1] = 2
    ones = np.ones((n, n))
    w = _dense_solve(cls, np.zeros((n, n)), f=ones)
    wmax = w.max()
    assert wmax <= orc.wbound(n, n)
    assert 0.25 * (n - 1) ** 2 < wmax  # not vacuous: the bound is within ~2x
    assert orc.wbound(n, n) < 2.5 * wmax
    # partially relaxed field with goal and obstacles
    rng = np.random.default_rng(n)
    cls2 = _random_classes(rng, n, n, p_obst=0.1)
    exact = _dense_solve(cls2, orc.field_init(cls2, None, orc.INIT_KEEP))
    psi = orc.field_init(cls2, None, orc.INIT_HALF)
    for sweeps in (1, 5, 25, 125):
        p = psi.copy()
        for _ in range(sweeps):
            p = orc.sor_sweep(cls2, p, 1.7)
        r = orc.residual(cls2, p)
        err = np.max(np.abs(p - exact))
        assert err <= r * orc.wbound(n, n) * (1 + 1e-12) + 1e-15
        # the sharp constant of this class map is no larger than the open one
        wc = _dense_solve(cls2, np.zeros((n, n)), f=np.ones((n, n))).max()
        assert err <= r * wc * (1 + 1e-9) + 1e-15


def test_relax_stop_rule_and_certificate(orc):
    rng = np.random.default_rng(5)
    cls = _random_classes(rng, 48, 40)
    psi, info = orc.relax(cls, tol=1e-9, tol_cert=1e-8, check_every=3)
    assert info["status"] == orc.OK
    assert info["residual"] <= 1e-9 and info["bound"] <= 1e-8
    assert abs(orc.residual(cls, psi) - info["residual"]) == 0.0
    ref = _dense_solve(cls, orc.field_init(cls, None, orc.INIT_KEEP))
    assert np.max(np.abs(psi - ref)) <= 1e-8
    # a cap that is too small reports NOT_CONVERGED with the partial residual
    _, info2 = orc.relax(cls, tol=1e-9, max_sweeps=7, check_every=3)
    assert info2["status"] == orc.NOT_CONVERGED and info2["sweeps"] == 7
    assert info2["residual"] > 1e-9


def test_residual_definition_matches_jacobi_change(orc):
    # R1: the residual is the change one Jacobi step (Eq. 1) would make.
    rng = np.random.default_rng(9)
    cls = _random_classes(rng, 30, 21)
    psi = orc.field_init(cls, rng.uniform(size=cls.shape), orc.INIT_KEEP)
    step = orc.jacobi_step(cls, psi)
    assert orc.residual(cls, psi) == np.max(np.abs(step - psi)[cls == 0])
    rf = orc.residual_field(cls, psi)
    np.testing.assert_array_equal(rf[cls == 0], (step - psi)[cls == 0])
    assert np.all(rf[cls != 0] == 0)


def _log_annulus(orc, n, r1_frac=0.125, r2_frac=0.45):
    c = (n - 1) / 2.0
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    r = np.hypot(xx - c, yy - c)
    r1, r2 = r1_frac * n, r2_frac * n
    cls = np.zeros((n, n), np.uint8)
    cls[(r <= r1) | (r >= r2)] = 4
    exact = np.log(np.maximum(r, 1e-300) / r1) / np.log(r2 / r1)
    psi0 = np.where(cls == 4, exact, 0.0)
    psi, info = orc.relax(cls, psi0, init=orc.INIT_HALF, tol=1e-13)
    assert info["status"] == orc.OK
    return np.max(np.abs(psi - exact)[cls == 0])


def test_log_annulus_second_order(orc):
    # P2: log r between two concentric circles; the discretisation error falls
    # about 4x each time the grid (and the radii) double: O(h^2).
    e1, e2, e3 = (_log_annulus(orc, n) for n in (32, 64, 128))
    assert e1 < 0.02
    assert 2.8 < e1 / e2 < 5.5, (e1, e2)
    assert 2.8 < e2 / e3 < 5.5, (e2, e3)


def test_maximum_principle_and_descent_everywhere(orc):
    # P5: boundary values bound the field; at convergence every FREE cell that
    # is connected to the goal has a strictly better neighbour (no interior
    # local minimum of phi), and goal-less components converge to phi = 1.
    # Behind long one-cell bottlenecks the exact psi falls by ~4x per cell and
    # drops below any FP64 resolution, so the descent part is asserted where
    # psi exceeds the certified error bound by 1e3.
    rng = np.random.default_rng(21)
    cls = _random_classes(rng, 60, 44, p_obst=0.25)
    psi, info = orc.relax(cls, tol=1e-15, tol_cert=1e-12)
    assert info["status"] == orc.OK
    free = cls == 0
    # the exact field lies in [0, 1]; the iterate is within the certified bound
    assert psi[free].min() >= -info["bound"] and psi[free].max() <= 1.0 + info["bound"]
    idx = orc.index_matrix(cls, psi)
    resolved = 0
    for y, x in np.argwhere(free):
        if orc.goal_reachable(cls, (x, y)):
            if psi[y, x] > 1e3 * info["bound"]:
                resolved += 1
                assert idx[y, x] != 4
                st, path = orc.descend(cls, psi, (x, y))
                assert st == orc.OK and cls[path[-1][1], path[-1][0]] == 3
        else:
            assert abs(psi[y, x]) <= info["bound"]
            st, _ = orc.descend(cls, psi, (x, y))
            assert st == orc.NO_PATH
    assert resolved > 400


def test_random_walk_probability(orc):
    # P6: psi(c) is the probability that a simple random walk from c reaches
    # the goal before any psi = 0 cell (harmonic measure).
    rng = np.random.default_rng(4)
    cls = _random_classes(rng, 10, 9, p_obst=0.15)
    psi, _ = orc.relax(cls, tol=1e-14)
    free = np.argwhere(cls == 0)
    pick = free[rng.choice(len(free), size=4, replace=False)]
    walks = 20000
    moves = np.array([(0, 1), (0, -1), (1, 0), (-1, 0)])
    for y0, x0 in pick:
        pos = np.tile([y0, x0], (walks, 1))
        alive = np.ones(walks, bool)
        hit_goal = np.zeros(walks, bool)
        while alive.any():
            step = moves[rng.integers(0, 4, size=alive.sum())]
            pos[alive] += step
            c = cls[pos[alive, 0], pos[alive, 1]]
            ended = c != 0
            ids = np.flatnonzero(alive)
            hit_goal[ids[ended & (c == 3)]] = True
            alive[ids[ended]] = False
        p = hit_goal.mean()
        se = np.sqrt(max(psi[y0, x0] * (1 - psi[y0, x0]), 1e-4) / walks)
        assert abs(p - psi[y0, x0]) < 2.58 * se + 1e-3


def test_mirror_symmetry(orc):
    # P7: mirroring the class map mirrors the converged field.
    rng = np.random.default_rng(8)
    cls = _random_classes(rng, 33, 26)
    a, _ = orc.relax(cls, tol=1e-14)
    b, _ = orc.relax(cls[:, ::-1].copy(), tol=1e-14)
    c, _ = orc.relax(cls.T.copy(), tol=1e-14)
    assert np.max(np.abs(a[:, ::-1] - b)) < 1e-12
    assert np.max(np.abs(a.T - c)) < 1e-12


def test_outside_grid_counts_as_fixed_zero(orc):
    # Without border walls the outside of the grid acts as psi = 0.
    cls = np.zeros((5, 5), np.uint8)
    cls[2, 2] = 3
    psi, _ = orc.relax(cls, tol=1e-15)
    padded = np.full((7, 7), 2, np.uint8)
    padded[1:6, 1:6] = cls
    psi2, _ = orc.relax(padded, tol=1e-15)
    assert np.max(np.abs(psi - psi2[1:6, 1:6])) < 1e-13


def _plain_red_black_sweep(cls, psi, omega, f=None, order=(0, 1)):
    """One red-black SOR sweep written from Eqs. (1)-(2) as plainly as NumPy
    allows: red cells ((x + y) even) first, then black, each FREE cell set to
    psi + omega * (mean of its four neighbours + f - psi), neighbours outside
    the grid counting as psi = 0.  Whole-array arithmetic, NumPy's own
    evaluation order, no fused operations."""
    ny, nx = cls.shape
    psi = psi.copy()
    yy, xx = np.mgrid[0:ny, 0:nx]
    for colour in order:
        p = np.pad(psi, 1)
        avg = (p[1:-1, 2:] + p[1:-1, :-2] + p[2:, 1:-1] + p[:-2, 1:-1]) / 4.0
        if f is not None:
            avg = avg + f
        new = psi + omega * (avg - psi)
        sel = (cls == 0) & (((xx + yy) % 2) == colour)
        psi[sel] = new[sel]
    return psi


@pytest.mark.parametrize("omega", [1.0, 1.5, 1.95])
@pytest.mark.parametrize("with_source", [False, True])
def test_sor_sweep_equals_plain_update_within_rounding(orc, omega, with_source):
    # R2: the oracle's sweep evaluates the update as
    # fma(omega, fma(1/4, ((E+W)+N)+S, f - psi), psi); the paper fixes the
    # update (Eqs. 1-2), not its evaluation order.  Against the plain form,
    # one sweep may differ only by rounding: on values in [0, 1] a handful of
    # unit roundoffs per half-sweep, growing at most linearly over sweeps
    # (the sweep is non-expansive in the max norm for omega <= 2 on these
    # fields' scale).  A wrong colour order, a dropped neighbour, a wrong
    # factor or a wrong sign differs by orders of magnitude more.
    rng = np.random.default_rng(int(omega * 100) + with_source)
    ny, nx = 37, 52
    cls = np.where(rng.uniform(size=(ny, nx)) < 0.15, 1, 0).astype(np.uint8)
    cls[0, :] = cls[-1, :] = cls[:, 0] = cls[:, -1] = 2
    cls[rng.uniform(size=(ny, nx)) < 0.03] = 4
    cls[10, 20] = 3
    psi0 = orc.field_init(cls, rng.uniform(size=(ny, nx)), orc.INIT_KEEP)
    f = rng.normal(size=(ny, nx)) * 1e-3 if with_source else None
    eps = np.finfo(np.float64).eps
    a, b = psi0.copy(), psi0.copy()
    for k in range(1, 11):
        a = orc.sor_sweep(cls, a, omega, f=f)
        b = _plain_red_black_sweep(cls, b, omega, f=f)
        assert np.max(np.abs(a - b)) <= 16 * k * eps, (k, np.max(np.abs(a - b)))
    # the pin has teeth: black first, or a factor off by one part in 10^4,
    # differs by far more than rounding
    black_first = _plain_red_black_sweep(cls, psi0, omega, f=f, order=(1, 0))
    other_factor = _plain_red_black_sweep(cls, psi0, omega * (1 + 1e-4), f=f)
    one = orc.sor_sweep(cls, psi0, omega, f=f)
    assert np.max(np.abs(one - black_first)) > 1e-3
    assert np.max(np.abs(one - other_factor)) > 1e3 * eps


def _tie_grid(values):
    """3 x 3 FREE block inside walls (5 x 5): the centre (2, 2) at psi 0.1,
    its E, W, S, N neighbours at the given psi values, every other cell a
    wall."""
    cls = np.full((5, 5), 2, np.uint8)
    psi = np.zeros((5, 5))
    cls[2, 2] = 0
    psi[2, 2] = 0.1
    for (dx, dy), v in zip(((1, 0), (-1, 0), (0, 1), (0, -1)), values):
        cls[2 + dy, 2 + dx] = 0
        psi[2 + dy, 2 + dx] = v
    return cls, psi


@pytest.mark.parametrize("values,want", [
    ((0.7, 0.7, 0.7, 0.7), 0),      # all four tie: E
    ((0.3, 0.7, 0.7, 0.7), 1),      # W, S, N tie: W
    ((0.3, 0.2, 0.7, 0.7), 2),      # S, N tie: S
    ((0.3, 0.2, 0.1, 0.7), 3),      # N alone
    ((0.7, 0.3, 0.2, 0.7), 0),      # E and N tie: E
    ((0.3, 0.7, 0.2, 0.7), 1),      # W and N tie: W
    ((0.1, 0.1, 0.1, 0.1), 4),      # no neighbour strictly better: no move
    ((0.1, 0.1, 0.1, 0.100001), 3),
])
def test_index_tie_break_order(orc, values, want):
    # R10 (Eq. 3 is garbled): among the neighbours with the highest psi the
    # first in the order E, W, S, N wins; a move needs a strictly higher psi.
    # Exact ties, hand-built, so any other order or a non-strict test fails.
    cls, psi = _tie_grid(values)
    assert orc.index_matrix(cls, psi)[2, 2] == want
    # the walk takes the same first step
    cls2 = cls.copy()
    if want != 4:
        dx, dy = ((1, 0), (-1, 0), (0, 1), (0, -1))[want]
        cls2[2 + dy, 2 + dx] = 3  # the chosen neighbour is the goal
        status, path = orc.descend(cls2, psi, (2, 2))
        assert status == orc.OK and path.tolist() == [[2, 2], [2 + dx, 2 + dy]]


def test_linear_ramp_init(orc):
    # the linear-ramp start: 1 at the goal, falling with the Euclidean
    # distance d to the goal as 1 - d / (max(nx, ny) sqrt 2), so it stays in
    # (0, 1] on the grid; fixed cells take their Dirichlet values
    ny, nx = 9, 13
    cls = np.zeros((ny, nx), np.uint8)
    cls[0, :] = 2
    cls[4, 6] = 1
    cls[2, 3] = 3
    psi = orc.field_init(cls, None, orc.INIT_LINEAR, goal=(3, 2))
    span = 13 * np.sqrt(2.0)
    assert psi[2, 3] == 1.0 and psi[4, 6] == 0.0 and np.all(psi[0] == 0.0)
    assert psi[2, 4] == 1.0 - 1.0 / span and psi[5, 7] == 1.0 - 5.0 / span  # 3-4-5 triangle
    assert psi[8, 12] == 1.0 - np.sqrt(81 + 36) / span
    free = cls == 0
    assert np.all((psi[free] > 0) & (psi[free] < 1))
