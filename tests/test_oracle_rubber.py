"""Pins of the oracle's rubber band (Eqs. 4-6; the candidate set, the vector
form of F and the update order are readings, see oracle/twg_oracle.c).
Parity unpinned beyond these properties: the band is a heuristic."""
import numpy as np

from paper_1903_07441_amd import scenarios


def boxed(nx, ny):
    cls = np.zeros((ny, nx), np.uint8)
    cls[0, :] = cls[-1, :] = cls[:, 0] = cls[:, -1] = 2
    return cls


def test_zero_tension_keeps_the_path(orc):
    # with k = 0 staying put has a zero resultant, and it is the first candidate
    sc = scenarios.scenario("static64", 3)
    cls, _ = orc.rasterize(sc)
    psi, _ = orc.relax(cls, tol=1e-12)
    st, path = orc.descend(cls, psi, sc["robot"])
    assert st == orc.OK and len(path) > 5
    assert np.array_equal(orc.rubber_band(cls, psi, path, k=0.0, iters=8), path)


def test_tension_straightens_a_bump_on_a_flat_field(orc):
    # equal potentials: F = 0, the tension (0, 2k) pulls the bump back in line
    cls = boxed(10, 10)
    cls[5, 8] = 3
    psi = np.ones((10, 10))
    p = np.array([(1, 5), (2, 5), (3, 4), (4, 5), (5, 5)], np.int32)
    out = orc.rubber_band(cls, psi, p, k=1.0, iters=1)
    assert out.tolist() == [[1, 5], [2, 5], [3, 5], [4, 5], [5, 5]]


def test_potential_force_resists_moving_towards_obstacles(orc):
    # moving the bump at (3,3) down to (3,2) zeroes the tension (|T|^2 = 4k^2
    # before) but costs |1/psi(3,2) - 1/psi(3,3)|^2 of potential force
    cls = boxed(8, 8)
    cls[6, 6] = 3
    psi = np.full((8, 8), 0.5)
    p = np.array([(1, 2), (2, 2), (3, 3), (4, 2), (5, 2)], np.int32)
    psi[2, 3] = 0.01  # 1/0.01 - 1/0.5 = 98: force^2 = 9604 > 4
    assert orc.rubber_band(cls, psi, p, k=1.0, iters=1)[2].tolist() == [3, 3]
    psi[2, 3] = 0.45  # 1/0.45 - 2 = 0.22: force^2 = 0.05 < 4
    assert orc.rubber_band(cls, psi, p, k=1.0, iters=1)[2].tolist() == [3, 2]


def test_band_invariants_on_scenarios(orc):
    for idx in (0, 1, 2, 4):
        sc = scenarios.scenario("static64", idx)
        cls, _ = orc.rasterize(sc)
        psi, _ = orc.relax(cls, tol=1e-12)
        st, path = orc.descend(cls, psi, sc["robot"])
        if st != orc.OK or len(path) < 3:
            continue
        for k in (0.25, 1.0, 4.0):
            out = orc.rubber_band(cls, psi, path, k=k, iters=32)
            assert out.shape == path.shape
            assert np.array_equal(out[0], path[0]) and np.array_equal(out[-1], path[-1])
            c = cls[out[:, 1], out[:, 0]]
            assert np.all((c == orc.FREE) | (c == orc.GOAL))
            assert np.all(np.abs(np.diff(out, axis=0)).max(axis=1) <= 1)
