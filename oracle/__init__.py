"""FP64 CPU oracle for the harmonic-potential-field path on the time-warped grid.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the product library never imports, links or calls
anything here.  It shares no code with the HIP path.

The arithmetic lives in ``twg_oracle.c`` (plain C, FP64, contraction off);
this module compiles it with gcc and wraps it with ctypes over contiguous
NumPy arrays.  The learned warm start's reference network is in ``unet.py``.

Conventions: arrays are indexed ``a[y, x]`` (row-major, x fastest); the field
is ``psi = 1 - phi`` (goal 1, obstacles 0); cell classes FREE 0, OBST 1,
WALL 2, GOAL 3, FIXED 4.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "twg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FREE, OBST, WALL, GOAL, FIXED = 0, 1, 2, 3, 4
OK, NOT_CONVERGED, NO_PATH, START_BLOCKED, PATH_TRUNCATED = 0, 1, 2, 3, 5

_lib = None


def build(force: bool = True) -> str:
    """Compile twg_oracle.c into liboracle.so next to it."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"  # one per process: parallel test workers may build at once
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    i32, i64, f64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    sig = {
        "orc_isqrt": (ctypes.c_uint64, [ctypes.c_uint64]),
        "orc_ring_of": (i32, [i64, i64, i32]),
        "orc_ring_map": (None, [i32, i32, i32, i32, i32, p]),
        "orc_num_rings": (i32, [i32, i32, i32, i32, i32]),
        "orc_ring_time": (f64, [i32, i32, f64]),
        "orc_predict_mean": (None, [p, p, f64, p]),
        "orc_kalman_predict_steps": (None, [p, p, f64, i32, p]),
        "orc_kalman_update": (None, [p, p, p, p]),
        "orc_rasterize_allpairs": (None, [i32, i32, i32, i32, i32, i32, i32, f64, i32, i32,
                                          p, p, p, p, p, p]),
        "orc_rasterize_perobs": (None, [i32, i32, i32, i32, i32, i32, i32, f64, i32, i32,
                                        p, p, p, p, p, p]),
        "orc_field_init": (None, [i32, i32, p, p, i32, i32, i32]),
        "orc_residual": (f64, [i32, i32, p, p, p]),
        "orc_residual_field": (None, [i32, i32, p, p, p, p]),
        "orc_sor_sweep": (None, [i32, i32, p, p, p, f64]),
        "orc_jacobi_step": (None, [i32, i32, p, p]),
        "orc_gs_lex_step": (None, [i32, i32, p, p]),
        "orc_wbound": (f64, [i32, i32]),
        "orc_relax": (i32, [i32, i32, p, p, p, f64, f64, f64, i64, i32, p]),
        "orc_index_of": (i32, [i32, i32, p, p, i32, i32]),
        "orc_index_matrix": (None, [i32, i32, p, p, p]),
        "orc_descend": (i32, [i32, i32, p, p, i32, i32, i32, p, p]),
        "orc_goal_reachable": (i32, [i32, i32, p, i32, i32]),
        "orc_rubber_band": (None, [i32, i32, p, p, p, i32, f64, i32]),
        "orc_ring_ellipse": (i32, [i64, i64, f64, f64, i32]),
        "orc_ring_map_mode": (None, [i32, i32, i32, i32, i32, i32, f64, f64, p]),
        "orc_pos_cov": (None, [p, f64, p]),
        "orc_inflated_radius": (f64, [f64, p, f64, f64, i32]),
        "orc_rasterize_modes": (None, [i32, i32, i32, i32, i32, i32, i32, f64, i32, i32, p, p, p, p,
                                       i32, f64, f64, i32, f64, p, p, p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


# --------------------------------------------------------------------------
# Time rings and prediction
# --------------------------------------------------------------------------

def isqrt(n: int) -> int:
    return int(_load().orc_isqrt(int(n)))


def ring_of(dx: int, dy: int, W: int) -> int:
    return int(_load().orc_ring_of(int(dx), int(dy), int(W)))


def ring_map(nx, ny, robot, W):
    out = np.empty((ny, nx), dtype=np.uint16)
    _load().orc_ring_map(nx, ny, int(robot[0]), int(robot[1]), int(W), _ptr(out))
    return out


def num_rings(nx, ny, robot, W) -> int:
    return int(_load().orc_num_rings(nx, ny, int(robot[0]), int(robot[1]), int(W)))


def ring_time(j, W, vr) -> float:
    return float(_load().orc_ring_time(int(j), int(W), float(vr)))


def predict_mean(p, v, t):
    p, v = _f64(p), _f64(v)
    mu = np.empty(2)
    _load().orc_predict_mean(_ptr(p), _ptr(v), float(t), _ptr(mu))
    return mu


def kalman_predict_steps(x, P, dt, steps, Q=None):
    x = _f64(x).copy()
    P = _f64(P).reshape(4, 4).copy()
    Qa = None if Q is None else _f64(Q).reshape(4, 4)
    _load().orc_kalman_predict_steps(_ptr(x), _ptr(P), float(dt), int(steps), _ptr(Qa))
    return x, P


def kalman_update(x, P, z, R):
    x = _f64(x).copy()
    P = _f64(P).reshape(4, 4).copy()
    z, R = _f64(z), _f64(R).reshape(2, 2)
    _load().orc_kalman_update(_ptr(x), _ptr(P), _ptr(z), _ptr(R))
    return x, P


def rasterize(sc, method="perobs", static_occ=None, border_walls=True):
    """Class map (uint8) and ring map (uint16) of a scenario.

    ``sc`` needs nx, ny, robot, goal, W, vr, pos (n,2), vel (n,2), rad (n,).
    ``method`` is "perobs" (per obstacle and ring) or "allpairs" (per cell).
    """
    nx, ny = int(sc["nx"]), int(sc["ny"])
    pos, vel, rad = _f64(sc["pos"]).reshape(-1, 2), _f64(sc["vel"]).reshape(-1, 2), _f64(sc["rad"])
    n = rad.shape[0]
    cls = np.empty((ny, nx), dtype=np.uint8)
    ring = np.empty((ny, nx), dtype=np.uint16)
    so = None if static_occ is None else _u8(static_occ)
    fn = _load().orc_rasterize_perobs if method == "perobs" else _load().orc_rasterize_allpairs
    fn(nx, ny, int(sc["robot"][0]), int(sc["robot"][1]), int(sc["goal"][0]), int(sc["goal"][1]),
       int(sc["W"]), float(sc["vr"]), int(bool(border_walls)), n,
       _ptr(pos), _ptr(vel), _ptr(rad), _ptr(so), _ptr(cls), _ptr(ring))
    return cls, ring


# --------------------------------------------------------------------------
# Field
# --------------------------------------------------------------------------

INIT_KEEP, INIT_HALF, INIT_ZERO, INIT_LINEAR = 0, 1, 2, 3


def field_init(cls, psi=None, mode=INIT_HALF, goal=(0, 0)):
    """Initial field (goal: the goal cell (x, y) of INIT_LINEAR)."""
    cls = _u8(cls)
    ny, nx = cls.shape
    out = np.zeros((ny, nx)) if psi is None else _f64(psi).copy()
    _load().orc_field_init(nx, ny, _ptr(cls), _ptr(out), int(mode), int(goal[0]), int(goal[1]))
    return out


def residual(cls, psi, f=None) -> float:
    cls, psi = _u8(cls), _f64(psi)
    ny, nx = cls.shape
    fa = None if f is None else _f64(f)
    return float(_load().orc_residual(nx, ny, _ptr(cls), _ptr(psi), _ptr(fa)))


def residual_field(cls, psi, f=None):
    cls, psi = _u8(cls), _f64(psi)
    ny, nx = cls.shape
    fa = None if f is None else _f64(f)
    r = np.empty((ny, nx))
    _load().orc_residual_field(nx, ny, _ptr(cls), _ptr(psi), _ptr(fa), _ptr(r))
    return r


def sor_sweep(cls, psi, omega, f=None):
    cls = _u8(cls)
    out = _f64(psi).copy()
    ny, nx = cls.shape
    fa = None if f is None else _f64(f)
    _load().orc_sor_sweep(nx, ny, _ptr(cls), _ptr(out), _ptr(fa), float(omega))
    return out


def jacobi_step(cls, psi):
    cls = _u8(cls)
    out = _f64(psi).copy()
    ny, nx = cls.shape
    _load().orc_jacobi_step(nx, ny, _ptr(cls), _ptr(out))
    return out


def gs_lex_step(cls, psi):
    cls = _u8(cls)
    out = _f64(psi).copy()
    ny, nx = cls.shape
    _load().orc_gs_lex_step(nx, ny, _ptr(cls), _ptr(out))
    return out


def wbound(nx, ny) -> float:
    return float(_load().orc_wbound(int(nx), int(ny)))


def omega_open(nx, ny) -> float:
    """SOR parameter that is optimal for the open rectangle: the Jacobi
    spectral radius of the 5-point average on an nx-by-ny grid with fixed
    outside values is (cos(pi/(nx+1)) + cos(pi/(ny+1)))/2, and Young's
    formula gives omega = 2 / (1 + sqrt(1 - rho^2))."""
    rho = 0.5 * (np.cos(np.pi / (nx + 1)) + np.cos(np.pi / (ny + 1)))
    return float(2.0 / (1.0 + np.sqrt(1.0 - rho * rho)))


def relax(cls, psi=None, init=INIT_HALF, omega=None, tol=1e-9, tol_cert=0.0,
          max_sweeps=10_000_000, check_every=10, f=None, goal=(0, 0)):
    """Red-black SOR in FP64 until ||r||inf <= tol and r * wbound <= tol_cert.

    Returns (psi, info) with info = dict(status, sweeps, residual, bound).
    """
    cls = _u8(cls)
    ny, nx = cls.shape
    out = field_init(cls, psi, init, goal)
    if omega is None:
        omega = omega_open(nx, ny)
    fa = None if f is None else _f64(f)
    info = np.zeros(3)
    st = _load().orc_relax(nx, ny, _ptr(cls), _ptr(out), _ptr(fa), float(omega), float(tol),
                           float(tol_cert), int(max_sweeps), int(check_every), _ptr(info))
    return out, dict(status=int(st), sweeps=int(info[0]), residual=float(info[1]),
                     bound=float(info[2]))


# --------------------------------------------------------------------------
# Descent
# --------------------------------------------------------------------------

def index_matrix(cls, psi):
    cls, psi = _u8(cls), _f64(psi)
    ny, nx = cls.shape
    out = np.empty((ny, nx), dtype=np.uint8)
    _load().orc_index_matrix(nx, ny, _ptr(cls), _ptr(psi), _ptr(out))
    return out


def descend(cls, psi, start, cap=None):
    """Steepest-descent walk; returns (status, path (len, 2) int32 [x, y])."""
    cls, psi = _u8(cls), _f64(psi)
    ny, nx = cls.shape
    if cap is None:
        cap = nx * ny
    path = np.zeros((max(cap, 1), 2), dtype=np.int32)
    n = ctypes.c_int32(0)
    st = _load().orc_descend(nx, ny, _ptr(cls), _ptr(psi), int(start[0]), int(start[1]),
                             int(cap), _ptr(path), ctypes.byref(n))
    return int(st), path[: n.value].copy()


def goal_reachable(cls, start) -> bool:
    cls = _u8(cls)
    ny, nx = cls.shape
    return bool(_load().orc_goal_reachable(nx, ny, _ptr(cls), int(start[0]), int(start[1])))


def rubber_band(cls, psi, path, k=1.0, iters=16):
    """Rubber-band smoothing of a path (Eqs. 4-6, reading in twg_oracle.c);
    returns the new (n, 2) int32 path [x, y]."""
    cls, psi = _u8(cls), _f64(psi)
    ny, nx = cls.shape
    out = np.ascontiguousarray(np.asarray(path, dtype=np.int32).reshape(-1, 2)).copy()
    _load().orc_rubber_band(nx, ny, _ptr(cls), _ptr(psi), _ptr(out), int(out.shape[0]), float(k), int(iters))
    return out


def ring_ellipse(dx, dy, hc, hs, W):
    """Elliptical warp ring of the cell at offset (dx, dy) from the robot."""
    return int(_load().orc_ring_ellipse(int(dx), int(dy), float(hc), float(hs), int(W)))


def pos_cov(P, t):
    """[a, b, d] of the 2x2 position covariance after horizon t."""
    P = _f64(np.asarray(P, dtype=np.float64).reshape(16))
    out = np.zeros(3)
    _load().orc_pos_cov(_ptr(P), float(t), _ptr(out))
    return out


def inflated_radius(r, P, t, kappa, W):
    P = None if P is None else _f64(np.asarray(P, dtype=np.float64).reshape(16))
    return float(_load().orc_inflated_radius(float(r), _ptr(P) if P is not None else None, float(t),
                                             float(kappa), int(W)))


def rasterize_modes(sc, ring_mode=0, heading=(1.0, 0.0), per_object=False, kappa=0.0, cov=None,
                    static_occ=None, border_walls=True):
    """Class and ring maps with the warp metric, horizon rule and covariance
    inflation chosen (see orc_rasterize_modes)."""
    nx, ny = int(sc["nx"]), int(sc["ny"])
    pos = _f64(np.asarray(sc["pos"], dtype=np.float64).reshape(-1, 2))
    vel = _f64(np.asarray(sc["vel"], dtype=np.float64).reshape(-1, 2))
    rad = _f64(np.asarray(sc["rad"], dtype=np.float64).reshape(-1))
    n = rad.shape[0]
    cv = None if cov is None else _f64(np.asarray(cov, dtype=np.float64).reshape(n, 16))
    so = None if static_occ is None else _u8(static_occ)
    cls = np.zeros((ny, nx), np.uint8)
    ring = np.zeros((ny, nx), np.uint16)
    _load().orc_rasterize_modes(nx, ny, int(sc["robot"][0]), int(sc["robot"][1]), int(sc["goal"][0]),
                                int(sc["goal"][1]), int(sc["W"]), float(sc["vr"]), int(bool(border_walls)), n,
                                _ptr(pos), _ptr(vel), _ptr(rad), _ptr(so) if so is not None else None,
                                int(ring_mode), float(heading[0]), float(heading[1]), int(bool(per_object)),
                                float(kappa), _ptr(cv) if cv is not None else None, _ptr(cls), _ptr(ring))
    return cls, ring
