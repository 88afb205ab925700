"""ctypes binding of libtwg.so (C ABI in include/twg.h).

Argument marshalling only: torch supplies device memory and the current HIP
stream; every step of the computation runs in the library's HIP kernels.
Importing this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtwg.so")

OK, NOT_CONVERGED, NO_PATH, START_BLOCKED, NET_FALLBACK, PATH_TRUNCATED = 0, 1, 2, 3, 4, 5
EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED = -1, -2, -3, -4
FREE, OBST, WALL, GOAL, FIXED = 0, 1, 2, 3, 4
INIT_KEEP, INIT_HALF, INIT_ZERO, INIT_LINEAR = 0, 1, 2, 3
GRID_LDS = 1  # twg_grid_desc.flags

i32, i64, f32, f64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double, ctypes.c_void_p


class Grid(ctypes.Structure):
    _fields_ = [("nx", i32), ("ny", i32), ("pitch", i32)]


class RasterParams(ctypes.Structure):
    _fields_ = [("robot_x", i32), ("robot_y", i32), ("goal_x", i32), ("goal_y", i32),
                ("ring_width", i32), ("border_walls", i32), ("robot_speed", f64),
                ("ring_mode", i32), ("per_object", i32), ("heading_x", f64), ("heading_y", f64),
                ("kappa", f64), ("cov", vp)]


class HpfParams(ctypes.Structure):
    _fields_ = [("tol", f64), ("tol_cert", f64), ("max_sweeps", i64), ("omega", f32),
                ("init", i32), ("polish", i32), ("sweeps_per_pass", i32), ("check_passes", i32),
                ("rows_per_tile", i32), ("goal_x", i32), ("goal_y", i32)]


class HpfStats(ctypes.Structure):
    _fields_ = [("sweeps", i64), ("polish_sweeps", i64), ("residual", f64), ("residual32", f64),
                ("cert_bound", f64), ("wbound", f64), ("omega", f32), ("status", i32),
                ("polish_rounds", i32), ("checks", i32), ("residual_rel", f64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


STATS_BYTES = ctypes.sizeof(HpfStats)


def stats_from_device(t):
    """hpf_stats dict from a device tensor written by relax_async (copies to the host, which
    waits for the stream)."""
    raw = bytes(t[:STATS_BYTES].cpu().numpy().tobytes())
    return HpfStats.from_buffer_copy(raw).as_dict()


def batch_stats_from_device(t, n):
    """hpf_stats dicts of a batch from a device tensor written by
    relax_batched(slots=...) (copies to the host, which waits for the stream)."""
    raw = bytes(t[:n * STATS_BYTES].cpu().numpy().tobytes())
    return [HpfStats.from_buffer_copy(raw[k * STATS_BYTES:(k + 1) * STATS_BYTES]).as_dict() for k in range(n)]


class GridDesc(ctypes.Structure):
    _fields_ = [("nx", i32), ("ny", i32), ("pitch", i32), ("flags", i32), ("offset", i64)]


class DescendParams(ctypes.Structure):
    _fields_ = [("start_x", i32), ("start_y", i32), ("cap", i32), ("reserved", i32)]


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_1903_07441_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    sigs = {
        "twg_version": (i32, []),
        "twg_ctx_create": (i32, [P(vp), i32]),
        "twg_ctx_destroy": (i32, [vp]),
        "twg_last_error": (ctypes.c_char_p, [vp]),
        "twg_ctx_set_graphs": (i32, [vp, i32]),
        "twg_rasterize": (i32, [vp, Grid, i32, vp, vp, vp, vp, P(RasterParams), vp, vp, vp]),
        "hpf_relax": (i32, [vp, Grid, vp, vp, vp, P(HpfParams), P(HpfStats), vp]),
        "hpf_relax_async": (i32, [vp, Grid, vp, vp, vp, P(HpfParams), i32, vp, vp]),
        "hpf_relax_async_noalloc": (i32, [vp, Grid, vp, vp, vp, P(HpfParams), i32, vp, vp]),
        "hpf_sweeps": (i32, [vp, Grid, vp, vp, vp, f32, i32, i32, i32, vp]),
        "hpf_relax_batched": (i32, [vp, i32, vp, vp, vp, P(HpfParams), vp, vp]),
        "hpf_relax_batched_async": (i32, [vp, i32, vp, vp, vp, vp, i32, vp, vp]),
        "hpf_residual": (i32, [vp, Grid, vp, vp, vp, vp, P(f64), vp]),
        "hpf_autotune": (i32, [vp, Grid, vp, vp, vp]),
        "hpf_autotune_batched": (i32, [vp, i32, vp, vp, vp, vp]),
        "hpf_sweeps64": (i32, [vp, Grid, vp, vp, f64, i32, i32, i32, vp]),
        "hpf_index_matrix": (i32, [vp, Grid, vp, vp, vp, vp, vp]),
        "hpf_descend": (i32, [vp, Grid, vp, vp, vp, P(DescendParams), vp, vp, vp]),
        "hpf_rubber_band": (i32, [vp, Grid, vp, vp, vp, vp, vp, i32, f64, i32, vp]),
        "hpf_merge_previous": (i32, [vp, Grid, vp, vp, vp, vp, vp]),
        "hpf_init_field": (i32, [vp, Grid, vp, vp, i32, i32, i32, vp]),
        "hpf_set_tiling": (i32, [vp, i32, i32, i32, i32, f32, i32, i32]),
        "twg_kalman_step": (i32, [vp, i32, vp, vp, vp, f64, vp, vp, vp, vp, vp]),
        "hpf_descent_all": (i32, [vp, Grid, vp, vp, vp, vp, i32, vp]),
        "twg_unet_num_params": (i32, []),
        "twg_unet_create": (i32, [vp, P(vp)]),
        "twg_unet_destroy": (i32, [vp]),
        "twg_unet_set_params": (i32, [vp, vp, vp]),
        "twg_unet_get_params": (i32, [vp, vp, vp]),
        "twg_unet_forward": (i32, [vp, i32, i32, i32, vp, vp, vp]),
        "twg_unet_loss_grad": (i32, [vp, i32, i32, i32, vp, vp, vp, vp, vp, vp]),
        "twg_unet_adam_step": (i32, [vp, f32, vp]),
        "twg_unet_features": (i32, [vp, Grid, vp, vp, i32, i32, i32, i32, vp, vp]),
        "twg_unet_warm_start": (i32, [vp, Grid, vp, vp, i32, i32, vp, vp, vp]),
        "twg_unet_coarse_frame": (i32, [Grid, i32, P(i32), P(i32)]),
        "twg_unet_features_coarse": (i32, [vp, Grid, vp, vp, i32, i32, i32, vp, vp, vp]),
        "twg_unet_coarse_target": (i32, [vp, Grid, vp, vp, i32, vp, vp]),
        "twg_unet_warm_start_coarse": (i32, [vp, Grid, vp, vp, i32, i32, i32, vp, vp, vp]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()
EXPORTED = ("twg_version", "twg_ctx_create", "twg_ctx_destroy", "twg_last_error", "twg_ctx_set_graphs",
            "twg_rasterize",
            "hpf_relax", "hpf_relax_async", "hpf_relax_async_noalloc", "hpf_relax_batched",
            "hpf_relax_batched_async", "hpf_sweeps", "hpf_sweeps64", "hpf_residual", "hpf_autotune",
            "hpf_autotune_batched",
            "hpf_index_matrix", "hpf_descend", "hpf_rubber_band", "hpf_merge_previous",
            "hpf_init_field", "hpf_set_tiling", "twg_kalman_step", "hpf_descent_all",
            "twg_unet_num_params", "twg_unet_create", "twg_unet_destroy",
            "twg_unet_set_params", "twg_unet_get_params", "twg_unet_forward", "twg_unet_loss_grad",
            "twg_unet_adam_step", "twg_unet_features", "twg_unet_warm_start", "twg_unet_coarse_frame",
            "twg_unet_features_coarse", "twg_unet_coarse_target", "twg_unet_warm_start_coarse")


class TwgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libtwg error {code}: {msg}")
        self.code = code


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _grid_of(t):
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("grid arrays must be 2-D [ny, >= nx] with unit x stride")
    if not t.is_cuda:
        raise ValueError("grid arrays must be device tensors")
    return t.shape[1], t.shape[0], t.stride(0)


class Context:
    """Owns one twg_ctx on a HIP device."""

    def __init__(self, device: int | None = None):
        if device is None:
            device = torch.cuda.current_device()
        h = ctypes.c_void_p()
        rc = lib.twg_ctx_create(ctypes.byref(h), int(device))
        if rc != OK:
            raise TwgError(rc, "twg_ctx_create failed")
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            lib.twg_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=(OK,)):
        if rc not in allow:
            msg = lib.twg_last_error(self.h)
            raise TwgError(rc, msg.decode() if msg else "")
        return rc

    def set_graphs(self, enable: bool):
        """Replay relaxation passes from captured HIP graphs (default) or
        launch them one by one."""
        self._check(lib.twg_ctx_set_graphs(self.h, int(bool(enable))))

    @staticmethod
    def grid(nx, ny, pitch):
        return Grid(int(nx), int(ny), int(pitch))

    # ---- map update ------------------------------------------------------
    def rasterize(self, nx, ny, robot, goal, pos, vel, rad, W=8, robot_speed=1.0,
                  border_walls=True, static_occ=None, cls=None, ring=None, want_ring=True,
                  ring_mode=0, heading=(1.0, 0.0), per_object=False, kappa=0.0, cov=None):
        dev = torch.device("cuda", self.device)
        if cls is None:
            cls = torch.empty((ny, nx), dtype=torch.uint8, device=dev)
        if ring is None and want_ring:
            ring = torch.empty((ny, nx), dtype=torch.uint16, device=dev)
        gx, gy, pitch = _grid_of(cls)
        assert (gx, gy) == (nx, ny)
        n = int(rad.numel()) if rad is not None else 0
        for t in (pos, vel, rad):
            if t is not None and (t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous()):
                raise ValueError("obstacle arrays must be contiguous float64 device tensors")
        if ring is not None and ring.stride(0) != pitch:
            raise ValueError("ring map must share the class map's pitch")
        if static_occ is not None and static_occ.stride(0) != pitch:
            raise ValueError("static map must share the class map's pitch")
        if cov is not None and (cov.dtype != torch.float64 or not cov.is_cuda or not cov.is_contiguous()
                                or cov.numel() != 16 * n):
            raise ValueError("cov must be a contiguous float64 device tensor of n_obs x 16")
        p = RasterParams(int(robot[0]), int(robot[1]), int(goal[0]), int(goal[1]), int(W),
                         int(bool(border_walls)), float(robot_speed), int(ring_mode), int(bool(per_object)),
                         float(heading[0]), float(heading[1]), float(kappa), _ptr(cov))
        rc = lib.twg_rasterize(self.h, Grid(nx, ny, pitch), n, _ptr(pos), _ptr(vel), _ptr(rad),
                               _ptr(static_occ), ctypes.byref(p), _ptr(cls), _ptr(ring), _stream())
        self._check(rc)
        return cls, ring

    def kalman_step(self, x, P, z=None, dt=1.0, Q=None, R=None, pos=None, vel=None):
        """One Kalman step for every obstacle; x [n, 4] and P [n, 16] float64
        device tensors are updated in place (z [n, 2] or None; Q [16] and
        R [4] float64 device tensors or None)."""
        n = int(x.shape[0])
        for t, m in ((x, 4), (P, 16)):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != n * m:
                raise ValueError("x and P must be contiguous float64 device tensors [n, 4] and [n, 16]")
        for t in (z, Q, R, pos, vel):
            if t is not None and (t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous()):
                raise ValueError("z, Q, R, pos, vel must be contiguous float64 device tensors")
        rc = lib.twg_kalman_step(self.h, n, _ptr(x), _ptr(P), _ptr(z), float(dt), _ptr(Q), _ptr(R), _ptr(pos),
                                 _ptr(vel), _stream())
        self._check(rc)
        return x, P

    # ---- relaxation --------------------------------------------------------
    @staticmethod
    def _relax_params(cls, psi, psi64, tol, tol_cert, max_sweeps, omega, init, polish, sweeps_per_pass,
                      check_passes, rows_per_tile, goal):
        nx, ny, pitch = _grid_of(psi)
        if psi.dtype != torch.float32 or cls.dtype != torch.uint8 or cls.stride(0) != pitch:
            raise ValueError("psi must be float32 and share its pitch with the uint8 class map")
        if psi64 is not None and (psi64.dtype != torch.float64 or psi64.stride(0) != pitch):
            raise ValueError("psi64 must be float64 with the same pitch")
        gx, gy = (int(goal[0]), int(goal[1])) if goal is not None else (-1, -1)
        prm = HpfParams(float(tol), float(tol_cert), int(max_sweeps), float(omega), int(init),
                        int(polish), int(sweeps_per_pass), int(check_passes), int(rows_per_tile), gx, gy)
        return Grid(nx, ny, pitch), prm

    def relax(self, cls, psi, psi64=None, tol=1e-6, tol_cert=0.0, max_sweeps=0, omega=0.0,
              init=INIT_HALF, polish=0, sweeps_per_pass=0, check_passes=0, rows_per_tile=0, goal=None):
        """polish: 0 FP32 only, 1 (or True) FP64 defect correction, 2 FP64 SOR
        sweeps.  goal (x, y): the goal cell of INIT_LINEAR."""
        g, prm = self._relax_params(cls, psi, psi64, tol, tol_cert, max_sweeps, omega, init, polish,
                                    sweeps_per_pass, check_passes, rows_per_tile, goal)
        st = HpfStats()
        rc = lib.hpf_relax(self.h, g, _ptr(cls), _ptr(psi), _ptr(psi64), ctypes.byref(prm), ctypes.byref(st),
                           _stream())
        self._check(rc, allow=(OK, NOT_CONVERGED))
        return st.as_dict()

    def relax_async(self, cls, psi, psi64=None, slots=1024, stats=None, tol=1e-6, tol_cert=0.0, max_sweeps=0,
                    omega=0.0, init=INIT_HALF, polish=0, sweeps_per_pass=0, check_passes=0, rows_per_tile=0,
                    goal=None, noalloc=False):
        """Enqueue the device-driven relaxation (slots launches and a final
        one) on the current stream and return at once; stats is a device
        uint8 tensor of STATS_BYTES bytes that receives the hpf_stats (read it
        with stats_from_device after the stream has passed).  noalloc=True
        calls hpf_relax_async_noalloc (the library's static scratch; pass
        stats to keep torch from allocating too)."""
        g, prm = self._relax_params(cls, psi, psi64, tol, tol_cert, max_sweeps, omega, init, polish,
                                    sweeps_per_pass, check_passes, rows_per_tile, goal)
        if stats is None:
            stats = torch.zeros(STATS_BYTES, dtype=torch.uint8, device=psi.device)
        if stats.dtype != torch.uint8 or stats.numel() < STATS_BYTES or not stats.is_cuda:
            raise ValueError(f"stats must be a device uint8 tensor of at least {STATS_BYTES} bytes")
        fn = lib.hpf_relax_async_noalloc if noalloc else lib.hpf_relax_async
        rc = fn(self.h, g, _ptr(cls), _ptr(psi), _ptr(psi64), ctypes.byref(prm), int(slots), _ptr(stats), _stream())
        self._check(rc)
        return stats

    def relax_batched(self, cls_flat, psi_flat, descs, tol=1e-6, max_sweeps=0, omega=0.0,
                      init=INIT_HALF, sweeps_per_pass=0, check_passes=0, rows_per_tile=0, slots=0, stats=None,
                      lds=False):
        """Relax many grids packed in one flat uint8 class buffer and one flat
        float32 field buffer; descs = [(nx, ny, pitch, offset), ...] (offsets in
        elements).  Returns one stats dict per grid.  slots > 0: enqueue
        hpf_relax_batched_async (slots launches and a final one) on the
        current stream and return the device stats tensor (n hpf_stats; read
        with batch_stats_from_device).  lds: every grid that fits in one
        workgroup's LDS is solved whole there (TWG_GRID_LDS) instead of by the
        tiled passes."""
        if cls_flat.dtype != torch.uint8 or psi_flat.dtype != torch.float32:
            raise ValueError("class buffer must be uint8 and field buffer float32")
        if not (cls_flat.is_cuda and psi_flat.is_cuda):
            raise ValueError("batch buffers must be device tensors")
        n = len(descs)
        flags = GRID_LDS if lds else 0
        arr = (GridDesc * n)(*[GridDesc(int(a), int(b), int(c), flags, int(d)) for a, b, c, d in descs])
        for a, b, c, d in descs:
            if d + c * b > min(cls_flat.numel(), psi_flat.numel()):
                raise ValueError("a grid extends past the batch buffers")
        prm = HpfParams(float(tol), 0.0, int(max_sweeps), float(omega), int(init), 0,
                        int(sweeps_per_pass), int(check_passes), int(rows_per_tile), -1, -1)
        if slots:
            if stats is None:
                stats = torch.zeros(n * STATS_BYTES, dtype=torch.uint8, device=psi_flat.device)
            if stats.dtype != torch.uint8 or stats.numel() < n * STATS_BYTES or not stats.is_cuda:
                raise ValueError(f"stats must be a device uint8 tensor of at least {n * STATS_BYTES} bytes")
            rc = lib.hpf_relax_batched_async(self.h, n, arr, _ptr(cls_flat), _ptr(psi_flat), ctypes.byref(prm),
                                             int(slots), _ptr(stats), _stream())
            self._check(rc)
            return stats
        st = (HpfStats * n)()
        rc = lib.hpf_relax_batched(self.h, n, arr, _ptr(cls_flat), _ptr(psi_flat), ctypes.byref(prm),
                                   st, _stream())
        self._check(rc, allow=(OK, NOT_CONVERGED))
        return [x.as_dict() for x in st]

    def sweeps(self, cls, psi, omega, n, tiled=True, sweeps_per_pass=0, f=None):
        nx, ny, pitch = _grid_of(psi)
        rc = lib.hpf_sweeps(self.h, Grid(nx, ny, pitch), _ptr(cls), _ptr(psi), _ptr(f), float(omega),
                            int(n), int(bool(tiled)), int(sweeps_per_pass), _stream())
        self._check(rc)

    def sweeps64(self, cls, psi64, omega, n, tiled=True, sweeps_per_pass=0):
        nx, ny, pitch = _grid_of(psi64)
        rc = lib.hpf_sweeps64(self.h, Grid(nx, ny, pitch), _ptr(cls), _ptr(psi64), float(omega), int(n),
                              int(bool(tiled)), int(sweeps_per_pass), _stream())
        self._check(rc)

    def autotune(self, cls):
        """Tune tiling (FP32 and FP64 sweeps), SOR factors and the correction
        solves' start phase for grids of cls's size; returns dict(S, RH,
        omega, cups, S64, RH64, cups64, omega_dc, lead_dc_omega,
        lead_dc_sweeps)."""
        nx, ny, pitch = _grid_of(cls)
        out = (ctypes.c_double * 10)()
        rc = lib.hpf_autotune(self.h, Grid(nx, ny, pitch), _ptr(cls), out, _stream())
        self._check(rc)
        return dict(S=int(out[0]), RH=int(out[1]), omega=float(out[2]), cups=float(out[3]), S64=int(out[4]),
                    RH64=int(out[5]), cups64=float(out[6]), omega_dc=float(out[7]), lead_dc_omega=float(out[8]),
                    lead_dc_sweeps=int(out[9]))

    def autotune_batched(self, cls_flat, descs):
        """Pick the batch tiling (sweeps per pass, rows per tile) for this
        batch by timing whole solves; later relax_batched calls with
        sweeps_per_pass = 0 use it.  Returns dict(S, RH, ms)."""
        n = len(descs)
        arr = (GridDesc * n)(*[GridDesc(int(a), int(b), int(c), 0, int(d)) for a, b, c, d in descs])
        out = (ctypes.c_double * 3)()
        self._check(lib.hpf_autotune_batched(self.h, n, arr, _ptr(cls_flat), out, _stream()))
        return dict(S=int(out[0]), RH=int(out[1]), ms=float(out[2]))

    def set_tiling(self, nx, ny, S, RH, omega=0.0, S64=0, RH64=0):
        """Fix the tiling (and SOR factor) used for grids of this size."""
        self._check(lib.hpf_set_tiling(self.h, int(nx), int(ny), int(S), int(RH), float(omega), int(S64), int(RH64)))

    def residual(self, cls, psi=None, psi64=None, f=None):
        t = psi if psi is not None else psi64
        nx, ny, pitch = _grid_of(t)
        out = ctypes.c_double()
        rc = lib.hpf_residual(self.h, Grid(nx, ny, pitch), _ptr(cls), _ptr(psi), _ptr(psi64), _ptr(f),
                              ctypes.byref(out), _stream())
        self._check(rc)
        return out.value

    # ---- descent -----------------------------------------------------------
    def index_matrix(self, cls, psi=None, psi64=None, idx=None):
        t = psi if psi is not None else psi64
        nx, ny, pitch = _grid_of(t)
        if idx is None:
            idx = torch.empty_strided((ny, nx), (pitch, 1), dtype=torch.uint8, device=t.device)
        rc = lib.hpf_index_matrix(self.h, Grid(nx, ny, pitch), _ptr(cls), _ptr(psi), _ptr(psi64),
                                  _ptr(idx), _stream())
        self._check(rc)
        return idx

    def descent_all(self, cls, psi=None, psi64=None, steps=None):
        """Descent length to the goal from every cell (-1: does not reach it);
        int32 device tensor [ny, nx]."""
        t = psi if psi is not None else psi64
        nx, ny, pitch = _grid_of(t)
        if steps is None:
            steps = torch.empty((ny, nx), dtype=torch.int32, device=t.device)
        if steps.dtype != torch.int32 or steps.stride(1) != 1:
            raise ValueError("steps must be an int32 grid")
        rc = lib.hpf_descent_all(self.h, Grid(nx, ny, pitch), _ptr(cls), _ptr(psi), _ptr(psi64), _ptr(steps),
                                 int(steps.stride(0)), _stream())
        self._check(rc)
        return steps

    def descend(self, cls, psi=None, psi64=None, start=(0, 0), cap=None, path=None, info=None):
        """Returns (path tensor [cap, 2] int32, info tensor [2] int32 = [len, status]);
        both stay on the device (the call is asynchronous)."""
        t = psi if psi is not None else psi64
        nx, ny, pitch = _grid_of(t)
        if cap is None:
            cap = nx * ny
        if path is None:
            path = torch.empty((cap, 2), dtype=torch.int32, device=t.device)
        if info is None:
            info = torch.empty(2, dtype=torch.int32, device=t.device)
        p = DescendParams(int(start[0]), int(start[1]), int(cap), 0)
        rc = lib.hpf_descend(self.h, Grid(nx, ny, pitch), _ptr(cls), _ptr(psi), _ptr(psi64),
                             ctypes.byref(p), _ptr(path), _ptr(info), _stream())
        self._check(rc)
        return path, info


def _rubber(ctx, cls, psi, psi64, path, info, k, iters):
    t = psi if psi is not None else psi64
    nx, ny, pitch = _grid_of(t)
    if path.dtype != torch.int32 or path.dim() != 2 or path.shape[1] != 2 or not path.is_contiguous():
        raise ValueError("path must be a contiguous int32 [cap, 2] device tensor")
    if info.dtype != torch.int32 or info.numel() < 1:
        raise ValueError("info must hold the path length as int32")
    rc = lib.hpf_rubber_band(ctx.h, Grid(nx, ny, pitch), _ptr(cls), _ptr(psi), _ptr(psi64), _ptr(path), _ptr(info),
                             int(path.shape[0]), float(k), int(iters), _stream())
    ctx._check(rc)
    return path


def _merge_previous(ctx, cls, cls_prev, psi_prev, psi):
    """cls_prev None: every FREE cell of cls takes psi_prev's value."""
    nx, ny, pitch = _grid_of(psi)
    for t in (cls, cls_prev, psi_prev):
        if t is not None and t.stride(0) != pitch:
            raise ValueError("all maps must share psi's pitch")
    ctx._check(lib.hpf_merge_previous(ctx.h, Grid(nx, ny, pitch), _ptr(cls), _ptr(cls_prev), _ptr(psi_prev),
                                      _ptr(psi), _stream()))
    return psi


def _init_field(ctx, cls, psi, init=INIT_HALF, goal=None):
    nx, ny, pitch = _grid_of(psi)
    if cls.stride(0) != pitch:
        raise ValueError("class map must share psi's pitch")
    gx, gy = (int(goal[0]), int(goal[1])) if goal is not None else (-1, -1)
    ctx._check(lib.hpf_init_field(ctx.h, Grid(nx, ny, pitch), _ptr(cls), _ptr(psi), int(init), gx, gy,
                                  _stream()))
    return psi


Context.merge_previous = _merge_previous
Context.init_field = _init_field
Context.rubber_band = lambda self, cls, path, info, psi=None, psi64=None, k=1.0, iters=16: _rubber(
    self, cls, psi, psi64, path, info, k, iters)


class UNet:
    """The learned warm start's network (twg_unet_*): parameters, forward,
    loss and gradients, Adam, features and warm start.  Tensors are device
    tensors; images are [batch, H, W] and inputs [batch, H, W, 3]."""

    def __init__(self, ctx: Context, params=None):
        self.ctx = ctx
        h = ctypes.c_void_p()
        ctx._check(lib.twg_unet_create(ctx.h, ctypes.byref(h)))
        self.h = h
        self.n_params = int(lib.twg_unet_num_params())
        if params is not None:
            self.set_params(params)

    def close(self):
        if self.h:
            lib.twg_unet_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self):
        return torch.device("cuda", self.ctx.device)

    def set_params(self, params):
        t = torch.as_tensor(params, dtype=torch.float32).to(self._dev()).contiguous()
        if t.numel() != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {t.numel()}")
        self.ctx._check(lib.twg_unet_set_params(self.h, _ptr(t), _stream()))
        torch.cuda.current_stream().synchronize()

    def get_params(self):
        t = torch.empty(self.n_params, dtype=torch.float32, device=self._dev())
        self.ctx._check(lib.twg_unet_get_params(self.h, _ptr(t), _stream()))
        return t

    @staticmethod
    def _img(t, dtype, last=None):
        if t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"expected a contiguous {dtype} device tensor")
        if last is not None and t.shape[-1] != last:
            raise ValueError(f"last dimension must be {last}")
        return t

    def forward(self, x, y=None):
        x = self._img(x, torch.float32, 3)
        B, H, W, _ = x.shape
        if y is None:
            y = torch.empty((B, H, W), dtype=torch.float32, device=x.device)
        self.ctx._check(lib.twg_unet_forward(self.h, B, H, W, _ptr(x), _ptr(y), _stream()))
        return y

    def loss_grad(self, x, target, cls, loss=None, grads=None):
        x = self._img(x, torch.float32, 3)
        B, H, W, _ = x.shape
        self._img(target, torch.float32)
        self._img(cls, torch.uint8)
        if tuple(target.shape) != (B, H, W) or tuple(cls.shape) != (B, H, W):
            raise ValueError("target and cls must be [batch, H, W]")
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=x.device)
        self.ctx._check(lib.twg_unet_loss_grad(self.h, B, H, W, _ptr(x), _ptr(target), _ptr(cls), _ptr(loss),
                                               _ptr(grads), _stream()))
        return loss

    def adam_step(self, lr):
        self.ctx._check(lib.twg_unet_adam_step(self.h, float(lr), _stream()))

    def train_step(self, x, target, cls, lr, loss=None):
        loss = self.loss_grad(x, target, cls, loss)
        self.adam_step(lr)
        return loss

    def features(self, cls, ring, goal, H=None, W=None, out=None):
        nx, ny, pitch = _grid_of(cls)
        H = H if H is not None else (ny + 7) // 8 * 8
        W = W if W is not None else (nx + 7) // 8 * 8
        if out is None:
            out = torch.empty((H, W, 3), dtype=torch.float32, device=cls.device)
        if ring is not None and ring.stride(0) != pitch:
            raise ValueError("ring map must share the class map's pitch")
        self.ctx._check(lib.twg_unet_features(self.h, Grid(nx, ny, pitch), _ptr(cls), _ptr(ring), int(goal[0]),
                                              int(goal[1]), int(H), int(W), _ptr(out), _stream()))
        return out

    @staticmethod
    def coarse_frame(nx, ny, factor):
        """(Hc, Wc) of the coarse frame of an nx x ny grid at 1/factor."""
        h, w = i32(), i32()
        rc = lib.twg_unet_coarse_frame(Grid(int(nx), int(ny), int(nx)), int(factor), ctypes.byref(h), ctypes.byref(w))
        if rc != OK:
            raise TwgError(rc, "bad grid or factor")
        return h.value, w.value

    def features_coarse(self, cls, ring, goal, factor, x=None, ccls=None):
        """Coarse input channels FP32 [Hc][Wc][3] and the coarse training mask
        uint8 [Hc][Wc] of a grid seen at 1/factor."""
        nx, ny, pitch = _grid_of(cls)
        if ring is not None and ring.stride(0) != pitch:
            raise ValueError("ring map must share the class map's pitch")
        Hc, Wc = self.coarse_frame(nx, ny, factor)
        if x is None:
            x = torch.empty((Hc, Wc, 3), dtype=torch.float32, device=self._dev())
        if ccls is None:
            ccls = torch.empty((Hc, Wc), dtype=torch.uint8, device=self._dev())
        if x.numel() != Hc * Wc * 3 or ccls.numel() != Hc * Wc or not (x.is_contiguous() and ccls.is_contiguous()):
            raise ValueError("x must be [Hc, Wc, 3] float32 and ccls [Hc, Wc] uint8, contiguous")
        self.ctx._check(lib.twg_unet_features_coarse(self.h, Grid(nx, ny, pitch), _ptr(cls), _ptr(ring), int(goal[0]),
                                                     int(goal[1]), int(factor), _ptr(x), _ptr(ccls), _stream()))
        return x, ccls

    def coarse_target(self, cls, psi, factor, out=None):
        """Mean of psi over the FREE cells of every coarse block, FP32 [Hc][Wc]."""
        nx, ny, pitch = _grid_of(psi)
        if cls.stride(0) != pitch:
            raise ValueError("class map must share psi's pitch")
        Hc, Wc = self.coarse_frame(nx, ny, factor)
        if out is None:
            out = torch.empty((Hc, Wc), dtype=torch.float32, device=self._dev())
        if out.numel() != Hc * Wc or not out.is_contiguous():
            raise ValueError("out must be a contiguous [Hc, Wc] float32 tensor")
        self.ctx._check(lib.twg_unet_coarse_target(self.h, Grid(nx, ny, pitch), _ptr(cls), _ptr(psi), int(factor),
                                                   _ptr(out), _stream()))
        return out

    def warm_start_coarse(self, cls, ring, goal, psi, factor, status=None):
        """Network field at 1/factor of the grid's resolution, interpolated
        into psi's FREE cells (fallback and status as warm_start)."""
        nx, ny, pitch = _grid_of(psi)
        if cls.stride(0) != pitch or (ring is not None and ring.stride(0) != pitch):
            raise ValueError("class and ring maps must share psi's pitch")
        if status is not None and (status.dtype != torch.int32 or not status.is_cuda):
            raise ValueError("status must be an int32 device tensor")
        self.ctx._check(lib.twg_unet_warm_start_coarse(self.h, Grid(nx, ny, pitch), _ptr(cls), _ptr(ring),
                                                       int(goal[0]), int(goal[1]), int(factor), _ptr(psi),
                                                       _ptr(status), _stream()))
        return psi

    def warm_start(self, cls, ring, goal, psi, status=None):
        """Network field into psi.  status: optional device int32 tensor that
        receives OK, or NET_FALLBACK when the network's output was not finite
        (psi then holds the plain start 0.5 on FREE cells)."""
        nx, ny, pitch = _grid_of(psi)
        if cls.stride(0) != pitch or (ring is not None and ring.stride(0) != pitch):
            raise ValueError("class and ring maps must share psi's pitch")
        if status is not None and (status.dtype != torch.int32 or not status.is_cuda):
            raise ValueError("status must be an int32 device tensor")
        self.ctx._check(lib.twg_unet_warm_start(self.h, Grid(nx, ny, pitch), _ptr(cls), _ptr(ring), int(goal[0]),
                                                int(goal[1]), _ptr(psi), _ptr(status), _stream()))
        return psi


def plan(ctx, cls, psi, psi64, start, tol=1e-6, tol_cert=5e-7, init=INIT_HALF, extra_sweeps=256,
         max_extra=8, path=None, info=None):
    """One replanning field and path: FP32 relaxation to `tol`, FP64 SOR polish
    to a certified error of `tol_cert`, then further FP64 sweeps, `extra_sweeps`
    at a time, until the steepest descent from `start` reaches the goal (at
    most `max_extra` times: far from the goal the potential can be ~1e-13 and
    only a well-converged FP64 field orders its neighbours).  Returns
    (plain_stats, polish_stats, path, info, extra_rounds)."""
    plain = ctx.relax(cls, psi, None, tol=tol, init=init)
    pol = ctx.relax(cls, psi, psi64, tol=tol, init=INIT_KEEP, polish=2, tol_cert=tol_cert)
    path, info = ctx.descend(cls, psi64=psi64, start=start, path=path, info=info)
    rounds = 0
    while int(info[1].item()) == NO_PATH and rounds < max_extra:
        ctx.sweeps64(cls, psi64, pol["omega"], extra_sweeps)
        path, info = ctx.descend(cls, psi64=psi64, start=start, path=path, info=info)
        rounds += 1
    return plain, pol, path, info, rounds


def version() -> int:
    return int(lib.twg_version())
