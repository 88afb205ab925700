"""The replanning step and loop of the paper's Algorithm 1 on the device.

One step is the "Map Update" block (Kalman estimates of the moving obstacles,
time rings around the robot, prediction of every obstacle to its ring's
horizon, marking) followed by the "Path Planning" block (harmonic potential
relaxed to convergence, index matrix, steepest-descent path from the robot),
all through the C ABI of libtwg.so:

    twg_kalman_step -> twg_rasterize -> field initialisation (previous field,
    network or the plain start) -> hpf_relax (FP32 red-black SOR to residual
    tol) -> hpf_relax (FP64 defect-correction polish to a certified bound) ->
    hpf_descend (+ FP64 sweeps while the descent from the robot does not
    resolve).

The loop moves the robot one cell per step along its own descent path
(Algorithm 1: plan, then move), while the true obstacles move at constant
velocity and reflect at the walls, and the filters see their positions with
Gaussian noise.  ``StepGraph`` captures the same step (without the
data-dependent extra FP64 rounds) into one HIP graph through
``hpf_relax_async``.  Every array stays on the device; the host reads only
the path's first move (and, for reporting, the solver statistics).
"""
from __future__ import annotations

import numpy as np
import torch

from . import twg

# certified bound on |psi - psi*| the step polishes to: with the oracle's
# own field within 1e-8 of psi*, the result is within 1e-6 of it
POLISH_CERT = 5e-7
TOL = 1e-6          # FP32-stage residual tolerance
# the plain initial field of a cold solve: psi = 0 (phi = 1) on FREE cells,
# as if every free cell were an obstacle until the relaxation shows
# otherwise; far from the goal the converged potential is ~0 anyway, and it
# needs 912 sweeps to residual 1e-6 on the 2048 x 2048 benchmark map against
# 1224 from the paper's 0.5 and 1278 from a linear ramp
PLAIN_INIT = twg.INIT_ZERO


def reflect(p, n):
    """Positions p (any shape) folded into [0, n - 1]: constant-velocity
    motion that reflects at the walls of an n-cell axis."""
    L = float(n - 1)
    q = np.mod(p, 2.0 * L)
    return np.where(q > L, 2.0 * L - q, q)


class Planner:
    """Buffers and calls of one replanning step on one nx x ny grid."""

    def __init__(self, ctx: twg.Context, sc: dict, net: twg.UNet | None = None, extra_sweeps=256,
                 max_extra=8):
        self.ctx, self.sc, self.net = ctx, sc, net
        self.nx, self.ny = sc["nx"], sc["ny"]
        dev = torch.device("cuda", ctx.device)
        self.dev = dev
        shape = (self.ny, self.nx)
        self.cls = torch.empty(shape, dtype=torch.uint8, device=dev)
        self.ring = torch.empty(shape, dtype=torch.uint16, device=dev)
        self.psi = torch.empty(shape, dtype=torch.float32, device=dev)
        self.psi64 = torch.empty(shape, dtype=torch.float64, device=dev)
        self.cap = self.nx * self.ny
        self.path = torch.empty((self.cap, 2), dtype=torch.int32, device=dev)
        self.info = torch.zeros(2, dtype=torch.int32, device=dev)
        self.rad = torch.as_tensor(sc["rad"], dtype=torch.float64, device=dev).contiguous()
        self.extra_sweeps, self.max_extra = extra_sweeps, max_extra

    def rasterize(self, robot, pos, vel):
        sc = self.sc
        self.ctx.rasterize(self.nx, self.ny, robot, sc["goal"], pos, vel, self.rad, W=sc["W"],
                           robot_speed=sc["vr"], cls=self.cls, ring=self.ring)

    def solve(self, robot, init=PLAIN_INIT, omega=0.0, ev_mid=None):
        """FP32 relaxation to TOL from `init` (INIT_KEEP: the field already in
        psi), FP64 defect correction to POLISH_CERT, descent from `robot`
        with FP64 sweeps added while it does not resolve.  Returns (plain
        stats, polish stats, extra FP64 rounds).  ev_mid: an event recorded
        after the FP32 stage."""
        ctx = self.ctx
        plain = ctx.relax(self.cls, self.psi, None, tol=TOL, init=init, omega=omega)
        if ev_mid is not None:
            ev_mid.record()
        pol = ctx.relax(self.cls, self.psi, self.psi64, tol=TOL, init=twg.INIT_KEEP, polish=1,
                        tol_cert=POLISH_CERT)
        ctx.descend(self.cls, psi64=self.psi64, start=robot, cap=self.cap, path=self.path, info=self.info)
        rounds = 0
        while int(self.info[1].item()) == twg.NO_PATH and rounds < self.max_extra:
            ctx.sweeps64(self.cls, self.psi64, pol["omega"], self.extra_sweeps)
            ctx.descend(self.cls, psi64=self.psi64, start=robot, cap=self.cap, path=self.path, info=self.info)
            rounds += 1
        return plain, pol, rounds


class StepGraph:
    """One replanning step (rasterise, FP32 relaxation, FP64 polish, descent)
    captured into one HIP graph: the relaxation runs through
    hpf_relax_async with fixed slot counts (surplus slots return at once),
    so the whole step replays with no host involvement.  Without the extra
    FP64 rounds of ``Planner.solve``: the graph reports the descent status
    as it is.  Slot counts come from an eager solve of the same map.  The
    graph holds the addresses of the context's scratch buffers: replay it
    only while no call on the context has needed larger scratch since the
    capture (a larger grid reallocates them)."""

    def __init__(self, planner: Planner, robot, pos, vel, plain_stats, pol_stats, S, margin=1.25):
        self.p = planner
        ctx, p = planner.ctx, planner
        passes = plain_stats["sweeps"] // S
        cpasses = pol_stats["polish_sweeps"] // S
        rounds = pol_stats["polish_rounds"]
        # a solve of P passes and R rounds of C_r correction passes takes
        # P + 1 + sum (C_r + 2) + 1 slots (hpf_relax_async)
        self.slots_plain = int(margin * (passes + 3)) + 8
        self.slots_pol = int(margin * (cpasses + 2 * rounds + 4)) + 8
        self.st_plain = torch.zeros(twg.STATS_BYTES, dtype=torch.uint8, device=p.dev)
        self.st_pol = torch.zeros(twg.STATS_BYTES, dtype=torch.uint8, device=p.dev)
        self.robot, self.pos, self.vel = robot, pos, vel
        self.graph = torch.cuda.CUDAGraph()
        self._enqueue()  # once outside capture: scratch of these sizes exists afterwards
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.graph.capture_begin()
            self._enqueue()
            self.graph.capture_end()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()

    def _enqueue(self):
        p, ctx = self.p, self.p.ctx
        p.rasterize(self.robot, self.pos, self.vel)
        ctx.relax_async(p.cls, p.psi, None, slots=self.slots_plain, stats=self.st_plain, tol=TOL,
                        init=PLAIN_INIT)
        ctx.relax_async(p.cls, p.psi, p.psi64, slots=self.slots_pol, stats=self.st_pol, tol=TOL,
                        init=twg.INIT_KEEP, polish=1, tol_cert=POLISH_CERT)
        ctx.descend(p.cls, psi64=p.psi64, start=self.robot, cap=p.cap, path=p.path, info=p.info)

    def replay(self):
        self.graph.replay()

    def stats(self):
        return twg.stats_from_device(self.st_plain), twg.stats_from_device(self.st_pol)


def run_loop(ctx, sc, steps, sigma=0.0, net=None, omega_warm=None, keep_first=0, cold_every=0,
             meas_seed=77, log=None, fill="half", net_factor=0):
    """The replanning loop of Algorithm 1 for `steps` steps on scenario sc.

    Each step: Kalman update of every obstacle from a position measurement
    with noise sigma (R = 0.25 I; step 0 starts from the scenario's state),
    rasterise around the robot, initial field = the previous step's field
    where the cell was and is FREE and, elsewhere, by `fill`: "half" the
    paper's 0.5, "network" the network's field (net; at 1/net_factor of the
    grid's resolution when net_factor > 0), "previous" the
    previous field there too (0 where an obstacle was; step 0 starts from
    PLAIN_INIT), FP32 relaxation to
    TOL, FP64 polish to
    POLISH_CERT, descent from the robot; then the robot moves one cell along
    its path.  omega_warm: SOR factor of the warm FP32 solves (None: picked
    on step 1 from a fixed family, untimed).  Every cold_every-th step is
    also solved cold (the plain start, tuned factor) for comparison, untimed.
    The first keep_first steps keep host copies of their inputs and outputs
    (for checks against the oracle).  Returns a dict of per-step records."""
    dev = torch.device("cuda", ctx.device)
    nx, ny = sc["nx"], sc["ny"]
    pos0 = np.asarray(sc["pos"], dtype=np.float64)
    vel0 = np.asarray(sc["vel"], dtype=np.float64)
    n_o = len(pos0)
    rng = np.random.default_rng(sc["seed"] + meas_seed)
    kx = torch.as_tensor(np.concatenate([pos0, vel0], axis=1), dtype=torch.float64, device=dev).contiguous()
    kP = torch.as_tensor(np.tile(0.25 * np.eye(4).reshape(16), (n_o, 1)), dtype=torch.float64,
                         device=dev).contiguous()
    kR = torch.as_tensor((0.25 * np.eye(2)).reshape(4), dtype=torch.float64, device=dev)
    est_p = kx[:, :2].contiguous()
    est_v = kx[:, 2:].contiguous()
    a, b = Planner(ctx, sc, net), Planner(ctx, sc, net)
    cold = Planner(ctx, sc) if cold_every else None
    robot = [int(sc["robot"][0]), int(sc["robot"][1])]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    recs, kept = [], []
    w_trials = {}
    for k in range(steps):
        truth = np.stack([reflect(pos0[:, 0] + k * vel0[:, 0], nx), reflect(pos0[:, 1] + k * vel0[:, 1], ny)], 1)
        zk = torch.as_tensor(truth + sigma * rng.normal(0.0, 1.0, size=(n_o, 2)), dtype=torch.float64,
                             device=dev).contiguous()
        torch.cuda.synchronize()
        ev[0].record()
        if k > 0:
            ctx.kalman_step(kx, kP, zk, dt=1.0, R=kR, pos=est_p, vel=est_v)
        a.rasterize(robot, est_p, est_v)
        if fill == "network" and net_factor:
            net.warm_start_coarse(a.cls, a.ring, sc["goal"], a.psi, net_factor)
        elif fill == "network":
            net.warm_start(a.cls, a.ring, sc["goal"], a.psi)
        else:
            ctx.init_field(a.cls, a.psi, twg.INIT_HALF if fill == "half" else PLAIN_INIT)
        if k > 0:
            ctx.merge_previous(a.cls, None if fill == "previous" else b.cls, b.psi, a.psi)
        if k == 1 and omega_warm is None:
            # untimed: the warm FP32 solves' SOR factor from a fixed family
            # (0 = the tuned factor), by the time of the whole certified
            # solve.  A factor below the optimum reaches residual TOL sooner
            # from a warm start but leaves the smooth error behind, which the
            # polish then pays for many times over
            base = a.psi.clone()
            for wc in (1.9, 1.95, 1.98, 0.0):
                a.psi.copy_(base)
                e_a, e_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e_a.record()
                ctx.relax(a.cls, a.psi, None, tol=TOL, init=twg.INIT_KEEP, omega=wc)
                ctx.relax(a.cls, a.psi, a.psi64, tol=TOL, init=twg.INIT_KEEP, polish=1, tol_cert=POLISH_CERT,
                          max_sweeps=20000)
                e_b.record()
                torch.cuda.synchronize()
                w_trials[wc] = e_a.elapsed_time(e_b)
            # another factor replaces the tuned one only when it wins
            # clearly: its polish cost varies from step to step with the
            # smooth error it leaves, which one step's trial cannot see
            best = min(w_trials, key=w_trials.get)
            omega_warm = best if w_trials[best] < 0.95 * w_trials[0.0] else 0.0
            a.psi.copy_(base)
            ev[0].record()  # the step's time starts after the trials
        w = 0.0 if k == 0 else (omega_warm or 0.0)
        ev[1].record()
        plain, pol, rounds = a.solve(robot, init=twg.INIT_KEEP, omega=w, ev_mid=ev[3])
        ev[2].record()
        torch.cuda.synchronize()
        n_p, status = [int(v) for v in a.info.cpu().tolist()]
        nxt = robot
        if status == twg.OK and n_p >= 2:
            nxt = [int(v) for v in a.path[1].cpu().tolist()]
        rec = {"step": k, "ms": ev[0].elapsed_time(ev[2]), "ms_relax_polish_descent": ev[1].elapsed_time(ev[2]),
               "ms_fp32": ev[1].elapsed_time(ev[3]),
               "sweeps": plain["sweeps"], "polish_sweeps": pol["polish_sweeps"], "rounds": pol["polish_rounds"],
               "extra_fp64_rounds": rounds, "cert_bound": pol["cert_bound"], "status": status,
               "path_len": n_p, "robot": list(robot), "fp32_residual": plain["residual"]}
        if k < keep_first:
            kept.append({"robot": list(robot), "cls": a.cls.cpu().numpy(), "psi64": a.psi64.cpu().numpy(),
                         "path": a.path[:max(n_p, 0)].cpu().numpy(), "status": status,
                         "est_pos": est_p.cpu().numpy(), "est_vel": est_v.cpu().numpy(),
                         "cert_bound": pol["cert_bound"]})
        if cold_every and k % cold_every == cold_every // 2:
            cold.cls.copy_(a.cls)
            ev[0].record()
            cp, cq, cr = cold.solve(robot, init=PLAIN_INIT, ev_mid=ev[3])
            ev[2].record()
            torch.cuda.synchronize()
            rec["cold_ms_relax_polish_descent"] = ev[0].elapsed_time(ev[2])
            rec["cold_ms_fp32"] = ev[0].elapsed_time(ev[3])
            rec["cold_sweeps"] = cp["sweeps"]
            rec["cold_polish_sweeps"] = cq["polish_sweeps"]
        recs.append(rec)
        if log is not None and (k % 20 == 0 or k == steps - 1):
            log(f"loop step {k}: {rec['ms']:.3f} ms, sweeps {rec['sweeps']} + {rec['polish_sweeps']}, "
                f"status {status}, robot {robot}")
        robot = nxt
        a, b = b, a
    return {"records": recs, "kept": kept, "omega_warm": omega_warm,
            "omega_trials_ms": {str(k): round(v, 3) for k, v in w_trials.items()}}


def summarize(loop, what):
    """p50 / p95 / max step latency and counts of a run_loop result."""
    recs = loop["records"]
    ms = np.array([r["ms"] for r in recs[1:]]) if len(recs) > 1 else np.array([recs[0]["ms"]])
    core = np.array([r["ms_relax_polish_descent"] for r in recs[1:]]) if len(recs) > 1 else ms
    cold = np.array([r["cold_ms_relax_polish_descent"] for r in recs if "cold_ms_relax_polish_descent" in r])
    cold32 = np.array([r["cold_ms_fp32"] for r in recs if "cold_ms_fp32" in r])
    fp32 = np.array([r["ms_fp32"] for r in recs[1:]]) if len(recs) > 1 else np.array([recs[0]["ms_fp32"]])
    out = {"steps": len(recs), "warm_start": what,
           "step_ms_p50": round(float(np.percentile(ms, 50)), 3),
           "step_ms_p95": round(float(np.percentile(ms, 95)), 3),
           "step_ms_max": round(float(ms.max()), 3),
           "first_step_ms": round(float(recs[0]["ms"]), 3),
           "relax_polish_descent_ms_p50": round(float(np.percentile(core, 50)), 3),
           "fp32_stage_ms_p50": round(float(np.percentile(fp32, 50)), 3),
           "sweeps_p50": int(np.median([r["sweeps"] for r in recs[1:]] or [recs[0]["sweeps"]])),
           "polish_sweeps_p50": int(np.median([r["polish_sweeps"] for r in recs[1:]] or [recs[0]["polish_sweeps"]])),
           "descent_reached_goal": f"{sum(1 for r in recs if r['status'] == twg.OK)}/{len(recs)}",
           "max_cert_bound": max(r["cert_bound"] for r in recs),
           "extra_fp64_rounds": sum(r["extra_fp64_rounds"] for r in recs),
           "robot_start": recs[0]["robot"], "robot_end": recs[-1]["robot"],
           "omega_warm": loop["omega_warm"], "omega_trials_ms": loop["omega_trials_ms"]}
    if len(cold):
        out["cold_relax_polish_descent_ms_p50"] = round(float(np.percentile(cold, 50)), 3)
        out["cold_samples"] = int(len(cold))
        out["speedup_vs_cold_p50"] = round(float(np.percentile(cold, 50) / np.percentile(core, 50)), 3)
        out["cold_fp32_stage_ms_p50"] = round(float(np.percentile(cold32, 50)), 3)
        out["fp32_stage_speedup_vs_cold_p50"] = round(float(np.percentile(cold32, 50) / np.percentile(fp32, 50)), 3)
    return out
