/*
 * twg.h -- C ABI of libtwg.so: harmonic potential fields on time-warped grids
 * for AMD Instinct MI355X (gfx950).
 *
 * Method: Farzan & DeSouza, "Path Planning in Dynamic Environments Using
 * Time-Warped Grids and a Parallel Implementation".  The library computes the
 * data-parallel part of each replanning step of Algorithm 1:
 *   twg_rasterize  -- "Map Update": time rings around the robot, Kalman
 *                     prediction of every moving obstacle to its ring's
 *                     horizon, and marking of the predicted poses.
 *   hpf_relax      -- "Path Planning", harmonic potential: Laplace's equation
 *                     (Eqs. 1-2) relaxed to convergence with Dirichlet goal,
 *                     obstacle and wall values.
 *   hpf_descend    -- index matrix (Eq. 3) and steepest-descent path.
 *
 * Conventions shared by every entry point
 *   - Array arguments are DEVICE pointers unless marked "host".  The caller
 *     owns every buffer it passes; the library never frees caller memory.  The
 *     context owns only its scratch buffers (allocated at first use of a size,
 *     released by twg_ctx_destroy).
 *   - Grids are row-major, x fastest: a[y * pitch + x], nx <= pitch <= 65536,
 *     in elements of the array's type, and pitch * ny < 2^31.
 *     1 <= nx, ny <= 32767.  Even nx and pitch (with bases aligned to two
 *     elements) take the faster paired-column relaxation.
 *   - The potential is stored as psi = 1 - phi, phi being the paper's
 *     potential: the goal holds psi = 1, obstacles and walls psi = 0, free
 *     space starts at psi = 0.5 (phi = 0.5).  The equation is linear, so psi
 *     is harmonic where phi is; the goal-side values keep FP32 relative
 *     precision far from the goal, where phi approaches 1.
 *   - A neighbour outside the grid acts as a fixed cell with psi = 0.
 *   - Every call is ordered on `stream` (a hipStream_t; NULL = the null
 *     stream).  Calls documented as "blocking" also wait for their own work.
 *   - Return value: 0 = TWG_OK; > 0 = finished with a non-fatal outcome;
 *     < 0 = error, outputs undefined.  twg_last_error() describes the last
 *     error or outcome of a context in words.
 */
#ifndef TWG_H
#define TWG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define TWG_OK 0
#define TWG_NOT_CONVERGED 1   /* max_sweeps reached; the partial field is returned */
#define TWG_NO_PATH 2         /* descent met a cell with no strictly better neighbour */
#define TWG_START_BLOCKED 3   /* the start cell is not FREE or GOAL */
#define TWG_NET_FALLBACK 4    /* learned warm start rejected; the plain initial field was used */
#define TWG_PATH_TRUNCATED 5  /* the path buffer filled before the goal */
#define TWG_EINVAL (-1)       /* invalid argument (checked on the host before any launch) */
#define TWG_ENOMEM (-2)       /* scratch allocation failed */
#define TWG_EDEVICE (-3)      /* a HIP call failed */
#define TWG_EUNSUPPORTED (-4) /* valid but unsupported option */

/* ---- cell classes (uint8 class map) ------------------------------------- */
#define TWG_CELL_FREE 0  /* relaxed */
#define TWG_CELL_OBST 1  /* obstacle, static or predicted: psi = 0 (phi = 1) */
#define TWG_CELL_WALL 2  /* border wall: psi = 0 */
#define TWG_CELL_GOAL 3  /* goal: psi = 1 (phi = 0) */
#define TWG_CELL_FIXED 4 /* Dirichlet cell holding the value the caller put in psi */

typedef struct twg_ctx twg_ctx;

typedef struct {
    int32_t nx, ny; /* cells */
    int32_t pitch;  /* row stride in elements, nx <= pitch <= 65536 */
} twg_grid;

/* Library version, major * 10000 + minor * 100 + patch. */
int32_t twg_version(void);

/* Create a context bound to HIP device `device`; *out receives it.
 * Errors: TWG_EINVAL (out NULL, no such device), TWG_EDEVICE. */
int32_t twg_ctx_create(twg_ctx **out, int32_t device);

/* Wait for the device, free the context's scratch and the context. */
int32_t twg_ctx_destroy(twg_ctx *ctx);

/* Text of the last error or non-fatal outcome of ctx ("" if none).  The
 * string belongs to ctx and is valid until its next call. */
const char *twg_last_error(const twg_ctx *ctx);

/* enable = 1 (default): runs of 64 relaxation passes are captured once into a
 * HIP graph (on a context-owned stream) and replayed on the caller's stream;
 * enable = 0: every pass is launched on its own.  Results are identical.
 * Errors: TWG_EINVAL for another value. */
int32_t twg_ctx_set_graphs(twg_ctx *ctx, int32_t enable);

/* ========================================================================= */
/* Map update: time rings, prediction, marking                               */
/* ========================================================================= */

typedef struct {
    int32_t robot_x, robot_y; /* robot cell (ring centre); inside the grid */
    int32_t goal_x, goal_y;   /* goal cell; inside the grid */
    int32_t ring_width;       /* W >= 1, cells per time ring */
    int32_t border_walls;     /* 1: cells on the grid border are WALL */
    double robot_speed;       /* v_r > 0, cells per step */
    /* The fields below may be left zero (circular rings, per-cell horizon,
     * no inflation). */
    int32_t ring_mode;        /* 0 circular rings; 1 elliptical warp metric (Eqs. 14-15) */
    int32_t per_object;       /* 0 per-cell horizon; 1 per-object horizon (Algorithm 1) */
    double heading_x, heading_y; /* robot heading (cos, sin) for ring_mode 1, used as given */
    double kappa;             /* covariance inflation factor >= 0 (0 = off) */
    const double *cov;        /* n_obs x 16 doubles (device): row-major 4x4 covariance of the
                                 state [x, y, vx, vy], or NULL (no inflation) */
} twg_raster_params;

/* twg_rasterize -- class map of one replanning step (Algorithm 1, "Map
 * Update"; section "Time-Warped Grid"; section "Integration of Kalman Filter
 * with Time-Warps").
 *
 * Every cell (x, y) lies in time ring
 *     j = floor(sqrt((x - robot_x)^2 + (y - robot_y)^2) / W)
 * (concentric rings of width W around the robot: the isotropic case of the
 * warp ellipses of Eqs. 14-15), computed exactly in integers.  Ring j's
 * horizon is t_j = j W / robot_speed steps: the time the robot needs to reach
 * the ring.  Obstacle i's constant-velocity Kalman state is predicted to t_j
 * by Eq. (9) with the state matrix of time step t_j: mu = p + t_j v (each
 * product and sum rounded once, FP64).  The cell is occupied by obstacle i
 * when its centre lies in the disc of radius r_i around mu, tested exactly in
 * Q.8 fixed point: C = rint(256 mu), R = rint(256 r) (round half to even) and
 * (256 x - C_x)^2 + (256 y - C_y)^2 <= R^2 in 64-bit integers.  A cell thus
 * sees every obstacle at the pose predicted for the time the robot would get
 * there.  Class, by precedence: WALL (border, if border_walls), GOAL (the goal
 * cell), OBST (static_occ nonzero, or occupied), FREE.
 *
 * ring_mode 1 replaces the circles by the paper's elliptical time warps
 * (Eqs. 14-15): the ellipse through a cell is centred 0.9 r_x ahead of the
 * robot along the heading with r_x = 4 r_y, i.e. with u = hx dx + hy dy and
 * v = hy dx - hx dy, r_x = (-1.8 u + sqrt(4 u^2 + 12.16 v^2)) / 0.38, and
 * j = floor(r_x / W), decided exactly: r_x >= j W when 0.38 j W + 1.8 u <= 0
 * or 4 u^2 + 12.16 v^2 >= (0.38 j W + 1.8 u)^2 (each operation rounded once).
 * per_object 1 follows Algorithm 1 literally: obstacle i is predicted once,
 * to the horizon of the ring of the cell nearest its current centre (round
 * half to even), and every cell of that disc is marked, whatever its ring.
 * kappa > 0 with cov grows each disc by min(W, kappa sqrt(lambda_max)),
 * lambda_max the larger eigenvalue of the predicted position covariance
 * P_pp + t (P_pv + P_vp) + t^2 P_vv at the disc's horizon t (the paper's
 * Gaussian marking of the prediction uncertainty, read as a capped radius).
 *
 *   pos, vel   n_obs x 2 doubles [x, y] (device): position in cells, velocity
 *              in cells per step.  Obstacles with a non-finite predicted
 *              position, or with |256 mu| >= 2^40, are ignored.
 *   radius     n_obs doubles (device), cells.  An obstacle whose radius is not
 *              a finite number in [0, 1e6] is ignored.
 *   static_occ optional uint8 map (device, pitch g.pitch): nonzero = static
 *              obstacle.  NULL = none.
 *   cls        out uint8 class map (device, pitch g.pitch).
 *   ring       optional out uint16 ring map (device, pitch g.pitch), or NULL.
 * Asynchronous.  Errors: TWG_EINVAL for a bad grid, robot or goal outside the
 * grid, W < 1, non-positive or non-finite speed, n_obs < 0, NULL cls, n_obs > 0
 * with NULL pos/vel/radius, ring_mode or per_object not 0/1, a heading that is
 * not finite or is zero with ring_mode 1, kappa negative or not finite;
 * TWG_EUNSUPPORTED when more than 65536 rings would touch the grid. */
int32_t twg_rasterize(twg_ctx *ctx, twg_grid g, int32_t n_obs, const double *pos,
                      const double *vel, const double *radius, const uint8_t *static_occ,
                      const twg_raster_params *params, uint8_t *cls, uint16_t *ring,
                      void *stream);

/* twg_kalman_step -- one step of the obstacles' Kalman filters (section
 * "Kalman Filter", Eqs. 9-13), one thread per obstacle, FP64.  State
 * [x, y, vx, vy] in cells and cells per step, constant-velocity model with
 * time step dt: time update x <- A x, P <- A P A^T + Q with A = [[I, dt I],
 * [0, I]] (Eqs. 9-10); then, if z is not NULL, measurement update with
 * H = [I 0]: K = P H^T (H P H^T + R)^-1, x <- x + K (z - H x),
 * P <- (I - K H) P (Eqs. 11-13, the 2x2 inverse written out).  Products are
 * summed in index order, each operation rounded once.
 *   x    n x 4 doubles (device), in/out.   P  n x 16 (row-major 4x4), in/out
 *        (the covariance layout twg_raster_params.cov takes).
 *   z    n x 2 measured positions (device) or NULL (prediction only).
 *   Q    16 doubles (device) or NULL (no process noise); R 4 doubles (device),
 *        required with z.
 *   pos, vel  optional n x 2 outputs (device): the new state's position and
 *        velocity, the arrays twg_rasterize takes.
 * Asynchronous.  Errors: TWG_EINVAL (n < 0, NULL x/P with n > 0, z without
 * R, dt not finite). */
int32_t twg_kalman_step(twg_ctx *ctx, int32_t n, double *x, double *P, const double *z, double dt,
                        const double *Q, const double *R, double *pos, double *vel, void *stream);

/* ========================================================================= */
/* Harmonic potential                                                        */
/* ========================================================================= */

#define HPF_INIT_KEEP 0   /* free cells keep the values in psi */
#define HPF_INIT_HALF 1   /* free cells start at phi = psi = 0.5 (the paper's choice) */
#define HPF_INIT_ZERO 2   /* free cells start at psi = 0 (phi = 1) */
#define HPF_INIT_LINEAR 3 /* free cells start on the ramp psi = 1 - d / (max(nx, ny) sqrt 2), d the
                             Euclidean distance to the goal cell (goal_x, goal_y), in FP64 rounded once */

typedef struct {
    double tol;              /* stop when max over FREE cells of |avg4(psi) - psi|,
                                evaluated in FP64, is <= tol (default 1e-6) */
    double tol_cert;         /* > 0: with polish, also require the certified error
                                bound residual * wbound <= tol_cert */
    int64_t max_sweeps;      /* cap on FP32 sweeps of the field (0 = 10^7) */
    float omega;             /* SOR factor in (0, 2); 0 = the autotuned factors of this grid
                                size (hpf_autotune), else the open-rectangle optimum */
    int32_t init;            /* HPF_INIT_* */
    int32_t polish;          /* 0: FP32 only; 1: FP64 defect correction (FP32 correction
                                solves); 2: FP64 red-black SOR sweeps */
    int32_t sweeps_per_pass; /* red-black sweeps per tile load (1 to 8); 0 = tuned */
    int32_t check_passes;    /* passes between residual checks; 0 = adaptive */
    int32_t rows_per_tile;   /* output rows per tile (even, >= 2); 0 = tuned */
    int32_t goal_x, goal_y;  /* goal cell of HPF_INIT_LINEAR (else unused) */
} hpf_params;

typedef struct {
    int64_t sweeps;        /* FP32 red-black sweeps on the field */
    int64_t polish_sweeps; /* FP32 sweeps on corrections */
    double residual;       /* FP64 residual of the returned field (psi64 if polished) */
    double residual32;     /* FP64 residual of the FP32 field after the FP32 phase */
    double cert_bound;     /* residual * wbound: bound on |psi - psi*| (max principle) */
    double wbound;         /* ((min(nx, ny) + 1)^2) / 2 >= ||(I - J)^-1 1||inf */
    float omega;           /* SOR factor used */
    int32_t status;        /* TWG_OK or TWG_NOT_CONVERGED */
    int32_t polish_rounds; /* defect-correction rounds */
    int32_t checks;        /* residual evaluations (fused checks and defects) */
    double residual_rel;   /* max |r| / |psi| over FREE cells with |psi| >= 1e-30 (FP32 phase);
                              far from the goal this stays large in FP32, whose rounding
                              noise there exceeds the field itself */
} hpf_stats;

/* hpf_relax -- converge the harmonic potential of one grid (Eqs. 1-2,
 * boundary values of section "Harmonic Potential Fields", Algorithm 1 "Path
 * Planning").
 *
 * Solves the discrete Laplace equation psi = avg4(psi) on FREE cells, where
 * avg4 is the mean of the four neighbours (Eq. 1), with Dirichlet values on
 * every other cell: OBST and WALL 0, GOAL 1, FIXED the input value.  The
 * iteration is red-black SOR (red = (x + y) even first; each FREE cell set to
 * psi + omega (avg4(psi) - psi), evaluated as fma(omega, fma(1/4,
 * ((E + W) + N) + S, -psi), psi) with N the row above and S the row below) in FP32,
 * several sweeps per tile load.  It stops when the FP64 residual
 * r = max |avg4(psi) - psi| over FREE cells is <= tol.  Because
 * |psi - psi*| <= r * ||(I - J)^-1 1||inf (discrete maximum principle), the
 * residual certifies the error.  With polish != 0 the field is then refined
 * in FP64 until r <= tol and r * wbound <= tol_cert, and the result is written
 * to psi64 (and rounded into psi): polish = 1 by defect correction (FP64
 * residual, FP32 correction solve, FP64 update), polish = 2 by FP64 SOR sweeps.
 * Far from the goal psi can be ~1e-13: FP32 sweeps leave rounding noise of
 * ~1e-12 there, so only an FP64-refined field resolves the descent far from
 * the goal.  Either polish gives one; on 2048 x 2048 fields, defect
 * correction to tol_cert = 1e-7 is faster than FP64 sweeps to 5e-7.  The
 * correction solves use the autotuned defect-correction factor (or omega if
 * given).  With omega = 0 on an autotuned size, each correction solve may
 * open with a start phase: a few passes at a smaller tuned factor (counted
 * in polish_sweeps).  A correction solve also ends early when, over a check
 * span of at least 128 sweeps, it contracts at less than half the speed its
 * factor omega gives every mode at or above a domain's optimum
 * (1 - q < (2 - omega) / 2 for the measured rate q per sweep): that is the
 * FP32 rounding floor of a correction with a large smooth part, which a
 * warm-started FP32 stage can leave; the FP64 update and the next round
 * carry on from there.
 *
 * Convergence is decided on the device (polish 0 and 1): the passes that
 * check measure the residual of their input field as they stream it, and the
 * last workgroup of each launch applies the stop rules (tolerance, sweep
 * budget, a stall at the FP32 rounding floor) and picks the next check from
 * the measured contraction; a solve that ends at a check returns the field
 * that check measured.  The sweep budget counts whole passes (max_sweeps is
 * rounded up to a multiple of the sweeps per pass).  The host only keeps
 * enough launches queued (it reads the device's decisions from pinned
 * memory and never waits for a residual).  With polish = 1 and
 * HPF_INIT_KEEP the solve opens with the first FP64 defect of the kept
 * field, which also gives the FP32 stage's initial residual: when that meets
 * tol the FP32 stage sweeps nothing (the usual call after an FP32 solve),
 * else the FP32 solve runs and the first defect comes again.  polish = 2
 * runs the FP64 sweeps with host-side checks.
 *
 *   cls    uint8 class map (device, pitch g.pitch).
 *   psi    in/out FP32 field (device, pitch g.pitch): FIXED cells must hold their
 *          values; with HPF_INIT_KEEP the FREE cells hold the initial field.
 *   psi64  FP64 field (device, pitch g.pitch) written when polish != 0; may be
 *          NULL when polish = 0.
 *   stats  host pointer or NULL.
 * Blocking: returns when the field is final.  Not for two streams at once on
 * one context (the control block and scratch belong to the context).
 * Returns TWG_OK or TWG_NOT_CONVERGED; errors TWG_EINVAL (bad grid, NULL
 * arrays, tol <= 0, omega outside [0, 2), polish without psi64, bad
 * sweeps_per_pass, HPF_INIT_LINEAR with the goal outside the grid, a
 * non-finite value in the field), TWG_ENOMEM, TWG_EDEVICE. */
int32_t hpf_relax(twg_ctx *ctx, twg_grid g, const uint8_t *cls, float *psi, double *psi64,
                  const hpf_params *params, hpf_stats *stats, void *stream);

/* hpf_relax_async -- hpf_relax (polish 0 or 1) with nothing done on the
 * host after the arguments are checked: field initialisation, then exactly
 * `slots` launches of the device-driven relaxation and one final launch, all
 * enqueued on `stream`, which a caller may capture into a graph.  Each
 * launch does one step the device decides (a pass of S sweeps, a defect, an
 * update); launches after the end return at once, and the final one ends a
 * solve still running (status TWG_NOT_CONVERGED, with the latest field).  A
 * solve of P FP32 passes and R polish rounds of C_r correction passes takes
 * P + 1 + sum_r (C_r + 2) + 1 slots.  stats is a DEVICE hpf_stats written
 * when the solve ends (status TWG_OK, TWG_NOT_CONVERGED or TWG_EINVAL for a
 * non-finite value); it is valid once the stream has passed the launches.
 * Scratch is allocated at the first call of a grid size: make that call
 * outside capture.  Returns TWG_OK when enqueued; errors as hpf_relax, and
 * TWG_EINVAL for slots < 1 or NULL stats, TWG_EUNSUPPORTED for polish = 2. */
int32_t hpf_relax_async(twg_ctx *ctx, twg_grid g, const uint8_t *cls, float *psi, double *psi64,
                        const hpf_params *params, int32_t slots, hpf_stats *stats, void *stream);

/* hpf_relax_async_noalloc -- hpf_relax_async for callers that cannot
 * allocate device memory: code under HIP graph capture (also at the first
 * call of a grid size), tight serving loops, harnesses that forbid
 * hipMalloc.  The same launches and the same results, bit for bit, with
 * every scratch buffer (control block, FP32 ping-pong partner, defect,
 * correction and the defect's products with the two correction factors,
 * free mask) inside one static device array of the library, 21 bytes per
 * cell for at most 4194304 cells plus 4 KiB (84 MiB and 4 KiB),
 * which each GPU the library runs on holds until the process ends.  The call
 * itself allocates nothing on the device (no hipMalloc, no hipFree).
 * Limit: pitch * ny <= 4194304 (e.g. 2048 x 2048); larger grids return
 * TWG_EUNSUPPORTED before any launch.  Every call on one GPU shares that
 * GPU's array, which keeps the last call's contents (each call resets its
 * control block with a kernel and writes every other buffer before reading
 * it): calls that overlap on one GPU -- on two streams, or from two contexts
 * -- race and give undefined results; serialise them.  hpf_relax and
 * hpf_relax_async use the context's own scratch and do not race with it.
 * Arguments, stats and errors as hpf_relax_async. */
int32_t hpf_relax_async_noalloc(twg_ctx *ctx, twg_grid g, const uint8_t *cls, float *psi, double *psi64,
                                const hpf_params *params, int32_t slots, hpf_stats *stats, void *stream);

typedef struct {
    int32_t nx, ny, pitch; /* as twg_grid */
    int32_t flags;  /* 0, or TWG_GRID_LDS */
    int64_t offset; /* element offset of this grid's arrays from the batch base pointers */
} twg_grid_desc;

/* twg_grid_desc.flags: solve the grid whole in one workgroup's LDS when it
 * fits there, instead of by the tiled passes */
#define TWG_GRID_LDS 1

/* hpf_relax_batched -- hpf_relax (FP32 phase) for n independent grids of any
 * sizes at once (Eqs. 1-2 on every grid; section "GPU-Based Parallel
 * Implementation").  Grid k's class map and field start at element offset
 * grids[k].offset of cls and psi (the grids must not overlap).  Every pass is
 * ONE launch over the tiles of all grids still above tolerance; each grid
 * runs its own solve on the device -- its own pass count, its own residual
 * checks (fused into the pass that checks, FP64 maxima per grid), its own
 * stop rules (tolerance, sweep budget per grid, a stall at the FP32
 * rounding floor) -- and drops out of the launches at the check where it
 * stops.  Checks fall on passes that are multiples of 4 (so that grids share
 * them), or every params->check_passes passes.  A grid whose descriptor
 * sets TWG_GRID_LDS and whose field and free mask fit in one workgroup's LDS
 * (5 bytes per cell: up to about 176 x 176 with 160 KiB of LDS) takes no part
 * in the passes: one workgroup loads it, checks its FP64 residual every S
 * sweeps and sweeps it in LDS until the same stop rules hold, and writes it
 * back once, before the first pass.  Its field after N sweeps has the bits
 * of N sweeps on the tiled path (its sweep count is a multiple of S).  On
 * MI355X the tiled passes are faster even for grids of 64 to 160 cells a
 * side (1024 such grids: 8.6 against 19.8 ms), so it is not the default.  The host never waits for a
 * residual: it only keeps launches queued (it reads the device's decisions
 * from pinned memory).  Sweeps per tile load and rows per tile come from
 * hpf_autotune_batched if it ran on this context, else from the
 * autotuned entry of the largest grid (or params->sweeps_per_pass /
 * rows_per_tile); each grid's SOR factor is params->omega, else its size's
 * autotuned factor, else its open-rectangle optimum.  init: HPF_INIT_KEEP,
 * HALF or ZERO; polish must be 0.  stats: host array of n entries, or NULL.
 * Blocking.  Returns TWG_OK when every grid converged, else
 * TWG_NOT_CONVERGED.  Errors: TWG_EINVAL (n < 1, NULL arrays, a bad grid,
 * offset or flags, polish set, a non-finite value in a grid),
 * TWG_EUNSUPPORTED (more than 65536 grids), TWG_ENOMEM, TWG_EDEVICE. */
int32_t hpf_relax_batched(twg_ctx *ctx, int32_t n, const twg_grid_desc *grids, const uint8_t *cls,
                          float *psi, const hpf_params *params, hpf_stats *stats, void *stream);

/* hpf_relax_batched_async -- hpf_relax_batched with nothing done on the host
 * after the arguments are checked: field initialisation, free masks, then
 * exactly `slots` launches of the batch and one final launch, all enqueued
 * on `stream` (a caller may capture them into a graph).  Each launch is one
 * pass over the tiles of the grids still active; launches after the end
 * return at once, and the final one ends the grids still running (status
 * TWG_NOT_CONVERGED, with their latest fields).  A batch whose slowest grid
 * needs P passes takes about P + 2 slots (its checks fall on multiples of 4
 * passes).  stats: DEVICE array of n hpf_stats, written when the batch ends.
 * The descriptor tables are uploaded (with a wait) only when they differ
 * from the last call's: make the first call of a batch outside capture.
 * Errors as hpf_relax_batched, and TWG_EINVAL for slots < 1 or NULL stats. */
int32_t hpf_relax_batched_async(twg_ctx *ctx, int32_t n, const twg_grid_desc *grids, const uint8_t *cls,
                                float *psi, const hpf_params *params, int32_t slots, hpf_stats *stats,
                                void *stream);

/* hpf_init_field -- the initial field of hpf_relax without relaxing: OBST
 * and WALL cells 0, GOAL 1, FIXED unchanged, FREE cells by `init`
 * (HPF_INIT_*; KEEP leaves them; LINEAR uses the goal cell (goal_x, goal_y),
 * ignored otherwise).  Asynchronous.  Errors: TWG_EINVAL. */
int32_t hpf_init_field(twg_ctx *ctx, twg_grid g, const uint8_t *cls, float *psi, int32_t init, int32_t goal_x,
                       int32_t goal_y, void *stream);

/* hpf_merge_previous -- warm start of a replanning step from the previous
 * step's field: every cell that is FREE in cls and was FREE in cls_prev takes
 * psi_prev's value; all other cells of psi are left as they are (so a
 * network warm start, or Dirichlet values, written to psi beforehand remain
 * where the map changed).  cls_prev NULL: every FREE cell of cls takes
 * psi_prev's value (a cell freed since the previous step starts from the
 * previous field there: 0 where an obstacle was).  All arrays device, pitch
 * g.pitch.  Asynchronous.  Errors: TWG_EINVAL (NULL cls, psi_prev or psi). */
int32_t hpf_merge_previous(twg_ctx *ctx, twg_grid g, const uint8_t *cls, const uint8_t *cls_prev,
                           const float *psi_prev, float *psi, void *stream);

/* hpf_sweeps -- exactly `sweeps` red-black SOR sweeps of the same update as
 * hpf_relax, with an optional FP32 source f (psi + omega (avg4(psi) + f - psi);
 * NULL = 0), no convergence test.  tiled = 0 runs one launch per colour
 * (each colour in place); tiled = 1 runs sweeps_per_pass sweeps per tile load
 * and gives bit-identical results.  Asynchronous.  Errors: TWG_EINVAL. */
int32_t hpf_sweeps(twg_ctx *ctx, twg_grid g, const uint8_t *cls, float *psi, const float *f,
                   float omega, int32_t sweeps, int32_t tiled, int32_t sweeps_per_pass,
                   void *stream);

/* hpf_sweeps64 -- exactly `sweeps` red-black SOR sweeps of an FP64 field
 * psi64, the update evaluated as fma(omega, fma(1/4, ((E + W) + N) + S,
 * -psi), psi) (N the row above, S the row below, each operation rounded
 * once), the expression the oracle's FP64 sweep evaluates, bit for bit.  tiled = 0: one launch per colour;
 * tiled = 1: sweeps_per_pass (1 to 8; 0 = the autotuned FP64
 * tiling of this grid size, else 4) sweeps per tile load, bit-identical.  Asynchronous.  Errors: TWG_EINVAL. */
int32_t hpf_sweeps64(twg_ctx *ctx, twg_grid g, const uint8_t *cls, double *psi64, double omega,
                     int32_t sweeps, int32_t tiled, int32_t sweeps_per_pass, void *stream);

/* hpf_autotune -- measure the relaxation kernel on grid g and class map cls
 * and remember, for grids of this exact size, the fastest tiling and an SOR
 * factor; later hpf_relax calls on this context with sweeps_per_pass = 0
 * and omega = 0 use them.  Tilings: sweeps per tile load S in
 * 1 to 8 x output rows per tile RH in {8, 16, 32, 64, 128} plus,
 * for k = 1..4, the smallest height whose tile count (one wave per tile) fits
 * k rounds of the device's SIMDs; each timed with HIP events over repeated
 * passes on context scratch, with and without a source term, and ranked by
 * the sum of the two times per sweep (the correction solves of a polish run
 * the passes with a source).  SOR factors:
 * omega = 2 / (1 + c sin(pi / (n + 1))), n = max(nx, ny), c in
 * {1, 1.4, 2, 2.4, 2.8, 3, 3.3, 3.6, 4, 4.5, 5, 6} (obstacles shrink the
 * effective domain, so the best factor is below the open-rectangle one):
 * the relaxation's factor by the fewest sweeps from the half-initialised
 * field to residual 1e-6, the defect-correction solves' factor (polish = 1)
 * by the fewest correction sweeps in polishing that field to a certified
 * 1e-7;
 * each keeps the next factor towards 2 unless that costs over 25 % more
 * sweeps (below the optimum the count climbs steeply).  Start phase: each
 * correction solve may open with sweeps at a smaller factor (c in
 * {12, 16, 24}, for about n / 40 or n / 20 sweeps), which damps the rough
 * start of its error (the correction starts from zero) faster; one is kept
 * when it saves over 5 % of the correction sweeps of a whole polish.
 * The FP64 sweeps (polish, hpf_sweeps64 with sweeps_per_pass = 0) get their
 * own tiling the same way, S in {2, 3, 4, 6, 8}.
 * out (host, optional, 10 doubles) receives [S, RH, omega, cell-updates per
 * second, S64, RH64, FP64 cell-updates per second, defect-correction
 * omega, correction start-phase omega, correction start-phase sweeps]
 * (sweeps 0: no start phase).
 * Blocking.  Errors: TWG_EINVAL, TWG_ENOMEM, TWG_EDEVICE. */
int32_t hpf_autotune(twg_ctx *ctx, twg_grid g, const uint8_t *cls, double *out, void *stream);

/* hpf_autotune_batched -- time the batched relaxation of this batch (n grid
 * descriptors and the packed class maps, as hpf_relax_batched takes them)
 * for the tilings (S, RH) = (4, 32), (6, 64), (8, 64), (6, 128), (8, 128):
 * each a whole solve from the 0.5 field to residual 1e-6 on a context-owned
 * field, timed with HIP events after an untimed set-up run.  The fastest is
 * remembered: later hpf_relax_batched(_async) calls on this context with
 * sweeps_per_pass = 0 use it (in place of the largest grid's single-grid
 * tiling).  Grids' SOR factors come from hpf_autotune of their sizes, as in
 * hpf_relax_batched.  out (host, optional, 3 doubles): [S, RH, ms of the
 * fastest].  Blocking.  Errors: TWG_EINVAL, TWG_ENOMEM, TWG_EDEVICE. */
int32_t hpf_autotune_batched(twg_ctx *ctx, int32_t n, const twg_grid_desc *grids, const uint8_t *cls,
                             double *out, void *stream);

/* hpf_set_tiling -- set, for grids of size nx x ny on this context, what
 * hpf_autotune would remember: FP32 sweeps per tile load S and rows per tile
 * RH, SOR factor omega (0 = the open-rectangle optimum), FP64 tiling S64 and
 * RH64 (S64 = 0: the FP64 default), and no start phase.  Host only.  Errors: TWG_EINVAL (S or
 * S64 not in 1 to 8, RH < 2, omega outside [0, 2)). */
int32_t hpf_set_tiling(twg_ctx *ctx, int32_t nx, int32_t ny, int32_t S, int32_t RH, float omega, int32_t S64,
                       int32_t RH64);

/* hpf_residual -- max over FREE cells of |avg4(u) + f - u| in FP64, where u
 * is psi64 if it is not NULL, else psi (FP32 values, FP64 arithmetic); f is
 * an optional FP32 source (NULL = 0).  *out is a host double.  Blocking. */
int32_t hpf_residual(twg_ctx *ctx, twg_grid g, const uint8_t *cls, const float *psi,
                     const double *psi64, const float *f, double *out, void *stream);

/* ========================================================================= */
/* Descent                                                                   */
/* ========================================================================= */

typedef struct {
    int32_t start_x, start_y; /* start cell (the robot) */
    int32_t cap;              /* capacity of path_xy in cells, >= 1 */
    int32_t reserved;
} hpf_descend_params;

/* hpf_index_matrix -- index matrix of Eq. (3): for every cell, the direction
 * of its FREE or GOAL neighbour with the lowest phi (highest psi), looked at
 * in the order E (x+1) = 0, W (x-1) = 1, S (y+1) = 2, N (y-1) = 3, the first
 * one winning a tie; 4 when no neighbour has a strictly higher psi than the
 * cell.  Compares psi64 if it is not NULL, else psi.  idx is a uint8 map
 * (device, pitch g.pitch).  Asynchronous.  Errors: TWG_EINVAL. */
int32_t hpf_index_matrix(twg_ctx *ctx, twg_grid g, const uint8_t *cls, const float *psi,
                         const double *psi64, uint8_t *idx, void *stream);

/* hpf_descend -- steepest-descent path (Algorithm 1: index matrix, then the
 * path from the robot's position).  From the start, repeatedly moves to the
 * neighbour given by the index matrix until a GOAL cell.  path_xy receives
 * (x, y) int32 pairs (device, 2 * cap), starting with the start cell.
 * info (device, 2 int32) receives [length, status] with status TWG_OK,
 * TWG_START_BLOCKED, TWG_NO_PATH (a cell with no strictly better neighbour:
 * the goal is unreachable or the field is not resolved there) or
 * TWG_PATH_TRUNCATED.  Asynchronous.  Errors: TWG_EINVAL (bad grid, start
 * outside the grid, cap < 1, NULL arrays). */
int32_t hpf_descend(twg_ctx *ctx, twg_grid g, const uint8_t *cls, const float *psi,
                    const double *psi64, const hpf_descend_params *params, int32_t *path_xy,
                    int32_t *info, void *stream);

/* hpf_descent_all -- the steepest descent of hpf_descend from every cell at
 * once: steps (device int32, row stride steps_pitch >= nx) receives, for each
 * FREE or GOAL cell, the number of moves its descent takes to reach a GOAL
 * cell (0 on GOAL cells), and -1 where the descent stops elsewhere (a cell
 * with no strictly better neighbour) or the cell is not walkable.  Computed
 * by pointer jumping over the index matrix (ceil(log2(nx ny)) rounds); on a
 * converged field every FREE cell connected to the goal gets a length
 * (discrete maximum principle).  Asynchronous.  Errors: TWG_EINVAL. */
int32_t hpf_descent_all(twg_ctx *ctx, twg_grid g, const uint8_t *cls, const float *psi, const double *psi64,
                        int32_t *steps, int32_t steps_pitch, void *stream);

/* hpf_rubber_band -- rubber-band smoothing of a path (section "Rubber Band
 * Model", Eqs. 4-6; Algorithm 1 "Path Planning").  The path's endpoints stay
 * fixed.  Each of `iters` iterations moves the interior points of odd index,
 * then those of even index, each to the best of the candidates c = p_i + d,
 * d in the order (0,0), E, W, S, N, (1,1), (-1,1), (1,-1), (-1,-1): in the
 * grid, FREE or GOAL, psi(c) > 0, and within one cell (Chebyshev) of both
 * neighbours, so the band stays 8-connected.  The best candidate minimises
 * |F + T|^2 with tension T = k ((p_{i-1} - c) + (p_{i+1} - c)) and potential
 * force F = -(1/psi(c) - 1/psi(p_i)) u, u the unit vector of d (F = 0 for
 * d = 0; 1/psi = 1/(1 - phi) as in Eq. 6, signed to resist moves towards
 * obstacles); the first candidate wins a tie.  Arithmetic is FP64 on psi64
 * if it is not NULL, else on psi widened to FP64.  path_xy (device, int32
 * (x, y) pairs, capacity cap) is updated in place; its length is read from
 * device memory at len[0] (e.g. hpf_descend's info).  Asynchronous.
 * Errors: TWG_EINVAL (bad grid, NULL arrays, cap < 1, iters < 0, k < 0 or
 * not finite). */
int32_t hpf_rubber_band(twg_ctx *ctx, twg_grid g, const uint8_t *cls, const float *psi, const double *psi64,
                        int32_t *path_xy, const int32_t *len, int32_t cap, double k, int32_t iters,
                        void *stream);

/* ========================================================================= */
/* Learned warm start (not in the paper: an initial field for hpf_relax)     */
/* ========================================================================= */

/* A small encoder-decoder network (4 levels, 32 base channels, 443,745
 * parameters) maps three input channels per cell -- occupancy (1 on OBST and
 * WALL), Euclidean distance to the goal / (max(nx, ny) sqrt 2), ring number /
 * largest ring -- to an initial psi.  Layers, in order (conv3 = 3x3
 * cross-correlation with zero padding 1 and a bias; pool = 2x2 mean; up = 2x
 * nearest; cat = channel concatenation):
 *   e0 = relu(conv3(x, 3->32)); e1 = relu(conv3(pool(e0), 32->64));
 *   e2 = relu(conv3(pool(e1), 64->128)); e3 = relu(conv3(pool(e2), 128->128));
 *   d2 = relu(conv3(cat(up(e3), e2), 256->64)); d1 = relu(conv3(cat(up(d2), e1), 128->32));
 *   d0 = relu(conv3(cat(up(d1), e0), 64->32)); y = conv1(d0, 32->1).
 * Every stored activation and the input are rounded to bf16 (nearest even);
 * products accumulate in FP32 on the matrix cores.  The relaxation always
 * finishes from the network's field, so results keep hpf_relax's tolerance.
 *
 * Parameter vectors (device, FP32, TWG_UNET_NUM_PARAMS entries) list the
 * layers in the order above, each as w[cout][cin][ky][kx] then b[cout].
 * Images are [batch][H][W] (x: [batch][H][W][3]), contiguous, H and W
 * multiples of 8, batch * H * W <= 2^28.  The network object owns its
 * parameters, optimiser state and activation buffers (allocated on first use
 * of a size); it must not be used by two streams at once. */
#define TWG_UNET_NUM_PARAMS 443745
typedef struct twg_unet twg_unet;

int32_t twg_unet_num_params(void);

/* Create a network on ctx's device with all parameters zero.  Errors:
 * TWG_EINVAL, TWG_ENOMEM, TWG_EDEVICE. */
int32_t twg_unet_create(twg_ctx *ctx, twg_unet **out);
int32_t twg_unet_destroy(twg_unet *net);

/* Load / read the parameters (device FP32 vector).  Loading resets the Adam
 * state.  Asynchronous. */
int32_t twg_unet_set_params(twg_unet *net, const float *params, void *stream);
int32_t twg_unet_get_params(twg_unet *net, float *params, void *stream);

/* y[b][h][w] = network output for input x[b][h][w][0..2] (device FP32).
 * Asynchronous.  Errors: TWG_EINVAL (shape, NULL), TWG_ENOMEM. */
int32_t twg_unet_forward(twg_unet *net, int32_t batch, int32_t H, int32_t W, const float *x, float *y,
                         void *stream);

/* Training loss and gradients: loss = mean over images of the mean over FREE
 * cells (cls[b][h][w] == TWG_CELL_FREE, uint8, device) of (y - target)^2;
 * *loss (device float) receives it.  The parameter gradients are kept for
 * twg_unet_adam_step and, if grads is not NULL, written there (device FP32,
 * parameter order).  Weight gradients are reduced in a fixed order
 * (deterministic).  Asynchronous. */
int32_t twg_unet_loss_grad(twg_unet *net, int32_t batch, int32_t H, int32_t W, const float *x,
                           const float *target, const uint8_t *cls, float *loss, float *grads,
                           void *stream);

/* One Adam step (b1 0.9, b2 0.999, eps 1e-8) with the gradients of the last
 * twg_unet_loss_grad.  Errors: TWG_EINVAL for lr outside (0, 1). */
int32_t twg_unet_adam_step(twg_unet *net, float lr, void *stream);

/* Network input channels of a grid, on an H x W frame (H >= ny, W >= nx,
 * multiples of 8; frame cells outside the grid read as walls), written to x
 * (device FP32 [H][W][3]).  ring may be NULL (ring channel 0).  Asynchronous. */
int32_t twg_unet_features(twg_unet *net, twg_grid g, const uint8_t *cls, const uint16_t *ring,
                          int32_t goal_x, int32_t goal_y, int32_t H, int32_t W, float *x, void *stream);

/* Warm start of one grid: features, network, and the field written to psi
 * (device FP32, pitch g.pitch): FREE cells clamp(y, 0, 1), OBST and WALL 0,
 * GOAL 1, FIXED cells unchanged.  If the network produces a non-finite value
 * at any FREE cell (e.g. NaN parameters), the network's field is rejected and
 * every FREE cell holds the plain start 0.5 (the paper's initial value)
 * instead; status (optional device int32, or NULL) receives TWG_OK or
 * TWG_NET_FALLBACK.  Follow with hpf_relax(init = HPF_INIT_KEEP).
 * Asynchronous; allocates nothing after the first call of a grid size (no
 * memset either), so it can be captured into a graph.  Errors: TWG_EINVAL
 * (bad grid, NULL cls or psi), TWG_ENOMEM. */
int32_t twg_unet_warm_start(twg_unet *net, twg_grid g, const uint8_t *cls, const uint16_t *ring,
                            int32_t goal_x, int32_t goal_y, float *psi, int32_t *status, void *stream);

/* Coarse-scale warm start: the network sees the grid at 1/factor of its
 * resolution (factor 2, 4, 8 or 16) on an Hc x Wc frame, the coarse sides
 * ceil(n / factor) rounded up to multiples of 8 (at least 8).  Coarse cell
 * (X, Y) covers the fine cells [factor X, factor X + factor) x [factor Y,
 * factor Y + factor), cells outside the grid reading as walls.  Its inputs:
 * occupancy = share of OBST, WALL and outside cells in the block; distance of
 * the block's centre (factor X + (factor - 1) / 2, ...) to the goal cell /
 * (max(nx, ny) sqrt 2); ring of the fine cell at (factor X + factor / 2,
 * factor Y + factor / 2), clamped into the grid, / largest ring (0 without a
 * ring map).  The network's output at that scale is interpolated back
 * (bilinear) to the grid's FREE cells. */

/* Hc and Wc of the coarse frame.  Host only.  Errors: TWG_EINVAL. */
int32_t twg_unet_coarse_frame(twg_grid g, int32_t factor, int32_t *Hc, int32_t *Wc);

/* Coarse input channels of a grid: x (device FP32 [Hc][Wc][3], or NULL) and
 * ccls (device uint8 [Hc][Wc], or NULL), the mask of the training loss:
 * TWG_CELL_FREE where the block holds a FREE cell, else TWG_CELL_OBST.
 * Asynchronous.  Errors: TWG_EINVAL. */
int32_t twg_unet_features_coarse(twg_unet *net, twg_grid g, const uint8_t *cls, const uint16_t *ring,
                                 int32_t goal_x, int32_t goal_y, int32_t factor, float *x, uint8_t *ccls,
                                 void *stream);

/* Coarse training target: out[Y][X] (device FP32 [Hc][Wc]) = the mean of psi
 * (device FP32, pitch g.pitch) over the FREE cells of block (X, Y), summed in
 * row order in FP32; 0 when the block has none.  Asynchronous.  Errors:
 * TWG_EINVAL. */
int32_t twg_unet_coarse_target(twg_unet *net, twg_grid g, const uint8_t *cls, const float *psi, int32_t factor,
                               float *out, void *stream);

/* Warm start of one grid from the network run at the coarse scale: coarse
 * features, network, then each FREE cell (x, y) of psi takes the bilinear
 * interpolation of the coarse output y at ((x + 1/2) / factor - 1/2,
 * (y + 1/2) / factor - 1/2), clamped to the frame, then to [0, 1]; OBST and
 * WALL 0, GOAL 1, FIXED unchanged; the same fallback and status as
 * twg_unet_warm_start.  Asynchronous.  Errors: TWG_EINVAL, TWG_ENOMEM. */
int32_t twg_unet_warm_start_coarse(twg_unet *net, twg_grid g, const uint8_t *cls, const uint16_t *ring,
                                   int32_t goal_x, int32_t goal_y, int32_t factor, float *psi, int32_t *status,
                                   void *stream);

#ifdef __cplusplus
}
#endif
#endif /* TWG_H */
