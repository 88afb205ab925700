/*
 * twg_oracle.c -- plain, slow, FP64 CPU oracle for the harmonic-potential-field
 * path on the time-warped grid (Farzan & DeSouza, "Path Planning in Dynamic
 * Environments Using Time-Warped Grids and a Parallel Implementation").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * path: the cell-class codes and status codes below are restated here on
 * purpose, from the same published definitions.
 *
 * Conventions (the readings of the paper this oracle takes):
 *   - Grids are row-major, x fastest, a[y*nx + x], no padding.
 *   - The field is stored as psi = 1 - phi (phi is the paper's potential):
 *     the goal holds psi = 1, obstacles and walls psi = 0.  The Laplace
 *     equation is linear, so psi is harmonic exactly where phi is.
 *   - A neighbour outside the grid counts as a fixed cell with psi = 0
 *     (an obstacle beyond the map's edge).
 *   - Cell classes: FREE 0, OBST 1, WALL 2, GOAL 3, FIXED 4 (fixed at the
 *     value the caller put in the field).  Precedence WALL > GOAL > OBST.
 *
 * Build: gcc -O2 -std=c11 -fopenmp -ffp-contract=off -fPIC -shared.
 * Contraction is off so that every product and sum is rounded once, exactly
 * as written.  OpenMP only splits rows inside one colour of a red-black sweep
 * and rows of the per-cell passes, which does not change any result.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { O_FREE = 0, O_OBST = 1, O_WALL = 2, O_GOAL = 3, O_FIXED = 4 };
enum { O_OK = 0, O_NOT_CONVERGED = 1, O_NO_PATH = 2, O_START_BLOCKED = 3,
       O_PATH_TRUNCATED = 5 };

/* ------------------------------------------------------------------------ */
/* Integer helpers                                                          */
/* ------------------------------------------------------------------------ */

/* Largest s with s*s <= n, by the classical digit-by-digit (base 4) method.
 * No floating point is involved, so the result is exact for every n. */
uint64_t orc_isqrt(uint64_t n)
{
    uint64_t rem = n, root = 0, bit = (uint64_t)1 << 62;
    while (bit > rem) bit >>= 2;
    while (bit != 0) {
        if (rem >= root + bit) {
            rem -= root + bit;
            root = (root >> 1) + bit;
        } else {
            root >>= 1;
        }
        bit >>= 2;
    }
    return root;
}

static int64_t floor_div(int64_t a, int64_t b) /* b > 0 */
{
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) q -= 1;
    return q;
}

/* ------------------------------------------------------------------------ */
/* Time rings (section "Time-Warped Grid", isotropic case of Eqs. 14-15)    */
/* ------------------------------------------------------------------------ */

/* Ring ("warp") number of cell (x, y) for a robot at (xr, yr): the index of
 * the annulus of width W cells that holds the cell's centre,
 *     j = floor( |(x, y) - (xr, yr)| / W ),
 * evaluated exactly as isqrt(dx^2 + dy^2) / W in integers. */
int32_t orc_ring_of(int64_t dx, int64_t dy, int32_t W)
{
    uint64_t d2 = (uint64_t)(dx * dx) + (uint64_t)(dy * dy);
    return (int32_t)(orc_isqrt(d2) / (uint64_t)W);
}

void orc_ring_map(int32_t nx, int32_t ny, int32_t xr, int32_t yr, int32_t W,
                  uint16_t *ring)
{
#pragma omp parallel for schedule(static)
    for (int32_t y = 0; y < ny; ++y)
        for (int32_t x = 0; x < nx; ++x)
            ring[(size_t)y * nx + x] =
                (uint16_t)orc_ring_of((int64_t)x - xr, (int64_t)y - yr, W);
}

/* Elliptical warp metric (Eqs. 14-15).  The ellipse through a point has its
 * centre 0.9 r_x ahead of the robot along the heading (hc, hs) and r_x = 4
 * r_y; with u = hc dx + hs dy and v = hs dx - hc dy relative to the robot,
 * Eq. (15) becomes r_x^2 = (u - 0.9 r_x)^2 + 16 v^2, whose positive root is
 *     r_x = (-1.8 u + sqrt(4 u^2 + 12.16 v^2)) / 0.38.
 * The ring j = floor(r_x / W) is decided without rounding a root: r_x >= j W
 * exactly when sqrt(4u^2 + 12.16v^2) >= 0.38 j W + 1.8 u, i.e. when the right
 * side is <= 0 or 4u^2 + 12.16v^2 >= (0.38 j W + 1.8 u)^2.  Every term is one
 * rounded IEEE operation, and the test is monotone in j. */
static int ellipse_reaches(double u, double v, int32_t j, int32_t W)
{
    const double q = 4.0 * (u * u) + 12.16 * (v * v);
    const double rhs = 0.38 * ((double)j * (double)W) + 1.8 * u;
    return rhs <= 0.0 || q >= rhs * rhs;
}

int32_t orc_ring_ellipse(int64_t dx, int64_t dy, double hc, double hs, int32_t W)
{
    const double u = hc * (double)dx + hs * (double)dy;
    const double v = hs * (double)dx - hc * (double)dy;
    /* estimate from the rounded root, then settle on the exact test */
    const double r = (-1.8 * u + sqrt(4.0 * (u * u) + 12.16 * (v * v))) / 0.38;
    int32_t j = (r > 0.0 && r < 1e9) ? (int32_t)(r / (double)W) : 0;
    while (j > 0 && !ellipse_reaches(u, v, j, W)) --j;
    while (ellipse_reaches(u, v, j + 1, W)) ++j;
    return j;
}

/* Ring of a cell in either mode: 0 circular (isotropic), 1 elliptical. */
static int32_t ring_any(int64_t dx, int64_t dy, int32_t W, int32_t mode, double hc, double hs)
{
    return mode == 1 ? orc_ring_ellipse(dx, dy, hc, hs, W) : orc_ring_of(dx, dy, W);
}

void orc_ring_map_mode(int32_t nx, int32_t ny, int32_t xr, int32_t yr, int32_t W, int32_t mode,
                       double hc, double hs, uint16_t *ring)
{
#pragma omp parallel for schedule(static)
    for (int32_t y = 0; y < ny; ++y)
        for (int32_t x = 0; x < nx; ++x)
            ring[(size_t)y * nx + x] =
                (uint16_t)ring_any((int64_t)x - xr, (int64_t)y - yr, W, mode, hc, hs);
}

/* Number of rings that touch the grid: one more than the largest ring
 * number, which is reached at one of the four corners. */
int32_t orc_num_rings(int32_t nx, int32_t ny, int32_t xr, int32_t yr, int32_t W)
{
    int32_t m = 0;
    int32_t cx[2] = {0, nx - 1}, cy[2] = {0, ny - 1};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            int32_t j = orc_ring_of((int64_t)cx[a] - xr, (int64_t)cy[b] - yr, W);
            if (j > m) m = j;
        }
    return m + 1;
}

/* Horizon of ring j: the time the robot, moving at vr cells per step, needs
 * to reach the ring's inner edge (the "next j-th step" reading of the
 * time-warp number, with the ring width as the unit of distance). */
double orc_ring_time(int32_t j, int32_t W, double vr)
{
    return ((double)j * (double)W) / vr;
}

/* ------------------------------------------------------------------------ */
/* Kalman prediction (Eqs. 9-10, constant-velocity model of the experiments) */
/* ------------------------------------------------------------------------ */

/* Predicted mean position after a horizon t: Eq. (9) with the
 * constant-velocity state matrix whose time step is t,
 *     x_hat = A(t) x,  A(t) = [[I, t I], [0, I]],  B = 0,
 * so the position part is p + t v (one product, one sum, each rounded). */
void orc_predict_mean(const double p[2], const double v[2], double t, double mu[2])
{
    for (int k = 0; k < 2; ++k) {
        double tv = t * v[k];
        mu[k] = p[k] + tv;
    }
}

/* Eqs. (9)-(10) applied literally 'steps' times with a time step dt:
 *     x <- A x,   P <- A P A^T + Q,
 * with full 4x4 matrix products.  State order [x, y, vx, vy]; P and Q are
 * row-major 4x4.  Used to pin the closed-form horizon prediction above. */
void orc_kalman_predict_steps(double x[4], double P[16], double dt, int32_t steps,
                              const double Q[16])
{
    double A[16] = {1, 0, dt, 0,
                    0, 1, 0, dt,
                    0, 0, 1, 0,
                    0, 0, 0, 1};
    for (int32_t s = 0; s < steps; ++s) {
        double nx4[4], AP[16], nP[16];
        for (int i = 0; i < 4; ++i) {
            double acc = 0.0;
            for (int k = 0; k < 4; ++k) acc += A[i * 4 + k] * x[k];
            nx4[i] = acc;
        }
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                double acc = 0.0;
                for (int k = 0; k < 4; ++k) acc += A[i * 4 + k] * P[k * 4 + j];
                AP[i * 4 + j] = acc;
            }
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                double acc = 0.0;
                for (int k = 0; k < 4; ++k) acc += AP[i * 4 + k] * A[j * 4 + k];
                nP[i * 4 + j] = acc + (Q ? Q[i * 4 + j] : 0.0);
            }
        memcpy(x, nx4, sizeof nx4);
        memcpy(P, nP, sizeof nP);
    }
}

/* Eqs. (11)-(13) for the position-only measurement H = [I 0]:
 *     K = P H^T (H P H^T + R)^-1,  x <- x + K (z - H x),  P <- (I - K H) P.
 * The 2x2 inverse is written out.  R is row-major 2x2. */
void orc_kalman_update(double x[4], double P[16], const double z[2], const double R[4])
{
    double S[4] = {P[0] + R[0], P[1] + R[1], P[4] + R[2], P[5] + R[3]};
    double det = S[0] * S[3] - S[1] * S[2];
    double Si[4] = {S[3] / det, -S[1] / det, -S[2] / det, S[0] / det};
    double K[8]; /* 4x2 = P[:, 0:2] * Si */
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 2; ++j)
            K[i * 2 + j] = P[i * 4 + 0] * Si[0 * 2 + j] + P[i * 4 + 1] * Si[1 * 2 + j];
    double innov[2] = {z[0] - x[0], z[1] - x[1]};
    for (int i = 0; i < 4; ++i) x[i] = x[i] + (K[i * 2 + 0] * innov[0] + K[i * 2 + 1] * innov[1]);
    double nP[16];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            nP[i * 4 + j] = P[i * 4 + j] - (K[i * 2 + 0] * P[0 * 4 + j] + K[i * 2 + 1] * P[1 * 4 + j]);
    memcpy(P, nP, sizeof nP);
}

/* Position covariance after a horizon t for the constant-velocity model:
 * the 2x2 position block of A(t) P A(t)^T,
 *     P_pos(t) = P_pp + t (P_pv + P_vp) + t^2 P_vv,
 * entries a = [0][0], b = [0][1], d = [1][1] (P row-major 4x4, state
 * [x, y, vx, vy]); summed as ((P_pp + t (P_pv + P_vp)) + (t t) P_vv). */
void orc_pos_cov(const double P[16], double t, double out[3])
{
    const double tt = t * t;
    out[0] = (P[0] + t * (P[2] + P[8])) + tt * P[10];
    out[1] = (P[1] + t * (P[3] + P[9])) + tt * P[11];
    out[2] = (P[5] + t * (P[7] + P[13])) + tt * P[15];
}

/* Disc radius with covariance inflation (reading of the paper's Gaussian
 * marking): r + min(W, kappa sqrt(lambda_max(P_pos(t)))), lambda_max =
 * (a + d) / 2 + sqrt(((a - d) / 2)^2 + b^2).  kappa = 0 or P = NULL: r. */
double orc_inflated_radius(double r, const double *P, double t, double kappa, int32_t W)
{
    if (!(kappa > 0.0) || !P) return r;
    double c[3];
    orc_pos_cov(P, t, c);
    const double h = (c[0] - c[2]) * 0.5;
    const double lam = (c[0] + c[2]) * 0.5 + sqrt(h * h + c[1] * c[1]);
    double g = kappa * sqrt(lam > 0.0 ? lam : 0.0);
    if (!(g <= (double)W)) g = (double)W; /* also catches NaN */
    return r + g;
}

/* ------------------------------------------------------------------------ */
/* Marking predicted poses on the grid (Algorithm 1, "Map Update")          */
/* ------------------------------------------------------------------------ */

/* Fixed-point Q.8 coordinate of a predicted position: round-to-nearest-even
 * of 256*mu.  Returns 0 and leaves *q alone when |256*mu| >= 2^40 (the disc
 * is then far outside any supported grid and is ignored). */
static int q8(double mu, int64_t *q)
{
    double s = 256.0 * mu;
    if (!(fabs(s) < 1099511627776.0)) return 0;
    *q = (int64_t)nearbyint(s);
    return 1;
}

/* Does the disc of Q.8 centre (cx, cy) and Q.8 radius R contain the centre
 * of cell (x, y)?  Inclusive, in exact 64-bit integers. */
static int disc_covers(int32_t x, int32_t y, int64_t cx, int64_t cy, int64_t R)
{
    int64_t dx = 256 * (int64_t)x - cx, dy = 256 * (int64_t)y - cy;
    if (dx > R || dx < -R || dy > R || dy < -R) return 0;
    return dx * dx + dy * dy <= R * R;
}

/* An obstacle radius is usable when it is a finite number in [0, 1e6]
 * cells; other obstacles are skipped (input-validity rule of the library). */
static int radius_ok(double r) { return r >= 0.0 && r <= 1e6; }

static uint8_t base_class(int32_t nx, int32_t ny, int32_t x, int32_t y,
                          int32_t xg, int32_t yg, int32_t border_walls)
{
    if (border_walls && (x == 0 || y == 0 || x == nx - 1 || y == ny - 1)) return O_WALL;
    if (x == xg && y == yg) return O_GOAL;
    return O_FREE;
}

/* All-pairs definition: each cell takes its own ring j, the ring's horizon
 * t_j, and tests every obstacle's disc predicted at t_j.  Static occupancy
 * (nonzero bytes of static_occ, may be NULL) marks OBST as well. */
void orc_rasterize_allpairs(int32_t nx, int32_t ny, int32_t xr, int32_t yr,
                            int32_t xg, int32_t yg, int32_t W, double vr,
                            int32_t border_walls, int32_t n_obs,
                            const double *pos, const double *vel, const double *rad,
                            const uint8_t *static_occ, uint8_t *cls, uint16_t *ring)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t y = 0; y < ny; ++y) {
        for (int32_t x = 0; x < nx; ++x) {
            size_t idx = (size_t)y * nx + x;
            int32_t j = orc_ring_of((int64_t)x - xr, (int64_t)y - yr, W);
            if (ring) ring[idx] = (uint16_t)j;
            uint8_t c = base_class(nx, ny, x, y, xg, yg, border_walls);
            if (c == O_FREE && static_occ && static_occ[idx]) c = O_OBST;
            if (c == O_FREE) {
                double t = orc_ring_time(j, W, vr);
                for (int32_t i = 0; i < n_obs; ++i) {
                    double mu[2];
                    int64_t cx, cy;
                    if (!radius_ok(rad[i])) continue;
                    orc_predict_mean(&pos[2 * i], &vel[2 * i], t, mu);
                    if (!q8(mu[0], &cx) || !q8(mu[1], &cy)) continue;
                    int64_t R = (int64_t)nearbyint(256.0 * rad[i]);
                    if (disc_covers(x, y, cx, cy, R)) { c = O_OBST; break; }
                }
            }
            cls[idx] = c;
        }
    }
}

/* All modes, all-pairs definition.
 *   ring_mode   0 circular rings, 1 elliptical warp metric (heading (hc, hs)).
 *   per_object  0: each cell sees every obstacle at its own ring's horizon;
 *               1 (Algorithm 1): obstacle i is predicted once, to the horizon
 *               of the ring of the cell nearest its current centre (round
 *               half to even), and its disc is marked on every ring.
 *   kappa, cov  covariance inflation (cov: n_obs x 16 doubles or NULL). */
void orc_rasterize_modes(int32_t nx, int32_t ny, int32_t xr, int32_t yr, int32_t xg, int32_t yg,
                         int32_t W, double vr, int32_t border_walls, int32_t n_obs, const double *pos,
                         const double *vel, const double *rad, const uint8_t *static_occ,
                         int32_t ring_mode, double hc, double hs, int32_t per_object, double kappa,
                         const double *cov, uint8_t *cls, uint16_t *ring)
{
    /* per-object discs, computed once */
    int64_t *ocx = (int64_t *)malloc((size_t)(n_obs > 0 ? n_obs : 1) * 3 * sizeof(int64_t));
    uint8_t *ook = (uint8_t *)calloc((size_t)(n_obs > 0 ? n_obs : 1), 1);
    if (per_object) {
        for (int32_t i = 0; i < n_obs; ++i) {
            if (!radius_ok(rad[i])) continue;
            const double px = nearbyint(pos[2 * i]), py = nearbyint(pos[2 * i + 1]);
            if (!(fabs(px) < 1e9) || !(fabs(py) < 1e9)) continue;
            const int32_t j = ring_any((int64_t)px - xr, (int64_t)py - yr, W, ring_mode, hc, hs);
            const double t = orc_ring_time(j, W, vr);
            double mu[2];
            int64_t cx, cy;
            orc_predict_mean(&pos[2 * i], &vel[2 * i], t, mu);
            if (!q8(mu[0], &cx) || !q8(mu[1], &cy)) continue;
            const double re = orc_inflated_radius(rad[i], cov ? cov + 16 * (size_t)i : NULL, t, kappa, W);
            ocx[3 * i] = cx;
            ocx[3 * i + 1] = cy;
            ocx[3 * i + 2] = (int64_t)nearbyint(256.0 * re);
            ook[i] = 1;
        }
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t y = 0; y < ny; ++y) {
        for (int32_t x = 0; x < nx; ++x) {
            size_t idx = (size_t)y * nx + x;
            int32_t j = ring_any((int64_t)x - xr, (int64_t)y - yr, W, ring_mode, hc, hs);
            if (ring) ring[idx] = (uint16_t)j;
            uint8_t c = base_class(nx, ny, x, y, xg, yg, border_walls);
            if (c == O_FREE && static_occ && static_occ[idx]) c = O_OBST;
            if (c == O_FREE) {
                double t = orc_ring_time(j, W, vr);
                for (int32_t i = 0; i < n_obs; ++i) {
                    int64_t cx, cy, R;
                    if (per_object) {
                        if (!ook[i]) continue;
                        cx = ocx[3 * i];
                        cy = ocx[3 * i + 1];
                        R = ocx[3 * i + 2];
                    } else {
                        double mu[2];
                        if (!radius_ok(rad[i])) continue;
                        orc_predict_mean(&pos[2 * i], &vel[2 * i], t, mu);
                        if (!q8(mu[0], &cx) || !q8(mu[1], &cy)) continue;
                        const double re =
                            orc_inflated_radius(rad[i], cov ? cov + 16 * (size_t)i : NULL, t, kappa, W);
                        R = (int64_t)nearbyint(256.0 * re);
                    }
                    if (disc_covers(x, y, cx, cy, R)) { c = O_OBST; break; }
                }
            }
            cls[idx] = c;
        }
    }
    free(ocx);
    free(ook);
}

/* Same result, organised per obstacle: for every (obstacle, ring) pair the
 * disc's bounding box is scanned and cells of that ring inside the disc are
 * marked.  Kept as a second, independent route to the same definition. */
void orc_rasterize_perobs(int32_t nx, int32_t ny, int32_t xr, int32_t yr,
                          int32_t xg, int32_t yg, int32_t W, double vr,
                          int32_t border_walls, int32_t n_obs,
                          const double *pos, const double *vel, const double *rad,
                          const uint8_t *static_occ, uint8_t *cls, uint16_t *ring)
{
    size_t n = (size_t)nx * ny;
    uint16_t *rg = ring ? ring : (uint16_t *)malloc(n * sizeof(uint16_t));
    uint8_t *occ = (uint8_t *)calloc(n, 1);
    orc_ring_map(nx, ny, xr, yr, W, rg);
    int32_t J = orc_num_rings(nx, ny, xr, yr, W);
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t i = 0; i < n_obs; ++i) {
        if (!radius_ok(rad[i])) continue;
        int64_t R = (int64_t)nearbyint(256.0 * rad[i]);
        for (int32_t j = 0; j < J; ++j) {
            double mu[2];
            int64_t cx, cy;
            orc_predict_mean(&pos[2 * i], &vel[2 * i], orc_ring_time(j, W, vr), mu);
            if (!q8(mu[0], &cx) || !q8(mu[1], &cy)) continue;
            /* cells whose Q.8 centre 256*x lies in [cx - R, cx + R] */
            int64_t x0 = -floor_div(-(cx - R), 256), x1 = floor_div(cx + R, 256);
            int64_t y0 = -floor_div(-(cy - R), 256), y1 = floor_div(cy + R, 256);
            if (x0 < 0) x0 = 0;
            if (y0 < 0) y0 = 0;
            if (x1 > nx - 1) x1 = nx - 1;
            if (y1 > ny - 1) y1 = ny - 1;
            for (int64_t y = y0; y <= y1; ++y)
                for (int64_t x = x0; x <= x1; ++x) {
                    size_t idx = (size_t)y * nx + x;
                    if (rg[idx] == j && disc_covers((int32_t)x, (int32_t)y, cx, cy, R))
                        occ[idx] = 1; /* same byte from every writer */
                }
        }
    }
#pragma omp parallel for schedule(static)
    for (int32_t y = 0; y < ny; ++y)
        for (int32_t x = 0; x < nx; ++x) {
            size_t idx = (size_t)y * nx + x;
            uint8_t c = base_class(nx, ny, x, y, xg, yg, border_walls);
            if (c == O_FREE && ((static_occ && static_occ[idx]) || occ[idx])) c = O_OBST;
            cls[idx] = c;
        }
    free(occ);
    if (!ring) free(rg);
}

/* ------------------------------------------------------------------------ */
/* Harmonic potential (Eqs. 1-2; boundary values of "Harmonic Potential     */
/* Fields")                                                                 */
/* ------------------------------------------------------------------------ */

static inline double at(const double *a, int32_t nx, int32_t ny, int32_t x, int32_t y)
{
    if (x < 0 || y < 0 || x >= nx || y >= ny) return 0.0;
    return a[(size_t)y * nx + x];
}

/* Average of the four neighbours, summed in the fixed order
 * ((E + W) + (S + N)) and scaled by 1/4 (exact). */
static inline double avg4(const double *a, int32_t nx, int32_t ny, int32_t x, int32_t y)
{
    double ew = at(a, nx, ny, x + 1, y) + at(a, nx, ny, x - 1, y);
    double sn = at(a, nx, ny, x, y + 1) + at(a, nx, ny, x, y - 1);
    return (ew + sn) * 0.25;
}

/* Dirichlet values: goal phi = 0 (psi = 1), obstacle and wall phi = 1
 * (psi = 0), FIXED cells keep the caller's value.  Free cells: mode 0 keeps
 * the input, 1 sets phi = 0.5 (the paper's initial value), 2 sets psi = 0,
 * 3 a linear ramp in the distance to the goal cell (gx, gy): psi = 1 - d /
 * (max(nx, ny) sqrt 2), d = sqrt(dx^2 + dy^2) (a starting field that falls
 * from the goal's value; max(nx, ny) sqrt 2 bounds any distance on the grid). */
void orc_field_init(int32_t nx, int32_t ny, const uint8_t *cls, double *psi, int32_t mode,
                    int32_t gx, int32_t gy)
{
    const double span = (double)(nx > ny ? nx : ny) * sqrt(2.0);
    for (int32_t y = 0; y < ny; ++y)
        for (int32_t x = 0; x < nx; ++x) {
            size_t i = (size_t)y * nx + x;
            switch (cls[i]) {
            case O_OBST: case O_WALL: psi[i] = 0.0; break;
            case O_GOAL: psi[i] = 1.0; break;
            case O_FREE:
                if (mode == 1) psi[i] = 0.5;
                else if (mode == 2) psi[i] = 0.0;
                else if (mode == 3) {
                    double dx = (double)(x - gx), dy = (double)(y - gy);
                    psi[i] = 1.0 - sqrt(dx * dx + dy * dy) / span;
                }
                break;
            default: break;
            }
        }
}

/* Residual of the discrete Laplace equation (the change one step of Eq. 1
 * would make) with an optional source f:  r = avg4(psi) + f - psi  on FREE
 * cells.  Returns max |r| over FREE cells; 0 when there are none. */
double orc_residual(int32_t nx, int32_t ny, const uint8_t *cls, const double *psi,
                    const double *f)
{
    double rmax = 0.0;
#pragma omp parallel for schedule(static) reduction(max : rmax) if ((int64_t)nx * ny > 65536)
    for (int32_t y = 0; y < ny; ++y)
        for (int32_t x = 0; x < nx; ++x) {
            size_t idx = (size_t)y * nx + x;
            if (cls[idx] != O_FREE) continue;
            double g = avg4(psi, nx, ny, x, y);
            if (f) g = g + f[idx];
            double r = fabs(g - psi[idx]);
            if (r > rmax) rmax = r;
        }
    return rmax;
}

/* Residual field r = avg4(psi) + f - psi on FREE cells, 0 elsewhere. */
void orc_residual_field(int32_t nx, int32_t ny, const uint8_t *cls, const double *psi,
                        const double *f, double *r)
{
#pragma omp parallel for schedule(static) if ((int64_t)nx * ny > 65536)
    for (int32_t y = 0; y < ny; ++y)
        for (int32_t x = 0; x < nx; ++x) {
            size_t idx = (size_t)y * nx + x;
            if (cls[idx] != O_FREE) { r[idx] = 0.0; continue; }
            double g = avg4(psi, nx, ny, x, y);
            if (f) g = g + f[idx];
            r[idx] = g - psi[idx];
        }
}

/* One red-black SOR sweep: red cells ((x + y) even) first, then black, each
 * FREE cell set to psi + omega * (avg4(psi) + f - psi).  With omega = 1 this
 * is Gauss-Seidel in red-black order: the in-place use of already updated
 * neighbours of Eq. (2), with a different visiting order.  The update is
 * evaluated as
 *     d = fma(1/4, ((E + W) + N) + S, f - psi),   psi' = fma(omega, d, psi)
 * (N the row above, S the row below, f = 0 without a source), one rounding
 * per operation; the GPU's FP64 sweeps use the same expression. */
void orc_sor_sweep(int32_t nx, int32_t ny, const uint8_t *cls, double *psi,
                   const double *f, double omega)
{
    for (int color = 0; color < 2; ++color) {
#pragma omp parallel for schedule(static) if ((int64_t)nx * ny > 65536)
        for (int32_t y = 0; y < ny; ++y)
            for (int32_t x = (y + color) & 1; x < nx; x += 2) {
                size_t idx = (size_t)y * nx + x;
                if (cls[idx] != O_FREE) continue;
                double e = at(psi, nx, ny, x + 1, y), w = at(psi, nx, ny, x - 1, y);
                double n = at(psi, nx, ny, x, y - 1), s = at(psi, nx, ny, x, y + 1);
                double sum = ((e + w) + n) + s;
                double rest = f ? f[idx] - psi[idx] : -psi[idx];
                double d = fma(0.25, sum, rest);
                psi[idx] = fma(omega, d, psi[idx]);
            }
    }
}

/* One Jacobi step, Eq. (1), written out: every FREE cell becomes the average
 * of its neighbours' previous values. */
void orc_jacobi_step(int32_t nx, int32_t ny, const uint8_t *cls, double *psi)
{
    size_t n = (size_t)nx * ny;
    double *old = (double *)malloc(n * sizeof(double));
    memcpy(old, psi, n * sizeof(double));
    for (int32_t y = 0; y < ny; ++y)
        for (int32_t x = 0; x < nx; ++x) {
            size_t idx = (size_t)y * nx + x;
            if (cls[idx] == O_FREE) psi[idx] = avg4(old, nx, ny, x, y);
        }
    free(old);
}

/* One lexicographic Gauss-Seidel step, Eq. (2), written out: cells visited
 * row by row, x fastest, each using the already updated left and upper
 * neighbours. */
void orc_gs_lex_step(int32_t nx, int32_t ny, const uint8_t *cls, double *psi)
{
    for (int32_t y = 0; y < ny; ++y)
        for (int32_t x = 0; x < nx; ++x) {
            size_t idx = (size_t)y * nx + x;
            if (cls[idx] == O_FREE) psi[idx] = avg4(psi, nx, ny, x, y);
        }
}

/* Cheap, rigorous bound on ||(I - J)^-1 1||_inf for any class map on an
 * nx-by-ny grid: the discrete maximum principle bounds the solution of
 * (I - J) w = 1 (w = 0 on fixed cells and outside the grid) by the
 * supersolution 2 (x + 1)(nx - x), whose maximum is (nx + 1)^2 / 2, and the
 * same in y. */
double orc_wbound(int32_t nx, int32_t ny)
{
    double n = (double)(nx < ny ? nx : ny) + 1.0;
    return n * n / 2.0;
}

/* Red-black SOR from the given field until, at a check every check_every
 * sweeps, the residual r satisfies r <= tol and (if tol_cert > 0)
 * r * orc_wbound <= tol_cert; or max_sweeps is reached.  The certificate is
 * the maximum-principle error bound |psi - psi*| <= r * ||(I-J)^-1 1||.
 * out[0] = sweeps, out[1] = final residual, out[2] = certified error bound.
 * Returns 0 when converged, 1 when max_sweeps ran out. */
int32_t orc_relax(int32_t nx, int32_t ny, const uint8_t *cls, double *psi,
                  const double *f, double omega, double tol, double tol_cert,
                  int64_t max_sweeps, int32_t check_every, double *out)
{
    double wb = orc_wbound(nx, ny);
    int64_t sweeps = 0;
    double r = orc_residual(nx, ny, cls, psi, f);
    int32_t status = O_NOT_CONVERGED;
    for (;;) {
        if (r <= tol && (tol_cert <= 0.0 || r * wb <= tol_cert)) { status = O_OK; break; }
        if (sweeps >= max_sweeps) break;
        for (int32_t k = 0; k < check_every && sweeps < max_sweeps; ++k, ++sweeps)
            orc_sor_sweep(nx, ny, cls, psi, f, omega);
        r = orc_residual(nx, ny, cls, psi, f);
    }
    if (out) { out[0] = (double)sweeps; out[1] = r; out[2] = r * wb; }
    return status;
}

/* ------------------------------------------------------------------------ */
/* Index matrix and steepest descent (Eq. 3, Algorithm 1 "Path Planning")   */
/* ------------------------------------------------------------------------ */

static int walkable(uint8_t c) { return c == O_FREE || c == O_GOAL; }

/* Index-matrix entry of a cell: among its in-grid walkable neighbours taken
 * in the order E (x+1), W (x-1), S (y+1), N (y-1), the one with the lowest
 * phi, i.e. the highest psi; the first one wins a tie.  Returns the
 * direction 0..3, or 4 when no neighbour has a strictly higher psi than the
 * cell itself. */
int32_t orc_index_of(int32_t nx, int32_t ny, const uint8_t *cls, const double *psi,
                     int32_t x, int32_t y)
{
    static const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};
    int32_t best = 4;
    double bv = 0.0;
    for (int d = 0; d < 4; ++d) {
        int32_t xx = x + dx[d], yy = y + dy[d];
        if (xx < 0 || yy < 0 || xx >= nx || yy >= ny) continue;
        size_t k = (size_t)yy * nx + xx;
        if (!walkable(cls[k])) continue;
        if (best == 4 || psi[k] > bv) { best = d; bv = psi[k]; }
    }
    if (best != 4 && !(bv > psi[(size_t)y * nx + x])) best = 4;
    return best;
}

void orc_index_matrix(int32_t nx, int32_t ny, const uint8_t *cls, const double *psi,
                      uint8_t *idx_out)
{
#pragma omp parallel for schedule(static)
    for (int32_t y = 0; y < ny; ++y)
        for (int32_t x = 0; x < nx; ++x)
            idx_out[(size_t)y * nx + x] = (uint8_t)orc_index_of(nx, ny, cls, psi, x, y);
}

/* Follow the index matrix from (sx, sy) until the goal.  The path holds the
 * start and every visited cell, as (x, y) pairs, at most cap cells.
 * Returns OK, START_BLOCKED (start not FREE or GOAL), NO_PATH (a cell with
 * no strictly better neighbour), or PATH_TRUNCATED (cap reached). */
int32_t orc_descend(int32_t nx, int32_t ny, const uint8_t *cls, const double *psi,
                    int32_t sx, int32_t sy, int32_t cap, int32_t *path, int32_t *len)
{
    static const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};
    *len = 0;
    if (sx < 0 || sy < 0 || sx >= nx || sy >= ny) return -1;
    uint8_t c0 = cls[(size_t)sy * nx + sx];
    if (!walkable(c0)) return O_START_BLOCKED;
    int32_t x = sx, y = sy, n = 0;
    if (cap < 1) return O_PATH_TRUNCATED;
    path[0] = x; path[1] = y; n = 1;
    for (;;) {
        if (cls[(size_t)y * nx + x] == O_GOAL) { *len = n; return O_OK; }
        int32_t d = orc_index_of(nx, ny, cls, psi, x, y);
        if (d == 4) { *len = n; return O_NO_PATH; }
        x += dx[d]; y += dy[d];
        if (n >= cap) { *len = n; return O_PATH_TRUNCATED; }
        path[2 * n] = x; path[2 * n + 1] = y; ++n;
    }
}

/* Is a GOAL cell 4-connected to (sx, sy) through walkable cells?  Plain
 * breadth-first search. */
int32_t orc_goal_reachable(int32_t nx, int32_t ny, const uint8_t *cls, int32_t sx, int32_t sy)
{
    static const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};
    size_t n = (size_t)nx * ny, head = 0, tail = 0;
    if (sx < 0 || sy < 0 || sx >= nx || sy >= ny) return 0;
    if (!walkable(cls[(size_t)sy * nx + sx])) return 0;
    uint8_t *seen = (uint8_t *)calloc(n, 1);
    int32_t *q = (int32_t *)malloc(n * sizeof(int32_t));
    int32_t found = 0;
    q[tail++] = sy * nx + sx;
    seen[(size_t)sy * nx + sx] = 1;
    while (head < tail) {
        int32_t k = q[head++];
        int32_t x = k % nx, y = k / nx;
        if (cls[k] == O_GOAL) { found = 1; break; }
        for (int d = 0; d < 4; ++d) {
            int32_t xx = x + dx[d], yy = y + dy[d];
            if (xx < 0 || yy < 0 || xx >= nx || yy >= ny) continue;
            size_t kk = (size_t)yy * nx + xx;
            if (seen[kk] || !walkable(cls[kk])) continue;
            seen[kk] = 1;
            q[tail++] = (int32_t)kk;
        }
    }
    free(seen);
    free(q);
    return found;
}

/* ------------------------------------------------------------------------ */
/* Rubber band (Eqs. 4-6, "Rubber Band Model"; Algorithm 1 "Path Planning")  */
/* ------------------------------------------------------------------------ */

/* The paper leaves the candidate set and the vector form of F open; the
 * reading taken here:
 *   - the band acts on an extracted path p_0 .. p_{n-1}; its endpoints (the
 *     robot and the goal) stay fixed;
 *   - one iteration updates the interior points of odd index, then those of
 *     even index, each from the current positions of its two neighbours;
 *   - candidates for point i are c = p_i + d, d in the order (0,0), E, W, S,
 *     N, (1,1), (-1,1), (1,-1), (-1,-1): in the grid, walkable, psi(c) > 0,
 *     and within one cell (Chebyshev) of both neighbours, so the band stays
 *     8-connected;
 *   - tension from the neighbours T = k ((p_{i-1} - c) + (p_{i+1} - c));
 *   - potential force F = -(1 / psi(c) - 1 / psi(p_i)) u, u the unit vector
 *     of d (F = 0 for d = 0); 1 / psi = 1 / (1 - phi) as in Eq. (6), signed
 *     so that it resists moves towards obstacles (lower psi);
 *   - the point moves to the candidate with the smallest |F + T|^2 (Eq. 4),
 *     the first one in order on a tie (Eq. 5 moves it one cell at most).
 * Points whose own psi is not positive do not move.
 * Parity unpinned beyond its properties (fixed endpoints, walkable and
 * 8-connected points, zero tension keeps the path, tension straightens a
 * bump, the force resists moves towards obstacles): Eq. (6) is garbled and
 * this reading is a heuristic. */
static const int rb_dx[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
static const int rb_dy[9] = {0, 0, 0, 1, -1, 1, 1, -1, -1};

static int32_t iabs32(int32_t v) { return v < 0 ? -v : v; }

void orc_rubber_band(int32_t nx, int32_t ny, const uint8_t *cls, const double *psi, int32_t *path,
                     int32_t n, double k, int32_t iters)
{
    const double inv_sqrt2 = 0.70710678118654752440;
    for (int32_t it = 0; it < iters; ++it) {
        for (int32_t color = 1; color >= 0; --color) {
            for (int32_t i = 1; i + 1 < n; ++i) {
                if ((i & 1) != color) continue;
                const int32_t px = path[2 * i], py = path[2 * i + 1];
                const int32_t ax = path[2 * i - 2], ay = path[2 * i - 1];
                const int32_t bx = path[2 * i + 2], by = path[2 * i + 3];
                const double p0 = psi[(size_t)py * nx + px];
                if (!(p0 > 0.0)) continue;
                const double g0 = 1.0 / p0;
                int32_t best = -1;
                double bestv = 0.0;
                for (int d = 0; d < 9; ++d) {
                    const int32_t cx = px + rb_dx[d], cy = py + rb_dy[d];
                    if (cx < 0 || cy < 0 || cx >= nx || cy >= ny) continue;
                    const size_t c = (size_t)cy * nx + cx;
                    if (!walkable(cls[c]) || !(psi[c] > 0.0)) continue;
                    if (iabs32(cx - ax) > 1 || iabs32(cy - ay) > 1 || iabs32(cx - bx) > 1 || iabs32(cy - by) > 1)
                        continue;
                    const double tx = k * (double)((ax - cx) + (bx - cx));
                    const double ty = k * (double)((ay - cy) + (by - cy));
                    double fx = 0.0, fy = 0.0;
                    if (d > 0) {
                        const double m = -(1.0 / psi[c] - g0);
                        const double u = (rb_dx[d] != 0 && rb_dy[d] != 0) ? inv_sqrt2 : 1.0;
                        fx = m * ((double)rb_dx[d] * u);
                        fy = m * ((double)rb_dy[d] * u);
                    }
                    const double rx = fx + tx, ry = fy + ty;
                    const double v = rx * rx + ry * ry;
                    if (best < 0 || v < bestv) { best = d; bestv = v; }
                }
                if (best > 0) {
                    path[2 * i] = px + rb_dx[best];
                    path[2 * i + 1] = py + rb_dy[best];
                }
            }
        }
    }
}
