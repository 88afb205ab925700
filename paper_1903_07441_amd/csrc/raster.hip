// Map update on the time-warped grid (Algorithm 1, "Map Update"; sections
// "Time-Warped Grid" and "Integration of Kalman Filter with Time-Warps").
//
//   k_raster_base  one thread per cell: ring number and the WALL / GOAL /
//                  static-OBST / FREE class.
//   k_pairs        one thread per (obstacle, ring): the constant-velocity
//                  Kalman prediction of Eq. (9) to the ring's horizon, its Q.8
//                  disc (optionally grown by the predicted position
//                  covariance), and a conservative test of whether the disc can
//                  touch the ring and the grid; survivors are appended to a
//                  list.  With the per-object horizon of Algorithm 1, one
//                  thread per obstacle, at the horizon of its own ring.
//   k_scatter      one workgroup per listed pair: exact integer test of every
//                  cell of the disc's bounding box (ring match + inside the
//                  disc); FREE cells become OBST.  Every writer stores the same
//                  byte, so the result does not depend on the order.
//
// Exactness: the horizon, the product and the sum of the prediction are each
// rounded once (contraction is off for this file), 256*mu is exact, and the
// Q.8 rounding is round-half-to-even; the inside test is in 64-bit integers.
#include "twg_internal.h"

namespace twg {

namespace {

struct Pair {
    long long cx, cy, R;  // Q.8 centre and radius
    int j;                // ring
    int pad;
};

__device__ __forceinline__ int dev_isqrt(long long n)
{
    long long s = (long long)sqrt((double)n);
    while (s * s > n) --s;
    while ((s + 1) * (s + 1) <= n) ++s;
    return (int)s;
}

__device__ __forceinline__ int ring_of(long long dx, long long dy, int W)
{
    return dev_isqrt(dx * dx + dy * dy) / W;
}

// Elliptical warp metric (Eqs. 14-15): relative to the robot, with heading
// (hc, hs), u = hc dx + hs dy and v = hs dx - hc dy; the ellipse through the
// cell has its centre 0.9 r_x ahead and r_x = 4 r_y, so
// r_x = (-1.8 u + sqrt(4 u^2 + 12.16 v^2)) / 0.38.  Ring j = floor(r_x / W)
// is settled by the exact, monotone test r_x >= j W  <=>  0.38 j W + 1.8 u
// <= 0 or 4 u^2 + 12.16 v^2 >= (0.38 j W + 1.8 u)^2 (each term one rounded
// IEEE operation, so host and device agree bit for bit).
__host__ __device__ inline bool ellipse_reaches(double u, double v, int j, int W)
{
    const double q = 4.0 * (u * u) + 12.16 * (v * v);
    const double rhs = 0.38 * ((double)j * (double)W) + 1.8 * u;
    return rhs <= 0.0 || q >= rhs * rhs;
}

__host__ __device__ inline int ring_ellipse(long long dx, long long dy, double hc, double hs, int W)
{
    const double u = hc * (double)dx + hs * (double)dy;
    const double v = hs * (double)dx - hc * (double)dy;
    const double r = (-1.8 * u + sqrt(4.0 * (u * u) + 12.16 * (v * v))) / 0.38;  // estimate only
    int j = (r > 0.0 && r < 1e9) ? (int)(r / (double)W) : 0;
    while (j > 0 && !ellipse_reaches(u, v, j, W)) --j;
    while (ellipse_reaches(u, v, j + 1, W)) ++j;
    return j;
}

struct WarpMode {
    int ring_mode;  // 0 circular, 1 elliptical
    double hc, hs;  // heading
};

__device__ __forceinline__ int ring_any(long long dx, long long dy, int W, const WarpMode &m)
{
    return m.ring_mode == 1 ? ring_ellipse(dx, dy, m.hc, m.hs, W) : ring_of(dx, dy, W);
}

// Disc radius with covariance inflation: r + min(W, kappa sqrt(lambda_max)),
// lambda_max the larger eigenvalue of the position covariance after horizon
// t, P_pos(t) = P_pp + t (P_pv + P_vp) + t^2 P_vv (P row-major 4x4, state
// [x, y, vx, vy]).  kappa = 0 or no covariance: r.
__device__ __forceinline__ double inflated_radius(double r, const double *P, double t, double kappa, int W)
{
    if (!(kappa > 0.0) || !P) return r;
    const double tt = t * t;
    const double a = (P[0] + t * (P[2] + P[8])) + tt * P[10];
    const double b = (P[1] + t * (P[3] + P[9])) + tt * P[11];
    const double d = (P[5] + t * (P[7] + P[13])) + tt * P[15];
    const double h = (a - d) * 0.5;
    const double lam = (a + d) * 0.5 + sqrt(h * h + b * b);
    double g = kappa * sqrt(lam > 0.0 ? lam : 0.0);
    if (!(g <= (double)W)) g = (double)W;
    return r + g;
}

__device__ __forceinline__ long long floor_div256(long long a)
{
    return a >= 0 ? a / 256 : -((-a + 255) / 256);
}

__global__ void k_raster_base(int nx, int ny, int pitch, int xr, int yr, int xg, int yg, int W,
                              int border, WarpMode wm, const uint8_t *__restrict__ static_occ,
                              uint8_t *__restrict__ cls, uint16_t *__restrict__ ring)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= nx || y >= ny) return;
    const size_t i = (size_t)y * pitch + x;
    uint8_t c = TWG_CELL_FREE;
    if (border && (x == 0 || y == 0 || x == nx - 1 || y == ny - 1)) c = TWG_CELL_WALL;
    else if (x == xg && y == yg) c = TWG_CELL_GOAL;
    else if (static_occ && static_occ[i]) c = TWG_CELL_OBST;
    cls[i] = c;
    if (ring) ring[i] = (uint16_t)ring_any(x - xr, y - yr, W, wm);
}

// Per-cell horizon: one thread per (obstacle, ring) pair j < J; the disc
// predicted to ring j's horizon is listed with ring j (its cells of ring j are
// marked).  Per-object horizon (Algorithm 1): one thread per obstacle; the
// disc predicted to the horizon of the ring of the cell nearest the
// obstacle's current centre is listed with ring -1 (all its cells marked).
__global__ void k_pairs(int n_obs, int J, int per_object, const double *__restrict__ pos,
                        const double *__restrict__ vel, const double *__restrict__ rad,
                        const double *__restrict__ cov, double kappa, WarpMode wm, int W, double vr, int nx,
                        int ny, int xr, int yr, Pair *__restrict__ list, unsigned int *count)
{
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long long)n_obs * (per_object ? 1 : J)) return;
    const int i = per_object ? (int)id : (int)(id / J);
    const double r = rad[i];
    if (!(r >= 0.0 && r <= 1e6)) return;
    int j;
    if (per_object) {
        const double px = rint(pos[2 * i]), py = rint(pos[2 * i + 1]);
        if (!(fabs(px) < 1e9) || !(fabs(py) < 1e9)) return;
        j = ring_any((long long)px - xr, (long long)py - yr, W, wm);
    } else {
        j = (int)(id % J);
    }
    // Eq. (9) with A(t): position p + t v, each operation rounded once
    const double t = ((double)j * (double)W) / vr;
    const double tvx = t * vel[2 * i], tvy = t * vel[2 * i + 1];
    const double mx = pos[2 * i] + tvx, my = pos[2 * i + 1] + tvy;
    const double sx = 256.0 * mx, sy = 256.0 * my;
    if (!(fabs(sx) < 1099511627776.0) || !(fabs(sy) < 1099511627776.0)) return;
    const long long cx = (long long)rint(sx), cy = (long long)rint(sy);
    const double re = inflated_radius(r, cov ? cov + 16 * (size_t)i : nullptr, t, kappa, W);
    const long long R = (long long)rint(256.0 * re);
    // disc must reach the grid
    if (cx + R < 0 || cx - R > 256LL * (nx - 1) || cy + R < 0 || cy - R > 256LL * (ny - 1)) return;
    if (!per_object) {
        // ...and ring j: cells of the disc lie within R of its centre; ring j
        // holds Euclidean distances [jW, (j+1)W) (circular) or, since the
        // elliptical r_x lies between d / 1.9 and 10 d, [jW / 10, 1.9 (j+1) W)
        // (elliptical); two cells of margin absorb rounding
        const double dx = (double)cx / 256.0 - xr, dy = (double)cy / 256.0 - yr;
        const double D = sqrt(dx * dx + dy * dy), Rc = (double)R / 256.0;
        const double lo = wm.ring_mode == 1 ? (double)j * W / 10.0 : (double)j * W;
        const double hi = wm.ring_mode == 1 ? 1.9 * (double)(j + 1) * W : (double)(j + 1) * W;
        if (D - Rc - 2.0 >= hi) return;
        if (D + Rc + 2.0 < lo) return;
    }
    const unsigned slot = atomicAdd(count, 1u);
    Pair p;
    p.cx = cx; p.cy = cy; p.R = R; p.j = per_object ? -1 : j; p.pad = 0;
    list[slot] = p;
}

__global__ __launch_bounds__(256) void k_scatter(const Pair *__restrict__ list,
                                                 const unsigned int *__restrict__ count, int nx,
                                                 int ny, int pitch, int xr, int yr, int W, WarpMode wm,
                                                 uint8_t *cls)
{
    const unsigned n = *count;
    for (unsigned e = blockIdx.x; e < n; e += gridDim.x) {
        const Pair p = list[e];
        long long x0 = -floor_div256(-(p.cx - p.R)), x1 = floor_div256(p.cx + p.R);
        long long y0 = -floor_div256(-(p.cy - p.R)), y1 = floor_div256(p.cy + p.R);
        if (x0 < 0) x0 = 0;
        if (y0 < 0) y0 = 0;
        if (x1 > nx - 1) x1 = nx - 1;
        if (y1 > ny - 1) y1 = ny - 1;
        if (x1 < x0 || y1 < y0) continue;
        const long long w = x1 - x0 + 1, total = w * (y1 - y0 + 1);
        for (long long k = threadIdx.x; k < total; k += blockDim.x) {
            const int x = (int)(x0 + k % w), y = (int)(y0 + k / w);
            if (p.j >= 0 && ring_any(x - xr, y - yr, W, wm) != p.j) continue;
            const long long dx = 256LL * x - p.cx, dy = 256LL * y - p.cy;
            if (dx * dx + dy * dy <= p.R * p.R) {
                const size_t i = (size_t)y * pitch + x;
                if (cls[i] == TWG_CELL_FREE) cls[i] = TWG_CELL_OBST;
            }
        }
    }
}

__global__ void k_zero_u32(unsigned int *w) { *w = 0u; }

int host_ring(long long dx, long long dy, int W)
{
    unsigned long long d2 = (unsigned long long)(dx * dx + dy * dy);
    unsigned long long s = (unsigned long long)std::sqrt((double)d2);
    while (s * s > d2) --s;
    while ((s + 1) * (s + 1) <= d2) ++s;
    return (int)(s / (unsigned long long)W);
}

}  // namespace

int launch_rasterize(twg_ctx *ctx, const twg_grid &g, int n_obs, const double *pos,
                     const double *vel, const double *rad, const uint8_t *static_occ,
                     const twg_raster_params &p, uint8_t *cls, uint16_t *ring, hipStream_t st)
{
    const int nx = g.nx, ny = g.ny, pitch = g.pitch;
    const WarpMode wm{p.ring_mode, p.heading_x, p.heading_y};
    // rings touching the grid: the metric is convex in the offset (a norm
    // plus a linear term), so the largest ring is reached at a corner
    int J = 0;
    const int cxs[2] = {0, nx - 1}, cys[2] = {0, ny - 1};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const long long dx = cxs[a] - p.robot_x, dy = cys[b] - p.robot_y;
            const int j = p.ring_mode == 1 ? ring_ellipse(dx, dy, wm.hc, wm.hs, p.ring_width)
                                           : host_ring(dx, dy, p.ring_width);
            if (j > J) J = j;
        }
    if (J > 65535) return set_err(ctx, TWG_EUNSUPPORTED, "more than 65536 rings: increase ring_width");
    J += 1;
    hipLaunchKernelGGL(k_raster_base, dim3((nx + 63) / 64, (ny + 3) / 4), dim3(256), 0, st, nx, ny,
                       pitch, p.robot_x, p.robot_y, p.goal_x, p.goal_y, p.ring_width,
                       p.border_walls, wm, static_occ, cls, ring);
    if (hipGetLastError() != hipSuccess) return set_err(ctx, TWG_EDEVICE, "k_raster_base launch failed");
    if (n_obs == 0) return TWG_OK;
    const long long pairs = (long long)n_obs * (p.per_object ? 1 : J);
    const size_t need = (size_t)pairs * sizeof(Pair);
    int rc = ensure(ctx, &ctx->pairs, &ctx->pairs_bytes, need);
    if (rc) return rc;
    unsigned int *count = reinterpret_cast<unsigned int *>(ctx->words + 32);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, count);
    hipLaunchKernelGGL(k_pairs, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, st, n_obs, J,
                       p.per_object, pos, vel, rad, p.cov, p.kappa, wm, p.ring_width, p.robot_speed, nx, ny,
                       p.robot_x, p.robot_y, reinterpret_cast<Pair *>(ctx->pairs), count);
    hipLaunchKernelGGL(k_scatter, dim3(1024), dim3(256), 0, st,
                       reinterpret_cast<const Pair *>(ctx->pairs), count, nx, ny, pitch, p.robot_x,
                       p.robot_y, p.ring_width, wm, cls);
    if (hipGetLastError() != hipSuccess) return set_err(ctx, TWG_EDEVICE, "rasterize launch failed");
    return TWG_OK;
}

}  // namespace twg
