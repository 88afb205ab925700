// Index matrix (Eq. 3) and steepest-descent path extraction (Algorithm 1,
// "Path Planning": index matrix, then the path from the robot's position).
//
//   k_index  one thread per cell: direction (E 0, W 1, S 2, N 3) of the
//            walkable neighbour with the highest psi (lowest phi), first one
//            on ties; 4 when none is strictly higher than the cell itself.
//   k_walk   one workgroup follows the index matrix from the start.  The
//            128 x 128 window of index codes and classes around the current
//            cell is staged in LDS by all 1024 threads; one thread then walks
//            inside the window (each step strictly raises psi, so the walk
//            never revisits a cell) and the window is re-centred when the
//            walk leaves it.
//   k_rubber one workgroup relaxes a path as a rubber band (Eqs. 4-6): per
//            iteration the interior points of odd index, then those of even
//            index, each move to the best of nine candidate cells given the
//            positions of their two neighbours (see hpf_rubber_band).
#include "twg_internal.h"

#include <utility>

namespace twg {

namespace {

__device__ __forceinline__ bool walkable(uint8_t c)
{
    return c == TWG_CELL_FREE || c == TWG_CELL_GOAL;
}

template <typename T>
__global__ void k_index(const uint8_t *__restrict__ cls, const T *__restrict__ u,
                        uint8_t *__restrict__ idx, int nx, int ny, int pitch)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= nx || y >= ny) return;
    const size_t i = (size_t)y * pitch + x;
    const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};
    int best = 4;
    T bv = T(0);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const int xx = x + dx[d], yy = y + dy[d];
        if (xx < 0 || yy < 0 || xx >= nx || yy >= ny) continue;
        const size_t k = (size_t)yy * pitch + xx;
        if (!walkable(cls[k])) continue;
        const T v = u[k];
        if (best == 4 || v > bv) {
            best = d;
            bv = v;
        }
    }
    if (best != 4 && !(bv > u[i])) best = 4;
    idx[i] = (uint8_t)best;
}

constexpr int kTile = 128;

__global__ __launch_bounds__(1024) void k_walk(const uint8_t *__restrict__ cls,
                                              const uint8_t *__restrict__ idx, int nx, int ny,
                                              int pitch, int sx, int sy, int cap,
                                              int32_t *__restrict__ path, int32_t *__restrict__ info)
{
    __shared__ uint8_t tidx[kTile * kTile];
    __shared__ uint8_t tcls[kTile * kTile];
    __shared__ int state[4];  // x, y, length, status (-1 = walking)
    if (threadIdx.x == 0) {
        const uint8_t c = cls[(size_t)sy * pitch + sx];
        state[0] = sx;
        state[1] = sy;
        if (!walkable(c)) {
            state[2] = 0;
            state[3] = TWG_START_BLOCKED;
        } else {
            path[0] = sx;
            path[1] = sy;
            state[2] = 1;
            state[3] = -1;
        }
    }
    __syncthreads();
    const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};
    while (state[3] < 0) {
        const int tx0 = state[0] - kTile / 2, ty0 = state[1] - kTile / 2;
        for (int k = threadIdx.x; k < kTile * kTile; k += blockDim.x) {
            const int x = tx0 + (k & (kTile - 1)), y = ty0 + k / kTile;
            uint8_t d = 4, c = TWG_CELL_WALL;
            if (x >= 0 && y >= 0 && x < nx && y < ny) {
                const size_t i = (size_t)y * pitch + x;
                d = idx[i];
                c = cls[i];
            }
            tidx[k] = d;
            tcls[k] = c;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int x = state[0], y = state[1], n = state[2], st = -1;
            for (;;) {
                const int lx = x - tx0, ly = y - ty0;
                if (lx < 0 || ly < 0 || lx >= kTile || ly >= kTile) break;
                const int k = ly * kTile + lx;
                if (tcls[k] == TWG_CELL_GOAL) { st = TWG_OK; break; }
                const int d = tidx[k];
                if (d == 4) { st = TWG_NO_PATH; break; }
                x += dx[d];
                y += dy[d];
                if (n >= cap) { st = TWG_PATH_TRUNCATED; break; }
                path[2 * n] = x;
                path[2 * n + 1] = y;
                ++n;
            }
            state[0] = x;
            state[1] = y;
            state[2] = n;
            state[3] = st;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        info[0] = state[2];
        info[1] = state[3];
    }
}

// Descent from every cell by pointer jumping over the index matrix: nxt[c]
// is the cell one descent step from c (c itself at a GOAL cell or where the
// index matrix has no move), len[c] the steps taken so far.  Each round
// doubles the steps covered: nxt'[c] = nxt[nxt[c]], len'[c] = len[c] +
// len[nxt[c]] (ping-pong buffers, so the rounds are order-free).  Descent
// strictly raises psi, so the chains have no cycles and ceil(log2(cells))
// rounds reach their ends.
__global__ void k_jump_init(const uint8_t *__restrict__ cls, const uint8_t *__restrict__ idx, int nx, int ny,
                            int pitch, int *__restrict__ nxt, int *__restrict__ len)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= nx || y >= ny) return;
    const int c = y * nx + x;
    const size_t i = (size_t)y * pitch + x;
    const uint8_t k = cls[i];
    const int d = idx[i];
    int n = c, l = 0;
    if (walkable(k) && k != TWG_CELL_GOAL && d < 4) {
        const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};
        n = (y + dy[d]) * nx + (x + dx[d]);
        l = 1;
    }
    nxt[c] = n;
    len[c] = l;
}

__global__ void k_jump(int total, const int *__restrict__ na, const int *__restrict__ la, int *__restrict__ nb,
                       int *__restrict__ lb)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= total) return;
    const int n = na[c];
    nb[c] = na[n];
    lb[c] = la[c] + la[n];
}

// steps[c] = descent length to a GOAL cell, or -1 (not walkable, or the
// descent ends elsewhere)
__global__ void k_jump_final(const uint8_t *__restrict__ cls, int nx, int ny, int pitch,
                             const int *__restrict__ nxt, const int *__restrict__ len, int32_t *__restrict__ steps,
                             int pitch_out)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= nx || y >= ny) return;
    const int c = y * nx + x;
    const int e = nxt[c];
    const bool ok = walkable(cls[(size_t)y * pitch + x]) &&
                    cls[(size_t)(e / nx) * pitch + (e % nx)] == TWG_CELL_GOAL;
    steps[(size_t)y * pitch_out + x] = ok ? len[c] : -1;
}

// Candidate offsets: stay, E, W, S, N, then the diagonals.
__constant__ int kRbDx[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
__constant__ int kRbDy[9] = {0, 0, 0, 1, -1, 1, 1, -1, -1};

template <typename T>
__global__ __launch_bounds__(1024) void k_rubber(const uint8_t *__restrict__ cls, const T *__restrict__ u,
                                                 int32_t *__restrict__ path, const int32_t *__restrict__ len,
                                                 int cap, int nx, int ny, int pitch, double k, int iters)
{
    const int n = min(*len, cap);
    const double inv_sqrt2 = 0.70710678118654752440;
    for (int it = 0; it < iters; ++it) {
        for (int color = 1; color >= 0; --color) {
            // points of this colour read only points of the other colour
            for (int i = 1 + (color ^ 1) + 2 * (int)threadIdx.x; i + 1 < n; i += 2 * (int)blockDim.x) {
                const int px = path[2 * i], py = path[2 * i + 1];
                const int ax = path[2 * i - 2], ay = path[2 * i - 1];
                const int bx = path[2 * i + 2], by = path[2 * i + 3];
                const double p0 = (double)u[(size_t)py * pitch + px];
                if (!(p0 > 0.0)) continue;
                const double g0 = 1.0 / p0;
                int best = -1;
                double bestv = 0.0;
                for (int d = 0; d < 9; ++d) {
                    const int cx = px + kRbDx[d], cy = py + kRbDy[d];
                    if (cx < 0 || cy < 0 || cx >= nx || cy >= ny) continue;
                    const size_t c = (size_t)cy * pitch + cx;
                    const double pc = (double)u[c];
                    if (!walkable(cls[c]) || !(pc > 0.0)) continue;
                    if (abs(cx - ax) > 1 || abs(cy - ay) > 1 || abs(cx - bx) > 1 || abs(cy - by) > 1) continue;
                    const double tx = k * (double)((ax - cx) + (bx - cx));
                    const double ty = k * (double)((ay - cy) + (by - cy));
                    double fx = 0.0, fy = 0.0;
                    if (d > 0) {
                        const double m = -(1.0 / pc - g0);
                        const double w = (kRbDx[d] != 0 && kRbDy[d] != 0) ? inv_sqrt2 : 1.0;
                        fx = m * ((double)kRbDx[d] * w);
                        fy = m * ((double)kRbDy[d] * w);
                    }
                    const double rx = fx + tx, ry = fy + ty;
                    const double v = rx * rx + ry * ry;
                    if (best < 0 || v < bestv) {
                        best = d;
                        bestv = v;
                    }
                }
                if (best > 0) {
                    path[2 * i] = px + kRbDx[best];
                    path[2 * i + 1] = py + kRbDy[best];
                }
            }
            __syncthreads();
        }
    }
}

}  // namespace

int launch_rubber(const uint8_t *cls, const float *psi, const double *psi64, int32_t *path, const int32_t *len,
                  int cap, int nx, int ny, int pitch, double k, int iters, hipStream_t st)
{
    if (psi64)
        hipLaunchKernelGGL(k_rubber<double>, dim3(1), dim3(1024), 0, st, cls, psi64, path, len, cap, nx, ny, pitch, k,
                           iters);
    else
        hipLaunchKernelGGL(k_rubber<float>, dim3(1), dim3(1024), 0, st, cls, psi, path, len, cap, nx, ny, pitch, k,
                           iters);
    return hipGetLastError() == hipSuccess ? TWG_OK : TWG_EDEVICE;
}

int launch_descent_all(const uint8_t *cls, const uint8_t *idx, int nx, int ny, int pitch, int *buf,
                       int32_t *steps, int pitch_out, hipStream_t st)
{
    const int total = nx * ny;
    int *na = buf, *la = buf + total, *nb = buf + 2 * (size_t)total, *lb = buf + 3 * (size_t)total;
    const dim3 grid((nx + 63) / 64, (ny + 3) / 4);
    hipLaunchKernelGGL(k_jump_init, grid, dim3(256), 0, st, cls, idx, nx, ny, pitch, na, la);
    int rounds = 1;
    while ((1LL << rounds) < (long long)total) ++rounds;
    for (int r = 0; r < rounds; ++r) {
        hipLaunchKernelGGL(k_jump, dim3((total + 255) / 256), dim3(256), 0, st, total, na, la, nb, lb);
        std::swap(na, nb);
        std::swap(la, lb);
    }
    hipLaunchKernelGGL(k_jump_final, grid, dim3(256), 0, st, cls, nx, ny, pitch, na, la, steps, pitch_out);
    return hipGetLastError() == hipSuccess ? TWG_OK : TWG_EDEVICE;
}

int launch_index(const uint8_t *cls, const float *psi, const double *psi64, uint8_t *idx, int nx,
                 int ny, int pitch, hipStream_t st)
{
    const dim3 grid((nx + 63) / 64, (ny + 3) / 4);
    if (psi64)
        hipLaunchKernelGGL(k_index<double>, grid, dim3(256), 0, st, cls, psi64, idx, nx, ny, pitch);
    else
        hipLaunchKernelGGL(k_index<float>, grid, dim3(256), 0, st, cls, psi, idx, nx, ny, pitch);
    return hipGetLastError() == hipSuccess ? TWG_OK : TWG_EDEVICE;
}

int launch_walk(const uint8_t *cls, const uint8_t *idx, int nx, int ny, int pitch, int sx, int sy,
                int cap, int32_t *path, int32_t *info, hipStream_t st)
{
    hipLaunchKernelGGL(k_walk, dim3(1), dim3(1024), 0, st, cls, idx, nx, ny, pitch, sx, sy, cap, path,
                       info);
    return hipGetLastError() == hipSuccess ? TWG_OK : TWG_EDEVICE;
}

}  // namespace twg
