// Index matrix (Eq. 3) and steepest-descent path extraction (Algorithm 1,
// "Path Planning": index matrix, then the path from the robot's position).
//
//   k_index  one thread per cell: direction (E 0, W 1, S 2, N 3) of the
//            walkable neighbour with the highest psi (lowest phi), first one
//            on ties; 4 when none is strictly higher than the cell itself.
//   k_walk   one workgroup follows the index matrix from the start.  The
//            64 x 64 window of index codes and classes around the current
//            cell is staged in LDS by all 256 threads; one thread then walks
//            inside the window (each step strictly raises psi, so the walk
//            never revisits a cell) and the window is re-centred when the
//            walk leaves it.
#include "twg_internal.h"

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

constexpr int kTile = 64;

__global__ __launch_bounds__(256) void k_walk(const uint8_t *__restrict__ cls,
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

}  // namespace

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
    hipLaunchKernelGGL(k_walk, dim3(1), dim3(256), 0, st, cls, idx, nx, ny, pitch, sx, sy, cap, path,
                       info);
    return hipGetLastError() == hipSuccess ? TWG_OK : TWG_EDEVICE;
}

}  // namespace twg
