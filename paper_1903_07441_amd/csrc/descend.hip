// Index matrix (Eq. 3) and steepest-descent path extraction (Algorithm 1,
// "Path Planning": index matrix, then the path from the robot's position).
//
//   k_index  one thread per cell: direction (E 0, W 1, S 2, N 3) of the
//            walkable neighbour with the highest psi (lowest phi), first one
//            on ties; 4 when none is strictly higher than the cell itself.
//   k_walk   one workgroup follows the index matrix from the start, reading
//            the walk codes (the index code, 5 on GOAL cells), turned into
//            in-window moves, from a 256 x 256 LDS window around the current
//            cell (see k_walk).
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

// WALK: the walk's code instead of the index matrix: 5 on GOAL cells, else
// the index code (so the walk reads one byte per step).
constexpr uint8_t kGoalCode = 5;
template <typename T, bool WALK>
__global__ void k_index(const uint8_t *__restrict__ cls, const T *__restrict__ u,
                        uint8_t *__restrict__ idx, int nx, int ny, int pitch)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= nx || y >= ny) return;
    const size_t i = (size_t)y * pitch + x;
    // every neighbour's class and value are loaded (clamped to the grid)
    // before any is compared, so no load waits inside a divergent branch
    const int xs[4] = {min(x + 1, nx - 1), max(x - 1, 0), x, x};
    const int ys[4] = {y, y, min(y + 1, ny - 1), max(y - 1, 0)};
    const bool inside[4] = {x + 1 < nx, x > 0, y + 1 < ny, y > 0};
    uint8_t c[4];
    T v[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const size_t k = (size_t)ys[d] * pitch + xs[d];
        c[d] = cls[k];
        v[d] = u[k];
    }
    const T self = u[i];
    int best = 4;
    T bv = T(0);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const bool ok = inside[d] && walkable(c[d]) && (best == 4 || v[d] > bv);
        best = ok ? d : best;
        bv = ok ? v[d] : bv;
    }
    if (best != 4 && !(bv > self)) best = 4;
    idx[i] = WALK && cls[i] == TWG_CELL_GOAL ? kGoalCode : (uint8_t)best;
}

constexpr int kTile = 256;

// Four walk codes (one per byte) to four 16-bit moves: the byte offset of the
// neighbour inside the 256-cell-wide LDS window (E +2, W -2, S +512, N -512),
// 0 for the codes 4 (no move) and 5 (goal).  v_perm_b32 looks the low and the
// high bytes up in two 4-byte tables (selectors 4 to 7 pick the zero word),
// then interleaves them.
__device__ __forceinline__ uint2 walk_moves(uint32_t codes)
{
    const uint32_t lo = __builtin_amdgcn_perm(0u, 0x0000fe02u, codes);
    const uint32_t hi = __builtin_amdgcn_perm(0u, 0xfe02ff00u, codes);
    return make_uint2(__builtin_amdgcn_perm(hi, lo, 0x05010400u), __builtin_amdgcn_perm(hi, lo, 0x07030602u));
}

// code: the walk codes of k_index<T, true> (direction, 4 = no move, 5 =
// goal).  The 256 x 256 window around the current cell is staged in LDS by
// all 1024 threads as 16-bit moves (unconditional loads: cells outside the
// grid read a clamped cell and become 4), with the window's border ring set
// to 0 so that no move leaves it.  The first wave then walks with every lane
// in step: per step one broadcast LDS read, a zero test and an add (each
// step strictly raises psi, so the walk never revisits a cell); lane k keeps
// the k-th cell of the current group of 64, stored in one coalesced write per
// group.  A 0 move ends the group: its cell's code, read from memory, tells
// the goal, a cell with no move, and the window's edge apart (at the edge the
// step is taken and the window is re-centred on the new cell).
__global__ __launch_bounds__(1024) void k_walk(const uint8_t *__restrict__ cls,
                                              const uint8_t *__restrict__ code, int nx, int ny,
                                              int pitch, int sx, int sy, int cap,
                                              int32_t *__restrict__ path, int32_t *__restrict__ info)
{
    __shared__ __align__(16) uint16_t tmove[kTile * kTile];
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
    while (state[3] < 0) {
        // window origin on a multiple of 16 columns, so that with pitch a
        // multiple of 16 (else 4) every 16-cell (4-cell) group is one
        // aligned 128-bit (32-bit) load; all of a thread's loads are issued
        // before its first LDS store, so a restage costs one memory latency,
        // not one per load
        const int tx0 = (state[0] - kTile / 2) & ~15, ty0 = state[1] - kTile / 2;
        if ((pitch & 15) == 0) {
            constexpr int PER = kTile * kTile / 16 / 1024;
            uint4 v[PER];
#pragma unroll
            for (int r = 0; r < PER; ++r) {
                const int q = threadIdx.x + r * 1024;  // 16-cell group
                const int x = tx0 + 16 * (q & (kTile / 16 - 1)), y = ty0 + q / (kTile / 16);
                const int xc = min(max(x, 0), pitch - 16), yc = min(max(y, 0), ny - 1);
                const uint4 w = *reinterpret_cast<const uint4 *>(code + (size_t)yc * pitch + xc);
                const uint32_t wv[4] = {w.x, w.y, w.z, w.w};
                uint32_t o[4];
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    o[h] = 0;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int xe = x + 4 * h + e;
                        const bool in = xe >= 0 && xe < nx && y >= 0 && y < ny && x == xc;
                        o[h] |= (in ? (wv[h] >> (8 * e)) & 0xffu : 4u) << (8 * e);
                    }
                }
                v[r] = make_uint4(o[0], o[1], o[2], o[3]);
            }
#pragma unroll
            for (int r = 0; r < PER; ++r) {
                const uint2 m0 = walk_moves(v[r].x), m1 = walk_moves(v[r].y);
                const uint2 m2 = walk_moves(v[r].z), m3 = walk_moves(v[r].w);
                uint4 *dst = reinterpret_cast<uint4 *>(tmove) + 2 * (threadIdx.x + r * 1024);
                dst[0] = make_uint4(m0.x, m0.y, m1.x, m1.y);
                dst[1] = make_uint4(m2.x, m2.y, m3.x, m3.y);
            }
        } else if ((pitch & 3) == 0) {
            constexpr int PER = kTile * kTile / 4 / 1024;
            uint32_t v[PER];
#pragma unroll
            for (int r = 0; r < PER; ++r) {
                const int q = threadIdx.x + r * 1024;  // 4-cell group
                const int x = tx0 + 4 * (q & (kTile / 4 - 1)), y = ty0 + q / (kTile / 4);
                const int xc = min(max(x, 0), pitch - 4), yc = min(max(y, 0), ny - 1);
                const uint32_t w = *reinterpret_cast<const uint32_t *>(code + (size_t)yc * pitch + xc);
                uint32_t o = 0;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const bool in = x + e >= 0 && x + e < nx && y >= 0 && y < ny && x == xc;
                    o |= (in ? (w >> (8 * e)) & 0xffu : 4u) << (8 * e);
                }
                v[r] = o;
            }
#pragma unroll
            for (int r = 0; r < PER; ++r)
                reinterpret_cast<uint2 *>(tmove)[threadIdx.x + r * 1024] = walk_moves(v[r]);
        } else {
            constexpr int PER = kTile * kTile / 1024;
            uint32_t v[PER];
#pragma unroll
            for (int r = 0; r < PER; ++r) {
                const int k = threadIdx.x + r * 1024;
                const int x = tx0 + (k & (kTile - 1)), y = ty0 + k / kTile;
                const bool in = x >= 0 && y >= 0 && x < nx && y < ny;
                const uint8_t d = code[(size_t)min(max(y, 0), ny - 1) * pitch + min(max(x, 0), nx - 1)];
                v[r] = in ? d : 4u;
            }
#pragma unroll
            for (int r = 0; r < PER; ++r) tmove[threadIdx.x + r * 1024] = (uint16_t)walk_moves(v[r]).x;
        }
        __syncthreads();
        {
            // border ring: rows 0 and 255, columns 0 and 255 (1020 cells)
            const int t = threadIdx.x, side = t >> 8, i = t & (kTile - 1);
            const int cell = side == 0 ? i : side == 1 ? (kTile - 1) * kTile + i : side == 2 ? i * kTile
                                                                                               : i * kTile + kTile - 1;
            tmove[cell] = 0;
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x;
            const int wx0 = __builtin_amdgcn_readfirstlane(tx0), wy0 = __builtin_amdgcn_readfirstlane(ty0);
            int n = __builtin_amdgcn_readfirstlane(state[2]);
            // byte offset of the current cell in the window
            int a = 2 * ((__builtin_amdgcn_readfirstlane(state[1]) - wy0) * kTile +
                         (__builtin_amdgcn_readfirstlane(state[0]) - wx0));
            const char *moves = reinterpret_cast<const char *>(tmove);
            for (;;) {
                const int lim = min(64, cap - n);
                int k = 0, rec = 0;
                int m = *reinterpret_cast<const int16_t *>(moves + a);
                while (m != 0 && k < lim) {
                    a += m;
                    rec = lane == k ? a : rec;
                    ++k;
                    m = *reinterpret_cast<const int16_t *>(moves + a);
                }
                if (lane < k) {
                    path[2 * (n + lane)] = wx0 + ((rec >> 1) & (kTile - 1));
                    path[2 * (n + lane) + 1] = wy0 + (rec >> 9);
                }
                n += k;
                if (k < 64) break;
            }
            int x = wx0 + ((a >> 1) & (kTile - 1)), y = wy0 + (a >> 9);
            const int d = code[(size_t)min(max(y, 0), ny - 1) * pitch + min(max(x, 0), nx - 1)];
            int st = -1;
            if (d == kGoalCode) {
                st = TWG_OK;
            } else if (d >= 4) {
                st = TWG_NO_PATH;
            } else {
                // the buffer is full (the step that did not fit is taken, not
                // stored), or the step leaves the window: take it here
                x += d < 2 ? 1 - 2 * d : 0;
                y += d < 2 ? 0 : 5 - 2 * d;
                if (n >= cap) {
                    st = TWG_PATH_TRUNCATED;
                } else {
                    if (lane == 0) {
                        path[2 * n] = x;
                        path[2 * n + 1] = y;
                    }
                    ++n;
                }
            }
            if (lane == 0) {
                state[0] = x;
                state[1] = y;
                state[2] = n;
                state[3] = st;
            }
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
                 int ny, int pitch, hipStream_t st, bool walk)
{
    const dim3 grid((nx + 63) / 64, (ny + 3) / 4);
    if (psi64) {
        if (walk)
            hipLaunchKernelGGL((k_index<double, true>), grid, dim3(256), 0, st, cls, psi64, idx, nx, ny, pitch);
        else
            hipLaunchKernelGGL((k_index<double, false>), grid, dim3(256), 0, st, cls, psi64, idx, nx, ny, pitch);
    } else {
        if (walk)
            hipLaunchKernelGGL((k_index<float, true>), grid, dim3(256), 0, st, cls, psi, idx, nx, ny, pitch);
        else
            hipLaunchKernelGGL((k_index<float, false>), grid, dim3(256), 0, st, cls, psi, idx, nx, ny, pitch);
    }
    return hipGetLastError() == hipSuccess ? TWG_OK : TWG_EDEVICE;
}

int launch_walk(const uint8_t *cls, const uint8_t *code, int nx, int ny, int pitch, int sx, int sy,
                int cap, int32_t *path, int32_t *info, hipStream_t st)
{
    hipLaunchKernelGGL(k_walk, dim3(1), dim3(1024), 0, st, cls, code, nx, ny, pitch, sx, sy, cap, path,
                       info);
    return hipGetLastError() == hipSuccess ? TWG_OK : TWG_EDEVICE;
}

}  // namespace twg
