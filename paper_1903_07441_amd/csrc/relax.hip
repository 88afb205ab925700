// Harmonic-potential relaxation kernels for gfx950 (Eqs. 1-2 of the paper;
// boundary values of section "Harmonic Potential Fields").
//
// Field layout: row-major, x fastest, pitch in elements; psi = 1 - phi.
// Red cells are (x + y) even.  One red-black SOR sweep sets every FREE cell of
// one colour, then of the other, to
//     psi + omega * (((E + W) + (S + N)) / 4 + f - psi)
// (f = optional source, 0 for the potential itself).  Fixed cells carry a
// per-cell factor 0 instead of omega, so they are rewritten unchanged.
//
// k_sor_stream is the production kernel: temporal blocking in registers.
// One wave owns a strip of 128 columns (each lane two adjacent columns, so in
// every row a lane holds exactly one red and one black cell) and streams it
// from top to bottom.  The S sweeps of a pass form a pipeline of 2S
// half-sweep stages; stage k lags the row loader by k + 1 rows, so every
// stage sees neighbour rows that are exactly one half-sweep older.  Vertical
// neighbours come from the rolling register window, horizontal ones from the
// adjacent lane through wave-wide DPP shifts (no LDS traffic at all).  Each
// half-sweep invalidates one column at each edge of the strip, so S lanes on
// each side are halo and 128 - 4S columns are written; the rows of a tile are
// likewise extended by 2S halo rows above and below.  Reads come from `src`
// and results go to `dst` (ping-pong), so the tiles of one launch never race.
#include "twg_internal.h"

namespace twg {

namespace {

constexpr int kWave = 64;

// ---- arithmetic shared by the untiled and the streamed kernels ----------
// FP32: d = avg4 (+ f) - old with the exact quarter folded into one fma,
// then old + w * d in a second fma.
template <bool RHS>
__device__ __forceinline__ float upd(float old, float ew, float sn, float w, float f)
{
    const float s = ew + sn;
    const float d = RHS ? __builtin_fmaf(0.25f, s, f) - old : __builtin_fmaf(0.25f, s, -old);
    return __builtin_fmaf(w, d, old);
}

// FP64: unfused, in the order of the definition (this file is compiled with
// contraction off), so one sweep reproduces a plain FP64 sweep bit for bit.
template <bool RHS>
__device__ __forceinline__ double upd(double old, double ew, double sn, double w, double f)
{
    double g = (ew + sn) * 0.25;
    if (RHS) g = g + f;
    const double d = g - old;
    return old + w * d;
}

// ---- wave-wide DPP shifts (gfx9 wave_shr:1 / wave_shl:1) ----------------
// shr: lane i receives lane i-1 (lane 0 receives 0); shl: lane i receives
// lane i+1 (lane 63 receives 0).
__device__ __forceinline__ float shr1(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float shl1(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double shr1(double v)
{
    int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, true);
    int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double shl1(double v)
{
    int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, true);
    int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of tiles so that its L2 sees a compact band of the grid.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    constexpr int X = 8;
    int per = nb / X, rem = nb % X;
    int xcd = b % X, local = b / X;
    return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// ---- streamed temporal-blocked red-black SOR ----------------------------
// Rows are prefetched one window (NW rows) ahead into a register queue, so a
// load has NW row-steps of arithmetic to arrive.  Loads use clamped (always
// in-bounds) addresses; cells outside the grid are zeroed with a fixed-cell
// factor when they are taken from the queue.
// One wave relaxes one tile: output columns [x0 + 2S, x0 + 128 - 2S) and
// rows [ybeg, yend) of a grid; x0 and ybeg are even, all tile values are
// wave-uniform.
template <typename T, int S, bool RHS>
__device__ __forceinline__ void stream_tile(const T *__restrict__ src, T *__restrict__ dst,
                                            const uint8_t *__restrict__ cls,
                                            const T *__restrict__ f, int nx, int ny, int pitch,
                                            T omega, int x0, int ybeg, int yend)
{
    constexpr int NW = 2 * S + 2;      // rolling window of rows (even)
    const int lane = threadIdx.x & (kWave - 1);
    const int r0 = ybeg - 2 * S;                   // first row streamed (even)
    const int T_rows = (yend - ybeg) + 4 * S;
    // per-lane constants
    const int xa = x0 + 2 * lane;
    const bool in0 = xa >= 0 && xa < nx, in1 = xa + 1 >= 0 && xa + 1 < nx;
    const int xc0 = min(max(xa, 0), nx - 1), xc1 = min(max(xa + 1, 0), nx - 1);
    const T om0 = in0 ? omega : T(0), om1 = in1 ? omega : T(0);
    const bool writer = lane >= S && lane < kWave - S;

    T qv0[NW], qv1[NW], qf0[NW], qf1[NW];
    uint32_t qc0[NW], qc1[NW];
    auto fetch = [&](int slot, int t) {
        const int yc = min(max(r0 + t, 0), ny - 1);
        const T *ps = src + yc * pitch;
        const uint8_t *pc = cls + yc * pitch;
        qv0[slot] = ps[xc0];
        qv1[slot] = ps[xc1];
        qc0[slot] = pc[xc0];
        qc1[slot] = pc[xc1];
        if (RHS) {
            const T *pf = f + yc * pitch;
            qf0[slot] = pf[xc0];
            qf1[slot] = pf[xc1];
        }
    };

    T R[NW], B[NW], wR[NW], wB[NW], fR[NW], fB[NW];
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        R[i] = B[i] = wR[i] = wB[i] = fR[i] = fB[i] = T(0);
        qf0[i] = qf1[i] = T(0);
        fetch(i, i);
    }

    for (int base = 0; base < T_rows; base += NW) {
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            const int t = base + u;
            if (t < T_rows) {
                const int y = r0 + t;  // parity of y == parity of u
                T v0 = T(0), v1 = T(0), w0 = T(0), w1 = T(0), f0 = T(0), f1 = T(0);
                if (y >= 0 && y < ny) {  // uniform
                    v0 = in0 ? qv0[u] : T(0);
                    v1 = in1 ? qv1[u] : T(0);
                    w0 = qc0[u] == TWG_CELL_FREE ? om0 : T(0);
                    w1 = qc1[u] == TWG_CELL_FREE ? om1 : T(0);
                    if (RHS) {
                        f0 = in0 ? qf0[u] : T(0);
                        f1 = in1 ? qf1[u] : T(0);
                    }
                }
                if (t + NW < T_rows) fetch(u, t + NW);
                if ((u & 1) == 0) {  // even row: red = first column
                    R[u] = v0; B[u] = v1; wR[u] = w0; wB[u] = w1; fR[u] = f0; fB[u] = f1;
                } else {
                    R[u] = v1; B[u] = v0; wR[u] = w1; wB[u] = w0; fR[u] = f1; fB[u] = f0;
                }
#pragma unroll
                for (int k = 0; k < 2 * S; ++k) {
                    const int s = (u - 1 - k + 4 * NW) % NW;  // slot of row y - 1 - k
                    const int sp = (s + 1) % NW, sm = (s + NW - 1) % NW;
                    if ((k & 1) == 0) {
                        // red half-sweep of sweep k/2 at row y - 1 - k
                        const T b = B[s];
                        const T ew = (s & 1) == 0 ? b + shr1(b) : shl1(b) + b;
                        const T sn = B[sp] + B[sm];
                        R[s] = upd<RHS>(R[s], ew, sn, wR[s], fR[s]);
                    } else {
                        const T r = R[s];
                        const T ew = (s & 1) == 0 ? shl1(r) + r : r + shr1(r);
                        const T sn = R[sp] + R[sm];
                        B[s] = upd<RHS>(B[s], ew, sn, wB[s], fB[s]);
                    }
                }
                const int ys = y - 2 * S;  // row finished by this step (uniform test)
                if (ys >= ybeg && ys < yend) {
                    const int s = (u - 2 * S + 4 * NW) % NW;
                    T *pd = dst + ys * pitch;
                    const T o0 = (s & 1) == 0 ? R[s] : B[s];
                    const T o1 = (s & 1) == 0 ? B[s] : R[s];
                    if (writer && in0) pd[xa] = o0;
                    if (writer && in1) pd[xa + 1] = o1;
                }
            }
        }
    }
}

template <typename T, int S, bool RHS>
__global__ __launch_bounds__(256) void k_sor_stream(const T *__restrict__ src, T *__restrict__ dst,
                                                    const uint8_t *__restrict__ cls,
                                                    const T *__restrict__ f, int nx, int ny,
                                                    int pitch, T omega, int strips, int RH,
                                                    int tiles)
{
    constexpr int VW = 128 - 4 * S;  // columns written per strip
    // everything that depends only on the tile is wave-uniform: keep it scalar
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
    if (tile >= tiles) return;  // whole wave
    const int strip = tile % strips, seg = tile / strips;
    const int ybeg = seg * RH;
    stream_tile<T, S, RHS>(src, dst, cls, f, nx, ny, pitch, omega, strip * VW - 2 * S, ybeg,
                           min(ybeg + RH, ny));
}

// Batched form: the tiles of many grids in one launch.  Grid g's arrays start
// at element offset desc.off of the batch base pointers; the tile count is
// read from device memory so that one captured launch serves any active set.
template <int S>
__global__ __launch_bounds__(256) void k_sor_stream_batch(const float *__restrict__ src,
                                                          float *__restrict__ dst,
                                                          const uint8_t *__restrict__ cls,
                                                          const BatchGrid *__restrict__ grids,
                                                          const BatchTile *__restrict__ tiles,
                                                          const int *__restrict__ n_tiles)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
    if (tile >= *n_tiles) return;  // whole wave
    const BatchTile t = tiles[tile];
    const BatchGrid g = grids[t.grid];
    stream_tile<float, S, false>(src + g.off, dst + g.off, cls + g.off, nullptr, g.nx, g.ny,
                                 g.pitch, g.omega, t.x0, t.ybeg, t.yend);
}

// ---- untiled half-sweep: one colour, in place -----------------------------
template <typename T, bool RHS>
__global__ __launch_bounds__(256) void k_sweep_color(const uint8_t *__restrict__ cls, T *psi,
                                                     const T *__restrict__ f, int nx, int ny,
                                                     int pitch, T omega, int color)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= nx || y >= ny || ((x + y) & 1) != color) return;
    const size_t i = (size_t)y * pitch + x;
    const T e = x + 1 < nx ? psi[i + 1] : T(0);
    const T w = x > 0 ? psi[i - 1] : T(0);
    const T s = y + 1 < ny ? psi[i + pitch] : T(0);
    const T n = y > 0 ? psi[i - pitch] : T(0);
    const T om = cls[i] == TWG_CELL_FREE ? omega : T(0);
    psi[i] = upd<RHS>(psi[i], e + w, s + n, om, RHS ? f[i] : T(0));
}

// ---- residual, FP64 arithmetic ------------------------------------------
// max that keeps a NaN (fmax would drop it)
__device__ __forceinline__ double nanmax(double a, double b) { return (b > a || b != b) ? b : a; }

__device__ __forceinline__ double block_max(double v)
{
    __shared__ double part[4];
    for (int o = 32; o > 0; o >>= 1) v = nanmax(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    return nanmax(nanmax(part[0], part[1]), nanmax(part[2], part[3]));
}

// Residual |avg4(u) + f - u| over FREE cells; the max's bit pattern goes to
// out[0] by atomicMax (non-negative doubles order like their bit patterns; a
// NaN anywhere yields a NaN pattern, which is larger than +inf).  out[1]
// receives max |r| / |u| over FREE cells with |u| >= 1e-30.
template <typename T, bool RHS, bool WRITE_R32>
__global__ __launch_bounds__(256) void k_resid(const uint8_t *__restrict__ cls,
                                               const T *__restrict__ u, const float *__restrict__ f,
                                               float *__restrict__ r32, int nx, int ny, int pitch,
                                               unsigned long long *out)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    double m = 0.0, mr = 0.0;
    for (int y = blockIdx.y * 4 + (threadIdx.x >> 6); y < ny; y += gridDim.y * 4) {
        if (x >= nx) break;
        const size_t i = (size_t)y * pitch + x;
        double r = 0.0;
        if (cls[i] == TWG_CELL_FREE) {
            const double e = x + 1 < nx ? (double)u[i + 1] : 0.0;
            const double w = x > 0 ? (double)u[i - 1] : 0.0;
            const double s = y + 1 < ny ? (double)u[i + pitch] : 0.0;
            const double n = y > 0 ? (double)u[i - pitch] : 0.0;
            double g = ((e + w) + (s + n)) * 0.25;
            if (RHS) g = g + (double)f[i];
            const double c = (double)u[i];
            r = g - c;
            const double ac = fabs(c);
            if (ac >= 1e-30) mr = nanmax(mr, fabs(r) / ac);
        }
        if (WRITE_R32) r32[i] = (float)r;
        m = nanmax(m, fabs(r));
    }
    m = block_max(m);
    __syncthreads();
    mr = block_max(mr);
    if (threadIdx.x == 0) {
        atomicMax(out, (unsigned long long)__double_as_longlong(m));
        atomicMax(out + 1, (unsigned long long)__double_as_longlong(mr));
    }
}

// Batched residual: block b handles 64 columns of one grid (all rows);
// out[2 g] and out[2 g + 1] receive grid g's max |r| and max |r| / |u|.
__global__ __launch_bounds__(256) void k_resid_batch(const uint8_t *__restrict__ cls,
                                                     const float *__restrict__ u,
                                                     const BatchGrid *__restrict__ grids,
                                                     const int2 *__restrict__ blocks,
                                                     unsigned long long *out)
{
    const int2 bk = blocks[blockIdx.x];
    const BatchGrid g = grids[bk.x];
    const uint8_t *c = cls + g.off;
    const float *v = u + g.off;
    const int x = bk.y * 64 + (threadIdx.x & 63);
    double m = 0.0, mr = 0.0;
    if (x < g.nx) {
        for (int y = threadIdx.x >> 6; y < g.ny; y += 4) {
            const size_t i = (size_t)y * g.pitch + x;
            if (c[i] != TWG_CELL_FREE) continue;
            const double e = x + 1 < g.nx ? (double)v[i + 1] : 0.0;
            const double w = x > 0 ? (double)v[i - 1] : 0.0;
            const double s = y + 1 < g.ny ? (double)v[i + g.pitch] : 0.0;
            const double n = y > 0 ? (double)v[i - g.pitch] : 0.0;
            const double cc = (double)v[i];
            const double r = ((e + w) + (s + n)) * 0.25 - cc;
            m = nanmax(m, fabs(r));
            if (fabs(cc) >= 1e-30) mr = nanmax(mr, fabs(r) / fabs(cc));
        }
    }
    m = block_max(m);
    __syncthreads();
    mr = block_max(mr);
    if (threadIdx.x == 0) {
        atomicMax(out + 2 * bk.x, (unsigned long long)__double_as_longlong(m));
        atomicMax(out + 2 * bk.x + 1, (unsigned long long)__double_as_longlong(mr));
    }
}

__global__ void k_field_init_batch(const uint8_t *__restrict__ cls, float *psi,
                                   const BatchGrid *__restrict__ grids,
                                   const int2 *__restrict__ blocks, int mode)
{
    const int2 bk = blocks[blockIdx.x];
    const BatchGrid g = grids[bk.x];
    const int x = bk.y * 64 + (threadIdx.x & 63);
    if (x >= g.nx) return;
    for (int y = threadIdx.x >> 6; y < g.ny; y += 4) {
        const size_t i = g.off + (size_t)y * g.pitch + x;
        switch (cls[i]) {
        case TWG_CELL_OBST:
        case TWG_CELL_WALL: psi[i] = 0.0f; break;
        case TWG_CELL_GOAL: psi[i] = 1.0f; break;
        case TWG_CELL_FREE:
            if (mode == HPF_INIT_HALF) psi[i] = 0.5f;
            else if (mode == HPF_INIT_ZERO) psi[i] = 0.0f;
            break;
        default: break;
        }
    }
}

__global__ void k_zero_words_n(unsigned long long *w, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) w[i] = 0ull;
}

__global__ void k_copy_batch(const float *__restrict__ s, float *__restrict__ d,
                             const BatchGrid *__restrict__ grids, const int2 *__restrict__ blocks)
{
    const int2 bk = blocks[blockIdx.x];
    const BatchGrid g = grids[bk.x];
    const int x = bk.y * 64 + (threadIdx.x & 63);
    if (x >= g.nx) return;
    for (int y = threadIdx.x >> 6; y < g.ny; y += 4) {
        const size_t i = g.off + (size_t)y * g.pitch + x;
        d[i] = s[i];
    }
}

// ---- element-wise helpers --------------------------------------------------
__global__ void k_field_init(const uint8_t *__restrict__ cls, float *psi, int nx, int ny, int pitch,
                             int mode)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= nx || y >= ny) return;
    const size_t i = (size_t)y * pitch + x;
    switch (cls[i]) {
    case TWG_CELL_OBST:
    case TWG_CELL_WALL: psi[i] = 0.0f; break;
    case TWG_CELL_GOAL: psi[i] = 1.0f; break;
    case TWG_CELL_FREE:
        if (mode == HPF_INIT_HALF) psi[i] = 0.5f;
        else if (mode == HPF_INIT_ZERO) psi[i] = 0.0f;
        break;
    default: break;
    }
}

__global__ void k_update64(const uint8_t *__restrict__ cls, double *u, const float *__restrict__ e,
                           float *psi, int nx, int ny, int pitch)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= nx || y >= ny) return;
    const size_t i = (size_t)y * pitch + x;
    double v = u[i];
    if (cls[i] == TWG_CELL_FREE) {
        v = v + (double)e[i];
        u[i] = v;
    }
    psi[i] = (float)v;
}

__global__ void k_widen(const float *__restrict__ psi, double *u, int nx, int ny, int pitch)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= nx || y >= ny) return;
    const size_t i = (size_t)y * pitch + x;
    u[i] = (double)psi[i];
}

__global__ void k_narrow(const double *__restrict__ u, float *psi, int nx, int ny, int pitch)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= nx || y >= ny) return;
    const size_t i = (size_t)y * pitch + x;
    psi[i] = (float)u[i];
}

__global__ void k_fill(float *a, float v, int nx, int ny, int pitch)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= nx || y >= ny) return;
    a[(size_t)y * pitch + x] = v;
}

__global__ void k_copy(const float *__restrict__ s, float *__restrict__ d, int nx, int ny, int pitch)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= nx || y >= ny) return;
    const size_t i = (size_t)y * pitch + x;
    d[i] = s[i];
}

__global__ void k_zero_words(unsigned long long *w, int n)
{
    if ((int)threadIdx.x < n) w[threadIdx.x] = 0ull;
}

dim3 cell_grid(int nx, int ny) { return dim3((nx + 63) / 64, (ny + 3) / 4); }

int last_status()
{
    return hipGetLastError() == hipSuccess ? TWG_OK : TWG_EDEVICE;
}

template <typename T, bool RHS>
int launch_stream(const T *src, T *dst, const uint8_t *cls, const T *f, int nx, int ny, int pitch,
                  T omega, const Geometry &g, hipStream_t st)
{
    const int blocks = (g.tiles + 3) / 4;
#define TWG_STREAM_CASE(SV)                                                                     \
    case SV:                                                                                    \
        hipLaunchKernelGGL((k_sor_stream<T, SV, RHS>), dim3(blocks), dim3(256), 0, st, src, dst, \
                           cls, f, nx, ny, pitch, omega, g.strips, g.RH, g.tiles);              \
        break;
    switch (g.S) {
        TWG_STREAM_CASE(1)
        TWG_STREAM_CASE(2)
        TWG_STREAM_CASE(3)
        TWG_STREAM_CASE(4)
        TWG_STREAM_CASE(6)
        TWG_STREAM_CASE(8)
    default: return TWG_EUNSUPPORTED;
    }
#undef TWG_STREAM_CASE
    return last_status();
}

}  // namespace

int launch_stream_batch(const float *src, float *dst, const uint8_t *cls, const BatchGrid *grids,
                        const BatchTile *tiles, const int *n_tiles, int max_tiles, int S,
                        hipStream_t st)
{
    const int blocks = (max_tiles + 3) / 4;
    if (blocks == 0) return TWG_OK;
#define TWG_BATCH_CASE(SV)                                                                       \
    case SV:                                                                                     \
        hipLaunchKernelGGL(k_sor_stream_batch<SV>, dim3(blocks), dim3(256), 0, st, src, dst, cls, \
                           grids, tiles, n_tiles);                                               \
        break;
    switch (S) {
        TWG_BATCH_CASE(1)
        TWG_BATCH_CASE(2)
        TWG_BATCH_CASE(3)
        TWG_BATCH_CASE(4)
        TWG_BATCH_CASE(6)
        TWG_BATCH_CASE(8)
    default: return TWG_EUNSUPPORTED;
    }
#undef TWG_BATCH_CASE
    return last_status();
}

int launch_resid_batch(const uint8_t *cls, const float *u, const BatchGrid *grids,
                       const int2 *blocks, int n_blocks, unsigned long long *out, int n_words,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_words_n, dim3(std::max(1, std::min(64, (n_words + 255) / 256))),
                       dim3(256), 0, st, out, n_words);
    if (n_blocks > 0)
        hipLaunchKernelGGL(k_resid_batch, dim3(n_blocks), dim3(256), 0, st, cls, u, grids, blocks, out);
    return last_status();
}

int launch_field_init_batch(const uint8_t *cls, float *psi, const BatchGrid *grids,
                            const int2 *blocks, int n_blocks, int mode, hipStream_t st)
{
    if (n_blocks > 0)
        hipLaunchKernelGGL(k_field_init_batch, dim3(n_blocks), dim3(256), 0, st, cls, psi, grids,
                           blocks, mode);
    return last_status();
}

int launch_copy_batch(const float *src, float *dst, const BatchGrid *grids, const int2 *blocks,
                      int n_blocks, hipStream_t st)
{
    if (n_blocks > 0)
        hipLaunchKernelGGL(k_copy_batch, dim3(n_blocks), dim3(256), 0, st, src, dst, grids, blocks);
    return last_status();
}

bool stream_depth_supported(int S) { return S == 1 || S == 2 || S == 3 || S == 4 || S == 6 || S == 8; }

Geometry stream_geometry(int nx, int ny, int S, int RH)
{
    Geometry g;
    g.S = S;
    g.RH = RH < 2 ? 2 : (RH & ~1);
    const int vw = 128 - 4 * S;
    g.strips = (nx + vw - 1) / vw;
    g.segs = (ny + g.RH - 1) / g.RH;
    g.tiles = g.strips * g.segs;
    return g;
}

int launch_field_init(const uint8_t *cls, float *psi, int nx, int ny, int pitch, int mode,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_field_init, cell_grid(nx, ny), dim3(256), 0, st, cls, psi, nx, ny, pitch,
                       mode);
    return last_status();
}

int launch_sweep_color_f32(const uint8_t *cls, float *psi, const float *f, int nx, int ny, int pitch,
                           float omega, int color, hipStream_t st)
{
    if (f)
        hipLaunchKernelGGL((k_sweep_color<float, true>), cell_grid(nx, ny), dim3(256), 0, st, cls,
                           psi, f, nx, ny, pitch, omega, color);
    else
        hipLaunchKernelGGL((k_sweep_color<float, false>), cell_grid(nx, ny), dim3(256), 0, st, cls,
                           psi, f, nx, ny, pitch, omega, color);
    return last_status();
}

int launch_sweep_color_f64(const uint8_t *cls, double *psi, const double *f, int nx, int ny,
                           int pitch, double omega, int color, hipStream_t st)
{
    if (f)
        hipLaunchKernelGGL((k_sweep_color<double, true>), cell_grid(nx, ny), dim3(256), 0, st, cls,
                           psi, f, nx, ny, pitch, omega, color);
    else
        hipLaunchKernelGGL((k_sweep_color<double, false>), cell_grid(nx, ny), dim3(256), 0, st, cls,
                           psi, f, nx, ny, pitch, omega, color);
    return last_status();
}

int launch_stream_f32(const float *src, float *dst, const uint8_t *cls, const float *f, int nx,
                      int ny, int pitch, float omega, const Geometry &geo, hipStream_t st)
{
    return f ? launch_stream<float, true>(src, dst, cls, f, nx, ny, pitch, omega, geo, st)
             : launch_stream<float, false>(src, dst, cls, f, nx, ny, pitch, omega, geo, st);
}

int launch_stream_f64(const double *src, double *dst, const uint8_t *cls, const double *f, int nx,
                      int ny, int pitch, double omega, const Geometry &geo, hipStream_t st)
{
    if (f) return TWG_EUNSUPPORTED;
    return launch_stream<double, false>(src, dst, cls, f, nx, ny, pitch, omega, geo, st);
}

static dim3 resid_grid(int nx, int ny)
{
    int gy = (ny + 3) / 4;
    if (gy > 64) gy = 64;
    return dim3((nx + 63) / 64, gy);
}

int launch_resid_f32(const uint8_t *cls, const float *u, const float *f, int nx, int ny, int pitch,
                     unsigned long long *out, hipStream_t st)
{
    if (f)
        hipLaunchKernelGGL((k_resid<float, true, false>), resid_grid(nx, ny), dim3(256), 0, st, cls, u,
                           f, nullptr, nx, ny, pitch, out);
    else
        hipLaunchKernelGGL((k_resid<float, false, false>), resid_grid(nx, ny), dim3(256), 0, st, cls,
                           u, f, nullptr, nx, ny, pitch, out);
    return last_status();
}

int launch_resid_f64(const uint8_t *cls, const double *u, const float *f, int nx, int ny, int pitch,
                     unsigned long long *out, hipStream_t st)
{
    if (f)
        hipLaunchKernelGGL((k_resid<double, true, false>), resid_grid(nx, ny), dim3(256), 0, st, cls,
                           u, f, nullptr, nx, ny, pitch, out);
    else
        hipLaunchKernelGGL((k_resid<double, false, false>), resid_grid(nx, ny), dim3(256), 0, st, cls,
                           u, f, nullptr, nx, ny, pitch, out);
    return last_status();
}

int launch_defect64(const uint8_t *cls, const double *u, float *r32, int nx, int ny, int pitch,
                    unsigned long long *out, hipStream_t st)
{
    hipLaunchKernelGGL((k_resid<double, false, true>), resid_grid(nx, ny), dim3(256), 0, st, cls, u,
                       nullptr, r32, nx, ny, pitch, out);
    return last_status();
}

int launch_update64(const uint8_t *cls, double *u, const float *e, float *psi, int nx, int ny,
                    int pitch, hipStream_t st)
{
    hipLaunchKernelGGL(k_update64, cell_grid(nx, ny), dim3(256), 0, st, cls, u, e, psi, nx, ny, pitch);
    return last_status();
}

int launch_widen(const float *psi, double *u, int nx, int ny, int pitch, hipStream_t st)
{
    hipLaunchKernelGGL(k_widen, cell_grid(nx, ny), dim3(256), 0, st, psi, u, nx, ny, pitch);
    return last_status();
}

int launch_narrow(const double *u, float *psi, int nx, int ny, int pitch, hipStream_t st)
{
    hipLaunchKernelGGL(k_narrow, cell_grid(nx, ny), dim3(256), 0, st, u, psi, nx, ny, pitch);
    return last_status();
}

int launch_fill_f32(float *a, float v, int nx, int ny, int pitch, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill, cell_grid(nx, ny), dim3(256), 0, st, a, v, nx, ny, pitch);
    return last_status();
}

int launch_copy_f32(const float *src, float *dst, int nx, int ny, int pitch, hipStream_t st)
{
    hipLaunchKernelGGL(k_copy, cell_grid(nx, ny), dim3(256), 0, st, src, dst, nx, ny, pitch);
    return last_status();
}

int launch_zero_words(unsigned long long *w, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, w, n);
    return last_status();
}

}  // namespace twg
