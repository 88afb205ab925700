// Streamed, temporally blocked red-black SOR for gfx950: the relaxation's
// hot loop (Eqs. 1-2 of the paper, boundary values of section "Harmonic
// Potential Fields").
//
// Field layout: row-major, x fastest, pitch in elements; psi = 1 - phi.  Red
// cells are (x + y) even.  One sweep sets every FREE cell of one colour, then
// of the other, to psi + omega * (((E + W) + (S + N)) / 4 + f - psi); fixed
// cells carry a factor 0 instead of omega and are rewritten unchanged.
//
// One wave owns a strip of 128 columns (each lane two adjacent columns, so in
// every row a lane holds exactly one red and one black cell) and streams it
// from top to bottom.  The S sweeps of a pass form a pipeline of 2S
// half-sweep stages; stage k lags the row loader by k + 1 rows, so every
// stage sees neighbour rows that are exactly one half-sweep older.  Vertical
// neighbours come from the rolling register window, horizontal ones from the
// adjacent lane through wave-wide DPP shifts (no LDS traffic).  The row loop
// has no per-row branches (its trip count is padded to whole windows, halo
// lanes store into a sink) and is fenced so that each prefetch stays in its
// row step: the compiler can then keep the prefetch queue in fixed registers
// and never has to wait for a load in flight before the window comes round.  Each
// half-sweep invalidates one column at each edge of the strip, so S lanes on
// each side are halo and 128 - 4S columns are written; the rows of a tile are
// likewise extended by 2S halo rows above and below.  Reads come from `src`
// and results go to `dst` (ping-pong), so the tiles of one launch never race.
#include "twg_internal.h"
#include "update.h"

namespace twg {

namespace {

constexpr int kWave = 64;

int last_status() { return hipGetLastError() == hipSuccess ? TWG_OK : TWG_EDEVICE; }

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
                                            T omega, int x0, int ybeg, int yend, T *__restrict__ sink)
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

    // the trip count is padded to whole windows so that the unrolled body
    // has no per-row branches: fetches are unconditional (clamped rows) and
    // rows past the tile are computed but never stored
    const int T_pad = ((T_rows + NW - 1) / NW) * NW;
    for (int base = 0; base < T_pad; base += NW) {
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            const int t = base + u;
            const int y = r0 + t;  // parity of y == parity of u
            const bool rowok = y >= 0 && y < ny;  // uniform
            const T v0 = rowok && in0 ? qv0[u] : T(0);
            const T v1 = rowok && in1 ? qv1[u] : T(0);
            const T w0 = rowok && qc0[u] == TWG_CELL_FREE ? om0 : T(0);
            const T w1 = rowok && qc1[u] == TWG_CELL_FREE ? om1 : T(0);
            T f0 = T(0), f1 = T(0);
            if (RHS) {
                f0 = rowok && in0 ? qf0[u] : T(0);
                f1 = rowok && in1 ? qf1[u] : T(0);
            }
            // the slot is refilled only after its values are taken, so the
            // queue keeps fixed registers across iterations
            __builtin_amdgcn_sched_barrier(0);
            fetch(u, t + NW);
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
                // halo lanes and columns outside the grid store into the
                // sink instead of branching around the store
                T *p0 = writer && in0 ? pd + xa : sink + 2 * lane;
                T *p1 = writer && in1 ? pd + xa + 1 : sink + 2 * lane + 1;
                *p0 = o0;
                *p1 = o1;
            }
            // keep this row's prefetch in this row step: without the fence
            // the scheduler sinks every prefetch of the window to its end
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

template <typename T, int S, bool RHS>
__global__ __launch_bounds__(256) void k_sor_stream(const T *__restrict__ src, T *__restrict__ dst,
                                                    const uint8_t *__restrict__ cls,
                                                    const T *__restrict__ f, int nx, int ny,
                                                    int pitch, T omega, int strips, int RH,
                                                    int tiles, T *__restrict__ sink)
{
    constexpr int VW = 128 - 4 * S;  // columns written per strip
    // everything that depends only on the tile is wave-uniform: keep it scalar
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
    if (tile >= tiles) return;  // whole wave
    const int strip = tile % strips, seg = tile / strips;
    const int ybeg = seg * RH;
    stream_tile<T, S, RHS>(src, dst, cls, f, nx, ny, pitch, omega, strip * VW - 2 * S, ybeg,
                           min(ybeg + RH, ny), sink);
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
                                                          const int *__restrict__ n_tiles,
                                                          float *__restrict__ sink)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
    if (tile >= *n_tiles) return;  // whole wave
    const BatchTile t = tiles[tile];
    const BatchGrid g = grids[t.grid];
    stream_tile<float, S, false>(src + g.off, dst + g.off, cls + g.off, nullptr, g.nx, g.ny,
                                 g.pitch, g.omega, t.x0, t.ybeg, t.yend, sink);
}

template <typename T, bool RHS>
int launch_stream(const T *src, T *dst, const uint8_t *cls, const T *f, int nx, int ny, int pitch,
                  T omega, const Geometry &g, void *sink, hipStream_t st)
{
    const int blocks = (g.tiles + 3) / 4;
#define TWG_STREAM_CASE(SV)                                                                     \
    case SV:                                                                                    \
        hipLaunchKernelGGL((k_sor_stream<T, SV, RHS>), dim3(blocks), dim3(256), 0, st, src, dst, \
                           cls, f, nx, ny, pitch, omega, g.strips, g.RH, g.tiles,               \
                           static_cast<T *>(sink));                                              \
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
                        const BatchTile *tiles, const int *n_tiles, int max_tiles, int S, void *sink,
                        hipStream_t st)
{
    const int blocks = (max_tiles + 3) / 4;
    if (blocks == 0) return TWG_OK;
#define TWG_BATCH_CASE(SV)                                                                       \
    case SV:                                                                                     \
        hipLaunchKernelGGL(k_sor_stream_batch<SV>, dim3(blocks), dim3(256), 0, st, src, dst, cls, \
                           grids, tiles, n_tiles, static_cast<float *>(sink));                   \
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

int launch_stream_f32(const float *src, float *dst, const uint8_t *cls, const float *f, int nx,
                      int ny, int pitch, float omega, const Geometry &geo, void *sink, hipStream_t st)
{
    return f ? launch_stream<float, true>(src, dst, cls, f, nx, ny, pitch, omega, geo, sink, st)
             : launch_stream<float, false>(src, dst, cls, f, nx, ny, pitch, omega, geo, sink, st);
}

int launch_stream_f64(const double *src, double *dst, const uint8_t *cls, const double *f, int nx,
                      int ny, int pitch, double omega, const Geometry &geo, void *sink, hipStream_t st)
{
    if (f) return TWG_EUNSUPPORTED;
    return launch_stream<double, false>(src, dst, cls, f, nx, ny, pitch, omega, geo, sink, st);
}

}  // namespace twg
