// Streamed, temporally blocked red-black SOR for gfx950: the relaxation's
// hot loop (Eqs. 1-2 of the paper, boundary values of section "Harmonic
// Potential Fields").
//
// Field layout: row-major, x fastest, pitch in elements; psi = 1 - phi.  Red
// cells are (x + y) even.  One sweep sets every FREE cell of one colour, then
// of the other, to psi + w * (avg4 + f - psi), evaluated as in update.h, where
// w is omega on FREE cells and 0 on fixed ones (which are thus rewritten
// unchanged).  The single-grid FP32 kernels read w from a factor map; the
// FP64 kernels, which move twice the bytes per cell, and the batched kernel,
// whose grids together outgrow the last-level cache, read a one-byte free
// mask and select omega or 0.  Both maps are built once per call from the
// class map.
//
// One wave owns a strip of 128 columns (each lane two adjacent columns, so in
// every row a lane holds exactly one red and one black cell) and streams it
// from top to bottom.  The S sweeps of a pass form a pipeline of 2S
// half-sweep stages; stage k lags the row loader by k + 1 rows, so every
// stage sees neighbour rows that are exactly one half-sweep older.  Vertical
// neighbours come from the rolling register window, horizontal ones from the
// adjacent lane through wave-wide DPP shifts (no LDS traffic).  The row loop
// has no per-row branches (its trip count is padded to whole windows, halo
// lanes store out of range) and is fenced so that each prefetch stays in its
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

// ---- buffer addressing ---------------------------------------------------
// A tile reads its rows through buffer resources based at its first row and
// writes through one based at its first output row, so every access is a
// scalar row offset plus a per-lane column offset.  The hardware checks the
// sum of the two against the resource's size and turns an access outside it
// into a zero read or a dropped store; the row loop relies on that instead
// of clamping: rows above or below the tile read zeros, rows that are not
// output rows (and halo lanes, whose column offset is kNoStore) are not
// stored.  A tile spans less than 2^30 bytes, so no offset sum wraps.
constexpr uint32_t kNoStore = 0x80000000u;
constexpr int64_t kMaxTileBytes = 1LL << 30;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float bload(float *, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0));
}
__device__ __forceinline__ double bload(double *, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 0));
}
// the 64- and 128-bit buffer builtins take and return these (GCC-style)
// vector types; they are only ever bit-cast or subscripted
typedef uint32_t bv2 __attribute__((__vector_size__(8)));
typedef uint32_t bv4 __attribute__((__vector_size__(16)));
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)vo, (int)so, 0);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(bv2, v), r, (int)vo, (int)so, 0);
}

// two adjacent elements in one access (PAIR tiles: even pitch, even nx and
// aligned bases, so a pair never straddles a row, the grid's edge or the
// resource's end)
template <typename T> struct Pair { T a, b; };
__device__ __forceinline__ Pair<float> bload2(float *, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
{
    // elements are copied out before the bit cast: clang bit-casts a vector
    // element lvalue from the vector's first element
    const bv2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 0);
    const uint32_t a = v[0], b = v[1];
    return {__builtin_bit_cast(float, a), __builtin_bit_cast(float, b)};
}
__device__ __forceinline__ Pair<double> bload2(double *, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
{
    struct D2 { double a, b; };
    const D2 v = __builtin_bit_cast(D2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)so, 0));
    return {v.a, v.b};
}
__device__ __forceinline__ void bstore2(float a, float b, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
{
    bv2 v;
    v[0] = __builtin_bit_cast(uint32_t, a);
    v[1] = __builtin_bit_cast(uint32_t, b);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)vo, (int)so, 0);
}
__device__ __forceinline__ void bstore2(double a, double b, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
{
    struct D2 { double a, b; };
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(bv4, D2{a, b}), r, (int)vo, (int)so, 0);
}

// ---- streamed temporal-blocked red-black SOR ----------------------------
// Rows are prefetched one window (NW rows) ahead into a register queue, so a
// load has NW row-steps of arithmetic to arrive.  Cells outside the grid are
// zeroed with a fixed-cell factor when they are taken from the queue.
// One wave relaxes one tile: output columns [x0 + 2S, x0 + 128 - 2S) and
// rows [ybeg, yend) of a grid; x0 and ybeg are even, all tile values are
// wave-uniform.  PAIR tiles move each lane's two columns in one access (three
// memory operations per row instead of six), which keeps a whole window of
// prefetches within the hardware's count of outstanding vector memory
// operations, so no row step ever waits for the loads of the rows after it.
// MASK: wsrc is the one-byte free mask (else the factor map of T).
template <typename T, int S, bool RHS, bool PAIR, bool MASK>
__device__ __forceinline__ void stream_tile(const T *__restrict__ src, T *__restrict__ dst,
                                            const void *__restrict__ wsrc, T omega,
                                            const T *__restrict__ f, int nx, int ny, int pitch,
                                            int x0, int ybeg, int yend)
{
    constexpr int NW = 2 * S + 2;      // rolling window of rows (even)
    const int lane = threadIdx.x & (kWave - 1);
    const int r0 = ybeg - 2 * S;                   // first row streamed (even)
    const int T_rows = (yend - ybeg) + 4 * S;
    // rows that can reach a stored row: [lo, hi)
    const int lo = max(r0, 0), hi = min(yend + 2 * S, ny);
    // read resources end at the last cell of row hi - 1 and the write
    // resource at the last cell of row yend - 1, so no access reaches past
    // the caller's last row even when its allocation ends there
    const uint32_t rowb = (uint32_t)pitch * sizeof(T);
    const uint32_t cells = (uint32_t)(hi - lo - 1) * (uint32_t)pitch + (uint32_t)nx;
    const uint32_t outc = (uint32_t)(yend - ybeg - 1) * (uint32_t)pitch + (uint32_t)nx;
    const size_t base = (size_t)lo * pitch;
    const __amdgpu_buffer_rsrc_t rs = rsrc(src + base, cells * sizeof(T));
    const __amdgpu_buffer_rsrc_t rw =
        MASK ? rsrc(static_cast<const uint8_t *>(wsrc) + base, cells)
             : rsrc(static_cast<const T *>(wsrc) + base, cells * sizeof(T));
    const __amdgpu_buffer_rsrc_t rf = rsrc(RHS ? f + base : src + base, cells * sizeof(T));
    const __amdgpu_buffer_rsrc_t rd = rsrc(dst + (size_t)ybeg * pitch, outc * sizeof(T));
    // per-lane constants: a column outside the grid gets an out-of-range
    // offset, so its value and factor read as zero; rows outside the grid
    // are out of range as well.  The row step thus uses the loads as they are.
    const int xa = x0 + 2 * lane;
    const bool in0 = xa >= 0 && xa < nx, in1 = xa + 1 >= 0 && xa + 1 < nx;
    const bool writer = lane >= S && lane < kWave - S;
    const uint32_t xb0 = in0 ? (uint32_t)xa * sizeof(T) : kNoStore;
    const uint32_t xb1 = in1 ? (uint32_t)(xa + 1) * sizeof(T) : kNoStore;
    const uint32_t xm0 = in0 ? (uint32_t)xa : kNoStore, xm1 = in1 ? (uint32_t)(xa + 1) : kNoStore;
    const uint32_t so0 = writer ? xb0 : kNoStore;
    const uint32_t so1 = writer ? xb1 : kNoStore;
    // row offsets (bytes) of streamed row t and of output row t - 4S;
    // negative ones are far out of range as unsigned sums
    const int vrow0 = (r0 - lo) * (int)rowb, mrow0 = (r0 - lo) * pitch;
    const int orow0 = (r0 - 2 * S - ybeg) * (int)rowb;

    T qv0[NW], qv1[NW], qw0[NW], qw1[NW], qf0[NW], qf1[NW];
    uint32_t qm0[NW], qm1[NW];
    auto fetch = [&](int slot, int t) {
        const uint32_t vo = (uint32_t)(vrow0 + t * (int)rowb), mo = (uint32_t)(mrow0 + t * pitch);
        if constexpr (MASK) {
            if constexpr (PAIR) {
                qm0[slot] = __builtin_amdgcn_raw_buffer_load_b16(rw, (int)xm0, (int)mo, 0);
            } else {
                qm0[slot] = __builtin_amdgcn_raw_buffer_load_b8(rw, (int)xm0, (int)mo, 0);
                qm1[slot] = __builtin_amdgcn_raw_buffer_load_b8(rw, (int)xm1, (int)mo, 0);
            }
        }
        if constexpr (PAIR) {
            const Pair<T> v = bload2((T *)nullptr, rs, xb0, vo);
            qv0[slot] = v.a;
            qv1[slot] = v.b;
            if constexpr (!MASK) {
                const Pair<T> w = bload2((T *)nullptr, rw, xb0, vo);
                qw0[slot] = w.a;
                qw1[slot] = w.b;
            }
            if (RHS) {
                const Pair<T> h = bload2((T *)nullptr, rf, xb0, vo);
                qf0[slot] = h.a;
                qf1[slot] = h.b;
            }
        } else {
            qv0[slot] = bload((T *)nullptr, rs, xb0, vo);
            qv1[slot] = bload((T *)nullptr, rs, xb1, vo);
            if constexpr (!MASK) {
                qw0[slot] = bload((T *)nullptr, rw, xb0, vo);
                qw1[slot] = bload((T *)nullptr, rw, xb1, vo);
            }
            if (RHS) {
                qf0[slot] = bload((T *)nullptr, rf, xb0, vo);
                qf1[slot] = bload((T *)nullptr, rf, xb1, vo);
            }
        }
    };

    T R[NW], B[NW], wR[NW], wB[NW], fR[NW], fB[NW];
    // the first window is fetched in slot order, so that slot 0's loads are
    // the oldest in flight when the loop starts, as on every later pass
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        R[i] = B[i] = wR[i] = wB[i] = fR[i] = fB[i] = T(0);
        qf0[i] = qf1[i] = T(0);
        fetch(i, i);
        __builtin_amdgcn_sched_barrier(0);
    }

    // the trip count is padded to whole windows so that the unrolled body
    // has no per-row branches: fetches are unconditional (rows past the grid
    // read zeros) and rows past the tile are computed but never stored
    const int T_pad = ((T_rows + NW - 1) / NW) * NW;
    for (int base = 0; base < T_pad; base += NW) {
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            const int t = base + u;
            const T v0 = qv0[u], v1 = qv1[u];
            T w0, w1;
            if constexpr (!MASK) {
                w0 = qw0[u];
                w1 = qw1[u];
            } else if constexpr (PAIR) {
                w0 = (qm0[u] & 0xffu) ? omega : T(0);
                w1 = (qm0[u] >> 8) ? omega : T(0);
            } else {
                w0 = qm0[u] ? omega : T(0);
                w1 = qm1[u] ? omega : T(0);
            }
            T f0 = T(0), f1 = T(0);
            if (RHS) {
                f0 = qf0[u];
                f1 = qf1[u];
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
            // stage k: half-sweep k of the pass (red for even k) at row
            // y - 1 - k (slot s).  Its E, W and N (row above, slot sm)
            // neighbours were finished in earlier row steps, so their sums
            // are formed first for all stages; S (row below, slot sp) is the
            // value stage k - 1 produces in this row step and is added last.
            T ewn[2 * S];
#pragma unroll
            for (int k = 0; k < 2 * S; ++k) {
                const int s = (u - 1 - k + 4 * NW) % NW;
                const int sm = (s + NW - 1) % NW;
                if ((k & 1) == 0) {
                    const T b = B[s];
                    ewn[k] = ((s & 1) == 0 ? b + shr1(b) : shl1(b) + b) + B[sm];
                } else {
                    const T r = R[s];
                    ewn[k] = ((s & 1) == 0 ? shl1(r) + r : r + shr1(r)) + R[sm];
                }
            }
#pragma unroll
            for (int k = 0; k < 2 * S; ++k) {
                const int s = (u - 1 - k + 4 * NW) % NW;
                const int sp = (s + 1) % NW;
                if ((k & 1) == 0)
                    R[s] = upd<RHS>(R[s], ewn[k], B[sp], wR[s], fR[s]);
                else
                    B[s] = upd<RHS>(B[s], ewn[k], R[sp], wB[s], fB[s]);
            }
            // the row finished by this step (row y - 2S) is stored; rows
            // outside [ybeg, yend) fall outside the write resource
            {
                const int s = (u - 2 * S + 4 * NW) % NW;
                const uint32_t ro = (uint32_t)(orow0 + t * (int)rowb);
                const T o0 = (s & 1) == 0 ? R[s] : B[s];
                const T o1 = (s & 1) == 0 ? B[s] : R[s];
                if constexpr (PAIR) {
                    bstore2(o0, o1, rd, so0, ro);
                } else {
                    bstore(o0, rd, so0, ro);
                    bstore(o1, rd, so1, ro);
                }
            }
            // keep this row's prefetch in this row step: without the fence
            // the scheduler sinks every prefetch of the window to its end
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

template <typename T, int S, bool RHS, bool PAIR>
__global__ __launch_bounds__(256) void k_sor_stream(const T *__restrict__ src, T *__restrict__ dst,
                                                    const void *__restrict__ wsrc, T omega,
                                                    const T *__restrict__ f, int nx, int ny,
                                                    int pitch, int strips, int RH, int tiles)
{
    constexpr int VW = 128 - 4 * S;  // columns written per strip
    // everything that depends only on the tile is wave-uniform: keep it scalar
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
    if (tile >= tiles) return;  // whole wave
    const int strip = tile % strips, seg = tile / strips;
    const int ybeg = seg * RH;
    stream_tile<T, S, RHS, PAIR, sizeof(T) == 8>(src, dst, wsrc, omega, f, nx, ny, pitch, strip * VW - 2 * S, ybeg,
                                 min(ybeg + RH, ny));
}

// Batched form: the tiles of many grids in one launch.  Grid g's arrays start
// at element offset desc.off of the batch base pointers; the tile count is
// read from device memory so that one captured launch serves any active set.
template <int S, bool PAIR>
__global__ __launch_bounds__(256) void k_sor_stream_batch(const float *__restrict__ src,
                                                          float *__restrict__ dst,
                                                          const uint8_t *__restrict__ fmask,
                                                          const BatchGrid *__restrict__ grids,
                                                          const BatchTile *__restrict__ tiles,
                                                          const int *__restrict__ n_tiles)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
    if (tile >= *n_tiles) return;  // whole wave
    const BatchTile t = tiles[tile];
    const BatchGrid g = grids[t.grid];
    stream_tile<float, S, false, PAIR, true>(src + g.off, dst + g.off, fmask + g.off, g.omega, nullptr,
                                             g.nx, g.ny, g.pitch, t.x0, t.ybeg, t.yend);
}

// Pair access needs even pitch and nx (a pair never leaves its row or the
// grid) and bases aligned to a pair.
// (wsrc holds elements of wbytes bytes: the factor map or the free mask)
template <typename T>
bool pairable(const T *src, const T *dst, const void *wsrc, size_t wbytes, const T *f, int nx, int pitch)
{
    const auto al = [](const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; };
    return nx % 2 == 0 && pitch % 2 == 0 && al(src, 2 * sizeof(T)) && al(dst, 2 * sizeof(T)) &&
           al(wsrc, 2 * wbytes) && (!f || al(f, 2 * sizeof(T)));
}

template <typename T, bool RHS, bool PAIR>
int launch_stream(const T *src, T *dst, const void *wsrc, T omega, const T *f, int nx, int ny, int pitch,
                  const Geometry &geo, hipStream_t st)
{
    const int cap = stream_rows_cap(pitch, sizeof(T), geo.S);
    const Geometry g = geo.RH > cap ? stream_geometry(nx, ny, geo.S, cap) : geo;
    const int blocks = (g.tiles + 3) / 4;
#define TWG_STREAM_CASE(SV)                                                                           \
    case SV:                                                                                          \
        hipLaunchKernelGGL((k_sor_stream<T, SV, RHS, PAIR>), dim3(blocks), dim3(256), 0, st, src, dst, \
                           wsrc, omega, f, nx, ny, pitch, g.strips, g.RH, g.tiles);                   \
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

int launch_stream_batch(const float *src, float *dst, const uint8_t *fmask, const BatchGrid *grids,
                        const BatchTile *tiles, const int *n_tiles, int max_tiles, int S, bool pair,
                        hipStream_t st)
{
    const int blocks = (max_tiles + 3) / 4;
    if (blocks == 0) return TWG_OK;
#define TWG_BATCH_CASE(SV)                                                                             \
    case SV:                                                                                           \
        if (pair)                                                                                      \
            hipLaunchKernelGGL((k_sor_stream_batch<SV, true>), dim3(blocks), dim3(256), 0, st, src, dst, \
                               fmask, grids, tiles, n_tiles);                                          \
        else                                                                                           \
            hipLaunchKernelGGL((k_sor_stream_batch<SV, false>), dim3(blocks), dim3(256), 0, st, src,     \
                               dst, fmask, grids, tiles, n_tiles);                                     \
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

int stream_rows_cap(int pitch, int elem_bytes, int S)
{
    // a tile's rows (RH + 4S of them) must span less than kMaxTileBytes
    const long long rows = (kMaxTileBytes - 1) / ((long long)pitch * elem_bytes);
    return (int)std::max(2LL, (rows - 4 * S - 2) & ~1LL);
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

int launch_stream_f32(const float *src, float *dst, const float *wmap, const float *f, int nx, int ny,
                      int pitch, const Geometry &geo, hipStream_t st)
{
    if (pairable(src, dst, wmap, sizeof(float), f, nx, pitch))
        return f ? launch_stream<float, true, true>(src, dst, wmap, 0.0f, f, nx, ny, pitch, geo, st)
                 : launch_stream<float, false, true>(src, dst, wmap, 0.0f, f, nx, ny, pitch, geo, st);
    return f ? launch_stream<float, true, false>(src, dst, wmap, 0.0f, f, nx, ny, pitch, geo, st)
             : launch_stream<float, false, false>(src, dst, wmap, 0.0f, f, nx, ny, pitch, geo, st);
}

int launch_stream_f64(const double *src, double *dst, const uint8_t *fmask, double omega, int nx, int ny,
                      int pitch, const Geometry &geo, hipStream_t st)
{
    if (pairable(src, dst, fmask, 1, (const double *)nullptr, nx, pitch))
        return launch_stream<double, false, true>(src, dst, fmask, omega, nullptr, nx, ny, pitch, geo, st);
    return launch_stream<double, false, false>(src, dst, fmask, omega, nullptr, nx, ny, pitch, geo, st);
}

}  // namespace twg
