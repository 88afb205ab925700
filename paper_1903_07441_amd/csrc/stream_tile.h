// Streamed, temporally blocked red-black SOR tile for gfx950, shared by the
// kernels of sor_stream.hip (fixed sweep counts, FP64 sweeps, batches) and
// solve.hip (the device-driven relaxation).  See sor_stream.hip for the
// scheme.
#pragma once

#include <type_traits>
#include <utility>

#include "twg_internal.h"
#include "update.h"

namespace twg {
namespace sdev {

constexpr int kWave = 64;

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
// Store cache policy of the field rows.  kStoreThrough (sc1): the L2 writes
// them through at agent scope, so its lines are clean when the kernel ends
// and the release between two passes has nothing to write back.  Measured
// on one 2048 x 2048 grid (one wave per SIMD): the gap from one pass's last
// wave to the next pass's first falls from 2.2 to 0.9 us, while a wave's own
// time grows by 0.15 us.  A batch pass (several waves per SIMD, long passes)
// is faster with the default write-back policy (kStoreBack): 44.8 against
// 47.4 ms for 256 grids.
constexpr int kStoreThrough = 16, kStoreBack = 0;

// the 64- and 128-bit buffer builtins take and return these (GCC-style)
// vector types; they are only ever bit-cast or subscripted
typedef uint32_t bv2 __attribute__((__vector_size__(8)));
typedef uint32_t bv4 __attribute__((__vector_size__(16)));
template <int AUX>
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)vo, (int)so, AUX);
}
template <int AUX>
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(bv2, v), r, (int)vo, (int)so, AUX);
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
template <int AUX>
__device__ __forceinline__ void bstore2(float a, float b, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
{
    bv2 v;
    v[0] = __builtin_bit_cast(uint32_t, a);
    v[1] = __builtin_bit_cast(uint32_t, b);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)vo, (int)so, AUX);
}
template <int AUX>
__device__ __forceinline__ void bstore2(double a, double b, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
{
    struct D2 { double a, b; };
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(bv4, D2{a, b}), r, (int)vo, (int)so, AUX);
}

// v where the sign-extended mask byte m is all ones (a FREE cell), +0 where it
// is zero: one AND (the compiler folds the byte's sign extension into it)
__device__ __forceinline__ float keep(float v, int32_t m) { return __int_as_float(__float_as_int(v) & m); }
__device__ __forceinline__ double keep(double v, int32_t m)
{
    return __hiloint2double(__double2hiint(v) & m, __double2loint(v) & m);
}

// Source term of a tile: none; f (the constants of update.h are formed from
// f as the rows arrive); or c = omega f already formed (0 on fixed cells),
// from which a row needs only a and b.  kSrcC gives the bits of kSrcF with
// c = fl(omega f): a = w / 4 and b = 1 - w = fma(a, -4, 1) are exact.
constexpr int kSrcNone = 0, kSrcF = 1, kSrcC = 2;

// ---- streamed temporal-blocked red-black SOR ----------------------------
// One wave relaxes one tile: output columns [x0 + 2S, x0 + 128 - 2S) and
// rows [ybeg, yend) of a grid; x0 and ybeg are even, all tile values are
// wave-uniform.  wsrc is the one-byte free mask (0xFF on FREE cells, else
// 0): a FREE cell takes the factor omega, any other cell 0 (it is rewritten
// unchanged).  f is the source term of mode RHS.  PAIR tiles move each
// lane's two columns in one access (three memory operations per row instead
// of six), which keeps a whole window of prefetches within the hardware's
// count of outstanding vector memory operations.
//
// Registers.  The pipeline needs NW = 2S + 2 rows at a time (the rows its
// stages touch and the row the last stage finishes), and each row is fetched
// NW row steps before it enters the pipeline.  Rows therefore live in a ring
// of 2 NW register slots: row t sits in slot t mod 2NW from its fetch to its
// last use, and the fetch of row t + NW refills the slot row t - NW has just
// left.  The loop body covers one turn of the ring, so every slot is a fixed
// register across iterations: no value is copied at the back edge, and no
// row step waits for a load younger than NW row steps.  Cells outside the
// grid read as zeros with factor 0, straight from the out-of-range loads.
//
// CHECK: the pass also measures the residual of its INPUT field, in FP64:
// r = ((E + W) + (S + N)) / 4 (+ f) - c over the FREE cells of its output
// rows and columns, the expression of the standalone residual kernels.  Row
// y's residual needs rows y - 1 and y + 1 as they were loaded; the pipeline's
// first stage rewrites row y - 1's red cells one row step before row y + 1
// arrives, so the loaded values of the previous row are kept in two extra
// registers.  rmax receives max |r| and rrel max |r| / |c| (|c| >= 1e-30,
// evaluated with the hardware reciprocal: a diagnostic), both per lane; a
// NaN residual propagates.
__device__ __forceinline__ double nan_max(double a, double b) { return (b > a || b != b) ? b : a; }

// f(integral_constant<int, U>) for U = 0, 1, ..., one inlined copy each: the
// row loop's body is one of these, so it is unrolled whatever its size (a
// rolled body would index the register ring at run time, i.e. in scratch)
template <class F, int... U>
__device__ __forceinline__ void static_for(std::integer_sequence<int, U...>, F &&f)
{
    (f(std::integral_constant<int, U>{}), ...);
}
__device__ __forceinline__ float nan_maxf(float a, float b) { return (b > a || b != b) ? b : a; }

template <typename T, int S, int RHS, bool PAIR, bool CHECK = false, int STORE = kStoreThrough, bool SLOT_OFS = true>
__device__ __forceinline__ void stream_tile(const T *__restrict__ src, T *__restrict__ dst,
                                            const uint8_t *__restrict__ wsrc, T omega,
                                            const T *__restrict__ f, int nx, int ny, int pitch,
                                            int x0, int ybeg, int yend, double *rmax = nullptr,
                                            float *rrel = nullptr)
{
    static_assert(RHS == kSrcNone || RHS == kSrcF || RHS == kSrcC, "source mode");
    static_assert(!(CHECK && RHS == kSrcC), "the residual check needs f");
    constexpr int NW = 2 * S + 2;      // rows the pipeline holds (even)
    constexpr int NR = 2 * NW;         // ring slots
    const T quarter = omega * T(0.25);  // exact
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
    const __amdgpu_buffer_rsrc_t rw = rsrc(wsrc + base, cells);
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

    // ring: the two columns of a row (P0 = column 2 lane, P1 = 2 lane + 1),
    // its raw mask bytes and, with a source term, its f (or c) values
    T P0[NR], P1[NR], F0[NR], F1[NR];
    uint32_t M0[NR], M1[NR];
    // factors of the rows in the pipeline, by row mod NW (red, black), and
    // with a source term the update constants of update.h
    T wR[NW], wB[NW];
    SrcConst<T> kR[NW], kB[NW];
    // loads of a row into ring slot `slot`: lane offsets (columns 2 lane and
    // 2 lane + 1 of the field, then of the mask) and scalar row offsets.
    // The field is loaded before the mask: the row step that takes the row
    // in needs both, and loads complete in order, so one wait (for the
    // mask) covers the two.
    auto fetch_at = [&](int slot, uint32_t b0, uint32_t b1, uint32_t m0, uint32_t m1, uint32_t vo, uint32_t mo) {
        if constexpr (PAIR) {
            const Pair<T> v = bload2((T *)nullptr, rs, b0, vo);
            P0[slot] = v.a;
            P1[slot] = v.b;
            M0[slot] = __builtin_amdgcn_raw_buffer_load_b16(rw, (int)m0, (int)mo, 0);
            if (RHS) {
                const Pair<T> h = bload2((T *)nullptr, rf, b0, vo);
                F0[slot] = h.a;
                F1[slot] = h.b;
            }
        } else {
            P0[slot] = bload((T *)nullptr, rs, b0, vo);
            P1[slot] = bload((T *)nullptr, rs, b1, vo);
            M0[slot] = __builtin_amdgcn_raw_buffer_load_b8(rw, (int)m0, (int)mo, 0);
            M1[slot] = __builtin_amdgcn_raw_buffer_load_b8(rw, (int)m1, (int)mo, 0);
            if (RHS) {
                F0[slot] = bload((T *)nullptr, rf, b0, vo);
                F1[slot] = bload((T *)nullptr, rf, b1, vo);
            }
        }
    };
    // The first window (stream rows 0 .. NW - 1, some of them above the
    // grid) puts the whole row offset, negative for rows above the grid, in
    // the scalar part.  The loop fetches stream rows from NW on, which lie
    // at or below the tile's first in-grid row lo (r0 + NW > ybeg >= lo), so
    // there the row offset of stream row tb + NW + u (tb: the turn's first
    // step) splits into u rows, added to the lane offsets once per tile,
    // and tb + NW rows in one scalar offset per turn.  Both parts are
    // non-negative and the sums are the same as in one piece, so the range
    // check sees the same offsets and no sum wraps; the row steps spend no
    // scalar instruction on load offsets.  That costs 2 NR registers (4 NR
    // unpaired); SLOT_OFS = false (kernels that run several waves per SIMD)
    // forms every fetch's offsets in the scalar part instead.
    uint32_t lb0[NR], lb1[NR], lm0[NR], lm1[NR];
#pragma unroll
    for (int u = 0; u < NR && SLOT_OFS; ++u) {
        lb0[u] = xb0 + (uint32_t)u * rowb;
        lm0[u] = xm0 + (uint32_t)u * (uint32_t)pitch;
        lb1[u] = PAIR ? 0u : xb1 + (uint32_t)u * rowb;
        lm1[u] = PAIR ? 0u : xm1 + (uint32_t)u * (uint32_t)pitch;
        // kept as registers (not re-formed in the loop, where they would
        // cost an instruction each)
        asm volatile("" : "+v"(lb0[u]), "+v"(lm0[u]));
        if constexpr (!PAIR) asm volatile("" : "+v"(lb1[u]), "+v"(lm1[u]));
    }
    auto fetch = [&](int slot, int t) {
        fetch_at(slot, xb0, xb1, xm0, xm1, (uint32_t)(vrow0 + t * (int)rowb), (uint32_t)(mrow0 + t * pitch));
    };
    auto fetch_loop = [&](int slot, int u, int tb) {
        if constexpr (SLOT_OFS)
            fetch_at(slot, lb0[u], lb1[u], lm0[u], lm1[u], (uint32_t)(vrow0 + (tb + NW) * (int)rowb),
                     (uint32_t)(mrow0 + (tb + NW) * pitch));
        else
            fetch(slot, tb + u + NW);
    };
    // red and black cells of the row in ring slot s (red is the first
    // column on even rows; r0 is even, so a row's parity is its slot's)
    auto red = [&](int s) -> T & { return (s & 1) == 0 ? P0[s] : P1[s]; };
    auto blk = [&](int s) -> T & { return (s & 1) == 0 ? P1[s] : P0[s]; };

    // CHECK: loaded values of the row above the checked one (columns 2 lane
    // and 2 lane + 1), and the running maxima
    T upa = T(0), upb = T(0);
    double cmax = 0.0;
    float crel = 0.0f;
    // rows t - 1 checked at row step t: t - 1 in [ybeg - r0, yend - r0)
    const int tchk0 = ybeg - r0 + 1, tchk1 = yend - r0 + 1;
    // rows before the first streamed one are zeros with factor 0; the first
    // window is fetched in slot order, so that slot 0's loads are the oldest
    // in flight when the loop starts
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        P0[i] = P1[i] = F0[i] = F1[i] = T(0);
        M0[i] = M1[i] = 0u;
    }
#pragma unroll
    for (int i = 0; i < NW; ++i) wR[i] = wB[i] = T(0);
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        fetch(i, i);
        __builtin_amdgcn_sched_barrier(0);
    }

    // One row step: row t (ring slot u, pipeline index u mod NW) enters the
    // pipeline, row t + NW is fetched, the 2S stages advance and row t - 2S
    // is stored.  u is a constant wherever the step is inlined.
    auto step = [&](const int u, const int t, const bool prefetch) __attribute__((always_inline)) {
        const int uw = u % NW;
        {
            // the mask bytes sign-extended (all ones on a FREE cell); the
            // factor is omega or +0, bit for bit omega x (0 or 1)
            const int32_t e0 = (int32_t)(M0[u] << 24) >> 24;
            const int32_t e1 = PAIR ? (int32_t)(M0[u] << 16) >> 24 : (int32_t)(M1[u] << 24) >> 24;
            const bool ev = (u & 1) == 0;
            if constexpr (RHS != kSrcC) {
                const T w0 = keep(omega, e0), w1 = keep(omega, e1);
                wR[uw] = ev ? w0 : w1;
                wB[uw] = ev ? w1 : w0;
                if constexpr (RHS == kSrcF) {
                    const SrcConst<T> k0 = src_const(w0, F0[u]), k1 = src_const(w1, F1[u]);
                    kR[uw] = ev ? k0 : k1;
                    kB[uw] = ev ? k1 : k0;
                }
            } else {
                const T a0 = keep(quarter, e0), a1 = keep(quarter, e1);
                const SrcConst<T> k0{a0, fused(a0, T(-4), T(1)), F0[u]}, k1{a1, fused(a1, T(-4), T(1)), F1[u]};
                kR[uw] = ev ? k0 : k1;
                kB[uw] = ev ? k1 : k0;
            }
        }
        if constexpr (CHECK) {
            // residual of row t - 1 (slot um, not yet touched by any
            // stage) from the kept row t - 2 and the new row t (slot u)
            const int um = (u + NR - 1) % NR, uwm = (uw + NW - 1) % NW;
            const T ca = P0[um], cb = P1[um];
            // only the tile's own rows (a uniform branch: the halo and
            // pipeline rows, two fifths of the steps, skip the FP64 work)
            if (t >= tchk0 && t < tchk1) {
                const bool ev = (um & 1) == 0;
                const T wa = ev ? wR[uwm] : wB[uwm], wb = ev ? wB[uwm] : wR[uwm];
                const T dna = P0[u], dnb = P1[u];
                const double ea = (double)cb, wwa = (double)shr1(cb);
                const double eb = (double)shl1(ca), wwb = (double)ca;
                double ga = ((ea + wwa) + ((double)dna + (double)upa)) * 0.25;
                double gb = ((eb + wwb) + ((double)dnb + (double)upb)) * 0.25;
                if constexpr (RHS == kSrcF) {
                    ga = ga + (double)F0[um];
                    gb = gb + (double)F1[um];
                }
                const double ra = ga - (double)ca, rb = gb - (double)cb;
                const bool oka = writer && wa != T(0), okb = writer && wb != T(0);
                cmax = nan_max(cmax, oka ? fabs(ra) : 0.0);
                cmax = nan_max(cmax, okb ? fabs(rb) : 0.0);
                const float aa = fabsf((float)ca), ab = fabsf((float)cb);
                const float qa = fabsf((float)ra) * __builtin_amdgcn_rcpf(aa);
                const float qb = fabsf((float)rb) * __builtin_amdgcn_rcpf(ab);
                crel = nan_maxf(crel, oka && aa >= 1e-30f ? qa : 0.0f);
                crel = nan_maxf(crel, okb && ab >= 1e-30f ? qb : 0.0f);
            }
            upa = ca;
            upb = cb;
        }
        // row t + NW goes to the slot row t - NW left at the last step
        __builtin_amdgcn_sched_barrier(0);
        if (prefetch) fetch_loop((u + NW) % NR, u, t - u);
        // stage k: half-sweep k of the pass (red for even k) at row
        // t - 1 - k (slot s).  Its E, W and N (row above, slot sm)
        // neighbours were finished in earlier row steps; S (row below, slot
        // sp) is the value stage k - 1 produces in this row step and is
        // added last, so the chain through the stages is three operations
        // deep per stage.
        // E + W + N of stage k (red cells for even k, black for odd)
        auto ewn = [&](const int k) __attribute__((always_inline)) -> T {
            const int s = (u - 1 - k + 2 * NR) % NR;
            const int sm = (s + NR - 1) % NR;
            if ((k & 1) == 0) {
                const T b = blk(s);
                return ((s & 1) == 0 ? shr1(b) + b : shl1(b) + b) + blk(sm);
            }
            const T r = red(s);
            return ((s & 1) == 0 ? shl1(r) + r : shr1(r) + r) + red(sm);
        };
        // each stage's sum is formed one stage ahead of its update, which
        // gives the scheduler two independent chains to interleave
        T e_next = ewn(0);
#pragma unroll
        for (int k = 0; k < 2 * S; ++k) {
            const int s = (u - 1 - k + 2 * NR) % NR;
            const int sp = (s + 1) % NR;
            const int sw = (uw - 1 - k + 2 * NW) % NW;
            const T e = e_next;
            if (k + 1 < 2 * S) e_next = ewn(k + 1);
            if constexpr (RHS != kSrcNone) {
                if ((k & 1) == 0)
                    red(s) = upd_src(red(s), e, blk(sp), kR[sw]);
                else
                    blk(s) = upd_src(blk(s), e, red(sp), kB[sw]);
            } else {
                if ((k & 1) == 0)
                    red(s) = upd(red(s), e, blk(sp), wR[sw]);
                else
                    blk(s) = upd(blk(s), e, red(sp), wB[sw]);
            }
        }
        // the row finished by this step (row t - 2S) is stored; rows
        // outside [ybeg, yend) fall outside the write resource
        {
            const int s = (u - 2 * S + 2 * NR) % NR;
            const uint32_t ro = (uint32_t)(orow0 + t * (int)rowb);
            if constexpr (PAIR) {
                bstore2<STORE>(P0[s], P1[s], rd, so0, ro);
            } else {
                bstore<STORE>(P0[s], rd, so0, ro);
                bstore<STORE>(P1[s], rd, so1, ro);
            }
        }
        // keep this row's prefetch in this row step: without the fence
        // the scheduler sinks every prefetch of the window to its end
        __builtin_amdgcn_sched_barrier(0);
    };

    // The trip count is padded to whole windows so that the unrolled body
    // has no per-row branches: fetches are unconditional (rows past the grid
    // read zeros) and rows past the tile are computed but never stored.  The
    // loop body is one turn of the ring (two windows); an odd window count
    // ends with one more window, which fetches nothing.
    const int windows = (T_rows + NW - 1) / NW;
    const int T_turns = (windows / 2) * NR;
    int tb = 0;
    for (; tb < T_turns; tb += NR)
        static_for(std::make_integer_sequence<int, NR>{},
                   [&](auto U) __attribute__((always_inline)) { step(decltype(U)::value, tb + U, true); });
    if (windows & 1)
        static_for(std::make_integer_sequence<int, NW>{},
                   [&](auto U) __attribute__((always_inline)) { step(decltype(U)::value, tb + U, false); });
    if constexpr (CHECK) {
        *rmax = nan_max(*rmax, cmax);
        *rrel = nan_maxf(*rrel, crel);
    }
}

}  // namespace sdev
}  // namespace twg
