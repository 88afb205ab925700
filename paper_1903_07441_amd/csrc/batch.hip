// Device-driven relaxation of a batch of independent grids of any sizes on
// gfx950 (Eqs. 1-2 relaxed to a residual tolerance on every grid; the
// paper's thread-per-cell launch of section "GPU-Based Parallel
// Implementation" applied to many grids at once).
//
// A batch solve is a sequence of launches of one kernel, k_batch_slot, each
// a "slot": one streamed pass of S red-black sweeps over every tile of every
// grid still active, the tiles of all grids in one launch.  Each grid runs
// its own solve: its pass number and ping-pong parity follow from the slot
// number and the slot at which its current run of passes began, its
// residual checks are fused into the pass that checks (stream_tile's CHECK
// path, one FP64 maximum per grid), and its stop rules are those of the
// single-grid solve (tolerance, sweep budget, a stall at the FP32 rounding
// floor).  Checks happen only at "event" slots, multiples of a quantum, so
// that many grids share them.  Each slot is followed by a one-workgroup
// launch, k_batch_ctrl: at an event it runs the controller with one thread
// per grid, then rebuilds the table of the active grids' tiles that the next
// slots enumerate (one wave per entry); after any other slot it returns at
// once.  When no grid is left, one finishing slot copies back every field
// that ended in the partner buffer, and its control launch writes the
// per-grid statistics.
#include "stream_tile.h"

#include <algorithm>
#include <climits>
#include <cmath>

namespace twg {

// per grid, read by its tiles: slot k of the grid's current run does pass
// pass0 + (k - run_slot) on parity parity0 ^ ((k - run_slot) & 1); a DONE
// grid's parity0 is the buffer its result ended in
struct GridRun {
    int32_t pass0, run_slot, next_check, parity0;
    int32_t strips, tiles, mode, status;
};
// per grid, controller only
struct GridCtl {
    double r_prev, best, rate, residual, residual_rel;
    int64_t since, last_chunk, sweeps;
    int32_t last_check, stalls, checks, solve_checks;
};

namespace {

using namespace sdev;

constexpr int64_t kStallSweepsB = 256;

// everything a slot reads before its tiles, in one load
struct alignas(32) BatchHdr {
    int32_t phase;        // BP_RUN, BP_FINISH, BP_DONE
    int32_t n_active;     // grids in the active list
    int32_t total_tiles;  // tiles of the active grids
    int32_t next_event;   // slot of the next event (a check of some grid)
    int32_t events;
    int32_t pad[3];
};
enum : int32_t { BP_RUN = 0, BP_FINISH = 1, BP_DONE = 2 };
enum : int32_t { BG_ACTIVE = 0, BG_DONE = 1 };

__device__ __forceinline__ unsigned long long dbits(double d) { return (unsigned long long)__double_as_longlong(d); }
__device__ __forceinline__ double bitsd(unsigned long long b) { return __longlong_as_double((long long)b); }

// passes to the next check of grid state c at residual r (the single-grid
// solve's prediction), at least one
__device__ int64_t predict_passes(GridCtl *c, double r, const BatchArgs &a, int64_t pass)
{
    const int S = a.S;
    int64_t chunk;
    if (a.check_passes > 0) {
        chunk = (int64_t)a.check_passes * S;
    } else {
        const double want = log(a.tol / r) / log(c->rate);
        const double k = c->checks <= 1 ? 0.8 : 1.05;
        chunk = (int64_t)fmin(ceil(want * k), 1e12) + S;
        chunk = chunk > 8 * S ? chunk : 8 * S;
        if (c->last_chunk > 0) {
            const int64_t cap = 2 * c->last_chunk > 64 * S ? 2 * c->last_chunk : 64 * S;
            chunk = chunk < cap ? chunk : cap;
        }
    }
    int64_t passes = (chunk + S - 1) / S;
    const int64_t pmax = a.max_sweeps / S;
    if (pass + passes > pmax) passes = pmax - pass;
    if (passes < 1) passes = 1;
    c->last_chunk = passes * S;
    return passes;
}

// the controller's work on grid k at event slot `slot` (one thread)
__device__ void grid_event(const BatchArgs &a, int k, int slot)
{
    GridRun *gr = a.run + k;
    if (gr->mode != BG_ACTIVE) return;
    const int dk = slot - gr->run_slot;
    const int64_t pass = (int64_t)gr->pass0 + dk;
    if (pass < gr->next_check) return;  // not this grid's check
    GridCtl *c = a.ctl + k;
    const int par = (gr->parity0 ^ dk) & 1;
    const double r = bitsd(__hip_atomic_exchange(a.rmax + k, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const double rel = bitsd(__hip_atomic_exchange(a.rrel + k, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    ++c->checks;
    const bool initial = c->solve_checks == 0;
    ++c->solve_checks;
    c->residual = r;
    c->residual_rel = rel;
    bool stop = false;
    int status = TWG_NOT_CONVERGED;
    if (r != r || rel != rel) {
        stop = true;
        status = TWG_EINVAL;
    } else {
        if (initial) {
            c->best = r;
            c->stalls = 0;
            c->since = 0;
        } else {
            const int64_t chunk = (pass - c->last_check) * a.S;
            if (r < c->r_prev && chunk > 0) {
                const double q = pow(r / c->r_prev, 1.0 / (double)chunk);
                if (q > 0.0 && q < 1.0) c->rate = q;
            }
            // the max-norm residual is not monotone: progress is judged
            // against the best residual, over a span of sweeps
            if (r < 0.9 * c->best) {
                c->best = r;
                c->stalls = 0;
                c->since = 0;
            } else {
                c->since += chunk;
                ++c->stalls;
            }
        }
        c->r_prev = r;
        c->last_check = (int32_t)pass;
        if (r <= a.tol) {
            stop = true;
            status = TWG_OK;
        } else if (pass * a.S >= a.max_sweeps || (c->stalls >= 3 && c->since >= kStallSweepsB)) {
            stop = true;
        }
    }
    if (stop) {
        // the result is this pass's input
        gr->mode = BG_DONE;
        gr->status = status;
        gr->parity0 = par;
        c->sweeps = pass * a.S;
        return;
    }
    // the pass ran: the next run starts at the next slot with its output;
    // the check's slot is rounded up to a multiple of the event quantum
    const int64_t passes = predict_passes(c, r, a, pass);
    const int64_t q = a.quantum > 0 ? a.quantum : 1;
    const int64_t cs = (((int64_t)slot + passes + q - 1) / q) * q;
    int64_t pcheck = pass + (cs - slot);
    const int64_t pmax = a.max_sweeps / a.S;
    if (pcheck > pmax) pcheck = pmax > pass ? pmax : pass + 1;
    gr->pass0 = (int32_t)(pass + 1);
    gr->run_slot = slot + 1;
    gr->parity0 = par ^ 1;
    gr->next_check = (int32_t)pcheck;
}

// decision published for a blocking caller: the slot of the next event
// (+1) in the low word, bit 63 when the solve is done
__device__ void publish_b(unsigned long long *mirror, const BatchHdr *h, int slot_now)
{
    if (!mirror) return;
    unsigned long long w;
    if (h->phase == BP_DONE) w = 1ull << 63;
    else if (h->phase == BP_FINISH) w = (unsigned long long)(slot_now + 2);
    else w = (unsigned long long)(h->next_event + 1);
    *reinterpret_cast<volatile unsigned long long *>(mirror) = w;
    __threadfence_system();
}

// the active list (every thread of one workgroup): the tiles of the grids
// still active, in grid order, and the slot of the next check of any of
// them; no grid left ends the run
__device__ void build_list(const BatchArgs &a, BatchHdr *h, int slot)
{
    __shared__ int gsum[256], tsum[256], smin[256];
    const int tid = threadIdx.x;
    const int per = (a.n + 255) / 256;
    const int k0 = min(tid * per, a.n), k1 = min(k0 + per, a.n);
    int cnt = 0, tiles = 0, nxt = INT_MAX;
    for (int k = k0; k < k1; ++k) {
        const GridRun gr = a.run[k];
        if (gr.mode != BG_ACTIVE) continue;
        ++cnt;
        tiles += gr.tiles;
        nxt = min(nxt, gr.run_slot + (gr.next_check - gr.pass0));
    }
    gsum[tid] = cnt;
    tsum[tid] = tiles;
    smin[tid] = nxt;
    __syncthreads();
    // inclusive scans (Hillis-Steele) of the counts, and the minimum
    for (int o = 1; o < 256; o <<= 1) {
        const int v1 = tid >= o ? gsum[tid - o] : 0;
        const int v2 = tid >= o ? tsum[tid - o] : 0;
        const int v3 = tid >= o ? smin[tid - o] : INT_MAX;
        __syncthreads();
        gsum[tid] += v1;
        tsum[tid] += v2;
        smin[tid] = min(smin[tid], v3);
        __syncthreads();
    }
    // the tile table of the next slots: entry i = (grid, tile of the grid)
    int tpos = tsum[tid] - tiles;
    for (int k = k0; k < k1; ++k) {
        const GridRun gr = a.run[k];
        if (gr.mode != BG_ACTIVE) continue;
        for (int t = 0; t < gr.tiles; ++t) a.tiles[tpos + t] = make_int2(k, t);
        tpos += gr.tiles;
    }
    __syncthreads();
    if (tid == 0) {
        const int n_act = gsum[255];
        h->n_active = n_act;
        h->total_tiles = tsum[255];
        if (n_act == 0) {
            h->phase = BP_FINISH;
            h->next_event = slot + 1;
        } else {
            h->next_event = smin[255];
        }
    }
}

// statistics of every grid (the last workgroup of the finishing slot);
// forced: grids still active end at the pass this slot would have run
__device__ void batch_stats(const BatchArgs &a, int slot, bool forced)
{
    for (int k = threadIdx.x; k < a.n; k += 256) {
        const GridRun gr = a.run[k];
        const GridCtl c = a.ctl[k];
        hpf_stats s = {};
        const int nx = a.grids[k].nx, ny = a.grids[k].ny;
        s.wbound = ((double)min(nx, ny) + 1.0) * ((double)min(nx, ny) + 1.0) / 2.0;
        if (gr.mode == BG_ACTIVE && forced) {
            s.sweeps = ((int64_t)gr.pass0 + (slot - gr.run_slot)) * a.S;
            s.status = TWG_NOT_CONVERGED;
        } else {
            s.sweeps = c.sweeps;
            s.status = gr.status;
        }
        s.residual = s.residual32 = c.residual;
        s.residual_rel = c.residual_rel;
        s.cert_bound = c.residual * s.wbound;
        s.omega = a.grids[k].omega;
        s.checks = c.checks;
        a.stats[k] = s;
    }
}

// At least three waves per SIMD (at most 168 VGPRs): the batch has several
// tiles per SIMD, and the deepest tiling (S = 8) otherwise takes 171 and
// runs at two (46.9 against 46.1 ms for the 256-grid batch).
template <int S, bool PAIR>
__global__ __launch_bounds__(256, 3) void k_batch_slot(BatchArgs a)
{
    BatchHdr *hp = static_cast<BatchHdr *>(a.hdr);
    const BatchHdr h = *hp;
    const int phase = __builtin_amdgcn_readfirstlane(h.phase);
    const int total = __builtin_amdgcn_readfirstlane(h.total_tiles);
    if (phase == BP_DONE) return;
    const int slot = a.slot;
    const bool forced = a.final_slot && phase == BP_RUN;
    const bool finish = phase == BP_FINISH || forced;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int gw = b * 4 + wave;

    if (!finish) {
        if (gw < total) {
            const int2 te = a.tiles[gw];
            const int k = __builtin_amdgcn_readfirstlane(te.x);
            const int t = __builtin_amdgcn_readfirstlane(te.y);
            const GridRun gr = a.run[k];
            const BatchGrid g = a.grids[k];
            const int strips = __builtin_amdgcn_readfirstlane(gr.strips);
            const int strip = t % strips, seg = t / strips;
            const int dk = slot - __builtin_amdgcn_readfirstlane(gr.run_slot);
            const int pass = __builtin_amdgcn_readfirstlane(gr.pass0) + dk;
            const bool check = pass >= __builtin_amdgcn_readfirstlane(gr.next_check);
            const int par = (__builtin_amdgcn_readfirstlane(gr.parity0) ^ dk) & 1;
            float *x0 = a.psi + g.off, *x1 = a.alt + g.off;
            float *src = par ? x1 : x0, *dst = par ? x0 : x1;
            const uint8_t *m = a.mask + g.off;
            constexpr int VW = 128 - 4 * S;
            const int ybeg = seg * a.RH, yend = min(ybeg + a.RH, g.ny);
            const int xs = strip * VW - 2 * S;
            if (check) {
                double rm = 0.0;
                float rr = 0.0f;
                stream_tile<float, S, kSrcNone, PAIR, true, kStoreBack, false>(src, dst, m, g.omega, nullptr, g.nx,
                                                                               g.ny, g.pitch, xs, ybeg, yend, &rm,
                                                                               &rr);
                for (int o = 32; o > 0; o >>= 1) {
                    rm = nan_max(rm, __shfl_xor(rm, o));
                    rr = nan_maxf(rr, __shfl_xor(rr, o));
                }
                if (lane == 0) {
                    __hip_atomic_fetch_max(a.rmax + k, dbits(rm), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_fetch_max(a.rrel + k, dbits((double)rr), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
            } else {
                stream_tile<float, S, kSrcNone, PAIR, false, kStoreBack, false>(src, dst, m, g.omega, nullptr,
                                                                                g.nx, g.ny, g.pitch, xs, ybeg,
                                                                                yend);
            }
        }
    } else {
        // copy back every field that ended in the partner buffer: work item
        // (entry e of the static column-block list, row chunk c of 32)
        const int items = a.n_blocks * 32;
        for (int it = gw; it < items; it += gridDim.x * 4) {
            const int e = it >> 5, c = it & 31;
            const int2 bk = a.blocks[e];
            const GridRun gr = a.run[bk.x];
            int par = gr.parity0;
            if (gr.mode == BG_ACTIVE) par = (par ^ (slot - gr.run_slot)) & 1;
            if (!par) continue;
            const BatchGrid g = a.grids[bk.x];
            const int x = bk.y * 64 + lane;
            const int rows = (g.ny + 31) / 32, y0 = c * rows, y1 = min(y0 + rows, g.ny);
            if (x < g.nx)
                for (int y = y0; y < y1; ++y) {
                    const size_t i = (size_t)g.off + (size_t)y * g.pitch + x;
                    a.psi[i] = a.alt[i];
                }
        }
    }

}

// The decision that follows every slot (one workgroup, launched after the
// slot on the same stream, so it sees every tile's maxima and fields): at an
// event, the controller of every grid that checked and the new active list;
// at the end, the per-grid statistics.  Any other slot returns at once.
__global__ __launch_bounds__(256) void k_batch_ctrl(BatchArgs a)
{
    BatchHdr *hp = static_cast<BatchHdr *>(a.hdr);
    const BatchHdr h = *hp;
    const int phase = __builtin_amdgcn_readfirstlane(h.phase);
    if (phase == BP_DONE) return;
    const int slot = a.slot;
    const bool forced = a.final_slot && phase == BP_RUN;
    if (phase == BP_FINISH || forced) {
        batch_stats(a, slot, forced);
        __syncthreads();
        if (threadIdx.x == 0) {
            hp->phase = BP_DONE;
            publish_b(a.mirror, hp, slot);
        }
        return;
    }
    if (slot < __builtin_amdgcn_readfirstlane(h.next_event)) return;
    for (int k = threadIdx.x; k < a.n; k += 256) grid_event(a, k, slot);
    __syncthreads();
    build_list(a, hp, slot);
    if (threadIdx.x == 0) {
        hp->events += 1;
        publish_b(a.mirror, hp, slot);
    }
}

// ---- small grids, each solved whole in one workgroup's LDS -------------
// (grids flagged TWG_GRID_LDS that fit).  The workgroup loads grid k's field
// (FP32) and free mask into LDS and runs
// its whole solve there: an FP64 residual check, then S red-black sweeps,
// repeated until a stop rule of the tiled path holds (tolerance, sweep
// budget, a stall: no 10 % gain on the best residual over three checks and
// at least kStallSweepsB sweeps).  A cell's update is the untiled sweep's
// (update.h), so the field after N sweeps has the bits the tiled path gives
// after N sweeps (red-black half-sweeps do not depend on the order of their
// cells), and the check is the fused check's expression.  The field goes
// back to HBM once; there is no launch per pass.  Every sweep still reads
// and writes each cell in LDS, where a streamed tile keeps S sweeps in
// registers per load: 1024 grids of 64 to 160 cells a side take 19.8 ms
// here against 8.6 ms in the tiled passes, so this is opt-in.
constexpr int kLdsThreads = 1024;
constexpr int kLdsWaves = kLdsThreads / 64;

__global__ __launch_bounds__(kLdsThreads) void k_batch_lds(BatchArgs a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ double part_r[kLdsWaves];
    __shared__ float part_q[kLdsWaves];
    const int k = a.lds_list[blockIdx.x];
    const BatchGrid g = a.grids[k];
    const int nx = g.nx, ny = g.ny;
    float *u = reinterpret_cast<float *>(lds_raw);
    uint8_t *m = lds_raw + (((size_t)nx * ny * sizeof(float) + 15) & ~size_t(15));
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // one wave per row, its lanes along the row
    for (int y = wave; y < ny; y += kLdsWaves)
        for (int x = lane; x < nx; x += 64) {
            const size_t gi = (size_t)g.off + (size_t)y * g.pitch + x;
            u[y * nx + x] = a.psi[gi];
            m[y * nx + x] = a.mask[gi];
        }
    __syncthreads();
    const float omega = g.omega;
    const int hw = (nx + 1) >> 1;
    // neighbours outside the grid read as fixed cells with value 0
    auto nbrs = [&](int x, int y, int i, float &e, float &w, float &s, float &n_) {
        e = x + 1 < nx ? u[i + 1] : 0.0f;
        w = x > 0 ? u[i - 1] : 0.0f;
        s = y + 1 < ny ? u[i + nx] : 0.0f;
        n_ = y > 0 ? u[i - nx] : 0.0f;
    };
    // colour c: the cells with (x + y) % 2 == c
    auto half_sweep = [&](int c) {
        for (int y = wave; y < ny; y += kLdsWaves) {
            const int x0 = (y + c) & 1;
            for (int kx = lane; kx < hw; kx += 64) {
                const int x = 2 * kx + x0;
                if (x >= nx) continue;
                const int i = y * nx + x;
                float e, w, s, n_;
                nbrs(x, y, i, e, w, s, n_);
                u[i] = upd(u[i], (e + w) + n_, s, m[i] ? omega : 0.0f);
            }
        }
        __syncthreads();
    };
    int64_t sweeps = 0, since = 0;
    int checks = 0, stalls = 0, status = TWG_NOT_CONVERGED;
    double best = 0.0, r = 0.0, rel = 0.0;
    for (;;) {
        // FP64 residual of the current field over its FREE cells (and the
        // relative one, a diagnostic, as the fused check evaluates it)
        double rm = 0.0;
        float qm = 0.0f;
        for (int y = wave; y < ny; y += kLdsWaves)
            for (int x = lane; x < nx; x += 64) {
                const int i = y * nx + x;
                if (!m[i]) continue;
                float e, w, s, n_;
                nbrs(x, y, i, e, w, s, n_);
                const double c0 = (double)u[i];
                const double d = ((((double)e + (double)w) + ((double)s + (double)n_)) * 0.25) - c0;
                rm = nan_max(rm, fabs(d));
                const float ac = fabsf(u[i]);
                qm = nan_maxf(qm, ac >= 1e-30f ? fabsf((float)d) * __builtin_amdgcn_rcpf(ac) : 0.0f);
            }
        for (int o = 32; o > 0; o >>= 1) {
            rm = nan_max(rm, __shfl_xor(rm, o));
            qm = nan_maxf(qm, __shfl_xor(qm, o));
        }
        if (lane == 0) {
            part_r[wave] = rm;
            part_q[wave] = qm;
        }
        __syncthreads();
        r = part_r[0];
        float q = part_q[0];
        for (int v = 1; v < kLdsWaves; ++v) {
            r = nan_max(r, part_r[v]);
            q = nan_maxf(q, part_q[v]);
        }
        rel = (double)q;
        __syncthreads();  // the partials are rewritten at the next check
        // every thread takes the same decision from the same maxima
        ++checks;
        bool stop = false;
        if (r != r || rel != rel) {
            stop = true;
            status = TWG_EINVAL;
        } else {
            if (checks == 1 || r < 0.9 * best) {
                best = r;
                stalls = 0;
                since = 0;
            } else {
                since += a.S;
                ++stalls;
            }
            if (r <= a.tol) {
                stop = true;
                status = TWG_OK;
            } else if (sweeps >= a.max_sweeps || (stalls >= 3 && since >= kStallSweepsB)) {
                stop = true;
            }
        }
        if (stop) break;
        for (int q2 = 0; q2 < a.S; ++q2) {
            half_sweep(0);
            half_sweep(1);
        }
        sweeps += a.S;
    }
    for (int y = wave; y < ny; y += kLdsWaves)
        for (int x = lane; x < nx; x += 64) a.psi[(size_t)g.off + (size_t)y * g.pitch + x] = u[y * nx + x];
    if (tid == 0) {
        GridRun *gr = a.run + k;
        gr->mode = BG_DONE;
        gr->status = status;
        gr->parity0 = 0;
        GridCtl *c = a.ctl + k;
        c->sweeps = sweeps;
        c->residual = r;
        c->residual_rel = rel;
        c->checks = checks;
    }
}

// set-up of a batch solve (one workgroup): every grid active, checking its
// initial field in slot 0
__global__ __launch_bounds__(256) void k_batch_begin(BatchArgs a)
{
    BatchHdr *h = static_cast<BatchHdr *>(a.hdr);
    const int VW = 128 - 4 * a.S;
    for (int k = threadIdx.x; k < a.n; k += 256) {
        const BatchGrid g = a.grids[k];
        GridRun gr;
        gr.strips = (g.nx + VW - 1) / VW;
        gr.tiles = g.lds ? 0 : gr.strips * ((g.ny + a.RH - 1) / a.RH);
        gr.pass0 = 0;
        gr.run_slot = 0;
        gr.next_check = 0;
        gr.parity0 = 0;
        // an LDS grid takes no part in the passes: k_batch_lds, launched
        // next, solves it and records its outcome
        gr.mode = g.lds ? BG_DONE : BG_ACTIVE;
        gr.status = TWG_NOT_CONVERGED;
        a.run[k] = gr;
        GridCtl c = {};
        c.rate = fmax((double)g.omega - 1.0, 0.5);
        a.ctl[k] = c;
        a.rmax[k] = 0ull;
        a.rrel[k] = 0ull;
    }
    if (threadIdx.x == 0) {
        h->phase = BP_RUN;
        h->events = 0;
    }
    __syncthreads();
    build_list(a, h, 0);
}

int last_status_b() { return hipGetLastError() == hipSuccess ? TWG_OK : TWG_EDEVICE; }

}  // namespace

size_t batch_hdr_bytes() { return (sizeof(BatchHdr) + 255) & ~size_t(255); }
size_t batch_run_bytes() { return sizeof(GridRun); }
size_t batch_ctl_bytes() { return sizeof(GridCtl); }

int launch_batch_begin(const BatchArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_batch_begin, dim3(1), dim3(256), 0, st, a);
    return last_status_b();
}

size_t batch_lds_bytes(long long cells)
{
    return (((size_t)cells * sizeof(float) + 15) & ~size_t(15)) + (size_t)cells;
}

int launch_batch_lds(const BatchArgs &a, size_t lds_bytes, size_t *lds_attr, hipStream_t st)
{
    if (a.n_lds < 1) return TWG_OK;
    // raised once per context and size (outside any capture: the first call
    // of a batch is made outside one)
    if (lds_bytes > *lds_attr) {
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_batch_lds),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes) != hipSuccess)
            return TWG_EDEVICE;
        *lds_attr = lds_bytes;
    }
    hipLaunchKernelGGL(k_batch_lds, dim3(a.n_lds), dim3(kLdsThreads), lds_bytes, st, a);
    return last_status_b();
}

int launch_batch_slot(const BatchArgs &a, int max_tiles, bool pair, hipStream_t st)
{
    // one wave per tile of the whole batch (the finishing slot's copy loops
    // over its items with the same waves)
    const int blocks = std::max(1, (max_tiles + 3) / 4);
#define TWG_BSLOT_CASE(SV)                                                                          \
    case SV:                                                                                        \
        if (pair)                                                                                   \
            hipLaunchKernelGGL((k_batch_slot<SV, true>), dim3(blocks), dim3(256), 0, st, a);        \
        else                                                                                        \
            hipLaunchKernelGGL((k_batch_slot<SV, false>), dim3(blocks), dim3(256), 0, st, a);       \
        break;
    switch (a.S) {
        TWG_BSLOT_CASE(1)
        TWG_BSLOT_CASE(2)
        TWG_BSLOT_CASE(3)
        TWG_BSLOT_CASE(4)
        TWG_BSLOT_CASE(5)
        TWG_BSLOT_CASE(6)
        TWG_BSLOT_CASE(7)
        TWG_BSLOT_CASE(8)
    default: return TWG_EUNSUPPORTED;
    }
#undef TWG_BSLOT_CASE
    hipLaunchKernelGGL(k_batch_ctrl, dim3(1), dim3(256), 0, st, a);
    return last_status_b();
}

}  // namespace twg
