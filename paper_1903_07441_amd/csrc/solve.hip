// Device-driven relaxation for gfx950: the convergence control of hpf_relax
// (Eqs. 1-2 relaxed to a residual tolerance; the FP64 defect-correction
// polish that certifies the field by the discrete maximum principle) runs on
// the GPU, so a solve needs no host round trip and can be captured into a
// graph.
//
// A solve is a sequence of launches of ONE kernel, k_relax_slot, each a
// "slot" whose work the device decides from a control block (RelaxCtl) in
// device memory:
//   PLAIN     one streamed pass of S red-black sweeps of the FP32 field
//             (ping-pong between the caller's psi and the context's alt);
//   DEFECT32  the first FP64 defect: psi64 = psi widened, r32 = the FP64
//             residual avg4(psi64) - psi64 rounded to FP32, e = 0;
//   CORR      one streamed pass of the FP32 correction solve
//             (I - J) e = r32 (ping-pong e / alt);
//   UPDATE    psi64 += e on FREE cells, psi = psi64 rounded, e = 0;
//   DEFECT64  the FP64 defect of psi64;
//   FINISH    the FP32 result into psi if it ended in alt, stats written;
//   DONE      nothing: surplus slots return at once.
// A pass measures the FP64 residual of its input field when the control
// block schedules a check there (stream_tile's CHECK path: no extra launch).
// Every workgroup of a slot adds its maxima to the block with atomics and
// then takes a ticket; the workgroup that takes the last ticket runs the
// controller (one thread):
// it reads the maxima, applies the stop rules (tolerance, sweep budget,
// rounding-floor stall), predicts the next check from the measured
// contraction, and moves the phase.  A decision is also published to a
// host-mapped word, which lets a blocking caller keep just enough slots
// queued; an asynchronous caller enqueues a fixed number of slots and one
// final slot that finishes whatever is left.
#include "stream_tile.h"

#include <cmath>

namespace twg {

namespace {

using namespace sdev;

enum : int { PH_PLAIN = 0, PH_DEFECT32, PH_CORR, PH_UPDATE, PH_DEFECT64, PH_FINISH, PH_DONE };

// a solve stops at the FP32 rounding floor after three checks without a 10 %
// gain on its best residual that together span at least this many sweeps
constexpr int64_t kStallSweeps = 256;

// The words every slot reads when it starts, loaded together (one scalar
// load): a run of passes of the current solve began at slot run_slot with
// pass number `pass` and the field (or correction) in buffer parity
// `parity` (`cparity`); slot k of the run does pass pass + (k - run_slot) on
// parity ^ ((k - run_slot) & 1), so a pass that does not check writes
// nothing to the control block.
struct alignas(32) RelaxHot {
    int32_t phase;
    int32_t parity;        // FP32 field at run_slot: 0 in psi, 1 in alt
    int32_t cparity;       // correction at run_slot: 0 in e, 1 in alt
    int32_t pass;          // pass number of slot run_slot
    int32_t run_slot;
    int32_t next_check;    // pass of the next residual check
    int32_t fresh;         // psi holds the rounded polished field
    int32_t wide;          // psi64 holds the (widened or polished) field
};

constexpr int kParts = 128;

struct RelaxCtl {
    RelaxHot h;
    RelaxConfig c;
    int32_t last_check;    // pass of the last check
    int32_t lead_check;    // the next check ends a correction start phase
    int32_t solve_checks;  // checks of the current solve
    int32_t stalls;
    int32_t checks;        // residual evaluations of the whole call
    int32_t rounds;        // defect-correction updates
    int32_t status;
    int32_t pad;
    uint32_t ticket;       // workgroups of the current slot that have finished
    uint32_t pad2;
    int64_t last_chunk, since, sweeps, polish_sweeps;
    double tol_cur, r_prev, best, rate, rate_dc;
    double residual32, residual_rel, residual;
    // bit patterns of the slot's maxima, spread over kParts words so that
    // the workgroups' atomics seldom meet on one address (workgroup b uses
    // part[b % kParts]); the slot's last workgroup combines and clears them
    unsigned long long part[kParts][2];
};

__device__ __forceinline__ unsigned long long dbits(double d) { return (unsigned long long)__double_as_longlong(d); }
__device__ __forceinline__ double bitsd(unsigned long long b) { return __longlong_as_double((long long)b); }

__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = nan_max(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_maxf(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = nan_maxf(v, __shfl_xor(v, o));
    return v;
}

// ---- controller (one thread of the last workgroup of a slot) --------------

// predicted passes to the next check of an FP32 solve at residual r
__device__ int32_t next_passes(RelaxCtl *c, double r)
{
    const int S = c->c.S;
    int64_t chunk;
    if (c->c.check_passes > 0) {
        chunk = (int64_t)c->c.check_passes * S;
    } else {
        // sweeps the measured contraction predicts, at most twice the last
        // chunk (a rate near 1 near the rounding floor must not turn into
        // one huge chunk); the prediction after the FP32 solve's initial
        // check (the first of a call, the rate still a guess) aims short
        const double want = log(c->tol_cur / r) / log(c->rate);
        const double k = c->h.phase == PH_PLAIN && c->solve_checks <= 1 ? 0.8 : 1.05;
        chunk = (int64_t)fmin(ceil(want * k), 1e12) + S;
        chunk = chunk > 8 * S ? chunk : 8 * S;
        if (c->last_chunk > 0) {
            const int64_t cap = 2 * c->last_chunk > 64 * S ? 2 * c->last_chunk : 64 * S;
            chunk = chunk < cap ? chunk : cap;
        }
    }
    int64_t passes = (chunk + S - 1) / S;
    const int64_t pmax = c->c.max_sweeps / S;
    if (c->h.pass + passes > pmax) passes = pmax - c->h.pass;
    if (passes < 1) passes = 1;
    c->last_chunk = passes * S;
    return (int32_t)passes;
}

// start the correction solve of one defect-correction round from residual r64
__device__ void start_correction(RelaxCtl *c, double r64, int32_t first_slot)
{
    c->h.phase = PH_CORR;
    c->h.pass = 0;
    c->h.cparity = 0;
    c->h.run_slot = first_slot;
    c->solve_checks = 0;
    // at most four decades per round (the FP32 correction keeps about that
    // much relative accuracy), and no further than the target with a 25 %
    // margin: after the FP64 update the field's residual is the correction
    // solve's own residual plus the rounding of the defect to FP32 (a
    // relative 6e-8) and of the update (about 1e-16)
    c->tol_cur = fmax(r64 * 1e-4, c->c.need / 1.25);
    c->r_prev = r64;
    c->best = r64;
    c->stalls = 0;
    c->since = 0;
    c->last_chunk = 0;
    c->last_check = 0;
    c->rate = (c->rate_dc > 0.0 && c->rate_dc < 1.0) ? c->rate_dc : fmax((double)c->c.omega_dc - 1.0, 0.5);
    if (c->c.lead_passes > 0 && c->c.max_sweeps >= c->c.S) {
        // the start phase runs at the smaller factor, then a check
        int32_t lp = c->c.lead_passes;
        const int32_t pmax = (int32_t)(c->c.max_sweeps / c->c.S);
        c->h.next_check = lp < pmax ? lp : pmax;
        c->lead_check = 1;
    } else {
        // the defect is the solve's initial residual (e = 0)
        c->solve_checks = 1;
        c->h.next_check = next_passes(c, r64);
        c->lead_check = 0;
    }
}

// end of the FP32 solve at pass p (the result is this pass's input)
__device__ void end_solve(RelaxCtl *c, bool conv, double r, double rel)
{
    if (c->h.phase == PH_PLAIN) {
        c->sweeps = (int64_t)c->h.pass * c->c.S;
        c->residual32 = r;
        c->residual_rel = rel;
        c->residual = r;
        c->status = conv ? TWG_OK : TWG_NOT_CONVERGED;
        c->h.phase = c->c.polish ? PH_DEFECT32 : PH_FINISH;
    } else {
        c->polish_sweeps += (int64_t)c->h.pass * c->c.S;
        c->rate_dc = c->rate;
        c->h.phase = PH_UPDATE;
    }
}

// a residual check of an FP32 solve at pass c->h.pass
__device__ void on_check(RelaxCtl *c, double r, double rel)
{
    ++c->checks;
    const bool initial = c->solve_checks == 0 || c->lead_check;
    ++c->solve_checks;
    if (r != r) {
        c->status = TWG_EINVAL;
        c->h.phase = PH_FINISH;
        return;
    }
    if (initial) {
        c->best = r;
        c->stalls = 0;
        c->since = 0;
        c->lead_check = 0;
    } else {
        const int64_t chunk = (int64_t)(c->h.pass - c->last_check) * c->c.S;
        double q = 1.0;
        if (r < c->r_prev && chunk > 0) {
            q = pow(r / c->r_prev, 1.0 / (double)chunk);
            if (q > 0.0 && q < 1.0) c->rate = q;
        }
        // A correction solve that contracts at less than half the speed its
        // factor gives every mode once the factor is at or above a domain's
        // optimum (omega - 1 per sweep) has met the FP32 rounding floor of
        // its correction: a correction with a large smooth part leaves FP32
        // residual noise of ~1e-7 times its own size, which can lie above
        // the solve's target.  The round ends there; the FP64 update and
        // the next round's exact defect carry on from it.  Judged over at
        // least 128 sweeps.
        if (c->h.phase == PH_CORR && chunk >= 128) {
            const double w = (double)c->c.omega_dc;
            if (q > 1.0 - 0.5 * (2.0 - w)) {
                // the next round's first prediction starts from the nominal
                // rate, not from the floor's
                c->rate = fmax(w - 1.0, 0.5);
                end_solve(c, false, r, rel);
                return;
            }
        }
        // the max-norm residual is not monotone, so progress is judged
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
    c->last_check = c->h.pass;
    if (r <= c->tol_cur) {
        end_solve(c, true, r, rel);
        return;
    }
    if ((int64_t)c->h.pass * c->c.S >= c->c.max_sweeps || (c->stalls >= 3 && c->since >= kStallSweeps)) {
        end_solve(c, false, r, rel);
        return;
    }
    c->h.next_check = c->h.pass + next_passes(c, r);
}

// a defect: polish done, or the next correction round.  The first defect
// of a kept field's polish (no check has run yet) also stands in for the
// FP32 stage's initial check: it evaluates the same FP64 expression over
// the same FREE cells of the same field, so when that residual meets tol the
// FP32 stage ends as it would at that check, with no sweep; else the FP32
// solve runs from its own initial check and the first defect comes again.
__device__ void on_defect(RelaxCtl *c, double r64, double rel, int32_t slot_now)
{
    if (c->h.phase == PH_DEFECT32 && c->checks == 0 && r64 == r64 && !(r64 <= c->tol_cur)) {
        ++c->checks;
        c->h.phase = PH_PLAIN;
        c->h.pass = 0;
        c->h.run_slot = slot_now + 1;
        c->h.next_check = 0;
        return;
    }
    if (c->h.phase == PH_DEFECT32 && c->checks == 0 && r64 == r64) {
        c->sweeps = 0;
        c->residual32 = r64;
        c->residual_rel = rel;
        c->status = TWG_OK;
    }
    ++c->checks;
    c->residual = r64;
    c->h.wide = 1;
    if (r64 != r64) {
        c->status = TWG_EINVAL;
        c->h.phase = PH_FINISH;
    } else if (r64 <= c->c.need) {
        c->status = TWG_OK;
        c->h.phase = PH_FINISH;
    } else if (c->rounds >= c->c.max_rounds) {
        c->status = TWG_NOT_CONVERGED;
        c->h.phase = PH_FINISH;
    } else {
        start_correction(c, r64, slot_now + 1);
    }
}

__device__ void write_stats(const RelaxCtl *c, hpf_stats *s)
{
    s->sweeps = c->sweeps;
    s->polish_sweeps = c->polish_sweeps;
    s->residual = c->residual;
    s->residual32 = c->residual32;
    s->cert_bound = c->residual * c->c.wbound;
    s->wbound = c->c.wbound;
    s->omega = c->c.omega;
    s->status = c->status;
    s->polish_rounds = c->rounds;
    s->checks = c->checks;
    s->residual_rel = c->residual_rel;
}

// decision published for a blocking caller: the slot of the next decision
// (+1) in the low word, bit 63 when the solve is done
__device__ void publish(const RelaxCtl *c, unsigned long long *mirror, int32_t slot_now)
{
    if (!mirror) return;
    unsigned long long w;
    if (c->h.phase == PH_DONE) {
        w = 1ull << 63;
    } else {
        int64_t next = slot_now + 1;  // DEFECT, UPDATE and FINISH decide in their own slot
        if (c->h.phase == PH_PLAIN || c->h.phase == PH_CORR) next = slot_now + (c->h.next_check - c->h.pass) + 1;
        w = (unsigned long long)(next + 1);
    }
    *reinterpret_cast<volatile unsigned long long *>(mirror) = w;
    __threadfence_system();
}

// The controller of a slot that decides: a checking pass (at pass p, on
// buffer parity par), a defect, an update, or the finish (`forced`: the
// final slot ends a solve whose phase was `was`, at pass p on parity par
// if that phase was a solve).
__device__ void controller_on(RelaxCtl *c, const SlotArgs &a, int phase, int was, bool forced, int32_t p,
                              int32_t par, double r, double rel)
{
    const int32_t slot_now = a.slot;
    switch (phase) {
    case PH_PLAIN:
    case PH_CORR: {
        // the run's state at this pass, then the check
        c->h.pass = p;
        c->h.run_slot = slot_now;
        if (phase == PH_PLAIN) c->h.parity = par;
        else c->h.cparity = par;
        on_check(c, r, rel);
        // the pass's output is the field from here on, unless the solve
        // ended at this check (its input is the result)
        if (c->h.phase == phase && c->h.pass == p) {
            if (phase == PH_PLAIN) c->h.parity = par ^ 1;
            else c->h.cparity = par ^ 1;
            c->h.pass = p + 1;
            c->h.run_slot = slot_now + 1;
        }
        break;
    }
    case PH_DEFECT32:
    case PH_DEFECT64: on_defect(c, r, rel, slot_now); break;
    case PH_UPDATE:
        ++c->rounds;
        c->h.fresh = 1;
        c->h.phase = PH_DEFECT64;
        break;
    case PH_FINISH:
        if (forced) {
            c->status = TWG_NOT_CONVERGED;
            // a solve cut short between checks: its passes so far count,
            // and the FP32 field is where its last pass wrote it
            if (was == PH_PLAIN) {
                c->h.parity = par;
                c->sweeps = (int64_t)p * c->c.S;
            } else if (was == PH_CORR) {
                c->polish_sweeps += (int64_t)p * c->c.S;
            }
        }
        write_stats(c, a.stats);
        c->h.phase = PH_DONE;
        break;
    }
    publish(c, a.mirror, slot_now);
}

// The controller works on a copy of the control block in registers: read in
// one batch of independent loads and written back once, instead of a chain
// of dependent global accesses (each a memory latency).  The words other
// workgroups update atomically (ticket, maxima) are read and reset here with
// atomics and not written back.
__device__ void controller(RelaxCtl *cg, const SlotArgs &a, int phase, int was, bool forced, int32_t p, int32_t par,
                           double r, double rel)
{
    RelaxCtl c = *cg;
    controller_on(&c, a, phase, was, forced, p, par, r, rel);
    cg->h = c.h;
    cg->last_check = c.last_check;
    cg->lead_check = c.lead_check;
    cg->solve_checks = c.solve_checks;
    cg->stalls = c.stalls;
    cg->checks = c.checks;
    cg->rounds = c.rounds;
    cg->status = c.status;
    cg->last_chunk = c.last_chunk;
    cg->since = c.since;
    cg->sweeps = c.sweeps;
    cg->polish_sweeps = c.polish_sweeps;
    cg->tol_cur = c.tol_cur;
    cg->r_prev = c.r_prev;
    cg->best = c.best;
    cg->rate = c.rate;
    cg->rate_dc = c.rate_dc;
    cg->residual32 = c.residual32;
    cg->residual_rel = c.residual_rel;
    cg->residual = c.residual;
}

// ---- element-wise and stencil phases ----------------------------------------

// the cells of a slot's elementwise phases: work items are (row, run of 256
// columns), spread over all waves of the launch; each lane takes four
// columns 64 apart
template <typename F>
__device__ __forceinline__ void for_cells(const SlotArgs &a, int gw, int nwaves, F fn)
{
    const int lane = threadIdx.x & 63;
    const int runs = (a.nx + 255) / 256;
    const int items = a.ny * runs;
    for (int it = gw; it < items; it += nwaves) {
        const int y = it / runs, x0 = (it - y * runs) * 256 + lane;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int x = x0 + 64 * j;
            if (x < a.nx) fn(x, y);
        }
    }
}

// The same cells, K work items at a time, each cell split into `load`
// (reads and arithmetic, returning a value) and `store` (writes): every load
// of the 4K cells is issued before the first store, so a wave has that many
// cells' loads in flight instead of one cell's (the stores could alias the
// loads, so the compiler keeps them in program order).  A cell outside the
// grid loads cell (0, 0) and stores nothing.
template <int K, typename L, typename St>
__device__ __forceinline__ void for_cells_batched(const SlotArgs &a, int gw, int nwaves, L load, St store)
{
    using V = decltype(load(0, 0));
    const int lane = threadIdx.x & 63;
    const int runs = (a.nx + 255) / 256;
    const int items = a.ny * runs;
    for (int it0 = gw; it0 < items; it0 += K * nwaves) {
        V v[K][4];
        int ys[K], xs[K][4];
        bool ok[K][4];
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const int it = it0 + q * nwaves;
            const bool in = it < items;
            const int y = in ? it / runs : 0;
            const int x0 = in ? (it - y * runs) * 256 + lane : 0;
            ys[q] = y;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                xs[q][j] = x0 + 64 * j;
                ok[q][j] = in && xs[q][j] < a.nx;
                v[q][j] = load(ok[q][j] ? xs[q][j] : 0, ok[q][j] ? y : 0);
            }
        }
#pragma unroll
        for (int q = 0; q < K; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (ok[q][j]) store(xs[q][j], ys[q], v[q][j]);
    }
}
// a store written through L2 at agent scope (sc1)
template <typename T>
__device__ __forceinline__ void st_through(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
struct DefectCell {
    double c, r;
    bool fr;
};
struct UpdateCell {
    double v;
    float e;
    bool fr;
};

// FP64 residual of u at (x, y) with the neighbours outside the grid at 0;
// every load unconditional (clamped, then zeroed), as in the standalone
// residual kernels
template <typename T>
__device__ __forceinline__ double defect_at(const T *u, int nx, int ny, int pitch, int x, int y, double *c_out)
{
    const size_t row = (size_t)y * pitch;
    const int xe = min(x + 1, nx - 1), xw = max(x - 1, 0);
    const double ue = (double)u[row + xe], uw = (double)u[row + xw];
    const double us = (double)u[(size_t)min(y + 1, ny - 1) * pitch + x];
    const double un = (double)u[(size_t)max(y - 1, 0) * pitch + x];
    const double c = (double)u[row + x];
    const double e = x + 1 < nx ? ue : 0.0;
    const double w = x > 0 ? uw : 0.0;
    const double s = y + 1 < ny ? us : 0.0;
    const double n = y > 0 ? un : 0.0;
    *c_out = c;
    return ((e + w) + (s + n)) * 0.25 - c;
}

template <int S, bool PAIR>
__global__ __launch_bounds__(256) void k_relax_slot(SlotArgs a)
{
    RelaxCtl *c = static_cast<RelaxCtl *>(a.ctl);
    // the hot words in one load; everything below is wave-uniform
    const RelaxHot h = *static_cast<const RelaxHot *>(a.ctl);
    const int was = __builtin_amdgcn_readfirstlane(h.phase);
    // position in the current run of passes (solve phases), derived before
    // any branch so that the words above arrive in one load
    const int k = __builtin_amdgcn_readfirstlane(a.slot - h.run_slot);
    const int pass = __builtin_amdgcn_readfirstlane(h.pass) + k;
    const int par = (__builtin_amdgcn_readfirstlane(was == PH_CORR ? h.cparity : h.parity) ^ k) & 1;
    const int next_check = __builtin_amdgcn_readfirstlane(h.next_check);
    const int hfresh = __builtin_amdgcn_readfirstlane(h.fresh), hwide = __builtin_amdgcn_readfirstlane(h.wide);
    const int hpar = __builtin_amdgcn_readfirstlane(h.parity), hcpar = __builtin_amdgcn_readfirstlane(h.cparity);
    if (was == PH_DONE) return;
    const bool forced = a.final_slot && was < PH_FINISH;
    const int phase = forced ? (int)PH_FINISH : was;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gw = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
    const int nwaves = gridDim.x * 4;
    double m = 0.0;
    float mr = 0.0f;
    bool reduce = false;

    if (phase == PH_PLAIN || phase == PH_CORR) {
        const bool corr = phase == PH_CORR;
        const bool check = pass >= next_check;
        reduce = check;
        float *x0 = corr ? a.e : a.psi;
        float *src = par ? a.alt : x0, *dst = par ? x0 : a.alt;
        const float om = corr ? (pass < a.lead_passes ? a.omega_lead : a.omega_dc) : a.omega;
        if (gw < a.tiles) {
            constexpr int VW = 128 - 4 * S;
            const int strip = gw % a.strips, seg = gw / a.strips;
            const int ybeg = seg * a.RH, yend = min(ybeg + a.RH, a.ny);
            const int xs = strip * VW - 2 * S;
            if (corr) {
                if (check)
                    stream_tile<float, S, kSrcF, PAIR, true>(src, dst, a.mask, om, a.r32, a.nx, a.ny, a.pitch,
                                                             xs, ybeg, yend, &m, &mr);
                else
                    stream_tile<float, S, kSrcC, PAIR, false>(src, dst, a.mask, om,
                                                              pass < a.lead_passes ? a.clead : a.cdc, a.nx,
                                                              a.ny, a.pitch, xs, ybeg, yend);
            } else {
                if (check)
                    stream_tile<float, S, kSrcNone, PAIR, true>(src, dst, a.mask, om, nullptr, a.nx, a.ny,
                                                                a.pitch, xs, ybeg, yend, &m, &mr);
                else
                    stream_tile<float, S, kSrcNone, PAIR, false>(src, dst, a.mask, om, nullptr, a.nx, a.ny,
                                                                 a.pitch, xs, ybeg, yend);
            }
        }
        // a pass that does not check decides nothing: the next slot derives
        // its pass and buffers from its own slot number
        if (!check) return;
    } else if (phase == PH_DEFECT32 || phase == PH_DEFECT64) {
        reduce = true;
        const bool first = phase == PH_DEFECT32;
        const int fpar = hpar;
        const float *u32 = fpar ? a.alt : a.psi;
        // the defect's maxima, and its outputs written through L2 (as the
        // passes' field rows are, so the kernel's end has nothing to write
        // back): the widened field and a cleared correction the first time
        auto store = [&](int x, int y, const DefectCell &d) {
            const size_t i = (size_t)y * a.pitch + x;
            if (first) {
                st_through(a.psi64 + i, d.c);
                st_through(a.e + i, 0.0f);
            }
            // the correction solves' source, and its products with their
            // two factors, formed here once instead of in every pass
            const float f = d.fr ? (float)d.r : 0.0f;
            st_through(a.r32 + i, f);
            st_through(a.cdc + i, a.omega_dc * f);
            if (a.lead_passes > 0) st_through(a.clead + i, a.omega_lead * f);
            m = nan_max(m, d.fr ? fabs(d.r) : 0.0);
            const float ac = fabsf((float)d.c);
            mr = nan_maxf(mr, d.fr && ac >= 1e-30f ? fabsf((float)d.r) * __builtin_amdgcn_rcpf(ac) : 0.0f);
        };
        auto load = [&](const auto *u, int x, int y) {
            DefectCell d;
            d.r = defect_at(u, a.nx, a.ny, a.pitch, x, y, &d.c);
            d.fr = a.mask[(size_t)y * a.pitch + x] != 0;
            return d;
        };
        if (first)
            for_cells_batched<2>(a, gw, nwaves, [&](int x, int y) { return load(u32, x, y); }, store);
        else
            for_cells_batched<2>(a, gw, nwaves, [&](int x, int y) { return load(a.psi64, x, y); }, store);
    } else if (phase == PH_UPDATE) {
        const int cpar = hcpar;
        const float *ecur = cpar ? a.alt : a.e;
        // ecur may be e itself: every cell's correction is read before any
        // cell's is cleared
        for_cells_batched<2>(
            a, gw, nwaves,
            [&](int x, int y) {
                const size_t i = (size_t)y * a.pitch + x;
                return UpdateCell{a.psi64[i], ecur[i], a.mask[i] != 0};
            },
            [&](int x, int y, const UpdateCell &u) {
                const size_t i = (size_t)y * a.pitch + x;
                double v = u.v;
                if (u.fr) {
                    v = v + (double)u.e;
                    st_through(a.psi64 + i, v);
                }
                st_through(a.psi + i, (float)v);
                st_through(a.e + i, 0.0f);
            });
    } else {  // PH_FINISH
        // the FP32 field's buffer: a solve cut short between checks left it
        // where its last pass wrote
        const int fpar = was == PH_PLAIN ? par : hpar;
        const bool copy = !hfresh && fpar;
        const bool widen = a.psi64 && a.polish && !hwide;
        if (copy || widen) {
            for_cells(a, gw, nwaves, [&](int x, int y) {
                const size_t i = (size_t)y * a.pitch + x;
                const float v = copy ? a.alt[i] : a.psi[i];
                if (copy) a.psi[i] = v;
                if (widen) a.psi64[i] = (double)v;
            });
        }
    }

    // maxima, then the ticket, one per workgroup: the block's maxima are
    // combined in LDS, its atomics are performed before it takes its ticket
    // (a wait on their results), so the block that takes the last ticket
    // reads the maxima of every block
    __shared__ double bm[4];
    __shared__ float br[4];
    __shared__ int last;
    if (reduce) {
        m = wave_max(m);
        mr = wave_maxf(mr);
        if (lane == 0) {
            bm[wave] = m;
            br[wave] = mr;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (reduce) {
            m = nan_max(nan_max(bm[0], bm[1]), nan_max(bm[2], bm[3]));
            mr = nan_maxf(nan_maxf(br[0], br[1]), nan_maxf(br[2], br[3]));
            unsigned long long *pp = c->part[blockIdx.x % kParts];
            __hip_atomic_fetch_max(pp, dbits(m), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_max(pp + 1, dbits((double)mr), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_s_waitcnt(0);
        }
        const unsigned int ticket =
            __hip_atomic_fetch_add(&c->ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        last = ticket == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    // the last workgroup: the slot's maxima from the kParts words (one
    // thread each, read and cleared), combined as bit patterns like the
    // atomics (non-negative doubles order like their patterns; a NaN's is
    // larger than +inf's)
    unsigned long long pr = 0ull, pq = 0ull;
    if (threadIdx.x < kParts) {
        pr = __hip_atomic_exchange(&c->part[threadIdx.x][0], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        pq = __hip_atomic_exchange(&c->part[threadIdx.x][1], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    for (int o = 32; o > 0; o >>= 1) {
        pr = max(pr, (unsigned long long)__shfl_xor((long long)pr, o));
        pq = max(pq, (unsigned long long)__shfl_xor((long long)pq, o));
    }
    __shared__ unsigned long long wr[4], wq[4];
    if (lane == 0) {
        wr[wave] = pr;
        wq[wave] = pq;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    pr = max(max(wr[0], wr[1]), max(wr[2], wr[3]));
    pq = max(max(wq[0], wq[1]), max(wq[2], wq[3]));
    __hip_atomic_exchange(&c->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    controller(c, a, phase, was, forced, pass, par, bitsd(pr), bitsd(pq));
}

__global__ void k_relax_begin(RelaxCtl *c, RelaxConfig cfg)
{
    if (blockIdx.x != 0) return;
    for (int i = threadIdx.x; i < kParts; i += blockDim.x) {
        __hip_atomic_store(&c->part[i][0], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&c->part[i][1], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x != 0) return;
    c->c = cfg;
    c->h.phase = cfg.kept ? PH_DEFECT32 : PH_PLAIN;
    c->h.parity = c->h.cparity = c->h.fresh = c->h.wide = 0;
    c->h.pass = 0;
    c->h.run_slot = 0;
    c->h.next_check = 0;  // the initial field's residual, fused into pass 0
    c->last_check = 0;
    c->lead_check = 0;
    c->solve_checks = 0;
    c->stalls = 0;
    c->checks = c->rounds = 0;
    c->status = TWG_NOT_CONVERGED;
    c->last_chunk = c->since = c->sweeps = c->polish_sweeps = 0;
    c->tol_cur = cfg.tol;
    c->r_prev = c->best = 0.0;
    c->rate = fmax((double)cfg.omega - 1.0, 0.5);
    c->rate_dc = 0.0;
    c->residual32 = c->residual_rel = c->residual = 0.0;
    __hip_atomic_exchange(&c->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

int last_status() { return hipGetLastError() == hipSuccess ? TWG_OK : TWG_EDEVICE; }

}  // namespace

size_t relax_ctl_bytes() { return (sizeof(RelaxCtl) + 255) & ~size_t(255); }

int launch_relax_begin(void *ctl, const RelaxConfig &cfg, hipStream_t st)
{
    hipLaunchKernelGGL(k_relax_begin, dim3(1), dim3(64), 0, st, static_cast<RelaxCtl *>(ctl), cfg);
    return last_status();
}

int launch_relax_slot(const SlotArgs &a, int S, hipStream_t st)
{
    const int blocks = (a.tiles + 3) / 4;
#define TWG_SLOT_CASE(SV)                                                                          \
    case SV:                                                                                       \
        if (a.pair)                                                                                \
            hipLaunchKernelGGL((k_relax_slot<SV, true>), dim3(blocks), dim3(256), 0, st, a);       \
        else                                                                                       \
            hipLaunchKernelGGL((k_relax_slot<SV, false>), dim3(blocks), dim3(256), 0, st, a);      \
        break;
    switch (S) {
        TWG_SLOT_CASE(1)
        TWG_SLOT_CASE(2)
        TWG_SLOT_CASE(3)
        TWG_SLOT_CASE(4)
        TWG_SLOT_CASE(5)
        TWG_SLOT_CASE(6)
        TWG_SLOT_CASE(7)
        TWG_SLOT_CASE(8)
    default: return TWG_EUNSUPPORTED;
    }
#undef TWG_SLOT_CASE
    return last_status();
}

}  // namespace twg
