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

struct RelaxCtl {
    RelaxConfig c;
    int32_t phase;
    int32_t parity;        // FP32 field: 0 in psi, 1 in alt
    int32_t cparity;       // correction: 0 in e, 1 in alt
    int32_t fresh;         // psi holds the rounded polished field
    int32_t wide;          // psi64 holds the (widened or polished) field
    int32_t pass;          // passes of the current solve
    int32_t next_check;    // pass of the next residual check
    int32_t last_check;    // pass of the last check
    int32_t lead_check;    // the next check ends a correction start phase
    int32_t solve_checks;  // checks of the current solve
    int32_t stalls;
    int32_t checks;        // residual evaluations of the whole call
    int32_t rounds;        // defect-correction updates
    int32_t slot;          // slots that did work
    int32_t status;
    int32_t pad;
    uint32_t ticket;       // workgroups of the current slot that have finished
    uint32_t pad2;
    unsigned long long rmax, rrel;  // bit patterns of the slot's maxima (atomic max)
    int64_t last_chunk, since, sweeps, polish_sweeps;
    double tol_cur, r_prev, best, rate, rate_dc;
    double residual32, residual_rel, residual;
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
        // one huge chunk); the first prediction of a call aims short
        const double want = log(c->tol_cur / r) / log(c->rate);
        const double k = c->checks <= 1 ? 0.8 : 1.05;
        chunk = (int64_t)fmin(ceil(want * k), 1e12) + S;
        chunk = chunk > 8 * S ? chunk : 8 * S;
        if (c->last_chunk > 0) {
            const int64_t cap = 2 * c->last_chunk > 64 * S ? 2 * c->last_chunk : 64 * S;
            chunk = chunk < cap ? chunk : cap;
        }
    }
    int64_t passes = (chunk + S - 1) / S;
    const int64_t pmax = c->c.max_sweeps / S;
    if (c->pass + passes > pmax) passes = pmax - c->pass;
    if (passes < 1) passes = 1;
    c->last_chunk = passes * S;
    return (int32_t)passes;
}

// start the correction solve of one defect-correction round from residual r64
__device__ void start_correction(RelaxCtl *c, double r64)
{
    c->phase = PH_CORR;
    c->pass = 0;
    c->cparity = 0;
    c->solve_checks = 0;
    // at most four decades per round (the FP32 correction keeps about that
    // much relative accuracy), and no further than a third of what is left
    c->tol_cur = fmax(r64 * 1e-4, c->c.need / 3.0);
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
        c->next_check = lp < pmax ? lp : pmax;
        c->lead_check = 1;
    } else {
        // the defect is the solve's initial residual (e = 0)
        c->solve_checks = 1;
        c->next_check = next_passes(c, r64);
        c->lead_check = 0;
    }
}

// end of the FP32 solve at pass p (the result is this pass's input)
__device__ void end_solve(RelaxCtl *c, bool conv, double r, double rel)
{
    if (c->phase == PH_PLAIN) {
        c->sweeps = (int64_t)c->pass * c->c.S;
        c->residual32 = r;
        c->residual_rel = rel;
        c->residual = r;
        c->status = conv ? TWG_OK : TWG_NOT_CONVERGED;
        c->phase = c->c.polish ? PH_DEFECT32 : PH_FINISH;
    } else {
        c->polish_sweeps += (int64_t)c->pass * c->c.S;
        c->rate_dc = c->rate;
        c->phase = PH_UPDATE;
    }
}

// a residual check of an FP32 solve at pass c->pass
__device__ void on_check(RelaxCtl *c, double r, double rel)
{
    ++c->checks;
    const bool initial = c->solve_checks == 0 || c->lead_check;
    ++c->solve_checks;
    if (r != r) {
        c->status = TWG_EINVAL;
        c->phase = PH_FINISH;
        return;
    }
    if (initial) {
        c->best = r;
        c->stalls = 0;
        c->since = 0;
        c->lead_check = 0;
    } else {
        const int64_t chunk = (int64_t)(c->pass - c->last_check) * c->c.S;
        if (r < c->r_prev && chunk > 0) {
            const double q = pow(r / c->r_prev, 1.0 / (double)chunk);
            if (q > 0.0 && q < 1.0) c->rate = q;
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
    c->last_check = c->pass;
    if (r <= c->tol_cur) {
        end_solve(c, true, r, rel);
        return;
    }
    if ((int64_t)c->pass * c->c.S >= c->c.max_sweeps || (c->stalls >= 3 && c->since >= kStallSweeps)) {
        end_solve(c, false, r, rel);
        return;
    }
    c->next_check = c->pass + next_passes(c, r);
}

// a defect: polish done, or the next correction round
__device__ void on_defect(RelaxCtl *c, double r64)
{
    ++c->checks;
    c->residual = r64;
    c->wide = 1;
    if (r64 != r64) {
        c->status = TWG_EINVAL;
        c->phase = PH_FINISH;
    } else if (r64 <= c->c.need) {
        c->status = TWG_OK;
        c->phase = PH_FINISH;
    } else if (c->rounds >= c->c.max_rounds) {
        c->status = TWG_NOT_CONVERGED;
        c->phase = PH_FINISH;
    } else {
        start_correction(c, r64);
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
    if (c->phase == PH_DONE) {
        w = 1ull << 63;
    } else {
        int64_t next = slot_now + 1;  // DEFECT, UPDATE and FINISH decide in their own slot
        if (c->phase == PH_PLAIN || c->phase == PH_CORR) next = slot_now + (c->next_check - c->pass) + 1;
        w = (unsigned long long)(next + 1);
    }
    *reinterpret_cast<volatile unsigned long long *>(mirror) = w;
    __threadfence_system();
}

__device__ void controller(RelaxCtl *c, const SlotArgs &a, int phase, bool check, bool forced)
{
    const int32_t slot_now = c->slot++;
    const double r = bitsd(__hip_atomic_exchange(&c->rmax, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const double rel = bitsd(__hip_atomic_exchange(&c->rrel, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    bool decided = true;
    switch (phase) {
    case PH_PLAIN:
    case PH_CORR: {
        const int32_t pass = c->pass;
        if (check) on_check(c, r, rel);
        // the pass's output is the field from here on, unless the solve
        // ended at this check (its input is the result)
        if (c->phase == phase && c->pass == pass) {
            if (phase == PH_PLAIN) c->parity ^= 1;
            else c->cparity ^= 1;
            c->pass = pass + 1;
            decided = check;
        }
        break;
    }
    case PH_DEFECT32:
    case PH_DEFECT64: on_defect(c, r); break;
    case PH_UPDATE:
        ++c->rounds;
        c->fresh = 1;
        c->phase = PH_DEFECT64;
        break;
    case PH_FINISH:
        if (forced) c->status = TWG_NOT_CONVERGED;
        write_stats(c, a.stats);
        c->phase = PH_DONE;
        break;
    }
    if (decided) publish(c, a.mirror, slot_now);
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
    int phase = __builtin_amdgcn_readfirstlane(c->phase);
    const bool forced = a.final_slot && phase < PH_FINISH;
    if (forced) phase = PH_FINISH;
    if (phase == PH_DONE) return;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gw = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
    const int nwaves = gridDim.x * 4;
    double m = 0.0;
    float mr = 0.0f;
    bool reduce = false, check = false;

    if (phase == PH_PLAIN || phase == PH_CORR) {
        const bool corr = phase == PH_CORR;
        const int pass = __builtin_amdgcn_readfirstlane(c->pass);
        check = pass == __builtin_amdgcn_readfirstlane(c->next_check);
        reduce = check;
        const int par = __builtin_amdgcn_readfirstlane(corr ? c->cparity : c->parity);
        float *x0 = corr ? a.e : a.psi;
        float *src = par ? a.alt : x0, *dst = par ? x0 : a.alt;
        const float om = corr ? (pass < c->c.lead_passes ? c->c.omega_lead : c->c.omega_dc) : c->c.omega;
        if (gw < a.tiles) {
            constexpr int VW = 128 - 4 * S;
            const int strip = gw % a.strips, seg = gw / a.strips;
            const int ybeg = seg * a.RH, yend = min(ybeg + a.RH, a.ny);
            const int xs = strip * VW - 2 * S;
            if (corr) {
                if (check)
                    stream_tile<float, S, true, PAIR, true, true>(src, dst, a.mask, om, a.r32, a.nx, a.ny, a.pitch,
                                                                  xs, ybeg, yend, &m, &mr);
                else
                    stream_tile<float, S, true, PAIR, true, false>(src, dst, a.mask, om, a.r32, a.nx, a.ny, a.pitch,
                                                                   xs, ybeg, yend);
            } else {
                if (check)
                    stream_tile<float, S, false, PAIR, true, true>(src, dst, a.mask, om, nullptr, a.nx, a.ny,
                                                                   a.pitch, xs, ybeg, yend, &m, &mr);
                else
                    stream_tile<float, S, false, PAIR, true, false>(src, dst, a.mask, om, nullptr, a.nx, a.ny,
                                                                    a.pitch, xs, ybeg, yend);
            }
        }
    } else if (phase == PH_DEFECT32 || phase == PH_DEFECT64) {
        reduce = true;
        const bool first = phase == PH_DEFECT32;
        const int par = __builtin_amdgcn_readfirstlane(c->parity);
        const float *u32 = par ? a.alt : a.psi;
        for_cells(a, gw, nwaves, [&](int x, int y) {
            const size_t i = (size_t)y * a.pitch + x;
            double cv;
            const double r = first ? defect_at(u32, a.nx, a.ny, a.pitch, x, y, &cv)
                                   : defect_at(a.psi64, a.nx, a.ny, a.pitch, x, y, &cv);
            const bool fr = a.mask[i] != 0;
            if (first) {
                a.psi64[i] = cv;
                a.e[i] = 0.0f;
            }
            a.r32[i] = fr ? (float)r : 0.0f;
            m = nan_max(m, fr ? fabs(r) : 0.0);
            const float ac = fabsf((float)cv);
            mr = nan_maxf(mr, fr && ac >= 1e-30f ? fabsf((float)r) * __builtin_amdgcn_rcpf(ac) : 0.0f);
        });
    } else if (phase == PH_UPDATE) {
        const int cpar = __builtin_amdgcn_readfirstlane(c->cparity);
        const float *ecur = cpar ? a.alt : a.e;
        for_cells(a, gw, nwaves, [&](int x, int y) {
            const size_t i = (size_t)y * a.pitch + x;
            double v = a.psi64[i];
            if (a.mask[i]) {
                v = v + (double)ecur[i];
                a.psi64[i] = v;
            }
            a.psi[i] = (float)v;
            a.e[i] = 0.0f;
        });
    } else {  // PH_FINISH
        const bool copy = !__builtin_amdgcn_readfirstlane(c->fresh) && __builtin_amdgcn_readfirstlane(c->parity);
        const bool widen = a.psi64 && c->c.polish && !__builtin_amdgcn_readfirstlane(c->wide);
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
    if (reduce) {
        m = wave_max(m);
        mr = wave_maxf(mr);
        if (lane == 0) {
            bm[wave] = m;
            br[wave] = mr;
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (reduce) {
        m = nan_max(nan_max(bm[0], bm[1]), nan_max(bm[2], bm[3]));
        mr = nan_maxf(nan_maxf(br[0], br[1]), nan_maxf(br[2], br[3]));
        __hip_atomic_fetch_max(&c->rmax, dbits(m), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_max(&c->rrel, dbits((double)mr), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_waitcnt(0);
    }
    const unsigned int ticket = __hip_atomic_fetch_add(&c->ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (ticket != gridDim.x - 1) return;
    __hip_atomic_exchange(&c->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    controller(c, a, phase, check, forced);
}

__global__ void k_relax_begin(RelaxCtl *c, RelaxConfig cfg)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    c->c = cfg;
    c->phase = PH_PLAIN;
    c->parity = c->cparity = c->fresh = c->wide = 0;
    c->pass = 0;
    c->next_check = 0;  // the initial field's residual, fused into pass 0
    c->last_check = 0;
    c->lead_check = 0;
    c->solve_checks = 0;
    c->stalls = 0;
    c->checks = c->rounds = c->slot = 0;
    c->status = TWG_NOT_CONVERGED;
    c->last_chunk = c->since = c->sweeps = c->polish_sweeps = 0;
    c->tol_cur = cfg.tol;
    c->r_prev = c->best = 0.0;
    c->rate = fmax((double)cfg.omega - 1.0, 0.5);
    c->rate_dc = 0.0;
    c->residual32 = c->residual_rel = c->residual = 0.0;
    __hip_atomic_exchange(&c->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_exchange(&c->rmax, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_exchange(&c->rrel, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
        TWG_SLOT_CASE(6)
        TWG_SLOT_CASE(8)
    default: return TWG_EUNSUPPORTED;
    }
#undef TWG_SLOT_CASE
    return last_status();
}

}  // namespace twg
