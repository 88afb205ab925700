// C ABI of libtwg.so: argument checks, scratch management and the host-side
// convergence control of the relaxation.  The arithmetic runs in the kernels
// of raster.hip, relax.hip and descend.hip.
#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "twg_internal.h"

// Scratch of hpf_relax_async_noalloc, for callers that cannot allocate: one
// file-scope device array, a copy of which each GPU the library runs on holds
// until the process ends.  Its layout for a grid of n = pitch * ny <=
// kNoAllocMaxCells cells: the control block and default stats at 0, then the
// FP32 ping-pong partner, the FP32 defect, correction and products of the
// defect with the correction factors, and the free mask,
// each at a fixed offset sized for the largest grid.  Host code never names
// the array in a launch or copy: it uses the device address that
// hipGetSymbolAddress gave for the current device (noalloc_scratch below).
namespace {
constexpr size_t kNoAllocMaxCells = size_t(1) << 22;  // e.g. 2048 x 2048
constexpr size_t kNoAllocCtlBytes = 4096;
constexpr size_t kNoAllocAlt = kNoAllocCtlBytes;
constexpr size_t kNoAllocPol = kNoAllocAlt + 4 * kNoAllocMaxCells;
constexpr size_t kNoAllocMask = kNoAllocPol + 16 * kNoAllocMaxCells;
constexpr size_t kNoAllocBytes = kNoAllocMask + kNoAllocMaxCells;
constexpr int kNoAllocDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kNoAllocDevices] = {};

// the device address of `scratch` on `device` (which must be current),
// looked up once per device
int noalloc_scratch(int device, void **out)
{
    if (device < 0 || device >= kNoAllocDevices) return TWG_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return TWG_EDEVICE;
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return TWG_OK;
}
}  // namespace

namespace twg {

int set_err(twg_ctx *ctx, int code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return code;
}

int ensure(twg_ctx *ctx, void **buf, size_t *have, size_t need)
{
    if (*have >= need) return TWG_OK;
    if (*buf) {
        hipDeviceSynchronize();
        hipFree(*buf);
        *buf = nullptr;
        *have = 0;
    }
    need = (need + 4095) & ~size_t(4095);
    if (hipMalloc(buf, need) != hipSuccess) {
        *buf = nullptr;
        return set_err(ctx, TWG_ENOMEM, "scratch allocation of " + std::to_string(need) + " bytes failed");
    }
    *have = need;
    return TWG_OK;
}

int check_grid(twg_ctx *ctx, const twg_grid &g)
{
    if (g.nx < 1 || g.ny < 1 || g.nx > 32767 || g.ny > 32767)
        return set_err(ctx, TWG_EINVAL, "grid sides must be in [1, 32767]");
    if (g.pitch < g.nx) return set_err(ctx, TWG_EINVAL, "pitch must be >= nx");
    if ((long long)g.pitch * g.ny >= (1LL << 31))
        return set_err(ctx, TWG_EINVAL, "pitch * ny must be below 2^31 elements");
    if (g.pitch > 65536) return set_err(ctx, TWG_EINVAL, "pitch must be <= 65536");
    return TWG_OK;
}

}  // namespace twg

using namespace twg;

namespace {

// passes per captured graph (even: the ping-pong ends where it began).  The
// GPU idles about 8 us between two graph launches but not between two plain
// kernel launches, so the graphs are long enough to make that idle time small
// (under 1 % of 64 passes at 2048 x 2048).
constexpr int kGraphPasses = 64;
// A solve counts as stalled (at its rounding floor) after three checks
// without a 10 % gain on its best residual that together span at least this
// many sweeps; at a useful SOR factor a 10 % gain takes tens of sweeps.
constexpr int64_t kStallSweeps = 256;
constexpr size_t kMaxGraphs = 16;

// Replay `times` copies of the launch sequence that `record` issues on a
// stream, as one instantiated graph on `st`.  The graph is captured once per
// key (the launch arguments) on the context's capture stream and cached.
template <typename F>
int graph_replay(twg_ctx *ctx, const std::vector<uintptr_t> &key, hipStream_t st, int64_t times, F record)
{
    hipGraphExec_t exec = nullptr;
    for (auto &g : ctx->graphs)
        if (g.key == key) exec = g.exec;
    if (!exec) {
        if (!ctx->cap && hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking) != hipSuccess) {
            ctx->cap = nullptr;
            return TWG_EDEVICE;
        }
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return TWG_EDEVICE;
        const int rc = record(ctx->cap);
        const hipError_t e = hipStreamEndCapture(ctx->cap, &graph);
        if (rc || e != hipSuccess || !graph) {
            if (graph) hipGraphDestroy(graph);
            return rc ? rc : TWG_EDEVICE;
        }
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (ei != hipSuccess) return TWG_EDEVICE;
        if (ctx->graphs.size() >= kMaxGraphs) {
            hipStreamSynchronize(st);
            hipGraphExecDestroy(ctx->graphs.front().exec);
            ctx->graphs.erase(ctx->graphs.begin());
        }
        ctx->graphs.push_back({key, exec});
    }
    for (int64_t t = 0; t < times; ++t)
        if (hipGraphLaunch(exec, st) != hipSuccess) return TWG_EDEVICE;
    return TWG_OK;
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

double bits_to_double(unsigned long long b)
{
    double d;
    std::memcpy(&d, &b, sizeof d);
    return d;
}

// Optimal SOR factor of the open rectangle: Jacobi spectral radius of the
// 5-point average with fixed values outside an nx-by-ny grid, then Young's
// formula omega = 2 / (1 + sqrt(1 - rho^2)).
// The autotuner's family of SOR factors for a grid of side n:
// 2 / (1 + c sin(pi / (n + 1))), c = 1 being the square's optimum.
float omega_family(int n, double c)
{
    const double pi = 3.14159265358979323846;
    return (float)(2.0 / (1.0 + c * std::sin(pi / (n + 1))));
}

double omega_open(int nx, int ny)
{
    const double pi = 3.14159265358979323846;
    const double rho = 0.5 * (std::cos(pi / (nx + 1)) + std::cos(pi / (ny + 1)));
    return 2.0 / (1.0 + std::sqrt(std::max(0.0, 1.0 - rho * rho)));
}

// Sweeps per tile load and rows per tile for a grid (fixed table; the
// autotuner may override through hpf_params.sweeps_per_pass).
void default_tiling(int nx, int ny, int *S, int *RH)
{
    const long long cells = (long long)nx * ny;
    if (cells >= (1LL << 22)) { *S = 4; *RH = 32; }
    else if (cells >= (1LL << 18)) { *S = 4; *RH = 16; }
    else { *S = 2; *RH = 8; }
}

// Tiling and SOR factor for a grid: the autotuned entry of this size if the
// context has one, else the fixed table and the open-rectangle optimum.
void tiling_for(twg_ctx *ctx, int nx, int ny, int *S, int *RH, float *omega)
{
    default_tiling(nx, ny, S, RH);
    *omega = (float)omega_open(nx, ny);
    auto it = ctx->tuned.find({nx, ny});
    if (it != ctx->tuned.end()) {
        *S = it->second.S;
        *RH = it->second.RH;
        if (it->second.omega > 0.0f) *omega = it->second.omega;
    }
}

// Tile heights to try for S sweeps per load: a fixed set plus, for k = 1..kmax,
// the smallest even height whose tile count (one wave per tile) fits k rounds
// of the device's SIMDs, and the tallest height with the same row steps per
// tile.  A tile streams RH + 4S rows in whole windows of 2S + 2 row steps, so
// that height fills the last window: the same time per wave, fewer tiles.
std::vector<int> tile_heights(const twg_ctx *ctx, int nx, int ny, int S, int kmax)
{
    std::vector<int> RHs = {8, 16, 32, 64, 128};
    const int simds = 4 * std::max(1, ctx->num_cu);
    const int strips = (nx + (128 - 4 * S) - 1) / (128 - 4 * S);
    const int NW = 2 * S + 2;
    auto add = [&](int RH) {
        if (RH >= 2 && std::find(RHs.begin(), RHs.end(), RH) == RHs.end()) RHs.push_back(RH);
    };
    for (int k = 1; k <= kmax; ++k) {
        const int segs = (k * simds) / strips;
        if (segs < 1) continue;
        int RH = (ny + segs - 1) / segs;
        RH += RH & 1;
        add(RH);
        add((RH + 4 * S + NW - 1) / NW * NW - 4 * S);  // even: NW and 4S are
    }
    return RHs;
}

// FP64 tiling for a grid: the autotuned one, else 4 sweeps per load and 32 rows
void tiling64_for(twg_ctx *ctx, int nx, int ny, int *S, int *RH)
{
    *S = 4;
    *RH = 32;
    auto it = ctx->tuned.find({nx, ny});
    if (it != ctx->tuned.end() && it->second.S64 > 0) {
        *S = it->second.S64;
        *RH = it->second.RH64;
    }
}

struct Runner {
    twg_ctx *ctx;
    twg_grid g;
    const uint8_t *cls;
    hipStream_t st;
    int checks = 0;

    // results the last residual reduction wrote to ctx->host_words_dev: poll
    // its sequence number in the pinned word 2 (the host sees it a few
    // microseconds before a stream synchronisation would return), asking the
    // stream every 1024 polls whether it failed, or finished without writing
    // the word (then the check fails)
    int wait_words()
    {
        const volatile unsigned long long *w = ctx->host_words;
        const unsigned long long seq = ctx->word_seq;
        for (unsigned k = 1; w[2] != seq; ++k) {
            if (k % 1024) continue;
            const hipError_t e = hipStreamQuery(st);
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess || w[2] != seq) return TWG_EDEVICE;
        }
        std::atomic_thread_fence(std::memory_order_acquire);
        ++checks;
        return TWG_OK;
    }


    bool have_fmask = false;
    int fmask(const uint8_t **m)
    {
        if (!have_fmask) {
            int rc = ensure(ctx, &ctx->fmask, &ctx->fmask_bytes, (size_t)g.pitch * g.ny);
            if (rc) return rc;
            rc = launch_fmask(cls, static_cast<uint8_t *>(ctx->fmask), g.nx, g.ny, g.pitch, st);
            if (rc) return set_err(ctx, rc, "free mask launch failed");
            have_fmask = true;
        }
        *m = static_cast<const uint8_t *>(ctx->fmask);
        return TWG_OK;
    }

    // `sweeps` FP32 sweeps on a <-> b, S per pass (remainder one per pass);
    // on return *a holds the newest field.  Runs of kGraphPasses full passes
    // are replayed from a captured graph.
    int sweep32(float **a, float **b, const float *f, float omega, int S, int RH, int64_t sweeps)
    {
        const uint8_t *m = nullptr;
        if (int rc = fmask(&m)) return rc;
        const Geometry geo = stream_geometry(g.nx, g.ny, S, RH);
        const Geometry geo1 = stream_geometry(g.nx, g.ny, 1, RH);
        int64_t done = 0;
        const int64_t reps = ctx->use_graphs ? sweeps / ((int64_t)S * kGraphPasses) : 0;
        if (reps > 0) {
            const std::vector<uintptr_t> key = {1, (uintptr_t)*a, (uintptr_t)*b, (uintptr_t)m, (uintptr_t)f,
                                                (uintptr_t)g.nx, (uintptr_t)g.ny, (uintptr_t)g.pitch,
                                                (uintptr_t)__builtin_bit_cast(uint32_t, omega), (uintptr_t)S,
                                                (uintptr_t)RH};
            float *x = *a, *y = *b;
            int rc = graph_replay(ctx, key, st, reps, [&](hipStream_t cs) {
                for (int k = 0; k < kGraphPasses; ++k) {
                    const int e = launch_stream_f32(k % 2 ? y : x, k % 2 ? x : y, m, omega, f, g.nx, g.ny, g.pitch,
                                                    geo, cs);
                    if (e) return e;
                }
                return TWG_OK;
            });
            if (rc) return set_err(ctx, rc, "relaxation graph failed");
            done = reps * S * kGraphPasses;
        }
        while (done < sweeps) {
            const bool full = sweeps - done >= S;
            int rc = launch_stream_f32(*a, *b, m, omega, f, g.nx, g.ny, g.pitch, full ? geo : geo1, st);
            if (rc) return set_err(ctx, rc, "relaxation kernel launch failed");
            std::swap(*a, *b);
            done += full ? S : 1;
        }
        return TWG_OK;
    }

    // FP64 residual of an FP64 field
    int residual64(const double *u, double *out)
    {
        int rc = launch_resid_f64(cls, u, nullptr, g.nx, g.ny, g.pitch, ctx->rpart, ctx->host_words_dev,
                                  ++ctx->word_seq, st);
        if (!rc) rc = wait_words();
        if (rc) return set_err(ctx, rc, "residual kernel failed");
        *out = bits_to_double(ctx->host_words[0]);
        return TWG_OK;
    }

    // FP64 red-black SOR on `field` (ping-pong with ctx->alt64), four sweeps
    // per tile load, until the FP64 residual is <= tol or the budget is spent.
    int solve64(double *field, double omega, double tol, int64_t max_sweeps, int64_t *sweeps_out,
                double *res_out, bool *converged)
    {
        int rc = ensure(ctx, &ctx->alt64, &ctx->alt64_bytes, (size_t)g.pitch * g.ny * sizeof(double));
        if (rc) return rc;
        int S, RH;
        tiling64_for(ctx, g.nx, g.ny, &S, &RH);
        const Geometry geo = stream_geometry(g.nx, g.ny, S, RH);
        const uint8_t *m = nullptr;
        if ((rc = fmask(&m))) return rc;
        double *a = field, *b = reinterpret_cast<double *>(ctx->alt64);
        double r;
        rc = residual64(a, &r);
        if (rc) return rc;
        int64_t done = 0, last_chunk = 0;
        int stalls = 0;
        double rate = std::max(omega - 1.0, 0.5);
        *converged = false;
        while (true) {
            if (std::isnan(r)) return set_err(ctx, TWG_EINVAL, "non-finite value in the field");
            if (r <= tol) { *converged = true; break; }
            if (done >= max_sweeps) break;
            const double want = std::log(tol / r) / std::log(rate);
            int64_t chunk = std::max<int64_t>((int64_t)std::min(std::ceil(want * 1.05), 1e12) + S, 8 * S);
            if (last_chunk > 0) chunk = std::min(chunk, std::max<int64_t>(2 * last_chunk, 64 * S));
            chunk = ((std::min(chunk, max_sweeps - done) + S - 1) / S) * S;
            last_chunk = chunk;
            for (int64_t k = 0; k < chunk; k += S) {
                rc = launch_stream_f64(a, b, m, omega, g.nx, g.ny, g.pitch, geo, st);
                if (rc) return set_err(ctx, rc, "relaxation kernel launch failed");
                std::swap(a, b);
            }
            done += chunk;
            const double r_prev = r;
            rc = residual64(a, &r);
            if (rc) return rc;
            if (r < r_prev * 0.999) {
                stalls = 0;
                const double q = std::pow(r / r_prev, 1.0 / (double)chunk);
                if (q > 0.0 && q < 1.0) rate = q;
            } else if (++stalls >= 3) {
                break;
            }
        }
        if (a != field &&
            hipMemcpy2DAsync(field, (size_t)g.pitch * 8, a, (size_t)g.pitch * 8, (size_t)g.nx * 8, g.ny,
                             hipMemcpyDeviceToDevice, st) != hipSuccess)
            return set_err(ctx, TWG_EDEVICE, "copy failed");
        *sweeps_out = done;
        *res_out = r;
        return TWG_OK;
    }
};

// What a relaxation call runs with: tiling, SOR factors and the correction
// solves' start phase.
struct RelaxPlan {
    int S = 4, RH = 32;
    float omega = 1.0f, omega_dc = 1.0f;
    StartPhase lead;
};

// The plan of hpf_relax for grid g and params p: the autotuned tiling and
// factors of this size if the context has them, else the fixed table, the
// open-rectangle optimum and the correction default 2 / (1 + 2.8 sin(pi /
// (n + 1))); a caller's omega (which also runs the correction solves, with
// no start phase) and tiling override them.
RelaxPlan plan_for(twg_ctx *ctx, const twg_grid &g, const hpf_params &p)
{
    RelaxPlan pl;
    float omega_t;
    tiling_for(ctx, g.nx, g.ny, &pl.S, &pl.RH, &omega_t);
    pl.omega = p.omega > 0.0f ? p.omega : omega_t;
    pl.omega_dc = omega_family(std::max(g.nx, g.ny), 2.8);
    if (p.omega > 0.0f) {
        pl.omega_dc = p.omega;
    } else {
        auto it = ctx->tuned.find({g.nx, g.ny});
        if (it != ctx->tuned.end()) {
            if (it->second.omega_dc > 0.0f) pl.omega_dc = it->second.omega_dc;
            pl.lead = it->second.lead_dc;
        }
    }
    if (p.sweeps_per_pass) pl.S = p.sweeps_per_pass;
    if (p.rows_per_tile) pl.RH = p.rows_per_tile;
    return pl;
}

// Defect-correction rounds a polish may take.
constexpr int kMaxRounds = 12;
// Slots a blocking solve keeps queued beyond the device's next decision.
constexpr int64_t kSlotMargin = 3;

// The device-driven solve of hpf_relax (polish 0 or 1): field init, free
// mask, the control block's begin kernel, then slots of k_relax_slot.
// slots > 0: exactly that many slots and a final one, all asynchronous;
// the stats land in stats_dev.  slots == 0: the host keeps slots queued just
// beyond the next decision the device publishes (it never waits for a
// residual), stops when the device reports the solve done, then waits for
// the stream and copies the stats to *stats_host.
// Scratch of the device-driven relaxation of a grid of n = pitch * ny cells:
// the FP32 ping-pong partner (4n bytes), with polish the FP32 defect, the
// correction and the defect's products with the two correction factors
// (16n), the free mask (n), and the control block followed by a default
// device hpf_stats (relax_ctl_bytes() + 256).
struct RelaxBufs {
    float *alt = nullptr;
    float *pol = nullptr;
    uint8_t *fmask = nullptr;
    char *ctl = nullptr;
};

// the context's scratch, allocated (or grown) here
int relax_bufs_ctx(twg_ctx *ctx, const twg_grid &g, bool polish, RelaxBufs *b)
{
    const size_t n = (size_t)g.pitch * g.ny;
    int rc = ensure(ctx, &ctx->alt, &ctx->alt_bytes, n * sizeof(float));
    if (!rc && polish) rc = ensure(ctx, &ctx->pol, &ctx->pol_bytes, 4 * n * sizeof(float));
    if (!rc) rc = ensure(ctx, &ctx->fmask, &ctx->fmask_bytes, n);
    if (!rc) rc = ensure(ctx, &ctx->ctl, &ctx->ctl_bytes, relax_ctl_bytes() + 256);
    if (rc) return rc;
    b->alt = static_cast<float *>(ctx->alt);
    b->pol = polish ? static_cast<float *>(ctx->pol) : nullptr;
    b->fmask = static_cast<uint8_t *>(ctx->fmask);
    b->ctl = static_cast<char *>(ctx->ctl);
    return TWG_OK;
}

int relax_device(twg_ctx *ctx, const twg_grid &g, const uint8_t *cls, float *psi, double *psi64,
                 const hpf_params &p, const RelaxPlan &pl, const RelaxBufs &bufs, int64_t slots,
                 hpf_stats *stats_dev, hpf_stats *stats_host, hipStream_t st)
{
    const size_t n = (size_t)g.pitch * g.ny;
    int rc = TWG_OK;
    char *ctl = bufs.ctl;
    hpf_stats *dstats = stats_dev ? stats_dev : reinterpret_cast<hpf_stats *>(ctl + relax_ctl_bytes());
    const int cap = stream_rows_cap(g.pitch, (int)sizeof(float), pl.S);
    const Geometry geo = stream_geometry(g.nx, g.ny, pl.S, std::min(pl.RH, cap));
    const double wb = std::pow((double)std::min(g.nx, g.ny) + 1.0, 2) / 2.0;

    rc = launch_field_init(cls, psi, g.nx, g.ny, g.pitch, p.init, p.goal_x, p.goal_y, st);
    if (!rc) rc = launch_fmask(cls, bufs.fmask, g.nx, g.ny, g.pitch, st);
    if (rc) return set_err(ctx, rc, "relaxation set-up launch failed");
    RelaxConfig cfg;
    cfg.tol = p.tol;
    cfg.need = p.polish ? (p.tol_cert > 0.0 ? std::min(p.tol, p.tol_cert / wb) : p.tol) : 0.0;
    cfg.wbound = wb;
    cfg.max_sweeps = p.max_sweeps;
    cfg.omega = pl.omega;
    cfg.omega_dc = pl.omega_dc;
    cfg.omega_lead = pl.lead.omega;
    cfg.lead_passes = pl.lead.sweeps > 0 ? (int32_t)((pl.lead.sweeps + pl.S - 1) / pl.S) : 0;
    cfg.S = pl.S;
    cfg.polish = p.polish ? 1 : 0;
    cfg.check_passes = p.check_passes;
    cfg.max_rounds = kMaxRounds;
    cfg.kept = cfg.polish && p.init == HPF_INIT_KEEP ? 1 : 0;
    rc = launch_relax_begin(ctl, cfg, st);
    if (rc) return set_err(ctx, rc, "relaxation begin launch failed");

    SlotArgs a;
    a.mask = bufs.fmask;
    a.psi = psi;
    a.alt = bufs.alt;
    a.r32 = p.polish ? bufs.pol : nullptr;
    a.e = p.polish ? a.r32 + n : nullptr;
    a.cdc = p.polish ? a.r32 + 2 * n : nullptr;
    a.clead = p.polish ? a.r32 + 3 * n : nullptr;
    a.psi64 = p.polish ? psi64 : nullptr;
    a.ctl = ctl;
    a.stats = dstats;
    a.nx = g.nx;
    a.ny = g.ny;
    a.pitch = g.pitch;
    a.strips = geo.strips;
    a.RH = geo.RH;
    a.tiles = geo.tiles;
    const auto al8 = [](const void *q) { return (reinterpret_cast<uintptr_t>(q) & 7) == 0; };
    a.pair = g.nx % 2 == 0 && g.pitch % 2 == 0 && al8(psi) && al8(a.alt) && (!p.polish || (al8(a.r32) && al8(a.e) && al8(a.cdc) && al8(a.clead)));
    a.final_slot = 0;
    a.slot = 0;
    a.polish = cfg.polish;
    a.omega = cfg.omega;
    a.omega_dc = cfg.omega_dc;
    a.omega_lead = cfg.omega_lead;
    a.lead_passes = cfg.lead_passes;

    if (slots > 0) {
        a.mirror = nullptr;
        for (int64_t k = 0; k < slots; ++k) {
            a.slot = (int)k;
            if ((rc = launch_relax_slot(a, pl.S, st))) return set_err(ctx, rc, "relaxation slot launch failed");
        }
        a.final_slot = 1;
        a.slot = (int)slots;
        rc = launch_relax_slot(a, pl.S, st);
        return rc ? set_err(ctx, rc, "relaxation slot launch failed") : TWG_OK;
    }

    // blocking: keep the slots up to the next published decision (plus a
    // margin) queued.  The device publishes, at every decision, the slot of
    // the next one; bit 63 marks the end.
    volatile unsigned long long *word = ctx->host_words + kMirrorWord;
    *word = 0ull;
    std::atomic_thread_fence(std::memory_order_seq_cst);
    a.mirror = ctx->host_words_dev + kMirrorWord;
    int64_t queued = 0, target = 1 + kSlotMargin;
    unsigned long long seen = 0;
    int idle = 0;
    for (unsigned polls = 0;;) {
        const unsigned long long w = *word;
        if (w >> 63) break;
        if (w != seen) {
            seen = w;
            idle = 0;
            target = std::max<int64_t>(target, (int64_t)(w & 0xffffffffull) + kSlotMargin);
        }
        if (queued < target) {
            a.slot = (int)queued;
            if ((rc = launch_relax_slot(a, pl.S, st))) return set_err(ctx, rc, "relaxation slot launch failed");
            ++queued;
            continue;
        }
        if (++polls % 1024) continue;
        const hipError_t e = hipStreamQuery(st);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) return set_err(ctx, TWG_EDEVICE, "relaxation stream failed");
        // the stream ran dry: every slot has run and its decisions are
        // visible, so the word must show a decision past the queue
        if (*word == seen && ++idle > 2)
            return set_err(ctx, TWG_EDEVICE, "relaxation control made no progress");
        target = queued + kSlotMargin;
    }
    if (hipMemcpyAsync(stats_host, dstats, sizeof(hpf_stats), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return set_err(ctx, TWG_EDEVICE, "relaxation stats read-back failed");
    return TWG_OK;
}

// relax_device on the context's scratch
int relax_device_ctx(twg_ctx *ctx, const twg_grid &g, const uint8_t *cls, float *psi, double *psi64,
                     const hpf_params &p, const RelaxPlan &pl, int64_t slots, hpf_stats *stats_dev,
                     hpf_stats *stats_host, hipStream_t st)
{
    RelaxBufs b;
    const int rc = relax_bufs_ctx(ctx, g, p.polish != 0, &b);
    if (rc) return rc;
    return relax_device(ctx, g, cls, psi, psi64, p, pl, b, slots, stats_dev, stats_host, st);
}

// Batch slots a blocking solve keeps queued beyond the device's next event.
constexpr int64_t kBatchSlotMargin = 3;
// Checks of a batch happen only at slots that are multiples of this, so that
// grids share them (an event costs every workgroup a ticket).
constexpr int kBatchQuantum = 4;
// LDS (bytes) left for the LDS worker's static variables (3 KiB at present)
constexpr size_t kLdsReserve = 8192;

// The device-driven batch relaxation (batch.hip): field init and free masks
// of every grid, the begin kernel, then slots.  slots > 0: exactly that many
// slots and a final one, asynchronous, stats into stats_dev (n entries).
// slots == 0: the host keeps slots queued just beyond the next event the
// device publishes, then copies the stats to stats_host.
int relax_batch_device(twg_ctx *ctx, int n, const twg_grid_desc *grids, const uint8_t *cls, float *psi,
                       const hpf_params *params, int64_t slots, hpf_stats *stats_dev, hpf_stats *stats_host,
                       hipStream_t st)
{
    if (n < 1 || !grids || !cls || !psi || !params)
        return set_err(ctx, TWG_EINVAL, "n >= 1, grids, cls, psi and params are required");
    if (n > kBatchMaxGrids)
        return set_err(ctx, TWG_EUNSUPPORTED, "a batch takes at most " + std::to_string(kBatchMaxGrids) + " grids");
    hpf_params p = *params;
    if (!(p.tol > 0.0)) return set_err(ctx, TWG_EINVAL, "tol must be > 0");
    if (!(p.omega >= 0.0f && p.omega < 2.0f)) return set_err(ctx, TWG_EINVAL, "omega must be in [0, 2)");
    if (p.init < HPF_INIT_KEEP || p.init > HPF_INIT_ZERO) return set_err(ctx, TWG_EINVAL, "bad init mode");
    if (p.polish) return set_err(ctx, TWG_EINVAL, "the batched relaxation has no polish");
    if (p.sweeps_per_pass && !stream_depth_supported(p.sweeps_per_pass))
        return set_err(ctx, TWG_EINVAL, "sweeps_per_pass must be 1 to 8");
    if (p.rows_per_tile && (p.rows_per_tile < 2 || (p.rows_per_tile & 1)))
        return set_err(ctx, TWG_EINVAL, "rows_per_tile must be even and >= 2");
    if (p.check_passes < 0) return set_err(ctx, TWG_EINVAL, "check_passes must be >= 0");
    if (p.max_sweeps <= 0) p.max_sweeps = 10000000;
    int big = 0;
    long long total = 0;
    for (int k = 0; k < n; ++k) {
        const twg_grid gk{grids[k].nx, grids[k].ny, grids[k].pitch};
        int rc = check_grid(ctx, gk);
        if (rc) return set_err(ctx, rc, "grid " + std::to_string(k) + ": " + ctx->err);
        if (grids[k].offset < 0) return set_err(ctx, TWG_EINVAL, "negative offset");
        if (grids[k].flags & ~TWG_GRID_LDS) return set_err(ctx, TWG_EINVAL, "unknown grid flags");
        total = std::max(total, (long long)grids[k].offset + (long long)grids[k].pitch * grids[k].ny);
        if ((long long)grids[k].nx * grids[k].ny > (long long)grids[big].nx * grids[big].ny) big = k;
    }
    hipSetDevice(ctx->device);
    int S, RH;
    float om_big;
    tiling_for(ctx, grids[big].nx, grids[big].ny, &S, &RH, &om_big);
    if (ctx->batch_S > 0) {
        S = ctx->batch_S;
        RH = ctx->batch_RH;
    }
    if (p.sweeps_per_pass) S = p.sweeps_per_pass;
    if (p.rows_per_tile) RH = p.rows_per_tile;
    const int VW = 128 - 4 * S;
    bool pair = (reinterpret_cast<uintptr_t>(psi) & 7) == 0;  // the partner and mask are context-owned (aligned)
    int max_pitch = 1;
    for (int k = 0; k < n; ++k) {
        pair = pair && grids[k].nx % 2 == 0 && grids[k].pitch % 2 == 0 && grids[k].offset % 2 == 0;
        max_pitch = std::max(max_pitch, grids[k].pitch);
    }
    RH = std::min(RH < 2 ? 2 : (RH & ~1), stream_rows_cap(max_pitch, (int)sizeof(float), S));

    // static tables: descriptors (with each grid's SOR factor), the
    // (grid, 64-column block) list and the grids small enough for one
    // workgroup's LDS that ask for it (TWG_GRID_LDS: solved whole there)
    std::vector<BatchGrid> bg(n);
    std::vector<int2> bl;
    std::vector<int> lds;
    long long max_tiles = 0;
    size_t lds_bytes = 0;
    const size_t lds_budget = ctx->lds_per_block > kLdsReserve ? ctx->lds_per_block - kLdsReserve : 0;
    for (int k = 0; k < n; ++k) {
        int s_, rh_;
        float om;
        tiling_for(ctx, grids[k].nx, grids[k].ny, &s_, &rh_, &om);
        const size_t need = batch_lds_bytes((long long)grids[k].nx * grids[k].ny);
        const int in_lds = (grids[k].flags & TWG_GRID_LDS) && need <= lds_budget;
        bg[k] = BatchGrid{grids[k].nx, grids[k].ny, grids[k].pitch, p.omega > 0.0f ? p.omega : om,
                          (long long)grids[k].offset, in_lds, 0};
        if (in_lds) {
            lds.push_back(k);
            lds_bytes = std::max(lds_bytes, need);
        } else {
            max_tiles += (long long)((grids[k].nx + VW - 1) / VW) * ((grids[k].ny + RH - 1) / RH);
        }
        for (int bx = 0; bx < (grids[k].nx + 63) / 64; ++bx) bl.push_back(make_int2(k, bx));
    }
    if (max_tiles > INT_MAX / 2 || (long long)bl.size() * 32 > INT_MAX / 2)
        return set_err(ctx, TWG_EUNSUPPORTED, "batch too large");
    // device layout: grids | blocks | LDS list | hdr | run | ctl | tile table | rmax | rrel | stats
    auto align = [](size_t v) { return (v + 255) & ~size_t(255); };
    const size_t o_grids = 0, o_blocks = align(o_grids + n * sizeof(BatchGrid));
    const size_t o_lds = align(o_blocks + bl.size() * sizeof(int2));
    const size_t o_hdr = align(o_lds + lds.size() * sizeof(int));
    const size_t o_run = align(o_hdr + batch_hdr_bytes());
    const size_t o_ctl = align(o_run + n * batch_run_bytes());
    const size_t o_tiles = align(o_ctl + n * batch_ctl_bytes());
    const size_t o_rmax = align(o_tiles + (size_t)max_tiles * sizeof(int2));
    const size_t o_rrel = align(o_rmax + n * sizeof(unsigned long long));
    const size_t o_stats = align(o_rrel + n * sizeof(unsigned long long));
    const size_t bytes = align(o_stats + n * sizeof(hpf_stats));
    const void *old_batch = ctx->batch;
    int rc = ensure(ctx, &ctx->batch, &ctx->batch_bytes, bytes);
    if (!rc) rc = ensure(ctx, &ctx->alt, &ctx->alt_bytes, (size_t)total * sizeof(float));
    if (!rc) rc = ensure(ctx, &ctx->fmask, &ctx->fmask_bytes, (size_t)total);
    if (rc) return rc;
    char *base = static_cast<char *>(ctx->batch);
    BatchGrid *d_grids = reinterpret_cast<BatchGrid *>(base + o_grids);
    int2 *d_blocks = reinterpret_cast<int2 *>(base + o_blocks);
    int *d_lds = reinterpret_cast<int *>(base + o_lds);
    // the tables are uploaded only when they differ from the last upload to
    // this buffer, so that an asynchronous call of an unchanged batch
    // enqueues kernels only (it can then be captured into a graph)
    const size_t sz_g = sizeof(BatchGrid) * bg.size(), sz_b = sizeof(int2) * bl.size(),
                 sz_l = sizeof(int) * lds.size();
    std::vector<char> sig(sz_g + sz_b + sz_l);
    std::memcpy(sig.data(), bg.data(), sz_g);
    std::memcpy(sig.data() + sz_g, bl.data(), sz_b);
    if (sz_l) std::memcpy(sig.data() + sz_g + sz_b, lds.data(), sz_l);
    if (old_batch != ctx->batch || sig != ctx->batch_sig) {
        if (hipMemcpyAsync(d_grids, bg.data(), sz_g, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(d_blocks, bl.data(), sz_b, hipMemcpyHostToDevice, st) != hipSuccess ||
            (sz_l && hipMemcpyAsync(d_lds, lds.data(), sz_l, hipMemcpyHostToDevice, st) != hipSuccess) ||
            hipStreamSynchronize(st) != hipSuccess)
            return set_err(ctx, TWG_EDEVICE, "batch table upload failed");
        ctx->batch_sig = std::move(sig);
    }
    uint8_t *const fmask = static_cast<uint8_t *>(ctx->fmask);
    rc = launch_field_init_batch(cls, psi, d_grids, d_blocks, (int)bl.size(), p.init, st);
    if (!rc) rc = launch_fmask_batch(cls, fmask, d_grids, d_blocks, (int)bl.size(), st);
    if (rc) return set_err(ctx, TWG_EDEVICE, "batch set-up failed");

    BatchArgs a;
    a.grids = d_grids;
    a.blocks = d_blocks;
    a.n_blocks = (int)bl.size();
    a.n = n;
    a.S = S;
    a.RH = RH;
    a.slot = 0;
    a.final_slot = 0;
    a.quantum = p.check_passes > 0 ? 1 : kBatchQuantum;
    a.check_passes = p.check_passes;
    a.tol = p.tol;
    a.max_sweeps = p.max_sweeps;
    a.psi = psi;
    a.alt = static_cast<float *>(ctx->alt);
    a.mask = fmask;
    a.hdr = base + o_hdr;
    a.run = reinterpret_cast<GridRun *>(base + o_run);
    a.ctl = reinterpret_cast<GridCtl *>(base + o_ctl);
    a.tiles = reinterpret_cast<int2 *>(base + o_tiles);
    a.rmax = reinterpret_cast<unsigned long long *>(base + o_rmax);
    a.rrel = reinterpret_cast<unsigned long long *>(base + o_rrel);
    a.stats = stats_dev ? stats_dev : reinterpret_cast<hpf_stats *>(base + o_stats);
    a.mirror = nullptr;
    a.lds_list = d_lds;
    a.n_lds = (int)lds.size();
    rc = launch_batch_begin(a, st);
    if (!rc) rc = launch_batch_lds(a, lds_bytes, &ctx->lds_attr, st);
    if (rc) return set_err(ctx, rc, "batch begin launch failed");
    const int mt = (int)max_tiles;

    if (slots > 0) {
        for (int64_t k = 0; k < slots; ++k) {
            a.slot = (int)k;
            if ((rc = launch_batch_slot(a, mt, pair, st))) return set_err(ctx, rc, "batch slot launch failed");
        }
        a.final_slot = 1;
        a.slot = (int)slots;
        rc = launch_batch_slot(a, mt, pair, st);
        return rc ? set_err(ctx, rc, "batch slot launch failed") : TWG_OK;
    }

    // blocking: keep the slots up to the next published event (plus a
    // margin) queued; bit 63 of the word marks the end
    volatile unsigned long long *word = ctx->host_words + kMirrorWord;
    *word = 0ull;
    std::atomic_thread_fence(std::memory_order_seq_cst);
    a.mirror = ctx->host_words_dev + kMirrorWord;
    int64_t queued = 0, target = 1 + kBatchSlotMargin;
    unsigned long long seen = 0;
    int idle = 0;
    for (unsigned polls = 0;;) {
        const unsigned long long w = *word;
        if (w >> 63) break;
        if (w != seen) {
            seen = w;
            idle = 0;
            target = std::max<int64_t>(target, (int64_t)(w & 0xffffffffull) + kBatchSlotMargin);
        }
        if (queued < target) {
            if (queued >= INT_MAX - 8) return set_err(ctx, TWG_EDEVICE, "batch slot count overflow");
            a.slot = (int)queued;
            if ((rc = launch_batch_slot(a, mt, pair, st))) return set_err(ctx, rc, "batch slot launch failed");
            ++queued;
            continue;
        }
        if (++polls % 1024) continue;
        const hipError_t e = hipStreamQuery(st);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) return set_err(ctx, TWG_EDEVICE, "batch stream failed");
        if (*word == seen && ++idle > 2) return set_err(ctx, TWG_EDEVICE, "batch control made no progress");
        target = queued + kBatchSlotMargin;
    }
    std::vector<hpf_stats> hs(n);
    if (hipMemcpyAsync(hs.data(), a.stats, n * sizeof(hpf_stats), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return set_err(ctx, TWG_EDEVICE, "batch stats read-back failed");
    bool all = true, bad = false;
    for (int k = 0; k < n; ++k) {
        all = all && hs[k].status == TWG_OK;
        bad = bad || hs[k].status == TWG_EINVAL;
        if (stats_host) stats_host[k] = hs[k];
    }
    if (bad) return set_err(ctx, TWG_EINVAL, "non-finite value in a grid of the batch");
    if (!all) set_err(ctx, TWG_NOT_CONVERGED, "some grids stopped before reaching the tolerance");
    return all ? TWG_OK : TWG_NOT_CONVERGED;
}

}  // namespace

extern "C" {

int32_t twg_version(void) { return 200; }

int32_t twg_ctx_create(twg_ctx **out, int32_t device)
{
    if (!out) return TWG_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return TWG_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return TWG_EDEVICE;
    twg_ctx *ctx = new twg_ctx();
    ctx->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        ctx->num_cu = prop.multiProcessorCount;
        ctx->lds_per_block = prop.sharedMemPerBlock;
    }
    if (hipMalloc(&ctx->words, kWords * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&ctx->rpart, 2 * kResidBlocks * sizeof(unsigned long long)) != hipSuccess ||
        hipHostMalloc(&ctx->host_words, kWords * sizeof(unsigned long long), hipHostMallocDefault) !=
            hipSuccess) {
        twg_ctx_destroy(ctx);
        return TWG_ENOMEM;
    }
    std::memset(ctx->host_words, 0, kWords * sizeof(unsigned long long));
    if (hipHostGetDevicePointer(reinterpret_cast<void **>(&ctx->host_words_dev), ctx->host_words, 0) !=
        hipSuccess) {
        twg_ctx_destroy(ctx);
        return TWG_EDEVICE;
    }
    // the static scratch of hpf_relax_async_noalloc on this device
    if (const int rc = noalloc_scratch(device, &ctx->noalloc)) {
        twg_ctx_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return TWG_OK;
}

int32_t twg_ctx_destroy(twg_ctx *ctx)
{
    if (!ctx) return TWG_EINVAL;
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    for (auto &g : ctx->graphs) hipGraphExecDestroy(g.exec);
    ctx->graphs.clear();
    if (ctx->cap) hipStreamDestroy(ctx->cap);
    void *bufs[] = {ctx->alt,   ctx->pol,   ctx->alt64,  ctx->fmask, ctx->pairs,   ctx->idxbuf,
                    ctx->batch, ctx->words, ctx->jumpbuf, ctx->rpart, ctx->tunebuf, ctx->ctl};
    for (void *b : bufs)
        if (b) hipFree(b);
    if (ctx->host_words) hipHostFree(ctx->host_words);
    delete ctx;
    return TWG_OK;
}

const char *twg_last_error(const twg_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int32_t twg_ctx_set_graphs(twg_ctx *ctx, int32_t enable)
{
    if (!ctx || (enable != 0 && enable != 1)) return TWG_EINVAL;
    ctx->use_graphs = enable;
    return TWG_OK;
}

int32_t twg_rasterize(twg_ctx *ctx, twg_grid g, int32_t n_obs, const double *pos, const double *vel,
                      const double *radius, const uint8_t *static_occ, const twg_raster_params *p,
                      uint8_t *cls, uint16_t *ring, void *stream)
{
    if (!ctx) return TWG_EINVAL;
    ctx->err.clear();
    int rc = check_grid(ctx, g);
    if (rc) return rc;
    if (!p || !cls) return set_err(ctx, TWG_EINVAL, "params and cls are required");
    if (n_obs < 0) return set_err(ctx, TWG_EINVAL, "n_obs < 0");
    if (n_obs > 0 && (!pos || !vel || !radius))
        return set_err(ctx, TWG_EINVAL, "obstacle arrays are required when n_obs > 0");
    if (p->robot_x < 0 || p->robot_y < 0 || p->robot_x >= g.nx || p->robot_y >= g.ny)
        return set_err(ctx, TWG_EINVAL, "robot outside the grid");
    if (p->goal_x < 0 || p->goal_y < 0 || p->goal_x >= g.nx || p->goal_y >= g.ny)
        return set_err(ctx, TWG_EINVAL, "goal outside the grid");
    if (p->ring_width < 1) return set_err(ctx, TWG_EINVAL, "ring_width < 1");
    if (!(p->robot_speed > 0.0) || !std::isfinite(p->robot_speed))
        return set_err(ctx, TWG_EINVAL, "robot_speed must be positive and finite");
    if ((p->ring_mode != 0 && p->ring_mode != 1) || (p->per_object != 0 && p->per_object != 1))
        return set_err(ctx, TWG_EINVAL, "ring_mode and per_object must be 0 or 1");
    if (p->ring_mode == 1 && (!std::isfinite(p->heading_x) || !std::isfinite(p->heading_y) ||
                              (p->heading_x == 0.0 && p->heading_y == 0.0)))
        return set_err(ctx, TWG_EINVAL, "ring_mode 1 needs a finite, nonzero heading");
    if (!(p->kappa >= 0.0) || !std::isfinite(p->kappa))
        return set_err(ctx, TWG_EINVAL, "kappa must be finite and >= 0");
    hipSetDevice(ctx->device);
    return launch_rasterize(ctx, g, n_obs, pos, vel, radius, static_occ, *p, cls, ring,
                            as_stream(stream));
}

namespace {

// argument checks shared by hpf_relax and hpf_relax_async
int check_relax_args(twg_ctx *ctx, const twg_grid &g, const uint8_t *cls, const float *psi, const double *psi64,
                     const hpf_params *params)
{
    int rc = check_grid(ctx, g);
    if (rc) return rc;
    if (!cls || !psi || !params) return set_err(ctx, TWG_EINVAL, "cls, psi and params are required");
    const hpf_params &p = *params;
    if (!(p.tol > 0.0)) return set_err(ctx, TWG_EINVAL, "tol must be > 0");
    if (!(p.omega >= 0.0f && p.omega < 2.0f)) return set_err(ctx, TWG_EINVAL, "omega must be in [0, 2)");
    if (p.init < HPF_INIT_KEEP || p.init > HPF_INIT_LINEAR) return set_err(ctx, TWG_EINVAL, "bad init mode");
    if (p.init == HPF_INIT_LINEAR && (p.goal_x < 0 || p.goal_y < 0 || p.goal_x >= g.nx || p.goal_y >= g.ny))
        return set_err(ctx, TWG_EINVAL, "HPF_INIT_LINEAR needs a goal inside the grid");
    if (p.polish < 0 || p.polish > 2) return set_err(ctx, TWG_EINVAL, "polish must be 0, 1 or 2");
    if (p.polish && !psi64) return set_err(ctx, TWG_EINVAL, "polish needs psi64");
    if (p.sweeps_per_pass && !stream_depth_supported(p.sweeps_per_pass))
        return set_err(ctx, TWG_EINVAL, "sweeps_per_pass must be 1 to 8");
    if (p.rows_per_tile && (p.rows_per_tile < 2 || (p.rows_per_tile & 1)))
        return set_err(ctx, TWG_EINVAL, "rows_per_tile must be even and >= 2");
    if (p.check_passes < 0) return set_err(ctx, TWG_EINVAL, "check_passes must be >= 0");
    return TWG_OK;
}

}  // namespace

int32_t hpf_relax(twg_ctx *ctx, twg_grid g, const uint8_t *cls, float *psi, double *psi64,
                  const hpf_params *params, hpf_stats *stats, void *stream)
{
    if (!ctx) return TWG_EINVAL;
    ctx->err.clear();
    int rc = check_relax_args(ctx, g, cls, psi, psi64, params);
    if (rc) return rc;
    hpf_params p = *params;
    if (p.max_sweeps <= 0) p.max_sweeps = 10000000;
    hipSetDevice(ctx->device);
    hipStream_t st = as_stream(stream);
    const RelaxPlan pl = plan_for(ctx, g, p);
    hpf_stats s;
    std::memset(&s, 0, sizeof s);
    if (p.polish == 2) {
        // FP32 solve on the device, then FP64 SOR sweeps driven from the host
        hpf_params p0 = p;
        p0.polish = 0;
        rc = relax_device_ctx(ctx, g, cls, psi, nullptr, p0, pl, 0, nullptr, &s, st);
        if (rc) return rc;
        if (s.status == TWG_EINVAL) return set_err(ctx, TWG_EINVAL, "non-finite value in the field");
        const double need = p.tol_cert > 0.0 ? std::min(p.tol, p.tol_cert / s.wbound) : p.tol;
        rc = launch_widen(psi, psi64, g.nx, g.ny, g.pitch, st);
        if (rc) return set_err(ctx, rc, "widen launch failed");
        Runner run{ctx, g, cls, st};
        bool done = false;
        double r64 = 0.0;
        rc = run.solve64(psi64, (double)pl.omega, need, p.max_sweeps, &s.polish_sweeps, &r64, &done);
        if (rc) return rc;
        rc = launch_narrow(psi64, psi, g.nx, g.ny, g.pitch, st);
        if (rc) return set_err(ctx, rc, "narrow launch failed");
        if (hipStreamSynchronize(st) != hipSuccess) return set_err(ctx, TWG_EDEVICE, "stream failed");
        s.residual = r64;
        s.cert_bound = r64 * s.wbound;
        s.status = done ? TWG_OK : TWG_NOT_CONVERGED;
        s.checks += run.checks;
    } else {
        rc = relax_device_ctx(ctx, g, cls, psi, psi64, p, pl, 0, nullptr, &s, st);
        if (rc) return rc;
    }
    if (stats) *stats = s;
    if (s.status == TWG_EINVAL) return set_err(ctx, TWG_EINVAL, "non-finite value in the field");
    if (s.status == TWG_NOT_CONVERGED)
        set_err(ctx, TWG_NOT_CONVERGED, "relaxation stopped before reaching the tolerance");
    return s.status;
}

int32_t hpf_relax_async(twg_ctx *ctx, twg_grid g, const uint8_t *cls, float *psi, double *psi64,
                        const hpf_params *params, int32_t slots, hpf_stats *stats, void *stream)
{
    if (!ctx) return TWG_EINVAL;
    ctx->err.clear();
    int rc = check_relax_args(ctx, g, cls, psi, psi64, params);
    if (rc) return rc;
    if (params->polish == 2) return set_err(ctx, TWG_EUNSUPPORTED, "the asynchronous relaxation polishes by defect correction only");
    if (slots < 1) return set_err(ctx, TWG_EINVAL, "slots must be >= 1");
    if (!stats) return set_err(ctx, TWG_EINVAL, "stats (device) is required");
    hpf_params p = *params;
    if (p.max_sweeps <= 0) p.max_sweeps = 10000000;
    hipSetDevice(ctx->device);
    const RelaxPlan pl = plan_for(ctx, g, p);
    return relax_device_ctx(ctx, g, cls, psi, psi64, p, pl, slots, stats, nullptr, as_stream(stream));
}

int32_t hpf_relax_async_noalloc(twg_ctx *ctx, twg_grid g, const uint8_t *cls, float *psi, double *psi64,
                                const hpf_params *params, int32_t slots, hpf_stats *stats, void *stream)
{
    if (!ctx) return TWG_EINVAL;
    ctx->err.clear();
    int rc = check_relax_args(ctx, g, cls, psi, psi64, params);
    if (rc) return rc;
    if (params->polish == 2) return set_err(ctx, TWG_EUNSUPPORTED, "the asynchronous relaxation polishes by defect correction only");
    if (slots < 1) return set_err(ctx, TWG_EINVAL, "slots must be >= 1");
    if (!stats) return set_err(ctx, TWG_EINVAL, "stats (device) is required");
    if ((size_t)g.pitch * (size_t)g.ny > kNoAllocMaxCells)
        return set_err(ctx, TWG_EUNSUPPORTED, "hpf_relax_async_noalloc takes grids of at most " +
                                                  std::to_string(kNoAllocMaxCells) + " cells (pitch * ny)");
    if (relax_ctl_bytes() + 256 > kNoAllocCtlBytes) return set_err(ctx, TWG_EDEVICE, "control block too large");
    if (!ctx->noalloc) return set_err(ctx, TWG_EDEVICE, "no static scratch on this device");
    hpf_params p = *params;
    if (p.max_sweeps <= 0) p.max_sweeps = 10000000;
    hipSetDevice(ctx->device);
    const RelaxPlan pl = plan_for(ctx, g, p);
    char *base = static_cast<char *>(ctx->noalloc);
    RelaxBufs b;
    b.ctl = base;
    b.alt = reinterpret_cast<float *>(base + kNoAllocAlt);
    b.pol = p.polish ? reinterpret_cast<float *>(base + kNoAllocPol) : nullptr;
    b.fmask = reinterpret_cast<uint8_t *>(base + kNoAllocMask);
    return relax_device(ctx, g, cls, psi, psi64, p, pl, b, slots, stats, nullptr, as_stream(stream));
}

int32_t hpf_relax_batched(twg_ctx *ctx, int32_t n, const twg_grid_desc *grids, const uint8_t *cls,
                          float *psi, const hpf_params *params, hpf_stats *stats, void *stream)
{
    if (!ctx) return TWG_EINVAL;
    ctx->err.clear();
    return relax_batch_device(ctx, n, grids, cls, psi, params, 0, nullptr, stats, as_stream(stream));
}

int32_t hpf_relax_batched_async(twg_ctx *ctx, int32_t n, const twg_grid_desc *grids, const uint8_t *cls,
                                float *psi, const hpf_params *params, int32_t slots, hpf_stats *stats,
                                void *stream)
{
    if (!ctx) return TWG_EINVAL;
    ctx->err.clear();
    if (slots < 1) return set_err(ctx, TWG_EINVAL, "slots must be >= 1");
    if (!stats) return set_err(ctx, TWG_EINVAL, "stats (device, n entries) is required");
    return relax_batch_device(ctx, n, grids, cls, psi, params, slots, stats, nullptr, as_stream(stream));
}

int32_t hpf_autotune_batched(twg_ctx *ctx, int32_t n, const twg_grid_desc *grids, const uint8_t *cls,
                             double *out, void *stream)
{
    if (!ctx) return TWG_EINVAL;
    ctx->err.clear();
    if (n < 1 || !grids || !cls) return set_err(ctx, TWG_EINVAL, "n >= 1, grids and cls are required");
    long long total = 0;
    for (int k = 0; k < n; ++k) {
        if (grids[k].offset < 0 || grids[k].pitch < 1 || grids[k].ny < 1)
            return set_err(ctx, TWG_EINVAL, "bad grid " + std::to_string(k));
        total = std::max(total, (long long)grids[k].offset + (long long)grids[k].pitch * grids[k].ny);
    }
    hipSetDevice(ctx->device);
    hipStream_t st = as_stream(stream);
    int rc = ensure(ctx, &ctx->tunebuf, &ctx->tunebuf_bytes, (size_t)total * sizeof(float));
    if (rc) return rc;
    float *fld = static_cast<float *>(ctx->tunebuf);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return set_err(ctx, TWG_EDEVICE, "event creation failed");
    // candidates: deeper passes and taller tiles pay off in a batch, which
    // has far more tiles than the device has SIMDs
    const int cand[][2] = {{4, 32}, {6, 64}, {8, 64}, {6, 128}, {8, 128}};
    int bS = 0, bRH = 0;
    float best = 0.0f;
    for (const auto &c : cand) {
        hpf_params p = {};
        p.tol = 1e-6;
        p.init = HPF_INIT_HALF;
        p.sweeps_per_pass = c[0];
        p.rows_per_tile = c[1];
        // once to set up (tables, scratch), once timed
        rc = relax_batch_device(ctx, n, grids, cls, fld, &p, 0, nullptr, nullptr, st);
        if (rc < 0) break;
        hipEventRecord(e0, st);
        rc = relax_batch_device(ctx, n, grids, cls, fld, &p, 0, nullptr, nullptr, st);
        hipEventRecord(e1, st);
        if (rc < 0 || hipEventSynchronize(e1) != hipSuccess) {
            rc = rc < 0 ? rc : TWG_EDEVICE;
            break;
        }
        float ms = 0.0f;
        hipEventElapsedTime(&ms, e0, e1);
        if (bS == 0 || ms < best) {
            bS = c[0];
            bRH = c[1];
            best = ms;
        }
        rc = TWG_OK;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    ctx->batch_S = bS;
    ctx->batch_RH = bRH;
    if (out) {
        out[0] = bS;
        out[1] = bRH;
        out[2] = best;
    }
    return TWG_OK;
}

int32_t hpf_autotune(twg_ctx *ctx, twg_grid g, const uint8_t *cls, double *out, void *stream)
{
    if (!ctx) return TWG_EINVAL;
    ctx->err.clear();
    int rc = check_grid(ctx, g);
    if (rc) return rc;
    if (!cls) return set_err(ctx, TWG_EINVAL, "cls is required");
    hipSetDevice(ctx->device);
    hipStream_t st = as_stream(stream);
    const size_t n32 = (size_t)g.pitch * g.ny;
    rc = ensure(ctx, &ctx->alt, &ctx->alt_bytes, n32 * sizeof(float));
    if (!rc) rc = ensure(ctx, &ctx->pol, &ctx->pol_bytes, 2 * n32 * sizeof(float));
    if (rc) return rc;
    float *a = reinterpret_cast<float *>(ctx->pol);
    float *b = reinterpret_cast<float *>(ctx->alt);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return set_err(ctx, TWG_EDEVICE, "event creation failed");
    Runner run{ctx, g, cls, st};
    const double cells = (double)g.nx * g.ny;
    // 1. tiling: the least time per sweep of a relaxation pass plus a pass
    //    with a source term (the correction solves' form), which differ in
    //    loads and per-row work; cups reports the relaxation pass's rate
    const int Ss[] = {1, 2, 3, 4, 5, 6, 7, 8};
    twg_tuning best;
    double best_score = 0.0;
    const float om0 = (float)omega_open(g.nx, g.ny);
    float *fsrc = a + n32;
    rc = launch_fill_f32(fsrc, 0.0f, g.nx, g.ny, g.pitch, st);
    for (int S : Ss) {
        if (rc) break;
        for (int RH : tile_heights(ctx, g.nx, g.ny, S, 4)) {
            if (RH > 2 * g.ny && RH > 8) continue;
            // passes for about 2 ms at 1e12 cell-updates/s
            int passes = (int)std::min(400.0, std::max(4.0, 2e9 / (cells * S)));
            passes += passes & 1;
            float ms[2] = {0.0f, 0.0f};
            for (int role = 0; role < 2 && !rc; ++role) {
                const float *f = role ? fsrc : nullptr;
                rc = launch_fill_f32(a, 0.5f, g.nx, g.ny, g.pitch, st);
                if (!rc) rc = launch_field_init(cls, a, g.nx, g.ny, g.pitch, HPF_INIT_KEEP, 0, 0, st);
                if (rc) break;
                float *x = a, *y = b;
                // warm-up: also captures the pass graph the timed run replays
                rc = run.sweep32(&x, &y, f, om0, S, RH, (int64_t)kGraphPasses * S);
                if (rc) break;
                hipEventRecord(e0, st);
                rc = run.sweep32(&x, &y, f, om0, S, RH, (int64_t)passes * S);
                hipEventRecord(e1, st);
                if (rc || hipEventSynchronize(e1) != hipSuccess) { rc = rc ? rc : TWG_EDEVICE; break; }
                hipEventElapsedTime(&ms[role], e0, e1);
            }
            if (rc) break;
            const double score = (double)(ms[0] + ms[1]) / ((double)S * passes);
            if (!best.S || score < best_score) {
                best.S = S;
                best.RH = RH;
                best.cups = cells * S * passes / (ms[0] * 1e-3);
                best_score = score;
            }
        }
    }
    // 2. FP64 tiling (the polish sweeps), on a widened copy of the field
    if (!rc) {
        rc = ensure(ctx, &ctx->alt64, &ctx->alt64_bytes, n32 * sizeof(double));
        if (!rc) rc = ensure(ctx, &ctx->pol, &ctx->pol_bytes, n32 * sizeof(double));
        double *a64 = reinterpret_cast<double *>(ctx->pol), *b64 = reinterpret_cast<double *>(ctx->alt64);
        if (!rc) rc = launch_fill_f32(b, 0.5f, g.nx, g.ny, g.pitch, st);
        if (!rc) rc = launch_field_init(cls, b, g.nx, g.ny, g.pitch, HPF_INIT_KEEP, 0, 0, st);
        if (!rc) rc = launch_widen(b, a64, g.nx, g.ny, g.pitch, st);
        const uint8_t *m64 = nullptr;
        if (!rc) rc = run.fmask(&m64);
        const int Ss64[] = {2, 3, 4, 5, 6, 7, 8};
        for (int S : Ss64) {
            if (rc) break;
            for (int RH : tile_heights(ctx, g.nx, g.ny, S, 3)) {
                if (RH > 2 * g.ny && RH > 8) continue;
                const Geometry geo = stream_geometry(g.nx, g.ny, S, RH);
                int passes = (int)std::min(200.0, std::max(4.0, 1e9 / (cells * S)));
                passes += passes & 1;
                double *x = a64, *y = b64;
                for (int k = 0; k < 2 && !rc; ++k) {  // warm-up
                    rc = launch_stream_f64(x, y, m64, (double)om0, g.nx, g.ny, g.pitch, geo, st);
                    std::swap(x, y);
                }
                hipEventRecord(e0, st);
                for (int k = 0; k < passes && !rc; ++k) {
                    rc = launch_stream_f64(x, y, m64, (double)om0, g.nx, g.ny, g.pitch, geo, st);
                    std::swap(x, y);
                }
                hipEventRecord(e1, st);
                if (rc || hipEventSynchronize(e1) != hipSuccess) { rc = rc ? rc : TWG_EDEVICE; break; }
                float ms = 0.0f;
                hipEventElapsedTime(&ms, e0, e1);
                const double cups = cells * S * passes / (ms * 1e-3);
                if (cups > best.cups64) { best.S64 = S; best.RH64 = RH; best.cups64 = cups; }
            }
        }
    }
    // 3. SOR factors, from the family 2 / (1 + c sin(pi / (n + 1))).  The
    // relaxation's: fewest sweeps from the paper's initial field (0.5) to
    // residual 1e-6.  The defect-correction solves': fewest correction sweeps
    // in the whole polish of that converged field to a certified 1e-7.
    // Below the optimum the sweep count climbs steeply (above it, gently),
    // and the optimum moves with the obstacles, so each keeps the next larger
    // factor of the family (one step towards 2) unless that costs over 25 %
    // more sweeps.  (The residual after a fixed sweep count does not rank
    // factors once it reaches the FP32 rounding floor.)
    if (!rc) {
        const int n = std::max(g.nx, g.ny);
        const double cs[] = {1.0, 1.4, 2.0, 2.4, 2.8, 3.0, 3.3, 3.6, 4.0, 4.5, 5.0, 6.0};
        constexpr int NC = sizeof(cs) / sizeof(cs[0]);
        const int64_t cap = std::max<int64_t>(256, (int64_t)(4.0 * n));
        auto pick = [&](const int64_t *sw) {
            int best_i = -1;
            for (int i = 0; i < NC; ++i)
                if (sw[i] > 0 && (best_i < 0 || sw[i] < sw[best_i])) best_i = i;
            if (best_i > 0 && sw[best_i - 1] > 0 && sw[best_i - 1] <= sw[best_i] * 1.25) --best_i;
            return best_i;
        };
        // one device-driven solve from the half-initialised field: the FP32
        // stage (and with polish the defect correction to a certified 1e-7)
        // under a trial plan; returns its stats
        rc = ensure(ctx, &ctx->tunebuf, &ctx->tunebuf_bytes, n32 * sizeof(float));
        if (!rc) rc = ensure(ctx, &ctx->alt64, &ctx->alt64_bytes, n32 * sizeof(double));
        float *fld = static_cast<float *>(ctx->tunebuf);
        double *f64 = reinterpret_cast<double *>(ctx->alt64);
        auto trial = [&](float om, float om_dc, StartPhase lp, bool polish, hpf_stats *s) {
            hpf_params tp;
            std::memset(&tp, 0, sizeof tp);
            tp.tol = 1e-6;
            tp.tol_cert = polish ? 1e-7 : 0.0;
            tp.max_sweeps = polish ? 3 * cap : cap;
            tp.init = HPF_INIT_HALF;
            tp.polish = polish ? 1 : 0;
            RelaxPlan pl;
            pl.S = best.S;
            pl.RH = best.RH;
            pl.omega = om;
            pl.omega_dc = om_dc;
            pl.lead = lp;
            return relax_device_ctx(ctx, g, cls, fld, f64, tp, pl, 0, nullptr, s, st);
        };
        int64_t sw_plain[NC] = {0};
        for (int i = 0; i < NC && !rc; ++i) {
            hpf_stats s;
            rc = trial(omega_family(n, cs[i]), 1.0f, {}, false, &s);
            if (!rc && s.status == TWG_OK) sw_plain[i] = s.sweeps;
        }
        const int ip = rc ? -1 : pick(sw_plain);
        if (ip >= 0) best.omega = omega_family(n, cs[ip]);
        // the whole defect-correction polish of that converged field to a
        // certified 1e-7, once per factor
        if (!rc && ip >= 0) {
            int64_t sw_dc[NC] = {0};
            for (int i = 0; i < NC && !rc; ++i) {
                hpf_stats s;
                rc = trial(best.omega, omega_family(n, cs[i]), {}, true, &s);
                if (!rc && s.status == TWG_OK && s.residual32 <= 1e-6) sw_dc[i] = s.polish_sweeps;
            }
            const int id = rc ? -1 : pick(sw_dc);
            if (id >= 0) best.omega_dc = omega_family(n, cs[id]);
            // start phase of the correction solves: candidates c' in
            // {12, 16, 24} for about n / 40 or n / 20 sweeps, kept when the
            // correction sweeps of a whole polish drop by over 5 %.  (The
            // relaxation itself gets none: a start phase there reaches the
            // residual sooner but leaves more smooth error, which costs the
            // polish more than it saves.)
            const double c_lead[] = {12.0, 16.0, 24.0};
            const int64_t k_lead[] = {std::max<int64_t>(n / 40, 2 * best.S), std::max<int64_t>(n / 20, 4 * best.S)};
            if (!rc && id >= 0) {
                const int64_t base = sw_dc[id];
                int64_t best_sw = base > 0 ? (int64_t)(0.95 * (double)base) : 0;
                for (double c1 : c_lead)
                    for (int64_t k : k_lead) {
                        if (rc) break;
                        const StartPhase lp{omega_family(n, c1), k};
                        hpf_stats s;
                        rc = trial(best.omega, best.omega_dc, lp, true, &s);
                        const int64_t sw = (!rc && s.status == TWG_OK && s.residual32 <= 1e-6) ? s.polish_sweeps : 0;
                        if (sw > 0 && best_sw > 0 && sw < best_sw) {
                            best_sw = sw;
                            best.lead_dc = lp;
                        }
                    }
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return set_err(ctx, rc, "autotune failed");
    ctx->tuned[{g.nx, g.ny}] = best;
    if (out) {
        out[0] = best.S;
        out[1] = best.RH;
        out[2] = best.omega;
        out[3] = best.cups;
        out[4] = best.S64;
        out[5] = best.RH64;
        out[6] = best.cups64;
        out[7] = best.omega_dc;
        out[8] = best.lead_dc.omega;
        out[9] = (double)best.lead_dc.sweeps;
    }
    return TWG_OK;
}

int32_t hpf_sweeps(twg_ctx *ctx, twg_grid g, const uint8_t *cls, float *psi, const float *f,
                   float omega, int32_t sweeps, int32_t tiled, int32_t sweeps_per_pass, void *stream)
{
    if (!ctx) return TWG_EINVAL;
    ctx->err.clear();
    int rc = check_grid(ctx, g);
    if (rc) return rc;
    if (!cls || !psi) return set_err(ctx, TWG_EINVAL, "cls and psi are required");
    if (sweeps < 0) return set_err(ctx, TWG_EINVAL, "sweeps < 0");
    if (!(omega > 0.0f && omega < 2.0f)) return set_err(ctx, TWG_EINVAL, "omega must be in (0, 2)");
    hipSetDevice(ctx->device);
    hipStream_t st = as_stream(stream);
    if (!tiled) {
        for (int k = 0; k < sweeps; ++k)
            for (int color = 0; color < 2; ++color) {
                rc = launch_sweep_color_f32(cls, psi, f, g.nx, g.ny, g.pitch, omega, color, st);
                if (rc) return set_err(ctx, rc, "sweep launch failed");
            }
        return TWG_OK;
    }
    int S = sweeps_per_pass, RH, dS;
    float om_unused;
    tiling_for(ctx, g.nx, g.ny, &dS, &RH, &om_unused);
    if (!S) S = dS;
    if (!stream_depth_supported(S))
        return set_err(ctx, TWG_EINVAL, "sweeps_per_pass must be 1 to 8");
    rc = ensure(ctx, &ctx->alt, &ctx->alt_bytes, (size_t)g.pitch * g.ny * sizeof(float));
    if (rc) return rc;
    Runner run{ctx, g, cls, st};
    float *a = psi, *b = reinterpret_cast<float *>(ctx->alt);
    rc = run.sweep32(&a, &b, f, omega, S, RH, sweeps);
    if (rc) return rc;
    if (a != psi) {
        rc = launch_copy_f32(a, psi, g.nx, g.ny, g.pitch, st);
        if (rc) return set_err(ctx, rc, "copy launch failed");
    }
    return TWG_OK;
}

int32_t hpf_sweeps64(twg_ctx *ctx, twg_grid g, const uint8_t *cls, double *psi64, double omega,
                     int32_t sweeps, int32_t tiled, int32_t sweeps_per_pass, void *stream)
{
    if (!ctx) return TWG_EINVAL;
    ctx->err.clear();
    int rc = check_grid(ctx, g);
    if (rc) return rc;
    if (!cls || !psi64) return set_err(ctx, TWG_EINVAL, "cls and psi64 are required");
    if (sweeps < 0) return set_err(ctx, TWG_EINVAL, "sweeps < 0");
    if (!(omega > 0.0 && omega < 2.0)) return set_err(ctx, TWG_EINVAL, "omega must be in (0, 2)");
    hipSetDevice(ctx->device);
    hipStream_t st = as_stream(stream);
    if (!tiled) {
        for (int k = 0; k < sweeps; ++k)
            for (int color = 0; color < 2; ++color) {
                rc = launch_sweep_color_f64(cls, psi64, nullptr, g.nx, g.ny, g.pitch, omega, color, st);
                if (rc) return set_err(ctx, rc, "sweep launch failed");
            }
        return TWG_OK;
    }
    int S, RH;
    tiling64_for(ctx, g.nx, g.ny, &S, &RH);
    if (sweeps_per_pass) S = sweeps_per_pass;
    if (!stream_depth_supported(S))
        return set_err(ctx, TWG_EINVAL, "sweeps_per_pass must be 1 to 8");
    rc = ensure(ctx, &ctx->alt64, &ctx->alt64_bytes, (size_t)g.pitch * g.ny * sizeof(double));
    if (rc) return rc;
    double *a = psi64, *b = reinterpret_cast<double *>(ctx->alt64);
    Runner run{ctx, g, cls, st};
    const uint8_t *m = nullptr;
    if ((rc = run.fmask(&m))) return rc;
    const Geometry geo = stream_geometry(g.nx, g.ny, S, RH), geo1 = stream_geometry(g.nx, g.ny, 1, RH);
    for (int64_t done = 0; done < sweeps;) {
        const bool full = sweeps - done >= S;
        rc = launch_stream_f64(a, b, m, omega, g.nx, g.ny, g.pitch, full ? geo : geo1, st);
        if (rc) return set_err(ctx, rc, "relaxation kernel launch failed");
        std::swap(a, b);
        done += full ? S : 1;
    }
    if (a != psi64 &&
        hipMemcpy2DAsync(psi64, (size_t)g.pitch * 8, a, (size_t)g.pitch * 8, (size_t)g.nx * 8, g.ny,
                         hipMemcpyDeviceToDevice, st) != hipSuccess)
        return set_err(ctx, TWG_EDEVICE, "copy failed");
    return TWG_OK;
}

int32_t hpf_residual(twg_ctx *ctx, twg_grid g, const uint8_t *cls, const float *psi,
                     const double *psi64, const float *f, double *out, void *stream)
{
    if (!ctx) return TWG_EINVAL;
    ctx->err.clear();
    int rc = check_grid(ctx, g);
    if (rc) return rc;
    if (!cls || (!psi && !psi64) || !out) return set_err(ctx, TWG_EINVAL, "missing argument");
    hipSetDevice(ctx->device);
    hipStream_t st = as_stream(stream);
    rc = psi64 ? launch_resid_f64(cls, psi64, f, g.nx, g.ny, g.pitch, ctx->rpart, ctx->host_words_dev, ++ctx->word_seq, st)
               : launch_resid_f32(cls, psi, f, g.nx, g.ny, g.pitch, ctx->rpart, ctx->host_words_dev, ++ctx->word_seq, st);
    Runner run{ctx, g, cls, st};
    if (!rc) rc = run.wait_words();
    if (rc) return set_err(ctx, rc, "residual kernel failed");
    *out = bits_to_double(ctx->host_words[0]);
    return TWG_OK;
}

int32_t hpf_index_matrix(twg_ctx *ctx, twg_grid g, const uint8_t *cls, const float *psi,
                         const double *psi64, uint8_t *idx, void *stream)
{
    if (!ctx) return TWG_EINVAL;
    ctx->err.clear();
    int rc = check_grid(ctx, g);
    if (rc) return rc;
    if (!cls || (!psi && !psi64) || !idx) return set_err(ctx, TWG_EINVAL, "missing argument");
    hipSetDevice(ctx->device);
    rc = launch_index(cls, psi, psi64, idx, g.nx, g.ny, g.pitch, as_stream(stream));
    return rc ? set_err(ctx, rc, "index launch failed") : TWG_OK;
}

int32_t hpf_descend(twg_ctx *ctx, twg_grid g, const uint8_t *cls, const float *psi,
                    const double *psi64, const hpf_descend_params *p, int32_t *path_xy,
                    int32_t *info, void *stream)
{
    if (!ctx) return TWG_EINVAL;
    ctx->err.clear();
    int rc = check_grid(ctx, g);
    if (rc) return rc;
    if (!cls || (!psi && !psi64) || !p || !path_xy || !info)
        return set_err(ctx, TWG_EINVAL, "missing argument");
    if (p->cap < 1) return set_err(ctx, TWG_EINVAL, "cap < 1");
    if (p->start_x < 0 || p->start_y < 0 || p->start_x >= g.nx || p->start_y >= g.ny)
        return set_err(ctx, TWG_EINVAL, "start outside the grid");
    hipSetDevice(ctx->device);
    hipStream_t st = as_stream(stream);
    rc = ensure(ctx, &ctx->idxbuf, &ctx->idxbuf_bytes, (size_t)g.pitch * g.ny);
    if (rc) return rc;
    uint8_t *idx = reinterpret_cast<uint8_t *>(ctx->idxbuf);
    rc = launch_index(cls, psi, psi64, idx, g.nx, g.ny, g.pitch, st, true);
    if (!rc) rc = launch_walk(cls, idx, g.nx, g.ny, g.pitch, p->start_x, p->start_y, p->cap, path_xy,
                              info, st);
    return rc ? set_err(ctx, rc, "descent launch failed") : TWG_OK;
}

int32_t hpf_rubber_band(twg_ctx *ctx, twg_grid g, const uint8_t *cls, const float *psi, const double *psi64,
                        int32_t *path_xy, const int32_t *len, int32_t cap, double k, int32_t iters, void *stream)
{
    if (!ctx) return TWG_EINVAL;
    ctx->err.clear();
    int rc = check_grid(ctx, g);
    if (rc) return rc;
    if (!cls || (!psi && !psi64) || !path_xy || !len) return set_err(ctx, TWG_EINVAL, "missing argument");
    if (cap < 1) return set_err(ctx, TWG_EINVAL, "cap < 1");
    if (iters < 0 || !(k >= 0.0) || !std::isfinite(k)) return set_err(ctx, TWG_EINVAL, "need iters >= 0 and finite k >= 0");
    hipSetDevice(ctx->device);
    rc = launch_rubber(cls, psi, psi64, path_xy, len, cap, g.nx, g.ny, g.pitch, k, iters, as_stream(stream));
    return rc ? set_err(ctx, rc, "rubber band launch failed") : TWG_OK;
}

int32_t hpf_merge_previous(twg_ctx *ctx, twg_grid g, const uint8_t *cls, const uint8_t *cls_prev,
                           const float *psi_prev, float *psi, void *stream)
{
    if (!ctx) return TWG_EINVAL;
    ctx->err.clear();
    int rc = check_grid(ctx, g);
    if (rc) return rc;
    if (!cls || !psi_prev || !psi) return set_err(ctx, TWG_EINVAL, "missing argument");
    hipSetDevice(ctx->device);
    rc = launch_merge_prev(cls, cls_prev, psi_prev, psi, g.nx, g.ny, g.pitch, as_stream(stream));
    return rc ? set_err(ctx, rc, "merge launch failed") : TWG_OK;
}

int32_t hpf_init_field(twg_ctx *ctx, twg_grid g, const uint8_t *cls, float *psi, int32_t init, int32_t goal_x,
                       int32_t goal_y, void *stream)
{
    if (!ctx) return TWG_EINVAL;
    ctx->err.clear();
    int rc = check_grid(ctx, g);
    if (rc) return rc;
    if (!cls || !psi) return set_err(ctx, TWG_EINVAL, "missing argument");
    if (init < HPF_INIT_KEEP || init > HPF_INIT_LINEAR) return set_err(ctx, TWG_EINVAL, "bad init mode");
    if (init == HPF_INIT_LINEAR && (goal_x < 0 || goal_y < 0 || goal_x >= g.nx || goal_y >= g.ny))
        return set_err(ctx, TWG_EINVAL, "HPF_INIT_LINEAR needs a goal inside the grid");
    hipSetDevice(ctx->device);
    rc = launch_field_init(cls, psi, g.nx, g.ny, g.pitch, init, goal_x, goal_y, as_stream(stream));
    return rc ? set_err(ctx, rc, "init launch failed") : TWG_OK;
}

int32_t hpf_set_tiling(twg_ctx *ctx, int32_t nx, int32_t ny, int32_t S, int32_t RH, float omega, int32_t S64,
                       int32_t RH64)
{
    if (!ctx) return TWG_EINVAL;
    ctx->err.clear();
    if (nx < 1 || ny < 1) return set_err(ctx, TWG_EINVAL, "bad grid size");
    if (!stream_depth_supported(S) || (S64 && !stream_depth_supported(S64)))
        return set_err(ctx, TWG_EINVAL, "sweeps per pass must be 1 to 8");
    if (RH < 2 || (S64 && RH64 < 2)) return set_err(ctx, TWG_EINVAL, "rows per tile must be >= 2");
    if (!(omega >= 0.0f && omega < 2.0f)) return set_err(ctx, TWG_EINVAL, "omega must be in [0, 2)");
    twg_tuning t;
    t.S = S;
    t.RH = RH;
    t.omega = omega;
    t.S64 = S64;
    t.RH64 = RH64;
    ctx->tuned[{nx, ny}] = t;
    return TWG_OK;
}

int32_t twg_kalman_step(twg_ctx *ctx, int32_t n, double *x, double *P, const double *z, double dt,
                        const double *Q, const double *R, double *pos, double *vel, void *stream)
{
    if (!ctx) return TWG_EINVAL;
    ctx->err.clear();
    if (n < 0) return set_err(ctx, TWG_EINVAL, "n < 0");
    if (n > 0 && (!x || !P)) return set_err(ctx, TWG_EINVAL, "x and P are required");
    if (z && !R) return set_err(ctx, TWG_EINVAL, "a measurement needs R");
    if (!std::isfinite(dt)) return set_err(ctx, TWG_EINVAL, "dt must be finite");
    hipSetDevice(ctx->device);
    const int rc = launch_kalman(n, x, P, z, dt, Q, R, pos, vel, as_stream(stream));
    return rc ? set_err(ctx, rc, "Kalman launch failed") : TWG_OK;
}

int32_t hpf_descent_all(twg_ctx *ctx, twg_grid g, const uint8_t *cls, const float *psi, const double *psi64,
                        int32_t *steps, int32_t steps_pitch, void *stream)
{
    if (!ctx) return TWG_EINVAL;
    ctx->err.clear();
    int rc = check_grid(ctx, g);
    if (rc) return rc;
    if (!cls || (!psi && !psi64) || !steps) return set_err(ctx, TWG_EINVAL, "missing argument");
    if (steps_pitch < g.nx) return set_err(ctx, TWG_EINVAL, "steps_pitch must be >= nx");
    hipSetDevice(ctx->device);
    hipStream_t st = as_stream(stream);
    const size_t cells = (size_t)g.nx * g.ny;
    rc = ensure(ctx, &ctx->idxbuf, &ctx->idxbuf_bytes, (size_t)g.pitch * g.ny);
    if (!rc) rc = ensure(ctx, &ctx->jumpbuf, &ctx->jumpbuf_bytes, 4 * cells * sizeof(int));
    if (rc) return rc;
    uint8_t *idx = reinterpret_cast<uint8_t *>(ctx->idxbuf);
    rc = launch_index(cls, psi, psi64, idx, g.nx, g.ny, g.pitch, st);
    if (!rc)
        rc = launch_descent_all(cls, idx, g.nx, g.ny, g.pitch, reinterpret_cast<int *>(ctx->jumpbuf), steps,
                                steps_pitch, st);
    return rc ? set_err(ctx, rc, "descent launch failed") : TWG_OK;
}

}  // extern "C"
