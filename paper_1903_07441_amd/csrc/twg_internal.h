// Internal declarations shared by the HIP translation units of libtwg.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "twg.h"

// Start phase of an FP32 solve: its first `sweeps` sweeps use the smaller
// factor `omega`, which damps the rough error of the initial field faster
// than the asymptotically best factor does (sweeps = 0: none).
struct StartPhase {
    float omega = 0.0f;
    int64_t sweeps = 0;
};

struct twg_tuning {
    int S = 0;        // sweeps per tile load
    int RH = 0;       // output rows per tile
    float omega = 0;     // 0 = open-rectangle optimum
    float omega_dc = 0;  // factor of the defect-correction solves (0 = default)
    StartPhase lead_dc;  // start phase of each correction solve
    double cups = 0;  // measured cell-updates per second
    int S64 = 0;      // the same for FP64 sweeps (0 = untuned)
    int RH64 = 0;
    double cups64 = 0;
};

struct twg_ctx {
    int device = 0;
    // autotuned tiling per grid size (nx, ny)
    std::map<std::pair<int, int>, twg_tuning> tuned;
    int num_cu = 0;
    size_t lds_per_block = 0;  // the device's LDS per workgroup (bytes)
    size_t lds_attr = 0;       // dynamic LDS the batch's LDS worker is allowed so far
    std::string err;
    // FP32 ping-pong partner of a relaxed field
    void *alt = nullptr;
    size_t alt_bytes = 0;
    // defect-correction buffers: FP32 defect, FP32 correction, its partner
    void *pol = nullptr;
    size_t pol_bytes = 0;
    // the autotuner's defect and correction while it times correction solves
    void *tunebuf = nullptr;
    size_t tunebuf_bytes = 0;
    // FP64 ping-pong partner (FP64 sweeps)
    void *alt64 = nullptr;
    size_t alt64_bytes = 0;
    // free mask of the streamed sweeps, rebuilt by every call that sweeps
    void *fmask = nullptr;
    size_t fmask_bytes = 0;
    // (obstacle, ring) work list of the rasteriser and its counter
    void *pairs = nullptr;
    size_t pairs_bytes = 0;
    // index matrix of hpf_descend
    void *idxbuf = nullptr;
    size_t idxbuf_bytes = 0;
    // pointer-jumping buffers of hpf_descent_all (4 int32 per cell)
    void *jumpbuf = nullptr;
    size_t jumpbuf_bytes = 0;
    // batched relaxation: descriptors, block list, control state and stats
    void *batch = nullptr;
    size_t batch_bytes = 0;
    // bytes of the descriptor and block tables last uploaded to `batch`
    std::vector<char> batch_sig;
    // tiling of batched relaxations picked by hpf_autotune_batched (0: none)
    int batch_S = 0, batch_RH = 0;
    // small device words: counters of the rasteriser
    unsigned long long *words = nullptr;
    // per-block partial maxima of the residual kernels (2 kResidBlocks words)
    unsigned long long *rpart = nullptr;
    // pinned host words: residual maxima (uint64 bit patterns) of the last
    // check in words 0 and 1, and in word 2 the sequence number of the
    // reduction that wrote them
    unsigned long long *host_words = nullptr;
    // the same pinned words as the device addresses them: the residual
    // reductions write their results there directly, so a check needs no
    // copy, only a wait for word 2 to show the last sequence number
    unsigned long long *host_words_dev = nullptr;
    // sequence number of the last residual reduction launched
    unsigned long long word_seq = 0;
    // control block of the device-driven relaxation and its device stats
    void *ctl = nullptr;
    size_t ctl_bytes = 0;
    // this device's copy of the static scratch of hpf_relax_async_noalloc
    // (its device address; not owned)
    void *noalloc = nullptr;
    // instantiated graphs of relaxation passes, keyed by their launch
    // arguments, and the stream they are captured on
    struct Graph {
        std::vector<uintptr_t> key;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
    hipStream_t cap = nullptr;
    int use_graphs = 1;
};

namespace twg {

constexpr int kWords = 64;
// host word the device-driven relaxation publishes its decisions to
constexpr int kMirrorWord = 8;

// one grid of a batch: arrays start at element offset `off` of the batch base
struct BatchGrid {
    int nx, ny, pitch;
    float omega;
    long long off;
    int lds;  // 1: solved whole in one workgroup's LDS (k_batch_lds), not by tiles
    int pad_;
};
int launch_field_init_batch(const uint8_t *cls, float *psi, const BatchGrid *grids,
                            const int2 *blocks, int n_blocks, int mode, hipStream_t st);

int set_err(twg_ctx *ctx, int code, const std::string &msg);
int ensure(twg_ctx *ctx, void **buf, size_t *have, size_t need);
int check_grid(twg_ctx *ctx, const twg_grid &g);

// relax.hip
struct Geometry {
    int S;       // sweeps per tile load
    int RH;      // output rows per tile (even)
    int strips;  // tiles across
    int segs;    // tiles down
    int tiles;
};
Geometry stream_geometry(int nx, int ny, int S, int RH);
// HPF_INIT_* on psi; HPF_INIT_LINEAR uses the goal cell (gx, gy)
int launch_field_init(const uint8_t *cls, float *psi, int nx, int ny, int pitch, int mode, int gx, int gy,
                      hipStream_t st);
int launch_sweep_color_f32(const uint8_t *cls, float *psi, const float *f, int nx, int ny, int pitch,
                           float omega, int color, hipStream_t st);
int launch_sweep_color_f64(const uint8_t *cls, double *psi, const double *f, int nx, int ny,
                           int pitch, double omega, int color, hipStream_t st);
bool stream_depth_supported(int S);
// largest RH whose tiles the streamed kernels can address (RH above it is
// lowered at launch)
int stream_rows_cap(int pitch, int elem_bytes, int S);
// streamed sweeps: fmask is the free mask (0xFF on FREE cells, 0 on the
// others) built by launch_fmask; w = omega on FREE cells, 0 elsewhere
int launch_stream_f32(const float *src, float *dst, const uint8_t *fmask, float omega, const float *f, int nx,
                      int ny, int pitch, const Geometry &geo, hipStream_t st);
int launch_stream_f64(const double *src, double *dst, const uint8_t *fmask, double omega, int nx, int ny,
                      int pitch, const Geometry &geo, hipStream_t st);
int launch_fmask(const uint8_t *cls, uint8_t *fmask, int nx, int ny, int pitch, hipStream_t st);
// the batch's free mask, over the batch's column blocks
int launch_fmask_batch(const uint8_t *cls, uint8_t *fmask, const BatchGrid *grids, const int2 *blocks,
                       int n_blocks, hipStream_t st);
// residual reductions: part = the context's block partials (2 kResidBlocks
// words), out = 3 words receiving max |r| and max |r| / |u|, then seq (after
// a system-scope fence, so a host that sees seq in out[2] reads final
// maxima)
constexpr int kResidBlocks = 4096;
int launch_resid_f32(const uint8_t *cls, const float *u, const float *f, int nx, int ny, int pitch,
                     unsigned long long *part, unsigned long long *out, unsigned long long seq, hipStream_t st);
int launch_resid_f64(const uint8_t *cls, const double *u, const float *f, int nx, int ny, int pitch,
                     unsigned long long *part, unsigned long long *out, unsigned long long seq, hipStream_t st);
int launch_defect64(const uint8_t *cls, const double *u, float *r32, int nx, int ny, int pitch,
                    unsigned long long *part, unsigned long long *out, unsigned long long seq, hipStream_t st);
int launch_update64(const uint8_t *cls, double *u, const float *e, float *psi, int nx, int ny,
                    int pitch, hipStream_t st);
int launch_widen(const float *psi, double *u, int nx, int ny, int pitch, hipStream_t st);
int launch_narrow(const double *u, float *psi, int nx, int ny, int pitch, hipStream_t st);
int launch_fill_f32(float *a, float v, int nx, int ny, int pitch, hipStream_t st);
int launch_copy_f32(const float *src, float *dst, int nx, int ny, int pitch, hipStream_t st);
int launch_merge_prev(const uint8_t *cls, const uint8_t *cls_prev, const float *psi_prev, float *psi, int nx,
                      int ny, int pitch, hipStream_t st);

// solve.hip: the device-driven relaxation.  One RelaxConfig per call, given
// to the begin kernel; SlotArgs are the arguments of every slot launch.
struct RelaxConfig {
    double tol;          // FP32-stage tolerance on the FP64 residual
    double need;         // residual the polish must reach (0 without polish)
    double wbound;       // maximum-principle bound on ||(I - J)^-1 1||inf
    int64_t max_sweeps;  // sweeps per solve (the FP32 solve, and each correction solve)
    float omega;         // SOR factor of the FP32 solve
    float omega_dc;      // SOR factor of the correction solves
    float omega_lead;    // factor of the correction solves' start phase
    int32_t lead_passes; // passes of that start phase (0: none)
    int32_t S;           // sweeps per pass
    int32_t polish;      // 1: FP64 defect correction after the FP32 solve
    int32_t check_passes;  // > 0: check every this many passes
    int32_t max_rounds;  // defect-correction rounds at most
    int32_t kept;        // 1: polish of the caller's kept FP32 field, whose first
                         // defect also checks the FP32 stage (0 sweeps when it
                         // meets tol)
};
struct SlotArgs {
    const uint8_t *mask;  // free mask (0xFF on FREE cells), the grid's layout
    float *psi;           // caller's FP32 field
    float *alt;           // its ping-pong partner (and the correction's)
    float *e;             // correction
    float *r32;           // FP32 defect f
    float *cdc, *clead;   // omega_dc f and omega_lead f (0 on fixed cells)
    double *psi64;        // caller's FP64 field (polish) or null
    void *ctl;            // device control block (relax_ctl_bytes())
    hpf_stats *stats;     // device stats, written when the solve ends
    unsigned long long *mirror;  // host-mapped decision word, or null
    int nx, ny, pitch;
    int strips, RH, tiles;  // SOR tiling (S sweeps per pass)
    int pair;             // paired-column access
    int final_slot;       // 1: finish what is left (the solve is then NOT_CONVERGED)
    int slot;             // this launch's number in the call's sequence (0, 1, ...)
    int polish;           // RelaxConfig::polish
    float omega, omega_dc, omega_lead;  // the RelaxConfig factors
    int lead_passes;      // RelaxConfig::lead_passes
};
size_t relax_ctl_bytes();
int launch_relax_begin(void *ctl, const RelaxConfig &cfg, hipStream_t st);
int launch_relax_slot(const SlotArgs &a, int S, hipStream_t st);

// batch.hip: the device-driven relaxation of a batch of grids.  BatchArgs
// are the arguments of the begin kernel and of every slot launch.
constexpr int kBatchMaxGrids = 65536;
struct GridRun;  // per-grid run state (batch.hip)
struct GridCtl;  // per-grid controller state (batch.hip)
struct BatchArgs {
    const BatchGrid *grids;  // n descriptors
    const int2 *blocks;      // static (grid, 64-column block) list of every grid
    int n_blocks, n;
    int S, RH;               // sweeps per pass, output rows per tile
    int slot, final_slot;    // this launch's number; 1: finish what is left
    int quantum;             // checks only at slots that are multiples of this
    int check_passes;        // > 0: a check every this many passes
    double tol;
    int64_t max_sweeps;      // per grid
    float *psi, *alt;        // batch fields and their ping-pong partner
    const uint8_t *mask;     // free masks, laid out as the fields
    void *hdr;               // batch_hdr_bytes()
    GridRun *run;            // n
    GridCtl *ctl;            // n
    int2 *tiles;             // one entry per tile of the batch: (grid, tile of the grid)
    unsigned long long *rmax, *rrel;  // n each: maxima of the checking passes
    hpf_stats *stats;        // n, device, written when the batch ends
    unsigned long long *mirror;       // host-mapped decision word, or null
    const int *lds_list;     // the grids solved in LDS (BatchGrid::lds), n_lds of them
    int n_lds;
};
size_t batch_hdr_bytes();
size_t batch_run_bytes();
size_t batch_ctl_bytes();
int launch_batch_begin(const BatchArgs &a, hipStream_t st);
int launch_batch_slot(const BatchArgs &a, int max_tiles, bool pair, hipStream_t st);
// LDS bytes k_batch_lds needs for a grid of `cells` cells; the solve of the
// LDS grids (one workgroup each), launched after launch_batch_begin
size_t batch_lds_bytes(long long cells);
int launch_batch_lds(const BatchArgs &a, size_t lds_bytes, size_t *lds_attr, hipStream_t st);

// raster.hip
int launch_rasterize(twg_ctx *ctx, const twg_grid &g, int n_obs, const double *pos,
                     const double *vel, const double *rad, const uint8_t *static_occ,
                     const twg_raster_params &p, uint8_t *cls, uint16_t *ring, hipStream_t st);

// kalman.hip
int launch_kalman(int n, double *x, double *P, const double *z, double dt, const double *Q, const double *R,
                  double *pos, double *vel, hipStream_t st);

// descend.hip.  walk: write the walk's codes (5 on GOAL cells, else the
// index code) instead of the index matrix; launch_walk reads those.
int launch_index(const uint8_t *cls, const float *psi, const double *psi64, uint8_t *idx, int nx,
                 int ny, int pitch, hipStream_t st, bool walk = false);
int launch_walk(const uint8_t *cls, const uint8_t *code, int nx, int ny, int pitch, int sx, int sy,
                int cap, int32_t *path, int32_t *info, hipStream_t st);
int launch_descent_all(const uint8_t *cls, const uint8_t *idx, int nx, int ny, int pitch, int *buf,
                       int32_t *steps, int pitch_out, hipStream_t st);
int launch_rubber(const uint8_t *cls, const float *psi, const double *psi64, int32_t *path, const int32_t *len,
                  int cap, int nx, int ny, int pitch, double k, int iters, hipStream_t st);

}  // namespace twg
