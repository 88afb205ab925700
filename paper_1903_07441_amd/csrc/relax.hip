// Relaxation support kernels for gfx950 (Eqs. 1-2 of the paper; boundary
// values of section "Harmonic Potential Fields"): the untiled one-colour
// sweep (the reference the streamed kernel in sor_stream.hip is tested
// against, bit for bit), FP64 residual reductions, field initialisation, the
// FP64 defect-correction kernels and the per-grid set-up of a batch.
//
// Field layout: row-major, x fastest, pitch in elements; psi = 1 - phi.
// Red cells are (x + y) even.
#include "twg_internal.h"
#include "update.h"

namespace twg {

namespace {

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
    if constexpr (RHS)
        psi[i] = upd_src(psi[i], (e + w) + n, s, src_const(om, f[i]));
    else
        psi[i] = upd(psi[i], (e + w) + n, s, om);
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

// Residual |avg4(u) + f - u| over FREE cells; each block writes the bit
// pattern of its max to part[2 b] (non-negative doubles order like their bit
// patterns; a NaN yields a NaN pattern, which is larger than +inf) and of its
// max |r| / |u| over FREE cells with |u| >= 1e-30 to part[2 b + 1];
// k_resid_reduce combines the blocks (no same-address atomics).
template <typename T, bool RHS, bool WRITE_R32>
__global__ __launch_bounds__(256) void k_resid(const uint8_t *__restrict__ cls,
                                               const T *__restrict__ u, const float *__restrict__ f,
                                               float *__restrict__ r32, int nx, int ny, int pitch,
                                               unsigned long long *__restrict__ part)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    double m = 0.0, mr = 0.0;
    // every load of a cell is unconditional (neighbours clamped to the grid,
    // then zeroed outside it; the class only selects the result), so none
    // waits inside a divergent branch, and four rows are in flight per thread
    if (x < nx) {
        const int xe = min(x + 1, nx - 1), xw = max(x - 1, 0);
#pragma unroll 4
        for (int y = blockIdx.y * 4 + (threadIdx.x >> 6); y < ny; y += gridDim.y * 4) {
            const size_t row = (size_t)y * pitch, i = row + x;
            const bool free_cell = cls[i] == TWG_CELL_FREE;
            const double ue = (double)u[row + xe], uw = (double)u[row + xw];
            const double us = (double)u[(size_t)min(y + 1, ny - 1) * pitch + x];
            const double un = (double)u[(size_t)max(y - 1, 0) * pitch + x];
            const double c = (double)u[i];
            const double e = x + 1 < nx ? ue : 0.0;
            const double w = x > 0 ? uw : 0.0;
            const double s = y + 1 < ny ? us : 0.0;
            const double n = y > 0 ? un : 0.0;
            double g = ((e + w) + (s + n)) * 0.25;
            if (RHS) g = g + (double)f[i];
            const double r = free_cell ? g - c : 0.0;
            const float ac = fabsf((float)c);
            // diagnostic ratio: single-precision division is enough
            const float q = fabsf((float)r) / ac;
            mr = nanmax(mr, free_cell && ac >= 1e-30f ? (double)q : 0.0);
            if (WRITE_R32) r32[i] = (float)r;
            m = nanmax(m, fabs(r));
        }
    }
    m = block_max(m);
    __syncthreads();
    mr = block_max(mr);
    if (threadIdx.x == 0) {
        const size_t b = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
        part[2 * b] = (unsigned long long)__double_as_longlong(m);
        part[2 * b + 1] = (unsigned long long)__double_as_longlong(mr);
    }
}

// out[0], out[1] = maxima of the n block partials (bit patterns of
// non-negative doubles, or NaN patterns, which compare larger); then, after
// a system-scope fence, out[2] = seq
__global__ __launch_bounds__(256) void k_resid_reduce(const unsigned long long *__restrict__ part, int n,
                                                      unsigned long long *out, unsigned long long seq)
{
    __shared__ unsigned long long red[2][256];
    unsigned long long a = 0, b = 0;
    for (int k = threadIdx.x; k < n; k += 256) {
        a = max(a, part[2 * k]);
        b = max(b, part[2 * k + 1]);
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] = max(red[0][threadIdx.x], red[0][threadIdx.x + w]);
            red[1][threadIdx.x] = max(red[1][threadIdx.x], red[1][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = red[0][0];
        out[1] = red[1][0];
        __threadfence_system();
        out[2] = seq;
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

// Warm start from a previous field: FREE cells that were FREE in the
// previous step take the previous value; every other cell keeps psi.
__global__ void k_merge_prev(const uint8_t *__restrict__ cls, const uint8_t *__restrict__ cls_prev,
                             const float *__restrict__ psi_prev, float *__restrict__ psi, int nx, int ny,
                             int pitch)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= nx || y >= ny) return;
    const size_t i = (size_t)y * pitch + x;
    // without a previous class map every FREE cell takes the previous value
    if (cls[i] == TWG_CELL_FREE && (!cls_prev || cls_prev[i] == TWG_CELL_FREE)) psi[i] = psi_prev[i];
}

// ---- element-wise helpers --------------------------------------------------
// Field initialisation: OBST and WALL 0, GOAL 1, FIXED unchanged; FREE cells
// by mode: HALF 0.5, ZERO 0, LINEAR the ramp 1 - d / (max(nx, ny) sqrt 2)
// of the Euclidean distance d to the goal cell (gx, gy), evaluated in FP64
// and rounded once; KEEP leaves them.
__global__ void k_field_init(const uint8_t *__restrict__ cls, float *psi, int nx, int ny, int pitch,
                             int mode, int gx, int gy)
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
        if (mode == HPF_INIT_HALF) {
            psi[i] = 0.5f;
        } else if (mode == HPF_INIT_ZERO) {
            psi[i] = 0.0f;
        } else if (mode == HPF_INIT_LINEAR) {
            const double dx = (double)(x - gx), dy = (double)(y - gy);
            const double d = sqrt(dx * dx + dy * dy);
            psi[i] = (float)(1.0 - d / ((double)max(nx, ny) * sqrt(2.0)));
        }
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

dim3 cell_grid(int nx, int ny) { return dim3((nx + 63) / 64, (ny + 3) / 4); }

// free mask of the streamed sweeps: 0xFF on FREE cells, 0 on the others
template <typename T>
__global__ void k_wmap(const uint8_t *__restrict__ cls, T *__restrict__ w, T omega, int nx, int ny, int pitch)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= nx || y >= ny) return;
    const size_t i = (size_t)y * pitch + x;
    w[i] = cls[i] == TWG_CELL_FREE ? omega : T(0);
}

__global__ void k_fmask_batch(const uint8_t *__restrict__ cls, uint8_t *__restrict__ m,
                              const BatchGrid *__restrict__ grids, const int2 *__restrict__ blocks)
{
    const int2 bk = blocks[blockIdx.x];
    const BatchGrid g = grids[bk.x];
    const int x = bk.y * 64 + (threadIdx.x & 63);
    if (x >= g.nx) return;
    for (int y = threadIdx.x >> 6; y < g.ny; y += 4) {
        const size_t i = g.off + (size_t)y * g.pitch + x;
        m[i] = cls[i] == TWG_CELL_FREE ? 0xff : 0;
    }
}

int last_status()
{
    return hipGetLastError() == hipSuccess ? TWG_OK : TWG_EDEVICE;
}

}  // namespace

int launch_field_init_batch(const uint8_t *cls, float *psi, const BatchGrid *grids,
                            const int2 *blocks, int n_blocks, int mode, hipStream_t st)
{
    if (n_blocks > 0)
        hipLaunchKernelGGL(k_field_init_batch, dim3(n_blocks), dim3(256), 0, st, cls, psi, grids,
                           blocks, mode);
    return last_status();
}


int launch_fmask(const uint8_t *cls, uint8_t *fmask, int nx, int ny, int pitch, hipStream_t st)
{
    hipLaunchKernelGGL(k_wmap<uint8_t>, cell_grid(nx, ny), dim3(256), 0, st, cls, fmask, (uint8_t)0xff, nx, ny,
                       pitch);
    return last_status();
}

int launch_fmask_batch(const uint8_t *cls, uint8_t *fmask, const BatchGrid *grids, const int2 *blocks,
                       int n_blocks, hipStream_t st)
{
    if (n_blocks > 0)
        hipLaunchKernelGGL(k_fmask_batch, dim3(n_blocks), dim3(256), 0, st, cls, fmask, grids, blocks);
    return last_status();
}

int launch_field_init(const uint8_t *cls, float *psi, int nx, int ny, int pitch, int mode, int gx, int gy,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_field_init, cell_grid(nx, ny), dim3(256), 0, st, cls, psi, nx, ny, pitch, mode, gx, gy);
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

// at most kResidBlocks blocks: 64 columns per block across, rows split so
// that the partial buffer of the context holds every block
static dim3 resid_grid(int nx, int ny)
{
    const int gx = (nx + 63) / 64;
    int gy = (ny + 3) / 4;
    if (gy > 64) gy = 64;
    const int cap = kResidBlocks / gx;
    if (gy > cap) gy = cap > 0 ? cap : 1;
    return dim3(gx, gy);
}

static int finish_resid(const dim3 &g, const unsigned long long *part, unsigned long long *out,
                        unsigned long long seq, hipStream_t st)
{
    hipLaunchKernelGGL(k_resid_reduce, dim3(1), dim3(256), 0, st, part, (int)(g.x * g.y), out, seq);
    return last_status();
}

int launch_resid_f32(const uint8_t *cls, const float *u, const float *f, int nx, int ny, int pitch,
                     unsigned long long *part, unsigned long long *out, unsigned long long seq, hipStream_t st)
{
    const dim3 g = resid_grid(nx, ny);
    if (f)
        hipLaunchKernelGGL((k_resid<float, true, false>), g, dim3(256), 0, st, cls, u, f, nullptr, nx, ny, pitch,
                           part);
    else
        hipLaunchKernelGGL((k_resid<float, false, false>), g, dim3(256), 0, st, cls, u, f, nullptr, nx, ny,
                           pitch, part);
    return finish_resid(g, part, out, seq, st);
}

int launch_resid_f64(const uint8_t *cls, const double *u, const float *f, int nx, int ny, int pitch,
                     unsigned long long *part, unsigned long long *out, unsigned long long seq, hipStream_t st)
{
    const dim3 g = resid_grid(nx, ny);
    if (f)
        hipLaunchKernelGGL((k_resid<double, true, false>), g, dim3(256), 0, st, cls, u, f, nullptr, nx, ny,
                           pitch, part);
    else
        hipLaunchKernelGGL((k_resid<double, false, false>), g, dim3(256), 0, st, cls, u, f, nullptr, nx, ny,
                           pitch, part);
    return finish_resid(g, part, out, seq, st);
}

int launch_defect64(const uint8_t *cls, const double *u, float *r32, int nx, int ny, int pitch,
                    unsigned long long *part, unsigned long long *out, unsigned long long seq, hipStream_t st)
{
    const dim3 g = resid_grid(nx, ny);
    hipLaunchKernelGGL((k_resid<double, false, true>), g, dim3(256), 0, st, cls, u, nullptr, r32, nx, ny, pitch,
                       part);
    return finish_resid(g, part, out, seq, st);
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

int launch_merge_prev(const uint8_t *cls, const uint8_t *cls_prev, const float *psi_prev, float *psi, int nx,
                      int ny, int pitch, hipStream_t st)
{
    hipLaunchKernelGGL(k_merge_prev, cell_grid(nx, ny), dim3(256), 0, st, cls, cls_prev, psi_prev, psi, nx, ny,
                       pitch);
    return last_status();
}

}  // namespace twg
