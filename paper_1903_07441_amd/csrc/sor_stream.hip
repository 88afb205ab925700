// Streamed, temporally blocked red-black SOR for gfx950: the relaxation's
// hot loop (Eqs. 1-2 of the paper, boundary values of section "Harmonic
// Potential Fields").
//
// Field layout: row-major, x fastest, pitch in elements; psi = 1 - phi.  Red
// cells are (x + y) even.  One sweep sets every FREE cell of one colour, then
// of the other, to psi + w * (avg4 + f - psi), evaluated as in update.h, where
// w is omega on FREE cells and 0 on fixed ones (which are thus rewritten
// unchanged).  Every kernel reads a one-byte free mask, built once per call
// from the class map, and selects omega or 0.
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
// row step; rows live in a register ring of two windows, so no value moves
// between registers and no row step waits for a load younger than a window.  Each
// half-sweep invalidates one column at each edge of the strip, so S lanes on
// each side are halo and 128 - 4S columns are written; the rows of a tile are
// likewise extended by 2S halo rows above and below.  Reads come from `src`
// and results go to `dst` (ping-pong), so the tiles of one launch never race.
#include "stream_tile.h"

namespace twg {

namespace {

using namespace sdev;

int last_status() { return hipGetLastError() == hipSuccess ? TWG_OK : TWG_EDEVICE; }

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
    stream_tile<T, S, RHS, PAIR>(src, dst, static_cast<const uint8_t *>(wsrc), omega, f, nx, ny, pitch,
                                 strip * VW - 2 * S, ybeg, min(ybeg + RH, ny));
}

// Batched form: the tiles of many grids in one launch.  Grid g's arrays start
// at element offset desc.off of the batch base pointers; the tile count is
// read from device memory so that one captured launch serves any active set.
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
        TWG_STREAM_CASE(5)
        TWG_STREAM_CASE(6)
        TWG_STREAM_CASE(7)
        TWG_STREAM_CASE(8)
    default: return TWG_EUNSUPPORTED;
    }
#undef TWG_STREAM_CASE
    return last_status();
}

}  // namespace

int stream_rows_cap(int pitch, int elem_bytes, int S)
{
    // a tile's rows (RH + 4S of them) must span less than kMaxTileBytes
    const long long rows = (kMaxTileBytes - 1) / ((long long)pitch * elem_bytes);
    return (int)std::max(2LL, (rows - 4 * S - 2) & ~1LL);
}

bool stream_depth_supported(int S) { return S >= 1 && S <= 8; }

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

int launch_stream_f32(const float *src, float *dst, const uint8_t *fmask, float omega, const float *f, int nx,
                      int ny, int pitch, const Geometry &geo, hipStream_t st)
{
    if (pairable(src, dst, fmask, 1, f, nx, pitch))
        return f ? launch_stream<float, true, true>(src, dst, fmask, omega, f, nx, ny, pitch, geo, st)
                 : launch_stream<float, false, true>(src, dst, fmask, omega, f, nx, ny, pitch, geo, st);
    return f ? launch_stream<float, true, false>(src, dst, fmask, omega, f, nx, ny, pitch, geo, st)
             : launch_stream<float, false, false>(src, dst, fmask, omega, f, nx, ny, pitch, geo, st);
}

int launch_stream_f64(const double *src, double *dst, const uint8_t *fmask, double omega, int nx, int ny,
                      int pitch, const Geometry &geo, hipStream_t st)
{
    if (pairable(src, dst, fmask, 1, (const double *)nullptr, nx, pitch))
        return launch_stream<double, false, true>(src, dst, fmask, omega, nullptr, nx, ny, pitch, geo, st);
    return launch_stream<double, false, false>(src, dst, fmask, omega, nullptr, nx, ny, pitch, geo, st);
}

}  // namespace twg
