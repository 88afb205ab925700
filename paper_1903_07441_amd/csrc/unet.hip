// Learned warm start for the relaxation: a small encoder-decoder network that
// maps occupancy, goal-distance and ring-time channels to an initial field
// psi0.  Inference and training run in the kernels below on gfx950 matrix
// cores (bf16 operands, FP32 accumulation).
//
// Network (4 levels, 32 base channels, 443,745 parameters):
//   e0 = relu(conv3(x, 3 -> 32))                H
//   e1 = relu(conv3(pool(e0), 32 -> 64))        H/2
//   e2 = relu(conv3(pool(e1), 64 -> 128))       H/4
//   e3 = relu(conv3(pool(e2), 128 -> 128))      H/8
//   d2 = relu(conv3(cat(up(e3), e2), 256 -> 64)) H/4
//   d1 = relu(conv3(cat(up(d2), e1), 128 -> 32)) H/2
//   d0 = relu(conv3(cat(up(d1), e0), 64 -> 32))  H
//   y  = conv1(d0, 32 -> 1)
// conv3: 3x3 cross-correlation, zero padding 1, bias; pool: 2x2 mean; up: 2x
// nearest; cat: channel concatenation.  Every stored activation is bf16
// (round to nearest even); products accumulate in FP32.
//
// Layout: activations NHWC (channels contiguous), [B][H][W][C] bf16.  The
// network input is padded from 3 to 32 channels (zeros) so that every conv
// has a channel count that is a multiple of 32.  Weights [Cout][9][Cin] bf16
// (K = tap * Cin + c contiguous: the operand order of the matrix
// instruction), tap = ky * 3 + kx; the FP32 masters and Adam moments share
// that layout.  The input-gradient pass uses a second copy with the taps
// flipped and the channel roles swapped, [Cin][9][Cout].
//
// Conv as implicit GEMM on v_mfma_f32_16x16x32_bf16: D[cout][pixel] =
// sum_k W[cout][k] * In[k][pixel].  A workgroup (4 waves) produces a 16 x 16
// pixel tile for all output channels; the 18 x 18 input halo of a 32-channel
// chunk is staged in LDS (pooling and upsample + concatenation are applied
// while staging, so pooled and concatenated tensors are never stored), the
// next chunk's global loads are in flight while the current one is
// multiplied.  Each wave owns 4 output rows; a lane's accumulator holds four
// consecutive output channels of one pixel, stored as one 8-byte bf16 vector.
//
// Weight gradient: dW[cout][tap][c] = sum_pixels dOut[p][cout] * In[p + tap][c]
// with the reduction over pixels on the matrix cores: the output-gradient tile
// is staged transposed ([cout][pixel]) and the input halo as three copies
// shifted by dx, so every operand is one aligned 16-byte LDS read.  The pixel
// reduction is split over workgroups; partial sums are added in a fixed order
// by a second kernel, so gradients are deterministic.
#include "twg_internal.h"
#include "unet.h"

#include <cmath>
#include <cstring>
#include <vector>

namespace twg {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

int last_status() { return hipGetLastError() == hipSuccess ? TWG_OK : TWG_EDEVICE; }

// ---- bf16 helpers -------------------------------------------------------
// round to nearest even; NaN stays a quiet NaN.  Both results are formed
// and one selected, so the conversion never branches.
__device__ __forceinline__ uint32_t f2bf(float f)
{
    const uint32_t u = __float_as_uint(f);
    const uint32_t rounded = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
    const uint32_t qnan = ((u >> 16) | 0x40u) & 0xffffu;
    return (u & 0x7fffffffu) > 0x7f800000u ? qnan : rounded;
}
__device__ __forceinline__ float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ uint32_t pack2(float lo, float hi) { return f2bf(lo) | (f2bf(hi) << 16); }
// ReLU that keeps a NaN a NaN (the hardware max would turn it into 0), so a
// broken parameter shows up in the network's output
__device__ __forceinline__ float relu(float v) { return v != v ? v : fmaxf(v, 0.f); }
__device__ __forceinline__ bool bf_pos(uint32_t h) { return (h & 0x8000u) == 0 && (h & 0x7fffu) != 0; }

__device__ __forceinline__ bf16x8 as_bf8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ void unpack8(uint4 v, float *f)
{
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        f[2 * i] = bf_lo(w[i]);
        f[2 * i + 1] = bf_hi(w[i]);
    }
}
__device__ __forceinline__ uint4 pack8(const float *f)
{
    return make_uint4(pack2(f[0], f[1]), pack2(f[2], f[3]), pack2(f[4], f[5]), pack2(f[6], f[7]));
}

constexpr int kPlain = 0, kPool = 1, kUpCat = 2, kIn4 = 3;

constexpr int kTS = 16;       // output tile side
constexpr int kHS = 18;       // halo side
constexpr int kCK = 32;       // input channels per chunk
constexpr int kPS = kCK + 8;  // LDS pixel stride (bf16), padded against bank conflicts
constexpr int kNV = kHS * kHS * (kCK / 8);
constexpr int kVPT = (kNV + 255) / 256;

// 8 channels [c, c + 8) of the conv input at pixel (yy, xx) of image b, at
// the conv's own resolution H x W (in bounds).
//   kPlain: A is [B][H][W][CIN].
//   kPool:  A is [B][2H][2W][CIN]; the 2x2 mean, rounded to bf16.
//   kUpCat: channels < CA from A = [B][H/2][W/2][CA] (nearest), the rest
//           from Bs = [B][H][W][CIN - CA].
//   kIn4:   A is the network input [B][H][W][4] (3 channels and a zero);
//           channels from 4 on read as zero.
template <int MODE, int CIN, int CA>
__device__ __forceinline__ uint4 gather8(const uint16_t *__restrict__ A, const uint16_t *__restrict__ Bs,
                                         int b, int yy, int xx, int c, int H, int W)
{
    if (MODE == kIn4) {
        if (c != 0) return make_uint4(0, 0, 0, 0);
        const uint2 v = *reinterpret_cast<const uint2 *>(A + (((size_t)b * H + yy) * W + xx) * 4);
        return make_uint4(v.x, v.y, 0, 0);
    } else if (MODE == kPlain) {
        return *reinterpret_cast<const uint4 *>(A + (((size_t)b * H + yy) * W + xx) * CIN + c);
    } else if (MODE == kPool) {
        const size_t W2 = 2 * (size_t)W;
        const uint16_t *p = A + (((size_t)b * 2 * H + 2 * yy) * W2 + 2 * xx) * CIN + c;
        float a[8], t[8];
        unpack8(*reinterpret_cast<const uint4 *>(p), a);
        unpack8(*reinterpret_cast<const uint4 *>(p + CIN), t);
        float s0[8], s1[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) s0[i] = a[i] + t[i];
        unpack8(*reinterpret_cast<const uint4 *>(p + W2 * CIN), a);
        unpack8(*reinterpret_cast<const uint4 *>(p + W2 * CIN + CIN), t);
#pragma unroll
        for (int i = 0; i < 8; ++i) s1[i] = (s0[i] + (a[i] + t[i])) * 0.25f;
        return pack8(s1);
    } else {
        // one load from whichever tensor holds channel c (no branch: the
        // channel group differs between lanes)
        const uint16_t *p = c < CA ? A + (((size_t)b * (H / 2) + yy / 2) * (W / 2) + xx / 2) * CA + c
                                   : Bs + (((size_t)b * H + yy) * W + xx) * (CIN - CA) + (c - CA);
        return *reinterpret_cast<const uint4 *>(p);
    }
}

// Halo element v (pixel v / 4 of the 18 x 18 halo of the tile at (x0, y0),
// channel group v % 4) of input chunk ch.  The load is unconditional: an
// element outside the halo or the image reads a clamped in-bounds pixel and
// is replaced by zero, so a wave issues all its halo loads back to back
// instead of waiting for each one inside a divergent branch.
template <int MODE, int CIN, int CA>
__device__ __forceinline__ uint4 halo8(const uint16_t *__restrict__ A, const uint16_t *__restrict__ Bs, int b,
                                       int v, int x0, int y0, int ch, int H, int W)
{
    const int vc = v < kNV ? v : 0;
    const int hp = vc >> 2, cg = vc & 3;
    const int hy = hp / kHS, hx = hp - hy * kHS;
    const int yy = y0 + hy - 1, xx = x0 + hx - 1;
    const bool in = v < kNV && yy >= 0 && yy < H && xx >= 0 && xx < W;
    const uint4 val = gather8<MODE, CIN, CA>(A, Bs, b, min(max(yy, 0), H - 1), min(max(xx, 0), W - 1),
                                             ch * kCK + cg * 8, H, W);
    return in ? val : make_uint4(0, 0, 0, 0);
}


// ---- bf16 output tile ----------------------------------------------------
// A lane's accumulators hold 4 consecutive output channels of one pixel,
// 8 bytes, every 2 COUT bytes apart, so storing them directly writes every
// output line in pieces.  Instead each wave puts its 4 rows x 16 pixels of
// bf16(relu(acc + bias)) into LDS (a slice of at most 64 channels at a time)
// and writes them back as 16-byte runs of consecutive channels.  stg must
// hold 4 x 64 x (min(COB, 64) + 8) bf16; all threads of the workgroup call
// this together (it synchronises).
template <int COUT, int COB>
__device__ __forceinline__ void store_tile(const f32x4 (&acc)[4][COB / 16], const float *__restrict__ bias,
                                           uint16_t *__restrict__ out, uint16_t *stg_all, int b, int co0, int x0,
                                           int y0, int H, int W)
{
    constexpr int CS = COB < 64 ? COB : 64, NS = COB / CS, RTS = CS / 16, PSO = CS + 8;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = lane & 15, g = lane >> 4;
    uint16_t *stg = stg_all + wave * 64 * PSO;
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int q = 0; q < RTS; ++q) {
                const int rt = sl * RTS + q, o = co0 + rt * 16 + g * 4;
                const f32x4 v = acc[ct][rt];
                const float r0 = relu(v[0] + bias[o]), r1 = relu(v[1] + bias[o + 1]);
                const float r2 = relu(v[2] + bias[o + 2]), r3 = relu(v[3] + bias[o + 3]);
                *reinterpret_cast<uint2 *>(&stg[(ct * 16 + j) * PSO + q * 16 + g * 4]) =
                    make_uint2(pack2(r0, r1), pack2(r2, r3));
            }
        __syncthreads();
#pragma unroll
        for (int q = lane; q < 64 * (CS / 8); q += 64) {
            const int p = q / (CS / 8), c8 = q - p * (CS / 8);
            const int y = y0 + wave * 4 + (p >> 4), x = x0 + (p & 15);
            const uint4 v = *reinterpret_cast<const uint4 *>(&stg[p * PSO + c8 * 8]);
            if (y < H && x < W)
                *reinterpret_cast<uint4 *>(out + (((size_t)b * H + y) * W + x) * COUT + co0 + sl * CS + c8 * 8) = v;
        }
        __syncthreads();
    }
}

// ---- forward conv (and input gradient with OUT_F32) ----------------------
// grid (ceil(W/16), ceil(H/16), B * max(1, COUT / 128)), 256 threads (a
// workgroup computes at most 128 output channels).  OUT_F32: FP32 output, no
// bias, no ReLU (input gradients); else bf16(relu(acc + bias)).
template <int CIN, int COUT, int MODE, int CA, bool OUT_F32>
__global__ __launch_bounds__(256) void k_conv3(const uint16_t *__restrict__ A, const uint16_t *__restrict__ Bs,
                                               const uint16_t *__restrict__ wt,
                                               const float *__restrict__ bias, void *__restrict__ out, int H,
                                               int W)
{
    // at most 128 output channels per workgroup (accumulator registers)
    constexpr int COB = COUT < 128 ? COUT : 128, NCO = COUT / COB;
    constexpr int NCH = CIN / kCK, RT = COB / 16;
    __shared__ __align__(16) uint16_t lds[2][kHS * kHS * kPS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = lane & 15, g = lane >> 4;
    const int b = blockIdx.z / NCO, co0 = (blockIdx.z % NCO) * COB;
    const int x0 = blockIdx.x * kTS, y0 = blockIdx.y * kTS;

    uint4 st[kVPT];
    auto fetch = [&](int ch) {
#pragma unroll
        for (int r = 0; r < kVPT; ++r) st[r] = halo8<MODE, CIN, CA>(A, Bs, b, tid + 256 * r, x0, y0, ch, H, W);
    };
    auto commit = [&](int buf) {
#pragma unroll
        for (int r = 0; r < kVPT; ++r) {
            const int v = tid + 256 * r;
            if (v < kNV) *reinterpret_cast<uint4 *>(&lds[buf][(v >> 2) * kPS + (v & 3) * 8]) = st[r];
        }
    };

    f32x4 acc[4][RT];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[ct][rt] = f32x4{0.f, 0.f, 0.f, 0.f};

    fetch(0);
    commit(0);
    __syncthreads();
    for (int ch = 0; ch < NCH; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < NCH) fetch(ch + 1);
        const uint16_t *wrow = wt + (size_t)(co0 + j) * 9 * CIN + ch * kCK + g * 8;
        uint4 a_next[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
            a_next[rt] = *reinterpret_cast<const uint4 *>(wrow + (size_t)rt * 16 * 9 * CIN);
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = tap / 3, dx = tap % 3;
            uint4 a[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) a[rt] = a_next[rt];
            if (tap + 1 < 9) {
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
                    a_next[rt] = *reinterpret_cast<const uint4 *>(wrow + (size_t)rt * 16 * 9 * CIN + (tap + 1) * CIN);
            }
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                const int row = wave * 4 + ct;
                const uint4 bv =
                    *reinterpret_cast<const uint4 *>(&lds[buf][((row + dy) * kHS + j + dx) * kPS + g * 8]);
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
                    acc[ct][rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(a[rt]), as_bf8(bv), acc[ct][rt], 0, 0, 0);
            }
        }
        if (ch + 1 < NCH) commit(buf ^ 1);
        __syncthreads();
    }

    if (OUT_F32) {
        const int x = x0 + j;
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int y = y0 + wave * 4 + ct;
            if (y >= H || x >= W) continue;
            const size_t pix = ((size_t)b * H + y) * W + x;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                const int o = co0 + rt * 16 + g * 4;
                const f32x4 v = acc[ct][rt];
                *reinterpret_cast<float4 *>(static_cast<float *>(out) + pix * COUT + o) =
                    make_float4(v[0], v[1], v[2], v[3]);
            }
        }
    } else {
        // the halo buffers are free after the loop's last barrier
        store_tile<COUT, COB>(acc, bias, static_cast<uint16_t *>(out), &lds[0][0], b, co0, x0, y0, H, W);
    }
}

// ---- first layer ---------------------------------------------------------
// The input has 3 real channels, so one K = 32 slice of the implicit GEMM
// covers all nine taps (k = 3 tap + c; k >= 27 is zero) and a 16-pixel row
// of 16 output channels takes one MFMA instead of nine.  x4 is
// [B][H][W][4] bf16 (channel 3 zero); the weights keep the layers' internal
// layout [32][9][32] (input channels padded to 32, only 0..2 used).  256
// threads; a workgroup builds its weight fragments once and then loops over
// 16 x 16 pixel tiles (t = blockIdx.x, + gridDim.x, ... < B tx ty), four
// rows per wave: every workgroup reading the same few weight lines for
// every tile would queue on the cache channels that hold them.
// out = bf16(relu(acc + bias)), [B][H][W][32].
__global__ __launch_bounds__(256) void k_conv3_in(const uint16_t *__restrict__ x4, const uint16_t *__restrict__ wt,
                                                  const float *__restrict__ bias, uint16_t *__restrict__ out, int nb,
                                                  int H, int W)
{
    constexpr int COUT = 32, RT = 2, ZERO = kHS * kHS * 4;  // lds[ZERO..ZERO + 3] stay zero
    __shared__ __align__(16) uint16_t lds[kHS * kHS * 4 + 4];
    __shared__ __align__(16) uint16_t stg[4 * 64 * (COUT + 8)];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = lane & 15, g = lane >> 4;
    const int tx = (W + kTS - 1) / kTS, ty = (H + kTS - 1) / kTS, ntile = nb * tx * ty;
    // this lane's k = 8 g + i: A element (output channel rt * 16 + j) and the
    // LDS offset of its B element from the pixel's own halo position.  Every
    // load is unconditional (k >= 27 reads a valid element and is zeroed, or
    // reads the zero slot), so no load waits inside a divergent branch.
    uint32_t a[RT][4];
    int off[8];
    bool live[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int k = 8 * g + i, tap = k / 3, c = k - 3 * tap;
        live[i] = k < 27;
        off[i] = live[i] ? ((tap / 3) * kHS + (tap % 3)) * 4 + c : 0;
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            uint32_t w2[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int k = 8 * g + 2 * h + e, tap = live[2 * h + e] ? k / 3 : 0, c = live[2 * h + e] ? k - 3 * tap : 0;
                const uint32_t w = wt[((size_t)(rt * 16 + j) * 9 + tap) * 32 + c];
                w2[e] = live[2 * h + e] ? w : 0u;
            }
            a[rt][h] = w2[0] | (w2[1] << 16);
        }
    if (tid == 0) *reinterpret_cast<uint2 *>(&lds[ZERO]) = make_uint2(0, 0);

    for (int t = blockIdx.x; t < ntile; t += gridDim.x) {
        const int b = t / (tx * ty), r = t - b * (tx * ty);
        const int x0 = (r % tx) * kTS, y0 = (r / tx) * kTS;
        for (int v = tid; v < kHS * kHS; v += 256) {
            const int hy = v / kHS, hx = v - hy * kHS;
            const int yy = y0 + hy - 1, xx = x0 + hx - 1;
            const bool in = yy >= 0 && yy < H && xx >= 0 && xx < W;
            const uint2 ld = *reinterpret_cast<const uint2 *>(
                x4 + (((size_t)b * H + min(max(yy, 0), H - 1)) * W + min(max(xx, 0), W - 1)) * 4);
            *reinterpret_cast<uint2 *>(&lds[v * 4]) = in ? ld : make_uint2(0, 0);
        }
        __syncthreads();

        f32x4 acc[4][RT];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int base = ((wave * 4 + ct) * kHS + j) * 4;
            uint32_t bw[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const uint32_t lo = lds[live[2 * h] ? base + off[2 * h] : ZERO];
                const uint32_t hi = lds[live[2 * h + 1] ? base + off[2 * h + 1] : ZERO];
                bw[h] = lo | (hi << 16);
            }
            const uint4 bv = make_uint4(bw[0], bw[1], bw[2], bw[3]);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
                acc[ct][rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    as_bf8(make_uint4(a[rt][0], a[rt][1], a[rt][2], a[rt][3])), as_bf8(bv),
                    f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        }
        // store_tile synchronises before and after its LDS round trip, so
        // the halo is free for the next tile when it returns
        store_tile<COUT, COUT>(acc, bias, out, stg, b, 0, x0, y0, H, W);
    }
}

// ---- weight gradient -----------------------------------------------------
constexpr int kOS = 256 + 8;              // LDS stride of one output channel's pixel row
constexpr int kIS = kHS * kTS + 8;        // LDS stride of one input channel (18 rows x 16)

// grid (CIN / 32, nsplit), 256 threads.  Workgroup (chunk, split) adds up
// the pixel tiles split, split + nsplit, ... of all images and writes
// part[split][cout][tap][chunk * 32 + c]; chunk 0 also writes the bias
// gradient's partial sums bpart[split][cout].
template <int CIN, int COUT, int MODE, int CA>
__global__ __launch_bounds__(256) void k_wgrad3(const uint16_t *__restrict__ A, const uint16_t *__restrict__ Bs,
                                                const uint16_t *__restrict__ dout, float *__restrict__ part,
                                                float *__restrict__ bpart, int nb, int H, int W, int nsplit)
{
    constexpr int NPAIR = (COUT / 16) * 2, PPW = NPAIR / 4;
    static_assert(NPAIR % 4 == 0, "pairs must split over 4 waves");
    __shared__ __align__(16) uint16_t ldo[COUT * kOS];
    __shared__ __align__(16) uint16_t ldi[3 * kCK * kIS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = lane & 15, g = lane >> 4;
    const int ch = blockIdx.x, split = blockIdx.y;
    const int tx = (W + kTS - 1) / kTS, ty = (H + kTS - 1) / kTS, per = tx * ty, ntile = nb * per;

    f32x4 acc[PPW][9];
#pragma unroll
    for (int q = 0; q < PPW; ++q)
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[q][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;

    for (int t = split; t < ntile; t += nsplit) {
        const int b = t / per, r = t - b * per;
        const int y0 = (r / tx) * kTS, x0 = (r % tx) * kTS;
        // output gradient tile, transposed to [cout][pixel]
        for (int v = tid; v < 256 * (COUT / 8); v += 256) {
            const int p = v & 255, cg = v >> 8;
            const int y = y0 + (p >> 4), x = x0 + (p & 15);
            const uint4 ld = *reinterpret_cast<const uint4 *>(
                dout + (((size_t)b * H + min(y, H - 1)) * W + min(x, W - 1)) * COUT + cg * 8);
            const uint4 val = y < H && x < W ? ld : make_uint4(0, 0, 0, 0);
            const uint32_t w4[4] = {val.x, val.y, val.z, val.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                ldo[(cg * 8 + 2 * e) * kOS + p] = (uint16_t)(w4[e] & 0xffffu);
                ldo[(cg * 8 + 2 * e + 1) * kOS + p] = (uint16_t)(w4[e] >> 16);
            }
        }
        // input halo of this channel chunk as three copies shifted by dx:
        // ldi[dx][c][hy][px] = In(y0 + hy - 1, x0 + px + dx - 1, c)
        for (int v = tid; v < kNV; v += 256) {
            const int hp = v >> 2, cg = v & 3;
            const int hy = hp / kHS, hx = hp - hy * kHS;
            const uint4 val = halo8<MODE, CIN, CA>(A, Bs, b, v, x0, y0, ch, H, W);
            const uint32_t w4[4] = {val.x, val.y, val.z, val.w};
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int px = hx - dx;
                if (px < 0 || px >= kTS) continue;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    ldi[(dx * kCK + cg * 8 + 2 * e) * kIS + hy * kTS + px] = (uint16_t)(w4[e] & 0xffffu);
                    ldi[(dx * kCK + cg * 8 + 2 * e + 1) * kIS + hy * kTS + px] = (uint16_t)(w4[e] >> 16);
                }
            }
        }
        __syncthreads();
        if (ch == 0 && tid < COUT) {
            const uint16_t *row = ldo + tid * kOS;
            for (int p = 0; p < 256; ++p) bsum += __uint_as_float((uint32_t)row[p] << 16);
        }
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) {
            const int row = 2 * kb + (g >> 1), col = (g & 1) * 8;
#pragma unroll
            for (int q = 0; q < PPW; ++q) {
                const int pair = wave * PPW + q, ot = pair >> 1, cti = pair & 1;
                const uint4 av = *reinterpret_cast<const uint4 *>(&ldo[(ot * 16 + j) * kOS + row * kTS + col]);
#pragma unroll
                for (int tap = 0; tap < 9; ++tap) {
                    const int dy = tap / 3, dx = tap % 3;
                    const uint4 bv = *reinterpret_cast<const uint4 *>(
                        &ldi[(dx * kCK + cti * 16 + j) * kIS + (row + dy) * kTS + col]);
                    acc[q][tap] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(av), as_bf8(bv), acc[q][tap], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < PPW; ++q) {
        const int pair = wave * PPW + q, ot = pair >> 1, cti = pair & 1;
        const int c = ch * kCK + cti * 16 + j;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int o = ot * 16 + g * 4 + v;
                part[(((size_t)split * COUT + o) * 9 + tap) * CIN + c] = acc[q][tap][v];
            }
    }
    if (ch == 0 && tid < COUT) bpart[(size_t)split * COUT + tid] = bsum;
}

// out[i] = sum over s < n of part[s * stride + i].  A block covers 64
// consecutive i with 4 lanes each; lane q adds s = q, q + 4, ... in order and
// the four lane sums are combined in a fixed order, so the result does not
// depend on scheduling.
__global__ __launch_bounds__(256) void k_sum_parts(const float *__restrict__ part, float *__restrict__ out,
                                                   int count, int n, size_t stride)
{
    __shared__ float red[4][64];
    const int q = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int i = blockIdx.x * 64 + l;
    float s = 0.f;
    if (i < count)
        for (int k = q; k < n; k += 4) s += part[(size_t)k * stride + i];
    red[q][l] = s;
    __syncthreads();
    if (q == 0 && i < count) out[i] = (red[0][l] + red[1][l]) + (red[2][l] + red[3][l]);
}

// ---- head, loss, routing ---------------------------------------------------
__device__ __forceinline__ float wave_sum(float v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// y = hb + sum_c hw[c] d0[c] for every pixel (FP32, channel order).
__device__ __forceinline__ float head_value(const uint16_t *__restrict__ d0p, const float *__restrict__ hw,
                                            float hb, float *d)
{
#pragma unroll
    for (int q = 0; q < 4; ++q) unpack8(reinterpret_cast<const uint4 *>(d0p)[q], d + 8 * q);
    float y = hb;
#pragma unroll
    for (int c = 0; c < 32; ++c) y = y + hw[c] * d[c];
    return y;
}

// Training head: masked MSE over FREE cells.  Per pixel: y, diff = y - t
// (0 outside the mask), loss += diff^2 / (n_b B), dy = 2 diff / (n_b B),
// dd0 = bf16(dy * hw * [d0 > 0]); block partial sums of the head gradients
// (hw: 32, hb: 1) and of the loss go to part[block][34].
__global__ __launch_bounds__(256) void k_head_loss(const uint16_t *__restrict__ d0, const float *__restrict__ hw,
                                                   const float *__restrict__ hb, const float *__restrict__ target,
                                                   const uint8_t *__restrict__ cls,
                                                   const unsigned int *__restrict__ cnt, int hw_pixels, int nb,
                                                   uint16_t *__restrict__ dd0, float *__restrict__ y_out,
                                                   float *__restrict__ part)
{
    __shared__ float red[4][34];
    const int p = blockIdx.x * 256 + threadIdx.x;
    const int total = hw_pixels * nb;
    float gw[32], gb = 0.f, lp = 0.f;
#pragma unroll
    for (int c = 0; c < 32; ++c) gw[c] = 0.f;
    if (p < total) {
        const int b = p / hw_pixels;
        float d[32];
        const float y = head_value(d0 + (size_t)p * 32, hw, hb[0], d);
        if (y_out) y_out[p] = y;
        const float diff = cls[p] == TWG_CELL_FREE ? y - target[p] : 0.f;
        const unsigned int nf = cnt[b];
        const float sc = (1.f / (float)(nf > 1u ? nf : 1u)) / (float)nb;
        lp = diff * diff * sc;
        const float dy = 2.f * diff * sc;
        gb = dy;
        float dd[32];
#pragma unroll
        for (int c = 0; c < 32; ++c) {
            gw[c] = dy * d[c];
            dd[c] = d[c] > 0.f ? dy * hw[c] : 0.f;
        }
        uint4 *o = reinterpret_cast<uint4 *>(dd0 + (size_t)p * 32);
#pragma unroll
        for (int q = 0; q < 4; ++q) o[q] = pack8(dd + 8 * q);
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int c = 0; c < 32; ++c) {
        const float s = wave_sum(gw[c]);
        if (lane == 0) red[wave][c] = s;
    }
    {
        const float s = wave_sum(gb);
        if (lane == 0) red[wave][32] = s;
        const float l = wave_sum(lp);
        if (lane == 0) red[wave][33] = l;
    }
    __syncthreads();
    if (threadIdx.x < 34) {
        const int c = threadIdx.x;
        part[(size_t)blockIdx.x * 34 + c] = ((red[0][c] + red[1][c]) + (red[2][c] + red[3][c]));
    }
}

// Inference head into a field: FREE cells get clamp(y, 0, 1); OBST/WALL 0,
// GOAL 1; FIXED cells keep their value.  The network runs on a padded
// Hp x Wp frame; only the grid's nx x ny cells are written.
// A non-finite output at a FREE cell sets *bad (the whole field then falls
// back to the plain start, k_net_fallback).
__global__ __launch_bounds__(256) void k_head_psi(const uint16_t *__restrict__ d0, const float *__restrict__ hw,
                                                  const float *__restrict__ hb, const uint8_t *__restrict__ cls,
                                                  float *__restrict__ psi, int nx, int ny, int pitch, int Wp,
                                                  unsigned int *bad)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= nx || y >= ny) return;
    const size_t i = (size_t)y * pitch + x;
    const uint8_t c = cls[i];
    if (c == TWG_CELL_FREE) {
        float d[32];
        const float v = head_value(d0 + ((size_t)y * Wp + x) * 32, hw, hb[0], d);
        if (!isfinite(v)) atomicOr(bad, 1u);
        psi[i] = fminf(fmaxf(v, 0.f), 1.f);
    } else if (c == TWG_CELL_OBST || c == TWG_CELL_WALL) {
        psi[i] = 0.f;
    } else if (c == TWG_CELL_GOAL) {
        psi[i] = 1.f;
    }
}

// Fallback of a warm start whose network produced a non-finite value: every
// FREE cell gets the plain start 0.5 (the fixed cells are already set);
// *status (if given) receives TWG_OK or TWG_NET_FALLBACK.
__global__ __launch_bounds__(256) void k_net_fallback(const uint8_t *__restrict__ cls, float *__restrict__ psi,
                                                      int nx, int ny, int pitch, const unsigned int *bad,
                                                      int32_t *status)
{
    const bool fall = *bad != 0u;
    if (status && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0)
        *status = fall ? TWG_NET_FALLBACK : TWG_OK;
    if (!fall) return;
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= nx || y >= ny) return;
    const size_t i = (size_t)y * pitch + x;
    if (cls[i] == TWG_CELL_FREE) psi[i] = 0.5f;
}

// Zero n device words (a kernel, so that the call can be captured into a
// graph without memset nodes).
__global__ void k_zero_words(unsigned int *w, int n)
{
    if (blockIdx.x == 0 && (int)threadIdx.x < n) w[threadIdx.x] = 0u;
}

// Plain head output y[p] (no field semantics).
__global__ __launch_bounds__(256) void k_head_plain(const uint16_t *__restrict__ d0, const float *__restrict__ hw,
                                                    const float *__restrict__ hb, float *__restrict__ y, int total)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= total) return;
    float d[32];
    y[p] = head_value(d0 + (size_t)p * 32, hw, hb[0], d);
}

// Gradient through up() into a low-resolution activation:
// dlow[b][Y][X][c] = bf16((sum_{2x2} dc[b][2Y+a][2X+e][c]) * [act > 0]) for
// c < CL, where dc is the FP32 input gradient of a concatenating conv with
// CT channels.  One thread per (low pixel, 8 channels).
template <int CL, int CT>
__global__ __launch_bounds__(256) void k_route_up(const float *__restrict__ dc, const uint16_t *__restrict__ act,
                                                  uint16_t *__restrict__ dlow, int nb, int Hl, int Wl)
{
    const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long total = (long long)nb * Hl * Wl * (CL / 8);
    if (v >= total) return;
    const int cg = (int)(v % (CL / 8));
    const long long lp = v / (CL / 8);
    const int X = (int)(lp % Wl);
    const long long t = lp / Wl;
    const int Y = (int)(t % Hl);
    const int b = (int)(t / Hl);
    const int Hh = 2 * Hl, Wh = 2 * Wl;
    float s[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) s[i] = 0.f;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const float *p = dc + (((size_t)b * Hh + 2 * Y + a) * Wh + 2 * X + e) * CT + cg * 8;
            const float4 u = reinterpret_cast<const float4 *>(p)[0], w = reinterpret_cast<const float4 *>(p)[1];
            s[0] += u.x; s[1] += u.y; s[2] += u.z; s[3] += u.w;
            s[4] += w.x; s[5] += w.y; s[6] += w.z; s[7] += w.w;
        }
    const uint4 av = *reinterpret_cast<const uint4 *>(act + (size_t)lp * CL + cg * 8);
    const uint32_t aw[4] = {av.x, av.y, av.z, av.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (!bf_pos(aw[i] & 0xffffu)) s[2 * i] = 0.f;
        if (!bf_pos(aw[i] >> 16)) s[2 * i + 1] = 0.f;
    }
    *reinterpret_cast<uint4 *>(dlow + (size_t)lp * CL + cg * 8) = pack8(s);
}

// Gradient of an encoder activation used by a skip connection and by pool():
// de[b][y][x][c] = bf16((dskip[...][OFF + c] + dp[b][y/2][x/2][c] / 4) * [e > 0]),
// dskip an FP32 input gradient with CT channels, dp the FP32 input gradient
// of the next encoder conv (C channels at half resolution).
template <int C, int OFF, int CT>
__global__ __launch_bounds__(256) void k_route_pool(const float *__restrict__ dskip, const float *__restrict__ dp,
                                                    const uint16_t *__restrict__ e, uint16_t *__restrict__ de,
                                                    int nb, int H, int W)
{
    const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long total = (long long)nb * H * W * (C / 8);
    if (v >= total) return;
    const int cg = (int)(v % (C / 8));
    const long long pix = v / (C / 8);
    const int x = (int)(pix % W);
    const long long t = pix / W;
    const int y = (int)(t % H);
    const int b = (int)(t / H);
    const float *ps = dskip + (size_t)pix * CT + OFF + cg * 8;
    const float *pp = dp + (((size_t)b * (H / 2) + y / 2) * (W / 2) + x / 2) * C + cg * 8;
    float s[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) s[i] = ps[i] + pp[i] * 0.25f;
    const uint4 av = *reinterpret_cast<const uint4 *>(e + (size_t)pix * C + cg * 8);
    const uint32_t aw[4] = {av.x, av.y, av.z, av.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (!bf_pos(aw[i] & 0xffffu)) s[2 * i] = 0.f;
        if (!bf_pos(aw[i] >> 16)) s[2 * i + 1] = 0.f;
    }
    *reinterpret_cast<uint4 *>(de + (size_t)pix * C + cg * 8) = pack8(s);
}

// ---- input packing and features ------------------------------------------
// x [P][3] FP32 -> xp [P][4] bf16 (channel 3 zero)
__global__ __launch_bounds__(256) void k_pack_input(const float *__restrict__ x, uint16_t *__restrict__ xp,
                                                    long long total)
{
    const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
    if (p >= total) return;
    *reinterpret_cast<uint2 *>(xp + (size_t)p * 4) = make_uint2(pack2(x[3 * p], x[3 * p + 1]), pack2(x[3 * p + 2], 0.f));
}

// Network input channels of a grid on an Hp x Wp frame (frame cells outside
// the grid read as walls): occupancy (1 on OBST and WALL), Euclidean goal
// distance / (max(nx, ny) sqrt 2), ring / max ring (0 without a ring map).
// Writes FP32 [Hp][Wp][3] to xf and/or bf16 [Hp][Wp][4] (channel 3 zero) to xp.
__global__ __launch_bounds__(256) void k_features(const uint8_t *__restrict__ cls, const uint16_t *__restrict__ ring,
                                                  int nx, int ny, int pitch, int Hp, int Wp, int gx, int gy,
                                                  float inv_diag, const unsigned int *__restrict__ jmax,
                                                  float *__restrict__ xf, uint16_t *__restrict__ xp)
{
    const unsigned int jm = ring ? *jmax : 0u;
    const float inv_jmax = jm > 0u ? 1.f / (float)jm : 0.f;
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= Wp || y >= Hp) return;
    float occ = 1.f, rt = 0.f;
    if (x < nx && y < ny) {
        const size_t i = (size_t)y * pitch + x;
        const uint8_t c = cls[i];
        occ = (c == TWG_CELL_OBST || c == TWG_CELL_WALL) ? 1.f : 0.f;
        if (ring) rt = (float)ring[i] * inv_jmax;
    }
    const float ddx = (float)(x - gx), ddy = (float)(y - gy);
    const float gd = sqrtf(ddx * ddx + ddy * ddy) * inv_diag;
    const size_t p = (size_t)y * Wp + x;
    if (xf) {
        xf[3 * p] = occ;
        xf[3 * p + 1] = gd;
        xf[3 * p + 2] = rt;
    }
    if (xp) *reinterpret_cast<uint2 *>(xp + p * 4) = make_uint2(pack2(occ, gd), pack2(rt, 0.f));
}

// ---- coarse-scale warm start ------------------------------------------------
// Input channels of a grid seen at 1/f of its resolution on an Hc x Wc frame:
// coarse cell (X, Y) covers the fine cells [fX, fX + f) x [fY, fY + f),
// cells outside the grid reading as walls.  Occupancy = share of OBST, WALL
// and outside cells in the block; goal distance of the block's centre
// (fX + (f - 1) / 2, fY + (f - 1) / 2) / (max(nx, ny) sqrt 2), the fine
// scale's normalisation; ring of the fine cell at the block's centre
// (fX + f / 2, fY + f / 2), clamped into the grid, / max ring (0 without a
// ring map).  ccls (optional): FREE where the block holds a FREE cell, else
// OBST (the training loss's mask at the coarse scale).
__global__ __launch_bounds__(256) void k_features_coarse(const uint8_t *__restrict__ cls,
                                                         const uint16_t *__restrict__ ring, int nx, int ny,
                                                         int pitch, int f, int Hc, int Wc, int gx, int gy,
                                                         float inv_diag, const unsigned int *__restrict__ jmax,
                                                         float *__restrict__ xf, uint16_t *__restrict__ xp,
                                                         uint8_t *__restrict__ ccls)
{
    const unsigned int jm = ring ? *jmax : 0u;
    const float inv_jmax = jm > 0u ? 1.f / (float)jm : 0.f;
    const int X = blockIdx.x * 64 + (threadIdx.x & 63);
    const int Y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (X >= Wc || Y >= Hc) return;
    int blocked = 0, nfree = 0;
    for (int dy = 0; dy < f; ++dy) {
        const int y = Y * f + dy;
        for (int dx = 0; dx < f; ++dx) {
            const int x = X * f + dx;
            if (x >= nx || y >= ny) {
                ++blocked;
                continue;
            }
            const uint8_t c = cls[(size_t)y * pitch + x];
            blocked += (c == TWG_CELL_OBST || c == TWG_CELL_WALL) ? 1 : 0;
            nfree += c == TWG_CELL_FREE ? 1 : 0;
        }
    }
    const float occ = (float)blocked / (float)(f * f);
    const float half = 0.5f * (float)(f - 1);
    const float ddx = ((float)(X * f) + half) - (float)gx, ddy = ((float)(Y * f) + half) - (float)gy;
    const float gd = sqrtf(ddx * ddx + ddy * ddy) * inv_diag;
    float rt = 0.f;
    if (ring && X * f < nx && Y * f < ny) {
        const int xc = min(X * f + f / 2, nx - 1), yc = min(Y * f + f / 2, ny - 1);
        rt = (float)ring[(size_t)yc * pitch + xc] * inv_jmax;
    }
    const size_t p = (size_t)Y * Wc + X;
    if (xf) {
        xf[3 * p] = occ;
        xf[3 * p + 1] = gd;
        xf[3 * p + 2] = rt;
    }
    if (xp) *reinterpret_cast<uint2 *>(xp + p * 4) = make_uint2(pack2(occ, gd), pack2(rt, 0.f));
    if (ccls) ccls[p] = nfree > 0 ? TWG_CELL_FREE : TWG_CELL_OBST;
}

// Coarse training target: out[Y][X] = mean of psi over the FREE fine cells of
// block (X, Y), summed in row order in FP32 (0 when the block has none).
__global__ __launch_bounds__(256) void k_coarse_target(const float *__restrict__ psi, const uint8_t *__restrict__ cls,
                                                       int nx, int ny, int pitch, int f, int Hc, int Wc,
                                                       float *__restrict__ out)
{
    const int X = blockIdx.x * 64 + (threadIdx.x & 63);
    const int Y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (X >= Wc || Y >= Hc) return;
    float sum = 0.f;
    int cnt = 0;
    for (int dy = 0; dy < f; ++dy) {
        const int y = Y * f + dy;
        if (y >= ny) break;
        for (int dx = 0; dx < f; ++dx) {
            const int x = X * f + dx;
            if (x >= nx) break;
            const size_t i = (size_t)y * pitch + x;
            if (cls[i] == TWG_CELL_FREE) {
                sum = sum + psi[i];
                ++cnt;
            }
        }
    }
    out[(size_t)Y * Wc + X] = cnt > 0 ? sum / (float)cnt : 0.f;
}

// Warm-start field from a coarse output yc [Hc][Wc]: a FREE cell (x, y) takes
// the bilinear interpolation of yc at coarse coordinates
// ((x + 1/2) / f - 1/2, (y + 1/2) / f - 1/2), clamped to the frame, then to
// [0, 1]; OBST and WALL 0, GOAL 1, FIXED unchanged.  A non-finite value at a
// FREE cell sets *bad.
__global__ __launch_bounds__(256) void k_up_psi(const float *__restrict__ yc, int Hc, int Wc, int f,
                                                const uint8_t *__restrict__ cls, float *__restrict__ psi, int nx,
                                                int ny, int pitch, unsigned int *bad)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= nx || y >= ny) return;
    const size_t i = (size_t)y * pitch + x;
    const uint8_t c = cls[i];
    if (c == TWG_CELL_FREE) {
        const float inv_f = 1.f / (float)f;  // f is a power of two: exact
        const float u = fminf(fmaxf(((float)x + 0.5f) * inv_f - 0.5f, 0.f), (float)(Wc - 1));
        const float v = fminf(fmaxf(((float)y + 0.5f) * inv_f - 0.5f, 0.f), (float)(Hc - 1));
        const int x0 = (int)u, y0 = (int)v;
        const int x1 = min(x0 + 1, Wc - 1), y1 = min(y0 + 1, Hc - 1);
        const float a = u - (float)x0, b = v - (float)y0;
        const float top = (1.f - a) * yc[(size_t)y0 * Wc + x0] + a * yc[(size_t)y0 * Wc + x1];
        const float bot = (1.f - a) * yc[(size_t)y1 * Wc + x0] + a * yc[(size_t)y1 * Wc + x1];
        const float val = (1.f - b) * top + b * bot;
        if (!isfinite(val)) atomicOr(bad, 1u);
        psi[i] = fminf(fmaxf(val, 0.f), 1.f);
    } else if (c == TWG_CELL_OBST || c == TWG_CELL_WALL) {
        psi[i] = 0.f;
    } else if (c == TWG_CELL_GOAL) {
        psi[i] = 1.f;
    }
}

// largest ring number of a grid; *out must be zero beforehand.  Grid-stride
// over rows, wave and block maxima, one atomic per block.
__global__ __launch_bounds__(256) void k_ring_max(const uint16_t *__restrict__ ring, int nx, int ny, int pitch,
                                                  unsigned int *out)
{
    __shared__ unsigned int red[4];
    unsigned int r = 0;
    for (int y = blockIdx.x; y < ny; y += gridDim.x)
        for (int x = threadIdx.x; x < nx; x += 256) r = max(r, (unsigned int)ring[(size_t)y * pitch + x]);
    for (int o = 32; o > 0; o >>= 1) r = max(r, (unsigned int)__shfl_xor((int)r, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        r = max(max(red[0], red[1]), max(red[2], red[3]));
        if (r) atomicMax(out, r);
    }
}

// ---- parameters ------------------------------------------------------------
// Element i of the internal parameter vector: layer, and for a conv weight
// its (o, tap, c).  Returns the layer or -1; *kind = 0 weight, 1 bias.
struct ParamPos {
    int layer, kind, o, tap, c;
};
__device__ __forceinline__ ParamPos locate(const NetLayout &L, int i)
{
    ParamPos r{-1, 0, 0, 0, 0};
#pragma unroll
    for (int l = 0; l < kNetLayers; ++l) {
        const int kk = L.k[l] * L.k[l];
        const int nw = L.cout[l] * kk * L.cinp[l];
        if (i >= L.offw[l] && i < L.offw[l] + nw) {
            const int q = i - L.offw[l];
            r.layer = l;
            r.kind = 0;
            r.c = q % L.cinp[l];
            r.tap = (q / L.cinp[l]) % kk;
            r.o = q / (L.cinp[l] * kk);
        } else if (i >= L.offb[l] && i < L.offb[l] + L.cout[l]) {
            r.layer = l;
            r.kind = 1;
            r.o = i - L.offb[l];
        }
    }
    return r;
}

// write the bf16 copies of weight element (o, tap, c) of a 3x3 layer
__device__ __forceinline__ void store_copies(const NetLayout &L, const ParamPos &pp, float v,
                                             uint16_t *__restrict__ wt, uint16_t *__restrict__ wf, int i)
{
    const uint16_t h = (uint16_t)f2bf(v);
    wt[i] = h;
    if (L.k[pp.layer] == 3)
        wf[L.offw[pp.layer] + ((size_t)pp.c * 9 + (8 - pp.tap)) * L.cout[pp.layer] + pp.o] = h;
}

// external (oracle order: per layer w[cout][cin][ky][kx], then b[cout]) ->
// internal masters + bf16 copies
__global__ void k_params_in(NetLayout L, const float *__restrict__ ext, float *__restrict__ master,
                            uint16_t *__restrict__ wt, uint16_t *__restrict__ wf)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.total_int) return;
    const ParamPos pp = locate(L, i);
    if (pp.layer < 0) return;
    const int l = pp.layer;
    float v;
    if (pp.kind == 1) {
        v = ext[L.extb[l] + pp.o];
    } else {
        const int k = L.k[l];
        v = pp.c < L.cin[l] ? ext[L.extw[l] + ((pp.o * L.cin[l] + pp.c) * k + pp.tap / k) * k + pp.tap % k] : 0.f;
    }
    master[i] = v;
    if (pp.kind == 0) store_copies(L, pp, v, wt, wf, i);
}

// internal -> external order
__global__ void k_params_out(NetLayout L, const float *__restrict__ master, float *__restrict__ ext)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.total_int) return;
    const ParamPos pp = locate(L, i);
    if (pp.layer < 0) return;
    const int l = pp.layer;
    if (pp.kind == 1) {
        ext[L.extb[l] + pp.o] = master[i];
    } else if (pp.c < L.cin[l]) {
        const int k = L.k[l];
        ext[L.extw[l] + ((pp.o * L.cin[l] + pp.c) * k + pp.tap / k) * k + pp.tap % k] = master[i];
    }
}

// Adam (Kingma & Ba) on the FP32 masters; bias corrections c1 = 1 / (1 -
// b1^t), c2 = 1 / (1 - b2^t) come from the host.  Padded input channels of
// the first layer stay zero.
__global__ void k_adam(NetLayout L, float *__restrict__ master, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ grad, uint16_t *__restrict__ wt, uint16_t *__restrict__ wf,
                       float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.total_int) return;
    const ParamPos pp = locate(L, i);
    if (pp.layer < 0) return;
    if (pp.kind == 0 && pp.c >= L.cin[pp.layer]) return;
    const float gi = grad[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi * c1, vh = vi * c2;
    const float p = master[i] - lr * mh / (sqrtf(vh) + eps);
    master[i] = p;
    if (pp.kind == 0) store_copies(L, pp, p, wt, wf, i);
}

__global__ void k_zero_u32n(unsigned int *__restrict__ w, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) w[i] = 0u;
}

// per-image count of FREE cells, added into cnt[b] (integer additions are
// exact in any order); grid (blocks per image, images)
__global__ __launch_bounds__(256) void k_count_free(const uint8_t *__restrict__ cls, int hw_pixels,
                                                    unsigned int *__restrict__ cnt)
{
    const int b = blockIdx.y;
    unsigned int n = 0;
    for (int p = blockIdx.x * 256 + threadIdx.x; p < hw_pixels; p += gridDim.x * 256)
        n += cls[(size_t)b * hw_pixels + p] == TWG_CELL_FREE;
    for (int o = 32; o > 0; o >>= 1) n += (unsigned int)__shfl_xor((int)n, o);
    if ((threadIdx.x & 63) == 0 && n) atomicAdd(cnt + b, n);
}

// column c < 34 of part[nblk][34] summed by block c: thread t adds rows t,
// t + 256, ... in order, then a fixed tree over the 256 thread sums.
__global__ __launch_bounds__(256) void k_sum_loss(const float *__restrict__ part, int nblk, float *__restrict__ loss,
                                                  float *__restrict__ head_grad)
{
    __shared__ float red[256];
    const int c = blockIdx.x;
    float s = 0.f;
    for (int k = threadIdx.x; k < nblk; k += 256) s += part[(size_t)k * 34 + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (c < 33) head_grad[c] = red[0];
        else if (loss) loss[0] = red[0];
    }
}

// ---- launch helpers -----------------------------------------------------------
template <int CIN, int COUT, int MODE, int CA, bool F32>
int conv(const uint16_t *A, const uint16_t *Bs, const uint16_t *wt, const float *bias, void *out, int nb, int H,
         int W, hipStream_t st)
{
    const dim3 grid((W + kTS - 1) / kTS, (H + kTS - 1) / kTS, nb * (COUT > 128 ? COUT / 128 : 1));
    hipLaunchKernelGGL((k_conv3<CIN, COUT, MODE, CA, F32>), grid, dim3(256), 0, st, A, Bs, wt, bias, out, H, W);
    return last_status();
}

int choose_split(int nchunk, int ntile)
{
    int s = std::max(1, 256 / nchunk);
    return std::min(s, ntile);
}

template <int CIN, int COUT, int MODE, int CA>
int wgrad(const uint16_t *A, const uint16_t *Bs, const uint16_t *dout, float *part, float *bpart, float *gw,
          float *gb, int nb, int H, int W, hipStream_t st)
{
    const int ntile = nb * ((H + kTS - 1) / kTS) * ((W + kTS - 1) / kTS);
    const int ns = choose_split(CIN / kCK, ntile);
    hipLaunchKernelGGL((k_wgrad3<CIN, COUT, MODE, CA>), dim3(CIN / kCK, ns), dim3(256), 0, st, A, Bs, dout, part,
                       bpart, nb, H, W, ns);
    const int nw = COUT * 9 * CIN;
    hipLaunchKernelGGL(k_sum_parts, dim3((nw + 63) / 64), dim3(256), 0, st, part, gw, nw, ns, (size_t)nw);
    hipLaunchKernelGGL(k_sum_parts, dim3((COUT + 63) / 64), dim3(256), 0, st, bpart, gb, COUT, ns, (size_t)COUT);
    return last_status();
}

template <int CL, int CT>
int route_up(const float *dc, const uint16_t *act, uint16_t *dlow, int nb, int Hl, int Wl, hipStream_t st)
{
    const long long total = (long long)nb * Hl * Wl * (CL / 8);
    hipLaunchKernelGGL((k_route_up<CL, CT>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, dc, act, dlow,
                       nb, Hl, Wl);
    return last_status();
}

template <int C, int OFF, int CT>
int route_pool(const float *dskip, const float *dp, const uint16_t *e, uint16_t *de, int nb, int H, int W,
               hipStream_t st)
{
    const long long total = (long long)nb * H * W * (C / 8);
    hipLaunchKernelGGL((k_route_pool<C, OFF, CT>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, dskip,
                       dp, e, de, nb, H, W);
    return last_status();
}

}  // namespace

// ---- host side ----------------------------------------------------------------

NetLayout net_layout()
{
    static const int spec[kNetLayers][3] = {{3, 32, 3},   {32, 64, 3},  {64, 128, 3}, {128, 128, 3},
                                            {256, 64, 3}, {128, 32, 3}, {64, 32, 3},  {32, 1, 1}};
    NetLayout L{};
    int oi = 0, oe = 0;
    for (int l = 0; l < kNetLayers; ++l) {
        L.cin[l] = spec[l][0];
        L.cinp[l] = spec[l][0] < 32 ? 32 : spec[l][0];
        L.cout[l] = spec[l][1];
        L.k[l] = spec[l][2];
        const int kk = L.k[l] * L.k[l];
        L.offw[l] = oi;
        oi += L.cout[l] * kk * L.cinp[l];
        L.offb[l] = oi;
        oi += L.cout[l];
        L.extw[l] = oe;
        oe += L.cout[l] * kk * L.cin[l];
        L.extb[l] = oe;
        oe += L.cout[l];
    }
    L.total_int = oi;
    L.total_ext = oe;
    return L;
}

int net_forward(twg_unet *n, int nb, int H, int W, hipStream_t st)
{
    const NetLayout &L = n->L;
    const uint16_t *wt = n->wt;
    const float *mb = n->master;
    auto W_ = [&](int l) { return wt + L.offw[l]; };
    auto B_ = [&](int l) { return mb + L.offb[l]; };
    const int H1 = H / 2, W1 = W / 2, H2 = H / 4, W2 = W / 4, H3 = H / 8, W3 = W / 8;
    {
        const long long ntile = (long long)nb * ((W + kTS - 1) / kTS) * ((H + kTS - 1) / kTS);
        const int grid = (int)std::max<long long>(1, std::min<long long>(ntile, 2048));
        hipLaunchKernelGGL(k_conv3_in, dim3(grid), dim3(256), 0, st, n->xp, W_(0), B_(0), n->e0, nb, H, W);
    }
    int rc = last_status();
    if (!rc) rc = conv<32, 64, kPool, 0, false>(n->e0, nullptr, W_(1), B_(1), n->e1, nb, H1, W1, st);
    if (!rc) rc = conv<64, 128, kPool, 0, false>(n->e1, nullptr, W_(2), B_(2), n->e2, nb, H2, W2, st);
    if (!rc) rc = conv<128, 128, kPool, 0, false>(n->e2, nullptr, W_(3), B_(3), n->e3, nb, H3, W3, st);
    if (!rc) rc = conv<256, 64, kUpCat, 128, false>(n->e3, n->e2, W_(4), B_(4), n->d2, nb, H2, W2, st);
    if (!rc) rc = conv<128, 32, kUpCat, 64, false>(n->d2, n->e1, W_(5), B_(5), n->d1, nb, H1, W1, st);
    if (!rc) rc = conv<64, 32, kUpCat, 32, false>(n->d1, n->e0, W_(6), B_(6), n->d0, nb, H, W, st);
    return rc;
}

int net_backward(twg_unet *n, int nb, int H, int W, const float *target, const uint8_t *cls, float *loss,
                 hipStream_t st)
{
    const NetLayout &L = n->L;
    const uint16_t *wf = n->wf;
    auto F_ = [&](int l) { return wf + L.offw[l]; };
    auto GW = [&](int l) { return n->grad + L.offw[l]; };
    auto GB = [&](int l) { return n->grad + L.offb[l]; };
    const int H1 = H / 2, W1 = W / 2, H2 = H / 4, W2 = W / 4, H3 = H / 8, W3 = W / 8;
    const int hwp = H * W, total = nb * hwp;
    // head and loss
    unsigned int *cnt = n->counts;
    hipLaunchKernelGGL(k_zero_u32n, dim3((nb + 255) / 256), dim3(256), 0, st, cnt, nb);
    hipLaunchKernelGGL(k_count_free, dim3(std::max(1, std::min(64, hwp / 4096)), nb), dim3(256), 0, st, cls, hwp,
                       cnt);
    const int nblk = (total + 255) / 256;
    hipLaunchKernelGGL(k_head_loss, dim3(nblk), dim3(256), 0, st, n->d0, n->master + L.offw[7],
                       n->master + L.offb[7], target, cls, cnt, hwp, nb, n->g_d0, nullptr, n->part);
    hipLaunchKernelGGL(k_sum_loss, dim3(34), dim3(256), 0, st, n->part, nblk, loss, n->grad + L.offw[7]);
    int rc = last_status();
    // d0: input cat(up(d1), e0) at H
    if (!rc) rc = wgrad<64, 32, kUpCat, 32>(n->d1, n->e0, n->g_d0, n->part, n->bpart, GW(6), GB(6), nb, H, W, st);
    if (!rc) rc = conv<32, 64, kPlain, 0, true>(n->g_d0, nullptr, F_(6), nullptr, n->f_c0, nb, H, W, st);
    if (!rc) rc = route_up<32, 64>(n->f_c0, n->d1, n->g_d1, nb, H1, W1, st);
    // d1: input cat(up(d2), e1) at H/2
    if (!rc) rc = wgrad<128, 32, kUpCat, 64>(n->d2, n->e1, n->g_d1, n->part, n->bpart, GW(5), GB(5), nb, H1, W1, st);
    if (!rc) rc = conv<32, 128, kPlain, 0, true>(n->g_d1, nullptr, F_(5), nullptr, n->f_c1, nb, H1, W1, st);
    if (!rc) rc = route_up<64, 128>(n->f_c1, n->d2, n->g_d2, nb, H2, W2, st);
    // d2: input cat(up(e3), e2) at H/4
    if (!rc) rc = wgrad<256, 64, kUpCat, 128>(n->e3, n->e2, n->g_d2, n->part, n->bpart, GW(4), GB(4), nb, H2, W2, st);
    if (!rc) rc = conv<64, 256, kPlain, 0, true>(n->g_d2, nullptr, F_(4), nullptr, n->f_c2, nb, H2, W2, st);
    if (!rc) rc = route_up<128, 256>(n->f_c2, n->e3, n->g_e3, nb, H3, W3, st);
    // e3: input pool(e2) at H/8
    if (!rc) rc = wgrad<128, 128, kPool, 0>(n->e2, nullptr, n->g_e3, n->part, n->bpart, GW(3), GB(3), nb, H3, W3, st);
    if (!rc) rc = conv<128, 128, kPlain, 0, true>(n->g_e3, nullptr, F_(3), nullptr, n->f_p2, nb, H3, W3, st);
    if (!rc) rc = route_pool<128, 128, 256>(n->f_c2, n->f_p2, n->e2, n->g_e2, nb, H2, W2, st);
    // e2: input pool(e1) at H/4
    if (!rc) rc = wgrad<64, 128, kPool, 0>(n->e1, nullptr, n->g_e2, n->part, n->bpart, GW(2), GB(2), nb, H2, W2, st);
    if (!rc) rc = conv<128, 64, kPlain, 0, true>(n->g_e2, nullptr, F_(2), nullptr, n->f_p1, nb, H2, W2, st);
    if (!rc) rc = route_pool<64, 64, 128>(n->f_c1, n->f_p1, n->e1, n->g_e1, nb, H1, W1, st);
    // e1: input pool(e0) at H/2
    if (!rc) rc = wgrad<32, 64, kPool, 0>(n->e0, nullptr, n->g_e1, n->part, n->bpart, GW(1), GB(1), nb, H1, W1, st);
    if (!rc) rc = conv<64, 32, kPlain, 0, true>(n->g_e1, nullptr, F_(1), nullptr, n->f_p0, nb, H1, W1, st);
    if (!rc) rc = route_pool<32, 32, 64>(n->f_c0, n->f_p0, n->e0, n->g_e0, nb, H, W, st);
    // e0: input x (padded to 32 channels)
    if (!rc) rc = wgrad<32, 32, kIn4, 0>(n->xp, nullptr, n->g_e0, n->part, n->bpart, GW(0), GB(0), nb, H, W, st);
    return rc;
}

int net_adam(twg_unet *n, float lr, hipStream_t st)
{
    const double b1 = 0.9, b2 = 0.999;
    n->adam_t += 1;
    const float c1 = (float)(1.0 / (1.0 - std::pow(b1, n->adam_t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(b2, n->adam_t)));
    hipLaunchKernelGGL(k_adam, dim3((n->L.total_int + 255) / 256), dim3(256), 0, st, n->L, n->master, n->m, n->v,
                       n->grad, n->wt, n->wf, lr, (float)b1, (float)b2, 1e-8f, c1, c2);
    return last_status();
}

int net_params_in(twg_unet *n, const float *ext, hipStream_t st)
{
    hipLaunchKernelGGL(k_params_in, dim3((n->L.total_int + 255) / 256), dim3(256), 0, st, n->L, ext, n->master,
                       n->wt, n->wf);
    return last_status();
}

int net_params_out(twg_unet *n, float *ext, hipStream_t st)
{
    hipLaunchKernelGGL(k_params_out, dim3((n->L.total_int + 255) / 256), dim3(256), 0, st, n->L, n->master, ext);
    return last_status();
}

int net_grads_out(twg_unet *n, float *ext, hipStream_t st)
{
    hipLaunchKernelGGL(k_params_out, dim3((n->L.total_int + 255) / 256), dim3(256), 0, st, n->L, n->grad, ext);
    return last_status();
}

int net_pack_input(twg_unet *n, const float *x, long long total, hipStream_t st)
{
    hipLaunchKernelGGL(k_pack_input, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, x, n->xp, total);
    return last_status();
}

int net_head_plain(twg_unet *n, float *y, int total, hipStream_t st)
{
    hipLaunchKernelGGL(k_head_plain, dim3((total + 255) / 256), dim3(256), 0, st, n->d0, n->master + n->L.offw[7],
                       n->master + n->L.offb[7], y, total);
    return last_status();
}

int net_head_psi(twg_unet *n, const uint8_t *cls, float *psi, int nx, int ny, int pitch, int Wp, int32_t *status,
                 hipStream_t st)
{
    const dim3 grid((nx + 63) / 64, (ny + 3) / 4);
    hipLaunchKernelGGL(k_head_psi, grid, dim3(256), 0, st, n->d0, n->master + n->L.offw[7],
                       n->master + n->L.offb[7], cls, psi, nx, ny, pitch, Wp, n->words + 1);
    hipLaunchKernelGGL(k_net_fallback, grid, dim3(256), 0, st, cls, psi, nx, ny, pitch, n->words + 1, status);
    return last_status();
}

int net_features_coarse(const uint8_t *cls, const uint16_t *ring, int nx, int ny, int pitch, int f, int Hc, int Wc,
                        int gx, int gy, const unsigned int *jmax, float *xf, uint16_t *xp, uint8_t *ccls,
                        hipStream_t st)
{
    const float inv_diag = (float)(1.0 / ((double)std::max(nx, ny) * std::sqrt(2.0)));
    hipLaunchKernelGGL(k_features_coarse, dim3((Wc + 63) / 64, (Hc + 3) / 4), dim3(256), 0, st, cls, ring, nx, ny,
                       pitch, f, Hc, Wc, gx, gy, inv_diag, jmax, xf, xp, ccls);
    return last_status();
}

int net_coarse_target(const float *psi, const uint8_t *cls, int nx, int ny, int pitch, int f, int Hc, int Wc,
                      float *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_coarse_target, dim3((Wc + 63) / 64, (Hc + 3) / 4), dim3(256), 0, st, psi, cls, nx, ny,
                       pitch, f, Hc, Wc, out);
    return last_status();
}

int net_up_psi(twg_unet *n, const float *yc, int Hc, int Wc, int f, const uint8_t *cls, float *psi, int nx, int ny,
               int pitch, int32_t *status, hipStream_t st)
{
    const dim3 grid((nx + 63) / 64, (ny + 3) / 4);
    hipLaunchKernelGGL(k_up_psi, grid, dim3(256), 0, st, yc, Hc, Wc, f, cls, psi, nx, ny, pitch, n->words + 1);
    hipLaunchKernelGGL(k_net_fallback, grid, dim3(256), 0, st, cls, psi, nx, ny, pitch, n->words + 1, status);
    return last_status();
}

int net_zero_words(twg_unet *n, int count, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, n->words, count);
    return last_status();
}

int net_features(const uint8_t *cls, const uint16_t *ring, int nx, int ny, int pitch, int Hp, int Wp, int gx,
                 int gy, const unsigned int *jmax, float *xf, uint16_t *xp, hipStream_t st)
{
    const float inv_diag = (float)(1.0 / ((double)std::max(nx, ny) * std::sqrt(2.0)));
    hipLaunchKernelGGL(k_features, dim3((Wp + 63) / 64, (Hp + 3) / 4), dim3(256), 0, st, cls, ring, nx, ny, pitch,
                       Hp, Wp, gx, gy, inv_diag, jmax, xf, xp);
    return last_status();
}

int net_ring_max(const uint16_t *ring, int nx, int ny, int pitch, unsigned int *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_ring_max, dim3(std::min(ny, 512)), dim3(256), 0, st, ring, nx, ny, pitch, out);
    return last_status();
}


}  // namespace twg
