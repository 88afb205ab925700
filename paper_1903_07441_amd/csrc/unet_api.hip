// C ABI of the learned warm start: argument checks, buffer management and
// the sequencing of the network's kernels (unet.hip).
#include <algorithm>
#include <cstring>
#include <string>

#include "twg_internal.h"
#include "unet.h"

using namespace twg;

namespace {

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

size_t al(size_t v) { return (v + 255) & ~size_t(255); }

// Forward activations for P = batch * H * W pixels (bf16 NHWC).
int ensure_fwd(twg_unet *n, long long P)
{
    if (P <= n->fwd_pixels) return TWG_OK;
    if (n->fblock) {
        hipDeviceSynchronize();
        hipFree(n->fblock);
        n->fblock = nullptr;
        n->fwd_pixels = 0;
    }
    const size_t s32 = al((size_t)P * 32 * 2), s4 = al((size_t)P * 4 * 2), s1 = al((size_t)P / 4 * 2),
                 s2 = al((size_t)P / 16 * 2), s3 = al((size_t)P / 64 * 2);
    const size_t bytes = s4 + 2 * s32 + 64 * s1 + 32 * s1 + 128 * s2 + 64 * s2 + 128 * s3;
    if (hipMalloc(&n->fblock, bytes) != hipSuccess) {
        n->fblock = nullptr;
        return set_err(n->ctx, TWG_ENOMEM, "network activation allocation failed");
    }
    char *p = static_cast<char *>(n->fblock);
    auto take = [&](size_t b) { uint16_t *r = reinterpret_cast<uint16_t *>(p); p += b; return r; };
    n->xp = take(s4);
    n->e0 = take(s32);
    n->d0 = take(s32);
    n->e1 = take(64 * s1);
    n->d1 = take(32 * s1);
    n->e2 = take(128 * s2);
    n->d2 = take(64 * s2);
    n->e3 = take(128 * s3);
    n->fwd_pixels = P;
    return TWG_OK;
}

// Backward buffers for P pixels.
int ensure_bwd(twg_unet *n, long long P)
{
    if (P <= n->bwd_pixels) return TWG_OK;
    if (n->bblock) {
        hipDeviceSynchronize();
        hipFree(n->bblock);
        n->bblock = nullptr;
        n->bwd_pixels = 0;
    }
    const size_t P0 = (size_t)P, P1 = P0 / 4, P2 = P0 / 16, P3 = P0 / 64;
    // bf16 gradients, FP32 input gradients, split-K partial sums
    const size_t parts = std::max<size_t>((size_t)16384 * 9 * 128, 34 * ((P0 + 255) / 256));
    const size_t sizes[] = {al(P0 * 32 * 2), al(P1 * 32 * 2), al(P2 * 64 * 2), al(P3 * 128 * 2), al(P2 * 128 * 2),
                            al(P1 * 64 * 2), al(P0 * 32 * 2), al(P0 * 64 * 4), al(P1 * 128 * 4), al(P2 * 256 * 4),
                            al(P3 * 128 * 4), al(P2 * 64 * 4), al(P1 * 32 * 4), al(parts * 4),
                            al((size_t)512 * 128 * 4), al((size_t)65536 * 4)};
    size_t bytes = 0;
    for (size_t s : sizes) bytes += s;
    if (hipMalloc(&n->bblock, bytes) != hipSuccess) {
        n->bblock = nullptr;
        return set_err(n->ctx, TWG_ENOMEM, "network gradient allocation failed");
    }
    char *p = static_cast<char *>(n->bblock);
    int k = 0;
    auto take = [&]() { char *r = p; p += sizes[k++]; return r; };
    n->g_d0 = reinterpret_cast<uint16_t *>(take());
    n->g_d1 = reinterpret_cast<uint16_t *>(take());
    n->g_d2 = reinterpret_cast<uint16_t *>(take());
    n->g_e3 = reinterpret_cast<uint16_t *>(take());
    n->g_e2 = reinterpret_cast<uint16_t *>(take());
    n->g_e1 = reinterpret_cast<uint16_t *>(take());
    n->g_e0 = reinterpret_cast<uint16_t *>(take());
    n->f_c0 = reinterpret_cast<float *>(take());
    n->f_c1 = reinterpret_cast<float *>(take());
    n->f_c2 = reinterpret_cast<float *>(take());
    n->f_p2 = reinterpret_cast<float *>(take());
    n->f_p1 = reinterpret_cast<float *>(take());
    n->f_p0 = reinterpret_cast<float *>(take());
    n->part = reinterpret_cast<float *>(take());
    n->bpart = reinterpret_cast<float *>(take());
    n->counts = reinterpret_cast<unsigned int *>(take());
    n->bwd_pixels = P;
    return TWG_OK;
}

int check_shape(twg_unet *n, int batch, int H, int W)
{
    if (batch < 1 || batch > 65536) return set_err(n->ctx, TWG_EINVAL, "batch must be in [1, 65536]");
    if (H < 8 || W < 8 || H % 8 || W % 8 || H > 32768 || W > 32768)
        return set_err(n->ctx, TWG_EINVAL, "H and W must be multiples of 8 in [8, 32768]");
    if ((long long)batch * H * W > (1LL << 28))
        return set_err(n->ctx, TWG_EINVAL, "batch * H * W must not exceed 2^28 pixels");
    return TWG_OK;
}

}  // namespace

extern "C" {

int32_t twg_unet_num_params(void) { return net_layout().total_ext; }

int32_t twg_unet_create(twg_ctx *ctx, twg_unet **out)
{
    if (!ctx || !out) return TWG_EINVAL;
    *out = nullptr;
    ctx->err.clear();
    hipSetDevice(ctx->device);
    twg_unet *n = new twg_unet();
    n->ctx = ctx;
    n->L = net_layout();
    const size_t N = (size_t)n->L.total_int;
    const size_t bytes = al(N * 4) * 4 + al(N * 2) * 2 + 256;
    if (hipMalloc(&n->pblock, bytes) != hipSuccess) {
        delete n;
        return set_err(ctx, TWG_ENOMEM, "network parameter allocation failed");
    }
    char *p = static_cast<char *>(n->pblock);
    n->master = reinterpret_cast<float *>(p); p += al(N * 4);
    n->m = reinterpret_cast<float *>(p); p += al(N * 4);
    n->v = reinterpret_cast<float *>(p); p += al(N * 4);
    n->grad = reinterpret_cast<float *>(p); p += al(N * 4);
    n->wt = reinterpret_cast<uint16_t *>(p); p += al(N * 2);
    n->wf = reinterpret_cast<uint16_t *>(p); p += al(N * 2);
    n->words = reinterpret_cast<unsigned int *>(p);
    if (hipMemset(n->pblock, 0, bytes) != hipSuccess) {
        hipFree(n->pblock);
        delete n;
        return set_err(ctx, TWG_EDEVICE, "network parameter initialisation failed");
    }
    *out = n;
    return TWG_OK;
}

int32_t twg_unet_destroy(twg_unet *n)
{
    if (!n) return TWG_EINVAL;
    hipSetDevice(n->ctx->device);
    hipDeviceSynchronize();
    if (n->pblock) hipFree(n->pblock);
    if (n->fblock) hipFree(n->fblock);
    if (n->bblock) hipFree(n->bblock);
    if (n->yc) hipFree(n->yc);
    delete n;
    return TWG_OK;
}

int32_t twg_unet_set_params(twg_unet *n, const float *params, void *stream)
{
    if (!n) return TWG_EINVAL;
    n->ctx->err.clear();
    if (!params) return set_err(n->ctx, TWG_EINVAL, "params is required");
    hipSetDevice(n->ctx->device);
    hipStream_t st = as_stream(stream);
    const size_t N = (size_t)n->L.total_int;
    // zero the masters (padding stays zero), reset Adam, then scatter
    if (hipMemsetAsync(n->master, 0, N * 4, st) != hipSuccess || hipMemsetAsync(n->m, 0, N * 4, st) != hipSuccess ||
        hipMemsetAsync(n->v, 0, N * 4, st) != hipSuccess || hipMemsetAsync(n->wt, 0, N * 2, st) != hipSuccess ||
        hipMemsetAsync(n->wf, 0, N * 2, st) != hipSuccess)
        return set_err(n->ctx, TWG_EDEVICE, "parameter reset failed");
    n->adam_t = 0;
    const int rc = net_params_in(n, params, st);
    return rc ? set_err(n->ctx, rc, "parameter upload kernel failed") : TWG_OK;
}

int32_t twg_unet_get_params(twg_unet *n, float *params, void *stream)
{
    if (!n) return TWG_EINVAL;
    n->ctx->err.clear();
    if (!params) return set_err(n->ctx, TWG_EINVAL, "params is required");
    hipSetDevice(n->ctx->device);
    const int rc = net_params_out(n, params, as_stream(stream));
    return rc ? set_err(n->ctx, rc, "parameter download kernel failed") : TWG_OK;
}

int32_t twg_unet_forward(twg_unet *n, int32_t batch, int32_t H, int32_t W, const float *x, float *y, void *stream)
{
    if (!n) return TWG_EINVAL;
    n->ctx->err.clear();
    int rc = check_shape(n, batch, H, W);
    if (rc) return rc;
    if (!x || !y) return set_err(n->ctx, TWG_EINVAL, "x and y are required");
    hipSetDevice(n->ctx->device);
    hipStream_t st = as_stream(stream);
    const long long P = (long long)batch * H * W;
    rc = ensure_fwd(n, P);
    if (!rc) rc = net_pack_input(n, x, P, st);
    if (!rc) rc = net_forward(n, batch, H, W, st);
    if (!rc) rc = net_head_plain(n, y, (int)P, st);
    return rc ? set_err(n->ctx, rc, n->ctx->err.empty() ? "network forward failed" : n->ctx->err) : TWG_OK;
}

int32_t twg_unet_loss_grad(twg_unet *n, int32_t batch, int32_t H, int32_t W, const float *x, const float *target,
                           const uint8_t *cls, float *loss, float *grads, void *stream)
{
    if (!n) return TWG_EINVAL;
    n->ctx->err.clear();
    int rc = check_shape(n, batch, H, W);
    if (rc) return rc;
    if (!x || !target || !cls || !loss) return set_err(n->ctx, TWG_EINVAL, "x, target, cls and loss are required");
    if (batch > 65536) return set_err(n->ctx, TWG_EINVAL, "batch too large");
    hipSetDevice(n->ctx->device);
    hipStream_t st = as_stream(stream);
    const long long P = (long long)batch * H * W;
    rc = ensure_fwd(n, P);
    if (!rc) rc = ensure_bwd(n, P);
    if (!rc) rc = net_pack_input(n, x, P, st);
    if (!rc) rc = net_forward(n, batch, H, W, st);
    if (!rc) rc = net_backward(n, batch, H, W, target, cls, loss, st);
    if (!rc && grads) rc = net_grads_out(n, grads, st);
    return rc ? set_err(n->ctx, rc, n->ctx->err.empty() ? "network backward failed" : n->ctx->err) : TWG_OK;
}

int32_t twg_unet_adam_step(twg_unet *n, float lr, void *stream)
{
    if (!n) return TWG_EINVAL;
    n->ctx->err.clear();
    if (!(lr > 0.0f) || !(lr < 1.0f)) return set_err(n->ctx, TWG_EINVAL, "lr must be in (0, 1)");
    hipSetDevice(n->ctx->device);
    const int rc = net_adam(n, lr, as_stream(stream));
    return rc ? set_err(n->ctx, rc, "Adam kernel failed") : TWG_OK;
}

int32_t twg_unet_features(twg_unet *n, twg_grid g, const uint8_t *cls, const uint16_t *ring, int32_t goal_x,
                          int32_t goal_y, int32_t H, int32_t W, float *x, void *stream)
{
    if (!n) return TWG_EINVAL;
    n->ctx->err.clear();
    int rc = check_grid(n->ctx, g);
    if (rc) return rc;
    if (!cls || !x) return set_err(n->ctx, TWG_EINVAL, "cls and x are required");
    if (H < g.ny || W < g.nx || H % 8 || W % 8) return set_err(n->ctx, TWG_EINVAL, "frame must cover the grid, sides multiples of 8");
    hipSetDevice(n->ctx->device);
    hipStream_t st = as_stream(stream);
    rc = net_zero_words(n, 2, st);
    if (!rc && ring) rc = net_ring_max(ring, g.nx, g.ny, g.pitch, n->words, st);
    if (!rc) rc = net_features(cls, ring, g.nx, g.ny, g.pitch, H, W, goal_x, goal_y, n->words, x, nullptr, st);
    return rc ? set_err(n->ctx, rc, "feature kernel failed") : TWG_OK;
}

int32_t twg_unet_warm_start(twg_unet *n, twg_grid g, const uint8_t *cls, const uint16_t *ring, int32_t goal_x,
                            int32_t goal_y, float *psi, int32_t *status, void *stream)
{
    if (!n) return TWG_EINVAL;
    n->ctx->err.clear();
    int rc = check_grid(n->ctx, g);
    if (rc) return rc;
    if (!cls || !psi) return set_err(n->ctx, TWG_EINVAL, "cls and psi are required");
    const int Hp = (g.ny + 7) / 8 * 8, Wp = (g.nx + 7) / 8 * 8;
    rc = check_shape(n, 1, std::max(Hp, 8), std::max(Wp, 8));
    if (rc) return rc;
    hipSetDevice(n->ctx->device);
    hipStream_t st = as_stream(stream);
    const int H = std::max(Hp, 8), W = std::max(Wp, 8);
    rc = ensure_fwd(n, (long long)H * W);
    if (rc) return rc;
    rc = net_zero_words(n, 2, st);
    if (!rc && ring) rc = net_ring_max(ring, g.nx, g.ny, g.pitch, n->words, st);
    if (!rc) rc = net_features(cls, ring, g.nx, g.ny, g.pitch, H, W, goal_x, goal_y, n->words, nullptr, n->xp, st);
    if (!rc) rc = net_forward(n, 1, H, W, st);
    if (!rc) rc = net_head_psi(n, cls, psi, g.nx, g.ny, g.pitch, W, status, st);
    return rc ? set_err(n->ctx, rc, "warm start failed") : TWG_OK;
}

namespace {

// the coarse frame of a grid at 1/f: sides rounded up to multiples of 8
void coarse_frame(const twg_grid &g, int f, int *Hc, int *Wc)
{
    *Hc = std::max(8, ((g.ny + f - 1) / f + 7) / 8 * 8);
    *Wc = std::max(8, ((g.nx + f - 1) / f + 7) / 8 * 8);
}

bool coarse_factor_ok(int f) { return f == 2 || f == 4 || f == 8 || f == 16; }

}  // namespace

int32_t twg_unet_coarse_frame(twg_grid g, int32_t factor, int32_t *Hc, int32_t *Wc)
{
    if (!Hc || !Wc || !coarse_factor_ok(factor) || g.nx < 1 || g.ny < 1) return TWG_EINVAL;
    int h, w;
    coarse_frame(g, factor, &h, &w);
    *Hc = h;
    *Wc = w;
    return TWG_OK;
}

int32_t twg_unet_features_coarse(twg_unet *n, twg_grid g, const uint8_t *cls, const uint16_t *ring, int32_t goal_x,
                                 int32_t goal_y, int32_t factor, float *x, uint8_t *ccls, void *stream)
{
    if (!n) return TWG_EINVAL;
    n->ctx->err.clear();
    int rc = check_grid(n->ctx, g);
    if (rc) return rc;
    if (!cls || (!x && !ccls)) return set_err(n->ctx, TWG_EINVAL, "cls and x or ccls are required");
    if (!coarse_factor_ok(factor)) return set_err(n->ctx, TWG_EINVAL, "factor must be 2, 4, 8 or 16");
    int Hc, Wc;
    coarse_frame(g, factor, &Hc, &Wc);
    hipSetDevice(n->ctx->device);
    hipStream_t st = as_stream(stream);
    rc = net_zero_words(n, 2, st);
    if (!rc && ring) rc = net_ring_max(ring, g.nx, g.ny, g.pitch, n->words, st);
    if (!rc) rc = net_features_coarse(cls, ring, g.nx, g.ny, g.pitch, factor, Hc, Wc, goal_x, goal_y, n->words, x,
                                      nullptr, ccls, st);
    return rc ? set_err(n->ctx, rc, "coarse feature kernel failed") : TWG_OK;
}

int32_t twg_unet_coarse_target(twg_unet *n, twg_grid g, const uint8_t *cls, const float *psi, int32_t factor,
                               float *out, void *stream)
{
    if (!n) return TWG_EINVAL;
    n->ctx->err.clear();
    int rc = check_grid(n->ctx, g);
    if (rc) return rc;
    if (!cls || !psi || !out) return set_err(n->ctx, TWG_EINVAL, "cls, psi and out are required");
    if (!coarse_factor_ok(factor)) return set_err(n->ctx, TWG_EINVAL, "factor must be 2, 4, 8 or 16");
    int Hc, Wc;
    coarse_frame(g, factor, &Hc, &Wc);
    hipSetDevice(n->ctx->device);
    rc = net_coarse_target(psi, cls, g.nx, g.ny, g.pitch, factor, Hc, Wc, out, as_stream(stream));
    return rc ? set_err(n->ctx, rc, "coarse target kernel failed") : TWG_OK;
}

int32_t twg_unet_warm_start_coarse(twg_unet *n, twg_grid g, const uint8_t *cls, const uint16_t *ring,
                                   int32_t goal_x, int32_t goal_y, int32_t factor, float *psi, int32_t *status,
                                   void *stream)
{
    if (!n) return TWG_EINVAL;
    n->ctx->err.clear();
    int rc = check_grid(n->ctx, g);
    if (rc) return rc;
    if (!cls || !psi) return set_err(n->ctx, TWG_EINVAL, "cls and psi are required");
    if (!coarse_factor_ok(factor)) return set_err(n->ctx, TWG_EINVAL, "factor must be 2, 4, 8 or 16");
    int Hc, Wc;
    coarse_frame(g, factor, &Hc, &Wc);
    rc = check_shape(n, 1, Hc, Wc);
    if (rc) return rc;
    hipSetDevice(n->ctx->device);
    hipStream_t st = as_stream(stream);
    const long long P = (long long)Hc * Wc;
    rc = ensure_fwd(n, P);
    if (rc) return rc;
    if (P > n->yc_pixels) {
        if (n->yc) {
            hipDeviceSynchronize();
            hipFree(n->yc);
            n->yc = nullptr;
            n->yc_pixels = 0;
        }
        if (hipMalloc(&n->yc, (size_t)P * sizeof(float)) != hipSuccess) {
            n->yc = nullptr;
            return set_err(n->ctx, TWG_ENOMEM, "coarse output allocation failed");
        }
        n->yc_pixels = P;
    }
    rc = net_zero_words(n, 2, st);
    if (!rc && ring) rc = net_ring_max(ring, g.nx, g.ny, g.pitch, n->words, st);
    if (!rc) rc = net_features_coarse(cls, ring, g.nx, g.ny, g.pitch, factor, Hc, Wc, goal_x, goal_y, n->words,
                                      nullptr, n->xp, nullptr, st);
    if (!rc) rc = net_forward(n, 1, Hc, Wc, st);
    if (!rc) rc = net_head_plain(n, n->yc, (int)P, st);
    if (!rc) rc = net_up_psi(n, n->yc, Hc, Wc, factor, cls, psi, g.nx, g.ny, g.pitch, status, st);
    return rc ? set_err(n->ctx, rc, "coarse warm start failed") : TWG_OK;
}

}  // extern "C"
