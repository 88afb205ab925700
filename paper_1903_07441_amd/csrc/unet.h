// Internal state of the learned warm start (unet.hip, unet_api.hip).
#pragma once

#include "twg_internal.h"

namespace twg {

constexpr int kNetLayers = 8;  // e0 e1 e2 e3 d2 d1 d0 head

// Offsets of every layer's weights and bias in the internal parameter vector
// (weights [cout][k*k][cinp], cinp = cin padded to >= 32) and in the external
// one (per layer w[cout][cin][ky][kx], then b[cout]).
struct NetLayout {
    int cin[kNetLayers], cinp[kNetLayers], cout[kNetLayers], k[kNetLayers];
    int offw[kNetLayers], offb[kNetLayers];
    int extw[kNetLayers], extb[kNetLayers];
    int total_int, total_ext;
};

NetLayout net_layout();

}  // namespace twg

struct twg_unet {
    twg_ctx *ctx = nullptr;
    twg::NetLayout L;
    // parameters (internal layout): FP32 masters, Adam moments, gradients,
    // bf16 forward copy and bf16 flipped copy (input gradients)
    void *pblock = nullptr;
    float *master = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    uint16_t *wt = nullptr, *wf = nullptr;
    long long adam_t = 0;
    // forward activations (bf16 NHWC) for up to fwd_pixels = batch * H * W
    void *fblock = nullptr;
    long long fwd_pixels = 0;
    uint16_t *xp = nullptr, *e0 = nullptr, *e1 = nullptr, *e2 = nullptr, *e3 = nullptr;
    uint16_t *d2 = nullptr, *d1 = nullptr, *d0 = nullptr;
    // backward buffers for up to bwd_pixels
    void *bblock = nullptr;
    long long bwd_pixels = 0;
    uint16_t *g_d0 = nullptr, *g_d1 = nullptr, *g_d2 = nullptr, *g_e3 = nullptr, *g_e2 = nullptr,
             *g_e1 = nullptr, *g_e0 = nullptr;
    float *f_c0 = nullptr, *f_c1 = nullptr, *f_c2 = nullptr, *f_p2 = nullptr, *f_p1 = nullptr,
          *f_p0 = nullptr;
    float *part = nullptr, *bpart = nullptr;
    unsigned int *counts = nullptr;  // FREE cells per image
    // small device words: [0] ring maximum, [1] non-finite network output flag
    unsigned int *words = nullptr;
    // coarse output of a coarse-scale warm start (yc_pixels floats)
    float *yc = nullptr;
    long long yc_pixels = 0;
};

namespace twg {

int net_forward(twg_unet *n, int nb, int H, int W, hipStream_t st);
int net_backward(twg_unet *n, int nb, int H, int W, const float *target, const uint8_t *cls, float *loss,
                 hipStream_t st);
int net_adam(twg_unet *n, float lr, hipStream_t st);
int net_params_in(twg_unet *n, const float *ext, hipStream_t st);
int net_params_out(twg_unet *n, float *ext, hipStream_t st);
int net_grads_out(twg_unet *n, float *ext, hipStream_t st);
int net_pack_input(twg_unet *n, const float *x, long long total, hipStream_t st);
int net_head_plain(twg_unet *n, float *y, int total, hipStream_t st);
// the field of a warm start; a non-finite network output at a FREE cell
// makes every FREE cell 0.5 instead, and *status (if given) receives
// TWG_OK or TWG_NET_FALLBACK
int net_head_psi(twg_unet *n, const uint8_t *cls, float *psi, int nx, int ny, int pitch, int Wp, int32_t *status,
                 hipStream_t st);
// coarse-scale warm start: input channels (xf FP32 and/or xp bf16) and the
// training mask ccls of a grid seen at 1/f on an Hc x Wc frame; the coarse
// training target (mean of psi over each block's FREE cells); the fine field
// from a coarse output (bilinear, then the fallback of net_head_psi)
int net_features_coarse(const uint8_t *cls, const uint16_t *ring, int nx, int ny, int pitch, int f, int Hc, int Wc,
                        int gx, int gy, const unsigned int *jmax, float *xf, uint16_t *xp, uint8_t *ccls,
                        hipStream_t st);
int net_coarse_target(const float *psi, const uint8_t *cls, int nx, int ny, int pitch, int f, int Hc, int Wc,
                      float *out, hipStream_t st);
int net_up_psi(twg_unet *n, const float *yc, int Hc, int Wc, int f, const uint8_t *cls, float *psi, int nx, int ny,
               int pitch, int32_t *status, hipStream_t st);
// zero the first `count` (<= 64) words of n->words
int net_zero_words(twg_unet *n, int count, hipStream_t st);
int net_features(const uint8_t *cls, const uint16_t *ring, int nx, int ny, int pitch, int Hp, int Wp, int gx,
                 int gy, const unsigned int *jmax, float *xf, uint16_t *xp, hipStream_t st);
int net_ring_max(const uint16_t *ring, int nx, int ny, int pitch, unsigned int *out, hipStream_t st);

}  // namespace twg
