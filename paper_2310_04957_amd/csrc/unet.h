// unet.h -- the learned preconditioner: a 5-level, 32-channel convolutional
// U-net on the r-z node image (rows z, columns r; the last node row and
// column, always conductors in the supported geometries, are left out).
// Parameters are one flat FP32 vector in the order of the layer list below:
// for each 3x3 convolution w[9][cout][cin] (tap t = (dy+1)*3 + (dx+1)) then
// b[cout]; finally the 1x1 output w[32], b[1].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

namespace pic {
namespace unet {

struct bf16 {
    unsigned short x;
};

constexpr int kC = 32;             // channels of every 3x3 convolution
constexpr int kLevels = 5;
constexpr int kConvs = 18;         // enc1a..enc4b, mid5a/b, dec4a..dec1b
constexpr int kIn = 3;             // input channels: residual, susceptibility, mask
constexpr int kInPad = 16;         // input channels as stored (multiple of the MFMA k step)
constexpr int kWgradBlocks = 512;  // per-block partials of a weight gradient
constexpr int kLossBlocks = 256;
constexpr int kMaxBatch = 16;
constexpr int kLossLog = 1024;
constexpr int kHarvestBlocks = 1024;
constexpr int kHarvestPerSolve = 16;   // Krylov iterates kept per harvested solve
constexpr int kMaxPairs = 1 << 16;

// launchers (unet_kernels.hip)
void conv_fwd(int cin, const bf16* X, const bf16* Wt, const float* bias, bf16* Y, int B, int H, int W, hipStream_t s);
void conv_dgrad(int cin_of_layer, const bf16* D, const bf16* Yout, const bf16* Wb, bf16* DX, int B, int H, int W,
                hipStream_t s);
int conv_wgrad(int cin, const bf16* X, const bf16* D, const bf16* Yout, float* part, float* gw, int B, int H, int W,
               hipStream_t s);
void pool(const bf16* X, bf16* Y, int B, int H, int W, int C, hipStream_t s);
void pool_bwd_add(const bf16* dY, const bf16* dS, bf16* dX, int B, int H, int W, int C, hipStream_t s);
void up_concat(const bf16* Xc, const bf16* S, bf16* Y, int B, int H, int W, int C, hipStream_t s);
void up_concat_bwd(const bf16* dY, bf16* dXc, bf16* dS, int B, int H, int W, int C, hipStream_t s);
void out_fwd(const bf16* last, const float* w, const float* b0, float* out, int B, int HW, int C, hipStream_t s);
void loss_out_bwd(const float* out, const float* target, const float* mask, const bf16* last, const float* w,
                  bf16* dlast, float* part, float* sums, int B, int HW, int C, float inv_n, hipStream_t s);
void adam(float* p, const float* g, float* m, float* v, int n, float lr, int t, hipStream_t s);
void pack_conv(const float* w, int cin, int cin_pad, int cout, bf16* fwd, bf16* bwd, hipStream_t s);
void input_from_grid(const double* r, double scale, const double* chi, const int8_t* nk, bf16* X, int H, int W, int w,
                     hipStream_t s);
void input_from_f32(const float* in3, bf16* X, size_t npix, hipStream_t s);

struct Net;
void gather_batch(const Net& n, const int* idx, int B, hipStream_t s);
void input_from_r32(const Net& n, const float* r, const double* rr, const double* chi, const int8_t* nk, int w,
                    double n_free, hipStream_t s);
void out_to_z(const Net& n, const double* rr, const int8_t* nk, float* z, int w, int nn, hipStream_t s);
// harvest of the Krylov iterates of an FP64 MG-PCG solve: residual r of the
// approximation x + dx
void harvest_iter(const Net& n, int slot, const double* r, const double* x, const double* dx, const double* chi,
                  const int8_t* nk, double* xk, const int* done, int w, int nn, hipStream_t s);
// the mask image (1 on unknown nodes) of the handle's geometry
void mask_from_nodes(const Net& n, const int8_t* nk, int w, hipStream_t s);
// part: >= 2 kHarvestBlocks doubles of scratch
void pair_finish(const Net& n, int slot, const double* xs, const double* xk, const int8_t* nk, int w, double n_free,
                 double* part, hipStream_t s);

struct Conv {
    int cin, cin_pad;
    size_t woff, boff;      // offsets in the flat parameter vector
    bf16 *wf, *wb;          // packed forward / data-gradient weights
};

// Device state of the network, carved from the library workspace.
struct Net {
    int H, W, B, nparam;
    int Hl[kLevels], Wl[kLevels];
    Conv conv[kConvs];
    size_t out_w, out_b;
    float *p, *g, *m, *v;                         // FP32 master parameters, gradient, Adam moments
    bf16* x0;                                     // [B][H][W][16]
    bf16 *enc_a[4], *enc_b[4], *pooled[4], *mid_a, *mid_b, *cat[4], *dec_a[4], *dec_b[4];
    bf16 *g_enc_a[4], *g_enc_b[4], *g_skip[4], *g_pool[4], *g_mid_a, *g_cat[4], *g_dec_a[4], *g_up[4], *g_last;
    float *out, *target, *mask;                   // [B][H][W]
    float *part, *sums, *gtmp;                    // reduction scratch
    // harvested (residual, error) pairs on the image
    int cap_pairs;
    int64_t n_pairs;
    float *h_r, *h_e, *h_chi, *h_mask;
    float* loss_log;                              // [kLossLog] losses of the last training steps
    int adam_t;
};

size_t layout(Net& n, int H, int W, int B, int pairs, char* base);  // bytes; assigns when base != nullptr
void init_layers(Net& n);
void pack_all(Net& n, hipStream_t s);
void forward(Net& n, int B, hipStream_t s);
void backward(Net& n, int B, float inv_n, hipStream_t s);   // needs target, mask and a forward pass
void adam_update(Net& n, float lr, hipStream_t s);          // Adam on n.g, then repack the weights
void log_loss(Net& n, int k, hipStream_t s);                // loss_log[k] = last loss

}  // namespace unet
}  // namespace pic
