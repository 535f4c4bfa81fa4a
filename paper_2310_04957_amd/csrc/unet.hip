// unet.hip -- host orchestration of the learned preconditioner: buffer
// layout in the library workspace, forward and backward passes over the
// five levels, the MSE loss on normalised errors and Adam, all queued on
// the caller's stream (kernels in unet_kernels.hip).
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "unet.h"

namespace pic {
namespace unet {

namespace {
size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct Carve {
    char* base;
    size_t off = 0;
    template <typename T>
    T* take(size_t n) {
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += al(std::max<size_t>(n, 1) * sizeof(T));
        return p;
    }
};
}  // namespace

// layer table in the flat-parameter order
void init_layers(Net& n) {
    size_t off = 0;
    int k = 0;
    auto add = [&](int cin, int cin_pad) {
        Conv& c = n.conv[k++];
        c.cin = cin;
        c.cin_pad = cin_pad;
        c.woff = off;
        off += (size_t)9 * kC * cin;
        c.boff = off;
        off += kC;
    };
    add(kIn, kInPad);               // enc1a
    add(kC, kC);                    // enc1b
    for (int l = 2; l < kLevels; ++l) {
        add(kC, kC);
        add(kC, kC);
    }
    add(kC, kC);                    // mid a
    add(kC, kC);                    // mid b
    for (int l = kLevels - 1; l >= 1; --l) {
        add(2 * kC, 2 * kC);        // dec a (concat input)
        add(kC, kC);                // dec b
    }
    n.out_w = off;
    off += kC;
    n.out_b = off;
    off += 1;
    n.nparam = (int)off;
}

size_t layout(Net& n, int H, int W, int B, int pairs, char* base) {
    Carve c{base};
    n.H = H; n.W = W; n.B = B;
    for (int l = 0; l < kLevels; ++l) { n.Hl[l] = H >> l; n.Wl[l] = W >> l; }
    init_layers(n);
    n.p = c.take<float>(n.nparam); n.g = c.take<float>(n.nparam);
    n.m = c.take<float>(n.nparam); n.v = c.take<float>(n.nparam);
    for (int k = 0; k < kConvs; ++k) {
        n.conv[k].wf = c.take<bf16>((size_t)9 * kC * n.conv[k].cin_pad);
        n.conv[k].wb = c.take<bf16>((size_t)9 * kC * n.conv[k].cin);
    }
    auto px = [&](int l) { return (size_t)B * n.Hl[l] * n.Wl[l]; };
    n.x0 = c.take<bf16>(px(0) * kInPad);
    for (int l = 0; l < 4; ++l) {
        n.enc_a[l] = c.take<bf16>(px(l) * kC);
        n.enc_b[l] = c.take<bf16>(px(l) * kC);
        n.pooled[l] = c.take<bf16>(px(l + 1) * kC);
        n.cat[l] = c.take<bf16>(px(l) * 2 * kC);
        n.dec_a[l] = c.take<bf16>(px(l) * kC);
        n.dec_b[l] = c.take<bf16>(px(l) * kC);
        n.g_enc_a[l] = c.take<bf16>(px(l) * kC);
        n.g_enc_b[l] = c.take<bf16>(px(l) * kC);
        n.g_skip[l] = c.take<bf16>(px(l) * kC);
        n.g_pool[l] = c.take<bf16>(px(l + 1) * kC);
        n.g_cat[l] = c.take<bf16>(px(l) * 2 * kC);
        n.g_dec_a[l] = c.take<bf16>(px(l) * kC);
        n.g_up[l] = c.take<bf16>(px(l + 1) * kC);
    }
    n.mid_a = c.take<bf16>(px(4) * kC);
    n.mid_b = c.take<bf16>(px(4) * kC);
    n.g_mid_a = c.take<bf16>(px(4) * kC);
    n.g_last = c.take<bf16>(px(0) * kC);
    n.out = c.take<float>(px(0));
    n.target = c.take<float>(px(0));
    n.mask = c.take<float>(px(0));
    n.part = c.take<float>((size_t)kWgradBlocks * (9 * kC * 2 * kC + kC));
    n.sums = c.take<float>(64);
    n.gtmp = c.take<float>((size_t)9 * kC * kInPad + kC);
    n.cap_pairs = pairs;
    const size_t img = (size_t)H * W;
    n.h_r = c.take<float>(img * std::max(pairs, 1));
    n.h_e = c.take<float>(img * std::max(pairs, 1));
    n.h_chi = c.take<float>(img * std::max(pairs, 1));
    n.h_mask = c.take<float>(img);
    n.loss_log = c.take<float>(kLossLog);
    return c.off;
}

void pack_all(Net& n, hipStream_t s) {
    for (int k = 0; k < kConvs; ++k) {
        Conv& c = n.conv[k];
        pack_conv(n.p + c.woff, c.cin, c.cin_pad, kC, c.wf, k == 0 ? nullptr : c.wb, s);
    }
}

void forward(Net& n, int B, hipStream_t s) {
    const bf16* h = n.x0;
    int ci = 0;
    for (int l = 0; l < 4; ++l) {
        const int H = n.Hl[l], W = n.Wl[l];
        Conv& a = n.conv[ci++];
        Conv& b = n.conv[ci++];
        conv_fwd(a.cin_pad, h, a.wf, n.p + a.boff, n.enc_a[l], B, H, W, s);
        conv_fwd(kC, n.enc_a[l], b.wf, n.p + b.boff, n.enc_b[l], B, H, W, s);
        pool(n.enc_b[l], n.pooled[l], B, H, W, kC, s);
        h = n.pooled[l];
    }
    {
        Conv& a = n.conv[ci++];
        Conv& b = n.conv[ci++];
        conv_fwd(kC, n.pooled[3], a.wf, n.p + a.boff, n.mid_a, B, n.Hl[4], n.Wl[4], s);
        conv_fwd(kC, n.mid_a, b.wf, n.p + b.boff, n.mid_b, B, n.Hl[4], n.Wl[4], s);
        h = n.mid_b;
    }
    for (int l = 3; l >= 0; --l) {
        const int H = n.Hl[l], W = n.Wl[l];
        Conv& a = n.conv[ci++];
        Conv& b = n.conv[ci++];
        up_concat(h, n.enc_b[l], n.cat[l], B, H, W, kC, s);
        conv_fwd(2 * kC, n.cat[l], a.wf, n.p + a.boff, n.dec_a[l], B, H, W, s);
        conv_fwd(kC, n.dec_a[l], b.wf, n.p + b.boff, n.dec_b[l], B, H, W, s);
        h = n.dec_b[l];
    }
    out_fwd(n.dec_b[0], n.p + n.out_w, n.p + n.out_b, n.out, B, n.H * n.W, kC, s);
}

__global__ void k_extract_first(const float* full, float* g, int cin, int cin_pad) {
    // the first layer's gradient over 16 padded channels -> its 3 real ones
    for (int e = threadIdx.x; e < 9 * kC * cin; e += blockDim.x) {
        const int c = e % cin, tn = e / cin;
        g[e] = full[tn * cin_pad + c];
    }
    for (int e = threadIdx.x; e < kC; e += blockDim.x) g[9 * kC * cin + e] = full[9 * kC * cin_pad + e];
}

__global__ void k_copy_out_grads(const float* sums, float* gw, float* gb, int C) {
    for (int c = threadIdx.x; c < C; c += blockDim.x) gw[c] = sums[2 + c];
    if (threadIdx.x == 0) gb[0] = sums[1];
}

// gradients of the loss of the last forward pass with respect to all
// parameters (target and mask already in place); n.sums[0] holds the loss
void backward(Net& n, int B, float inv_n, hipStream_t s) {
    const int HW = n.H * n.W;
    loss_out_bwd(n.out, n.target, n.mask, n.dec_b[0], n.p + n.out_w, n.g_last, n.part, n.sums, B, HW, kC, inv_n, s);
    hipLaunchKernelGGL(k_copy_out_grads, dim3(1), dim3(64), 0, s, (const float*)n.sums, n.g + n.out_w,
                       n.g + n.out_b, kC);
    const bf16* gh = n.g_last;
    int ci = kConvs - 1;
    for (int l = 0; l < 4; ++l) {
        const int H = n.Hl[l], W = n.Wl[l];
        Conv& b = n.conv[ci--];
        Conv& a = n.conv[ci--];
        conv_wgrad(kC, n.dec_a[l], gh, n.dec_b[l], n.part, n.g + b.woff, B, H, W, s);
        conv_dgrad(kC, gh, n.dec_b[l], b.wb, n.g_dec_a[l], B, H, W, s);
        conv_wgrad(2 * kC, n.cat[l], n.g_dec_a[l], n.dec_a[l], n.part, n.g + a.woff, B, H, W, s);
        conv_dgrad(2 * kC, n.g_dec_a[l], n.dec_a[l], a.wb, n.g_cat[l], B, H, W, s);
        up_concat_bwd(n.g_cat[l], n.g_up[l], n.g_skip[l], B, H, W, kC, s);
        gh = n.g_up[l];
    }
    {
        const int H = n.Hl[4], W = n.Wl[4];
        Conv& b = n.conv[ci--];
        Conv& a = n.conv[ci--];
        conv_wgrad(kC, n.mid_a, gh, n.mid_b, n.part, n.g + b.woff, B, H, W, s);
        conv_dgrad(kC, gh, n.mid_b, b.wb, n.g_mid_a, B, H, W, s);
        conv_wgrad(kC, n.pooled[3], n.g_mid_a, n.mid_a, n.part, n.g + a.woff, B, H, W, s);
        conv_dgrad(kC, n.g_mid_a, n.mid_a, a.wb, n.g_pool[3], B, H, W, s);
    }
    for (int l = 3; l >= 0; --l) {
        const int H = n.Hl[l], W = n.Wl[l];
        Conv& b = n.conv[ci--];
        Conv& a = n.conv[ci--];
        pool_bwd_add(n.g_pool[l], n.g_skip[l], n.g_enc_b[l], B, H, W, kC, s);
        conv_wgrad(kC, n.enc_a[l], n.g_enc_b[l], n.enc_b[l], n.part, n.g + b.woff, B, H, W, s);
        conv_dgrad(kC, n.g_enc_b[l], n.enc_b[l], b.wb, n.g_enc_a[l], B, H, W, s);
        if (l > 0) {
            conv_wgrad(kC, n.pooled[l - 1], n.g_enc_a[l], n.enc_a[l], n.part, n.g + a.woff, B, H, W, s);
            conv_dgrad(kC, n.g_enc_a[l], n.enc_a[l], a.wb, n.g_pool[l - 1], B, H, W, s);
        } else {
            conv_wgrad(kInPad, n.x0, n.g_enc_a[0], n.enc_a[0], n.part, n.gtmp, B, H, W, s);
            hipLaunchKernelGGL(k_extract_first, dim3(1), dim3(256), 0, s, (const float*)n.gtmp, n.g + a.woff, kIn,
                               kInPad);
        }
    }
}

void adam_update(Net& n, float lr, hipStream_t s) {
    n.adam_t += 1;
    adam(n.p, n.g, n.m, n.v, n.nparam, lr, n.adam_t, s);
    pack_all(n, s);
}

__global__ void k_log_loss(const float* sums, float* log, int k) { log[k] = sums[0]; }

void log_loss(Net& n, int k, hipStream_t s) {
    hipLaunchKernelGGL(k_log_loss, dim3(1), dim3(1), 0, s, (const float*)n.sums, n.loss_log, k);
}

}  // namespace unet
}  // namespace pic
