// unet_kernels.hip -- kernels of the learned preconditioner: a 5-level
// convolutional U-net on the r-z node image (rows z, columns r) that
// approximates the inverse of the finite-volume operator of Eq. (1) on a
// normalised residual.  Activations are NHWC bfloat16; 3x3 convolutions run
// as implicit GEMMs on gfx950 BF16 matrix cores (v_mfma_f32_32x32x16_bf16)
// with FP32 accumulation; master weights and the Adam state are FP32.
#include <hip/hip_runtime.h>

#include "unet.h"

namespace pic {
namespace unet {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));   // 8 bf16 moved as raw bits
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float bf2f(bf16 v) {
    return __uint_as_float(((unsigned)v.x) << 16);
}
__device__ __forceinline__ float bf2f(__bf16 v) {
    return __uint_as_float(((unsigned)__builtin_bit_cast(unsigned short, v)) << 16);
}
__device__ __forceinline__ bf16 f2bf(float f) {
    // round to nearest even: one hardware conversion on gfx950
    bf16 r;
    r.x = __builtin_bit_cast(unsigned short, (__bf16)f);
    return r;
}
__device__ __forceinline__ __bf16 f2raw(float f) { return __builtin_bit_cast(__bf16, f2bf(f).x); }
__device__ __forceinline__ __bf16 raw(bf16 v) { return __builtin_bit_cast(__bf16, v.x); }

// ------------------------------------------------------------- 3x3 conv
// Y[b][y][x][n] = act(bias[n] + sum_t sum_c Wt[t][n][c] * Xin[b][y+dy_t][x+dx_t][c])
// with zero padding, Xin = X (optionally multiplied by the ReLU mask
// M > 0 of the layer whose gradient X is).  Tile: 16x16 output pixels per
// block iteration, 4 wavefronts x 4 rows; each wavefront computes two
// 32-pixel x 32-channel MFMA tiles per 32 output channels.  The input
// channels are staged in LDS 32 (or all, if fewer) at a time with the
// tile's halo; the weights of all taps and channels stay in LDS for the
// whole launch.  The next chunk's input is loaded into registers while the
// current one is multiplied out of LDS.  Each thread's place in the staged
// halo tile is fixed, so its load offsets are computed once per launch.
template <int CIN>
struct Stage {
    static constexpr int CH = CIN < 32 ? CIN : 32;   // channels per staged chunk
    static constexpr int NCH = CIN / CH;             // chunks per tile
    static constexpr int G = CH / 8;                 // 8-channel groups per pixel of a chunk
    static constexpr int N = 18 * 18 * G;            // groups of one staged halo tile
    static constexpr int Q = (N + 255) / 256;        // groups per thread
};

template <int CIN>
struct LoadPlan {
    int py[Stage<CIN>::Q], px[Stage<CIN>::Q], c8[Stage<CIN>::Q];
};

template <int CIN>
__device__ __forceinline__ void make_plan(int tid, LoadPlan<CIN>& lp) {
    using S = Stage<CIN>;
#pragma unroll
    for (int q = 0; q < S::Q; ++q) {
        const int e = tid + q * 256;
        const int pix = e / S::G;
        lp.c8[q] = e % S::G;
        lp.py[q] = e < S::N ? pix / 18 : -1000000;   // an idle group is never in the image
        lp.px[q] = pix % 18;
    }
}

// keep each of the eight bf16 in t whose mask value in m is > 0 (the mask is
// a ReLU output: never NaN)
__device__ __forceinline__ void relu_mask(u32x4& t, const u32x4 m) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const unsigned lo = (m[k] << 16), hi = (m[k] & 0xffff0000u);
        const unsigned keep = (__uint_as_float(lo) > 0.0f ? 0x0000ffffu : 0u) |
                              (__uint_as_float(hi) > 0.0f ? 0xffff0000u : 0u);
        t[k] &= keep;
    }
}

// chunk ch of the halo tile at (b, y0 - 1, x0 - 1) into registers, as raw
// bits (a bf16 vector type here costs a repacking per element on the way
// to LDS)
template <int CIN, bool MASK>
__device__ __forceinline__ void load_chunk(const bf16* __restrict__ X, const bf16* __restrict__ M,
                                           const LoadPlan<CIN>& lp, int b, int y0, int x0, int ch, int H, int W,
                                           u32x4* v) {
    using S = Stage<CIN>;
#pragma unroll
    for (int q = 0; q < S::Q; ++q) {
        const int yy = y0 - 1 + lp.py[q], xx = x0 - 1 + lp.px[q];
        u32x4 t = {0u, 0u, 0u, 0u};
        if (yy >= 0 && yy < H && xx >= 0 && xx < W) {
            const size_t g = (((size_t)b * H + yy) * W + xx) * CIN + ch * S::CH + lp.c8[q] * 8;
            t = *(const u32x4*)&X[g];
            if (MASK) relu_mask(t, *(const u32x4*)&M[g]);
        }
        v[q] = t;
    }
}

template <int CIN, int COUT, bool RELU, bool MASK>
__global__ __launch_bounds__(256) void k_conv3x3(const bf16* __restrict__ X, const bf16* __restrict__ Wt,
                                                 const float* __restrict__ bias, const bf16* __restrict__ M,
                                                 bf16* __restrict__ Y, int B, int H, int W) {
    using S = Stage<CIN>;
    constexpr int CP = S::CH + 8;         // padded channel stride of the staged chunk (bank spread)
    constexpr int CW = CIN + 8;           // padded channel stride of the weights
    constexpr int NT = COUT / 32;
    __shared__ __attribute__((aligned(16))) bf16 xs[18 * 18 * CP];
    __shared__ __attribute__((aligned(16))) bf16 ws[9 * COUT * CW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // weights once per block
    for (int e = tid; e < 9 * COUT * (CIN / 8); e += 256) {
        const int c8 = e % (CIN / 8), tn = e / (CIN / 8);
        *(u32x4*)&ws[tn * CW + c8 * 8] = *(const u32x4*)&Wt[(size_t)tn * CIN + c8 * 8];
    }
    LoadPlan<CIN> lp;
    make_plan<CIN>(tid, lp);
    const int kh = (lane >> 5) * 8;      // this lane's 8 channels of a 16-wide k step
    const int m = lane & 31;             // this lane's pixel row of the A tile / output channel of B
    // this lane's bias values, once per launch (a load inside the epilogue
    // makes every store there wait for all earlier memory operations)
    float bb[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) bb[nt] = bias ? bias[nt * 32 + m] : 0.0f;
    const int tx = (W + 15) / 16, ty = (H + 15) / 16;
    // tile indices fit in 32 bits (images of at most 2^31 16x16 tiles)
    const unsigned txy = (unsigned)(tx * ty), utx = (unsigned)tx, nti = (unsigned)((long long)tx * ty * B);
    u32x4 next[S::Q];
    // the staged chunk in registers into LDS, between barriers (every
    // wavefront's MFMAs are done with the previous chunk)
    auto stage = [&]() {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < S::Q; ++q)
            if (lp.py[q] >= 0) *(u32x4*)&xs[(lp.py[q] * 18 + lp.px[q]) * CP + lp.c8[q] * 8] = next[q];
        __syncthreads();
    };
    if (blockIdx.x < nti) {
        const unsigned tile = blockIdx.x;
        const int b = (int)(tile / txy);
        const unsigned rem = tile % txy;
        load_chunk<CIN, MASK>(X, M, lp, b, (int)(rem / utx) * 16, (int)(rem % utx) * 16, 0, H, W, next);
        stage();
    }
    for (unsigned tile = blockIdx.x; tile < nti; tile += gridDim.x) {
        const int b = (int)(tile / txy);
        const unsigned rem = tile % txy;
        const int y0 = (int)(rem / utx) * 16, x0 = (int)(rem % utx) * 16;
        f32x16 acc[2][NT];
        for (int s = 0; s < 2; ++s)
            for (int nt = 0; nt < NT; ++nt) acc[s][nt] = {};
#pragma unroll
        for (int ch = 0; ch < S::NCH; ++ch) {
            if (ch > 0) stage();   // the first chunk is staged before the loop or the previous epilogue
            // the next chunk of this tile, else the first of the next tile
            if (ch + 1 < S::NCH) {
                load_chunk<CIN, MASK>(X, M, lp, b, y0, x0, ch + 1, H, W, next);
            } else {
                const unsigned nt2 = tile + gridDim.x;
                if (nt2 < nti) {
                    const int b2 = (int)(nt2 / txy);
                    const unsigned rem2 = nt2 % txy;
                    load_chunk<CIN, MASK>(X, M, lp, b2, (int)(rem2 / utx) * 16, (int)(rem2 % utx) * 16, 0, H, W,
                                          next);
                }
            }
            // steps k = (tap, 16-channel slice); the fragments of step k + 1
            // are read from LDS before the MFMAs of step k are issued (the
            // scheduling barriers keep that order)
            constexpr int KS = S::CH / 16, NK = 9 * KS;
            auto frag = [&](int k, bf16x8* a, bf16x8* bq) {
                const int t = k / KS, c0 = (k % KS) * 16;
                const int dy = t / 3, dx = t % 3;   // halo coordinates: +1 offsets folded in
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    bq[nt] = *(const bf16x8*)&ws[(t * COUT + nt * 32 + m) * CW + ch * S::CH + c0 + kh];
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const int py = wave * 4 + s * 2 + m / 16, px = m % 16;
                    a[s] = *(const bf16x8*)&xs[((py + dy) * 18 + (px + dx)) * CP + c0 + kh];
                }
            };
            bf16x8 afr[2][2], bfr[2][NT];
            frag(0, afr[0], bfr[0]);
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                if (k + 1 < NK) frag(k + 1, afr[(k + 1) & 1], bfr[(k + 1) & 1]);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int s = 0; s < 2; ++s)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        acc[s][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(afr[k & 1][s], bfr[k & 1][nt],
                                                                              acc[s][nt], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // the next tile's first chunk goes to LDS before this tile's results
        // are stored: the wait for its loads then waits for no store
        if (tile + gridDim.x < nti) stage();
        // D layout: lane holds column n = lane % 32, rows pm = 8(r/4) +
        // 4(lane/32) + r%4, i.e. tile row pm/16 = (r >= 8) and column
        // pm % 16 = 8((r/4) & 1) + 4(lane/32) + r%4.  One base address per
        // lane and compile-time offsets; interior tiles store without any
        // check (one branch for the whole tile), edge tiles check each
        // value; bf16 by the hardware's round-to-nearest-even conversion.
        const bool full = y0 + 16 <= H && x0 + 16 <= W;
        const int cx = 4 * (lane >> 5);
        const size_t row = (size_t)W * COUT;
        auto out = [&](int s, int nt, int r) {
            float v = acc[s][nt][r] + bb[nt];
            if (RELU) v = fmaxf(v, 0.0f);
            return __builtin_bit_cast(unsigned short, (__bf16)v);
        };
        if (full) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                unsigned short* const Yb = reinterpret_cast<unsigned short*>(Y) +
                                           (((size_t)b * H + y0 + wave * 4 + s * 2) * W + x0 + cx) * COUT + m;
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int dy = r >= 8 ? 1 : 0, dx = 8 * ((r / 4) & 1) + (r % 4);
                        Yb[dy * row + dx * COUT + nt * 32] = out(s, nt, r);
                    }
            }
        } else {
            for (int s = 0; s < 2; ++s) {
                const int py0 = y0 + wave * 4 + s * 2;
                unsigned short* const Yb = reinterpret_cast<unsigned short*>(Y) +
                                           (((size_t)b * H + py0) * W + x0 + cx) * COUT + m;
                for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int dy = r >= 8 ? 1 : 0, dx = 8 * ((r / 4) & 1) + (r % 4);
                        if (py0 + dy < H && x0 + cx + dx < W) Yb[dy * row + dx * COUT + nt * 32] = out(s, nt, r);
                    }
            }
        }
    }
}

// ------------------------------------------------------- weight gradient
// dW[t][n][c] = sum_p Dm[p][n] * Xpad[p + off_t][c] and db[n] = sum_p Dm[p][n],
// Dm = D * (Yout > 0).  Per 16x16 tile and tap a GEMM with M = 32 output
// channels, N = the input channels (padded to whole 32-channel tiles) and
// K = the tile's 256 pixels.  Dm and the halo tile of X are staged
// transposed in LDS (channel-major, two pixels per 32-bit word); the halo
// rows are padded to 24 pixels, so that for one tile row and one tap row dy
// a 16-byte and a 4-byte read give the B fragments of all three dx (dx = 1
// by a 16-bit funnel shift).  Wavefront w takes all nine taps over the tile
// rows w, w + 4, ... (with 64 input channels: channel tile w & 1 over the
// rows w/2, w/2 + 2, ...).  At the end the wavefronts' sums are added in LDS
// in a fixed order and each block writes one partial, reduced later in a
// fixed order.
__device__ __forceinline__ float bf_lo(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf_hi(unsigned w) { return __uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

template <int CIN>
__global__ __launch_bounds__(256) void k_wgrad(const bf16* __restrict__ X, const bf16* __restrict__ D,
                                               const bf16* __restrict__ Yout, float* __restrict__ part, int B, int H,
                                               int W) {
    constexpr int NT = (CIN + 31) / 32;
    constexpr int CT = NT * 32;            // channels padded to whole N tiles
    constexpr int DS = 256 + 8;            // dT[n][pixel], pixel = 16 row + column
    constexpr int HR = 24;                 // padded halo row
    constexpr int XS = 18 * HR + 8;        // xT[c][halo row][halo column]
    constexpr int RS = 4 / NT;             // tile-row stride of a wavefront
    constexpr int NX = 18 * 9 * (CT / 8);  // X staging tasks: (halo row, column pair, 8-channel group)
    constexpr int QX = (NX + 255) / 256;
    constexpr int kStage = 32 * DS * 2 + CT * XS * 2;
    constexpr int kRed = 9 * 32 * CT * 4;
    __shared__ __attribute__((aligned(16))) unsigned char smem[kStage > kRed ? kStage : kRed];
    __shared__ float dbred[4][16];
    bf16* const dT = reinterpret_cast<bf16*>(smem);
    bf16* const xT = dT + 32 * DS;
    float* const red = reinterpret_cast<float*>(smem);   // after the last tile
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 31, kh = (lane >> 5) * 8;
    const int nt = NT == 1 ? 0 : (wave & 1);
    const int row0 = NT == 1 ? wave : (wave >> 1);
    f32x16 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = {};
    // this thread's pixel pair (tile row prow, columns pcol, pcol + 1) and
    // 16 channels of Dm, and its share of db
    const int pp = tid & 127, dh = tid >> 7;
    const int prow = pp >> 3, pcol = (pp & 7) * 2;
    float dbp[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) dbp[j] = 0.0f;
    const int tx = (W + 15) / 16, ty = (H + 15) / 16;
    const long long ntile = (long long)tx * ty * B;
    for (long long tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const int b = (int)(tile / (tx * ty));
        const int rem = (int)(tile % (tx * ty));
        const int y0 = (rem / tx) * 16, x0 = (rem % tx) * 16;
        u32x4 dv[2][2], xv[QX][2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int py = y0 + prow, px = x0 + pcol + k;
            dv[k][0] = dv[k][1] = u32x4{0u, 0u, 0u, 0u};
            if (py < H && px < W) {
                const size_t g = (((size_t)b * H + py) * W + px) * 32 + dh * 16;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    dv[k][h] = *(const u32x4*)&D[g + 8 * h];
                    relu_mask(dv[k][h], *(const u32x4*)&Yout[g + 8 * h]);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < QX; ++q) {
            const int e = tid + 256 * q;
            const int g8 = e % (CT / 8), cp = (e / (CT / 8)) % 9, hy = e / (CT / 8) / 9;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int yy = y0 - 1 + hy, xx = x0 - 1 + 2 * cp + k;
                xv[q][k] = u32x4{0u, 0u, 0u, 0u};
                if (e < NX && g8 * 8 < CIN && yy >= 0 && yy < H && xx >= 0 && xx < W)
                    xv[q][k] = *(const u32x4*)&X[(((size_t)b * H + yy) * W + xx) * CIN + g8 * 8];
            }
        }
        __syncthreads();   // every wavefront is done with the previous tile's fragments
        // word (channel, pixel pair): the first pixel in the low half
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const unsigned a = dv[0][h][i], c = dv[1][h][i];
                const int j = h * 8 + 2 * i, n0 = dh * 16 + j;
                *(unsigned*)&dT[n0 * DS + prow * 16 + pcol] = (a & 0xffffu) | (c << 16);
                *(unsigned*)&dT[(n0 + 1) * DS + prow * 16 + pcol] = (a >> 16) | (c & 0xffff0000u);
                dbp[j] += bf_lo(a) + bf_lo(c);
                dbp[j + 1] += bf_hi(a) + bf_hi(c);
            }
#pragma unroll
        for (int q = 0; q < QX; ++q) {
            const int e = tid + 256 * q;
            if (e < NX) {
                const int g8 = e % (CT / 8), cp = (e / (CT / 8)) % 9, hy = e / (CT / 8) / 9;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const unsigned a = xv[q][0][i], c = xv[q][1][i];
                    const int c0 = g8 * 8 + 2 * i;
                    *(unsigned*)&xT[c0 * XS + hy * HR + 2 * cp] = (a & 0xffffu) | (c << 16);
                    *(unsigned*)&xT[(c0 + 1) * XS + hy * HR + 2 * cp] = (a >> 16) | (c & 0xffff0000u);
                }
            }
        }
        __syncthreads();
#pragma unroll 1
        for (int r = 0; r < 16 / RS; ++r) {
            const int ks = row0 + r * RS;   // tile row = k step of 16 pixels
            const bf16x8 afr = as_bf16x8(*(const u32x4*)&dT[m * DS + ks * 16 + kh]);
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) {
                const bf16* src = &xT[(nt * 32 + m) * XS + (ks + dy) * HR + kh];
                const u32x4 v = *(const u32x4*)src;
                const unsigned v4 = *(const unsigned*)(src + 8);
                const u32x4 s1 = {__builtin_amdgcn_alignbit(v[1], v[0], 16), __builtin_amdgcn_alignbit(v[2], v[1], 16),
                                  __builtin_amdgcn_alignbit(v[3], v[2], 16), __builtin_amdgcn_alignbit(v4, v[3], 16)};
                const u32x4 s2 = {v[1], v[2], v[3], v4};
                acc[dy * 3 + 0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(afr, as_bf16x8(v), acc[dy * 3 + 0], 0, 0, 0);
                acc[dy * 3 + 1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(afr, as_bf16x8(s1), acc[dy * 3 + 1], 0, 0, 0);
                acc[dy * 3 + 2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(afr, as_bf16x8(s2), acc[dy * 3 + 2], 0, 0, 0);
            }
        }
    }
    // the wavefronts' sums: the buffer cleared, then each wavefront adds its
    // own, one wavefront at a time in wavefront order (a fixed order; the
    // LDS atomic takes the accumulators as they are).  D layout: lane holds
    // input channel nt 32 + lane % 32, output channels 8(r/4) + 4(lane/32) +
    // r%4
    __syncthreads();
    for (int e = tid; e < 9 * 32 * CT; e += 256) red[e] = 0.0f;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        __syncthreads();
        if (wave == w) {
#pragma unroll
            for (int t = 0; t < 9; ++t)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int n = 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
                    atomicAdd(&red[(t * 32 + n) * CT + nt * 32 + m], acc[t][r]);
                }
        }
    }
    // db: over the 64 lanes of a wavefront, then the two wavefronts of a
    // channel half
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        float v = dbp[j];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) dbred[wave][j] = v;
    }
    __syncthreads();
    // partial layout per block: [9][32][CIN] weights then [32] bias
    float* const out = part + (size_t)blockIdx.x * (9 * 32 * CIN + 32);
    for (int e = tid; e < 9 * 32 * CIN; e += 256) out[e] = red[(e / CIN) * CT + e % CIN];
    if (tid < 32) out[9 * 32 * CIN + tid] = dbred[2 * (tid >> 4)][tid & 15] + dbred[2 * (tid >> 4) + 1][tid & 15];
}

// sum of per-block partials in a fixed order: the 8 thread groups of a block
// add the partials k, k + 8, ... of 32 consecutive elements, then the 8 sums
// are added in order
__global__ __launch_bounds__(256) void k_sum_parts(const float* part, int nblk, int len, float* out) {
    __shared__ float sh[256];
    const int k = threadIdx.x >> 5, i = blockIdx.x * 32 + (threadIdx.x & 31);
    float s = 0.0f;
    if (i < len)
        for (int b = k; b < nblk; b += 8) s += part[(size_t)b * len + i];
    sh[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < 32 && i < len) {
        float t = 0.0f;
        for (int j = 0; j < 8; ++j) t += sh[j * 32 + threadIdx.x];
        out[i] = t;
    }
}

static void sum_parts(const float* part, int nblk, int len, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_parts, dim3((len + 31) / 32), dim3(256), 0, s, part, nblk, len, out);
}

// ---------------------------------------------- pooling, upsampling, concat
// All four move whole 8-channel groups (16 bytes) per thread; C is a
// multiple of 8.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void unpack8(u32x4 v, float* f) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        f[2 * k] = __uint_as_float(v[k] << 16);
        f[2 * k + 1] = __uint_as_float(v[k] & 0xFFFF0000u);
    }
}
__device__ __forceinline__ u32x4 pack8(const float* f) {
    u32x4 v;
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (unsigned)f2bf(f[2 * k]).x | ((unsigned)f2bf(f[2 * k + 1]).x << 16);
    return v;
}
__device__ __forceinline__ u32x4 ld8(const bf16* p) { return *reinterpret_cast<const u32x4*>(p); }
__device__ __forceinline__ void st8(bf16* p, u32x4 v) { *reinterpret_cast<u32x4*>(p) = v; }

__global__ __launch_bounds__(256) void k_pool(const bf16* X, bf16* Y, int B, int H, int W, int C) {
    const int Ho = H / 2, Wo = W / 2, G = C / 8;
    const size_t n = (size_t)B * Ho * Wo * G;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int c8 = (int)(e % G);
        const size_t q = e / G;
        const int xo = q % Wo, yo = (q / Wo) % Ho, b = q / ((size_t)Wo * Ho);
        const size_t g = (((size_t)b * H + 2 * yo) * W + 2 * xo) * C + c8 * 8;
        float s[8], t[8];
        unpack8(ld8(X + g), s);
        unpack8(ld8(X + g + C), t);
        for (int k = 0; k < 8; ++k) s[k] += t[k];
        unpack8(ld8(X + g + (size_t)W * C), t);
        for (int k = 0; k < 8; ++k) s[k] += t[k];
        unpack8(ld8(X + g + (size_t)W * C + C), t);
        for (int k = 0; k < 8; ++k) s[k] = 0.25f * (s[k] + t[k]);
        st8(Y + q * C + c8 * 8, pack8(s));
    }
}

// dX = pool^T(dY) + dS (the skip-path gradient), fine resolution
__global__ __launch_bounds__(256) void k_pool_bwd_add(const bf16* dY, const bf16* dS, bf16* dX, int B, int H, int W,
                                                      int C) {
    const int G = C / 8, Wo = W / 2, Ho = H / 2;
    const size_t n = (size_t)B * H * W * G;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int c8 = (int)(e % G);
        const size_t q = e / G;
        const int x = q % W, y = (q / W) % H, b = q / ((size_t)W * H);
        float u[8], v[8];
        unpack8(ld8(dY + (((size_t)b * Ho + y / 2) * Wo + x / 2) * C + c8 * 8), u);
        unpack8(ld8(dS + q * C + c8 * 8), v);
        for (int k = 0; k < 8; ++k) u[k] = 0.25f * u[k] + v[k];
        st8(dX + q * C + c8 * 8, pack8(u));
    }
}

// Y = [up2(Xc), S]: 2C channels at the fine resolution
__global__ __launch_bounds__(256) void k_up_concat(const bf16* Xc, const bf16* S, bf16* Y, int B, int H, int W, int C) {
    const int G = C / 8;
    const size_t n = (size_t)B * H * W * 2 * G;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int c8 = (int)(e % (2 * G));
        const size_t q = e / (2 * G);
        const int x = q % W, y = (q / W) % H, b = q / ((size_t)W * H);
        const u32x4 v = (c8 < G) ? ld8(Xc + (((size_t)b * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c8 * 8)
                                 : ld8(S + q * C + (c8 - G) * 8);
        st8(Y + q * 2 * C + c8 * 8, v);
    }
}

// from the 2C-channel concat gradient: dXc = up^T(first C), dS = last C
__global__ __launch_bounds__(256) void k_up_concat_bwd(const bf16* dY, bf16* dXc, bf16* dS, int B, int H, int W,
                                                       int C) {
    const int Ho = H / 2, Wo = W / 2, G = C / 8;
    const size_t nc = (size_t)B * Ho * Wo * G;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < nc; e += (size_t)gridDim.x * blockDim.x) {
        const int c8 = (int)(e % G);
        const size_t q = e / G;
        const int xo = q % Wo, yo = (q / Wo) % Ho, b = q / ((size_t)Wo * Ho);
        float s[8] = {}, t[8];
        for (int d = 0; d < 4; ++d) {
            const size_t p = ((size_t)b * H + 2 * yo + d / 2) * W + 2 * xo + d % 2;
            unpack8(ld8(dY + p * 2 * C + c8 * 8), t);
            for (int k = 0; k < 8; ++k) s[k] += t[k];
        }
        st8(dXc + q * C + c8 * 8, pack8(s));
    }
    const size_t nf = (size_t)B * H * W * G;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < nf; e += (size_t)gridDim.x * blockDim.x) {
        const size_t p = e / G;
        const int c8 = (int)(e % G);
        st8(dS + p * C + c8 * 8, ld8(dY + p * 2 * C + C + c8 * 8));
    }
}

// ------------------------------------------------------------ output layer
// out[p] = scale_b * (w . last[p] + b0) on unknown nodes (0 elsewhere)
__global__ __launch_bounds__(256) void k_out(const bf16* last, const float* w, const float* b0, float* out, int B,
                                             int HW, int C) {
    const size_t n = (size_t)B * HW;
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
        float s = b0[0];
        for (int c8 = 0; c8 < C / 8; ++c8) {
            float x[8];
            unpack8(ld8(last + p * C + c8 * 8), x);
            for (int k = 0; k < 8; ++k) s += w[c8 * 8 + k] * x[k];
        }
        out[p] = s;
    }
}

// loss = mean over masked pixels of (out - target)^2; dz; dlast = w dz;
// per-block partials of the loss, dw and db
__global__ __launch_bounds__(256) void k_loss_out_bwd(const float* out, const float* target, const float* mask,
                                                      const bf16* last, const float* w, bf16* dlast, float* part,
                                                      int B, int HW, float inv_n) {
    constexpr int C = kC;
    __shared__ float sh[256];
    float acc[C + 2];
#pragma unroll
    for (int k = 0; k < C + 2; ++k) acc[k] = 0.0f;
    const size_t n = (size_t)B * HW;
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
        const float mk = mask[p];
        const float d = (out[p] - target[p]) * mk;
        const float dz = 2.0f * d * inv_n;
        acc[0] += d * d * inv_n;
        acc[1] += dz;
#pragma unroll
        for (int c8 = 0; c8 < C / 8; ++c8) {
            float x[8], g[8];
            unpack8(ld8(last + p * C + c8 * 8), x);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                acc[2 + c8 * 8 + k] += x[k] * dz;
                g[k] = w[c8 * 8 + k] * dz;
            }
            st8(dlast + p * C + c8 * 8, pack8(g));
        }
    }
#pragma unroll
    for (int k = 0; k < C + 2; ++k) {
        sh[threadIdx.x] = acc[k];
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * (C + 2) + k] = sh[0];
        __syncthreads();
    }
}

// ------------------------------------------------------------------ Adam
// master FP32 parameters p, gradients g, moments m, v; t is the step count
__global__ __launch_bounds__(256) void k_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1,
                                              float b2, float eps, float c1, float c2) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// bfloat16 copies of one conv layer's weights: forward layout [t][co][cin_pad]
// and, for the data gradient, [t'][ci][co] = W[8 - t'][co][ci]
__global__ __launch_bounds__(256) void k_pack_conv(const float* w, int cin, int cin_pad, int cout, bf16* fwd,
                                                   bf16* bwd) {
    const int n = 9 * cout * cin_pad;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int ci = e % cin_pad, co = (e / cin_pad) % cout, t = e / (cin_pad * cout);
        fwd[e] = f2bf(ci < cin ? w[(t * cout + co) * cin + ci] : 0.0f);
    }
    if (!bwd) return;
    const int nb = 9 * cin * cout;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nb; e += gridDim.x * blockDim.x) {
        const int co = e % cout, ci = (e / cout) % cin, t = e / (cout * cin);
        bwd[e] = f2bf(w[((8 - t) * cout + co) * cin + ci]);
    }
}

// network input from a residual on the node grid (FP64), chi and node kinds:
// channels [r * scale, chi / (1 + chi), 1 on unknown nodes], 16 padded
__global__ __launch_bounds__(256) void k_input_from_grid(const double* r, double scale, const double* chi,
                                                         const int8_t* nk, bf16* X, int H, int W, int w) {
    const size_t n = (size_t)H * W;
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
        const int y = p / W, x = p % W;
        const int node = y * w + x;
        const bool free = nk[node] < 0;
        bf16x8 v0 = {}, v1 = {};
        v0[0] = f2raw(free ? (float)(r[node] * scale) : 0.0f);
        const float c = (float)chi[node];
        v0[1] = f2raw(c / (1.0f + c));
        v0[2] = f2raw(free ? 1.0f : 0.0f);
        *(bf16x8*)&X[p * 16] = v0;
        *(bf16x8*)&X[p * 16 + 8] = v1;
    }
}

// network input from host-provided FP32 channels [H][W][3]
__global__ __launch_bounds__(256) void k_input_from_f32(const float* in3, bf16* X, size_t npix) {
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < npix; p += (size_t)gridDim.x * blockDim.x) {
        bf16x8 v0 = {}, v1 = {};
        v0[0] = f2raw(in3[p * 3]);
        v0[1] = f2raw(in3[p * 3 + 1]);
        v0[2] = f2raw(in3[p * 3 + 2]);
        *(bf16x8*)&X[p * 16] = v0;
        *(bf16x8*)&X[p * 16 + 8] = v1;
    }
}

// training batch from harvested pairs: inputs [r, chi', mask], target e
struct BatchIdx {
    int idx[kMaxBatch];
};
__global__ __launch_bounds__(256) void k_gather_batch(BatchIdx bi, int B, const float* hr, const float* he,
                                                      const float* hchi, const float* hmask, bf16* X, float* target,
                                                      float* mask, size_t img) {
    const size_t n = (size_t)B * img;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int b = (int)(e / img);
        const size_t p = e % img;
        const size_t src = (size_t)bi.idx[b] * img + p;
        bf16x8 v0 = {}, v1 = {};
        v0[0] = f2raw(hr[src]);
        v0[1] = f2raw(hchi[src]);
        v0[2] = f2raw(hmask[p]);
        *(bf16x8*)&X[e * 16] = v0;
        *(bf16x8*)&X[e * 16 + 8] = v1;
        target[e] = he[src];
        mask[e] = hmask[p];
    }
}

// preconditioner input from an FP32 inner residual on the node grid,
// scaled to unit RMS over the unknown nodes: r sqrt(n_free / (r.r))
__global__ __launch_bounds__(256) void k_input_from_r32(const float* r, const double* rr, const double* chi,
                                                        const int8_t* nk, bf16* X, int H, int W, int w,
                                                        double n_free) {
    const float sc = (float)sqrt(n_free / *rr);
    const size_t n = (size_t)H * W;
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
        const int node = (int)(p / W) * w + (int)(p % W);
        const bool free = nk[node] < 0;
        bf16x8 v0 = {}, v1 = {};
        v0[0] = f2raw(free ? r[node] * sc : 0.0f);
        const float c = (float)chi[node];
        v0[1] = f2raw(c / (1.0f + c));
        v0[2] = f2raw(free ? 1.0f : 0.0f);
        *(bf16x8*)&X[p * 16] = v0;
        *(bf16x8*)&X[p * 16 + 8] = v1;
    }
}

// z = ||r|| * out on unknown nodes of the image, 0 elsewhere (flexible CG
// is blind to a scalar factor on z; this one keeps z on the scale of r)
__global__ __launch_bounds__(256) void k_out_to_z(const float* out, const double* rr, const int8_t* nk, float* z, int H,
                                                  int W, int w, int nn) {
    const float sc = (float)sqrt(*rr);
    for (int node = blockIdx.x * blockDim.x + threadIdx.x; node < nn; node += gridDim.x * blockDim.x) {
        const int i = node % w, j = node / w;
        float v = 0.0f;
        if (i < W && j < H && nk[node] < 0) v = sc * out[(size_t)j * W + i];
        z[node] = v;
    }
}

// harvest, inside an FP64 MG-PCG solve: a residual (FP32, image layout,
// not yet scaled), chi / (1 + chi), the mask, and the approximation x + dx it
// belongs to (FP64, node layout) for the error computed once the solve is
// done.  Skipped once the solve has converged (*done).
__global__ __launch_bounds__(256) void k_harvest_iter(const double* r, const double* x, const double* dx,
                                                      const double* chi, const int8_t* nk, float* hr, float* hchi,
                                                      float* hmask, double* xk, const int* done, int H, int W, int w,
                                                      int nn) {
    if (*done) return;
    const size_t n = (size_t)H * W;
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
        const int node = (int)(p / W) * w + (int)(p % W);
        const bool free = nk[node] < 0;
        hr[p] = free ? (float)r[node] : 0.0f;
        const double c = chi[node];
        hchi[p] = (float)(c / (1.0 + c));
        hmask[p] = free ? 1.0f : 0.0f;
    }
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += gridDim.x * blockDim.x) xk[e] = x[e] + dx[e];
}

// after the solve: the error of iterate k, e = x* - x_k (FP64 difference),
// and per-block partial sums of e^2 and r^2
__global__ __launch_bounds__(256) void k_pair_error(const double* xs, const double* xk, const int8_t* nk,
                                                    const float* hr, float* he, double* part, int H, int W, int w) {
    __shared__ double sa[256], sb[256];
    const size_t n = (size_t)H * W;
    double a = 0.0, b = 0.0;
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
        const int node = (int)(p / W) * w + (int)(p % W);
        const double d = nk[node] < 0 ? xs[node] - xk[node] : 0.0;
        he[p] = (float)d;
        a += d * d;
        b += (double)hr[p] * (double)hr[p];
    }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sa[threadIdx.x] += sa[threadIdx.x + o];
            sb[threadIdx.x] += sb[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sa[0];
        part[2 * blockIdx.x + 1] = sb[0];
    }
}

// ... then both scaled to unit RMS over the unknown nodes (every block sums
// the partials in the same order)
__global__ __launch_bounds__(256) void k_pair_norm(float* hr, float* he, const double* part, int nparts, size_t n,
                                                   double n_free) {
    __shared__ double sa[256], sb[256];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nparts; k += blockDim.x) {
        a += part[2 * k];
        b += part[2 * k + 1];
    }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sa[threadIdx.x] += sa[threadIdx.x + o];
            sb[threadIdx.x] += sb[threadIdx.x + o];
        }
        __syncthreads();
    }
    const float se = sa[0] > 0.0 ? (float)sqrt(n_free / sa[0]) : 0.0f;
    const float sr = sb[0] > 0.0 ? (float)sqrt(n_free / sb[0]) : 0.0f;
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
        he[p] *= se;
        hr[p] *= sr;
    }
}

// --------------------------------------------------------------- launchers
static dim3 tiles_grid(int B, int H, int W) {
    const long long nt = (long long)((W + 15) / 16) * ((H + 15) / 16) * B;
    return dim3((unsigned)std::min<long long>(nt, 2048));
}

void conv_fwd(int cin, const bf16* X, const bf16* Wt, const float* bias, bf16* Y, int B, int H, int W,
              hipStream_t s) {
    const dim3 g = tiles_grid(B, H, W);
    if (cin == 16) hipLaunchKernelGGL((k_conv3x3<16, 32, true, false>), g, dim3(256), 0, s, X, Wt, bias, nullptr, Y, B, H, W);
    else if (cin == 32) hipLaunchKernelGGL((k_conv3x3<32, 32, true, false>), g, dim3(256), 0, s, X, Wt, bias, nullptr, Y, B, H, W);
    else hipLaunchKernelGGL((k_conv3x3<64, 32, true, false>), g, dim3(256), 0, s, X, Wt, bias, nullptr, Y, B, H, W);
}

void conv_dgrad(int cin_of_layer, const bf16* D, const bf16* Yout, const bf16* Wb, bf16* DX, int B, int H, int W,
                hipStream_t s) {
    const dim3 g = tiles_grid(B, H, W);
    if (cin_of_layer == 32)
        hipLaunchKernelGGL((k_conv3x3<32, 32, false, true>), g, dim3(256), 0, s, D, Wb, (const float*)nullptr, Yout, DX, B, H, W);
    else
        hipLaunchKernelGGL((k_conv3x3<32, 64, false, true>), g, dim3(256), 0, s, D, Wb, (const float*)nullptr, Yout, DX, B, H, W);
}

int conv_wgrad(int cin, const bf16* X, const bf16* D, const bf16* Yout, float* part, float* gw, int B, int H, int W,
               hipStream_t s) {
    const dim3 g = tiles_grid(B, H, W);
    const int nb = (int)std::min<unsigned>(g.x, kWgradBlocks);
    const int len = 9 * 32 * cin + 32;
    if (cin == 16) hipLaunchKernelGGL((k_wgrad<16>), dim3(nb), dim3(256), 0, s, X, D, Yout, part, B, H, W);
    else if (cin == 32) hipLaunchKernelGGL((k_wgrad<32>), dim3(nb), dim3(256), 0, s, X, D, Yout, part, B, H, W);
    else hipLaunchKernelGGL((k_wgrad<64>), dim3(nb), dim3(256), 0, s, X, D, Yout, part, B, H, W);
    sum_parts(part, nb, len, gw, s);
    return nb;
}

static dim3 ew_grid(size_t n) { return dim3((unsigned)std::min<size_t>((n + 255) / 256, 4096)); }

void pool(const bf16* X, bf16* Y, int B, int H, int W, int C, hipStream_t s) {
    hipLaunchKernelGGL(k_pool, ew_grid((size_t)B * H * W * C / 32), dim3(256), 0, s, X, Y, B, H, W, C);
}
void pool_bwd_add(const bf16* dY, const bf16* dS, bf16* dX, int B, int H, int W, int C, hipStream_t s) {
    hipLaunchKernelGGL(k_pool_bwd_add, ew_grid((size_t)B * H * W * C / 8), dim3(256), 0, s, dY, dS, dX, B, H, W, C);
}
void up_concat(const bf16* Xc, const bf16* S, bf16* Y, int B, int H, int W, int C, hipStream_t s) {
    hipLaunchKernelGGL(k_up_concat, ew_grid((size_t)B * H * W * C / 4), dim3(256), 0, s, Xc, S, Y, B, H, W, C);
}
void up_concat_bwd(const bf16* dY, bf16* dXc, bf16* dS, int B, int H, int W, int C, hipStream_t s) {
    hipLaunchKernelGGL(k_up_concat_bwd, ew_grid((size_t)B * H * W * C / 8), dim3(256), 0, s, dY, dXc, dS, B, H, W, C);
}
void out_fwd(const bf16* last, const float* w, const float* b0, float* out, int B, int HW, int C, hipStream_t s) {
    hipLaunchKernelGGL(k_out, ew_grid((size_t)B * HW), dim3(256), 0, s, last, w, b0, out, B, HW, C);
}
void loss_out_bwd(const float* out, const float* target, const float* mask, const bf16* last, const float* w,
                  bf16* dlast, float* part, float* sums, int B, int HW, int C, float inv_n, hipStream_t s) {
    hipLaunchKernelGGL(k_loss_out_bwd, dim3(kLossBlocks), dim3(256), 0, s, out, target, mask, last, w, dlast, part, B,
                       HW, inv_n);
    sum_parts(part, kLossBlocks, C + 2, sums, s);
}
void adam(float* p, const float* g, float* m, float* v, int n, float lr, int t, hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, ew_grid(n), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, 1e-8f, c1, c2);
}
void pack_conv(const float* w, int cin, int cin_pad, int cout, bf16* fwd, bf16* bwd, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_conv, dim3(64), dim3(256), 0, s, w, cin, cin_pad, cout, fwd, bwd);
}
void input_from_grid(const double* r, double scale, const double* chi, const int8_t* nk, bf16* X, int H, int W,
                     int w, hipStream_t s) {
    hipLaunchKernelGGL(k_input_from_grid, ew_grid((size_t)H * W), dim3(256), 0, s, r, scale, chi, nk, X, H, W, w);
}
void input_from_f32(const float* in3, bf16* X, size_t npix, hipStream_t s) {
    hipLaunchKernelGGL(k_input_from_f32, ew_grid(npix), dim3(256), 0, s, in3, X, npix);
}
void gather_batch(const Net& n, const int* idx, int B, hipStream_t s) {
    BatchIdx bi;
    for (int b = 0; b < kMaxBatch; ++b) bi.idx[b] = b < B ? idx[b] : 0;
    const size_t img = (size_t)n.H * n.W;
    hipLaunchKernelGGL(k_gather_batch, ew_grid(B * img), dim3(256), 0, s, bi, B, (const float*)n.h_r,
                       (const float*)n.h_e, (const float*)n.h_chi, (const float*)n.h_mask, n.x0, n.target, n.mask,
                       img);
}
void input_from_r32(const Net& n, const float* r, const double* rr, const double* chi, const int8_t* nk, int w,
                    double n_free, hipStream_t s) {
    hipLaunchKernelGGL(k_input_from_r32, ew_grid((size_t)n.H * n.W), dim3(256), 0, s, r, rr, chi, nk, n.x0, n.H, n.W,
                       w, n_free);
}
void out_to_z(const Net& n, const double* rr, const int8_t* nk, float* z, int w, int nn, hipStream_t s) {
    hipLaunchKernelGGL(k_out_to_z, ew_grid(nn), dim3(256), 0, s, (const float*)n.out, rr, nk, z, n.H, n.W, w, nn);
}
void harvest_iter(const Net& n, int slot, const double* r, const double* x, const double* dx, const double* chi,
                  const int8_t* nk, double* xk, const int* done, int w, int nn, hipStream_t s) {
    const size_t img = (size_t)n.H * n.W;
    hipLaunchKernelGGL(k_harvest_iter, ew_grid(std::max<size_t>(img, nn)), dim3(256), 0, s, r, x, dx, chi, nk,
                       n.h_r + slot * img, n.h_chi + slot * img, n.h_mask, xk, done, n.H, n.W, w, nn);
}
__global__ __launch_bounds__(256) void k_mask_from_nodes(const int8_t* nk, float* hmask, int H, int W, int w) {
    const size_t n = (size_t)H * W;
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x)
        hmask[p] = nk[(int)(p / W) * w + (int)(p % W)] < 0 ? 1.0f : 0.0f;
}
void mask_from_nodes(const Net& n, const int8_t* nk, int w, hipStream_t s) {
    hipLaunchKernelGGL(k_mask_from_nodes, ew_grid((size_t)n.H * n.W), dim3(256), 0, s, nk, n.h_mask, n.H, n.W, w);
}
void pair_finish(const Net& n, int slot, const double* xs, const double* xk, const int8_t* nk, int w, double n_free,
                 double* part, hipStream_t s) {
    const size_t img = (size_t)n.H * n.W;
    const dim3 g((unsigned)std::min<size_t>((img + 255) / 256, kHarvestBlocks));
    hipLaunchKernelGGL(k_pair_error, g, dim3(256), 0, s, xs, xk, nk, (const float*)(n.h_r + slot * img),
                       n.h_e + slot * img, part, n.H, n.W, w);
    hipLaunchKernelGGL(k_pair_norm, g, dim3(256), 0, s, n.h_r + slot * img, n.h_e + slot * img, (const double*)part,
                       (int)g.x, img, n_free);
}

}  // namespace unet
}  // namespace pic
