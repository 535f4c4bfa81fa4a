// sort.hip -- periodic stable sort of a species' slots by the 16x16-cell
// tile of the predicted position, which also removes dead slots.  LSD radix
// sort on 8-bit digits: per-chunk digit histograms, one exclusive scan in
// digit-major order, and a stable scatter whose in-chunk ranks come from
// wavefront ballots (no atomics decide an order, so the permutation is
// deterministic).  The particle arrays are then gathered through the
// permutation, usually by the next particle step.  The keys usually come
// from the species' particle step just before (it locates every particle
// anyway); the key pass then covers only the slots appended after it.
#include <hip/hip_runtime.h>

#include "pic_internal.h"

namespace pic {

constexpr int kSeg = 4096;   // elements per block of the scan kernels

struct KeyArgs {
    Geo g;
    const f32x4* rz;          // the particles' first vector group (r, z, ...)
    tkey_t* keys;
    const long long* n_slots;
    const long long* start;   // non-null: keys below *start are already written
    unsigned int* dead;
    int sp, kmul;             // tile key multiplier
    uint32_t dead_key;
};

__global__ __launch_bounds__(kBlock) void k_keys(KeyArgs a) {
    const long long n = a.n_slots[a.sp];
    const long long p0 = a.start ? *a.start : 0;
    unsigned int dead = 0;
    for (long long p = p0 + blockIdx.x * (long long)blockDim.x + threadIdx.x; p < n;
         p += (long long)gridDim.x * blockDim.x) {
        const f32x4 x = a.rz[p];
        uint32_t key = a.dead_key;
        if (x.x >= 0.0f) {
            Loc L = locate(x.x, x.y, a.g);
            if (L.inside) key = tile_key(L, a.kmul);
        }
        dead += (key == a.dead_key);
        a.keys[p] = (tkey_t)key;
    }
    // wave reduction then one atomic per wave
    for (int o = 32; o > 0; o >>= 1) dead += __shfl_down(dead, o);
    if ((threadIdx.x & 63) == 0 && dead) atomicAdd(a.dead, dead);
}

// eight 16-bit keys from one 16-byte load
__device__ __forceinline__ void unpack8(const uint4 v, uint32_t* k) {
    k[0] = v.x & 0xFFFFu; k[1] = v.x >> 16; k[2] = v.y & 0xFFFFu; k[3] = v.y >> 16;
    k[4] = v.z & 0xFFFFu; k[5] = v.z >> 16; k[6] = v.w & 0xFFFFu; k[7] = v.w >> 16;
}

// Digit counts per chunk.  Each thread counts kItems consecutive keys and
// adds a run of equal digits with one LDS atomic: sorted or nearly sorted
// keys (the usual case between two sorts) then cost about one atomic per
// thread instead of one per key on the same few bins.
__global__ __launch_bounds__(kBlock) void k_hist(const tkey_t* keys, const long long* n_slots, int sp, int shift,
                                                 uint32_t mask, uint32_t* hist) {
    __shared__ unsigned int h[256];
    const long long n = n_slots[sp];
    const long long nch = (n + kChunk - 1) / kChunk;
    for (long long c = blockIdx.x; c < nch; c += gridDim.x) {
        h[threadIdx.x] = 0u;
        __syncthreads();
        const long long p0 = c * kChunk + (long long)threadIdx.x * kItems;
        uint32_t kv[kItems];
        if (p0 + kItems <= n) {
#pragma unroll
            for (int q = 0; q < kItems / 8; ++q) unpack8(*reinterpret_cast<const uint4*>(keys + p0 + 8 * q), kv + 8 * q);
        } else {
#pragma unroll
            for (int q = 0; q < kItems; ++q) kv[q] = p0 + q < n ? keys[p0 + q] : 0u;
        }
        const int cnt = (int)min((long long)kItems, max(0LL, n - p0));
        uint32_t run_d = 0u, run_n = 0u;
#pragma unroll
        for (int q = 0; q < kItems; ++q) {
            if (q < cnt) {
                const uint32_t d = (kv[q] >> shift) & mask;
                if (run_n != 0u && d != run_d) {
                    atomicAdd(&h[run_d], run_n);
                    run_n = 0u;
                }
                run_d = d;
                ++run_n;
            }
        }
        if (run_n != 0u) atomicAdd(&h[run_d], run_n);
        __syncthreads();
        hist[(long long)threadIdx.x * nch + c] = h[threadIdx.x];
        __syncthreads();
    }
}

// exclusive scan of hist[0 .. 256 * nch) in three kernels
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t* v, const long long* n_slots, int sp,
                                                        uint32_t* bsum) {
    __shared__ unsigned int s[kBlock];
    const long long nch = (n_slots[sp] + kChunk - 1) / kChunk;
    const long long len = 256 * nch;
    const long long nseg = (len + kSeg - 1) / kSeg;
    for (long long b = blockIdx.x; b < nseg; b += gridDim.x) {
        unsigned int t = 0;
        for (int k = 0; k < kSeg / kBlock; ++k) {
            long long i = b * kSeg + (long long)k * kBlock + threadIdx.x;
            if (i < len) t += v[i];
        }
        s[threadIdx.x] = t;
        __syncthreads();
        for (int o = kBlock / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) bsum[b] = s[0];
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void k_scan_top(uint32_t* bsum, const long long* n_slots, int sp) {
    __shared__ unsigned int s[1024];
    __shared__ unsigned int carry;
    const long long nch = (n_slots[sp] + kChunk - 1) / kChunk;
    const long long nseg = (256 * nch + kSeg - 1) / kSeg;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (long long b0 = 0; b0 < nseg; b0 += 1024) {
        long long i = b0 + threadIdx.x;
        unsigned int v = (i < nseg) ? bsum[i] : 0u;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            unsigned int t = ((int)threadIdx.x >= o) ? s[threadIdx.x - o] : 0u;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nseg) bsum[i] = carry + s[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 0) carry += s[1023];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_down(uint32_t* v, const uint32_t* bsum, const long long* n_slots,
                                                      int sp) {
    __shared__ unsigned int s[kBlock];
    const long long nch = (n_slots[sp] + kChunk - 1) / kChunk;
    const long long len = 256 * nch;
    const long long nseg = (len + kSeg - 1) / kSeg;
    constexpr int per = kSeg / kBlock;  // 16 consecutive elements per thread
    for (long long b = blockIdx.x; b < nseg; b += gridDim.x) {
        unsigned int loc[per];
        unsigned int t = 0;
        const long long i0 = b * kSeg + (long long)threadIdx.x * per;
        for (int k = 0; k < per; ++k) {
            long long i = i0 + k;
            loc[k] = (i < len) ? v[i] : 0u;
            t += loc[k];
        }
        s[threadIdx.x] = t;
        __syncthreads();
        for (int o = 1; o < kBlock; o <<= 1) {
            unsigned int u = ((int)threadIdx.x >= o) ? s[threadIdx.x - o] : 0u;
            __syncthreads();
            s[threadIdx.x] += u;
            __syncthreads();
        }
        unsigned int run = bsum[b] + s[threadIdx.x] - t;
        for (int k = 0; k < per; ++k) {
            long long i = i0 + k;
            if (i < len) v[i] = run;
            run += loc[k];
        }
        __syncthreads();
    }
}

__device__ __forceinline__ unsigned long long lanemask_lt_s() {
    return (1ull << (threadIdx.x & 63)) - 1ull;
}

// peers of a lane: the valid lanes of its wavefront holding the same digit
__device__ __forceinline__ unsigned long long digit_peers(bool valid, uint32_t d) {
    // one ballot per distinct digit present in the wavefront (a few: the
    // keys are nearly sorted), taking the digits in the order of their
    // first lane
    unsigned long long left = __ballot(valid), peers = 0ull;
    while (left) {
        const uint32_t d0 = __builtin_amdgcn_readlane(d, __ffsll((long long)left) - 1);
        const bool same = valid && d == d0;
        const unsigned long long m = __ballot(same);
        if (same) peers = m;
        left &= ~m;
    }
    return peers;
}

// Stable scatter of one 8-bit digit.  Each wavefront owns a contiguous
// quarter of the chunk and walks it twice: first counting its digits, then
// (after one block-wide offset computation) placing every element at
// chunk offset + earlier wavefronts' counts + its rank among equal digits
// before it.  Ranks come from wavefront ballots, so the order is fixed.
__global__ __launch_bounds__(kBlock) void k_scatter(const tkey_t* kin, const uint32_t* vin, tkey_t* kout,
                                                    uint32_t* vout, const uint32_t* offs, const long long* n_slots,
                                                    int sp, int shift, uint32_t mask) {
    __shared__ unsigned int wcnt[kWaves][256];
    __shared__ unsigned int wbase[kWaves][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int slice = kChunk / kWaves;
    static_assert(slice == 64 * kItems, "a wavefront's slice is kItems keys per lane");
    const long long n = n_slots[sp];
    const long long nch = (n + kChunk - 1) / kChunk;
    for (long long c = blockIdx.x; c < nch; c += gridDim.x) {
        for (int w2 = 0; w2 < kWaves; ++w2) wcnt[w2][tid] = 0u;
        __syncthreads();
        const long long s0 = c * kChunk + (long long)wave * slice;
        // counts of the wavefront's slice: each lane counts kItems
        // consecutive keys (slice = 64 kItems) by runs of equal digits
        {
            const long long p0 = s0 + (long long)lane * kItems;
            uint32_t kv[kItems];
            if (p0 + kItems <= n) {
#pragma unroll
                for (int q = 0; q < kItems / 8; ++q) unpack8(*reinterpret_cast<const uint4*>(kin + p0 + 8 * q), kv + 8 * q);
            } else {
#pragma unroll
                for (int q = 0; q < kItems; ++q) kv[q] = p0 + q < n ? kin[p0 + q] : 0u;
            }
            const int cnt = (int)min((long long)kItems, max(0LL, n - p0));
            uint32_t run_d = 0u, run_n = 0u;
#pragma unroll
            for (int q = 0; q < kItems; ++q) {
                if (q < cnt) {
                    const uint32_t d = (kv[q] >> shift) & mask;
                    if (run_n != 0u && d != run_d) {
                        atomicAdd(&wcnt[wave][run_d], run_n);
                        run_n = 0u;
                    }
                    run_d = d;
                    ++run_n;
                }
            }
            if (run_n != 0u) atomicAdd(&wcnt[wave][run_d], run_n);
        }
        __syncthreads();
        {
            unsigned int run = offs[(long long)tid * nch + c];
            for (int w2 = 0; w2 < kWaves; ++w2) {
                wbase[w2][tid] = run;
                run += wcnt[w2][tid];
            }
        }
        __syncthreads();
        // the slice's keys and values, all requested before the first is used
        uint32_t kk[slice / 64], vv[slice / 64];
#pragma unroll
        for (int it = 0; it < slice / 64; ++it) {
            const long long p = s0 + it * 64 + lane;
            const bool valid = p < n;
            kk[it] = valid ? kin[p] : 0u;
            // the first pass's values are the slots
            vv[it] = vin ? (valid ? vin[p] : 0u) : (uint32_t)p;
        }
#pragma unroll
        for (int it = 0; it < slice / 64; ++it) {
            const long long p = s0 + it * 64 + lane;
            const bool valid = p < n;
            const uint32_t key = kk[it];
            const uint32_t d = (key >> shift) & mask;
            const unsigned long long peers = digit_peers(valid, d);
            const int rank = __popcll(peers & lanemask_lt_s());
            if (valid) {
                const unsigned int pos = wbase[wave][d] + rank;
                if (kout != nullptr) kout[pos] = (tkey_t)key;   // (the last pass keeps no keys)
                vout[pos] = vv[it];
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (valid && rank == 0) wbase[wave][d] += (unsigned int)__popcll(peers);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
    }
}

struct GatherArgs {
    Species src;
    Species dst;
    const uint32_t* idx;
    const long long* n_slots;
    int sp;
};

__global__ __launch_bounds__(kBlock) void k_gather(GatherArgs a) {
    const long long n = a.n_slots[a.sp];
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        store9(a.dst, (uint32_t)q, load9(a.src, a.idx[q]));
    }
}

__global__ void k_finish_sort(long long* n_slots, unsigned int* dead, int sp) {
    n_slots[sp] -= (long long)dead[sp];
    dead[sp] = 0u;
}

__global__ void k_zero_u32(unsigned int* p) { *p = 0u; }

// keyed: the particle step just before wrote the keys of its slots and
// counted their dead ones (no sort is pending then); the key pass covers
// the slots appended since (births, split copies)
void launch_sort(pic_handle* h, int sp, bool deferred, bool keyed) {
    hipStream_t st = h->stream;
    materialize(h, sp);   // a sort reads the particles as they stand
    const long long* ns = (const long long*)h->ctr->n_slots;
    unsigned int* dead = &h->ctr->dead[0];
    if (!keyed) hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, dead + sp);
    Species& S = h->buf[sp][h->cur[sp]];
    KeyArgs ka;
    ka.g.nr = h->nr; ka.g.nz = h->nz; ka.g.w = h->w;
    ka.g.R = h->cfg.geom.R; ka.g.Z = h->cfg.geom.Z; ka.g.Sr = h->Sr; ka.g.Sz = h->Sz;
    ka.g.inv_dr = (float)(1.0 / h->dr); ka.g.inv_dz = (float)(1.0 / h->dz);
    ka.g.invd = h->invd; ka.g.cell_kind = h->cell_kind; ka.g.node_kind = h->node_kind;
    for (int k = 0; k < 3; ++k) ka.g.edge_bc[k] = h->cfg.geom.edge_bc[k];
    ka.rz = S.a;
    // the species' keys: the electrons' in the first shared buffer, the ions'
    // in their own (the radix passes then ping-pong with the second shared one)
    tkey_t* kb[2] = {sp == 0 ? h->keys[0] : h->keys_ion, h->keys[1]};
    ka.keys = kb[0];
    ka.n_slots = ns; ka.dead = dead + sp; ka.sp = sp; ka.kmul = h->kmul;
    ka.start = keyed ? (const long long*)&h->ctr->n_keyed[sp] : nullptr;
    ka.dead_key = (uint32_t)(h->ntz * h->kmul);   // past the last tile's key: sorts last
    hipLaunchKernelGGL(k_keys, dim3(2048), dim3(kBlock), 0, st, ka);
    // the passes' digits: the tile column, then the tile row (power-of-two
    // key multiplier), else 8-bit digits
    int pshift[3], pmask[3], np = 0;
    if (h->row_bits > 0) {
        pshift[0] = 0;
        pmask[0] = (1 << h->row_bits) - 1;
        pshift[1] = h->row_bits;
        pmask[1] = 0xFF;
        np = 2;
    } else {
        for (int sh = 0; sh < h->key_bits && np < 3; sh += 8) {
            pshift[np] = sh;
            pmask[np] = 0xFF;
            ++np;
        }
    }
    int src = 0;
    for (int ip = 0; ip < np; ++ip) {
        const int shift = pshift[ip];
        const uint32_t mask = (uint32_t)pmask[ip];
        // the last pass writes the permutation to the species' own buffer
        const bool last = ip + 1 == np;
        hipLaunchKernelGGL(k_hist, dim3(2048), dim3(kBlock), 0, st, kb[src], ns, sp, shift, mask, h->hist);
        hipLaunchKernelGGL(k_scan_reduce, dim3(2048), dim3(kBlock), 0, st, h->hist, ns, sp, h->bsum);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, h->bsum, ns, sp);
        hipLaunchKernelGGL(k_scan_down, dim3(2048), dim3(kBlock), 0, st, h->hist, h->bsum, ns, sp);
        hipLaunchKernelGGL(k_scatter, dim3(2048), dim3(kBlock), 0, st, kb[src], ip == 0 ? nullptr : h->idx[src],
                           last ? nullptr : kb[1 - src],
                           last ? h->perm[sp] : h->idx[1 - src], h->hist, ns, sp, shift, mask);
        src = 1 - src;
    }
    hipLaunchKernelGGL(k_finish_sort, dim3(1), dim3(1), 0, st, h->ctr->n_slots, dead, sp);
    // the particles move with the next particle step (deferred) or now
    h->pending[sp] = true;
    if (!deferred) materialize(h, sp);
}

// apply a deferred sort: gather the current buffer through the permutation
// into the other one (the slot count is already that of the sorted view)
void materialize(pic_handle* h, int sp) {
    if (!h->pending[sp]) return;
    GatherArgs ga;
    const Species& S = h->buf[sp][h->cur[sp]];
    Species& D = h->buf[sp][1 - h->cur[sp]];
    ga.src = S;
    ga.dst = D;
    ga.idx = h->perm[sp];
    ga.n_slots = h->ctr->n_slots;
    ga.sp = sp;
    hipLaunchKernelGGL(k_gather, dim3(2048), dim3(kBlock), 0, h->stream, ga);
    h->cur[sp] = 1 - h->cur[sp];
    h->pending[sp] = false;
}

// ---------------------------------------------------- particle splitting
// (Sec. 3, particle splitting against on-axis heating.)  A live particle
// inside the domain whose weight is at least 2^m reference weights of its
// cell column (m <= 3, compared in FP32) becomes 2^m identical particles of
// a 2^m-th of the weight: the parent keeps its slot, the copies follow the
// last slot in parent-slot order.  Three passes over the chunks of kChunk
// slots: count, one exclusive scan of the chunk counts, write (the count is
// recomputed, so no per-slot storage); order comes from block scans, never
// from atomics, so the result is deterministic.
struct SplitArgs {
    Geo g;
    Species f;
    const float* wt;          // reference weight per cell column
    DevCounters* ctr;
    long long* off;           // per chunk: copies, then their exclusive offsets
    long long cap;
    int sp;
};

__device__ __forceinline__ int split_doublings(float w, float t) {
    int m = 0;
    while (m < 3 && w >= t * (float)(2 << m)) ++m;
    return m;
}

__device__ __forceinline__ int split_m(const SplitArgs& a, long long p) {
    const f32x4 x = a.f.a[p];
    if (!(x.x >= 0.0f)) return 0;
    const Loc L = locate(x.x, x.y, a.g);
    if (!L.inside) return 0;
    return split_doublings(a.f.w[p], a.wt[L.i]);
}

// exclusive scan of v over the block (kBlock threads); *total gets the sum
__device__ __forceinline__ int block_exscan(int v, int* sh, int* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    int before = 0, all = 0;
    for (int w2 = 0; w2 < kBlock / 64; ++w2) {
        if (w2 < wave) before += sh[w2];
        all += sh[w2];
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

__global__ __launch_bounds__(kBlock) void k_split_count(SplitArgs a) {
    __shared__ int sh[kBlock / 64];
    const long long n = a.ctr->n_slots[a.sp];
    const long long nch = (n + kChunk - 1) / kChunk;
    for (long long c = blockIdx.x; c < nch; c += gridDim.x) {
        int cnt = 0;
        for (int it = 0; it < kItems; ++it) {
            const long long p = c * kChunk + (long long)it * kBlock + threadIdx.x;
            if (p < n) cnt += (1 << split_m(a, p)) - 1;
        }
        int total;
        block_exscan(cnt, sh, &total);
        if (threadIdx.x == 0) a.off[c] = total;
    }
}

// one block: chunk counts -> exclusive offsets; the pass is cancelled
// (split_total = -1, capacity error) when the copies do not fit
__global__ __launch_bounds__(1024) void k_split_scan(SplitArgs a) {
    __shared__ long long sh[1024];
    const long long n = a.ctr->n_slots[a.sp];
    const long long nch = (n + kChunk - 1) / kChunk;
    const long long per = (nch + 1023) / 1024;
    const long long b0 = threadIdx.x * per, b1 = min(nch, b0 + per);
    long long s = 0;
    for (long long c = b0; c < b1; ++c) s += a.off[c];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const long long y = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += y;
        __syncthreads();
    }
    long long run = sh[threadIdx.x] - s;
    for (long long c = b0; c < b1; ++c) {
        const long long v = a.off[c];
        a.off[c] = run;
        run += v;
    }
    if (threadIdx.x == 1023) {
        const long long total = sh[1023];
        if (n + total > a.cap) {
            a.ctr->split_total = -1;
            atomicOr(&a.ctr->err, kErrSplit);
        } else {
            a.ctr->split_total = total;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_split_write(SplitArgs a) {
    __shared__ int sh[kBlock / 64];
    if (a.ctr->split_total <= 0) return;
    const long long n = a.ctr->n_slots[a.sp];
    const long long nch = (n + kChunk - 1) / kChunk;
    for (long long c = blockIdx.x; c < nch; c += gridDim.x) {
        long long out = n + a.off[c];
        for (int it = 0; it < kItems; ++it) {
            const long long p = c * kChunk + (long long)it * kBlock + threadIdx.x;
            const int m = (p < n) ? split_m(a, p) : 0;
            const int e = (1 << m) - 1;
            int total;
            const int ex = block_exscan(e, sh, &total);
            if (e > 0) {
                P9 v = load9(a.f, (uint32_t)p);
                v.w = v.w / (float)(1 << m);
                a.f.w[p] = v.w;
                for (int q = 0; q < e; ++q) store9(a.f, (uint32_t)(out + ex + q), v);
            }
            out += total;
        }
    }
}

__global__ void k_split_commit(DevCounters* c, int sp) {
    if (c->split_total > 0) {
        c->n_slots[sp] += c->split_total;
        c->split_added[sp] += c->split_total;
    }
}

void launch_split(pic_handle* h, int sp) {
    materialize(h, sp);
    SplitArgs a;
    a.g.nr = h->nr; a.g.nz = h->nz; a.g.w = h->w;
    a.g.R = h->cfg.geom.R; a.g.Z = h->cfg.geom.Z; a.g.Sr = h->Sr; a.g.Sz = h->Sz;
    a.g.inv_dr = (float)(1.0 / h->dr); a.g.inv_dz = (float)(1.0 / h->dz);
    a.g.invd = h->invd; a.g.cell_kind = h->cell_kind; a.g.node_kind = h->node_kind;
    for (int k = 0; k < 3; ++k) a.g.edge_bc[k] = h->cfg.geom.edge_bc[k];
    a.f = h->buf[sp][h->cur[sp]];
    a.wt = h->wtcol[sp];
    a.ctr = h->ctr;
    a.off = h->split_off;
    a.cap = h->cap[sp];
    a.sp = sp;
    hipLaunchKernelGGL(k_split_count, dim3(2048), dim3(kBlock), 0, h->stream, a);
    hipLaunchKernelGGL(k_split_scan, dim3(1), dim3(1024), 0, h->stream, a);
    hipLaunchKernelGGL(k_split_write, dim3(2048), dim3(kBlock), 0, h->stream, a);
    hipLaunchKernelGGL(k_split_commit, dim3(1), dim3(1), 0, h->stream, h->ctr, sp);
}

}  // namespace pic
