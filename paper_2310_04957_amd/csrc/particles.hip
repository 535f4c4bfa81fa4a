// particles.hip -- the per-step particle loop on gfx950: field gather, D1
// implicit correction, absorption, null-collision MCC with wavefront-ballot
// compaction of colliders, D1 prediction and the fixed-point charge /
// susceptibility deposit through an LDS window flushed with 64-bit integer
// atomics (arXiv 2310.04957, Sec. 2: implicit push around Eq. 1, unequal
// weights, collision paragraph).  Births are appended in parent order.
#include <hip/hip_runtime.h>

#include "pic_internal.h"

namespace pic {

constexpr int kHalo = 8;                      // cells of halo around a 16x16-cell tile
constexpr int kWin = kTile + 2 * kHalo + 1;   // LDS window nodes per side
constexpr int kQCap = 512;                    // deferred colliders per block

struct PushArgs {
    Geo g;
    Mcc m;
    float* f[9];
    const float2* E;
    unsigned long long* dep;
    unsigned long long* wallq;
    DevCounters* ctr;
    Birth* stage;
    int* stage_cnt;
    int sp, sign;
    float qm, dt;
    uint32_t key0, key1, step;
};

__device__ __forceinline__ unsigned long long lanemask_lt() {
    return (1ull << (threadIdx.x & 63)) - 1ull;
}

// Charge of a removed particle: to the conductor it hit, or deposited at the
// landing point into the dielectric surface-charge grid (the share on
// conductor nodes goes to that conductor).  Returns true if removed.
__device__ __forceinline__ bool absorb(const Geo& g, const Loc& L, float w, int sign,
                                       unsigned long long* s_abs, unsigned long long* wallq) {
    if (L.inside && g.cell_kind[L.j * g.nr + L.i] == 0) return false;
    if (!L.inside) {
        int bc = g.edge_bc[L.edge];
        int slot = bc >= 0 ? (bc < 2 ? bc : 0) : 2;
        atomicAdd(&s_abs[slot], (unsigned long long)total_share((double)w));
        return true;
    }
    int ck = g.cell_kind[L.j * g.nr + L.i];
    if (ck >= 2) {
        int id = ck - 2;
        atomicAdd(&s_abs[id < 2 ? id : 0], (unsigned long long)total_share((double)w));
        return true;
    }
    int64_t c[4];
    node_shares(L, (double)w, g.invd, c);
    int n00 = L.j * g.w + L.i;
    int nodes[4] = {n00, n00 + 1, n00 + g.w, n00 + g.w + 1};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int nk = g.node_kind[nodes[k]];
        if (nk >= 0) {
            atomicAdd(&s_abs[nk < 2 ? nk : 0], (unsigned long long)c[k]);
        } else {
            atomicAdd(&wallq[nodes[k]], (unsigned long long)(sign * c[k]));
            atomicAdd(&s_abs[3], (unsigned long long)c[k]);
        }
    }
    return true;
}

// Deposit into the LDS window when all four nodes fall inside it, else
// straight to the global grid (the result is identical: integer sums).
__device__ __forceinline__ void deposit(const Geo& g, const Loc& L, float w, unsigned long long* win, int wi0,
                                        int wj0, unsigned long long* dep, unsigned int* s_fallback) {
    int64_t c[4];
    node_shares(L, (double)w, g.invd, c);
    int li = L.i - wi0, lj = L.j - wj0;
    if (li >= 0 && li + 1 < kWin && lj >= 0 && lj + 1 < kWin) {
        int b = lj * kWin + li;
        atomicAdd(&win[b], (unsigned long long)c[0]);
        atomicAdd(&win[b + 1], (unsigned long long)c[1]);
        atomicAdd(&win[b + kWin], (unsigned long long)c[2]);
        atomicAdd(&win[b + kWin + 1], (unsigned long long)c[3]);
    } else {
        int n00 = L.j * g.w + L.i;
        atomicAdd(&dep[n00], (unsigned long long)c[0]);
        atomicAdd(&dep[n00 + 1], (unsigned long long)c[1]);
        atomicAdd(&dep[n00 + g.w], (unsigned long long)c[2]);
        atomicAdd(&dep[n00 + g.w + 1], (unsigned long long)c[3]);
        atomicAdd(s_fallback, 1u);
    }
}

__device__ __forceinline__ P9 load9(float* const* f, long long p) {
    P9 s;
    s.r = f[0][p]; s.z = f[1][p]; s.vr = f[2][p]; s.vt = f[3][p]; s.vz = f[4][p];
    s.ar = f[5][p]; s.at = f[6][p]; s.az = f[7][p]; s.w = f[8][p];
    return s;
}

__device__ __forceinline__ void store8(float* const* f, long long p, const P9& s) {
    f[0][p] = s.r; f[1][p] = s.z; f[2][p] = s.vr; f[3][p] = s.vt; f[4][p] = s.vz;
    f[5][p] = s.ar; f[6][p] = s.at; f[7][p] = s.az;
}

// One time step for every particle of one species.  A block owns whole
// chunks of 4096 consecutive slots; the chunks of one XCD are contiguous so
// neighbouring (cell-sorted) chunks share that XCD's L2.  Colliding
// particles are compacted by wavefront ballots into an LDS queue and
// processed by full waves; births are staged per chunk in slot order.
__global__ __launch_bounds__(kBlock) void k_particles(PushArgs a) {
    __shared__ unsigned long long win[kWin * kWin];
    __shared__ float qst[9][kQCap];
    __shared__ unsigned int qslot[kQCap];
    __shared__ int wave_cnt[kBlock / 64];
    __shared__ int s_qn, s_nb;
    __shared__ unsigned long long s_abs[4];
    __shared__ unsigned int s_coll[4];
    __shared__ unsigned int s_fallback;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const Geo& g = a.g;
    const long long n = a.ctr->n_slots[a.sp];
    const long long nch = (n + kChunk - 1) / kChunk;
    const int nx = 8;  // XCDs: consecutive block ids go round-robin over them
    const int xcd = blockIdx.x % nx, per = gridDim.x / nx, lb = blockIdx.x / nx;
    const long long c_begin = nch * xcd / nx, c_end = nch * (xcd + 1) / nx;

    for (int k = tid; k < kWin * kWin; k += kBlock) win[k] = 0ull;
    if (tid < 4) { s_abs[tid] = 0ull; s_coll[tid] = 0u; }
    if (tid == 0) s_fallback = 0u;
    __syncthreads();

    for (long long chunk = c_begin + lb; chunk < c_end; chunk += per) {
        const long long base = chunk * kChunk;
        // LDS window: the 16x16 tile of the chunk's first particle plus halo
        int wi0 = -(1 << 28), wj0 = -(1 << 28);
        {
            Loc L0 = locate(a.f[0][base], a.f[1][base], g);
            if (L0.inside && a.f[0][base] >= 0.0f) {
                wi0 = ((L0.i >> kTileShift) << kTileShift) - kHalo;
                wj0 = ((L0.j >> kTileShift) << kTileShift) - kHalo;
            }
        }
        if (tid == 0) { s_qn = 0; s_nb = 0; }
        __syncthreads();

        for (int it = 0; it < kItems; ++it) {
            const long long p = base + (long long)it * kBlock + tid;
            bool live = p < n;
            bool coll = false;
            P9 s;
            if (live) {
                s.r = a.f[0][p];
                live = s.r >= 0.0f;
            }
            if (live) {
                s = load9(a.f, p);
                float Er, Ez;
                gather_E(a.E, g, s.r, s.z, Er, Ez);
                d1_correct(s, Er, Ez, a.qm, a.dt);
                Loc L = locate(s.r, s.z, g);
                if (absorb(g, L, s.w, a.sign, s_abs, a.wallq)) {
                    a.f[0][p] = -1.0f;
                    live = false;
                } else {
                    uint4 x = draw((uint32_t)p, a.step, kPurposeMcc, a.sp, 0, a.key0, a.key1);
                    coll = x.x < a.m.thresh;
                    if (!coll) {
                        d1_predict(s, a.dt);
                        Loc L2 = locate(s.r, s.z, g);
                        if (absorb(g, L2, s.w, a.sign, s_abs, a.wallq)) {
                            a.f[0][p] = -1.0f;
                        } else {
                            deposit(g, L2, s.w, win, wi0, wj0, a.dep, &s_fallback);
                            store8(a.f, p, s);
                        }
                    }
                }
            }
            // ballot compaction of this round's colliders, in slot order
            unsigned long long mask = __ballot(coll);
            if (lane == 0) wave_cnt[wave] = __popcll(mask);
            __syncthreads();
            if (coll) {
                int q = s_qn + __popcll(mask & lanemask_lt());
                for (int w2 = 0; w2 < wave; ++w2) q += wave_cnt[w2];
                qslot[q] = (unsigned int)p;
                qst[0][q] = s.r; qst[1][q] = s.z; qst[2][q] = s.vr; qst[3][q] = s.vt; qst[4][q] = s.vz;
                qst[5][q] = s.ar; qst[6][q] = s.at; qst[7][q] = s.az; qst[8][q] = s.w;
            }
            __syncthreads();
            if (tid == 0) {
                int t = 0;
                for (int w2 = 0; w2 < kBlock / 64; ++w2) t += wave_cnt[w2];
                s_qn += t;
            }
            __syncthreads();
            const int qn = s_qn;
            if (qn > kQCap - kBlock || it == kItems - 1) {
                // process the queue with full waves
                for (int b0 = 0; b0 < qn; b0 += kBlock) {
                    const int q = b0 + tid;
                    const bool has = q < qn;
                    int proc = -1;
                    float b6[6];
                    P9 c;
                    unsigned int slot = 0;
                    if (has) {
                        slot = qslot[q];
                        c.r = qst[0][q]; c.z = qst[1][q]; c.vr = qst[2][q]; c.vt = qst[3][q]; c.vz = qst[4][q];
                        c.ar = qst[5][q]; c.at = qst[6][q]; c.az = qst[7][q]; c.w = qst[8][q];
                        uint4 x = draw(slot, a.step, kPurposeMcc, a.sp, 0, a.key0, a.key1);
                        proc = collide(a.sp, x, c.vr, c.vt, c.vz, a.m, slot, a.step, a.key0, a.key1, b6,
                                       &a.ctr->viol);
                        atomicAdd(&s_coll[proc], 1u);
                    }
                    const bool born = has && proc == 2 && a.stage != nullptr;
                    unsigned long long bm = __ballot(born);
                    __syncthreads();
                    if (lane == 0) wave_cnt[wave] = __popcll(bm);
                    __syncthreads();
                    if (born) {
                        int idx = s_nb + __popcll(bm & lanemask_lt());
                        for (int w2 = 0; w2 < wave; ++w2) idx += wave_cnt[w2];
                        if (idx < kStageCap) {
                            Birth bb;
                            bb.r = c.r; bb.z = c.z; bb.w = c.w;
                            for (int k = 0; k < 6; ++k) bb.v[k] = b6[k];
                            a.stage[chunk * kStageCap + idx] = bb;
                        } else {
                            atomicMax(&a.ctr->err, 2);
                        }
                    }
                    __syncthreads();
                    if (tid == 0) {
                        int t = 0;
                        for (int w2 = 0; w2 < kBlock / 64; ++w2) t += wave_cnt[w2];
                        s_nb += t;
                    }
                    if (has) {
                        d1_predict(c, a.dt);
                        Loc L2 = locate(c.r, c.z, g);
                        if (absorb(g, L2, c.w, a.sign, s_abs, a.wallq)) {
                            a.f[0][slot] = -1.0f;
                        } else {
                            deposit(g, L2, c.w, win, wi0, wj0, a.dep, &s_fallback);
                            store8(a.f, slot, c);
                        }
                    }
                }
                __syncthreads();
                if (tid == 0) s_qn = 0;
                __syncthreads();
            }
        }
        // flush the window to the global grid and clear it
        __syncthreads();
        for (int k = tid; k < kWin * kWin; k += kBlock) {
            unsigned long long v = win[k];
            if (v != 0ull) {
                int gi = wi0 + k % kWin, gj = wj0 + k / kWin;
                if (gi >= 0 && gi <= g.nr && gj >= 0 && gj <= g.nz) atomicAdd(&a.dep[gj * g.w + gi], v);
                win[k] = 0ull;
            }
        }
        if (tid == 0 && a.stage_cnt != nullptr) a.stage_cnt[chunk] = min(s_nb, kStageCap);
        __syncthreads();
    }
    if (tid < 4) {
        if (s_abs[tid]) atomicAdd(&a.ctr->absorbed[a.sp][tid], s_abs[tid]);
        if (s_coll[tid]) atomicAdd(&a.ctr->coll[a.sp][tid], (unsigned long long)s_coll[tid]);
    }
    if (tid == 0 && s_fallback) atomicAdd(&a.ctr->fallback, (unsigned long long)s_fallback);
}

static int grid_blocks() {
    // persistent-style grid: 8 XCDs x 32 CUs x 4 blocks, a multiple of 8
    return 1024;
}

static Geo make_geo(pic_handle* h) {
    Geo g;
    g.nr = h->nr; g.nz = h->nz; g.w = h->w;
    g.R = h->cfg.geom.R; g.Z = h->cfg.geom.Z; g.Sr = h->Sr; g.Sz = h->Sz;
    g.inv_dr = (float)(1.0 / h->dr); g.inv_dz = (float)(1.0 / h->dz);
    g.invd = h->invd;
    g.cell_kind = h->cell_kind;
    g.node_kind = h->node_kind;
    for (int k = 0; k < 3; ++k) g.edge_bc[k] = h->cfg.geom.edge_bc[k];
    return g;
}

static Mcc make_mcc(pic_handle* h, int sp) {
    const double QE = 1.602176634e-19, ME = 9.1093837015e-31, MAR = 39.948 * 1.66053906660e-27;
    Mcc m;
    m.n_gas = (float)h->n_gas;
    m.nu_max = (float)h->nu_max[sp];
    m.vth_gas = (float)h->vth_gas;
    m.half_m_over_e = (float)(0.5 * ME / QE);
    m.two_e_over_m = (float)(2.0 * QE / ME);
    m.m_ratio2 = (float)(2.0 * ME / MAR);
    m.thresh = h->thresh[sp];
    return m;
}

static float qm_of(int sp) {
    const double QE = 1.602176634e-19, ME = 9.1093837015e-31, MAR = 39.948 * 1.66053906660e-27;
    return (float)(sp == 0 ? -QE / ME : QE / MAR);
}

void launch_particles(pic_handle* h, int sp) {
    PushArgs a;
    a.g = make_geo(h);
    a.m = make_mcc(h, sp);
    for (int k = 0; k < 9; ++k) a.f[k] = h->buf[sp][h->cur[sp]].f[k];
    a.E = h->E;
    a.dep = h->dep[h->dep_cur][sp];
    a.wallq = h->wallq;
    a.ctr = h->ctr;
    a.stage = sp == 0 ? h->stage : nullptr;
    a.stage_cnt = sp == 0 ? h->stage_cnt : nullptr;
    a.sp = sp;
    a.sign = sp == 0 ? -1 : 1;
    a.qm = qm_of(sp);
    a.dt = (float)h->dt;
    a.key0 = (uint32_t)(h->cfg.run.seed & 0xFFFFFFFFu);
    a.key1 = (uint32_t)(h->cfg.run.seed >> 32);
    a.step = (uint32_t)(h->step + 1);
    hipLaunchKernelGGL(k_particles, dim3(grid_blocks()), dim3(kBlock), 0, h->stream, a);
}

// ---------------------------------------------------------------- births
// One block: exclusive scan of the per-chunk birth counts of the electron
// pass (slot order), capacity check, append bases.
__global__ __launch_bounds__(1024) void k_birth_scan(DevCounters* c, const int* cnt, int* off, long long cap_e,
                                                     long long cap_i) {
    __shared__ long long s_part[1024];
    __shared__ long long s_carry;
    const int tid = threadIdx.x;
    const long long nch = (c->n_slots[0] + kChunk - 1) / kChunk;
    if (tid == 0) s_carry = 0;
    __syncthreads();
    for (long long b0 = 0; b0 < nch; b0 += 1024) {
        long long i = b0 + tid;
        long long v = (i < nch) ? (long long)cnt[i] : 0;
        s_part[tid] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            long long t = (tid >= o) ? s_part[tid - o] : 0;
            __syncthreads();
            s_part[tid] += t;
            __syncthreads();
        }
        if (i < nch) off[i] = (int)(s_carry + s_part[tid] - v);
        __syncthreads();
        if (tid == 0) s_carry += s_part[1023];
        __syncthreads();
    }
    if (tid == 0) {
        long long B = s_carry;
        c->base[0] = c->n_slots[0];
        c->base[1] = c->n_slots[1];
        c->nch_births = nch;
        if (c->n_slots[0] + B > cap_e || c->n_slots[1] + B > cap_i) {
            atomicMax(&c->err, 2);
            B = 0;
        }
        c->births_step = B;
        c->born += B;
        c->n_slots[0] += B;
        c->n_slots[1] += B;
    }
}

struct BirthArgs {
    Geo g;
    float* fe[9];
    float* fi[9];
    unsigned long long* dep_e;
    unsigned long long* dep_i;
    unsigned long long* wallq;
    DevCounters* ctr;
    const Birth* stage;
    const int* cnt;
    const int* off;
    float dt;
};

// Newborn electron and ion: a_bar = 0, predict, absorption, deposit.
__device__ __forceinline__ void place_newborn(const Geo& g, float* const* f, long long slot, P9 s, float dt,
                                              int sp, unsigned long long* dep, unsigned long long* wallq,
                                              DevCounters* ctr) {
    d1_predict(s, dt);
    Loc L = locate(s.r, s.z, g);
    bool removed;
    {
        unsigned long long loc[4] = {0ull, 0ull, 0ull, 0ull};
        // absorption accounting straight to the global counters (rare)
        if (L.inside && g.cell_kind[L.j * g.nr + L.i] == 0) {
            removed = false;
        } else {
            removed = true;
            if (!L.inside) {
                int bc = g.edge_bc[L.edge];
                loc[bc >= 0 ? (bc < 2 ? bc : 0) : 2] += (unsigned long long)total_share((double)s.w);
            } else {
                int ck = g.cell_kind[L.j * g.nr + L.i];
                if (ck >= 2) {
                    loc[(ck - 2) < 2 ? ck - 2 : 0] += (unsigned long long)total_share((double)s.w);
                } else {
                    int64_t c[4];
                    node_shares(L, (double)s.w, g.invd, c);
                    int n00 = L.j * g.w + L.i;
                    int nodes[4] = {n00, n00 + 1, n00 + g.w, n00 + g.w + 1};
                    for (int k = 0; k < 4; ++k) {
                        int nk = g.node_kind[nodes[k]];
                        if (nk >= 0) loc[nk < 2 ? nk : 0] += (unsigned long long)c[k];
                        else {
                            atomicAdd(&wallq[nodes[k]], (unsigned long long)((sp == 0 ? -1 : 1) * c[k]));
                            loc[3] += (unsigned long long)c[k];
                        }
                    }
                }
            }
            for (int k = 0; k < 4; ++k)
                if (loc[k]) atomicAdd(&ctr->absorbed[sp][k], loc[k]);
        }
    }
    f[0][slot] = removed ? -1.0f : s.r;
    f[1][slot] = s.z; f[2][slot] = s.vr; f[3][slot] = s.vt; f[4][slot] = s.vz;
    f[5][slot] = s.ar; f[6][slot] = s.at; f[7][slot] = s.az; f[8][slot] = s.w;
    if (!removed) {
        int64_t c[4];
        node_shares(L, (double)s.w, g.invd, c);
        int n00 = L.j * g.w + L.i;
        atomicAdd(&dep[n00], (unsigned long long)c[0]);
        atomicAdd(&dep[n00 + 1], (unsigned long long)c[1]);
        atomicAdd(&dep[n00 + g.w], (unsigned long long)c[2]);
        atomicAdd(&dep[n00 + g.w + 1], (unsigned long long)c[3]);
    }
}

__global__ __launch_bounds__(kBlock) void k_birth_append(BirthArgs a) {
    const long long nch = a.ctr->nch_births;
    if (a.ctr->births_step == 0) return;
    const long long be = a.ctr->base[0], bi = a.ctr->base[1];
    for (long long chunk = blockIdx.x; chunk < nch; chunk += gridDim.x) {
        int cnt = a.cnt[chunk];
        if (cnt == 0) continue;
        long long o = a.off[chunk];
        for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
            Birth b = a.stage[chunk * kStageCap + k];
            P9 e;
            e.r = b.r; e.z = b.z; e.vr = b.v[0]; e.vt = b.v[1]; e.vz = b.v[2];
            e.ar = 0.0f; e.at = 0.0f; e.az = 0.0f; e.w = b.w;
            place_newborn(a.g, a.fe, be + o + k, e, a.dt, 0, a.dep_e, a.wallq, a.ctr);
            P9 i = e;
            i.vr = b.v[3]; i.vt = b.v[4]; i.vz = b.v[5];
            place_newborn(a.g, a.fi, bi + o + k, i, a.dt, 1, a.dep_i, a.wallq, a.ctr);
        }
    }
}

void launch_births(pic_handle* h) {
    hipLaunchKernelGGL(k_birth_scan, dim3(1), dim3(1024), 0, h->stream, h->ctr, h->stage_cnt, h->stage_off,
                       (long long)h->cap[0], (long long)h->cap[1]);
    BirthArgs a;
    a.g = make_geo(h);
    for (int k = 0; k < 9; ++k) {
        a.fe[k] = h->buf[0][h->cur[0]].f[k];
        a.fi[k] = h->buf[1][h->cur[1]].f[k];
    }
    a.dep_e = h->dep[h->dep_cur][0];
    a.dep_i = h->dep[h->dep_cur][1];
    a.wallq = h->wallq;
    a.ctr = h->ctr;
    a.stage = h->stage;
    a.cnt = h->stage_cnt;
    a.off = h->stage_off;
    a.dt = (float)h->dt;
    hipLaunchKernelGGL(k_birth_append, dim3(512), dim3(kBlock), 0, h->stream, a);
}

// ------------------------------------------------------------------ loader
struct LoadArgs {
    float* f[9];
    const double* cdf;
    const int* cell;
    int nv, nr;
    double vvac, dr, dz;
    long long n;
    float W, vth;
    int sp;
    uint32_t key0, key1;
};

// Uniform plasma (Sec. 3, first paragraph): a vacuum cell by inverse CDF of
// cell volume, r^2 and z uniform inside it, Maxwellian velocity.
__global__ __launch_bounds__(kBlock) void k_load(LoadArgs a) {
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < a.n;
         p += (long long)gridDim.x * blockDim.x) {
        uint4 x = draw((uint32_t)p, 0u, kPurposeLoad, a.sp, 0, a.key0, a.key1);
        uint4 y = draw((uint32_t)p, 0u, kPurposeLoad, a.sp, 1, a.key0, a.key1);
        double target = (double)u01(x.x) * a.vvac;
        int lo = 0, hi = a.nv - 1;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (a.cdf[mid] > target) hi = mid; else lo = mid + 1;
        }
        int c = a.cell[lo];
        int ci = c % a.nr, cj = c / a.nr;
        double r0 = ci * a.dr, r1 = (ci + 1) * a.dr;
        double r = sqrt(r0 * r0 + (double)u01(x.y) * (r1 * r1 - r0 * r0));
        double z = (cj + (double)u01(x.z)) * a.dz;
        float vr, vt, vz;
        maxwell3(y, a.vth, vr, vt, vz);
        a.f[0][p] = (float)r; a.f[1][p] = (float)z;
        a.f[2][p] = vr; a.f[3][p] = vt; a.f[4][p] = vz;
        a.f[5][p] = 0.0f; a.f[6][p] = 0.0f; a.f[7][p] = 0.0f;
        a.f[8][p] = a.W;
    }
}

void launch_load(pic_handle* h, int sp, const double* cdf, const int* cell, int nv, double vvac, int64_t n,
                 float W, float vth) {
    LoadArgs a;
    for (int k = 0; k < 9; ++k) a.f[k] = h->buf[sp][h->cur[sp]].f[k];
    a.cdf = cdf; a.cell = cell; a.nv = nv; a.nr = h->nr;
    a.vvac = vvac; a.dr = h->dr; a.dz = h->dz;
    a.n = n; a.W = W; a.vth = vth; a.sp = sp;
    a.key0 = (uint32_t)(h->cfg.run.seed & 0xFFFFFFFFu);
    a.key1 = (uint32_t)(h->cfg.run.seed >> 32);
    if (n > 0) hipLaunchKernelGGL(k_load, dim3(2048), dim3(kBlock), 0, h->stream, a);
}

// First prediction after the load (a_bar = 0), absorption and deposit; or,
// with predict = 0, a plain deposit of the stored positions.
struct PDArgs {
    Geo g;
    float* f[9];
    unsigned long long* dep;
    unsigned long long* wallq;
    DevCounters* ctr;
    int sp, predict;
    float dt;
};

__global__ __launch_bounds__(kBlock) void k_predict_deposit(PDArgs a) {
    const long long n = a.ctr->n_slots[a.sp];
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < n;
         p += (long long)gridDim.x * blockDim.x) {
        P9 s = load9(a.f, p);
        if (!(s.r >= 0.0f)) continue;
        if (a.predict) {
            place_newborn(a.g, a.f, p, s, a.dt, a.sp, a.dep, a.wallq, a.ctr);
        } else {
            Loc L = locate(s.r, s.z, a.g);
            if (!L.inside) continue;
            int64_t c[4];
            node_shares(L, (double)s.w, a.g.invd, c);
            int n00 = L.j * a.g.w + L.i;
            atomicAdd(&a.dep[n00], (unsigned long long)c[0]);
            atomicAdd(&a.dep[n00 + 1], (unsigned long long)c[1]);
            atomicAdd(&a.dep[n00 + a.g.w], (unsigned long long)c[2]);
            atomicAdd(&a.dep[n00 + a.g.w + 1], (unsigned long long)c[3]);
        }
    }
}

static void launch_pd(pic_handle* h, int sp, int predict) {
    PDArgs a;
    a.g = make_geo(h);
    for (int k = 0; k < 9; ++k) a.f[k] = h->buf[sp][h->cur[sp]].f[k];
    a.dep = h->dep[h->dep_cur][sp];
    a.wallq = h->wallq;
    a.ctr = h->ctr;
    a.sp = sp;
    a.predict = predict;
    a.dt = (float)h->dt;
    hipLaunchKernelGGL(k_predict_deposit, dim3(2048), dim3(kBlock), 0, h->stream, a);
}

void launch_predict_deposit(pic_handle* h, int sp) { launch_pd(h, sp, 1); }

void launch_redeposit(pic_handle* h) {
    for (int sp = 0; sp < 2; ++sp) {
        launch_zero_u64(h->dep[h->dep_cur][sp], (size_t)h->nn, h->stream);
        launch_pd(h, sp, 0);
    }
}

__global__ __launch_bounds__(kBlock) void k_count_alive(const float* r, const long long* n_slots, int sp,
                                                        unsigned long long* out) {
    __shared__ unsigned int s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const long long n = n_slots[sp];
    unsigned int c = 0;
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < n;
         p += (long long)gridDim.x * blockDim.x)
        c += (r[p] >= 0.0f);
    atomicAdd(&s_cnt, c);
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out, (unsigned long long)s_cnt);
}

void launch_count_alive(pic_handle* h, long long* out2) {
    // uses the pad words of the device counters as scratch
    unsigned long long* d = (unsigned long long*)&h->ctr->pad[0];
    launch_zero_u64(d, 2, h->stream);
    for (int sp = 0; sp < 2; ++sp)
        hipLaunchKernelGGL(k_count_alive, dim3(512), dim3(kBlock), 0, h->stream, h->buf[sp][h->cur[sp]].f[0],
                           (const long long*)h->ctr->n_slots, sp, d + sp);
    hipMemcpyAsync(out2, d, 2 * sizeof(long long), hipMemcpyDeviceToHost, h->stream);
    hipStreamSynchronize(h->stream);
}

}  // namespace pic
