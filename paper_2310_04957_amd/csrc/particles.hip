// particles.hip -- the per-step particle loop on gfx950: field gather, D1
// implicit correction, absorption, null-collision MCC on the colliding
// lanes, D1 prediction and the fixed-point charge /
// susceptibility deposit through an LDS window flushed with 64-bit integer
// atomics (arXiv 2310.04957, Sec. 2: implicit push around Eq. 1, unequal
// weights, collision paragraph).  Births are appended in parent order.
#include <hip/hip_runtime.h>

#include "pic_internal.h"

namespace pic {

// LDS deposit window: the 16x16-cell tile of a particle from the middle of a
// chunk plus a halo of H cells, (16 + 2H + 1)^2 nodes; electrons (fast,
// dispersing between sorts) use H = 24, ions H = 16
constexpr int win_nodes(int halo) { return kTile + 2 * halo + 1; }
constexpr int kRounds = kSlice / 64;
static_assert(kSlice % 256 == 0 && kRounds % 4 == 0, "decision words are shared by four aligned rounds");

struct PushArgs {
    Geo g;
    Mcc m;
    Species f;                   // particles written here (read here too unless perm is set)
    Species src;                 // with perm: slot p reads src at perm[p] (a deferred sort)
    const uint32_t* perm;
    tkey_t* keys;                // non-null: write each slot's sort key (a sort follows this step)
    Species sink;                // 64 slots written by the lanes past the last slot
    tkey_t* ksink;               // 64 keys likewise
    uint32_t dead_key;
    int kmul;                    // tile key multiplier
    const float2* E;
    unsigned long long* dep;
    unsigned long long* wallq;
    DevCounters* ctr;
    Birth* stage;
    int* stage_cnt;
    int stage_w;                 // births per staging row
    int sp, sign;
    float qm, dt;
    uint32_t key0, key1, step;
};

__device__ __forceinline__ unsigned long long lanemask_lt() {
    return (1ull << (threadIdx.x & 63)) - 1ull;
}

// The radial factor 2^-2F / (2i + 1) of column i, as the grid's table holds
// it (a correctly rounded FP64 division, bit for bit the table's value).
// Computed, not read from the table, on the paths of particles outside the
// LDS window: a load there would make its wait also wait for the next
// round's state, which is in flight.
__device__ __forceinline__ double radial_factor(int i) {
    return __builtin_ldexp(1.0, -2 * kFBits) / (double)(2 * i + 1);
}

// Charge of a removed particle: to the conductor it hit, or deposited at the
// landing point into the dielectric surface-charge grid (the share on
// conductor nodes goes to that conductor).  Returns true if removed.
// Cell kinds come from the window's LDS copy s_ck when the cell lies in it,
// else from the LDS copy s_vt of the all-vacuum tile bitmap when that marks
// the cell's tile, else from the global grid.
template <int kWin>
__device__ __forceinline__ bool absorb(const Geo& g, const Loc& L, float w, int sign,
                                       unsigned long long* s_abs, unsigned long long* wallq, bool vac, int wi0,
                                       int wj0, const uint8_t* s_ck, const uint32_t* s_vt) {
    if (!L.inside) {
        // (a select of the three, not an indexed read of the argument block,
        // which would be a vector memory load)
        const int bc = L.edge == 0 ? g.edge_bc[0] : L.edge == 1 ? g.edge_bc[1] : g.edge_bc[2];
        int slot = bc >= 0 ? slot_of(bc) : 2;
        atomicAdd(&s_abs[slot], (unsigned long long)total_share((double)w));
        return true;
    }
    const int li = L.i - wi0, lj = L.j - wj0;
    const bool inw = (unsigned)li < (unsigned)(kWin - 1) && (unsigned)lj < (unsigned)(kWin - 1);
    // vac: every domain cell of the window is vacuum
    if (inw && vac) return false;
    // the LDS read (index clamped into the window) is replaced from the
    // global grid for a cell outside the window
    int ck = s_ck[min(max(lj, 0), kWin - 2) * (kWin - 1) + min(max(li, 0), kWin - 2)];
    // (as the aligned 32-bit word holding the byte, inside the grid's
    // 256-byte-padded buffer, which also keeps the compiler from merging
    // the two reads into one generic-address load)
    if (!inw) {
        // a vacuum tile needs no global read (whose wait would also wait
        // for the next round's state, in flight)
        const int t = (L.j >> kTileShift) * g.ntr + (L.i >> kTileShift);
        if (t < 32 * kVacWords && ((s_vt[t >> 5] >> (t & 31)) & 1u)) return false;
        const uint32_t c = (uint32_t)(L.j * g.nr + L.i);
        const uint32_t wd = *reinterpret_cast<const uint32_t*>(g.cell_kind + (c & ~3u));
        ck = (int)((wd >> (8u * (c & 3u))) & 0xFFu);
    }
    if (ck == 0) return false;
    if (ck >= 2) {
        int id = ck - 2;
        atomicAdd(&s_abs[slot_of(id)], (unsigned long long)total_share((double)w));
        return true;
    }
    int64_t c[4];
    node_shares(L, (double)w, radial_factor(L.i), c);
    int n00 = L.j * g.w + L.i;
    int nodes[4] = {n00, n00 + 1, n00 + g.w, n00 + g.w + 1};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int nk = g.node_kind[nodes[k]];
        if (nk >= 0) {
            atomicAdd(&s_abs[slot_of(nk)], (unsigned long long)c[k]);
        } else {
            atomicAdd(&wallq[nodes[k]], (unsigned long long)(sign * c[k]));
            atomicAdd(&s_abs[3], (unsigned long long)c[k]);
        }
    }
    return true;
}

// Deposit into the LDS window when all four nodes fall inside it, else
// straight to the global grid (the result is identical: integer sums).
// Returns 1 for a global-fallback deposit.
// The radial factor of the particle's column comes from the window's LDS
// copy s_invd (columns wi0 ... wi0 + kWin - 1) in the first case.
template <int kWin>
__device__ __forceinline__ unsigned int deposit(const Geo& g, const Loc& L, float w, unsigned long long* win,
                                                const double* s_invd, int wi0, int wj0, unsigned long long* dep) {
    int64_t c[4];
    const int li = L.i - wi0, lj = L.j - wj0;
    if (li >= 0 && li + 1 < kWin && lj >= 0 && lj + 1 < kWin) {
        node_shares(L, (double)w, s_invd[li], c);
        const int b = lj * kWin + li;
        atomicAdd(&win[b], (unsigned long long)c[0]);
        atomicAdd(&win[b + 1], (unsigned long long)c[1]);
        atomicAdd(&win[b + kWin], (unsigned long long)c[2]);
        atomicAdd(&win[b + kWin + 1], (unsigned long long)c[3]);
        return 0u;
    }
    node_shares(L, (double)w, radial_factor(L.i), c);
    const int n00 = L.j * g.w + L.i;
    atomicAdd(&dep[n00], (unsigned long long)c[0]);
    atomicAdd(&dep[n00 + 1], (unsigned long long)c[1]);
    atomicAdd(&dep[n00 + g.w], (unsigned long long)c[2]);
    atomicAdd(&dep[n00 + g.w + 1], (unsigned long long)c[3]);
    return 1u;
}

// slot p of this step: in place, or through the permutation of a deferred
// sort.  Unconditional (no branch, so the loads stay where they are
// issued): a slot beyond the last, n - 1, is read in its place and the
// caller ignores it.  Needs n >= 1.  In place the state is read once, in
// order, so it streams past the caches (non-temporal), leaving them to the
// grids; through a permutation the lines of the old order are picked
// several times and stay cached.
template <bool kMoved>
__device__ __forceinline__ P9 load_slot(const Species& f, const Species& src, const uint32_t* perm, long long p,
                                        long long n) {
    const uint32_t q = (uint32_t)(p < n ? p : n - 1);
    if (kMoved) return load9(src, perm[q]);
    const f32x4 x = __builtin_nontemporal_load(&f.a[q]), y = __builtin_nontemporal_load(&f.b[q]);
    P9 s;
    s.r = x.x; s.z = x.y; s.vr = x.z; s.vt = x.w;
    s.vz = y.x; s.ar = y.y; s.at = y.z; s.az = y.w;
    s.w = __builtin_nontemporal_load(&f.w[q]);
    return s;
}

// One time step for every particle of one species.  A block of eight
// wavefronts owns one chunk of 8192 consecutive slots and each of its
// wavefronts a contiguous slice of 1024 of them, processed 64 at a time
// with the next 64 already in flight; every live slot is stored once per
// round.  A colliding particle scatters in its own round, on its lane
// alone (about one lane in thirty collides per step, and the kernel waits
// on memory far more than on arithmetic), then is predicted and deposited
// with the others; births are staged per slice in slot order.  A window (the tile of a particle from
// the middle of the chunk plus halo) lives in LDS: E at its nodes, the
// radial factors of its columns and the kinds of its cells are read there,
// and the deposit goes there, flushed at the end.  So the only global
// traffic of a particle inside the window is its own state.
template <int kHalo, bool kMoved, bool kKeys>
__global__ __launch_bounds__(kPushBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_particles(PushArgs a) {
    constexpr int kWin = win_nodes(kHalo);
    __shared__ unsigned long long win[kWin * kWin];
    __shared__ float2 ewin[kWin * kWin];
    __shared__ double s_invd[kWin];
    __shared__ uint8_t s_ck[(kWin - 1) * (kWin - 1)];
    __shared__ uint32_t s_vt[kVacWords];
    __shared__ int s_org[2];
    __shared__ unsigned long long s_abs[kSlots];
    __shared__ unsigned int s_coll[4];
    __shared__ unsigned int s_fallback;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const Geo& g = a.g;
    const long long n = a.ctr->n_slots[a.sp];
    const long long nch = (n + kPushChunk - 1) / kPushChunk;
    // one block per chunk: the grid has ceil(capacity / chunk) blocks and
    // n never exceeds the capacity (a single pass rather than a loop over
    // chunks, so nothing of the setup below is kept live across one)
    const Species& f = a.f;
    constexpr bool moved = kMoved;
    unsigned int fallback = 0;
    unsigned int ndead = 0;   // dead keys written (uniform in the wavefront)

    for (int k = tid; k < kWin * kWin; k += kPushBlock) win[k] = 0ull;
    if (tid < kSlots) s_abs[tid] = 0ull;
    if (tid < 4) s_coll[tid] = 0u;
    if (tid == 0) s_fallback = 0u;

    // the window's deposits go to the global grid (64-bit atomics) at the end
    int wi0 = -(1 << 28), wj0 = -(1 << 28);
    bool vac = false, have = false;
    auto flush = [&]() {
        __syncthreads();
        for (int k = tid; k < kWin * kWin; k += kPushBlock) {
            const unsigned long long v = win[k];
            if (v != 0ull) {
                const int gi = wi0 + k % kWin, gj = wj0 + k / kWin;
                if (gi >= 0 && gi <= g.nr && gj >= 0 && gj <= g.nz) atomicAdd(&a.dep[gj * g.w + gi], v);
                win[k] = 0ull;
            }
        }
        __syncthreads();
    };

    if (blockIdx.x < nch) {
        const long long chunk = blockIdx.x;
        const long long base = chunk * kPushChunk;
        // this wavefront's slice, whose first round is requested before the
        // window is probed and filled (its latency overlaps theirs)
        const long long sbase = base + (long long)wave * kSlice;
        // this lane's slot in round r (after the last round the last one's,
        // beyond the last slot the last slot: read and ignored)
        auto slot_in = [&](int r) -> long long {
            const long long q = sbase + (long long)min(r, kRounds - 1) * 64 + lane;
            return q < n ? q : n - 1;
        };
        P9 cur = load_slot<kMoved>(f, a.src, a.perm, sbase + lane, n);
        // after a deferred sort the permutation entries run two rounds
        // ahead: the entry of round r is requested in round r - 2, the state
        // it points to in round r - 1 (the wait for the entry then waits for
        // nothing issued since); here the entry of the second round (r = 1)
        uint32_t pq_next = kMoved ? a.perm[slot_in(1)] : 0u;
        // LDS window origin: tile of a live particle from the middle of the
        // chunk (else from its start), plus halo.  Sorted chunks that span
        // several tiles then keep both ends inside the window.
        if (wave == 0) {
            const long long mid = max(base, base + min((long long)kPushChunk, n - base) / 2 - 32);
            auto probe = [&](long long p, Loc& L) {
                if (p >= n) return false;
                const uint32_t q = kMoved ? a.perm[p] : (uint32_t)p;
                const f32x4 x = (kMoved ? a.src : f).a[q];
                const float r = x.x;
                L = locate(r, x.y, g);
                return (r >= 0.0f) && L.inside;
            };
            Loc Lm, Lb;
            const bool okm = probe(mid + lane, Lm), okb = probe(base + lane, Lb);
            const unsigned long long mm = __ballot(okm), mb = __ballot(okb);
            const unsigned long long m = mm ? mm : mb;
            const int first = m ? __ffsll((long long)m) - 1 : -1;
            if (lane == first) {
                const Loc& L = mm ? Lm : Lb;
                s_org[0] = ((L.i >> kTileShift) << kTileShift) - kHalo;
                s_org[1] = ((L.j >> kTileShift) << kTileShift) - kHalo;
            }
            if (first < 0 && lane == 0) { s_org[0] = -(1 << 28); s_org[1] = -(1 << 28); }
        }
        __syncthreads();
        {
            wi0 = s_org[0];
            wj0 = s_org[1];
            have = true;
            // the window's copies of E, of the radial factors and of the
            // cell kinds (zero outside the domain); are all its domain
            // cells vacuum?  A thread requests all its values before it
            // stores the first, so their latencies overlap.
            constexpr int kNE = (kWin * kWin + kPushBlock - 1) / kPushBlock;
            constexpr int kNC = ((kWin - 1) * (kWin - 1) + kPushBlock - 1) / kPushBlock;
            static_assert(kWin <= kPushBlock, "one radial factor per thread");
            float2 ev[kNE];
            uint32_t cv[kNC];
            double dv = 0.0;
#pragma unroll
            for (int q = 0; q < kNE; ++q) {
                const int k = tid + q * kPushBlock;
                const int gi = wi0 + k % kWin, gj = wj0 + k / kWin;
                ev[q] = make_float2(0.0f, 0.0f);
                if (k < kWin * kWin && gi >= 0 && gi <= g.nr && gj >= 0 && gj <= g.nz) ev[q] = a.E[gj * g.w + gi];
            }
#pragma unroll
            for (int q = 0; q < kNC; ++q) {
                const int k = tid + q * kPushBlock;
                const int ci = wi0 + k % (kWin - 1), cj = wj0 + k / (kWin - 1);
                cv[q] = 0u;
                if (k < (kWin - 1) * (kWin - 1) && ci >= 0 && ci < g.nr && cj >= 0 && cj < g.nz)
                    cv[q] = g.cell_kind[cj * g.nr + ci];
            }
            if (tid < kWin && wi0 + tid >= 0 && wi0 + tid < g.nr) dv = g.invd[wi0 + tid];
            static_assert(kVacWords <= kPushBlock, "one bitmap word per thread");
            const uint32_t vtw = tid < kVacWords ? g.vac_tiles[tid] : 0u;
#pragma unroll
            for (int q = 0; q < kNE; ++q)
                if (tid + q * kPushBlock < kWin * kWin) ewin[tid + q * kPushBlock] = ev[q];
            if (tid < kWin) s_invd[tid] = dv;
            if (tid < kVacWords) s_vt[tid] = vtw;
            bool cells_ok = true;
#pragma unroll
            for (int q = 0; q < kNC; ++q)
                if (tid + q * kPushBlock < (kWin - 1) * (kWin - 1)) {
                    s_ck[tid + q * kPushBlock] = (uint8_t)cv[q];
                    if (cv[q] != 0u) cells_ok = false;
                }
            vac = __syncthreads_and(cells_ok) != 0;
        }

        // Cell-index range (in units of cells, FP32) whose positions are
        // certainly inside the domain and whose cell, computed exactly, is
        // certainly inside the window: one cell of margin on every side,
        // far above the FP32 error of r / dr.  In a vacuum window a
        // corrected position in this range is not absorbed, without the
        // exact location.
        const float fxlo = (float)(wi0 + 1), fxhi = (float)min(wi0 + kWin - 2, g.nr - 1);
        const float fylo = (float)max(wj0 + 1, 1), fyhi = (float)min(wj0 + kWin - 2, g.nz - 1);

        const long long stage_row = chunk * kPushWaves + wave;
        int nb = 0;

        uint4 dec4 = make_uint4(0u, 0u, 0u, 0u);
        for (int it = 0; it < kRounds; ++it) {
            const long long p = sbase + (long long)it * 64 + lane;
            P9 s = cur;
            const bool live = p < n && s.r >= 0.0f;
            // E at the particle's position: its cell and weights, and for a
            // cell outside the window the four nodes from the global grid,
            // requested before the next round's state (waiting for them then
            // does not wait for that state)
            const EW ew = e_weights(g, s.r, s.z);
            const int eli = ew.i - wi0, elj = ew.j - wj0;
            const bool eout = live && !((unsigned)eli < (unsigned)(kWin - 1) && (unsigned)elj < (unsigned)(kWin - 1));
            float2 eg[4];
            if (eout) {
                const int n00 = ew.j * g.w + ew.i;
                eg[0] = a.E[n00];
                eg[1] = a.E[n00 + 1];
                eg[2] = a.E[n00 + g.w];
                eg[3] = a.E[n00 + g.w + 1];
            }
            // the next round's state is requested here and pinned by a
            // scheduling barrier, so its latency hides behind this round
            uint32_t pq_after = 0u;
            P9 nxt;
            if (kMoved) {
                pq_after = a.perm[slot_in(it + 2)];
                nxt = load9(a.src, pq_next);
            } else {
                nxt = load_slot<false>(f, a.src, a.perm, it + 1 < kRounds ? p + 64 : p, n);
            }
            __builtin_amdgcn_sched_barrier(0);
            // decision words of this lane's slots in rounds it .. it+3 (sbase is
            // a multiple of 256, so the four share one counter)
            if ((it & 3) == 0) dec4 = draw(decision_ctr((uint32_t)p), a.step, kPurposeDecide, a.sp, 0, a.key0, a.key1);
            const uint32_t dword = (it & 3) == 0 ? dec4.x : (it & 3) == 1 ? dec4.y : (it & 3) == 2 ? dec4.z : dec4.w;
            bool born = false;
            uint32_t key = a.dead_key;
            float b6[6], br = 0.0f, bz = 0.0f;
            if (live) {
                float Er, Ez;
                {
                    // read in the window (clamped into it), then replaced by
                    // the global grid's values for a cell outside the window
                    const int b = min(max(elj, 0), kWin - 2) * kWin + min(max(eli, 0), kWin - 2);
                    e_combine(ew, ewin[b], ewin[b + 1], ewin[b + kWin], ewin[b + kWin + 1], Er, Ez);
                }
                if (eout) e_combine(ew, eg[0], eg[1], eg[2], eg[3], Er, Ez);
                d1_correct(s, Er, Ez, a.qm, a.dt);
                const float cx = s.r * g.inv_dr, cy = s.z * g.inv_dz;
                bool gone = false;
                if (!(vac && cx >= fxlo && cx < fxhi && cy >= fylo && cy < fyhi)) {
                    const Loc L = locate(s.r, s.z, g);
                    gone = absorb<kWin>(g, L, s.w, a.sign, s_abs, a.wallq, vac, wi0, wj0, s_ck, s_vt);
                }
                if (gone) {
                    s.r = -1.0f;
                } else {
                    // a collider scatters at its corrected position (only
                    // these lanes run the collision), then moves on with
                    // the others
                    if (dword < a.m.thresh) {
                        const uint4 x = draw((uint32_t)p, a.step, kPurposeMcc, a.sp, 0, a.key0, a.key1);
                        const int proc = collide(a.sp, x, s.vr, s.vt, s.vz, a.m, (uint32_t)p, a.step, a.key0, a.key1,
                                                 b6, &a.ctr->viol);
                        atomicAdd(&s_coll[proc], 1u);
                        born = proc == 2 && a.stage != nullptr;
                        br = s.r;
                        bz = s.z;
                    }
                    d1_predict(s, a.dt);
                    const Loc L2 = locate(s.r, s.z, g);
                    if (absorb<kWin>(g, L2, s.w, a.sign, s_abs, a.wallq, vac, wi0, wj0, s_ck, s_vt)) {
                        s.r = -1.0f;
                    } else {
                        fallback += deposit<kWin>(g, L2, s.w, win, s_invd, wi0, wj0, a.dep);
                        key = tile_key(L2, a.kmul);
                    }
                }
            }
            // one store per round for every slot: the predicted state, r = -1
            // for a removed particle, a dead slot's state unchanged; a lane
            // past the last slot writes the sink.  The stores are issued by
            // every wavefront in every round, so the compiler counts them
            // exactly: the wait for the next round's state above then lets
            // them stay in flight.
            {
                const bool in = p < n;
                // (a choice between two computed addresses: a choice between
                // the arrays' pointers becomes a per-lane load of the pointer)
                auto pick = [&](auto* base, auto* sink) {
                    return reinterpret_cast<decltype(base)>(in ? reinterpret_cast<uintptr_t>(base + p)
                                                               : reinterpret_cast<uintptr_t>(sink + lane));
                };
                __builtin_nontemporal_store(group_a(s), pick(f.a, a.sink.a));
                __builtin_nontemporal_store(group_b(s), pick(f.b, a.sink.b));
                if (moved) __builtin_nontemporal_store(s.w, pick(f.w, a.sink.w));
                // the key of the tile sort that follows: the tile of the
                // predicted position, or the dead key (as the key pass
                // computes it)
                if (kKeys) {
                    *pick(a.keys, a.ksink) = (tkey_t)key;
                    ndead += __popcll(__ballot(in && key == a.dead_key));
                }
            }
            // births of this round, staged in slot order
            const unsigned long long bm = __ballot(born);
            if (born) {
                const int idx = nb + __popcll(bm & lanemask_lt());
                if (idx < a.stage_w) {
                    Birth bb;
                    bb.r = br; bb.z = bz; bb.w = s.w;
                    for (int k = 0; k < 6; ++k) bb.v[k] = b6[k];
                    a.stage[stage_row * a.stage_w + idx] = bb;
                } else {
                    atomicOr(&a.ctr->err, kErrStage);
                }
            }
            nb += __popcll(bm);
            cur = nxt;
            pq_next = pq_after;
        }
        if (lane == 0 && a.stage_cnt != nullptr) a.stage_cnt[stage_row] = min(nb, a.stage_w);
    }
    if (have) flush();
    for (int o = 32; o > 0; o >>= 1) fallback += __shfl_down(fallback, o);
    if (lane == 0 && fallback) atomicAdd(&s_fallback, fallback);
    __syncthreads();
    if (tid < kSlots && s_abs[tid]) atomicAdd(&a.ctr->absorbed[a.sp][tid], s_abs[tid]);
    if (tid < 4 && s_coll[tid]) atomicAdd(&a.ctr->coll[a.sp][tid], (unsigned long long)s_coll[tid]);
    if (tid == 0 && s_fallback) atomicAdd(&a.ctr->fallback, (unsigned long long)s_fallback);
    if (kKeys) {
        if (lane == 0 && ndead) atomicAdd(&a.ctr->dead[a.sp], ndead);
        if (blockIdx.x == 0 && tid == 0) a.ctr->n_keyed[a.sp] = n;
    }
}

// one block per chunk of the species' capacity (blocks past the last slot
// exit at once): the hardware dispatches them in order, which keeps the
// chunks in flight close together and balances uneven chunks (colliders,
// window misses) better than a persistent grid
static unsigned grid_blocks(const pic_handle* h, int sp) {
    return (unsigned)std::max<int64_t>(1, (h->cap[sp] + kPushChunk - 1) / kPushChunk);
}

static Geo make_geo(pic_handle* h) {
    Geo g;
    g.nr = h->nr; g.nz = h->nz; g.w = h->w;
    g.R = h->cfg.geom.R; g.Z = h->cfg.geom.Z; g.Sr = h->Sr; g.Sz = h->Sz;
    g.inv_dr = (float)(1.0 / h->dr); g.inv_dz = (float)(1.0 / h->dz);
    g.invd = h->invd;
    g.cell_kind = h->cell_kind;
    g.vac_tiles = h->vac_tiles;
    g.ntr = h->ntr;
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

void launch_particles(pic_handle* h, int sp, bool emit_keys) {
    PushArgs a;
    a.g = make_geo(h);
    a.m = make_mcc(h, sp);
    // a deferred sort is applied on the way: read through the permutation,
    // write the other buffer
    const bool moved = h->pending[sp];
    a.src = h->buf[sp][h->cur[sp]];
    a.f = h->buf[sp][moved ? 1 - h->cur[sp] : h->cur[sp]];
    a.perm = moved ? h->perm[sp] : nullptr;
    a.E = h->E;
    a.dep = h->dep[h->dep_cur][sp];
    a.wallq = h->wallq;
    a.ctr = h->ctr;
    a.stage = sp == 0 ? h->stage : nullptr;
    a.stage_cnt = sp == 0 ? h->stage_cnt : nullptr;
    a.stage_w = h->stage_w;
    a.sp = sp;
    a.sign = sp == 0 ? -1 : 1;
    a.qm = qm_of(sp);
    a.dt = (float)h->dt;
    a.key0 = (uint32_t)(h->cfg.run.seed & 0xFFFFFFFFu);
    a.key1 = (uint32_t)(h->cfg.run.seed >> 32);
    a.step = (uint32_t)(h->step + 1);
    a.keys = emit_keys ? (sp == 0 ? h->keys[0] : h->keys_ion) : nullptr;
    a.sink = h->sink;
    a.ksink = h->ksink;
    a.dead_key = (uint32_t)(h->ntz * h->kmul);
    a.kmul = h->kmul;
    const dim3 grid(grid_blocks(h, sp)), block(kPushBlock);
    if (sp == 0) {
        if (emit_keys) {
            if (moved) hipLaunchKernelGGL((k_particles<24, true, true>), grid, block, 0, h->stream, a);
            else hipLaunchKernelGGL((k_particles<24, false, true>), grid, block, 0, h->stream, a);
        } else {
            if (moved) hipLaunchKernelGGL((k_particles<24, true, false>), grid, block, 0, h->stream, a);
            else hipLaunchKernelGGL((k_particles<24, false, false>), grid, block, 0, h->stream, a);
        }
    } else {
        if (emit_keys) {
            if (moved) hipLaunchKernelGGL((k_particles<16, true, true>), grid, block, 0, h->stream, a);
            else hipLaunchKernelGGL((k_particles<16, false, true>), grid, block, 0, h->stream, a);
        } else {
            if (moved) hipLaunchKernelGGL((k_particles<16, true, false>), grid, block, 0, h->stream, a);
            else hipLaunchKernelGGL((k_particles<16, false, false>), grid, block, 0, h->stream, a);
        }
    }
    if (moved) {
        h->cur[sp] = 1 - h->cur[sp];
        h->pending[sp] = false;
    }
}

// ---------------------------------------------------------------- births
// Births are appended in parent-slot order: the staged counts of the
// (chunk, wavefront) rows are summed per segment of 1024 rows (coalesced),
// the segment sums are scanned by one block (which also checks capacity and
// sets the append bases), and the append kernel scans each segment locally.
constexpr int kSegRows = 1024;

__global__ __launch_bounds__(kSegRows) void k_birth_segsum(const DevCounters* c, const int* cnt, int* segsum) {
    __shared__ int sh[kSegRows / 64];
    const long long rows = stage_rows(c->n_slots[0]);
    const long long nseg = (rows + kSegRows - 1) / kSegRows;
    for (long long b = blockIdx.x; b < nseg; b += gridDim.x) {
        const long long i = b * kSegRows + threadIdx.x;
        int v = (i < rows) ? cnt[i] : 0;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = 0;
            for (int w = 0; w < kSegRows / 64; ++w) t += sh[w];
            segsum[b] = t;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void k_birth_scan(DevCounters* c, const int* segsum, int* segoff, long long cap_e,
                                                     long long cap_i) {
    __shared__ long long s_part[1024];
    const int tid = threadIdx.x;
    const long long rows = stage_rows(c->n_slots[0]);
    const long long nseg = (rows + kSegRows - 1) / kSegRows;
    long long carry = 0;
    for (long long b0 = 0; b0 < nseg; b0 += 1024) {
        const long long i = b0 + tid;
        const long long v = (i < nseg) ? segsum[i] : 0;
        s_part[tid] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const long long t = (tid >= o) ? s_part[tid - o] : 0;
            __syncthreads();
            s_part[tid] += t;
            __syncthreads();
        }
        if (i < nseg) segoff[i] = (int)(carry + s_part[tid] - v);
        carry += s_part[1023];
        __syncthreads();
    }
    if (tid == 0) {
        long long B = carry;
        c->base[0] = c->n_slots[0];
        c->base[1] = c->n_slots[1];
        c->nch_births = rows;
        if (c->n_slots[0] + B > cap_e || c->n_slots[1] + B > cap_i) {
            atomicOr(&c->err, kErrBirths);
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
    Species fe;
    Species fi;
    unsigned long long* dep_e;
    unsigned long long* dep_i;
    unsigned long long* wallq;
    DevCounters* ctr;
    const Birth* stage;
    const int* cnt;
    const int* segoff;
    int stage_w;
    float dt;
};

// Newborn electron and ion: a_bar = 0, predict, absorption, deposit.
__device__ __forceinline__ void place_newborn(const Geo& g, const Species& f, long long slot, P9 s, float dt,
                                              int sp, unsigned long long* dep, unsigned long long* wallq,
                                              DevCounters* ctr) {
    d1_predict(s, dt);
    Loc L = locate(s.r, s.z, g);
    bool removed;
    {
        unsigned long long loc[kSlots] = {0ull, 0ull, 0ull, 0ull, 0ull, 0ull, 0ull, 0ull};
        // absorption accounting straight to the global counters (rare)
        if (L.inside && g.cell_kind[L.j * g.nr + L.i] == 0) {
            removed = false;
        } else {
            removed = true;
            if (!L.inside) {
                int bc = g.edge_bc[L.edge];
                loc[bc >= 0 ? slot_of(bc) : 2] += (unsigned long long)total_share((double)s.w);
            } else {
                int ck = g.cell_kind[L.j * g.nr + L.i];
                if (ck >= 2) {
                    loc[slot_of(ck - 2)] += (unsigned long long)total_share((double)s.w);
                } else {
                    int64_t c[4];
                    node_shares(L, (double)s.w, g.invd[L.i], c);
                    int n00 = L.j * g.w + L.i;
                    int nodes[4] = {n00, n00 + 1, n00 + g.w, n00 + g.w + 1};
                    for (int k = 0; k < 4; ++k) {
                        int nk = g.node_kind[nodes[k]];
                        if (nk >= 0) loc[slot_of(nk)] += (unsigned long long)c[k];
                        else {
                            atomicAdd(&wallq[nodes[k]], (unsigned long long)((sp == 0 ? -1 : 1) * c[k]));
                            loc[3] += (unsigned long long)c[k];
                        }
                    }
                }
            }
            for (int k = 0; k < kSlots; ++k)
                if (loc[k]) atomicAdd(&ctr->absorbed[sp][k], loc[k]);
        }
    }
    if (removed) s.r = -1.0f;
    store9(f, (uint32_t)slot, s);
    if (!removed) {
        int64_t c[4];
        node_shares(L, (double)s.w, g.invd[L.i], c);
        int n00 = L.j * g.w + L.i;
        atomicAdd(&dep[n00], (unsigned long long)c[0]);
        atomicAdd(&dep[n00 + 1], (unsigned long long)c[1]);
        atomicAdd(&dep[n00 + g.w], (unsigned long long)c[2]);
        atomicAdd(&dep[n00 + g.w + 1], (unsigned long long)c[3]);
    }
}

__global__ __launch_bounds__(kSegRows) void k_birth_append(BirthArgs a) {
    __shared__ int sh[kSegRows];
    const long long rows = a.ctr->nch_births;
    if (a.ctr->births_step == 0) return;
    const long long be = a.ctr->base[0], bi = a.ctr->base[1];
    const long long nseg = (rows + kSegRows - 1) / kSegRows;
    for (long long b = blockIdx.x; b < nseg; b += gridDim.x) {
        const long long row = b * kSegRows + threadIdx.x;
        const int cnt = (row < rows) ? a.cnt[row] : 0;
        sh[threadIdx.x] = cnt;
        __syncthreads();
        for (int o = 1; o < kSegRows; o <<= 1) {
            const int t = ((int)threadIdx.x >= o) ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        // the segment's births, spread over the block: birth idx (in row
        // order) belongs to the first row whose inclusive count exceeds idx
        // and goes to slot base + segoff + idx
        const int total = sh[kSegRows - 1];
        const long long o0 = (long long)a.segoff[b];
        for (int idx = threadIdx.x; idx < total; idx += kSegRows) {
            int lo = 0, hi = kSegRows - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (sh[mid] > idx) hi = mid; else lo = mid + 1;
            }
            const int k = idx - (lo > 0 ? sh[lo - 1] : 0);
            const Birth bb = a.stage[(b * kSegRows + lo) * a.stage_w + k];
            P9 e;
            e.r = bb.r; e.z = bb.z; e.vr = bb.v[0]; e.vt = bb.v[1]; e.vz = bb.v[2];
            e.ar = 0.0f; e.at = 0.0f; e.az = 0.0f; e.w = bb.w;
            place_newborn(a.g, a.fe, be + o0 + idx, e, a.dt, 0, a.dep_e, a.wallq, a.ctr);
            P9 i = e;
            i.vr = bb.v[3]; i.vt = bb.v[4]; i.vz = bb.v[5];
            place_newborn(a.g, a.fi, bi + o0 + idx, i, a.dt, 1, a.dep_i, a.wallq, a.ctr);
        }
        __syncthreads();   // sh is rewritten by the next segment
    }
}

void launch_births(pic_handle* h) {
    hipLaunchKernelGGL(k_birth_segsum, dim3(256), dim3(kSegRows), 0, h->stream, (const DevCounters*)h->ctr,
                       (const int*)h->stage_cnt, h->stage_off);
    hipLaunchKernelGGL(k_birth_scan, dim3(1), dim3(1024), 0, h->stream, h->ctr, (const int*)h->stage_off,
                       h->stage_segoff, (long long)h->cap[0], (long long)h->cap[1]);
    BirthArgs a;
    a.g = make_geo(h);
    a.fe = h->buf[0][h->cur[0]];
    a.fi = h->buf[1][h->cur[1]];
    a.dep_e = h->dep[h->dep_cur][0];
    a.dep_i = h->dep[h->dep_cur][1];
    a.wallq = h->wallq;
    a.ctr = h->ctr;
    a.stage = h->stage;
    a.cnt = h->stage_cnt;
    a.segoff = h->stage_segoff;
    a.stage_w = h->stage_w;
    a.dt = (float)h->dt;
    hipLaunchKernelGGL(k_birth_append, dim3(256), dim3(kSegRows), 0, h->stream, a);
}

// ------------------------------------------------------------------ loader
struct LoadArgs {
    Species f;
    const double* cdf;
    const int* cell;
    int nv, nr;
    double vvac, dr, dz;
    long long n;
    float W, vth;
    int sp;
    uint32_t key0, key1;
    int weights;              // PIC_WEIGHTS_CELL: cell uniform over vacuum cells, weight wt[column]
    const float* wt;
};

// Uniform plasma (Sec. 3, first paragraph): a vacuum cell by inverse CDF of
// cell volume (equal weights) or uniformly over the vacuum cells with the
// weight of the cell's column (unequal weights), r^2 and z uniform inside
// it, Maxwellian velocity.
__global__ __launch_bounds__(kBlock) void k_load(LoadArgs a) {
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < a.n;
         p += (long long)gridDim.x * blockDim.x) {
        uint4 x = draw((uint32_t)p, 0u, kPurposeLoad, a.sp, 0, a.key0, a.key1);
        uint4 y = draw((uint32_t)p, 0u, kPurposeLoad, a.sp, 1, a.key0, a.key1);
        int lo = 0;
        if (a.weights == PIC_WEIGHTS_CELL) {
            lo = min((int)floor((double)u01(x.x) * (double)a.nv), a.nv - 1);
        } else {
            const double target = (double)u01(x.x) * a.vvac;
            int hi = a.nv - 1;
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (a.cdf[mid] > target) hi = mid; else lo = mid + 1;
            }
        }
        int c = a.cell[lo];
        int ci = c % a.nr, cj = c / a.nr;
        double r0 = ci * a.dr, r1 = (ci + 1) * a.dr;
        double r = sqrt(r0 * r0 + (double)u01(x.y) * (r1 * r1 - r0 * r0));
        double z = (cj + (double)u01(x.z)) * a.dz;
        float vr, vt, vz;
        maxwell3(y, a.vth, vr, vt, vz);
        P9 s;
        s.r = (float)r; s.z = (float)z;
        s.vr = vr; s.vt = vt; s.vz = vz;
        s.ar = 0.0f; s.at = 0.0f; s.az = 0.0f;
        s.w = a.weights == PIC_WEIGHTS_CELL ? a.wt[ci] : a.W;
        store9(a.f, (uint32_t)p, s);
    }
}

void launch_load(pic_handle* h, int sp, const double* cdf, const int* cell, int nv, double vvac, int64_t n,
                 float W, float vth) {
    LoadArgs a;
    a.f = h->buf[sp][h->cur[sp]];
    a.cdf = cdf; a.cell = cell; a.nv = nv; a.nr = h->nr;
    a.vvac = vvac; a.dr = h->dr; a.dz = h->dz;
    a.n = n; a.W = W; a.vth = vth; a.sp = sp;
    a.key0 = (uint32_t)(h->cfg.run.seed & 0xFFFFFFFFu);
    a.key1 = (uint32_t)(h->cfg.run.seed >> 32);
    a.weights = h->cfg.run.weights;
    a.wt = h->wtcol[sp];
    if (n > 0) hipLaunchKernelGGL(k_load, dim3(2048), dim3(kBlock), 0, h->stream, a);
}

// First prediction after the load (a_bar = 0), absorption and deposit; or,
// with predict = 0, a plain deposit of the stored positions.
struct PDArgs {
    Geo g;
    Species f;
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
        P9 s = load9(a.f, (uint32_t)p);
        if (!(s.r >= 0.0f)) continue;
        if (a.predict) {
            place_newborn(a.g, a.f, p, s, a.dt, a.sp, a.dep, a.wallq, a.ctr);
        } else {
            Loc L = locate(s.r, s.z, a.g);
            if (!L.inside) continue;
            int64_t c[4];
            node_shares(L, (double)s.w, a.g.invd[L.i], c);
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
    a.f = h->buf[sp][h->cur[sp]];
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

struct MomArgs {
    Geo g;
    Species f;
    const long long* n_slots;
    int sp;
    double half_m_over_e;
    unsigned long long *N, *E;
};

__global__ __launch_bounds__(kBlock) void k_count_alive(const f32x4* ra, const long long* n_slots, int sp,
                                                        unsigned long long* out) {
    __shared__ unsigned int s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const long long n = n_slots[sp];
    unsigned int c = 0;
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < n;
         p += (long long)gridDim.x * blockDim.x)
        c += (ra[p].x >= 0.0f);
    atomicAdd(&s_cnt, c);
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out, (unsigned long long)s_cnt);
}

// Energy moment of one species at the stored positions and velocities v*:
// node sums of the deposit shares c_k and of c_k floor(16 eps / eV) with
// eps = (m / 2e)((v_r^2 + v_t^2) + v_z^2) evaluated in FP64 (capped at 2^20).
// Integer sums: order-independent.
__global__ __launch_bounds__(kBlock) void k_moments(MomArgs a) {
#pragma clang fp contract(off)
    const long long n = a.n_slots[a.sp];
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < n;
         p += (long long)gridDim.x * blockDim.x) {
        const P9 s = load9(a.f, (uint32_t)p);
        if (!(s.r >= 0.0f)) continue;
        const Loc L = locate(s.r, s.z, a.g);
        if (!L.inside) continue;
        int64_t c[4];
        node_shares(L, (double)s.w, a.g.invd[L.i], c);
        const double vr = s.vr, vt = s.vt, vz = s.vz;
        double v2 = vr * vr;
        v2 = v2 + vt * vt;
        v2 = v2 + vz * vz;
        const double eq = floor(a.half_m_over_e * v2 * 16.0);
        const long long q = eq < 1048576.0 ? (long long)eq : 1048576ll;
        const int n00 = L.j * a.g.w + L.i;
        const int nodes[4] = {n00, n00 + 1, n00 + a.g.w, n00 + a.g.w + 1};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            atomicAdd(&a.N[nodes[k]], (unsigned long long)c[k]);
            atomicAdd(&a.E[nodes[k]], (unsigned long long)(c[k] * q));
        }
    }
}

void launch_moments(pic_handle* h, int sp, unsigned long long* N, unsigned long long* E) {
    MomArgs a;
    a.g = make_geo(h);
    a.f = h->buf[sp][h->cur[sp]];
    a.n_slots = (const long long*)h->ctr->n_slots;
    a.sp = sp;
    const double QE = 1.602176634e-19, ME = 9.1093837015e-31, MAR = 39.948 * 1.66053906660e-27;
    a.half_m_over_e = 0.5 * (sp == 0 ? ME : MAR) / QE;
    a.N = N;
    a.E = E;
    launch_zero_u64(N, (size_t)h->nn, h->stream);
    launch_zero_u64(E, (size_t)h->nn, h->stream);
    hipLaunchKernelGGL(k_moments, dim3(2048), dim3(kBlock), 0, h->stream, a);
}

int launch_count_alive(pic_handle* h, long long* out2) {
    // uses the pad words of the device counters as scratch
    unsigned long long* d = (unsigned long long*)&h->ctr->pad[0];
    launch_zero_u64(d, 2, h->stream);
    for (int sp = 0; sp < 2; ++sp)
        hipLaunchKernelGGL(k_count_alive, dim3(512), dim3(kBlock), 0, h->stream, (const f32x4*)h->buf[sp][h->cur[sp]].a,
                           (const long long*)h->ctr->n_slots, sp, d + sp);
    if (hipMemcpyAsync(out2, d, 2 * sizeof(long long), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
        return PIC_E_HIP;
    return PIC_OK;
}

}  // namespace pic
