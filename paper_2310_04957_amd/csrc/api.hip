// api.hip -- the C ABI of include/pic.h: configuration checks, geometry,
// workspace layout, the multigrid plan, and the time-step driver that queues
// the kernels of particles.hip, sort.hip and field.hip on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "pic_internal.h"

using namespace pic;

namespace {

constexpr double kQE = 1.602176634e-19;
constexpr double kME = 9.1093837015e-31;
constexpr double kMAr = 39.948 * 1.66053906660e-27;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kKB = 1.380649e-23;
constexpr double kPi = 3.14159265358979323846;
constexpr int64_t kMaxSlots = (1LL << 30) - 16;   // slot indices and sort permutations are 32-bit

// Fixed scratch of the allocation-free entry points: two int64 node grids
// (the energy moments' N and E), one copy per GPU for the process's life.
// Host code never uses the array's name as an address: each device's copy
// is found once with hipGetSymbolAddress, with that device current.
constexpr size_t kNoAllocNodes = PIC_NOALLOC_MAX_NODES;
__device__ __align__(256) unsigned long long scratch[2 * kNoAllocNodes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long* g_scratch_ptr[kMaxDevices];

// the current device's copy of the scratch array (nullptr on failure)
unsigned long long* noalloc_scratch() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[dev] = static_cast<unsigned long long*>(p);
    }
    return g_scratch_ptr[dev];
}

#define HIP_OK(x)                               \
    do {                                        \
        if ((x) != hipSuccess) return PIC_E_HIP; \
    } while (0)

int validate(const pic_config* c) {
    if (!c || c->abi_version != PIC_ABI_VERSION) return PIC_E_CONFIG;
    const pic_geometry& g = c->geom;
    if (g.nr < 4 || g.nz < 4 || (g.nr & 1) || (g.nz & 1) || g.nr > 4096 || g.nz > 4096) return PIC_E_CONFIG;
    // 16-bit sort keys: the tiles and the dead key after them
    if (((g.nr + kTile - 1) / kTile) * ((g.nz + kTile - 1) / kTile) > 65535) return PIC_E_CONFIG;
    if (!(g.R > 0) || !(g.Z > 0) || g.n_regions < 0 || g.n_regions > PIC_MAX_REGIONS) return PIC_E_CONFIG;
    if (c->n_el < 0 || c->n_el > PIC_MAX_ELECTRODES) return PIC_E_CONFIG;
    const int n_el = c->n_el > 0 ? c->n_el : 1;
    for (int k = 0; k < 3; ++k)
        if (g.edge_bc[k] < -1 || g.edge_bc[k] > n_el) return PIC_E_CONFIG;
    for (int k = 0; k < g.n_regions; ++k) {
        const pic_region& r = g.regions[k];
        if (r.kind < 0 || r.kind > 2) return PIC_E_CONFIG;
        if (r.kind == PIC_COND && (r.cond_id < 0 || r.cond_id > n_el)) return PIC_E_CONFIG;
        if (r.kind == PIC_DIEL && !(r.eps_r >= 1.0)) return PIC_E_CONFIG;
    }
    for (int e = 0; e < n_el; ++e) {
        const pic_circuit& ci = e == 0 ? c->circ : c->circ_el[e - 1];
        if (!(ci.freq > 0) || ci.kind < 0 || ci.kind > 2 || ci.substeps < 1) return PIC_E_CONFIG;
        if (ci.kind == PIC_LMATCH && !(ci.C_m1 > 0 && ci.C_m2 > 0 && ci.L_m > 0 && ci.R_s > 0 && ci.C_stray > 0 &&
                                       ci.L_stray > 0))
            return PIC_E_CONFIG;
        if (ci.kind == PIC_SERIES_RLC && !(ci.C_b > 0 && ci.L_b > 0)) return PIC_E_CONFIG;
    }
    const pic_run& r = c->run;
    if (r.steps_per_period < 1 || r.n_e < 0 || r.n_i < 0 || r.cap_e < r.n_e || r.cap_i < r.n_i) return PIC_E_CONFIG;
    if (r.weights < PIC_WEIGHTS_EQUAL || r.weights > PIC_WEIGHTS_CELL || r.split < 0 || r.split > 1) return PIC_E_CONFIG;
    if (r.cap_e > kMaxSlots || r.cap_i > kMaxSlots || r.sort_every < 0 || r.sort_every_ion < 0)
        return PIC_E_CONFIG;
    if (!(c->gas.p_Pa >= 0) || !(c->gas.T_gas_K > 0) || !(r.n0 >= 0)) return PIC_E_CONFIG;
    if (c->solver.method < 0 || c->solver.method > 3 || !(c->solver.tol > 0) || c->solver.max_iter < 1)
        return PIC_E_CONFIG;
    const int ub = c->solver.unet_batch, up = c->solver.unet_pairs;
    if (ub < 0 || ub > unet::kMaxBatch || up < 0 || up > unet::kMaxPairs) return PIC_E_CONFIG;
    if (c->solver.method == PIC_SOLVE_IR_UNET && ub == 0) return PIC_E_CONFIG;
    if (ub > 0 && ((g.nr % 16) || (g.nz % 16))) return PIC_E_CONFIG;
    return PIC_OK;
}

// the network sees nodes i < nr, j < nz: the rest must be conductors
int unet_geometry_ok(const pic_handle* h) {
    if (h->cfg.solver.unet_batch == 0) return PIC_OK;
    for (int j = 0; j <= h->nz; ++j)
        for (int i = 0; i <= h->nr; ++i)
            if ((i == h->nr || j == h->nz) && h->h_node_kind[(size_t)j * h->w + i] < 0) return PIC_E_CONFIG;
    return PIC_OK;
}

// He-normal initial weights from a splitmix64 stream (Box-Muller), zero biases
uint64_t splitmix64(uint64_t& x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
double unit_open(uint64_t& x) { return ((double)(splitmix64(x) >> 11) + 0.5) * 0x1.0p-53; }

std::vector<float> unet_initial_params(const unet::Net& n, uint64_t seed) {
    std::vector<float> p((size_t)n.nparam, 0.0f);
    uint64_t st = seed;
    auto normal = [&]() {
        const double u = unit_open(st), v = unit_open(st);
        return std::sqrt(-2.0 * std::log(u)) * std::cos(2.0 * kPi * v);
    };
    for (int k = 0; k < unet::kConvs; ++k) {
        const unet::Conv& c = n.conv[k];
        const double sd = std::sqrt(2.0 / (9.0 * c.cin));
        for (size_t e = 0; e < (size_t)9 * unet::kC * c.cin; ++e) p[c.woff + e] = (float)(sd * normal());
    }
    for (int e = 0; e < unet::kC; ++e) p[n.out_w + e] = (float)(std::sqrt(1.0 / unet::kC) * normal());
    return p;
}

// cross sections for the electron null-collision bound (analytic argon
// stand-ins: elastic, excitation 11.5 eV, ionisation 15.76 eV)
double sigma_total_e(double eps) {
    double el = 1.0e-19 / std::sqrt(1.0 + eps / 10.0);
    double ex = (eps > 11.5) ? 2.7e-20 * std::log(eps / 11.5) / (eps / 11.5) : 0.0;
    double io = (eps > 15.76) ? 8.0e-20 * std::log(eps / 15.76) / (eps / 15.76) : 0.0;
    return el + ex + io;
}

void derive(pic_handle* h) {
    const pic_config& c = h->cfg;
    h->nr = c.geom.nr; h->nz = c.geom.nz; h->w = h->nr + 1;
    h->n_el = c.n_el > 0 ? c.n_el : 1;
    h->nn = (h->nr + 1) * (h->nz + 1);
    h->ncell = h->nr * h->nz;
    h->dr = c.geom.R / h->nr;
    h->dz = c.geom.Z / h->nz;
    h->dt = 1.0 / (c.circ.freq * c.run.steps_per_period);
    h->Sr = std::ldexp(1.0, kFBits) / h->dr;
    h->Sz = std::ldexp(1.0, kFBits) / h->dz;
    h->ntr = (h->nr + kTile - 1) / kTile;
    h->ntz = (h->nz + kTile - 1) / kTile;
    h->ntiles = h->ntr * h->ntz;
    // tile keys ty kmul + tx, the dead key ntz kmul after them: kmul the
    // tiles per row rounded up to a power of two 2^row_bits when the tile
    // column and the tile row (dead key included) each fit one 8-bit radix
    // digit, so each pass sorts one coordinate (a wavefront of nearly sorted
    // keys then holds few distinct digits); else the tiles per row, sorted in
    // 8-bit digits.  The tile order, and so the sort, is the same.
    int rb = 0;
    while ((1 << rb) < h->ntr) ++rb;
    if (rb >= 1 && rb <= 8 && h->ntz <= 255) {
        h->kmul = 1 << rb;
        h->row_bits = rb;
    } else {
        h->kmul = h->ntr;
        h->row_bits = 0;
    }
    int bits = 1;
    while ((1u << bits) <= (unsigned)(h->ntz * h->kmul)) ++bits;   // keys 0 .. ntz kmul (dead)
    h->key_bits = bits;
    h->cap[0] = c.run.cap_e;
    h->cap[1] = c.run.cap_i;
    int64_t capmax = std::max<int64_t>(std::max(h->cap[0], h->cap[1]), 1);
    h->max_chunks = (capmax + kChunk - 1) / kChunk;
    h->max_rows = stage_rows(capmax);
    // null-collision constants (Vahedi & Surendra 1995)
    h->n_gas = c.gas.p_Pa / (kKB * c.gas.T_gas_K);
    const int N = 2000000;
    double best = 0.0;
    for (int k = 0; k < N; ++k) {
        double eps = std::pow(10.0, -4.0 + 9.0 * (double)k / (double)(N - 1));
        double sv = sigma_total_e(eps) * std::sqrt(2.0 * kQE * eps / kME);
        best = std::max(best, sv);
    }
    h->nu_max[0] = h->n_gas * best * 1.001;
    const double gmax = std::sqrt(2.0 * kQE * 2000.0 / kMAr) + 5.0 * std::sqrt(kKB * c.gas.T_gas_K / kMAr);
    h->nu_max[1] = h->n_gas * (5.0e-19 + 5.0e-19) * gmax;
    h->vth_gas = std::sqrt(kKB * c.gas.T_gas_K / kMAr);
    for (int sp = 0; sp < 2; ++sp) {
        double P = -std::expm1(-h->nu_max[sp] * h->dt);
        double T = std::floor(P * 4294967296.0);
        h->thresh[sp] = (T >= 4294967295.0) ? 0xFFFFFFFFu : (uint32_t)T;
    }
    // births of a 1024-slot slice are at most its null-collision candidates,
    // binomial(1024, P): the row holds the mean plus eight standard
    // deviations plus 32, in whole 64s
    {
        const double P = (double)h->thresh[0] * 0x1p-32, m = kSlice * P;
        const double need = m + 8.0 * std::sqrt(m * (1.0 - P)) + 32.0;
        h->stage_w = std::min(kSlice, std::max(kStageWMin, ((int)std::ceil(need) + 63) / 64 * 64));
    }
}

}  // namespace

namespace pic {

// Cells: the last region containing the centre; nodes: conductor if an
// adjacent cell is a conductor or it lies on a conductor edge, ground
// winning over the driven electrode where both touch.  Host only.
int host_geometry(pic_handle* h) {
    const pic_geometry& g = h->cfg.geom;
    const int nr = h->nr, nz = h->nz, w = h->w;
    h->h_cell_kind.assign((size_t)nr * nz, 0);
    std::vector<double> eps((size_t)nr * nz, 1.0);
    for (int j = 0; j < nz; ++j)
        for (int i = 0; i < nr; ++i) {
            const double rc = (i + 0.5) * h->dr, zc = (j + 0.5) * h->dz;
            uint8_t kind = 0;
            double e = 1.0;
            for (int k = 0; k < g.n_regions; ++k) {
                const pic_region& q = g.regions[k];
                if (rc >= q.r0 && rc < q.r1 && zc >= q.z0 && zc < q.z1) {
                    if (q.kind == PIC_COND) { kind = (uint8_t)(2 + q.cond_id); e = 1.0; }
                    else if (q.kind == PIC_DIEL) { kind = 1; e = q.eps_r; }
                    else { kind = 0; e = 1.0; }
                }
            }
            h->h_cell_kind[(size_t)j * nr + i] = kind;
            eps[(size_t)j * nr + i] = e;
        }
    h->h_node_kind.assign((size_t)h->nn, -1);
    for (int j = 0; j <= nz; ++j)
        for (int i = 0; i <= nr; ++i) {
            // conductor ids 0 .. kMaxEl (validated); the lowest id touching
            // the node wins, so ground wins
            bool touch[1 + kMaxEl] = {};
            for (int cj = j - 1; cj <= j; ++cj)
                for (int ci = i - 1; ci <= i; ++ci) {
                    if (ci < 0 || cj < 0 || ci >= nr || cj >= nz) continue;
                    const uint8_t k = h->h_cell_kind[(size_t)cj * nr + ci];
                    if (k >= 2) touch[k - 2] = true;
                }
            if (i == nr && g.edge_bc[0] >= 0) touch[g.edge_bc[0]] = true;
            if (j == 0 && g.edge_bc[1] >= 0) touch[g.edge_bc[1]] = true;
            if (j == nz && g.edge_bc[2] >= 0) touch[g.edge_bc[2]] = true;
            int8_t kind = -1;
            for (int k = kMaxEl; k >= 0; --k)
                if (touch[k]) kind = (int8_t)k;
            h->h_node_kind[(size_t)j * w + i] = kind;
        }
    // node volumes: half of each adjacent annulus (r^2 weights), half again on z edges
    h->h_vol.assign((size_t)h->nn, 0.0);
    h->h_gr.assign((size_t)h->nn, 0.0);
    h->h_gz.assign((size_t)h->nn, 0.0);
    const double dr = h->dr, dz = h->dz;
    for (int j = 0; j <= nz; ++j)
        for (int i = 0; i <= nr; ++i) {
            const double rlo = (i > 0) ? (i - 1) * dr : 0.0;
            const double ri = i * dr;
            const double rhi = (i < nr) ? (i + 1) * dr : ri;
            double v = (i == 0) ? kPi * dz * dr * dr * 0.5 : kPi * dz * (rhi * rhi - rlo * rlo) * 0.5;
            if (j == 0 || j == nz) v *= 0.5;
            const size_t n = (size_t)j * w + i;
            h->h_vol[n] = v;
            // finite-volume faces over the node control volume
            if (i < nr) {
                const double hz = (j == 0 || j == nz) ? 0.5 * dz : dz;
                double e = 0.0, cnt = 0.0;
                if (j > 0) { e += eps[(size_t)(j - 1) * nr + i]; cnt += 1.0; }
                if (j < nz) { e += eps[(size_t)j * nr + i]; cnt += 1.0; }
                h->h_gr[n] = 2.0 * kPi * (i + 0.5) * dr * hz * kEps0 * (e / cnt) / dr;
            }
            if (j < nz) {
                const double a = (i > 0) ? (i - 0.5) * dr : 0.0;
                const double b = (i < nr) ? (i + 0.5) * dr : h->cfg.geom.R;
                double num = 0.0;
                if (i > 0) num += eps[(size_t)j * nr + i - 1] * (ri * ri - a * a);
                if (i < nr) num += eps[(size_t)j * nr + i] * (b * b - ri * ri);
                h->h_gz[n] = kPi * (b * b - a * a) * kEps0 * (num / (b * b - a * a)) / dz;
            }
        }
    return PIC_OK;
}

int upload_geometry(pic_handle* h) {
    std::vector<double> invd((size_t)h->nr);
    for (int i = 0; i < h->nr; ++i) invd[i] = std::ldexp(1.0, -2 * kFBits) / (double)(2 * i + 1);
    hipStream_t s = h->stream;
    HIP_OK(hipMemcpyAsync(h->cell_kind, h->h_cell_kind.data(), h->h_cell_kind.size(), hipMemcpyHostToDevice, s));
    // tiles whose cells are all vacuum (the particle kernel answers the
    // absorption test of a cell outside its window from this bitmap)
    std::vector<uint32_t> vt(kVacWords, 0u);
    for (int t = 0; t < std::min(h->ntiles, 32 * kVacWords); ++t) {
        const int ti = t % h->ntr, tj = t / h->ntr;
        bool vac = true;
        for (int j = tj * kTile; j < std::min((tj + 1) * kTile, h->nz) && vac; ++j)
            for (int i = ti * kTile; i < std::min((ti + 1) * kTile, h->nr); ++i)
                if (h->h_cell_kind[(size_t)j * h->nr + i] != 0) { vac = false; break; }
        if (vac) vt[t >> 5] |= 1u << (t & 31);
    }
    HIP_OK(hipMemcpyAsync(h->vac_tiles, vt.data(), vt.size() * 4, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(h->node_kind, h->h_node_kind.data(), h->h_node_kind.size(), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(h->vol, h->h_vol.data(), h->h_vol.size() * 8, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(h->gr, h->h_gr.data(), h->h_gr.size() * 8, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(h->gz, h->h_gz.data(), h->h_gz.size() * 8, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(h->invd, invd.data(), invd.size() * 8, hipMemcpyHostToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
    return PIC_OK;
}

// Level sizes: coarsen in z only while cells are much wider in r (strong
// axial coupling), in r only in the opposite case, else in both; stop at
// kCoarsestNodes nodes or fewer.  A grid too small to coarsen gets one
// identity level so the coarse solve is exact.
int mg_plan(pic_handle* h) {
    int nr = h->nr, nz = h->nz;
    double dr = h->dr, dz = h->dz;
    int l = 0;
    h->lv[0].nr = nr; h->lv[0].nz = nz;
    for (;;) {
        const long nn = (long)(nr + 1) * (nz + 1);
        if (nn <= kCoarsestNodes || l + 1 >= kMaxLevels) break;
        const bool can_r = (nr % 2 == 0) && nr >= 4, can_z = (nz % 2 == 0) && nz >= 4;
        int cr = 1, cz = 1;
        if (dr > 1.5 * dz) { if (can_z) cz = 2; else if (can_r) cr = 2; }
        else if (dz > 1.5 * dr) { if (can_r) cr = 2; else if (can_z) cz = 2; }
        else { if (can_r) cr = 2; if (can_z) cz = 2; }
        if (cr == 1 && cz == 1) break;
        h->lv[l].cr = cr; h->lv[l].cz = cz;
        nr /= cr; nz /= cz; dr *= cr; dz *= cz;
        ++l;
        h->lv[l].nr = nr; h->lv[l].nz = nz;
    }
    if (l == 0) {
        h->lv[0].cr = h->lv[0].cz = 1;
        l = 1;
        h->lv[1].nr = nr; h->lv[1].nz = nz;
    }
    h->nlev = l + 1;
    for (int k = 0; k < h->nlev; ++k) {
        h->lv[k].w = h->lv[k].nr + 1;
        h->lv[k].nn = h->lv[k].w * (h->lv[k].nz + 1);
    }
    h->lv[h->nlev - 1].cr = h->lv[h->nlev - 1].cz = 1;
    // activity of the coarsest nodes follows the injection chain from level 0
    int cnr = h->lv[h->nlev - 1].nr, cnz = h->lv[h->nlev - 1].nz;
    int cnt = 0;
    for (int J = 0; J <= cnz; ++J)
        for (int I = 0; I <= cnr; ++I) {
            int i = I, j = J;
            for (int k = h->nlev - 2; k >= 0; --k) { i *= h->lv[k].cr; j *= h->lv[k].cz; }
            if (h->h_node_kind[(size_t)j * h->w + i] < 0) ++cnt;
        }
    if (cnt > kMaxCoarse) return PIC_E_CONFIG;
    h->ncoarse = cnt;
    return PIC_OK;
}

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Carver {
    char* base;
    size_t off = 0;
    template <typename T>
    T* take(size_t count) {
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += align_up(std::max<size_t>(count, 1) * sizeof(T));
        return p;
    }
};

size_t layout(pic_handle* h, char* base) {
    Carver c{base};
    const size_t nn = (size_t)h->nn, nc = (size_t)h->ncell;
    h->cell_kind = c.take<uint8_t>(nc);
    h->vac_tiles = c.take<uint32_t>(kVacWords);
    h->node_kind = c.take<int8_t>(nn);
    h->vol = c.take<double>(nn);
    h->gr = c.take<double>(nn);
    h->gz = c.take<double>(nn);
    h->invd = c.take<double>((size_t)h->nr);
    for (int sp = 0; sp < 2; ++sp) h->wtcol[sp] = c.take<float>((size_t)h->nr);
    size_t capmax = (size_t)std::max<int64_t>(std::max(h->cap[0], h->cap[1]), 1);
    for (int sp = 0; sp < 2; ++sp)
        for (int b = 0; b < 2; ++b) {
            const size_t cs = (size_t)std::max<int64_t>(h->cap[sp], 1);
            h->buf[sp][b].a = c.take<f32x4>(cs);
            h->buf[sp][b].b = c.take<f32x4>(cs);
            h->buf[sp][b].w = c.take<float>(cs);
        }
    for (int b = 0; b < 2; ++b) {
        h->keys[b] = c.take<tkey_t>(capmax);
        h->idx[b] = c.take<uint32_t>(capmax);
    }
    for (int sp = 0; sp < 2; ++sp) h->perm[sp] = c.take<uint32_t>((size_t)std::max<int64_t>(h->cap[sp], 1));
    h->keys_ion = c.take<tkey_t>((size_t)std::max<int64_t>(h->cap[1], 1));
    h->sink.a = c.take<f32x4>(64);
    h->sink.b = c.take<f32x4>(64);
    h->sink.w = c.take<float>(64);
    h->ksink = c.take<tkey_t>(64);
    const size_t mch = (size_t)h->max_chunks;
    h->hist = c.take<uint32_t>(256 * mch);
    h->bsum = c.take<uint32_t>((256 * mch + 4095) / 4096 + 1);
    h->split_off = c.take<long long>(mch + 1);
    const size_t mrows = (size_t)h->max_rows;
    h->stage = c.take<Birth>(mrows * h->stage_w);
    h->stage_cnt = c.take<int>(mrows);
    h->stage_off = c.take<int>(mrows / 1024 + 2);
    h->stage_segoff = c.take<int>(mrows / 1024 + 2);
    for (int b = 0; b < 2; ++b)
        for (int sp = 0; sp < 2; ++sp) h->dep[b][sp] = c.take<unsigned long long>(nn);
    h->wallq = c.take<unsigned long long>(nn);
    for (int sp = 0; sp < 2; ++sp) {
        h->psum[sp] = c.take<unsigned long long>(nn);
        h->plast[sp] = c.take<unsigned long long>(nn);
    }
    h->chi = c.take<double>(nn); h->Q = c.take<double>(nn);
    h->ar = c.take<double>(nn); h->az = c.take<double>(nn);
    h->phi = c.take<double>(nn); h->zeroQ = c.take<double>(nn);
    for (int e = 0; e < kMaxEl; ++e) h->phiL[e] = e < h->n_el ? c.take<double>(nn) : nullptr;
    h->phi_prev = c.take<double>(nn);
    h->phi_prev2 = c.take<double>(nn);
    h->ar32 = c.take<float>(nn); h->az32 = c.take<float>(nn);
    h->E = c.take<float2>(nn);
    h->r64 = c.take<double>(nn); h->x64 = c.take<double>(nn); h->z64 = c.take<double>(nn);
    h->p64 = c.take<double>(nn); h->q64 = c.take<double>(nn);
    h->r32 = c.take<float>(nn); h->x32 = c.take<float>(nn); h->z32 = c.take<float>(nn);
    h->p32 = c.take<float>(nn); h->q32 = c.take<float>(nn);
    h->part = c.take<double>(kMaxEl * kRedBlocks);
    // partials of the fused CG: r.z and p.q (one per level-0 tile of the
    // fused multigrid; 16-node tiles in FP64 are the most), r.r
    h->cgpart_n = std::max(((h->nr + 16) / 16) * ((h->nz + 16) / 16), kCgBlocks);
    h->cgpart = c.take<double>(3 * (size_t)h->cgpart_n);
    for (int l = 0; l < h->nlev; ++l) {
        Level& L = h->lv[l];
        const size_t m = (size_t)L.nn;
        for (int k = 0; k < 9; ++k) {
            L.A64[k] = (l > 0) ? c.take<double>(m) : nullptr;
            L.A32[k] = (l > 0) ? c.take<float>(m) : nullptr;
        }
        L.x64 = c.take<double>(m); L.y64 = c.take<double>(m); L.b64 = c.take<double>(m); L.res64 = c.take<double>(m);
        L.x32 = c.take<float>(m); L.y32 = c.take<float>(m); L.b32 = c.take<float>(m); L.res32 = c.take<float>(m);
    }
    const size_t cnn = (size_t)h->lv[h->nlev - 1].nn;
    h->cmap = c.take<int>(cnn + kMaxCoarse);
    h->cinv64 = c.take<double>((size_t)kMaxCoarse * kMaxCoarse);
    h->cinv32 = c.take<float>((size_t)kMaxCoarse * kMaxCoarse);
    const size_t spp = (size_t)h->cfg.run.steps_per_period;
    h->serU = c.take<double>(kMaxEl * spp); h->serI = c.take<double>(kMaxEl * spp);
    h->lastU = c.take<double>(kMaxEl * spp); h->lastI = c.take<double>(kMaxEl * spp);
    h->serVin = c.take<double>(spp); h->serI1 = c.take<double>(spp);
    h->lastVin = c.take<double>(spp); h->lastI1 = c.take<double>(spp);
    h->ctr = c.take<DevCounters>(1);
    h->sc = c.take<DevScalars>(1);
    h->unet_on = h->cfg.solver.unet_batch > 0;
    if (h->unet_on) {
        const int B = h->cfg.solver.unet_batch;
        h->hx64 = c.take<double>(h->cfg.solver.unet_pairs > 0 ? (size_t)unet::kHarvestPerSolve * nn : 1);
        h->unet_stage = c.take<float>((size_t)B * h->nr * h->nz * 3);
        c.off = (c.off + 255) & ~(size_t)255;
        c.off += unet::layout(h->net, h->nz, h->nr, B, h->cfg.solver.unet_pairs, base ? base + c.off : nullptr);
    }
    return c.off;
}

}  // namespace pic

namespace {

void ev_record(pic_handle* h, int phase, hipEvent_t* begin) {
    if (!h->timing) return;
    hipEvent_t e;
    if (h->ev_pool.empty()) {
        if (hipEventCreate(&e) != hipSuccess) return;
    } else {
        e = h->ev_pool.back();
        h->ev_pool.pop_back();
    }
    if (hipEventRecord(e, h->stream) != hipSuccess) {
        h->ev_pool.push_back(e);
        return;
    }
    if (phase < 0) {
        *begin = e;
    } else {
        h->ev_pending.push_back({phase, {*begin, e}});
    }
}

void ev_collect(pic_handle* h) {
    for (auto& p : h->ev_pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.second.first, p.second.second) == hipSuccess) h->ms[p.first] += ms;
        h->ev_pool.push_back(p.second.first);
        h->ev_pool.push_back(p.second.second);
    }
    h->ev_pending.clear();
}

struct InitCirc {
    double U0[kMaxEl];
    int n_el;
};

// initial electrode state: voltages U0 (an ideal source's DC value, else 0)
// held by the charges Q = C U + Q_P
__global__ void k_init_circuit(const double* part, DevScalars* s, const DevCounters* ctr, InitCirc ic) {
    __shared__ double a[kRedBlocks];
    __shared__ double qp[kMaxEl];
    for (int e = 0; e < ic.n_el; ++e) {
        for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) a[i] = part[e * kRedBlocks + i];
        __syncthreads();
        for (int o = kRedBlocks / 2; o > 0; o >>= 1) {
            for (int i = threadIdx.x; i < o; i += blockDim.x) a[i] += a[i + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) qp[e] = a[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int e = 0; e < ic.n_el; ++e) {
            s->Q_P[e] = qp[e];
            s->U_E[e] = ic.U0[e];
        }
        for (int e = 0; e < ic.n_el; ++e) {
            double q = 0.0;
            for (int f = 0; f < ic.n_el; ++f) q += s->Cm[e][f] * ic.U0[f];
            s->Q_E[e] = q + qp[e];
            const int sl = slot_of(e + 1);
            s->el_prev[e] = (double)((long long)ctr->absorbed[1][sl] - (long long)ctr->absorbed[0][sl]);
        }
    }
}

__global__ void k_set_slots(DevCounters* c, long long ne, long long ni) {
    c->n_slots[0] = ne;
    c->n_slots[1] = ni;
}

__global__ void k_set_state(DevScalars* s, double t, double QE, double UE, double c0, double c1, double c2, double c3,
                            double c4, double Ceq) {
    s->t = t; s->Q_E[0] = QE; s->U_E[0] = UE;
    s->circ[0][0] = c0; s->circ[0][1] = c1; s->circ[0][2] = c2; s->circ[0][3] = c3; s->circ[0][4] = c4;
    s->Cm[0][0] = Ceq;
}

// identity rows: the Dirichlet values of the electrodes' Laplace problems
__global__ void k_set_units(DevScalars* s) {
    for (int e = 0; e < kMaxEl; ++e)
        for (int f = 0; f < kMaxEl; ++f) s->unit[e][f] = e == f ? 1.0 : 0.0;
}

struct Uvec {
    double U[kMaxEl];
};

__global__ void k_set_U(DevScalars* s, Uvec u) {
    for (int e = 0; e < kMaxEl; ++e) s->Uset[e] = u.U[e];
}

__global__ void k_set_cmap(int* cmap, const int* src, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) cmap[i] = src[i];
}

int build_cmap(pic_handle* h) {
    const Level& L = h->lv[h->nlev - 1];
    std::vector<int> m((size_t)L.nn + kMaxCoarse, -1);
    int cnt = 0;
    for (int J = 0; J <= L.nz; ++J)
        for (int I = 0; I <= L.nr; ++I) {
            int i = I, j = J;
            for (int k = h->nlev - 2; k >= 0; --k) { i *= h->lv[k].cr; j *= h->lv[k].cz; }
            if (h->h_node_kind[(size_t)j * h->w + i] < 0) {
                m[(size_t)J * L.w + I] = cnt;
                m[(size_t)L.nn + cnt] = J * L.w + I;
                ++cnt;
            }
        }
    HIP_OK(hipMemcpyAsync(h->cmap, m.data(), m.size() * sizeof(int), hipMemcpyHostToDevice, h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    return PIC_OK;
}

int load_plasma(pic_handle* h) {
    const pic_run& r = h->cfg.run;
    std::vector<double> cdf;
    std::vector<int> cell;
    double acc = 0.0;
    for (int j = 0; j < h->nz; ++j)
        for (int i = 0; i < h->nr; ++i) {
            if (h->h_cell_kind[(size_t)j * h->nr + i] != 0) continue;
            const double r0 = i * h->dr, r1 = (i + 1) * h->dr;
            acc += kPi * (r1 * r1 - r0 * r0) * h->dz;
            cdf.push_back(acc);
            cell.push_back(j * h->nr + i);
        }
    const double vvac = acc;
    h->w_unit = r.n0 * vvac / (double)(r.n_e > 0 ? r.n_e : 1);
    // reference weight of each cell column (splitting, unequal-weight load):
    // loading weight x column cell volume / mean vacuum-cell volume
    {
        const int64_t nreq[2] = {r.n_e, r.n_i};
        const double nv = (double)cdf.size();
        for (int sp = 0; sp < 2; ++sp) {
            const double wref = nreq[sp] > 0 ? (r.n0 * vvac / (double)nreq[sp]) / h->w_unit : 1.0;
            std::vector<float> wt((size_t)h->nr);
            for (int i = 0; i < h->nr; ++i) {
                const double r0 = i * h->dr, r1 = (i + 1) * h->dr;
                const double vi = kPi * (r1 * r1 - r0 * r0) * h->dz;
                wt[(size_t)i] = (float)(wref * vi * nv / vvac);
            }
            HIP_OK(hipMemcpyAsync(h->wtcol[sp], wt.data(), wt.size() * 4, hipMemcpyHostToDevice, h->stream));
        }
        HIP_OK(hipStreamSynchronize(h->stream));
    }
    h->qunit = kQE * h->w_unit * std::ldexp(1.0, -kKBits);
    const double base = 0.5 * h->dt * h->dt * kQE * kQE * h->w_unit * std::ldexp(1.0, -kKBits) / kEps0;
    h->chi_c[0] = base / kME;
    h->chi_c[1] = base / kMAr;
    if (!r.load || cdf.empty()) return PIC_OK;
    if ((size_t)cdf.size() > (size_t)h->nn) return PIC_E_CONFIG;
    // the solver vectors serve as upload space for the CDF
    double* d_cdf = h->r64;
    int* d_cell = reinterpret_cast<int*>(h->x64);
    HIP_OK(hipMemcpyAsync(d_cdf, cdf.data(), cdf.size() * 8, hipMemcpyHostToDevice, h->stream));
    HIP_OK(hipMemcpyAsync(d_cell, cell.data(), cell.size() * 4, hipMemcpyHostToDevice, h->stream));
    const int64_t n[2] = {r.n_e, r.n_i};
    const double T[2] = {r.Te_eV, r.Ti_eV}, M[2] = {kME, kMAr};
    for (int sp = 0; sp < 2; ++sp) {
        if (n[sp] <= 0) continue;
        const double W = (r.n0 * vvac / (double)n[sp]) / h->w_unit;
        const double vth = std::sqrt(kQE * T[sp] / M[sp]);
        launch_load(h, sp, d_cdf, d_cell, (int)cdf.size(), vvac, n[sp], (float)W, (float)vth);
    }
    HIP_OK(hipStreamSynchronize(h->stream));
    return PIC_OK;
}

// fundamental (k = 1) of N samples: X_1 = (2/N) sum x_n e^{-2 pi i n / N}
void fundamental(const std::vector<double>& x, double* re, double* im) {
    const int N = (int)x.size();
    double a = 0.0, b = 0.0;
    for (int n = 0; n < N; ++n) {
        const double ph = 2.0 * kPi * (double)n / (double)N;
        a += x[n] * std::cos(ph);
        b -= x[n] * std::sin(ph);
    }
    *re = a * 2.0 / N;
    *im = b * 2.0 / N;
}

// Electrical characterisation of the last RF period (Sec. 3, Eqs. 11-14).
// Voltages are samples at step ends, currents step averages, whose
// fundamental carries sinc(pi/N) e^{-i pi/N} relative to an end sample;
// impedances divide it out.  Powers are the period-averaged element energies.
void characterise(const pic_handle* h, const std::vector<double>& U, const std::vector<double>& I,
                  const std::vector<double>& Vin, const std::vector<double>& I1, const double* energy,
                  pic_diag_out* out) {
    const int N = (int)U.size();
    const double x = kPi / N, sinc = std::sin(x) / x;
    const std::complex<double> bias = std::polar(sinc, -x);
    double ur, ui, ir, ii, vr, vi, jr, ji;
    fundamental(U, &ur, &ui);
    fundamental(I, &ir, &ii);
    fundamental(Vin, &vr, &vi);
    fundamental(I1, &jr, &ji);
    const std::complex<double> zc = std::complex<double>(ur, ui) * bias / std::complex<double>(ir, ii);
    const std::complex<double> zl = std::complex<double>(vr, vi) * bias / std::complex<double>(jr, ji);
    out->Z_ccp_re = zc.real(); out->Z_ccp_im = zc.imag();
    out->Z_load_re = zl.real(); out->Z_load_im = zl.imag();
    const double T = 1.0 / h->cfg.circ.freq;
    out->P_source = energy[0] / T;
    out->P_Rs = energy[1] / T;
    out->P_imn = energy[2] / T;
    out->P_stray = energy[3] / T;
    out->P_ccp = energy[4] / T;
    const double Rs = h->cfg.circ.kind == PIC_LMATCH ? h->cfg.circ.R_s : 0.0;
    out->gamma_abs = Rs > 0.0 ? std::abs((zl - Rs) / (zl + Rs)) : 0.0;
    out->P_forward = out->P_source - out->P_Rs;
    out->P_ref = out->P_forward * out->gamma_abs * out->gamma_abs;
}

int sync_err(pic_handle* h) {
    if (hipStreamSynchronize(h->stream) != hipSuccess) return PIC_E_HIP;
    if (hipMemcpy(h->h_ctr, h->ctr, sizeof(DevCounters), hipMemcpyDeviceToHost) != hipSuccess) return PIC_E_HIP;
    if (h->h_ctr->err != 0) h->sticky_err = PIC_E_CAPACITY;
    return PIC_OK;
}

}  // namespace

extern "C" {

int pic_workspace_size(const pic_config* cfg, size_t* bytes_out) {
    if (!bytes_out) return PIC_E_ARG;
    int rc = validate(cfg);
    if (rc) return rc;
    pic_handle* h = new (std::nothrow) pic_handle();
    if (!h) return PIC_E_ARG;
    h->cfg = *cfg;
    derive(h);
    host_geometry(h);
    rc = unet_geometry_ok(h);
    if (rc == PIC_OK) rc = mg_plan(h);
    if (rc == PIC_OK) *bytes_out = layout(h, nullptr) + 256;
    delete h;
    return rc;
}

int pic_init(const pic_config* cfg, void* dev_workspace, size_t bytes, void* hip_stream, pic_handle** out) {
    if (!out || !dev_workspace) return PIC_E_ARG;
    *out = nullptr;
    size_t need = 0;
    int rc = pic_workspace_size(cfg, &need);
    if (rc) return rc;
    if (bytes < need) return PIC_E_ARG;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return PIC_E_NODEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return PIC_E_NODEVICE;
    pic_handle* h = new (std::nothrow) pic_handle();
    if (!h) return PIC_E_ARG;
    h->cfg = *cfg;
    h->stream = (hipStream_t)hip_stream;
    h->timing = cfg->run.timing != 0;
    derive(h);
    host_geometry(h);
    rc = mg_plan(h);
    if (rc) { delete h; return rc; }
    char* base = (char*)(((uintptr_t)dev_workspace + 255) & ~(uintptr_t)255);
    h->ws = base;
    h->ws_bytes = bytes;
    const size_t used = layout(h, base);
    if (used + (size_t)(base - (char*)dev_workspace) > bytes) { delete h; return PIC_E_ARG; }
    if (hipHostMalloc((void**)&h->h_sc, sizeof(DevScalars), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h->h_ctr, sizeof(DevCounters), hipHostMallocDefault) != hipSuccess) {
        pic_free(h);
        return PIC_E_HIP;
    }
    // zero the whole workspace with a fill kernel
    launch_zero_u64((unsigned long long*)base, used / 8, h->stream);
    rc = upload_geometry(h);
    if (rc == PIC_OK) rc = build_cmap(h);
    if (rc == PIC_OK) rc = load_plasma(h);
    if (rc) { pic_free(h); return rc; }
    const int64_t n0[2] = {cfg->run.load ? cfg->run.n_e : 0, cfg->run.load ? cfg->run.n_i : 0};
    hipLaunchKernelGGL(k_set_slots, dim3(1), dim3(1), 0, h->stream, h->ctr, (long long)n0[0], (long long)n0[1]);
    hipLaunchKernelGGL(k_set_units, dim3(1), dim3(1), 0, h->stream, h->sc);
    h->dep_cur = 0;
    h->cur[0] = h->cur[1] = 0;
    // first prediction (a_bar = 0) and deposit; the loaded plasma starts tile-sorted
    for (int sp = 0; sp < 2; ++sp) launch_predict_deposit(h, sp);
    launch_sort(h, 0);
    launch_sort(h, 1);
    // vacuum operator, multigrid, Laplace solution and C_eq (Eqs. 6-7)
    launch_faces(h);                 // chi = 0 from the zeroed workspace
    rc = refresh_laplace(h);
    if (rc) { pic_free(h); return rc; }
    // initial electrode charge: U_E(0) with the induced charge of the load
    launch_assemble(h);
    {
        InitCirc ic;
        ic.n_el = h->n_el;
        for (int e = 0; e < kMaxEl; ++e) ic.U0[e] = 0.0;
        for (int e = 0; e < h->n_el; ++e) {
            const pic_circuit& ce = e == 0 ? cfg->circ : cfg->circ_el[e - 1];
            ic.U0[e] = ce.kind == PIC_IDEAL_SOURCE ? ce.U_dc : 0.0;
        }
        hipLaunchKernelGGL(k_init_circuit, dim3(1), dim3(256), 0, h->stream, (const double*)h->part, h->sc,
                           (const DevCounters*)h->ctr, ic);
    }
    // the assembly above added the first deposit to the period sums: undo
    launch_zero_u64(h->psum[0], (size_t)h->nn, h->stream);
    launch_zero_u64(h->psum[1], (size_t)h->nn, h->stream);
    if (h->unet_on) {
        unet::Net& n = h->net;
        const std::vector<float> p0 = unet_initial_params(n, cfg->run.seed);
        if (hipMemcpyAsync(n.p, p0.data(), p0.size() * 4, hipMemcpyHostToDevice, h->stream) != hipSuccess) {
            pic_free(h);
            return PIC_E_HIP;
        }
        unet::pack_all(n, h->stream);
        h->img_free = 0;
        for (int j = 0; j < h->nz; ++j)
            for (int i = 0; i < h->nr; ++i) h->img_free += h->h_node_kind[(size_t)j * h->w + i] < 0;
    }
    rc = sync_err(h);
    if (rc) { pic_free(h); return rc; }
    *out = h;
    return PIC_OK;
}

int pic_step(pic_handle* h, int32_t nsteps) {
    if (!h) return PIC_E_ARG;
    if (nsteps < 0) return PIC_E_ARG;
    if (h->halted) return PIC_E_CAPACITY;
    const pic_config& c = h->cfg;
    const int spp = c.run.steps_per_period;
    for (int32_t k = 0; k < nsteps; ++k) {
        hipEvent_t b0 = nullptr, b1 = nullptr, b2 = nullptr, b3 = nullptr;
        ev_record(h, -1, &b0);
        launch_assemble(h);
        launch_faces(h);
        launch_circuit(h);
        int32_t it = 0;
        double rel = 0.0;
        h->harvest_now = h->harvest_every > 0 && h->step % h->harvest_every == 0;
        launch_extrapolate(h);
        int rc = field_solve(h, h->phi, h->Q, h->sc->U_E, c.solver.tol, c.solver.method, &it, &rel);
        h->harvest_now = false;
        h->solver_iters = it;
        h->solver_relres = rel;
        if (rc != PIC_OK) return rc;
        // the solve's residual read waited for the previous step's births:
        // if some did not fit, stop before this step moves any particle
        if (h->h_sc->cap_err & (kErrBirths | kErrStage)) {
            h->halted = true;
            h->sticky_err = PIC_E_CAPACITY;
            return PIC_E_CAPACITY;
        }
        launch_efield(h);
        ev_record(h, 4, &b0);
        h->dep_cur = 1 - h->dep_cur;
        ev_record(h, -1, &b1);
        // a species writes its sort keys in the particle step that its sort
        // ends (the ions into a key buffer of their own: the electrons' sort
        // runs first and uses the shared ones)
        const bool se_next = c.run.sort_every > 0 && (h->step + 1) % c.run.sort_every == 0;
        const bool si_next = c.run.sort_every_ion > 0 && (h->step + 1) % c.run.sort_every_ion == 0;
        launch_particles(h, 0, se_next);
        ev_record(h, 0, &b1);
        ev_record(h, -1, &b1);
        launch_particles(h, 1, si_next);
        ev_record(h, 1, &b1);
        ev_record(h, -1, &b2);
        launch_births(h);
        ev_record(h, 2, &b2);
        h->step++;
        const bool se = c.run.sort_every > 0 && h->step % c.run.sort_every == 0;
        const bool si = c.run.sort_every_ion > 0 && h->step % c.run.sort_every_ion == 0;
        if (se || si) {
            // deferred: the particles move during the next particle step
            ev_record(h, -1, &b3);
            // particle splitting runs at a species' tile sort, before it
            if (se && c.run.split) launch_split(h, 0);
            if (se) launch_sort(h, 0, true, true);
            if (si && c.run.split) launch_split(h, 1);
            if (si) launch_sort(h, 1, true, true);
            ev_record(h, 3, &b3);
        }
        if (h->step % spp == 0) {
            ev_record(h, -1, &b3);
            rc = refresh_laplace(h);
            if (rc) return rc;
            launch_period_roll(h);
            ev_record(h, 5, &b3);
            h->periods_done++;
            h->have_last = 1;
        }
        if (h->timing) h->timed_steps++;
    }
    if (hipGetLastError() != hipSuccess) return PIC_E_HIP;
    return PIC_OK;
}

int pic_reset_timers(pic_handle* h) {
    if (!h) return PIC_E_ARG;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return PIC_E_HIP;
    ev_collect(h);
    for (double& m : h->ms) m = 0.0;
    h->timed_steps = 0;
    return PIC_OK;
}

int pic_diag(pic_handle* h, pic_diag_out* out, const pic_diag_buffers* bufs) {
    if (!h || !out) return PIC_E_ARG;
    materialize(h, 0);
    materialize(h, 1);
    int rc = sync_err(h);
    if (rc) return rc;
    ev_collect(h);
    DevScalars sc;
    if (hipMemcpy(&sc, h->sc, sizeof(sc), hipMemcpyDeviceToHost) != hipSuccess) return PIC_E_HIP;
    const DevCounters& ct = *h->h_ctr;
    std::memset(out, 0, sizeof(*out));
    out->t = sc.t; out->U_E = sc.U_E[0]; out->Q_E = sc.Q_E[0]; out->C_eq = sc.Cm[0][0]; out->Q_P = sc.Q_P[0];
    out->I_ccp = sc.I_ccp[0]; out->dt = h->dt; out->w_unit = h->w_unit; out->n_gas = h->n_gas;
    for (int k = 0; k < 5; ++k) out->circ[k] = sc.circ[0][k];
    out->n_el = h->n_el;
    for (int e = 0; e < h->n_el; ++e) {
        out->U_el[e] = sc.U_E[e]; out->Q_el[e] = sc.Q_E[e]; out->QP_el[e] = sc.Q_P[e]; out->I_el[e] = sc.I_ccp[e];
        for (int f = 0; f < h->n_el; ++f) out->C_el[e * PIC_MAX_ELECTRODES + f] = sc.Cm[e][f];
        for (int sp = 0; sp < 2; ++sp) out->absorbed_el[sp][e] = (int64_t)ct.absorbed[sp][slot_of(e + 1)];
    }
    for (int sp = 0; sp < 2; ++sp) {
        out->nu_max[sp] = h->nu_max[sp];
        out->thresh[sp] = h->thresh[sp];
        out->n_slots[sp] = ct.n_slots[sp];
        for (int k = 0; k < 4; ++k) {
            out->absorbed[sp][k] = (int64_t)ct.absorbed[sp][k];
            out->coll[sp][k] = (int64_t)ct.coll[sp][k];
        }
    }
    long long alive[2] = {0, 0};
    rc = launch_count_alive(h, alive);
    if (rc) return rc;
    out->n_alive[0] = alive[0];
    out->n_alive[1] = alive[1];
    out->step = h->step;
    out->periods_done = h->periods_done;
    out->born = ct.born;
    out->numax_violations = ct.viol;
    out->solver_iters = h->solver_iters;
    out->solver_outer = h->solver_outer;
    out->solver_relres = h->solver_relres;
    out->ms_particles[0] = h->ms[0]; out->ms_particles[1] = h->ms[1];
    out->ms_births = h->ms[2]; out->ms_sort = h->ms[3]; out->ms_field = h->ms[4]; out->ms_refresh = h->ms[5];
    out->timed_steps = h->timed_steps;
    out->deposit_fallback = (int64_t)ct.fallback;
    out->error = h->sticky_err;
    out->unet_pairs = h->net.n_pairs;
    out->unet_fallbacks = h->unet_fallbacks;
    out->unet_applications = h->unet_apps;
    out->unet_disabled = h->unet_off ? 1 : 0;
    out->capacity_bits = h->h_ctr->err;
    out->split_added[0] = ct.split_added[0];
    out->split_added[1] = ct.split_added[1];
    const int spp = h->cfg.run.steps_per_period;
    std::vector<double> UA((size_t)kMaxEl * spp), IA((size_t)kMaxEl * spp);
    if (hipMemcpy(UA.data(), h->lastU, UA.size() * 8, hipMemcpyDeviceToHost) != hipSuccess) return PIC_E_HIP;
    if (hipMemcpy(IA.data(), h->lastI, IA.size() * 8, hipMemcpyDeviceToHost) != hipSuccess) return PIC_E_HIP;
    std::vector<double> U(UA.begin(), UA.begin() + spp), I(IA.begin(), IA.begin() + spp);
    if (h->have_last) {
        // harmonics 0..5 of each electrode's voltage and current
        for (int e = 0; e < h->n_el; ++e)
            for (int k = 0; k < 6; ++k) {
                double a = 0, b = 0, c = 0, d = 0;
                for (int n = 0; n < spp; ++n) {
                    const double ph = 2.0 * kPi * (double)k * (double)n / (double)spp;
                    const double u = UA[(size_t)e * spp + n], i = IA[(size_t)e * spp + n];
                    a += u * std::cos(ph); b -= u * std::sin(ph);
                    c += i * std::cos(ph); d -= i * std::sin(ph);
                }
                const double s = (k == 0) ? 1.0 / spp : 2.0 / spp;
                out->hU_re[e][k] = a * s; out->hU_im[e][k] = b * s;
                out->hI_re[e][k] = c * s; out->hI_im[e][k] = d * s;
            }
        std::vector<double> V(spp), J(spp);
        if (hipMemcpy(V.data(), h->lastVin, spp * 8, hipMemcpyDeviceToHost) != hipSuccess) return PIC_E_HIP;
        if (hipMemcpy(J.data(), h->lastI1, spp * 8, hipMemcpyDeviceToHost) != hipSuccess) return PIC_E_HIP;
        characterise(h, U, I, V, J, sc.last_energy, out);
        for (int k = 0; k < 6; ++k) {
            double a = 0, b = 0, c = 0, d = 0;
            for (int n = 0; n < spp; ++n) {
                const double ph = 2.0 * kPi * (double)k * (double)n / (double)spp;
                a += U[n] * std::cos(ph); b -= U[n] * std::sin(ph);
                c += I[n] * std::cos(ph); d -= I[n] * std::sin(ph);
            }
            const double s = (k == 0) ? 1.0 / spp : 2.0 / spp;
            out->harm_U_re[k] = a * s; out->harm_U_im[k] = b * s;
            out->harm_I_re[k] = c * s; out->harm_I_im[k] = d * s;
        }
    }
    if (bufs) {
        if (bufs->U_E) std::memcpy(bufs->U_E, U.data(), spp * 8);
        if (bufs->I_ccp) std::memcpy(bufs->I_ccp, I.data(), spp * 8);
        if (bufs->phi && hipMemcpy(bufs->phi, h->phi, (size_t)h->nn * 8, hipMemcpyDeviceToHost) != hipSuccess)
            return PIC_E_HIP;
        double* dens[2] = {bufs->n_e, bufs->n_i};
        for (int sp = 0; sp < 2; ++sp) {
            if (!dens[sp]) continue;
            std::vector<unsigned long long> s((size_t)h->nn);
            if (hipMemcpy(s.data(), h->plast[sp], (size_t)h->nn * 8, hipMemcpyDeviceToHost) != hipSuccess)
                return PIC_E_HIP;
            const double u = h->w_unit * std::ldexp(1.0, -kKBits) / spp;
            for (size_t n = 0; n < s.size(); ++n) dens[sp][n] = (double)(long long)s[n] * u / h->h_vol[n];
        }
    }
    return PIC_OK;
}

int pic_free(pic_handle* h) {
    if (!h) return PIC_E_ARG;
    // teardown: errors here cannot be acted on, the handle goes away regardless
    (void)hipStreamSynchronize(h->stream);
    ev_collect(h);
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    for (auto& g : h->cg_graph)
        for (hipGraphExec_t e : g)
            if (e) (void)hipGraphExecDestroy(e);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->h_sc) (void)hipHostFree(h->h_sc);
    if (h->h_ctr) (void)hipHostFree(h->h_ctr);
    delete h;
    return PIC_OK;
}

const char* pic_strerror(int code) {
    switch (code) {
    case PIC_OK: return "ok";
    case PIC_E_CONFIG: return "invalid configuration";
    case PIC_E_CAPACITY: return "particle capacity exceeded by births";
    case PIC_E_SOLVER: return "field solve did not converge";
    case PIC_E_HIP: return "HIP runtime error";
    case PIC_E_NONFINITE: return "non-finite value in the field solve";
    case PIC_E_STATE: return "call not valid in this state";
    case PIC_E_ARG: return "bad argument";
    case PIC_E_NODEVICE: return "no gfx950 device is current";
    case PIC_E_TOOBIG: return "grid larger than the allocation-free scratch";
    }
    return "unknown error";
}

int pic_get_particles(pic_handle* h, int32_t species, float* host9, int64_t* n) {
    if (!h || !host9 || !n || species < 0 || species > 1) return PIC_E_ARG;
    materialize(h, species);
    int rc = sync_err(h);
    if (rc) return rc;
    const int64_t m = h->h_ctr->n_slots[species];
    const size_t cap = (size_t)h->cap[species];
    const Species& S = h->buf[species][h->cur[species]];
    if (m > 0) {
        // the two vector groups through a host buffer, split into the
        // caller's nine arrays
        std::vector<float> g((size_t)m * 4);
        for (int grp = 0; grp < 2; ++grp) {
            if (hipMemcpy(g.data(), grp ? S.b : S.a, (size_t)m * 16, hipMemcpyDeviceToHost) != hipSuccess)
                return PIC_E_HIP;
            for (int k = 0; k < 4; ++k) {
                float* out = host9 + (size_t)(4 * grp + k) * cap;
                for (int64_t p = 0; p < m; ++p) out[p] = g[(size_t)p * 4 + k];
            }
        }
        if (hipMemcpy(host9 + 8 * cap, S.w, (size_t)m * 4, hipMemcpyDeviceToHost) != hipSuccess) return PIC_E_HIP;
    }
    *n = m;
    return PIC_OK;
}

int pic_set_particles(pic_handle* h, int32_t species, const float* host9, int64_t n) {
    if (!h || (!host9 && n > 0) || species < 0 || species > 1 || n < 0 || n > h->cap[species]) return PIC_E_ARG;
    h->pending[species] = false;   // the new particles replace the old, sorted or not
    if (hipStreamSynchronize(h->stream) != hipSuccess) return PIC_E_HIP;
    const Species& S = h->buf[species][h->cur[species]];
    if (n > 0) {
        std::vector<float> g((size_t)n * 4);
        for (int grp = 0; grp < 2; ++grp) {
            for (int k = 0; k < 4; ++k) {
                const float* in = host9 + (size_t)(4 * grp + k) * n;
                for (int64_t p = 0; p < n; ++p) g[(size_t)p * 4 + k] = in[p];
            }
            if (hipMemcpy(grp ? S.b : S.a, g.data(), (size_t)n * 16, hipMemcpyHostToDevice) != hipSuccess)
                return PIC_E_HIP;
        }
        if (hipMemcpy(S.w, host9 + 8 * (size_t)n, (size_t)n * 4, hipMemcpyHostToDevice) != hipSuccess)
            return PIC_E_HIP;
    }
    long long ns[2];
    DevCounters ct;
    if (hipMemcpy(&ct, h->ctr, sizeof(ct), hipMemcpyDeviceToHost) != hipSuccess) return PIC_E_HIP;
    ns[0] = ct.n_slots[0];
    ns[1] = ct.n_slots[1];
    ns[species] = n;
    hipLaunchKernelGGL(k_set_slots, dim3(1), dim3(1), 0, h->stream, h->ctr, ns[0], ns[1]);
    return hipStreamSynchronize(h->stream) == hipSuccess ? PIC_OK : PIC_E_HIP;
}

int pic_redeposit(pic_handle* h) {
    if (!h) return PIC_E_ARG;
    materialize(h, 0);
    materialize(h, 1);
    launch_redeposit(h);
    return hipStreamSynchronize(h->stream) == hipSuccess ? PIC_OK : PIC_E_HIP;
}

int pic_get_grid(pic_handle* h, int32_t which, void* host) {
    if (!h || !host) return PIC_E_ARG;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return PIC_E_HIP;
    const size_t nn = (size_t)h->nn;
    const void* src = nullptr;
    size_t bytes = nn * 8;
    switch (which) {
    case PIC_G_DEP_E: src = h->dep[h->dep_cur][0]; break;
    case PIC_G_DEP_I: src = h->dep[h->dep_cur][1]; break;
    case PIC_G_PHI: src = h->phi; break;
    case PIC_G_CHI: src = h->chi; break;
    case PIC_G_WALLQ: src = h->wallq; break;
    case PIC_G_PHI_L: src = h->phiL[0]; break;
    case PIC_G_PHI_L2:
    case PIC_G_PHI_L3:
    case PIC_G_PHI_L4:
        if (which - PIC_G_PHI_L2 + 1 >= h->n_el) return PIC_E_ARG;
        src = h->phiL[which - PIC_G_PHI_L2 + 1];
        break;
    case PIC_G_Q: src = h->Q; break;
    case PIC_G_AR: src = h->ar; break;
    case PIC_G_AZ: src = h->az; break;
    case PIC_G_ER:
    case PIC_G_EZ: {
        std::vector<float2> e(nn);
        if (hipMemcpy(e.data(), h->E, nn * sizeof(float2), hipMemcpyDeviceToHost) != hipSuccess) return PIC_E_HIP;
        float* o = (float*)host;
        for (size_t n = 0; n < nn; ++n) o[n] = (which == PIC_G_ER) ? e[n].x : e[n].y;
        return PIC_OK;
    }
    default: return PIC_E_ARG;
    }
    return hipMemcpy(host, src, bytes, hipMemcpyDeviceToHost) == hipSuccess ? PIC_OK : PIC_E_HIP;
}

int pic_set_grid(pic_handle* h, int32_t which, const void* host) {
    if (!h || !host) return PIC_E_ARG;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return PIC_E_HIP;
    void* dst = nullptr;
    switch (which) {
    case PIC_G_DEP_E: dst = h->dep[h->dep_cur][0]; break;
    case PIC_G_DEP_I: dst = h->dep[h->dep_cur][1]; break;
    case PIC_G_WALLQ: dst = h->wallq; break;
    case PIC_G_PHI: dst = h->phi; h->have_prev = 0; break;
    case PIC_G_PHI_L: dst = h->phiL[0]; break;
    default: return PIC_E_ARG;
    }
    return hipMemcpy(dst, host, (size_t)h->nn * 8, hipMemcpyHostToDevice) == hipSuccess ? PIC_OK : PIC_E_HIP;
}

int pic_sort_now(pic_handle* h, int32_t species, int64_t* perm_out) {
    if (!h || species < 0 || species > 1) return PIC_E_ARG;
    launch_sort(h, species);
    int rc = sync_err(h);
    if (rc) return rc;
    if (perm_out) {
        const int64_t n = h->h_ctr->n_slots[species];
        std::vector<uint32_t> p((size_t)std::max<int64_t>(n, 1));
        if (n > 0 && hipMemcpy(p.data(), h->perm[species], (size_t)n * 4, hipMemcpyDeviceToHost) != hipSuccess)
            return PIC_E_HIP;
        for (int64_t k = 0; k < n; ++k) perm_out[k] = p[k];
    }
    return PIC_OK;
}

int pic_split_now(pic_handle* h, int32_t species, int64_t* added) {
    if (!h || species < 0 || species > 1) return PIC_E_ARG;
    launch_split(h, species);
    int rc = sync_err(h);
    if (rc) return rc;
    const long long t = h->h_ctr->split_total;
    if (t < 0) return PIC_E_CAPACITY;
    if (added) *added = t;
    return PIC_OK;
}

int pic_solve_once_el(pic_handle* h, const double* Q, const double* chi, const double* U, double tol,
                      double* phi_inout, int32_t* iters, double* relres) {
    if (!h || !Q || !chi || !phi_inout || !U) return PIC_E_ARG;
    const size_t nn = (size_t)h->nn;
    if (hipMemcpyAsync(h->Q, Q, nn * 8, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(h->chi, chi, nn * 8, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(h->phi, phi_inout, nn * 8, hipMemcpyHostToDevice, h->stream) != hipSuccess)
        return PIC_E_HIP;
    Uvec u;
    for (int e = 0; e < kMaxEl; ++e) u.U[e] = e < h->n_el ? U[e] : 0.0;
    hipLaunchKernelGGL(k_set_U, dim3(1), dim3(1), 0, h->stream, h->sc, u);
    launch_faces(h);
    mg_rebuild(h);
    h->harvest_now = h->harvest_every > 0;
    h->have_prev = 0;
    int rc = field_solve(h, h->phi, h->Q, h->sc->Uset, tol, h->cfg.solver.method, iters, relres);
    h->harvest_now = false;
    if (hipMemcpy(phi_inout, h->phi, nn * 8, hipMemcpyDeviceToHost) != hipSuccess) return PIC_E_HIP;
    return rc;
}

int pic_solve_once(pic_handle* h, const double* Q, const double* chi, double U_E, double tol, double* phi_inout,
                   int32_t* iters, double* relres) {
    double U[kMaxEl] = {U_E, 0.0, 0.0, 0.0};
    return pic_solve_once_el(h, Q, chi, U, tol, phi_inout, iters, relres);
}

int pic_match_design(pic_handle* h, int32_t apply, double* out2) {
    if (!h || !out2) return PIC_E_ARG;
    pic_circuit& c = h->cfg.circ;
    if (c.kind != PIC_LMATCH) return PIC_E_CONFIG;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return PIC_E_HIP;
    double Ceq = 0.0;
    if (hipMemcpy(&Ceq, &h->sc->Cm[0][0], sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return PIC_E_HIP;
    // load: C_eq in parallel with the stray branch; the network's input
    // admittance j w C_m1 + 1/Z_b, Z_b = R_m + j w L_m + 1/(j w C_m2) + Z_load
    // = R_b + j X_b, equals 1/R_s iff R_b/(R_b^2 + X_b^2) = 1/R_s and
    // w C_m1 = X_b/(R_b^2 + X_b^2): X_b = sqrt(R_b (R_s - R_b)) > 0
    using cd = std::complex<double>;
    const double w = 2.0 * kPi * c.freq;
    const cd zc = 1.0 / cd(0.0, w * Ceq);
    const cd zs = cd(c.R_stray, w * c.L_stray) + 1.0 / cd(0.0, w * c.C_stray);
    const cd zl = zc * zs / (zc + zs);
    const double Rb = c.R_m + zl.real();
    if (!(Ceq > 0.0) || !(Rb > 0.0) || !(Rb < c.R_s)) return PIC_E_CONFIG;
    const double Xb = std::sqrt(Rb * (c.R_s - Rb));
    const double xc2 = w * c.L_m + zl.imag() - Xb;   // reactance 1/(w C_m2) the series branch needs
    if (!(xc2 > 0.0)) return PIC_E_CONFIG;
    out2[0] = Xb / (Rb * c.R_s) / w;
    out2[1] = 1.0 / (w * xc2);
    if (apply) {
        c.C_m1 = out2[0];
        c.C_m2 = out2[1];
    }
    return PIC_OK;
}

int pic_set_state(pic_handle* h, const double* st9) {
    if (!h || !st9) return PIC_E_ARG;
    hipLaunchKernelGGL(k_set_state, dim3(1), dim3(1), 0, h->stream, h->sc, st9[0], st9[1], st9[2], st9[3], st9[4],
                       st9[5], st9[6], st9[7], st9[8]);
    return hipStreamSynchronize(h->stream) == hipSuccess ? PIC_OK : PIC_E_HIP;
}

int pic_moments(pic_handle* h, int32_t species, int64_t* N, int64_t* E) {
    if (!h || !N || !E || species < 0 || species > 1) return PIC_E_ARG;
    materialize(h, species);
    // the solver's FP64 work vectors are free between steps and hold the sums
    unsigned long long* dN = reinterpret_cast<unsigned long long*>(h->x64);
    unsigned long long* dE = reinterpret_cast<unsigned long long*>(h->z64);
    launch_moments(h, species, dN, dE);
    HIP_OK(hipStreamSynchronize(h->stream));
    HIP_OK(hipMemcpy(N, dN, (size_t)h->nn * 8, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(E, dE, (size_t)h->nn * 8, hipMemcpyDeviceToHost));
    return PIC_OK;
}

int pic_moments_noalloc(pic_handle* h, int32_t species, int64_t* N, int64_t* E) {
    if (!h || !N || !E || species < 0 || species > 1) return PIC_E_ARG;
    if ((size_t)h->nn > kNoAllocNodes) return PIC_E_TOOBIG;
    unsigned long long* base = noalloc_scratch();
    if (!base) return PIC_E_HIP;
    materialize(h, species);
    unsigned long long* dN = base;
    unsigned long long* dE = base + kNoAllocNodes;
    launch_moments(h, species, dN, dE);   // clears the nn entries it uses with a fill kernel
    HIP_OK(hipStreamSynchronize(h->stream));
    HIP_OK(hipMemcpy(N, dN, (size_t)h->nn * 8, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(E, dE, (size_t)h->nn * 8, hipMemcpyDeviceToHost));
    return PIC_OK;
}

int pic_set_solver(pic_handle* h, const pic_solver* sv) {
    if (!h || !sv) return PIC_E_ARG;
    pic_config c = h->cfg;
    if (sv->unet_batch != c.solver.unet_batch || sv->unet_pairs != c.solver.unet_pairs) return PIC_E_CONFIG;
    c.solver = *sv;
    int rc = validate(&c);
    if (rc) return rc;
    h->cfg.solver = *sv;
    return PIC_OK;
}

// ---- learned preconditioner

int pic_unet_num_params(pic_handle* h, int64_t* n) {
    if (!h || !n) return PIC_E_ARG;
    if (!h->unet_on) return PIC_E_STATE;
    *n = h->net.nparam;
    return PIC_OK;
}

int pic_unet_set_params(pic_handle* h, const float* p, int64_t n) {
    if (!h || !p) return PIC_E_ARG;
    if (!h->unet_on) return PIC_E_STATE;
    if (n != h->net.nparam) return PIC_E_ARG;
    unet::Net& net = h->net;
    HIP_OK(hipMemcpyAsync(net.p, p, (size_t)n * 4, hipMemcpyHostToDevice, h->stream));
    // new weights start a new optimisation: Adam moments and step count reset
    // (the moment arrays are padded to 256 bytes, so whole 8-byte words fit)
    launch_zero_u64((unsigned long long*)net.m, ((size_t)n + 1) / 2, h->stream);
    launch_zero_u64((unsigned long long*)net.v, ((size_t)n + 1) / 2, h->stream);
    net.adam_t = 0;
    unet::pack_all(net, h->stream);
    h->unet_off = false;
    h->unet_strikes = 0;
    HIP_OK(hipStreamSynchronize(h->stream));
    return PIC_OK;
}

int pic_unet_get_params(pic_handle* h, float* p, int64_t n) {
    if (!h || !p) return PIC_E_ARG;
    if (!h->unet_on) return PIC_E_STATE;
    if (n != h->net.nparam) return PIC_E_ARG;
    HIP_OK(hipStreamSynchronize(h->stream));
    HIP_OK(hipMemcpy(p, h->net.p, (size_t)n * 4, hipMemcpyDeviceToHost));
    return PIC_OK;
}

static int unet_stage_inputs(pic_handle* h, const float* in3, int32_t batch) {
    unet::Net& n = h->net;
    const size_t npix = (size_t)batch * n.H * n.W;
    HIP_OK(hipMemcpyAsync(h->unet_stage, in3, npix * 3 * 4, hipMemcpyHostToDevice, h->stream));
    unet::input_from_f32(h->unet_stage, n.x0, npix, h->stream);
    return PIC_OK;
}

int pic_unet_forward(pic_handle* h, const float* in3, int32_t batch, float* out) {
    if (!h || !in3 || !out) return PIC_E_ARG;
    if (!h->unet_on) return PIC_E_STATE;
    if (batch < 1 || batch > h->net.B) return PIC_E_ARG;
    int rc = unet_stage_inputs(h, in3, batch);
    if (rc) return rc;
    unet::forward(h->net, batch, h->stream);
    HIP_OK(hipStreamSynchronize(h->stream));
    HIP_OK(hipMemcpy(out, h->net.out, (size_t)batch * h->net.H * h->net.W * 4, hipMemcpyDeviceToHost));
    return PIC_OK;
}

int pic_unet_grads(pic_handle* h, const float* in3, const float* target, const float* mask, int32_t batch,
                   float* grads, double* loss) {
    if (!h || !in3 || !target || !mask || !grads) return PIC_E_ARG;
    if (!h->unet_on) return PIC_E_STATE;
    unet::Net& n = h->net;
    if (batch < 1 || batch > n.B) return PIC_E_ARG;
    const size_t npix = (size_t)batch * n.H * n.W;
    double cnt = 0.0;
    for (size_t e = 0; e < npix; ++e) cnt += mask[e];
    if (!(cnt > 0.0)) return PIC_E_ARG;
    int rc = unet_stage_inputs(h, in3, batch);
    if (rc) return rc;
    HIP_OK(hipMemcpyAsync(n.target, target, npix * 4, hipMemcpyHostToDevice, h->stream));
    HIP_OK(hipMemcpyAsync(n.mask, mask, npix * 4, hipMemcpyHostToDevice, h->stream));
    unet::forward(n, batch, h->stream);
    unet::backward(n, batch, (float)(1.0 / cnt), h->stream);
    HIP_OK(hipStreamSynchronize(h->stream));
    HIP_OK(hipMemcpy(grads, n.g, (size_t)n.nparam * 4, hipMemcpyDeviceToHost));
    float l = 0.0f;
    HIP_OK(hipMemcpy(&l, n.sums, 4, hipMemcpyDeviceToHost));
    if (loss) *loss = l;
    return PIC_OK;
}

int pic_unet_harvest(pic_handle* h, int32_t every) {
    if (!h || every < 0) return PIC_E_ARG;
    if (!h->unet_on) return PIC_E_STATE;
    if (every > 0 && h->net.cap_pairs < 1) return PIC_E_CONFIG;
    h->harvest_every = every;
    return PIC_OK;
}

int pic_unet_get_pair(pic_handle* h, int32_t slot, float* r, float* e, float* chi, float* mask) {
    if (!h) return PIC_E_ARG;
    if (!h->unet_on) return PIC_E_STATE;
    const unet::Net& n = h->net;
    if (slot < 0 || slot >= std::min<int64_t>(n.n_pairs, n.cap_pairs)) return PIC_E_ARG;
    HIP_OK(hipStreamSynchronize(h->stream));
    const size_t img = (size_t)n.H * n.W;
    if (r) HIP_OK(hipMemcpy(r, n.h_r + slot * img, img * 4, hipMemcpyDeviceToHost));
    if (e) HIP_OK(hipMemcpy(e, n.h_e + slot * img, img * 4, hipMemcpyDeviceToHost));
    if (chi) HIP_OK(hipMemcpy(chi, n.h_chi + slot * img, img * 4, hipMemcpyDeviceToHost));
    if (mask) HIP_OK(hipMemcpy(mask, n.h_mask, img * 4, hipMemcpyDeviceToHost));
    return PIC_OK;
}

int pic_unet_put_pair(pic_handle* h, int32_t slot, const float* r, const float* e, const float* chi) {
    if (!h || !r || !e || !chi) return PIC_E_ARG;
    if (!h->unet_on) return PIC_E_STATE;
    unet::Net& n = h->net;
    if (slot < 0 || slot >= n.cap_pairs) return PIC_E_ARG;
    const size_t img = (size_t)n.H * n.W;
    HIP_OK(hipMemcpyAsync(n.h_r + slot * img, r, img * 4, hipMemcpyHostToDevice, h->stream));
    HIP_OK(hipMemcpyAsync(n.h_e + slot * img, e, img * 4, hipMemcpyHostToDevice, h->stream));
    HIP_OK(hipMemcpyAsync(n.h_chi + slot * img, chi, img * 4, hipMemcpyHostToDevice, h->stream));
    // the mask of the handle's own geometry (unknown nodes of the image)
    if (n.n_pairs == 0) unet::mask_from_nodes(n, h->node_kind, h->w, h->stream);
    HIP_OK(hipStreamSynchronize(h->stream));
    if (n.n_pairs < (int64_t)slot + 1) n.n_pairs = (int64_t)slot + 1;
    return PIC_OK;
}

int pic_unet_train(pic_handle* h, int32_t steps, int32_t batch, double lr, uint64_t seed, double* loss_curve) {
    if (!h || steps < 0 || !(lr > 0)) return PIC_E_ARG;
    if (!h->unet_on) return PIC_E_STATE;
    unet::Net& n = h->net;
    if (batch < 1 || batch > n.B) return PIC_E_ARG;
    const int64_t avail = std::min<int64_t>(n.n_pairs, n.cap_pairs);
    if (avail < 1 || h->img_free < 1) return PIC_E_STATE;
    const float inv_n = (float)(1.0 / ((double)batch * (double)h->img_free));
    h->unet_off = false;
    h->unet_strikes = 0;
    uint64_t st = seed ^ 0x5DEECE66Dull;
    std::vector<float> log(unet::kLossLog);
    for (int32_t k = 0; k < steps; ++k) {
        int idx[unet::kMaxBatch];
        for (int b = 0; b < batch; ++b) idx[b] = (int)(splitmix64(st) % (uint64_t)avail);
        unet::gather_batch(n, idx, batch, h->stream);
        unet::forward(n, batch, h->stream);
        unet::backward(n, batch, inv_n, h->stream);
        unet::log_loss(n, k % unet::kLossLog, h->stream);
        unet::adam_update(n, (float)lr, h->stream);
        if ((k + 1) % unet::kLossLog == 0 || k + 1 == steps) {
            HIP_OK(hipStreamSynchronize(h->stream));
            const int m = k % unet::kLossLog + 1;
            HIP_OK(hipMemcpy(log.data(), n.loss_log, (size_t)m * 4, hipMemcpyDeviceToHost));
            if (loss_curve)
                for (int e = 0; e < m; ++e) loss_curve[k + 1 - m + e] = log[e];
        }
    }
    HIP_OK(hipStreamSynchronize(h->stream));
    return PIC_OK;
}

}  // extern "C"
