// pic_internal.h -- runtime state behind the C ABI and the host-side
// launchers of the HIP kernels (one process, one gfx950 device, the
// caller's stream).  Device buffers are carved from the caller's workspace.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/pic.h"
#include "pic_device.h"
#include "unet.h"

namespace pic {

// tile sort key of a slot: its tile, or the tile count for a dead slot (at
// most 65535 tiles, checked at init)
typedef uint16_t tkey_t;
constexpr int kBlock = 256;           // threads per block for sort and helper kernels
constexpr int kItems = 16;            // particles per thread per sort chunk
constexpr int kChunk = kBlock * kItems;
constexpr int kWaves = kBlock / 64;   // wavefronts per block of the sort kernels
// the particle kernel: a block of kPushWaves wavefronts owns chunks of
// kPushChunk consecutive slots, each wavefront a slice of kSlice of them
constexpr int kPushWaves = 8;
constexpr int kPushBlock = 64 * kPushWaves;
constexpr int kSlice = 1024;
constexpr int kPushChunk = kSlice * kPushWaves;
// staged ionisation births per slice (one row per slice): at least this
// many, and enough that a slice overflows its row with a probability below
// 1e-15 per step (set with the null-collision constants)
constexpr int kStageWMin = 64;
// rows of the birth staging area for n slots (whole chunks)
__host__ __device__ constexpr long long stage_rows(long long n) {
    return (n + kPushChunk - 1) / kPushChunk * kPushWaves;
}
constexpr int kMaxLevels = 16;
constexpr int kMaxCoarse = 320;       // active nodes of the coarsest multigrid level
constexpr int kCoarsestNodes = 100;   // coarsening stops at this many nodes (or when it cannot go on)
constexpr int kRedBlocks = 4096;      // partial sums of a grid reduction
constexpr int kCgBlocks = 512;        // blocks (and partial sums) of the fused CG vector kernels
constexpr int kMaxEl = PIC_MAX_ELECTRODES;   // driven electrodes
// absorption counter slot of conductor id: 0 ground, 1 electrode 1, 2 lost
// (Neumann edge), 3 dielectric, 4 .. 6 electrodes 2 .. 4
__host__ __device__ constexpr int slot_of(int id) { return id <= 1 ? id : 2 + id; }
constexpr int kSlots = 8;
// bits of DevCounters::err: births that did not fit a species' slots or a
// slice's staging row were dropped (the run stops at the next step); a
// splitting pass did not fit and changed nothing
constexpr int kErrBirths = 1;
constexpr int kErrStage = 2;   // births dropped too: a slice's staging row was full
constexpr int kErrSplit = 4;

// counters that kernels update; lives in device memory
struct DevCounters {
    long long n_slots[2];
    long long born;
    unsigned long long absorbed[2][kSlots];
    unsigned long long coll[2][4];
    unsigned int viol;
    int err;
    unsigned long long fallback;
    long long births_step;
    long long base[2];
    long long nch_births;
    unsigned int dead[2];
    long long split_total;        // copies of the current splitting pass (-1: they do not fit)
    long long split_added[2];     // copies since init, per species
    long long n_keyed[2];         // slots whose sort keys the last particle step wrote
    long long pad[2];
};

// FP64 scalars of the field solve and the circuit; device memory
struct DevScalars {
    // driven electrodes e (index e - 1): voltage, charge, induced charge,
    // circuit current and state, capacitance matrix (Cm[0][0] = C_eq of
    // electrode 1), integer absorbed charge at the last circuit step
    double U_E[kMaxEl], Q_E[kMaxEl], Q_P[kMaxEl], I_ccp[kMaxEl], circ[kMaxEl][5];
    double Cm[kMaxEl][kMaxEl];
    double el_prev[kMaxEl];
    double unit[kMaxEl][kMaxEl];   // identity rows: Dirichlet values of the Laplace problems
    double Uset[kMaxEl];           // Dirichlet values of pic_solve_once
    double t;
    double bb, rr, rz, rz_new, pq, alpha, beta, target, scale, relres, rr0;
    double rr_net, c_net;    // learned preconditioner: |res|^2 at the network, its Galerkin weight
    double energy[5];        // circuit element energies of the running RF period
    double last_energy[5];   // ... of the last complete one
    int done, iters, nonfinite, fallback;
    int cap_err;             // DevCounters::err as the last residual reduction saw it
    // refinement with the control on the device: the solve is finished
    // (every later launch of it returns at once), the residual reductions
    // done, the Krylov iterations of each pass and in all
    int outer_done, outer, its_pass[4], iters_total;
};

struct Level {
    int nr, nz, w, nn, cr, cz;   // cr/cz: factor to the next (coarser) level
    double* A64[9];              // 9-point stencils (levels >= 1)
    float* A32[9];
    double *x64, *y64, *b64, *res64;
    float *x32, *y32, *b32, *res32;
};

}  // namespace pic

struct pic_handle {
    pic_config cfg;
    hipStream_t stream;
    char* ws;
    size_t ws_bytes;
    // derived constants
    int nr, nz, w, nn, ncell, ntr, ntz, ntiles, key_bits;
    int kmul, row_bits;           // tile keys ty kmul + tx; row_bits > 0: kmul = 2^row_bits
    double dr, dz, dt, Sr, Sz, w_unit, n_gas, nu_max[2], vth_gas, qunit, chi_c[2];
    uint32_t thresh[2];
    int64_t cap[2];
    int64_t max_chunks;
    int64_t max_rows;             // birth staging rows
    int stage_w;                  // births per staging row
    // geometry (device)
    uint8_t* cell_kind;
    uint32_t* vac_tiles;          // kVacWords words: bit t, every cell of tile t is vacuum
    int8_t* node_kind;
    double *vol, *gr, *gz, *invd;
    std::vector<int8_t> h_node_kind;
    std::vector<uint8_t> h_cell_kind;
    std::vector<double> h_vol, h_gr, h_gz;
    // particles: two buffers per species for the sort
    pic::Species buf[2][2];
    int cur[2];
    pic::tkey_t* keys[2];
    uint32_t* idx[2];
    pic::tkey_t* keys_ion;    // the ions' sort keys, written by the ion step before their sort
    pic::Species sink;               // 64 slots the particle kernel's lanes past the last slot write
    pic::tkey_t* ksink;              // 64 keys likewise
    uint32_t* perm[2];        // per species: the permutation of the last sort
    bool pending[2];          // a sort whose particle movement is still to be applied
    uint32_t* hist;
    uint32_t* bsum;
    // particle splitting: reference weight per cell column, per species;
    // per-chunk copy counts and offsets of a pass
    float* wtcol[2];
    long long* split_off;
    // births
    pic::Birth* stage;
    int *stage_cnt, *stage_off, *stage_segoff;   // stage_off holds segment sums
    // deposits and grids
    unsigned long long* dep[2][2];  // [buffer][species]
    int dep_cur;
    unsigned long long *wallq, *psum[2], *plast[2];
    double *chi, *Q, *ar, *az, *phi, *zeroQ;
    int n_el;               // driven electrodes
    double* phiL[pic::kMaxEl];  // Laplace solution of each driven electrode
    double* phi_prev;       // the previous step's solution (initial-guess extrapolation)
    double* phi_prev2;      // ... and the one before
    int have_prev;          // solutions in the history (0 .. 2)
    float *ar32, *az32;
    float2* E;
    // solver vectors
    double *r64, *x64, *z64, *p64, *q64;
    float *r32, *x32, *z32, *p32, *q32;
    double* part;           // reduction partials
    double* cgpart;         // fused CG partials: r.z (cgpart_n, one per level-0 multigrid tile), p.q, r.r
    int cgpart_n;
    int tail_lds_max = -1;  // dynamic LDS bytes the multigrid tail may use (-1: not yet asked)
    // HIP graphs of the fused CG, per precision (0 FP32, 1 FP64): the start
    // (k_begin_cg and the first V-cycle) and the iterations 0, odd, even
    // (which differ in the direction buffers and the first-iteration flag);
    // captured on a private stream at the first solve, replayed on `stream`
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t cg_graph[2][4] = {};
    bool cg_graph_tried[2] = {false, false};
    bool cg_graph_ok[2] = {false, false};
    pic::Level lv[pic::kMaxLevels];
    int nlev;
    int* cmap;              // coarsest node -> dense index, -1 inactive
    int ncoarse;
    double* cinv64;
    float* cinv32;
    // time series
    double *serU, *serI, *lastU, *lastI;          // kMaxEl x steps_per_period each
    double *serVin, *serI1, *lastVin, *lastI1;   // source-side voltage and current per step
    // device counters / scalars and their pinned host mirrors
    pic::DevCounters* ctr;
    pic::DevScalars* sc;
    pic::DevScalars* h_sc;     // pinned
    pic::DevCounters* h_ctr;   // pinned
    // host-side bookkeeping
    int64_t step, periods_done;
    int have_last;
    int64_t solver_iters, solver_outer;
    int cg_guess[2][4];           // Krylov iterations of the last solve, per precision and outer pass
    int ir_passes = 0;            // refinement passes of the last device-controlled solve (0: none yet)
    double solver_relres;
    int sticky_err;
    bool halted;                  // births were dropped: no further steps
    // learned preconditioner
    bool unet_on;
    pic::unet::Net net;
    float* unet_stage;      // host-provided inputs, [B][H][W][3]
    double* hx64;           // [kHarvestPerSolve][nn] Krylov iterates of a harvested solve
    int harvest_every, harvest_limit;
    bool harvest_now, harvesting;
    int64_t unet_fallbacks, unet_apps, img_free;
    int unet_strikes;       // consecutive solves the network gave back to multigrid
    bool unet_off;          // switched off after three of them, until new parameters
    // phase timing
    bool timing;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
    double ms[6];
    int64_t timed_steps;
};

namespace pic {

// geometry and layout on the host
int host_geometry(pic_handle* h);          // host rasterisation, volumes, faces
int upload_geometry(pic_handle* h);
size_t layout(pic_handle* h, char* base);   // returns bytes; assigns pointers when base != nullptr
int mg_plan(pic_handle* h);                 // level sizes and coarsening factors (host)

// particle kernels
void launch_load(pic_handle* h, int sp, const double* cdf, const int* cell, int nv, double vvac, int64_t n,
                 float W, float vth);
void launch_predict_deposit(pic_handle* h, int sp);
void launch_redeposit(pic_handle* h);
void launch_particles(pic_handle* h, int sp, bool emit_keys = false);
void launch_births(pic_handle* h);
int launch_count_alive(pic_handle* h, long long* out2);
void launch_moments(pic_handle* h, int sp, unsigned long long* N, unsigned long long* E);

// sort
void launch_sort(pic_handle* h, int sp, bool deferred = false, bool keyed = false);
void launch_split(pic_handle* h, int sp);
void materialize(pic_handle* h, int sp);

// field
void launch_assemble(pic_handle* h);
void launch_faces(pic_handle* h);
void launch_circuit(pic_handle* h);
int field_solve(pic_handle* h, double* phi, const double* Q, const double* Uptr, double tol, int method,
                int32_t* iters_out, double* relres_out);
int refresh_laplace(pic_handle* h);
void mg_rebuild(pic_handle* h);
void launch_efield(pic_handle* h);
void launch_extrapolate(pic_handle* h);
void launch_period_roll(pic_handle* h);
void launch_zero_u64(unsigned long long* p, size_t n, hipStream_t s);
void launch_zero_f64(double* p, size_t n, hipStream_t s);

}  // namespace pic
