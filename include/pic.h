/*
 * pic.h -- C ABI of the MI355X (gfx950) implementation of the hot path of
 * the 2D axisymmetric (r-z) electrostatic implicit PIC/MCC model with
 * equivalent-capacitance circuit coupling of arXiv 2310.04957 (Sec. 2).
 *
 * The calls follow the paper's statement of the problem: a reactor made of
 * metal electrodes and dielectrics on a regular r-z grid (Sec. 2, reactor
 * geometry paragraph), one RF-driven electrode coupled to an external
 * circuit (Eqs. 5 and 8-10), argon with electrons and Ar+ (collision
 * paragraph), a time step (Sec. 3, first paragraph), and outputs of
 * period-averaged densities and electrode voltage/current harmonics (Sec. 3).
 *
 * Conventions for every entry point:
 *   - Return value: PIC_OK (0) or a negative PIC_E_* code; pic_strerror()
 *     names it.  No C++ exception crosses this boundary.
 *   - Device memory and the HIP stream are owned by the caller: pic_init
 *     receives one device workspace of at least pic_workspace_size() bytes,
 *     which must stay allocated and untouched until pic_free(); all work is
 *     queued on the caller's stream.  The library allocates no device memory
 *     of its own.
 *   - The library copies the configuration at pic_init; caller buffers
 *     passed to other calls are read or written only during the call.
 *   - A handle is not thread safe: one caller at a time.
 *   - Grids are node arrays of (nr+1)*(nz+1) values, index j*(nr+1)+i with
 *     r_i = i*R/nr, z_j = j*Z/nz (r fastest).
 */
#ifndef PIC_H
#define PIC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_ABI_VERSION 2
#define PIC_MAX_REGIONS 32
#define PIC_MAX_ELECTRODES 4           /* driven electrodes: conductor ids 1 .. 4 */

enum {
    PIC_OK = 0,
    PIC_E_CONFIG = -1,    /* invalid configuration (sizes, regions, circuit values) */
    PIC_E_CAPACITY = -2,  /* births exceeded a species capacity (or a slice's staging row): the births
                             that did not fit were dropped in that step, pic_step returns this code at
                             the next step, before moving any particle, and refuses every later call;
                             a splitting pass that does not fit changes nothing and reports it too */
    PIC_E_SOLVER = -3,    /* field solve did not reach the tolerance within max_iter */
    PIC_E_HIP = -4,       /* a HIP runtime call failed */
    PIC_E_NONFINITE = -5, /* a non-finite value reached the field solve */
    PIC_E_STATE = -6,     /* call not valid in the handle's state */
    PIC_E_ARG = -7,       /* bad argument (null pointer, size too small, bad id) */
    PIC_E_NODEVICE = -8,  /* no gfx950 device is current */
    PIC_E_TOOBIG = -9     /* the grid exceeds the fixed scratch of an allocation-free entry point */
};

enum { PIC_VACUUM = 0, PIC_DIEL = 1, PIC_COND = 2 };                 /* region kinds */
enum { PIC_GROUND = 0, PIC_POWERED = 1, PIC_NEUMANN = -1 };           /* conductor ids / edge bc */
enum { PIC_IDEAL_SOURCE = 0, PIC_SERIES_RLC = 1, PIC_LMATCH = 2 };    /* circuits */
/* field-solve methods: FP64 MG-PCG; FP64 iterative refinement around an FP32
   inner solve by MG-PCG, by flexible CG preconditioned with the U-net below
   (MG-PCG takes over when the network fails), or by CG without a
   preconditioner (the reference point of what the network gains) */
enum { PIC_SOLVE_MGPCG_FP64 = 0, PIC_SOLVE_IR_MG = 1, PIC_SOLVE_IR_UNET = 2, PIC_SOLVE_IR_CG = 3 };
enum { PIC_WEIGHTS_EQUAL = 0, PIC_WEIGHTS_CELL = 1 };                /* initial macro-particle weights */

/* A rectangle [r0,r1) x [z0,z1) in metres.  Each cell takes the last region
   that contains its centre.  kind PIC_COND uses cond_id (0 ground, 1 .. n_el
   a driven electrode); PIC_DIEL uses eps_r. */
typedef struct {
    double r0, r1, z0, z1;
    int32_t kind, cond_id;
    double eps_r;
} pic_region;

typedef struct {
    int32_t nr, nz;             /* cells; both even, 4 <= n <= 4096, at most 65535 tiles of 16 x 16 cells */
    double R, Z;                /* domain [0,R] x [0,Z], metres; r = 0 is the axis */
    int32_t n_regions;
    int32_t edge_bc[3];         /* r=R, z=0, z=Z edges: conductor id or PIC_NEUMANN */
    pic_region regions[PIC_MAX_REGIONS];
} pic_geometry;

/* Eq. (9) series R_b L_b C_b, Eq. (10) L-type network (C_m1 shunt, R_m L_m
   C_m2 series, stray branch R_stray L_stray C_stray), or an ideal source on
   the electrode.  Source U_amp sin(2 pi f t) + U_dc. */
typedef struct {
    int32_t kind, substeps;     /* substeps: RK4 substeps per PIC step */
    double freq, U_amp, U_dc, R_s, C_m1, C_m2, L_m, R_m, C_stray, L_stray, R_stray, C_b, R_b, L_b;
} pic_circuit;

typedef struct {
    double p_Pa, T_gas_K;       /* background argon, fixed (no depletion) */
} pic_gas;

typedef struct {
    int64_t n_e, n_i;           /* initial macro-particles */
    int64_t cap_e, cap_i;       /* slots reserved per species, at most 2^30 - 16 */
    double n0, Te_eV, Ti_eV;    /* initial uniform plasma density (m^-3) and temperatures */
    int32_t steps_per_period;   /* dt = 1 / (freq * steps_per_period) */
    int32_t sort_every;         /* electron tile sort every K steps (0: never) */
    int32_t sort_every_ion;     /* ion tile sort every K steps (0: never) */
    uint64_t seed;              /* Philox key */
    int32_t load;               /* 1: load the Maxwellian plasma at init; 0: start empty */
    int32_t timing;             /* 1: time each phase with HIP events (pic_diag reports ms) */
    /* Unequal weights and particle splitting (Sec. 3, particle splitting
       against on-axis heating).  weights: PIC_WEIGHTS_EQUAL loads equal
       weights uniformly in volume; PIC_WEIGHTS_CELL loads every vacuum cell
       with the same expected count, each particle weighted by the volume of
       its cell over the mean vacuum-cell volume (the reference weight of
       the cell's column).  split = 1: at every tile sort of a species, a
       particle whose weight is at least 2^m reference weights of its
       column is first replaced by 2^m identical particles (m <= 3). */
    int32_t weights;
    int32_t split;
} pic_run;

typedef struct {
    int32_t method;             /* PIC_SOLVE_* */
    double tol;                 /* ||b - K phi||_2 / ||b||_2 at which a solve stops */
    int32_t max_iter;           /* Krylov iterations per solve */
    double inner_tol;           /* IR: relative tolerance of each FP32 inner solve */
    int32_t unet_batch;         /* learned preconditioner: training batch capacity (0: no U-net) */
    int32_t unet_pairs;         /* learned preconditioner: harvested (residual, error) pair slots */
    int32_t graphs;             /* 1: each iteration of the multigrid-preconditioned CG (its two
                                   vector launches and the V-cycle's launches) is replayed from a HIP
                                   graph captured once per handle, so the host issues one launch per
                                   iteration instead of ~15; 0: every kernel is launched on its own
                                   (for callers that capture pic_step into graphs of their own).  The
                                   results are the same bit for bit. */
} pic_solver;

typedef struct {
    int32_t abi_version;        /* PIC_ABI_VERSION */
    pic_geometry geom;
    pic_circuit circ;
    pic_gas gas;
    pic_run run;
    pic_solver solver;
    /* Several driven electrodes (Sec. 2: each metal electrode has its own
       equivalent capacitance and circuit): conductor ids 1 .. n_el (0 means
       1).  Electrode 1 uses circ, electrode e >= 2 circ_el[e - 2].  The
       electrodes couple through the capacitance matrix C (the field-energy
       bilinear form of their Laplace solutions): Q = C U + Q_P, so an ideal
       source fixes its electrode's voltage and the other voltages follow
       from their charges.  One time step's substep count is the largest of
       the circuits'. */
    int32_t n_el;
    pic_circuit circ_el[PIC_MAX_ELECTRODES - 1];
} pic_config;

typedef struct pic_handle pic_handle;

/* Scalars and counters returned by pic_diag.  Grids and time series are
   copied into the optional caller buffers of pic_diag_buffers. */
typedef struct {
    double t, U_E, Q_E, C_eq, Q_P, I_ccp, dt, w_unit, n_gas;
    double circ[5];
    double nu_max[2];
    uint32_t thresh[2];
    int64_t step, periods_done;
    int64_t n_slots[2], n_alive[2];
    int64_t absorbed[2][4];     /* per species: ground, powered, lost (Neumann edge), dielectric */
    int64_t born, coll[2][4], numax_violations;
    int64_t solver_iters, solver_outer;
    double solver_relres;
    double harm_U_re[6], harm_U_im[6], harm_I_re[6], harm_I_im[6];
    double ms_particles[2], ms_births, ms_sort, ms_field, ms_refresh; /* accumulated since last reset */
    int64_t timed_steps, deposit_fallback;
    int32_t error;              /* sticky error raised on the device (PIC_E_CAPACITY ...) */
    int64_t unet_pairs, unet_fallbacks, unet_applications;
    /* last complete RF period (Sec. 3, Eqs. 11-14): CCP and load impedances
       at the fundamental (ohm), |Gamma| against R_s (circuit II only), and
       period-averaged powers (W) of the source, R_s, the matching network's
       R_m (circuit II) or the series branch's R_b (circuit I), the stray
       branch, the plasma load; the forward power into the matching network
       and the reflected power */
    double Z_ccp_re, Z_ccp_im, Z_load_re, Z_load_im, gamma_abs;
    double P_source, P_Rs, P_imn, P_stray, P_ccp, P_forward, P_ref;
    int64_t split_added[2];     /* particles added by splitting since init, per species */
    /* per driven electrode e = 1 .. n_el at index e - 1: voltage, charge,
       induced charge Q_P, circuit current, the capacitance matrix (row-major
       PIC_MAX_ELECTRODES x PIC_MAX_ELECTRODES, F), harmonics 0..5 of voltage
       and current over the last RF period of electrode 1's source, and the
       charge absorbed per species (units 2^-32 w_unit).  U_E, Q_E, C_eq, Q_P,
       I_ccp, the harmonics and the characterisation above are electrode 1's. */
    int32_t n_el;
    double U_el[PIC_MAX_ELECTRODES], Q_el[PIC_MAX_ELECTRODES], QP_el[PIC_MAX_ELECTRODES];
    double I_el[PIC_MAX_ELECTRODES];
    double C_el[PIC_MAX_ELECTRODES * PIC_MAX_ELECTRODES];
    double hU_re[PIC_MAX_ELECTRODES][6], hU_im[PIC_MAX_ELECTRODES][6];
    double hI_re[PIC_MAX_ELECTRODES][6], hI_im[PIC_MAX_ELECTRODES][6];
    int64_t absorbed_el[2][PIC_MAX_ELECTRODES];
    /* 1 when the learned preconditioner is switched off: three solves in a
       row gave it back to multigrid (it stays off until pic_unet_set_params
       or pic_unet_train; PIC_SOLVE_IR_UNET then runs as PIC_SOLVE_IR_MG) */
    int32_t unet_disabled;
    /* what raised PIC_E_CAPACITY: bit 0 the births of a step exceeded a
       species' slot capacity, bit 1 a slice's births exceeded its staging
       row, bit 2 a splitting pass did not fit */
    int32_t capacity_bits;
} pic_diag_out;

typedef struct {
    double* n_e;                /* period-averaged densities, m^-3, node grid (or NULL) */
    double* n_i;
    double* phi;                /* potential at the last step, V (or NULL) */
    double* U_E;                /* electrode voltage over the last complete period, steps_per_period values */
    double* I_ccp;              /* circuit current over the last complete period */
} pic_diag_buffers;

/* Bytes of device workspace needed for cfg.  Host-only, no device access. */
int pic_workspace_size(const pic_config* cfg, size_t* bytes_out);

/* Validate cfg, carve the workspace, build the geometry, load the plasma
   (Sec. 3: uniform density, Maxwellian), deposit the first predicted
   positions, compute the vacuum C_eq (Eqs. 6-7) and the multigrid
   hierarchy.  Synchronises the stream before returning. */
int pic_init(const pic_config* cfg, void* dev_workspace, size_t bytes, void* hip_stream, pic_handle** out);

/* Queue nsteps time steps on the stream (Sec. 2 order: assembly of Eq. 1,
   circuit and electrode charge, implicit field solve, particle push with
   MCC and deposit, births, periodic sort, per-period Laplace/C_eq refresh).
   Returns after queueing; the field solve reads one convergence flag back
   every few Krylov iterations. */
int pic_step(pic_handle* h, int32_t nsteps);

/* Synchronise and fill `out` (and the buffers of `bufs` that are non-NULL). */
int pic_diag(pic_handle* h, pic_diag_out* out, const pic_diag_buffers* bufs);
int pic_reset_timers(pic_handle* h);

int pic_free(pic_handle* h);
const char* pic_strerror(int code);

/* ---- introspection for parity tests (synchronous, host buffers) ---- */
enum { PIC_P_R = 0, PIC_P_Z, PIC_P_VR, PIC_P_VT, PIC_P_VZ, PIC_P_AR, PIC_P_AT, PIC_P_AZ, PIC_P_W };
/* Particle slots of a species as 9 field-major FP32 arrays (r z vr vt vz ar
   at az w); a dead slot has r < 0.  get: `host9` holds 9*cap floats and
   *n receives the slot count.  set: n slots are copied in. */
int pic_get_particles(pic_handle* h, int32_t species, float* host9, int64_t* n);
int pic_set_particles(pic_handle* h, int32_t species, const float* host9, int64_t n);

enum {
    PIC_G_DEP_E = 0, PIC_G_DEP_I = 1, /* int64 fixed-point deposits of the predicted positions */
    PIC_G_PHI = 2,                    /* double */
    PIC_G_ER = 3, PIC_G_EZ = 4,       /* float, node electric field */
    PIC_G_CHI = 5,                    /* double */
    PIC_G_WALLQ = 6,                  /* int64 dielectric surface charge */
    PIC_G_PHI_L = 10, PIC_G_Q = 11, PIC_G_AR = 12, PIC_G_AZ = 13, /* double */
    /* double: Laplace solutions of driven electrodes 2, 3, 4 (PHI_L is electrode 1's) */
    PIC_G_PHI_L2 = 14, PIC_G_PHI_L3 = 15, PIC_G_PHI_L4 = 16
};
int pic_get_grid(pic_handle* h, int32_t which, void* host);
int pic_set_grid(pic_handle* h, int32_t which, const void* host); /* DEP_E, DEP_I, WALLQ, PHI */

/* Zero both deposit grids and deposit the current slots at their stored
   (predicted) positions, with the same fixed-point kernel as the step. */
int pic_redeposit(pic_handle* h);

/* Tile sort of one species now (stable, dead slots dropped); perm_out (or
   NULL) receives, for each new slot, the old slot it came from. */
int pic_sort_now(pic_handle* h, int32_t species, int64_t* perm_out);

/* One particle-splitting pass over a species now (Sec. 3, particle
   splitting): a live particle inside the domain in cell column i whose
   weight w is at least 2 w_ref(i) becomes k = 2^m particles of weight w/k
   (m the largest with w >= 2^m w_ref(i), at most 3; compared in FP32) with
   the same position, velocity and averaged acceleration.  w_ref(i) = W_s
   V_i / V_mean: W_s the species' loading weight (units of w_unit), V_i the
   cell volume of column i, V_mean the mean vacuum-cell volume.  The parent
   keeps its slot; the k - 1 copies follow the last slot in parent-slot
   order.  *added (or NULL) receives the number of copies.  Returns
   PIC_E_CAPACITY when the copies do not fit: no particle changes, and the
   handle keeps the capacity error that pic_diag reports. */
int pic_split_now(pic_handle* h, int32_t species, int64_t* added);

/* One solve of Eq. (1) on given node charges Q (C) and susceptibility chi
   with driven electrode 1 at U_E (any others at 0 V); phi_inout is the warm
   start and the result.  Uses the configured method; tol overrides the
   configured one. */
int pic_solve_once(pic_handle* h, const double* Q, const double* chi, double U_E, double tol,
                   double* phi_inout, int32_t* iters, double* relres);

/* The same with driven electrode e at U[e - 1], e = 1 .. n_el (host array). */
int pic_solve_once_el(pic_handle* h, const double* Q, const double* chi, const double* U, double tol,
                      double* phi_inout, int32_t* iters, double* relres);

/* Matching design (Sec. 3, first paragraph: the vacuum equivalent
   capacitance gives the L-network's elements for a perfect match).  For
   electrode 1's circuit II (PIC_LMATCH): the shunt C_m1 and series C_m2
   for which the network, with its R_m and L_m, presents exactly R_s to the
   source when loaded by the current C_eq in parallel with the stray branch
   R_stray, L_stray, C_stray (Eq. 10).  Called right after pic_init, C_eq is
   the vacuum one, as in the paper.  out2 (host, 2 doubles) receives C_m1
   and C_m2 in farads; apply = 1 also makes them the circuit's elements for
   the following steps (the circuit state is kept).  Synchronises the
   stream.  PIC_E_CONFIG when the circuit is not PIC_LMATCH or no such
   network exists (R_m + Re Z_load >= R_s, or a series reactance above
   w L_m would be needed); nothing changes then. */
int pic_match_design(pic_handle* h, int32_t apply, double* out2);

/* Set t, Q_E, U_E, circ[5], C_eq (9 doubles) -- for single-step parity. */
int pic_set_state(pic_handle* h, const double* st9);

/* Energy moment of a species at its stored (predicted) positions and
   explicit velocities v* (the state between steps): N and E node grids
   (int64, nr+1 by nz+1, host buffers) of the deposit's integer weight
   shares c_k (units 2^-32 of a weight) and of c_k floor(16 eps), eps the
   particle's kinetic energy in eV (capped at 2^20 / 16 eV).  Mean energy
   per node E / (16 N) eV, electron temperature two thirds of it (Sec. 3,
   the T_e maps).  Exact integer sums: bit-identical to any order. */
int pic_moments(pic_handle* h, int32_t species, int64_t* N, int64_t* E);

/* pic_moments for callers that cannot allocate device memory (code under
   HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
   the same results, bit for bit, but the two device node grids it
   accumulates in live in a fixed scratch array of the library (one per GPU,
   held until the process ends) instead of the handle's solver work vectors,
   which it leaves untouched.  It calls no allocating routine.  Limit: grids
   of at most PIC_NOALLOC_MAX_NODES nodes ((nr+1)(nz+1); 1024 x 2048 cells
   fit), PIC_E_TOOBIG beyond.  Every call on one GPU shares that GPU's
   scratch: calls that overlap on one GPU (several threads or streams) race
   and must be serialised by the caller. */
#define PIC_NOALLOC_MAX_NODES (1025 * 2049)
int pic_moments_noalloc(pic_handle* h, int32_t species, int64_t* N, int64_t* E);

/* ---- learned preconditioner (requires solver.unet_batch > 0; nr and nz
   multiples of 16) ----
   A 5-level, 32-channel U-net on the node image of nz rows (z) by nr
   columns (r); the node row z = Z and column r = R must be conductors and
   are left out.  Input channels per pixel: the residual scaled to unit RMS
   over the unknown nodes, chi/(1+chi), and 1 on unknown nodes (0 on
   conductors).  Output: the error K^-1 r of that residual, also at unit RMS;
   it preconditions flexible CG (method PIC_SOLVE_IR_UNET), which does not
   depend on a scalar factor of the preconditioner output.  MG-PCG takes over
   a solve in which the output stops being a descent direction.
   Parameters: one FP32 vector, per 3x3 convolution w[9][cout][cin] (tap
   t = 3 (dy+1) + (dx+1), dy along z) then b[cout], in the order enc1a enc1b
   ... enc4b mid5a mid5b dec4a dec4b ... dec1a dec1b, then the 1x1 output
   w[32] and b[1].  BF16 weights and activations, FP32 accumulation; the
   master weights and Adam moments stay FP32. */
int pic_unet_num_params(pic_handle* h, int64_t* n);
/* n must equal pic_unet_num_params; setting parameters also resets the Adam
   moments and step count. */
int pic_unet_set_params(pic_handle* h, const float* p, int64_t n);
int pic_unet_get_params(pic_handle* h, float* p, int64_t n);
/* Replace the solver settings (method, tol, max_iter, inner_tol); unet_batch
   and unet_pairs must equal the values given to pic_init. */
int pic_set_solver(pic_handle* h, const pic_solver* s);
/* in3: [batch][nz][nr][3] FP32 input channels; out: [batch][nz][nr]. */
int pic_unet_forward(pic_handle* h, const float* in3, int32_t batch, float* out);
/* Gradient of the mean over mask of (out - target)^2 (mask, target:
   [batch][nz][nr]) with respect to every parameter, and the loss. */
int pic_unet_grads(pic_handle* h, const float* in3, const float* target, const float* mask, int32_t batch,
                   float* grads, double* loss);
/* During pic_step, store one (first residual, error removed) pair of the
   field solve every `every` steps, both at unit RMS as above, in a ring of
   solver.unet_pairs slots (every > 0 also harvests each pic_solve_once;
   0 stops).  A solve that does not converge leaves no pair. */
int pic_unet_harvest(pic_handle* h, int32_t every);
/* Copy harvested pair `slot` (< min(pairs harvested, unet_pairs)): the
   normalised residual, the normalised error, chi/(1+chi) and the mask, each
   [nz][nr] FP32 (NULL skips one). */
int pic_unet_get_pair(pic_handle* h, int32_t slot, float* r, float* e, float* chi, float* mask);
/* Store a pair in slot `slot` (< solver.unet_pairs) of the ring, in the
   layout pic_unet_get_pair returns (normalised residual, normalised error,
   chi/(1+chi), each [nz][nr] FP32; the mask is the handle's own), so that
   pairs harvested by several runs train one network.  The pair count
   becomes at least slot + 1. */
int pic_unet_put_pair(pic_handle* h, int32_t slot, const float* r, const float* e, const float* chi);
/* Adam (lr, betas 0.9/0.999) on random batches of the harvested pairs;
   loss_curve (or NULL) receives the loss of each step. */
int pic_unet_train(pic_handle* h, int32_t steps, int32_t batch, double lr, uint64_t seed, double* loss_curve);

#ifdef __cplusplus
}
#endif
#endif
