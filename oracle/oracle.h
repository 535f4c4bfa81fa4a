/*
 * oracle.h -- plain FP64 CPU oracle for the r-z implicit PIC/MCC step with
 * equivalent-capacitance circuit coupling (arXiv 2310.04957, Sec. 2).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no source with
 * the HIP path; both consume the same plain-data configuration and seeded
 * inputs.  Everything here is written for a reader to check against the
 * paper by eye: no blocking, no fusion, single-threaded, FP64 throughout
 * (the deposit is an exact integer definition).
 *
 * Readings of passages the paper leaves open are marked [Rn] in the sources;
 * the list is kept with the design notes of the repository.
 *
 * Parity unpinned: conformance of Philox4x32-10 to the published
 * known-answer vectors (not available); the 4x64 instantiation of the same
 * round structure is pinned to numpy's Philox instead.
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_REGIONS 32
#define ORC_NCNT 4 /* absorption counter slots: 0 ground, 1 powered, 2 lost (Neumann edge), 3 dielectric */
#define ORC_MAX_EL 4 /* driven electrodes: conductor ids 1 .. ORC_MAX_EL */

typedef struct {
    double r0, r1, z0, z1;
    int32_t kind;    /* 0 vacuum, 1 dielectric, 2 conductor */
    int32_t cond_id; /* 0 ground, 1 RF-driven electrode */
    double eps_r;
} orc_region;

/* the external circuit of one driven electrode (fields as in orc_config) */
typedef struct {
    int32_t kind, substeps;
    double freq, U_amp, U_dc, R_s, C_m1, C_m2, L_m, R_m, C_stray, L_stray, R_stray, C_b, R_b, L_b;
} orc_circ;

typedef struct {
    /* geometry: cells nr x nz on [0,R] x [0,Z] */
    int32_t nr, nz;
    double R, Z;
    int32_t n_regions;
    int32_t edge_bc[3]; /* r=R, z=0, z=Z: conductor id, or -1 Neumann */
    orc_region regions[ORC_MAX_REGIONS];
    /* circuit: 0 ideal source on the electrode, 1 series R_b L_b C_b (Eq. 9),
       2 L-type matching network with stray branch (Eq. 10) */
    int32_t circ_kind, substeps;
    double freq, U_amp, U_dc, R_s, C_m1, C_m2, L_m, R_m, C_stray, L_stray, R_stray, C_b, R_b, L_b;
    /* background argon */
    double p_Pa, T_gas_K;
    /* particles and run */
    int64_t n_e, n_i, cap_e, cap_i;
    double n0, Te_eV, Ti_eV;
    int32_t steps_per_period, sort_every, sort_every_ion;
    uint64_t seed;
    double tol;
    int32_t max_iter;
    int32_t load; /* 1: Maxwellian uniform load at creation, 0: no particles */
    /* [R32] weights: 0 equal; 1 per cell volume (equal count per vacuum cell).
       split: 1 splits heavy particles at every tile sort of their species */
    int32_t weights, split;
    /* [R33] driven electrodes 1 .. n_el (0 counts as 1): electrode 1 uses
       the circuit above, electrode e >= 2 circ_el[e - 2] */
    int32_t n_el;
    orc_circ circ_el[ORC_MAX_EL - 1];
} orc_config;

typedef struct {
    double t, U_E, Q_E, C_eq, Q_P, I_ccp, dt, w_unit, n_gas;
    double circ[5];
    double nu_max[2];
    uint32_t thresh[2];
    int64_t step, periods_done;
    int64_t n_slots[2], n_alive[2];
    int64_t absorbed[2][ORC_NCNT];
    int64_t born, coll[2][4], numax_violations;
    int64_t solver_iters;
    double solver_relres;
    double harm_U_re[6], harm_U_im[6], harm_I_re[6], harm_I_im[6];
    /* last complete period (Eqs. 11-14): Z_ccp re/im, Z_load re/im, |Gamma|,
       P_source, P_Rs, P_IMN, P_stray, P_ccp, P_forward, P_ref */
    double elec[12];
    int64_t split_added[2]; /* particles added by splitting since creation */
    /* [R33] per driven electrode e = 1 .. n_el (index e - 1): voltage,
       charge, induced charge, circuit current, capacitance matrix (row-major
       ORC_MAX_EL x ORC_MAX_EL), harmonics 0..5 of the last period, charge
       absorbed per species (units 2^-32 w_unit) */
    int32_t n_el;
    double U_el[ORC_MAX_EL], Q_el[ORC_MAX_EL], QP_el[ORC_MAX_EL], I_el[ORC_MAX_EL];
    double C_el[ORC_MAX_EL * ORC_MAX_EL];
    double hU_re[ORC_MAX_EL][6], hU_im[ORC_MAX_EL][6], hI_re[ORC_MAX_EL][6], hI_im[ORC_MAX_EL][6];
    int64_t absorbed_el[2][ORC_MAX_EL];
} orc_diag;

typedef struct orc_sim orc_sim;

/* grid ids for orc_get_grid / orc_set_grid */
enum {
    ORC_G_DEP_E = 0, ORC_G_DEP_I = 1, /* int64 fixed-point node sums of the predicted positions */
    ORC_G_PHI = 2, ORC_G_ER = 3, ORC_G_EZ = 4, ORC_G_CHI = 5,
    ORC_G_WALLQ = 6,       /* int64 dielectric surface charge, signed */
    ORC_G_NODE_KIND = 7,   /* int32: -1 unknown, >=0 conductor id */
    ORC_G_CELL_KIND = 8,   /* int32: 0 vacuum, 1 dielectric, 2+id conductor */
    ORC_G_VOL = 9, ORC_G_PHI_L = 10, ORC_G_Q = 11, ORC_G_AR = 12, ORC_G_AZ = 13,
    ORC_G_NE_AVG = 14, ORC_G_NI_AVG = 15
};

int orc_create(const orc_config* cfg, orc_sim** out);
void orc_destroy(orc_sim* s);
int orc_step(orc_sim* s, int32_t nsteps);
int orc_diag_get(orc_sim* s, orc_diag* d);
int orc_series(orc_sim* s, int32_t last, double* U_out, double* I_out);

/* particles as 9 field-major arrays of length n: r z vr vt vz ar at az w */
int64_t orc_num_slots(orc_sim* s, int32_t species);
int orc_get_particles(orc_sim* s, int32_t species, double* out9);
int orc_set_particles(orc_sim* s, int32_t species, int64_t n, const double* in9);
int orc_redeposit(orc_sim* s);
int orc_get_grid(orc_sim* s, int32_t which, void* out);
int orc_set_grid(orc_sim* s, int32_t which, const void* in);
int orc_set_state(orc_sim* s, const double* st); /* t, Q_E, U_E, circ[5], C_eq */
/* [R32] one splitting pass over a species now; *added = copies appended */
int orc_split_now(orc_sim* s, int32_t species, int64_t* added);
/* [R33] one solve with the driven electrodes at U[0 .. n_el-1] */
int orc_solve_qv(orc_sim* s, const double* Q, const double* chi, const double* U, double tol,
                 double* phi_inout, int32_t* iters, double* relres);
/* [R33] Laplace solution of driven electrode e (1-based) at 1 V, others 0 */
int orc_get_phiL(orc_sim* s, int32_t e, double* out);
/* [R32] reference weight of a particle in cell column i (units of w_unit) */
double orc_split_target(orc_sim* s, int32_t species, int32_t i);

/* pure pieces, for pins */
int orc_assemble_now(orc_sim* s);        /* CHI and Q grids from the deposits as they stand */
int orc_efield_now(orc_sim* s);          /* ER and EZ grids from the PHI grid as it stands */
int orc_gather(orc_sim* s, int64_t n, const double* r, const double* z, double* Er, double* Ez);
int orc_solve_q(orc_sim* s, const double* Q, const double* chi, double U_E, double tol,
                double* phi_inout, int32_t* iters, double* relres);
double orc_refresh_laplace(orc_sim* s); /* recompute phi_L and C_eq with the current chi */
double orc_ceq_flux(orc_sim* s);         /* C_eq as the flux out of the electrode */
int orc_deposit(orc_sim* s, int64_t n, const double* r, const double* z, const double* w, int64_t* grid);
/* energy moment of species sp: node sums of the integer weight shares (N)
   and of shares times floor(16 kinetic energy / eV) (E); mean energy
   E / (16 N) eV */
int orc_moments(orc_sim* s, int sp, int64_t* N, int64_t* E);
int orc_tile_keys(orc_sim* s, int64_t n, const double* r, const double* z, uint32_t* keys);
int orc_stable_perm(int64_t n, const uint32_t* keys, int64_t* perm);
int orc_predict(orc_sim* s, int64_t n, double* p9);
int orc_correct(orc_sim* s, int32_t species, int64_t n, double* p9, const double* Er, const double* Ez);
int orc_mcc(orc_sim* s, int32_t species, int64_t n, double* v3, uint32_t slot0, uint32_t step,
            int32_t* proc, double* birth6);
void orc_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
void orc_xsec_e(double eps_eV, double out3[3]);
/* |Gamma| (Eq. 12), forward and reflected power (Eq. 14) of a load Z_load
   against R_s: out3 = |Gamma|, P_forward, P_ref */
void orc_reflection(double z_re, double z_im, double R_s, double P_source, double P_Rs, double* out3);

/* matching design (Sec. 3): C_m1, C_m2 of the L-network of cfg (its R_s,
   R_m, L_m and stray branch) that match a load C_eq perfectly; out2 =
   C_m1, C_m2.  -1 when no such network exists. */
int orc_match_design(const orc_config* cfg, double C_eq, double* out2);

/* the circuit alone with a fixed C_eq and no plasma; chars (or NULL): the
   electrical characterisation of the last period, as orc_diag.elec */
int orc_circuit_vacuum(const orc_config* cfg, double C_eq, int64_t nsteps, double* U_out, double* I_out,
                       double* chars);

#ifdef __cplusplus
}
#endif
#endif
