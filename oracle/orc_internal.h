/* Internal state of the oracle (test infrastructure only; see oracle.h). */
#ifndef PIC_ORC_INTERNAL_H
#define PIC_ORC_INTERNAL_H
#include "oracle.h"
#include <stddef.h>

/* CODATA 2018 */
#define O_QE 1.602176634e-19
#define O_ME 9.1093837015e-31
#define O_AMU 1.66053906660e-27
#define O_MAR (39.948 * O_AMU)
#define O_EPS0 8.8541878128e-12
#define O_KB 1.380649e-23
#define O_PI 3.14159265358979323846

/* fixed-point deposit definition: F fraction bits of position, K bits of weight */
#define O_FBITS 20
#define O_KBITS 32
#define O_TILE_SHIFT 4 /* sort tiles of 16x16 cells */

typedef struct {
    int64_t n, cap;
    double *r, *z, *vr, *vt, *vz, *ar, *at, *az, *w;
} o_parts;

typedef struct { /* one multigrid level: 9-point stencil, (nr+1)*(nz+1) nodes */
    int nr, nz, cr, cz; /* cr/cz: coarsening factor from this level to the next */
    double dr, dz;
    double* A[9];       /* A[k][n]: coupling of node n with neighbour offset k (k = (dj+1)*3 + (di+1)) */
    double *x, *b, *res;
} o_level;

struct orc_sim {
    orc_config cfg;
    int nr, nz, nn; /* cells, nodes = (nr+1)*(nz+1) */
    double dr, dz, dt, Sr, Sz;
    double* invd; /* 2^-2F / (2i+1) */
    int32_t *cell_kind, *node_kind;
    double *cell_eps, *vol, *gr, *gz; /* gr/gz: face factors without (1+chi) */
    /* particles */
    o_parts p[2];
    double qm[2], mass[2];
    int sign[2];
    double w_unit, n_gas, nu_max[2], vth_gas;
    double vvac, wref[2];   /* vacuum volume; loading weight of each species */
    int nvac;               /* vacuum cells */
    int64_t split_added[2];
    uint32_t thresh[2];
    /* grids */
    int64_t *dep[2], *wallq, *psum[2], *plast[2];
    double *phi, *Er, *Ez, *chi, *Q, *ar, *az;
    /* driven electrodes e = 0 .. n_el-1 (conductor id e + 1) [R33]: Laplace
       solutions, capacitance matrix, charges, voltages, induced charges,
       circuit currents and states */
    int n_el;
    double* phiL[ORC_MAX_EL];
    double Cm[ORC_MAX_EL][ORC_MAX_EL];
    double t, Q_E[ORC_MAX_EL], U_E[ORC_MAX_EL], Q_P[ORC_MAX_EL], I_ccp[ORC_MAX_EL], circ[ORC_MAX_EL][5];
    /* absorption counters: slot_of(conductor id); 2 lost, 3 dielectric */
    int64_t cnt[2][8], cnt_prev[ORC_MAX_EL];
    /* diagnostics */
    int64_t step, periods_done, born, coll[2][4], viol;
    double *serU[ORC_MAX_EL], *serI[ORC_MAX_EL], *lastU[ORC_MAX_EL], *lastI[ORC_MAX_EL];
    double *serVin, *serI1, *lastVin, *lastI1;   /* source-side voltage and current per step */
    double energy[5], last_energy[5];            /* element energies of the current / last period */
    int64_t solver_iters;
    double solver_relres;
    int have_last;
};

void o_characterise(const orc_config* c, const double* U, const double* I, const double* Vin, const double* I1,
                    const double* energy, double* chars);

/* field (orc_field.c) */
int o_geometry(orc_sim* s);
void o_assemble(orc_sim* s);
void o_faces_from_chi(orc_sim* s, const double* chi, double* ar, double* az);
int o_solve(orc_sim* s, const double* ar, const double* az, const double* Q, const double* U, double tol,
            double* phi, int* iters, double* relres);
/* absorption counter slot of conductor id: 0 ground, 1 electrode 1, 4 + (id - 2) electrodes >= 2 */
static inline int o_slot_of(int id) { return id <= 1 ? id : 2 + id; }
double o_laplace(orc_sim* s);
void o_efield(orc_sim* s);

/* particles (orc_particles.c) */
typedef struct { int inside, edge; int64_t qr, qz; int i, j; int64_t fr, fz; } o_loc;
o_loc o_locate(const orc_sim* s, double r, double z);
double o_split_target(const orc_sim* s, int sp, int i);
void o_deposit_one(const orc_sim* s, double r, double z, double W, int64_t* grid);
void o_node_weights(const orc_sim* s, const o_loc* L, double W, int64_t c[4]);
void o_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double o_u01(uint32_t x);
void o_predict1(const orc_sim* s, double* st);
void o_correct1(const orc_sim* s, int sp, double* st, double Er, double Ez);
void o_gather(const orc_sim* s, double r, double z, double* Er, double* Ez);
int o_mcc1(orc_sim* s, int sp, double* v, uint32_t slot, uint32_t step, double* birth6);
void o_xsec_e(double eps, double* el, double* ex, double* io);
int o_absorb_check(orc_sim* s, int sp, double r, double z, double W);
void o_set_collision_constants(orc_sim* s);
int o_load(orc_sim* s);

/* circuit (orc_sim.c) */
void o_circuit_advance(orc_sim* s);

#endif
