/*
 * orc_sim.c -- oracle (test infrastructure only): the external circuit
 * (Eqs. 8-10) coupled by the equivalent capacitance (Eq. 5), the time step
 * in the paper's order, sorting, diagnostics (Sec. 3: period-averaged
 * densities, electrode voltage and current harmonics), and the C entry
 * points used by the Python tests.
 */
#include "orc_internal.h"
#include <stdio.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- circuit */
/* the external circuit of driven electrode e (0-based) [R33] */
static orc_circ circ_of(const orc_config* c, int e) {
    if (e > 0) return c->circ_el[e - 1];
    orc_circ k;
    k.kind = c->circ_kind; k.substeps = c->substeps;
    k.freq = c->freq; k.U_amp = c->U_amp; k.U_dc = c->U_dc; k.R_s = c->R_s;
    k.C_m1 = c->C_m1; k.C_m2 = c->C_m2; k.L_m = c->L_m; k.R_m = c->R_m;
    k.C_stray = c->C_stray; k.L_stray = c->L_stray; k.R_stray = c->R_stray;
    k.C_b = c->C_b; k.R_b = c->R_b; k.L_b = c->L_b;
    return k;
}

static double source_v(const orc_circ* c, double t) { return c->U_amp * sin(2.0 * O_PI * c->freq * t) + c->U_dc; }

/* State y: L-match (Eq. 10) y0..y4 = Q1, Q2, I2, Q_ccp, I_stray;
   series RLC (Eq. 9) y0, y1 = Q_b, I_b; y5 = Q_E, the electrode charge of
   Eq. (8), dQ_E/dt = I_ccp + I_conv, for the electrode voltage U_E. */
static void circ_rhs(const orc_circ* c, double U_E, double t, const double* y, double I_conv, double* dy) {
    double Us = source_v(c, t);
    for (int k = 0; k < 6; k++) dy[k] = 0.0;
    if (c->kind == 2) {
        double Um1 = (y[0] - y[1]) / c->C_m1;
        dy[0] = (Us - Um1) / c->R_s;
        dy[1] = y[2];
        dy[2] = (Um1 - U_E - y[1] / c->C_m2 - y[2] * c->R_m) / c->L_m;
        dy[3] = y[2] - y[4];
        dy[4] = (U_E - (y[1] - y[3]) / c->C_stray - y[4] * c->R_stray) / c->L_stray;
        dy[5] = (y[2] - y[4]) + I_conv;
    } else if (c->kind == 1) {
        dy[0] = y[1];
        dy[1] = (Us - U_E - y[0] / c->C_b - y[1] * c->R_b) / c->L_b;
        dy[5] = y[1] + I_conv;
    }
}

/* Instantaneous powers of the circuit elements for state y at time t
   (Eq. 13 integrands) [R30]: 0 delivered by the source, 1 lost in R_s,
   2 lost in the matching network (R_m) or in the series branch (R_b),
   3 lost in the stray branch, 4 delivered to the plasma load U_E I_ccp. */
static void circ_powers(const orc_circ* c, double U_E, double t, const double* y, double* p) {
    double Us = source_v(c, t);
    for (int k = 0; k < 5; k++) p[k] = 0.0;
    if (c->kind == 2) {
        double I1 = (Us - (y[0] - y[1]) / c->C_m1) / c->R_s;
        p[0] = Us * I1;
        p[1] = c->R_s * I1 * I1;
        p[2] = c->R_m * y[2] * y[2];
        p[3] = c->R_stray * y[4] * y[4];
        p[4] = U_E * (y[2] - y[4]);
    } else if (c->kind == 1) {
        p[0] = Us * y[1];
        p[2] = c->R_b * y[1] * y[1];
        p[4] = U_E * y[1];
    }
}

/* The driven electrodes' circuits, coupled through the capacitance matrix.
   [R16] with one electrode U_E = (Q_E - Q_P)/C_eq, Q_P = -sum phi_L Q the
   charge the space charge induces on it (Green reciprocity); in vacuum
   Eq. (5).  [R33] with several: Q = C U + Q_P, so an ideal source fixes its
   electrode's voltage and the others solve C_NN U_N = Q_N - Q_P,N - C_NK U_K. */
typedef struct {
    int M;
    orc_circ c[ORC_MAX_EL];
    double C[ORC_MAX_EL][ORC_MAX_EL];
    double QP[ORC_MAX_EL], Iconv[ORC_MAX_EL];
} o_circset;

static void volts(const o_circset* cs, double t, double Y[][6], double* U) {
    int N[ORC_MAX_EL], nN = 0;
    for (int e = 0; e < cs->M; e++) {
        if (cs->c[e].kind == 0) U[e] = source_v(&cs->c[e], t);
        else N[nN++] = e;
    }
    if (nN == 0) return;
    double A[ORC_MAX_EL][ORC_MAX_EL], b[ORC_MAX_EL];
    for (int a = 0; a < nN; a++) {
        int e = N[a];
        b[a] = Y[e][5] - cs->QP[e];
        for (int f = 0; f < cs->M; f++)
            if (cs->c[f].kind == 0) b[a] -= cs->C[e][f] * U[f];
        for (int q = 0; q < nN; q++) A[a][q] = cs->C[e][N[q]];
    }
    /* Gaussian elimination; A is symmetric positive definite */
    for (int p = 0; p < nN; p++)
        for (int a = p + 1; a < nN; a++) {
            double m = A[a][p] / A[p][p];
            for (int q = p; q < nN; q++) A[a][q] -= m * A[p][q];
            b[a] -= m * b[p];
        }
    for (int a = nN - 1; a >= 0; a--) {
        double x = b[a];
        for (int q = a + 1; q < nN; q++) x -= A[a][q] * U[N[q]];
        U[N[a]] = x / A[a][a];
    }
}

/* [R17] classical RK4 of the coupled circuit states over one PIC step, the
   largest substep count of the circuits; I_conv and Q_P are held over the
   step.  Iavg: each circuit's step-averaged current.  With e5, adds the
   element energies of electrode 1's circuit (trapezoid rule on the substep
   end points). */
static void circ_step(const o_circset* cs, double dt, double t0, double Y[][6], double* e5, double* Iavg) {
    int M = 0, qi[ORC_MAX_EL];
    double q0[ORC_MAX_EL];
    for (int e = 0; e < cs->M; e++) {
        qi[e] = (cs->c[e].kind == 2) ? 3 : 0;
        q0[e] = Y[e][qi[e]];
        if (cs->c[e].kind != 0) {
            int ms = cs->c[e].substeps > 0 ? cs->c[e].substeps : 1;
            if (ms > M) M = ms;
        }
    }
    if (M == 0) return;
    double h = dt / M;
    double U[ORC_MAX_EL], pa[5], pb[5];
    int pe = (e5 != NULL) && cs->c[0].kind != 0;
    if (pe) {
        volts(cs, t0, Y, U);
        circ_powers(&cs->c[0], U[0], t0, Y[0], pa);
    }
    for (int m = 0; m < M; m++) {
        double t = t0 + m * h;
        double k1[ORC_MAX_EL][6], k2[ORC_MAX_EL][6], k3[ORC_MAX_EL][6], k4[ORC_MAX_EL][6], yt[ORC_MAX_EL][6];
        volts(cs, t, Y, U);
        for (int e = 0; e < cs->M; e++) if (cs->c[e].kind) circ_rhs(&cs->c[e], U[e], t, Y[e], cs->Iconv[e], k1[e]);
        for (int e = 0; e < cs->M; e++) for (int k = 0; k < 6; k++) yt[e][k] = Y[e][k] + 0.5 * h * k1[e][k];
        volts(cs, t + 0.5 * h, yt, U);
        for (int e = 0; e < cs->M; e++) if (cs->c[e].kind) circ_rhs(&cs->c[e], U[e], t + 0.5 * h, yt[e], cs->Iconv[e], k2[e]);
        for (int e = 0; e < cs->M; e++) for (int k = 0; k < 6; k++) yt[e][k] = Y[e][k] + 0.5 * h * k2[e][k];
        volts(cs, t + 0.5 * h, yt, U);
        for (int e = 0; e < cs->M; e++) if (cs->c[e].kind) circ_rhs(&cs->c[e], U[e], t + 0.5 * h, yt[e], cs->Iconv[e], k3[e]);
        for (int e = 0; e < cs->M; e++) for (int k = 0; k < 6; k++) yt[e][k] = Y[e][k] + h * k3[e][k];
        volts(cs, t + h, yt, U);
        for (int e = 0; e < cs->M; e++) if (cs->c[e].kind) circ_rhs(&cs->c[e], U[e], t + h, yt[e], cs->Iconv[e], k4[e]);
        for (int e = 0; e < cs->M; e++)
            if (cs->c[e].kind)
                for (int k = 0; k < 6; k++) Y[e][k] += h / 6.0 * (k1[e][k] + 2.0 * k2[e][k] + 2.0 * k3[e][k] + k4[e][k]);
        if (pe) {
            volts(cs, t + h, Y, U);
            circ_powers(&cs->c[0], U[0], t + h, Y[0], pb);
            for (int k = 0; k < 5; k++) {
                e5[k] += 0.5 * h * (pa[k] + pb[k]);
                pa[k] = pb[k];
            }
        }
    }
    for (int e = 0; e < cs->M; e++)
        if (cs->c[e].kind) Iavg[e] = (Y[e][qi[e]] - q0[e]) / dt;
}

/* Source-side samples of a step for the load impedance: the voltage at the
   matching network's input (across C_m1) or the source voltage, at t1. */
static double circ_vin(const orc_circ* c, double t1, const double* y) {
    if (c->kind == 2) return (y[0] - y[1]) / c->C_m1;
    return source_v(c, t1);
}

/* net charge absorbed by driven electrode e (units 2^-32 w_unit) */
static double electrode_count(const orc_sim* s, int e) {
    int slot = o_slot_of(e + 1);
    return (double)(s->sign[1] * s->cnt[1][slot] + s->sign[0] * s->cnt[0][slot]);
}

static double induced_charge(const orc_sim* s, int e) {
    double qp = 0.0;
    for (int n = 0; n < s->nn; n++)
        if (s->node_kind[n] < 0) qp -= s->phiL[e][n] * s->Q[n];
    return qp;
}

static void circset_of(const orc_sim* s, o_circset* cs) {
    cs->M = s->n_el;
    for (int e = 0; e < s->n_el; e++) {
        cs->c[e] = circ_of(&s->cfg, e);
        for (int f = 0; f < s->n_el; f++) cs->C[e][f] = s->Cm[e][f];
        cs->QP[e] = 0.0;
        cs->Iconv[e] = 0.0;
    }
}

/* charge of an electrode held by an ideal source: Q = sum_f C_ef U_f + Q_P */
static double held_charge(const o_circset* cs, int e, const double* U) {
    double q = 0.0;
    for (int f = 0; f < cs->M; f++) q += cs->C[e][f] * U[f];
    return q + cs->QP[e];
}

void o_circuit_advance(orc_sim* s) {
    double unit = O_QE * s->w_unit * ldexp(1.0, -O_KBITS);
    int k = (int)(s->step % s->cfg.steps_per_period);
    o_circset cs;
    circset_of(s, &cs);
    for (int e = 0; e < s->n_el; e++) {
        double pc = electrode_count(s, e);
        cs.Iconv[e] = (pc - (double)s->cnt_prev[e]) * unit / s->dt;
        s->cnt_prev[e] = (int64_t)pc;
        cs.QP[e] = induced_charge(s, e);
        s->Q_P[e] = cs.QP[e];
    }
    double t1 = s->t + s->dt;
    double U0 = s->U_E[0];
    double Y[ORC_MAX_EL][6], Iavg[ORC_MAX_EL], U[ORC_MAX_EL];
    for (int e = 0; e < s->n_el; e++) {
        for (int q = 0; q < 5; q++) Y[e][q] = s->circ[e][q];
        Y[e][5] = s->Q_E[e];
    }
    double q1 = Y[0][0];
    circ_step(&cs, s->dt, s->t, Y, s->energy, Iavg);
    volts(&cs, t1, Y, U);
    for (int e = 0; e < s->n_el; e++) {
        if (cs.c[e].kind == 0) {
            double QE = held_charge(&cs, e, U);
            s->I_ccp[e] = (QE - s->Q_E[e]) / s->dt - cs.Iconv[e];
            s->Q_E[e] = QE;
        } else {
            for (int q = 0; q < 5; q++) s->circ[e][q] = Y[e][q];
            s->Q_E[e] = Y[e][5];
            s->I_ccp[e] = Iavg[e];
        }
        s->U_E[e] = U[e];
    }
    /* electrode 1: source-side samples and, for an ideal source, energies */
    if (cs.c[0].kind == 0) {
        /* the source is the electrode: the mean voltage over the step times
           the step-averaged current */
        double e = s->dt * 0.5 * (U0 + U[0]) * s->I_ccp[0];
        s->energy[0] += e;
        s->energy[4] += e;
        s->serVin[k] = U[0];
        s->serI1[k] = s->I_ccp[0];
    } else {
        s->serVin[k] = circ_vin(&cs.c[0], t1, Y[0]);
        s->serI1[k] = (cs.c[0].kind == 2) ? (Y[0][0] - q1) / s->dt : s->I_ccp[0];
    }
    s->t = t1;
}

int orc_circuit_vacuum(const orc_config* cfg, double C_eq, int64_t nsteps, double* U_out, double* I_out,
                       double* chars) {
    double dt = 1.0 / (cfg->freq * cfg->steps_per_period);
    int spp = cfg->steps_per_period;
    o_circset cs;
    cs.M = 1;
    cs.c[0] = circ_of(cfg, 0);
    cs.C[0][0] = C_eq;
    cs.QP[0] = 0.0;
    cs.Iconv[0] = 0.0;
    double Y[1][6] = {{0, 0, 0, 0, 0, 0}};
    double t = 0.0, e[5] = {0, 0, 0, 0, 0};
    double* vin = calloc((size_t)spp, sizeof(double));
    double* i1 = calloc((size_t)spp, sizeof(double));
    double* uu = calloc((size_t)spp, sizeof(double));
    double* ii = calloc((size_t)spp, sizeof(double));
    if (!vin || !i1 || !uu || !ii) { free(vin); free(i1); free(uu); free(ii); return -1; }
    for (int64_t n = 0; n < nsteps; n++) {
        int last_period = n >= nsteps - spp;
        double q1 = Y[0][0];
        double I = 0.0;
        circ_step(&cs, dt, t, Y, last_period ? e : NULL, &I);
        t += dt;
        U_out[n] = Y[0][5] / C_eq;
        I_out[n] = I;
        if (last_period) {
            int k = (int)(n - (nsteps - spp));
            uu[k] = U_out[n];
            ii[k] = I;
            vin[k] = circ_vin(&cs.c[0], t, Y[0]);
            i1[k] = (cfg->circ_kind == 2) ? (Y[0][0] - q1) / dt : I;
        }
    }
    if (chars && nsteps >= spp) o_characterise(cfg, uu, ii, vin, i1, e, chars);
    free(vin); free(i1); free(uu); free(ii);
    return 0;
}

/* ---------------------------------------------------------------- helpers */
static int parts_alloc(o_parts* P, int64_t cap) {
    P->cap = cap;
    P->n = 0;
    double** f[9] = {&P->r, &P->z, &P->vr, &P->vt, &P->vz, &P->ar, &P->at, &P->az, &P->w};
    for (int k = 0; k < 9; k++) {
        *f[k] = calloc((size_t)(cap > 0 ? cap : 1), sizeof(double));
        if (!*f[k]) return -1;
    }
    return 0;
}

static void parts_free(o_parts* P) {
    free(P->r); free(P->z); free(P->vr); free(P->vt); free(P->vz);
    free(P->ar); free(P->at); free(P->az); free(P->w);
}

static void get1(const o_parts* P, int64_t k, double* st) {
    st[0] = P->r[k]; st[1] = P->z[k]; st[2] = P->vr[k]; st[3] = P->vt[k]; st[4] = P->vz[k];
    st[5] = P->ar[k]; st[6] = P->at[k]; st[7] = P->az[k]; st[8] = P->w[k];
}

static void put1(o_parts* P, int64_t k, const double* st) {
    P->r[k] = st[0]; P->z[k] = st[1]; P->vr[k] = st[2]; P->vt[k] = st[3]; P->vz[k] = st[4];
    P->ar[k] = st[5]; P->at[k] = st[6]; P->az[k] = st[7]; P->w[k] = st[8];
}

static uint32_t tile_key(const orc_sim* s, double r, double z) {
    if (r < 0.0) return 0xFFFFFFFFu;
    o_loc L = o_locate(s, r, z);
    if (!L.inside) return 0xFFFFFFFFu;
    int ntr = (s->nr + (1 << O_TILE_SHIFT) - 1) >> O_TILE_SHIFT;
    return (uint32_t)((L.j >> O_TILE_SHIFT) * ntr + (L.i >> O_TILE_SHIFT));
}

typedef struct { uint32_t key; int64_t idx; } kv;
static int kv_cmp(const void* a, const void* b) {
    const kv *x = a, *y = b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

int orc_stable_perm(int64_t n, const uint32_t* keys, int64_t* perm) {
    kv* a = malloc(sizeof(kv) * (size_t)(n > 0 ? n : 1));
    for (int64_t k = 0; k < n; k++) { a[k].key = keys[k]; a[k].idx = k; }
    qsort(a, (size_t)n, sizeof(kv), kv_cmp);
    for (int64_t k = 0; k < n; k++) perm[k] = a[k].idx;
    free(a);
    return 0;
}

/* stable sort by tile key of the predicted position; dead slots dropped */
static void sort_species(orc_sim* s, int sp) {
    o_parts* P = &s->p[sp];
    int64_t n = P->n;
    uint32_t* keys = calloc((size_t)(n > 0 ? n : 1), sizeof(uint32_t));
    int64_t* perm = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!keys || !perm) {
        fprintf(stderr, "oracle: out of memory in the tile sort\n");
        abort();
    }
    for (int64_t k = 0; k < n; k++) keys[k] = tile_key(s, P->r[k], P->z[k]);
    orc_stable_perm(n, keys, perm);
    o_parts Q;
    parts_alloc(&Q, P->cap);
    int64_t m = 0;
    double st[9];
    for (int64_t k = 0; k < n; k++) {
        if (keys[perm[k]] == 0xFFFFFFFFu) break;
        get1(P, perm[k], st);
        put1(&Q, m++, st);
    }
    Q.n = m;
    parts_free(P);
    *P = Q;
    free(keys);
    free(perm);
}

/* [R32] Particle splitting.  A live particle inside the domain whose weight
   w (compared in single precision) is at least 2^m times the reference
   weight of its cell column is replaced by k = 2^m identical particles of
   weight w / k, m at most 3: the parent keeps its slot with weight w / k and
   the k - 1 copies follow the last slot, in parent order.  Position,
   velocity and averaged acceleration are copied, so charge, momentum and
   kinetic energy are unchanged exactly (k is a power of two). */
static int split_doublings(float w, float t) {
    int m = 0;
    while (m < 3 && w >= t * (float)(2 << m)) m++;
    return m;
}

static int split_of(orc_sim* s, int sp, int64_t k) {
    const o_parts* P = &s->p[sp];
    if (!(P->r[k] >= 0.0)) return 0;
    o_loc L = o_locate(s, P->r[k], P->z[k]);
    if (!L.inside) return 0;
    return split_doublings((float)P->w[k], (float)o_split_target(s, sp, L.i));
}

/* nothing changes when the copies would not fit (returns -2) */
static int split_species(orc_sim* s, int sp, int64_t* added) {
    o_parts* P = &s->p[sp];
    int64_t n = P->n, m = n, total = 0;
    double st[9];
    for (int64_t k = 0; k < n; k++) total += (1 << split_of(s, sp, k)) - 1;
    if (n + total > P->cap) return -2;
    for (int64_t k = 0; k < n; k++) {
        int d = split_of(s, sp, k);
        if (d == 0) continue;
        int kk = 1 << d;
        get1(P, k, st);
        st[8] = st[8] / kk;
        put1(P, k, st);
        for (int c = 1; c < kk; c++) put1(P, m++, st);
    }
    P->n = m;
    s->split_added[sp] += m - n;
    if (added) *added = m - n;
    return 0;
}

/* ------------------------------------------------------------------ step */
typedef struct { double r, z, W, v[6]; } o_birth;

static int particle_pass(orc_sim* s, int sp, o_birth** births, int64_t* nb, int64_t* capb, uint32_t step) {
    o_parts* P = &s->p[sp];
    double st[9];
    for (int64_t k = 0; k < P->n; k++) {
        if (P->r[k] < 0.0) continue;
        get1(P, k, st);
        double Er, Ez;
        o_gather(s, st[0], st[1], &Er, &Ez);
        o_correct1(s, sp, st, Er, Ez);
        if (o_absorb_check(s, sp, st[0], st[1], st[8])) { P->r[k] = -1.0; continue; }
        double v[3] = {st[2], st[3], st[4]}, b6[6];
        int proc = o_mcc1(s, sp, v, (uint32_t)k, step, b6);
        if (proc >= 0) s->coll[sp][proc]++;
        st[2] = v[0]; st[3] = v[1]; st[4] = v[2];
        if (proc == 2 && sp == 0) {
            if (*nb == *capb) {
                *capb = *capb * 2 + 16;
                *births = realloc(*births, sizeof(o_birth) * (size_t)*capb);
            }
            o_birth* b = &(*births)[(*nb)++];
            b->r = st[0]; b->z = st[1]; b->W = st[8];
            memcpy(b->v, b6, sizeof(b6));
        }
        o_predict1(s, st);
        if (o_absorb_check(s, sp, st[0], st[1], st[8])) { P->r[k] = -1.0; continue; }
        put1(P, k, st);
        o_deposit_one(s, st[0], st[1], st[8], s->dep[sp]);
    }
    return 0;
}

static int append_births(orc_sim* s, const o_birth* b, int64_t nb) {
    if (s->p[0].n + nb > s->p[0].cap || s->p[1].n + nb > s->p[1].cap) return -2;
    for (int64_t k = 0; k < nb; k++) {
        for (int sp = 0; sp < 2; sp++) {
            double st[9] = {b[k].r, b[k].z, b[k].v[3 * sp], b[k].v[3 * sp + 1], b[k].v[3 * sp + 2],
                            0.0, 0.0, 0.0, b[k].W};
            o_predict1(s, st);
            o_parts* P = &s->p[sp];
            int64_t slot = P->n++;
            if (o_absorb_check(s, sp, st[0], st[1], st[8])) {
                put1(P, slot, st);
                P->r[slot] = -1.0;
                continue;
            }
            put1(P, slot, st);
            o_deposit_one(s, st[0], st[1], st[8], s->dep[sp]);
        }
        s->born++;
    }
    return 0;
}

/* One time step in the paper's order (Sec. 2): the susceptibility and the
   predicted charge define Eq. (1); the electrode voltage comes from the
   electrode charge and the equivalent capacitance (Eqs. 5, 8-10); the field
   solve; then the particle loop (gather, implicit correction, absorption,
   null-collision MCC, prediction and deposit of the next predicted
   positions), births, the periodic sort and the once-per-period refresh of
   the Laplace solution and C_eq. */
static int step1(orc_sim* s) {
    int spp = s->cfg.steps_per_period;
    int k = (int)(s->step % spp);
    o_assemble(s);
    for (int sp = 0; sp < 2; sp++)
        for (int n = 0; n < s->nn; n++) s->psum[sp][n] += s->dep[sp][n];
    o_circuit_advance(s);
    int it;
    double rel;
    int rc = o_solve(s, s->ar, s->az, s->Q, s->U_E, s->cfg.tol, s->phi, &it, &rel);
    s->solver_iters = it;
    s->solver_relres = rel;
    if (rc) return rc;
    o_efield(s);
    for (int e = 0; e < s->n_el; e++) {
        s->serU[e][k] = s->U_E[e];
        s->serI[e][k] = s->I_ccp[e];
    }
    for (int sp = 0; sp < 2; sp++) memset(s->dep[sp], 0, sizeof(int64_t) * s->nn);
    uint32_t stepc = (uint32_t)(s->step + 1);
    o_birth* births = NULL;
    int64_t nb = 0, capb = 0;
    particle_pass(s, 0, &births, &nb, &capb, stepc);
    particle_pass(s, 1, &births, &nb, &capb, stepc);
    rc = append_births(s, births, nb);
    free(births);
    if (rc) return rc;
    s->step++;
    for (int sp = 0; sp < 2; sp++) {
        int every = sp == 0 ? s->cfg.sort_every : s->cfg.sort_every_ion;
        if (every > 0 && s->step % every == 0) {
            /* [R32] splitting runs at the species' tile sort, before it */
            if (s->cfg.split && split_species(s, sp, NULL)) return -2;
            sort_species(s, sp);
        }
    }
    if (s->step % spp == 0) {
        o_laplace(s);
        for (int e = 0; e < s->n_el; e++) {
            memcpy(s->lastU[e], s->serU[e], sizeof(double) * spp);
            memcpy(s->lastI[e], s->serI[e], sizeof(double) * spp);
        }
        memcpy(s->lastVin, s->serVin, sizeof(double) * spp);
        memcpy(s->lastI1, s->serI1, sizeof(double) * spp);
        for (int q = 0; q < 5; q++) { s->last_energy[q] = s->energy[q]; s->energy[q] = 0.0; }
        for (int sp = 0; sp < 2; sp++) {
            memcpy(s->plast[sp], s->psum[sp], sizeof(int64_t) * s->nn);
            memset(s->psum[sp], 0, sizeof(int64_t) * s->nn);
        }
        s->periods_done++;
        s->have_last = 1;
    }
    return 0;
}

int orc_step(orc_sim* s, int32_t nsteps) {
    for (int32_t k = 0; k < nsteps; k++) {
        int rc = step1(s);
        if (rc) return rc;
    }
    return 0;
}

/* ------------------------------------------------------------ create/free */
int orc_create(const orc_config* cfg, orc_sim** out) {
    if (cfg->nr < 2 || cfg->nz < 2 || cfg->R <= 0 || cfg->Z <= 0 || cfg->steps_per_period < 1 ||
        cfg->n_regions < 0 || cfg->n_regions > ORC_MAX_REGIONS || cfg->freq <= 0 || cfg->n_el < 0 ||
        cfg->n_el > ORC_MAX_EL)
        return -1;
    orc_sim* s = calloc(1, sizeof(orc_sim));
    s->cfg = *cfg;
    s->n_el = cfg->n_el > 0 ? cfg->n_el : 1;
    s->nr = cfg->nr;
    s->nz = cfg->nz;
    s->nn = (cfg->nr + 1) * (cfg->nz + 1);
    s->dt = 1.0 / (cfg->freq * cfg->steps_per_period);
    if (o_geometry(s)) { orc_destroy(s); return -1; }
    s->Sr = ldexp(1.0, O_FBITS) / s->dr;
    s->Sz = ldexp(1.0, O_FBITS) / s->dz;
    s->invd = malloc(sizeof(double) * s->nr);
    for (int i = 0; i < s->nr; i++) s->invd[i] = ldexp(1.0, -2 * O_FBITS) / (double)(2 * i + 1);
    s->mass[0] = O_ME;
    s->mass[1] = O_MAR;
    s->qm[0] = -O_QE / O_ME;
    s->qm[1] = O_QE / O_MAR;
    s->sign[0] = -1;
    s->sign[1] = 1;
    o_set_collision_constants(s);
    int64_t caps[2] = {cfg->cap_e, cfg->cap_i};
    for (int sp = 0; sp < 2; sp++) {
        if (parts_alloc(&s->p[sp], caps[sp])) { orc_destroy(s); return -1; }
        s->dep[sp] = calloc(s->nn, sizeof(int64_t));
        s->psum[sp] = calloc(s->nn, sizeof(int64_t));
        s->plast[sp] = calloc(s->nn, sizeof(int64_t));
    }
    s->wallq = calloc(s->nn, sizeof(int64_t));
    double** g[7] = {&s->phi, &s->Er, &s->Ez, &s->chi, &s->Q, &s->ar, &s->az};
    for (int k = 0; k < 7; k++) *g[k] = calloc(s->nn, sizeof(double));
    int spp = cfg->steps_per_period;
    for (int e = 0; e < s->n_el; e++) {
        s->phiL[e] = calloc(s->nn, sizeof(double));
        s->serU[e] = calloc(spp, sizeof(double));
        s->serI[e] = calloc(spp, sizeof(double));
        s->lastU[e] = calloc(spp, sizeof(double));
        s->lastI[e] = calloc(spp, sizeof(double));
    }
    s->serVin = calloc(spp, sizeof(double));
    s->serI1 = calloc(spp, sizeof(double));
    s->lastVin = calloc(spp, sizeof(double));
    s->lastI1 = calloc(spp, sizeof(double));
    /* particles: the load fixes w_unit; with load = 0 the slots stay empty */
    orc_config save = s->cfg;
    if (!cfg->load) { s->cfg.n_e = 0; s->cfg.n_i = 0; }
    /* w_unit from the requested counts even when nothing is loaded */
    {
        double vv = 0.0;
        int nv = 0;
        for (int j = 0; j < s->nz; j++)
            for (int i = 0; i < s->nr; i++)
                if (s->cell_kind[j * s->nr + i] == 0) {
                    double r0 = i * s->dr, r1 = (i + 1) * s->dr;
                    vv += O_PI * (r1 * r1 - r0 * r0) * s->dz;
                    nv++;
                }
        s->w_unit = cfg->n0 * vv / (double)(cfg->n_e > 0 ? cfg->n_e : 1);
        /* loading weight of each species from the requested counts [R32] */
        s->vvac = vv;
        s->nvac = nv;
        int64_t nreq[2] = {cfg->n_e, cfg->n_i};
        for (int sp = 0; sp < 2; sp++)
            s->wref[sp] = (nreq[sp] > 0) ? (cfg->n0 * vv / (double)nreq[sp]) / s->w_unit : 1.0;
    }
    int rc = o_load(s);
    s->cfg = save;
    if (rc) { orc_destroy(s); return rc; }
    /* [R8] a_bar = 0 at start: the first prediction is a plain move */
    for (int sp = 0; sp < 2; sp++) {
        o_parts* P = &s->p[sp];
        double st[9];
        for (int64_t k = 0; k < P->n; k++) {
            get1(P, k, st);
            o_predict1(s, st);
            if (o_absorb_check(s, sp, st[0], st[1], st[8])) { put1(P, k, st); P->r[k] = -1.0; continue; }
            put1(P, k, st);
            o_deposit_one(s, st[0], st[1], st[8], s->dep[sp]);
        }
    }
    /* the loaded plasma starts tile-sorted, like every later sort */
    sort_species(s, 0);
    sort_species(s, 1);
    /* vacuum equivalent capacitance and Laplace solution at start [R21] */
    o_faces_from_chi(s, s->chi, s->ar, s->az);
    o_laplace(s);
    o_assemble(s);
    /* initial electrode voltages: an ideal source's DC value, else 0, with
       the charge Q = C U + Q_P that holds them */
    {
        o_circset cs;
        circset_of(s, &cs);
        double U[ORC_MAX_EL];
        for (int e = 0; e < s->n_el; e++) {
            cs.QP[e] = induced_charge(s, e);
            s->Q_P[e] = cs.QP[e];
            U[e] = (cs.c[e].kind == 0) ? cs.c[e].U_dc : 0.0;
            s->U_E[e] = U[e];
        }
        for (int e = 0; e < s->n_el; e++) {
            s->Q_E[e] = held_charge(&cs, e, U);
            s->cnt_prev[e] = (int64_t)electrode_count(s, e);
        }
    }
    *out = s;
    return 0;
}

void orc_destroy(orc_sim* s) {
    if (!s) return;
    free(s->invd); free(s->cell_kind); free(s->node_kind); free(s->cell_eps);
    free(s->vol); free(s->gr); free(s->gz);
    for (int sp = 0; sp < 2; sp++) {
        parts_free(&s->p[sp]);
        free(s->dep[sp]); free(s->psum[sp]); free(s->plast[sp]);
    }
    free(s->wallq);
    free(s->phi); free(s->Er); free(s->Ez); free(s->chi); free(s->Q);
    free(s->ar); free(s->az);
    for (int e = 0; e < ORC_MAX_EL; e++) {
        free(s->phiL[e]); free(s->serU[e]); free(s->serI[e]); free(s->lastU[e]); free(s->lastI[e]);
    }
    free(s->serVin); free(s->serI1); free(s->lastVin); free(s->lastI1);
    free(s);
}

/* ------------------------------------------------------------ diagnostics */
/* [R23] harmonics over the last complete RF period of N = steps_per_period
   samples: X_k = (2/N) sum_n x_n exp(-2 pi i k n / N), X_0 the mean (the DC
   self-bias for the voltage). */
static void harmonics(const double* x, int N, double* re, double* im) {
    for (int k = 0; k < 6; k++) {
        double a = 0.0, b = 0.0;
        for (int n = 0; n < N; n++) {
            double ph = 2.0 * O_PI * (double)k * (double)n / (double)N;
            a += x[n] * cos(ph);
            b -= x[n] * sin(ph);
        }
        double sc = (k == 0) ? 1.0 / N : 2.0 / N;
        re[k] = a * sc;
        im[k] = b * sc;
    }
}

/* Electrical characterisation of one RF period (Sec. 3, Eqs. 11-14)
   [R30].  Voltages are sampled at the end of each step, currents are step
   averages: the fundamental of a step average equals that of the sample at
   the step end times sinc(pi/N) exp(-i pi/N), which is divided out.
   chars: Z_ccp (re, im), Z_load (re, im), |Gamma|, P_source, P_Rs, P_IMN,
   P_stray, P_ccp, P_forward, P_ref. */
void o_characterise(const orc_config* c, const double* U, const double* I, const double* Vin, const double* I1,
                    const double* energy, double* chars) {
    int N = c->steps_per_period;
    double hu[2][6], hi[2][6], hv[2][6], h1[2][6];
    harmonics(U, N, hu[0], hu[1]);
    harmonics(I, N, hi[0], hi[1]);
    harmonics(Vin, N, hv[0], hv[1]);
    harmonics(I1, N, h1[0], h1[1]);
    double x = O_PI / N, sinc = sin(x) / x;
    double fr = sinc * cos(-x), fi = sinc * sin(-x);   /* sinc(pi/N) e^{-i pi/N} */
    /* complex a / (b / f) = a f / b */
    double zc[2], zl[2];
    {
        double nr = hu[0][1] * fr - hu[1][1] * fi, ni = hu[0][1] * fi + hu[1][1] * fr;
        double dd = hi[0][1] * hi[0][1] + hi[1][1] * hi[1][1];
        zc[0] = (nr * hi[0][1] + ni * hi[1][1]) / dd;
        zc[1] = (ni * hi[0][1] - nr * hi[1][1]) / dd;
    }
    {
        double nr = hv[0][1] * fr - hv[1][1] * fi, ni = hv[0][1] * fi + hv[1][1] * fr;
        double dd = h1[0][1] * h1[0][1] + h1[1][1] * h1[1][1];
        zl[0] = (nr * h1[0][1] + ni * h1[1][1]) / dd;
        zl[1] = (ni * h1[0][1] - nr * h1[1][1]) / dd;
    }
    const double T = 1.0 / c->freq;   /* one RF period */
    double P[5];
    for (int k = 0; k < 5; k++) P[k] = energy[k] / T;
    chars[0] = zc[0]; chars[1] = zc[1]; chars[2] = zl[0]; chars[3] = zl[1];
    for (int k = 0; k < 5; k++) chars[5 + k] = P[k];
    double gp[3];
    orc_reflection(zl[0], zl[1], c->circ_kind == 2 ? c->R_s : 0.0, P[0], P[1], gp);
    chars[4] = gp[0];
    chars[10] = gp[1];
    chars[11] = gp[2];
}

/* Eq. 12 and Eq. 14: |Gamma| of a load Z against the source resistance R_s
   (0 when there is none), the forward power into the matching network (the
   source's power less its internal loss) and the reflected power. */
void orc_reflection(double z_re, double z_im, double R_s, double P_source, double P_Rs, double* out3) {
    double gam = 0.0;
    if (R_s > 0.0) {
        double ar = z_re - R_s, br = z_re + R_s;
        gam = sqrt((ar * ar + z_im * z_im) / (br * br + z_im * z_im));
    }
    out3[0] = gam;
    out3[1] = P_source - P_Rs;
    out3[2] = out3[1] * gam * gam;
}

/* Matching design from the equivalent capacitance (Sec. 3, first
   paragraph: the vacuum C_eq gives the L-network's C_m1 and C_m2 for a
   perfect match).  Load: C_eq in parallel with the stray branch
   R_stray + j w L_stray + 1/(j w C_stray) (Eq. 10).  The network's input
   admittance j w C_m1 + 1/Z_b, with Z_b = R_m + j w L_m + 1/(j w C_m2) +
   Z_load = R_b + j X_b, equals 1/R_s when
     R_b / (R_b^2 + X_b^2) = 1/R_s   and   w C_m1 = X_b / (R_b^2 + X_b^2),
   i.e. X_b = +sqrt(R_b (R_s - R_b)) (C_m1 > 0), w C_m1 = X_b / (R_b R_s) and
   1/(w C_m2) = w L_m + Im Z_load - X_b.  Returns -1 when no such network
   exists (R_b >= R_s or a non-positive C_m2). */
int orc_match_design(const orc_config* c, double C_eq, double* out2) {
    double w = 2.0 * O_PI * c->freq;
    /* Z_C = 1/(j w C_eq) = -j / (w C_eq) */
    double zc_re = 0.0, zc_im = -1.0 / (w * C_eq);
    double zs_re = c->R_stray, zs_im = w * c->L_stray - 1.0 / (w * c->C_stray);
    /* parallel combination Z_C Z_s / (Z_C + Z_s) */
    double num_re = zc_re * zs_re - zc_im * zs_im, num_im = zc_re * zs_im + zc_im * zs_re;
    double den_re = zc_re + zs_re, den_im = zc_im + zs_im;
    double dd = den_re * den_re + den_im * den_im;
    double zl_re = (num_re * den_re + num_im * den_im) / dd;
    double zl_im = (num_im * den_re - num_re * den_im) / dd;
    double Rb = c->R_m + zl_re;
    if (!(Rb > 0.0) || !(Rb < c->R_s)) return -1;
    double Xb = sqrt(Rb * (c->R_s - Rb));
    double Cm1 = Xb / (Rb * c->R_s) / w;
    double xc2 = w * c->L_m + zl_im - Xb;
    if (!(xc2 > 0.0)) return -1;
    out2[0] = Cm1;
    out2[1] = 1.0 / (w * xc2);
    return 0;
}

int orc_split_now(orc_sim* s, int32_t sp, int64_t* added) {
    if (sp < 0 || sp > 1) return -1;
    return split_species(s, sp, added);
}

double orc_split_target(orc_sim* s, int32_t sp, int32_t i) { return o_split_target(s, sp, i); }

int orc_diag_get(orc_sim* s, orc_diag* d) {
    memset(d, 0, sizeof(*d));
    d->t = s->t; d->U_E = s->U_E[0]; d->Q_E = s->Q_E[0]; d->C_eq = s->Cm[0][0]; d->Q_P = s->Q_P[0];
    d->I_ccp = s->I_ccp[0]; d->dt = s->dt; d->w_unit = s->w_unit; d->n_gas = s->n_gas;
    d->n_el = s->n_el;
    for (int e = 0; e < s->n_el; e++) {
        d->U_el[e] = s->U_E[e]; d->Q_el[e] = s->Q_E[e]; d->QP_el[e] = s->Q_P[e]; d->I_el[e] = s->I_ccp[e];
        for (int f = 0; f < s->n_el; f++) d->C_el[e * ORC_MAX_EL + f] = s->Cm[e][f];
        for (int sp = 0; sp < 2; sp++) d->absorbed_el[sp][e] = s->cnt[sp][o_slot_of(e + 1)];
    }
    memcpy(d->circ, s->circ, sizeof(d->circ));
    d->nu_max[0] = s->nu_max[0]; d->nu_max[1] = s->nu_max[1];
    d->thresh[0] = s->thresh[0]; d->thresh[1] = s->thresh[1];
    d->step = s->step; d->periods_done = s->periods_done;
    for (int sp = 0; sp < 2; sp++) {
        d->n_slots[sp] = s->p[sp].n;
        int64_t a = 0;
        for (int64_t k = 0; k < s->p[sp].n; k++) a += (s->p[sp].r[k] >= 0.0);
        d->n_alive[sp] = a;
        for (int c = 0; c < ORC_NCNT; c++) d->absorbed[sp][c] = s->cnt[sp][c];
        for (int c = 0; c < 4; c++) d->coll[sp][c] = s->coll[sp][c];
    }
    d->born = s->born;
    d->split_added[0] = s->split_added[0];
    d->split_added[1] = s->split_added[1];
    d->numax_violations = s->viol;
    d->solver_iters = s->solver_iters;
    d->solver_relres = s->solver_relres;
    if (s->have_last) {
        harmonics(s->lastU[0], s->cfg.steps_per_period, d->harm_U_re, d->harm_U_im);
        harmonics(s->lastI[0], s->cfg.steps_per_period, d->harm_I_re, d->harm_I_im);
        for (int e = 0; e < s->n_el; e++) {
            harmonics(s->lastU[e], s->cfg.steps_per_period, d->hU_re[e], d->hU_im[e]);
            harmonics(s->lastI[e], s->cfg.steps_per_period, d->hI_re[e], d->hI_im[e]);
        }
        o_characterise(&s->cfg, s->lastU[0], s->lastI[0], s->lastVin, s->lastI1, s->last_energy, d->elec);
    }
    return 0;
}

int orc_series(orc_sim* s, int32_t last, double* U_out, double* I_out) {
    int spp = s->cfg.steps_per_period;
    memcpy(U_out, last ? s->lastU[0] : s->serU[0], sizeof(double) * spp);
    memcpy(I_out, last ? s->lastI[0] : s->serI[0], sizeof(double) * spp);
    return 0;
}

/* --------------------------------------------------------- introspection */
int64_t orc_num_slots(orc_sim* s, int32_t sp) { return (sp == 0 || sp == 1) ? s->p[sp].n : -1; }

int orc_get_particles(orc_sim* s, int32_t sp, double* out9) {
    o_parts* P = &s->p[sp];
    int64_t n = P->n;
    double* f[9] = {P->r, P->z, P->vr, P->vt, P->vz, P->ar, P->at, P->az, P->w};
    for (int k = 0; k < 9; k++) memcpy(out9 + (size_t)k * n, f[k], sizeof(double) * n);
    return 0;
}

int orc_set_particles(orc_sim* s, int32_t sp, int64_t n, const double* in9) {
    o_parts* P = &s->p[sp];
    if (n > P->cap) return -2;
    double* f[9] = {P->r, P->z, P->vr, P->vt, P->vz, P->ar, P->at, P->az, P->w};
    for (int k = 0; k < 9; k++) memcpy(f[k], in9 + (size_t)k * n, sizeof(double) * n);
    P->n = n;
    return 0;
}

int orc_redeposit(orc_sim* s) {
    for (int sp = 0; sp < 2; sp++) {
        memset(s->dep[sp], 0, sizeof(int64_t) * s->nn);
        o_parts* P = &s->p[sp];
        for (int64_t k = 0; k < P->n; k++)
            if (P->r[k] >= 0.0) o_deposit_one(s, P->r[k], P->z[k], P->w[k], s->dep[sp]);
    }
    return 0;
}

int orc_get_grid(orc_sim* s, int32_t which, void* out) {
    size_t nn = (size_t)s->nn, nc = (size_t)s->nr * s->nz;
    switch (which) {
    case ORC_G_DEP_E: memcpy(out, s->dep[0], nn * 8); return 0;
    case ORC_G_DEP_I: memcpy(out, s->dep[1], nn * 8); return 0;
    case ORC_G_PHI: memcpy(out, s->phi, nn * 8); return 0;
    case ORC_G_ER: memcpy(out, s->Er, nn * 8); return 0;
    case ORC_G_EZ: memcpy(out, s->Ez, nn * 8); return 0;
    case ORC_G_CHI: memcpy(out, s->chi, nn * 8); return 0;
    case ORC_G_WALLQ: memcpy(out, s->wallq, nn * 8); return 0;
    case ORC_G_NODE_KIND: memcpy(out, s->node_kind, nn * 4); return 0;
    case ORC_G_CELL_KIND: memcpy(out, s->cell_kind, nc * 4); return 0;
    case ORC_G_VOL: memcpy(out, s->vol, nn * 8); return 0;
    case ORC_G_PHI_L: memcpy(out, s->phiL[0], nn * 8); return 0;
    case ORC_G_Q: memcpy(out, s->Q, nn * 8); return 0;
    case ORC_G_AR: memcpy(out, s->ar, nn * 8); return 0;
    case ORC_G_AZ: memcpy(out, s->az, nn * 8); return 0;
    case ORC_G_NE_AVG:
    case ORC_G_NI_AVG: {
        int sp = which - ORC_G_NE_AVG;
        double* o = out;
        double unit = s->w_unit * ldexp(1.0, -O_KBITS) / s->cfg.steps_per_period;
        for (size_t n = 0; n < nn; n++) o[n] = (double)s->plast[sp][n] * unit / s->vol[n];
        return 0;
    }
    }
    return -1;
}

int orc_set_grid(orc_sim* s, int32_t which, const void* in) {
    size_t nn = (size_t)s->nn;
    switch (which) {
    case ORC_G_DEP_E: memcpy(s->dep[0], in, nn * 8); return 0;
    case ORC_G_DEP_I: memcpy(s->dep[1], in, nn * 8); return 0;
    case ORC_G_PHI: memcpy(s->phi, in, nn * 8); return 0;
    case ORC_G_WALLQ: memcpy(s->wallq, in, nn * 8); return 0;
    case ORC_G_PHI_L: memcpy(s->phiL[0], in, nn * 8); return 0;
    case ORC_G_ER: memcpy(s->Er, in, nn * 8); return 0;
    case ORC_G_EZ: memcpy(s->Ez, in, nn * 8); return 0;
    }
    return -1;
}

int orc_set_state(orc_sim* s, const double* st) {
    s->t = st[0]; s->Q_E[0] = st[1]; s->U_E[0] = st[2];
    for (int k = 0; k < 5; k++) s->circ[0][k] = st[3 + k];
    s->Cm[0][0] = st[8];
    return 0;
}

/* ------------------------------------------------------------ pure pieces */
/* Eq. (1)'s susceptibility and right-hand side from the deposit grids as
   they stand (the first step of every time step), without stepping. */
int orc_assemble_now(orc_sim* s) {
    o_assemble(s);
    return 0;
}

/* E = -grad phi at the nodes from the potential grid as it stands [R9]. */
int orc_efield_now(orc_sim* s) {
    o_efield(s);
    return 0;
}

/* The field the particle step gathers at n positions, from the node field
   grids as they stand (0 outside the domain). */
int orc_gather(orc_sim* s, int64_t n, const double* r, const double* z, double* Er, double* Ez) {
    for (int64_t k = 0; k < n; k++) o_gather(s, r[k], z[k], &Er[k], &Ez[k]);
    return 0;
}

int orc_solve_qv(orc_sim* s, const double* Q, const double* chi, const double* U, double tol, double* phi_inout,
                 int32_t* iters, double* relres) {
    double* ar = calloc(s->nn, sizeof(double));
    double* az = calloc(s->nn, sizeof(double));
    o_faces_from_chi(s, chi, ar, az);
    int it;
    double rel;
    double Uv[ORC_MAX_EL] = {0.0};
    for (int e = 0; e < s->n_el; e++) Uv[e] = U[e];
    int rc = o_solve(s, ar, az, Q, Uv, tol, phi_inout, &it, &rel);
    if (iters) *iters = it;
    if (relres) *relres = rel;
    free(ar);
    free(az);
    return rc;
}

int orc_solve_q(orc_sim* s, const double* Q, const double* chi, double U_E, double tol, double* phi_inout,
                int32_t* iters, double* relres) {
    double U[ORC_MAX_EL] = {U_E, 0.0, 0.0, 0.0};
    return orc_solve_qv(s, Q, chi, U, tol, phi_inout, iters, relres);
}

int orc_get_phiL(orc_sim* s, int32_t e, double* out) {
    if (e < 1 || e > s->n_el) return -1;
    memcpy(out, s->phiL[e - 1], sizeof(double) * s->nn);
    return 0;
}

double orc_refresh_laplace(orc_sim* s) { return o_laplace(s); }

int orc_deposit(orc_sim* s, int64_t n, const double* r, const double* z, const double* w, int64_t* grid) {
    memset(grid, 0, sizeof(int64_t) * s->nn);
    for (int64_t k = 0; k < n; k++)
        if (r[k] >= 0.0) o_deposit_one(s, r[k], z[k], w[k], grid);
    return 0;
}

/* Energy moment of species sp at the stored (predicted) positions and
   explicit velocities v* [R31]: per particle the kinetic energy
   eps = (m / 2e)((v_r v_r + v_t v_t) + v_z v_z) in eV, quantised as
   e_q = floor(16 eps) (capped at 2^20), and node sums N += c_k,
   E += c_k e_q with the deposit's integer shares c_k.  Mean energy per
   node E / (16 N) eV; temperature (2/3) of it. */
int orc_moments(orc_sim* s, int sp, int64_t* N, int64_t* E) {
    memset(N, 0, sizeof(int64_t) * s->nn);
    memset(E, 0, sizeof(int64_t) * s->nn);
    const o_parts* P = &s->p[sp];
    const double half_m_over_e = 0.5 * s->mass[sp] / O_QE;
    for (int64_t k = 0; k < P->n; k++) {
        if (!(P->r[k] >= 0.0)) continue;
        o_loc L = o_locate(s, P->r[k], P->z[k]);
        if (!L.inside) continue;
        int64_t c[4];
        o_node_weights(s, &L, P->w[k], c);
        double v2 = P->vr[k] * P->vr[k];
        v2 = v2 + P->vt[k] * P->vt[k];
        v2 = v2 + P->vz[k] * P->vz[k];
        double eq = floor(half_m_over_e * v2 * 16.0);
        int64_t q = eq < 1048576.0 ? (int64_t)eq : 1048576;
        int nodes[4] = {L.j * (s->nr + 1) + L.i, L.j * (s->nr + 1) + L.i + 1, (L.j + 1) * (s->nr + 1) + L.i,
                        (L.j + 1) * (s->nr + 1) + L.i + 1};
        for (int m = 0; m < 4; m++) {
            N[nodes[m]] += c[m];
            E[nodes[m]] += c[m] * q;
        }
    }
    return 0;
}

int orc_tile_keys(orc_sim* s, int64_t n, const double* r, const double* z, uint32_t* keys) {
    for (int64_t k = 0; k < n; k++) keys[k] = tile_key(s, r[k], z[k]);
    return 0;
}

int orc_predict(orc_sim* s, int64_t n, double* p9) {
    double st[9];
    for (int64_t k = 0; k < n; k++) {
        for (int f = 0; f < 9; f++) st[f] = p9[(size_t)f * n + k];
        o_predict1(s, st);
        for (int f = 0; f < 9; f++) p9[(size_t)f * n + k] = st[f];
    }
    return 0;
}

int orc_correct(orc_sim* s, int32_t sp, int64_t n, double* p9, const double* Er, const double* Ez) {
    double st[9];
    for (int64_t k = 0; k < n; k++) {
        for (int f = 0; f < 9; f++) st[f] = p9[(size_t)f * n + k];
        o_correct1(s, sp, st, Er[k], Ez[k]);
        for (int f = 0; f < 9; f++) p9[(size_t)f * n + k] = st[f];
    }
    return 0;
}

int orc_mcc(orc_sim* s, int32_t sp, int64_t n, double* v3, uint32_t slot0, uint32_t step, int32_t* proc,
            double* birth6) {
    for (int64_t k = 0; k < n; k++) {
        double v[3] = {v3[3 * k], v3[3 * k + 1], v3[3 * k + 2]}, b6[6] = {0, 0, 0, 0, 0, 0};
        proc[k] = o_mcc1(s, sp, v, slot0 + (uint32_t)k, step, b6);
        for (int c = 0; c < 3; c++) v3[3 * k + c] = v[c];
        if (birth6) for (int c = 0; c < 6; c++) birth6[6 * k + c] = b6[c];
    }
    return 0;
}
