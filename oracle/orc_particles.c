/*
 * orc_particles.c -- oracle (test infrastructure only): fixed-point charge
 * deposit with cylindrical-volume weights, the direct-implicit push, particle
 * absorption, Philox random streams and null-collision Monte Carlo
 * collisions (Sec. 2: implicit scheme around Eq. 1, unequal weights and the
 * collision paragraph).
 */
#include "orc_internal.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NODE(i, j) ((j) * (s->nr + 1) + (i))

/* -------------------------------------------------------------- locate */
/* Fixed-point position: q = floor((double)x * 2^F / dx); cell index
   q >> F, fraction q & (2^F - 1).  A particle is inside when r < R and
   0 < z < Z and its cell index is in range; otherwise `edge` names the
   domain edge it left by (0: r=R, 1: z=0, 2: z=Z). */
o_loc o_locate(const orc_sim* s, double r, double z) {
    o_loc L;
    memset(&L, 0, sizeof(L));
    L.inside = 0;
    if (!(r < s->cfg.R)) { L.edge = 0; return L; }
    if (!(z > 0.0)) { L.edge = 1; return L; }
    if (!(z < s->cfg.Z)) { L.edge = 2; return L; }
    double xr = r * s->Sr, xz = z * s->Sz;
    L.qr = (int64_t)floor(xr);
    L.qz = (int64_t)floor(xz);
    L.i = (int)(L.qr >> O_FBITS);
    L.j = (int)(L.qz >> O_FBITS);
    if (L.i >= s->nr) { L.edge = 0; return L; }
    if (L.j >= s->nz) { L.edge = 2; return L; }
    L.fr = L.qr & ((1LL << O_FBITS) - 1);
    L.fz = L.qz & ((1LL << O_FBITS) - 1);
    L.inside = 1;
    return L;
}

/* [R6] cylindrical-volume weights: radial weight to node i+1 is the volume
   fraction (r^2 - r_i^2)/(r_{i+1}^2 - r_i^2), axial weights linear.  Exact
   integer definition, no fused multiply-add:
     n_r = 2 i f_r 2^F + f_r^2  (integer),  w_r = n_r * invd[i],
     invd[i] = 2^-2F / (2i+1),  w_z = f_z 2^-F,
     c11 = floor(((W w_r) w_z) 2^K), c10 = floor(((W w_r)(1-w_z)) 2^K),
     c01 = floor(((W (1-w_r)) w_z) 2^K), c00 = floor(W 2^K) - c11 - c10 - c01.
   Order of c: (i,j), (i+1,j), (i,j+1), (i+1,j+1). */
void o_node_weights(const orc_sim* s, const o_loc* L, double W, int64_t c[4]) {
    int64_t nrr = 2LL * L->i * L->fr * (1LL << O_FBITS) + L->fr * L->fr;
    double wr = (double)nrr * s->invd[L->i];
    double wrb = 1.0 - wr;
    double wz = (double)L->fz * ldexp(1.0, -O_FBITS);
    double wzb = (double)((1LL << O_FBITS) - L->fz) * ldexp(1.0, -O_FBITS);
    double K = ldexp(1.0, O_KBITS);
    double t;
    t = W * wr; t = t * wz; t = t * K; int64_t c11 = (int64_t)floor(t);
    t = W * wr; t = t * wzb; t = t * K; int64_t c10 = (int64_t)floor(t);
    t = W * wrb; t = t * wz; t = t * K; int64_t c01 = (int64_t)floor(t);
    t = W * K; int64_t tot = (int64_t)floor(t);
    c[0] = tot - c11 - c10 - c01;
    c[1] = c10;
    c[2] = c01;
    c[3] = c11;
}

void o_deposit_one(const orc_sim* s, double r, double z, double W, int64_t* grid) {
    o_loc L = o_locate(s, r, z);
    if (!L.inside) return;
    int64_t c[4];
    o_node_weights(s, &L, W, c);
    grid[NODE(L.i, L.j)] += c[0];
    grid[NODE(L.i + 1, L.j)] += c[1];
    grid[NODE(L.i, L.j + 1)] += c[2];
    grid[NODE(L.i + 1, L.j + 1)] += c[3];
}

/* Gather E at a position with the same cylindrical-volume weights, in
   floating point. */
void o_gather(const orc_sim* s, double r, double z, double* Er, double* Ez) {
    o_loc L = o_locate(s, r, z);
    if (!L.inside) { *Er = 0.0; *Ez = 0.0; return; }
    double f = (double)L.fr * ldexp(1.0, -O_FBITS);
    double wr = (2.0 * L.i * f + f * f) / (2.0 * L.i + 1.0);
    double wz = (double)L.fz * ldexp(1.0, -O_FBITS);
    int n00 = NODE(L.i, L.j), n10 = n00 + 1, n01 = n00 + s->nr + 1, n11 = n01 + 1;
    double w00 = (1 - wr) * (1 - wz), w10 = wr * (1 - wz), w01 = (1 - wr) * wz, w11 = wr * wz;
    *Er = w00 * s->Er[n00] + w10 * s->Er[n10] + w01 * s->Er[n01] + w11 * s->Er[n11];
    *Ez = w00 * s->Ez[n00] + w10 * s->Ez[n10] + w01 * s->Ez[n01] + w11 * s->Ez[n11];
}

/* ------------------------------------------------------------- push (D1) */
/* [R7] direct-implicit D1 scheme: with state (x~, v*, a_bar),
   correct:  a = (q/m) E(x~);  x = x~ + dt^2/2 a;  v = v* + dt/2 a;
             a_bar = (a_bar + a)/2;  a particle crossing the axis is reflected.
   predict:  v* = v + dt/2 a_bar;  Cartesian move X = r + dt v*_r,
             Y = dt v*_t, z~ = z + dt v*_z; r~ = sqrt(X^2+Y^2); v* and a_bar
             are rotated into the new local (r, theta) frame. */
enum { P_R = 0, P_Z, P_VR, P_VT, P_VZ, P_AR, P_AT, P_AZ, P_W };

void o_correct1(const orc_sim* s, int sp, double* st, double Er, double Ez) {
    double dt = s->dt;
    double ar = s->qm[sp] * Er, az = s->qm[sp] * Ez;
    st[P_R] = st[P_R] + 0.5 * dt * dt * ar;
    st[P_Z] = st[P_Z] + 0.5 * dt * dt * az;
    st[P_VR] = st[P_VR] + 0.5 * dt * ar;
    st[P_VZ] = st[P_VZ] + 0.5 * dt * az;
    st[P_AR] = 0.5 * (st[P_AR] + ar);
    st[P_AT] = 0.5 * st[P_AT];
    st[P_AZ] = 0.5 * (st[P_AZ] + az);
    if (st[P_R] < 0.0) {
        st[P_R] = -st[P_R];
        st[P_VR] = -st[P_VR]; st[P_VT] = -st[P_VT];
        st[P_AR] = -st[P_AR]; st[P_AT] = -st[P_AT];
    }
}

void o_predict1(const orc_sim* s, double* st) {
    double dt = s->dt;
    double vr = st[P_VR] + 0.5 * dt * st[P_AR];
    double vt = st[P_VT] + 0.5 * dt * st[P_AT];
    double vz = st[P_VZ] + 0.5 * dt * st[P_AZ];
    double X = st[P_R] + dt * vr, Y = dt * vt;
    double rn = sqrt(X * X + Y * Y);
    double c = 1.0, sn = 0.0;
    if (rn > 0.0) { c = X / rn; sn = Y / rn; }
    st[P_R] = rn;
    st[P_Z] = st[P_Z] + dt * vz;
    st[P_VR] = c * vr + sn * vt;
    st[P_VT] = -sn * vr + c * vt;
    st[P_VZ] = vz;
    double ar = st[P_AR], at = st[P_AT];
    st[P_AR] = c * ar + sn * at;
    st[P_AT] = -sn * ar + c * at;
}

/* ------------------------------------------------------------ absorption */
/* [R10] after the correction and after the prediction, a particle outside
   the domain or in a non-vacuum cell is removed.  Its integer charge
   floor(W 2^K) goes to the counter of the conductor it hit (or of the domain
   edge; a Neumann edge counts as lost).  In a dielectric cell the charge is
   deposited with the node weights at the landing point into the persistent
   surface-charge grid; the part that falls on conductor nodes goes to that
   conductor's counter.  Returns 1 if the particle was removed. */
int o_absorb_check(orc_sim* s, int sp, double r, double z, double W) {
    o_loc L = o_locate(s, r, z);
    int64_t tot = (int64_t)floor(W * ldexp(1.0, O_KBITS));
    if (!L.inside) {
        int bc = s->cfg.edge_bc[L.edge];
        int slot = (bc >= 0) ? o_slot_of(bc) : 2;
        s->cnt[sp][slot] += tot;
        return 1;
    }
    int ck = s->cell_kind[L.j * s->nr + L.i];
    if (ck == 0) return 0;
    if (ck >= 2) {
        int id = ck - 2;
        s->cnt[sp][o_slot_of(id)] += tot;
        return 1;
    }
    int64_t c[4];
    o_node_weights(s, &L, W, c);
    int nodes[4] = {NODE(L.i, L.j), NODE(L.i + 1, L.j), NODE(L.i, L.j + 1), NODE(L.i + 1, L.j + 1)};
    for (int k = 0; k < 4; k++) {
        int nk = s->node_kind[nodes[k]];
        if (nk >= 0) s->cnt[sp][o_slot_of(nk)] += c[k];
        else {
            s->wallq[nodes[k]] += s->sign[sp] * c[k];
            s->cnt[sp][3] += c[k];
        }
    }
    return 1;
}

/* -------------------------------------------------------------- Philox */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
   (c0,c1,c2,c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1,
   lo(M0 c0)), with the key bumped by the Weyl constants between rounds. */
void o_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void orc_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    o_philox4x32(ctr, key, out);
}

/* the same round structure with 64-bit words (Philox4x64-10) */
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ull * c0;
        unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ull * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform in (0,1): ((x >> 9) + 1/2) 2^-23, exact in FP32 and FP64 */
double o_u01(uint32_t x) { return ((double)(x >> 9) + 0.5) * ldexp(1.0, -23); }

static void draw(const orc_sim* s, uint32_t slot, uint32_t step, uint32_t purpose, int sp, uint32_t k,
                 uint32_t out[4]) {
    uint32_t ctr[4] = {slot, step, purpose * 2u + (uint32_t)sp, k};
    uint32_t key[2] = {(uint32_t)(s->cfg.seed & 0xFFFFFFFFu), (uint32_t)(s->cfg.seed >> 32)};
    o_philox4x32(ctr, key, out);
}

/* ------------------------------------------------------- cross sections */
/* [R11] synthetic analytic argon cross sections (m^2, energy in eV):
   elastic 1e-19/sqrt(1+e/10); excitation 2.7e-20 ln(x)/x, x = e/11.5 (e>11.5);
   ionisation 8e-20 ln(x)/x, x = e/15.76 (e>15.76); Ar+ on Ar isotropic and
   charge exchange 5e-19 each [R12]. */
#define E_EXC 11.5
#define E_ION 15.76
#define B_ION 10.0
#define SIG_ISO 5.0e-19
#define SIG_CX 5.0e-19

void o_xsec_e(double eps, double* el, double* ex, double* io) {
    *el = 1.0e-19 / sqrt(1.0 + eps / 10.0);
    *ex = (eps > E_EXC) ? 2.7e-20 * log(eps / E_EXC) / (eps / E_EXC) : 0.0;
    *io = (eps > E_ION) ? 8.0e-20 * log(eps / E_ION) / (eps / E_ION) : 0.0;
}

void orc_xsec_e(double eps, double out3[3]) { o_xsec_e(eps, &out3[0], &out3[1], &out3[2]); }

/* Null-collision constants (Vahedi & Surendra 1995): nu_max is the maximum
   of n_g sigma_T(e) v(e) over a dense logarithmic energy scan times 1.001
   for electrons, n_g (sigma_iso + sigma_cx) g_max for ions; the per-step
   collision probability 1 - exp(-nu_max dt) becomes an integer threshold on
   a 32-bit random word [R13]. */
void o_set_collision_constants(orc_sim* s) {
    s->n_gas = s->cfg.p_Pa / (O_KB * s->cfg.T_gas_K);
    const int N = 2000000;
    double best = 0.0;
    for (int k = 0; k < N; k++) {
        double eps = pow(10.0, -4.0 + 9.0 * (double)k / (double)(N - 1));
        double el, ex, io;
        o_xsec_e(eps, &el, &ex, &io);
        double sv = (el + ex + io) * sqrt(2.0 * O_QE * eps / O_ME);
        if (sv > best) best = sv;
    }
    s->nu_max[0] = s->n_gas * best * 1.001;
    double gmax = sqrt(2.0 * O_QE * 2000.0 / O_MAR) + 5.0 * sqrt(O_KB * s->cfg.T_gas_K / O_MAR);
    s->nu_max[1] = s->n_gas * (SIG_ISO + SIG_CX) * gmax;
    s->vth_gas = sqrt(O_KB * s->cfg.T_gas_K / O_MAR);
    for (int sp = 0; sp < 2; sp++) {
        double P = -expm1(-s->nu_max[sp] * s->dt);
        double T = floor(P * 4294967296.0);
        s->thresh[sp] = (T >= 4294967295.0) ? 0xFFFFFFFFu : (uint32_t)T;
    }
}

/* scattering by polar angle chi (cos cchi) and azimuth phi about the unit
   direction d (standard rotation formula) */
static void rotate_dir(double d[3], double cchi, double phi) {
    double schi = sqrt(fmax(0.0, 1.0 - cchi * cchi));
    double cp = cos(phi), sp = sin(phi);
    double u = d[0], v = d[1], w = d[2];
    double st = sqrt(u * u + v * v); /* = sqrt(1 - w^2) without cancellation near the pole */
    if (st > 1e-10) {
        d[0] = u * cchi + schi * (u * w * cp - v * sp) / st;
        d[1] = v * cchi + schi * (v * w * cp + u * sp) / st;
        d[2] = w * cchi - st * schi * cp;
    } else {
        d[0] = schi * cp;
        d[1] = schi * sp;
        d[2] = (w >= 0 ? 1.0 : -1.0) * cchi;
    }
}

/* electron scattering angle (Vahedi & Surendra 1995):
   cos chi = (2 + e - 2 (1+e)^u) / e */
static double e_cos_chi(double eps, double u) {
    if (eps < 1e-10) return 1.0 - 2.0 * u;
    double c = (2.0 + eps - 2.0 * pow(1.0 + eps, u)) / eps;
    return fmin(1.0, fmax(-1.0, c));
}

/* One null-collision test for a particle (species sp, slot, step) with
   velocity v (m/s, local r,theta,z components).  Returns the process:
   -1 no collision, 0 elastic / isotropic, 1 excitation / charge exchange,
   2 ionisation, 3 null.  For ionisation birth6 = (ejected electron v,
   new ion v). */
/* The null-collision decision word of a slot at a step [R27]: one
   Philox4x32-10 block (purpose 2) serves the four slots that agree in the
   low six bits and in bits 8 and up, c0 = (slot mod 64) + 64 floor(slot/256);
   the slot takes word floor(slot / 64) mod 4 of it. */
static uint32_t decision_word(const orc_sim* s, uint32_t slot, uint32_t step, int sp) {
    uint32_t x[4];
    draw(s, (slot & 63u) | ((slot >> 8) << 6), step, 2, sp, 0, x);
    return x[(slot >> 6) & 3u];
}

int o_mcc1(orc_sim* s, int sp, double* v, uint32_t slot, uint32_t step, double* birth6) {
    uint32_t x[4];
    if (!(decision_word(s, slot, step, sp) < s->thresh[sp])) return -1;
    draw(s, slot, step, 1, sp, 0, x);
    double u1 = o_u01(x[1]), u2 = o_u01(x[2]), u3 = o_u01(x[3]);
    double R = u1 * s->nu_max[sp];
    if (sp == 0) {
        double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        double vm = sqrt(v2);
        double eps = 0.5 * O_ME * v2 / O_QE;
        double el, ex, io;
        o_xsec_e(eps, &el, &ex, &io);
        double n_el = s->n_gas * el * vm, n_ex = s->n_gas * ex * vm, n_io = s->n_gas * io * vm;
        if (vm == 0.0) return 3;
        double d[3] = {v[0] / vm, v[1] / vm, v[2] / vm};
        if (R < n_el) {
            double cc = e_cos_chi(eps, u2);
            double e2 = eps * (1.0 - 2.0 * O_ME / O_MAR * (1.0 - cc));
            rotate_dir(d, cc, 2.0 * O_PI * u3);
            double sp2 = sqrt(2.0 * O_QE * e2 / O_ME);
            for (int k = 0; k < 3; k++) v[k] = sp2 * d[k];
            return 0;
        } else if (R < n_el + n_ex) {
            double e1 = eps - E_EXC;
            double cc = e_cos_chi(e1, u2);
            rotate_dir(d, cc, 2.0 * O_PI * u3);
            double sp2 = sqrt(2.0 * O_QE * e1 / O_ME);
            for (int k = 0; k < 3; k++) v[k] = sp2 * d[k];
            return 1;
        } else if (R < n_el + n_ex + n_io) {
            uint32_t y[4], z4[4];
            draw(s, slot, step, 1, sp, 1, y);
            draw(s, slot, step, 1, sp, 2, z4);
            double e1 = eps - E_ION;
            double eej = B_ION * tan(o_u01(y[0]) * atan(e1 / (2.0 * B_ION)));
            double esc = e1 - eej;
            double d2[3] = {d[0], d[1], d[2]};
            rotate_dir(d, e_cos_chi(esc, u2), 2.0 * O_PI * u3);
            rotate_dir(d2, e_cos_chi(eej, o_u01(y[1])), 2.0 * O_PI * o_u01(y[2]));
            double s1 = sqrt(2.0 * O_QE * esc / O_ME), s2 = sqrt(2.0 * O_QE * eej / O_ME);
            for (int k = 0; k < 3; k++) { v[k] = s1 * d[k]; birth6[k] = s2 * d2[k]; }
            /* the new ion: Maxwellian at the gas temperature */
            double a = sqrt(-2.0 * log(o_u01(z4[0]))), b = 2.0 * O_PI * o_u01(z4[1]);
            double c = sqrt(-2.0 * log(o_u01(z4[2]))), e = 2.0 * O_PI * o_u01(z4[3]);
            birth6[3] = s->vth_gas * a * cos(b);
            birth6[4] = s->vth_gas * a * sin(b);
            birth6[5] = s->vth_gas * c * cos(e);
            return 2;
        }
        return 3;
    }
    /* Ar+ on Ar: collision partner sampled from the 300 K Maxwellian
       (Sec. 2, collision paragraph); relative speed g */
    uint32_t y[4];
    draw(s, slot, step, 1, sp, 1, y);
    double a = sqrt(-2.0 * log(o_u01(y[0]))), b = 2.0 * O_PI * o_u01(y[1]);
    double c = sqrt(-2.0 * log(o_u01(y[2]))), e = 2.0 * O_PI * o_u01(y[3]);
    double vn[3] = {s->vth_gas * a * cos(b), s->vth_gas * a * sin(b), s->vth_gas * c * cos(e)};
    double g[3] = {v[0] - vn[0], v[1] - vn[1], v[2] - vn[2]};
    double gm = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    double n_iso = s->n_gas * SIG_ISO * gm, n_cx = s->n_gas * SIG_CX * gm;
    double tot = n_iso + n_cx;
    if (tot > s->nu_max[1]) {
        s->viol++;
        double f = s->nu_max[1] / tot;
        n_iso *= f;
        n_cx *= f;
    }
    if (R < n_iso) {
        /* isotropic in the centre of mass, equal masses: in the neutral rest
           frame cos chi = sqrt(1-u), |g'| = |g| cos chi */
        double cc = sqrt(1.0 - u2);
        double d[3] = {g[0] / gm, g[1] / gm, g[2] / gm};
        rotate_dir(d, cc, 2.0 * O_PI * u3);
        double gp = gm * cc;
        for (int k = 0; k < 3; k++) v[k] = vn[k] + gp * d[k];
        return 0;
    } else if (R < n_iso + n_cx) {
        for (int k = 0; k < 3; k++) v[k] = vn[k];
        return 1;
    }
    return 3;
}

/* [R32] Reference weight in cell column i: the species' loading weight
   times the column's cell volume over the mean vacuum-cell volume, so that
   particles of this weight fill every cell with the same count. */
double o_split_target(const orc_sim* s, int sp, int i) {
    double r0 = i * s->dr, r1 = (i + 1) * s->dr;
    double vi = O_PI * (r1 * r1 - r0 * r0) * s->dz;
    return s->wref[sp] * vi * (double)s->nvac / s->vvac;
}

/* --------------------------------------------------------------- loader */
/* Uniform plasma (Sec. 3, first paragraph): particles uniform in volume over
   the vacuum cells (cell chosen by inverse CDF of cell volume, then r^2 and
   z uniform inside it), Maxwellian velocities by Box-Muller. */
int o_load(orc_sim* s) {
    int nr = s->nr, nz = s->nz;
    double* cdf = malloc(sizeof(double) * ((size_t)nr * nz + 1));
    int* cell = malloc(sizeof(int) * ((size_t)nr * nz + 1));
    int nv = 0;
    double acc = 0.0;
    for (int j = 0; j < nz; j++)
        for (int i = 0; i < nr; i++) {
            if (s->cell_kind[j * nr + i] != 0) continue;
            double r0 = i * s->dr, r1 = (i + 1) * s->dr;
            acc += O_PI * (r1 * r1 - r0 * r0) * s->dz;
            cdf[nv] = acc;
            cell[nv] = j * nr + i;
            nv++;
        }
    double vvac = acc;
    for (int sp = 0; sp < 2; sp++) {
        int64_t n = sp == 0 ? s->cfg.n_e : s->cfg.n_i;
        double W = (n > 0) ? (s->cfg.n0 * vvac / (double)n) / s->w_unit : 1.0;
        double T = sp == 0 ? s->cfg.Te_eV : s->cfg.Ti_eV;
        double vth = sqrt(O_QE * T / s->mass[sp]);
        o_parts* P = &s->p[sp];
        if (n > P->cap) { free(cdf); free(cell); return -2; }
        for (int64_t k = 0; k < n; k++) {
            uint32_t x[4], y[4];
            draw(s, (uint32_t)k, 0, 0, sp, 0, x);
            draw(s, (uint32_t)k, 0, 0, sp, 1, y);
            int lo;
            if (s->cfg.weights == 1) {
                /* [R32] every vacuum cell equally likely, weight by cell volume */
                lo = (int)floor(o_u01(x[0]) * (double)nv);
                if (lo > nv - 1) lo = nv - 1;
            } else {
                double target = o_u01(x[0]) * vvac;
                lo = 0; /* first c with cdf[c] > target */
                int hi = nv - 1;
                while (lo < hi) {
                    int mid = (lo + hi) / 2;
                    if (cdf[mid] > target) hi = mid; else lo = mid + 1;
                }
            }
            int ci = cell[lo] % nr, cj = cell[lo] / nr;
            double r0 = ci * s->dr, r1 = (ci + 1) * s->dr;
            double r = sqrt(r0 * r0 + o_u01(x[1]) * (r1 * r1 - r0 * r0));
            double z = (cj + o_u01(x[2])) * s->dz;
            double a = sqrt(-2.0 * log(o_u01(y[0]))), b = 2.0 * O_PI * o_u01(y[1]);
            double c = sqrt(-2.0 * log(o_u01(y[2]))), e = 2.0 * O_PI * o_u01(y[3]);
            P->r[k] = r; P->z[k] = z;
            P->vr[k] = vth * a * cos(b);
            P->vt[k] = vth * a * sin(b);
            P->vz[k] = vth * c * cos(e);
            P->ar[k] = P->at[k] = P->az[k] = 0.0; /* [R8] */
            P->w[k] = (s->cfg.weights == 1) ? o_split_target(s, sp, ci) : W;
        }
        P->n = n;
    }
    free(cdf);
    free(cell);
    return 0;
}
