/*
 * orc_field.c -- oracle (test infrastructure only): geometry, node volumes,
 * the finite-volume form of the implicit Poisson equation (Eq. 1), its
 * solution by multigrid-preconditioned CG, the Laplace problem behind the
 * equivalent capacitance (Eqs. 5-7) and the node electric field.
 */
#include "orc_internal.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NODE(i, j) ((j) * (s->nr + 1) + (i))

/* ---------------------------------------------------------------- geometry */
/* Cells take the last region containing their centre (Sec. 2, reactor
   geometry paragraph: metal and dielectric materials on a regular grid).
   A node is a conductor node if an adjacent cell is a conductor or it lies
   on a conductor domain edge.  [R1] a node touching two conductors belongs
   to ground, otherwise to the lowest id. */
int o_geometry(orc_sim* s) {
    const orc_config* c = &s->cfg;
    int nr = s->nr, nz = s->nz;
    s->dr = c->R / nr;
    s->dz = c->Z / nz;
    s->cell_kind = calloc((size_t)nr * nz, sizeof(int32_t));
    s->cell_eps = calloc((size_t)nr * nz, sizeof(double));
    s->node_kind = calloc((size_t)s->nn, sizeof(int32_t));
    s->vol = calloc((size_t)s->nn, sizeof(double));
    s->gr = calloc((size_t)s->nn, sizeof(double));
    s->gz = calloc((size_t)s->nn, sizeof(double));
    if (!s->cell_kind || !s->cell_eps || !s->node_kind || !s->vol || !s->gr || !s->gz) return -1;
    for (int j = 0; j < nz; j++)
        for (int i = 0; i < nr; i++) {
            double rc = (i + 0.5) * s->dr, zc = (j + 0.5) * s->dz;
            int kind = 0;
            double eps = 1.0;
            for (int k = 0; k < c->n_regions; k++) {
                const orc_region* g = &c->regions[k];
                if (rc >= g->r0 && rc < g->r1 && zc >= g->z0 && zc < g->z1) {
                    if (g->kind == 2) { kind = 2 + g->cond_id; eps = 1.0; }
                    else if (g->kind == 1) { kind = 1; eps = g->eps_r; }
                    else { kind = 0; eps = 1.0; }
                }
            }
            s->cell_kind[j * nr + i] = kind;
            s->cell_eps[j * nr + i] = eps;
        }
    for (int j = 0; j <= nz; j++)
        for (int i = 0; i <= nr; i++) {
            int mark[16] = {0};
            for (int dj = -1; dj <= 0; dj++)
                for (int di = -1; di <= 0; di++) {
                    int ci = i + di, cj = j + dj;
                    if (ci < 0 || cj < 0 || ci >= nr || cj >= nz) continue;
                    int k = s->cell_kind[cj * nr + ci];
                    if (k >= 2 && k - 2 < 16) mark[k - 2] = 1;
                }
            if (i == nr && c->edge_bc[0] >= 0) mark[c->edge_bc[0]] = 1;
            if (j == 0 && c->edge_bc[1] >= 0) mark[c->edge_bc[1]] = 1;
            if (j == nz && c->edge_bc[2] >= 0) mark[c->edge_bc[2]] = 1;
            int kind = -1;
            for (int k = 15; k >= 0; k--)
                if (mark[k]) kind = k; /* lowest id wins, so ground (0) wins */
            s->node_kind[NODE(i, j)] = kind;
        }
    /* Node volumes consistent with r^2 (volume-fraction) radial weights and
       linear axial weights: node i receives half of each adjacent annulus. */
    double dr = s->dr, dz = s->dz;
    for (int j = 0; j <= nz; j++)
        for (int i = 0; i <= nr; i++) {
            double rm = (i > 0) ? (i - 1) * dr : 0.0;
            double rp = (i < nr) ? (i + 1) * dr : i * dr;
            double ri = i * dr;
            double v;
            if (i == 0) v = O_PI * dz * (dr * dr) / 2.0;
            else if (i == nr) v = O_PI * dz * (ri * ri - rm * rm) / 2.0;
            else v = O_PI * dz * (rp * rp - rm * rm) / 2.0;
            if (j == 0 || j == nz) v *= 0.5;
            s->vol[NODE(i, j)] = v;
        }
    /* Face factors of the finite-volume operator over control volumes
       [r_{i-1/2}, r_{i+1/2}] x [z_{j-1/2}, z_{j+1/2}], clipped at the edges.
       [R3] eps = eps0 * eps_r of the material, chi the implicit susceptibility. */
    for (int j = 0; j <= nz; j++)
        for (int i = 0; i <= nr; i++) {
            int n = NODE(i, j);
            if (i < nr) { /* radial edge (i,j)-(i+1,j) */
                double h = (j == 0 || j == nz) ? 0.5 * dz : dz;
                double e = 0.0, cnt = 0.0;
                if (j > 0) { e += s->cell_eps[(j - 1) * nr + i]; cnt += 1.0; }
                if (j < nz) { e += s->cell_eps[j * nr + i]; cnt += 1.0; }
                e /= cnt;
                double rh = (i + 0.5) * dr;
                s->gr[n] = 2.0 * O_PI * rh * h * O_EPS0 * e / dr;
            }
            if (j < nz) { /* axial edge (i,j)-(i,j+1) */
                double rlo = (i > 0) ? (i - 0.5) * dr : 0.0;
                double rhi = (i < nr) ? (i + 0.5) * dr : c->R;
                double ri = i * dr;
                double num = 0.0;
                if (i > 0) num += s->cell_eps[j * nr + i - 1] * (ri * ri - rlo * rlo);
                if (i < nr) num += s->cell_eps[j * nr + i] * (rhi * rhi - ri * ri);
                double area = rhi * rhi - rlo * rlo;
                double e = num / area;
                s->gz[n] = O_PI * area * O_EPS0 * e / dz;
            }
        }
    return 0;
}

void o_faces_from_chi(orc_sim* s, const double* chi, double* ar, double* az) {
    int nr = s->nr, nz = s->nz;
    for (int j = 0; j <= nz; j++)
        for (int i = 0; i <= nr; i++) {
            int n = NODE(i, j);
            ar[n] = (i < nr) ? s->gr[n] * (1.0 + 0.5 * (chi[n] + chi[n + 1])) : 0.0;
            az[n] = (j < nz) ? s->gz[n] * (1.0 + 0.5 * (chi[n] + chi[n + nr + 1])) : 0.0;
        }
}

/* Eq. (1) right-hand side and susceptibility from the deposits of the
   predicted positions.  chi_n = 1/2 dt^2 sum_s (q_s^2/m_s) n_s / eps0 is the
   D1 linearised response (beta = 1/2) [R7]; rho~ is the charge of the
   predicted positions (Sec. 2, text after Eq. 1). */
void o_assemble(orc_sim* s) {
    double unit = s->w_unit * ldexp(1.0, -O_KBITS);
    for (int n = 0; n < s->nn; n++) {
        double Ne = (double)s->dep[0][n], Ni = (double)s->dep[1][n];
        double dens_over_m = (Ne * unit / O_ME + Ni * unit / O_MAR) / s->vol[n];
        s->chi[n] = 0.5 * s->dt * s->dt * O_QE * O_QE * dens_over_m / O_EPS0;
        s->Q[n] = O_QE * unit * ((double)s->dep[1][n] - (double)s->dep[0][n] + (double)s->wallq[n]);
    }
    o_faces_from_chi(s, s->chi, s->ar, s->az);
}

/* ---------------------------------------------------------- multigrid PCG */
static const int OFF_DI[9] = {-1, 0, 1, -1, 0, 1, -1, 0, 1};
static const int OFF_DJ[9] = {-1, -1, -1, 0, 0, 0, 1, 1, 1};

static double p1d(int i, int I, int c) {
    if (c == 1) return i == I ? 1.0 : 0.0;
    int d = i - 2 * I;
    if (d == 0) return 1.0;
    if (d == 1 || d == -1) return 0.5;
    return 0.0;
}

static void lev_alloc(o_level* L, int nr, int nz, double dr, double dz) {
    L->nr = nr; L->nz = nz; L->dr = dr; L->dz = dz; L->cr = L->cz = 1;
    size_t nn = (size_t)(nr + 1) * (nz + 1);
    for (int k = 0; k < 9; k++) L->A[k] = calloc(nn, sizeof(double));
    L->x = calloc(nn, sizeof(double));
    L->b = calloc(nn, sizeof(double));
    L->res = calloc(nn, sizeof(double));
}

static void lev_free(o_level* L) {
    for (int k = 0; k < 9; k++) free(L->A[k]);
    free(L->x); free(L->b); free(L->res);
}

static void lev_apply(const o_level* L, const double* x, double* y) {
    int nr = L->nr, nz = L->nz, w = nr + 1;
    for (int j = 0; j <= nz; j++)
        for (int i = 0; i <= nr; i++) {
            int n = j * w + i;
            if (L->A[4][n] == 0.0) { y[n] = 0.0; continue; }
            double acc = 0.0;
            for (int k = 0; k < 9; k++) {
                int i2 = i + OFF_DI[k], j2 = j + OFF_DJ[k];
                if (i2 < 0 || j2 < 0 || i2 > nr || j2 > nz) continue;
                acc += L->A[k][n] * x[j2 * w + i2];
            }
            y[n] = acc;
        }
}

typedef struct {
    int nlev;
    o_level lv[24];
    int nc;        /* active nodes on the coarsest level */
    int* cidx;     /* coarsest node -> dense index or -1 */
    double* chol;  /* dense Cholesky factor (lower, row-major nc x nc) */
} o_mg;

static void mg_build(o_mg* mg, orc_sim* s, const double* ar, const double* az) {
    int nr = s->nr, nz = s->nz, w = nr + 1;
    memset(mg, 0, sizeof(*mg));
    o_level* L0 = &mg->lv[0];
    lev_alloc(L0, nr, nz, s->dr, s->dz);
    for (int j = 0; j <= nz; j++)
        for (int i = 0; i <= nr; i++) {
            int n = j * w + i;
            if (s->node_kind[n] >= 0) continue;
            double d = 0.0;
            if (i > 0) { d += ar[n - 1]; if (s->node_kind[n - 1] < 0) L0->A[3][n] = -ar[n - 1]; }
            if (i < nr) { d += ar[n]; if (s->node_kind[n + 1] < 0) L0->A[5][n] = -ar[n]; }
            if (j > 0) { d += az[n - w]; if (s->node_kind[n - w] < 0) L0->A[1][n] = -az[n - w]; }
            if (j < nz) { d += az[n]; if (s->node_kind[n + w] < 0) L0->A[7][n] = -az[n]; }
            L0->A[4][n] = d;
        }
    int l = 0;
    for (;;) {
        o_level* F = &mg->lv[l];
        size_t nn = (size_t)(F->nr + 1) * (F->nz + 1);
        if (nn <= 300 || l == 23) break;
        int can_r = (F->nr % 2 == 0) && F->nr >= 4;
        int can_z = (F->nz % 2 == 0) && F->nz >= 4;
        int cr = 1, cz = 1;
        if (F->dr > 1.5 * F->dz) { if (can_z) cz = 2; else if (can_r) cr = 2; }
        else if (F->dz > 1.5 * F->dr) { if (can_r) cr = 2; else if (can_z) cz = 2; }
        else { if (can_r) cr = 2; if (can_z) cz = 2; }
        if (cr == 1 && cz == 1) break;
        F->cr = cr; F->cz = cz;
        o_level* C = &mg->lv[l + 1];
        lev_alloc(C, F->nr / cr, F->nz / cz, F->dr * cr, F->dz * cz);
        int fw = F->nr + 1, cw = C->nr + 1;
        /* Galerkin coarse operator A_c = P^T A_f P, P bilinear (or linear in
           one direction), P rows of inactive fine nodes zero.  A coarse node
           is active only if the fine node it injects into is active: each
           column of P then holds a 1 that no other column touches, so P has
           full column rank and A_c stays positive definite. */
#define CACT(I_, J_) (F->A[4][(cz * (J_)) * fw + cr * (I_)] != 0.0)
        for (int J = 0; J <= C->nz; J++)
            for (int I = 0; I <= C->nr; I++) {
                int Nc = J * cw + I;
                if (!CACT(I, J)) continue;
                for (int j = cz * J - (cz - 1); j <= cz * J + (cz - 1); j++)
                    for (int i = cr * I - (cr - 1); i <= cr * I + (cr - 1); i++) {
                        if (i < 0 || j < 0 || i > F->nr || j > F->nz) continue;
                        int nf = j * fw + i;
                        if (F->A[4][nf] == 0.0) continue;
                        double pw1 = p1d(i, I, cr) * p1d(j, J, cz);
                        if (pw1 == 0.0) continue;
                        for (int k = 0; k < 9; k++) {
                            double a = F->A[k][nf];
                            if (a == 0.0) continue;
                            int i2 = i + OFF_DI[k], j2 = j + OFF_DJ[k];
                            for (int k2 = 0; k2 < 9; k2++) {
                                int I2 = I + OFF_DI[k2], J2 = J + OFF_DJ[k2];
                                if (I2 < 0 || J2 < 0 || I2 > C->nr || J2 > C->nz) continue;
                                if (!CACT(I2, J2)) continue;
                                double pw2 = p1d(i2, I2, cr) * p1d(j2, J2, cz);
                                if (pw2 == 0.0) continue;
                                C->A[k2][Nc] += pw1 * a * pw2;
                            }
                        }
                    }
            }
#undef CACT
        l++;
    }
    mg->nlev = l + 1;
    /* dense Cholesky of the coarsest operator over its active nodes */
    o_level* C = &mg->lv[l];
    int cw = C->nr + 1, cn = cw * (C->nz + 1);
    mg->cidx = malloc(sizeof(int) * cn);
    int nc = 0;
    for (int n = 0; n < cn; n++) mg->cidx[n] = (C->A[4][n] != 0.0) ? nc++ : -1;
    mg->nc = nc;
    mg->chol = calloc((size_t)nc * nc + 1, sizeof(double));
    double* M = mg->chol;
    for (int J = 0; J <= C->nz; J++)
        for (int I = 0; I <= C->nr; I++) {
            int n = J * cw + I, a = mg->cidx[n];
            if (a < 0) continue;
            for (int k = 0; k < 9; k++) {
                int I2 = I + OFF_DI[k], J2 = J + OFF_DJ[k];
                if (I2 < 0 || J2 < 0 || I2 > C->nr || J2 > C->nz) continue;
                int b = mg->cidx[J2 * cw + I2];
                if (b < 0) continue;
                M[(size_t)a * nc + b] += C->A[k][n];
            }
        }
    for (int k = 0; k < nc; k++) {
        double d = M[(size_t)k * nc + k];
        for (int p = 0; p < k; p++) d -= M[(size_t)k * nc + p] * M[(size_t)k * nc + p];
        d = sqrt(d);
        M[(size_t)k * nc + k] = d;
        for (int i = k + 1; i < nc; i++) {
            double v = M[(size_t)i * nc + k];
            for (int p = 0; p < k; p++) v -= M[(size_t)i * nc + p] * M[(size_t)k * nc + p];
            M[(size_t)i * nc + k] = v / d;
        }
    }
}

static void mg_free(o_mg* mg) {
    for (int l = 0; l < mg->nlev; l++) lev_free(&mg->lv[l]);
    free(mg->cidx);
    free(mg->chol);
}

#define MG_OMEGA 0.7
#define MG_NU 2

static void smooth(o_level* L, int first_from_zero) {
    int nn = (L->nr + 1) * (L->nz + 1);
    if (first_from_zero) {
        for (int n = 0; n < nn; n++) L->x[n] = (L->A[4][n] != 0.0) ? MG_OMEGA * L->b[n] / L->A[4][n] : 0.0;
        return;
    }
    lev_apply(L, L->x, L->res);
    for (int n = 0; n < nn; n++)
        if (L->A[4][n] != 0.0) L->x[n] += MG_OMEGA * (L->b[n] - L->res[n]) / L->A[4][n];
}

/* symmetric V-cycle: x_l ~= A_l^{-1} b_l */
static void vcycle(o_mg* mg, int l) {
    o_level* L = &mg->lv[l];
    int nn = (L->nr + 1) * (L->nz + 1);
    if (l == mg->nlev - 1) {
        int nc = mg->nc;
        double* y = malloc(sizeof(double) * (nc + 1));
        for (int n = 0; n < nn; n++) if (mg->cidx[n] >= 0) y[mg->cidx[n]] = L->b[n];
        const double* M = mg->chol;
        for (int i = 0; i < nc; i++) {
            double v = y[i];
            for (int p = 0; p < i; p++) v -= M[(size_t)i * nc + p] * y[p];
            y[i] = v / M[(size_t)i * nc + i];
        }
        for (int i = nc - 1; i >= 0; i--) {
            double v = y[i];
            for (int p = i + 1; p < nc; p++) v -= M[(size_t)p * nc + i] * y[p];
            y[i] = v / M[(size_t)i * nc + i];
        }
        for (int n = 0; n < nn; n++) L->x[n] = (mg->cidx[n] >= 0) ? y[mg->cidx[n]] : 0.0;
        free(y);
        return;
    }
    smooth(L, 1);
    for (int k = 1; k < MG_NU; k++) smooth(L, 0);
    lev_apply(L, L->x, L->res);
    for (int n = 0; n < nn; n++) L->res[n] = L->b[n] - L->res[n];
    o_level* C = &mg->lv[l + 1];
    int cr = L->cr, cz = L->cz, fw = L->nr + 1, cw = C->nr + 1;
    for (int J = 0; J <= C->nz; J++)
        for (int I = 0; I <= C->nr; I++) {
            double acc = 0.0;
            for (int j = cz * J - (cz - 1); j <= cz * J + (cz - 1); j++)
                for (int i = cr * I - (cr - 1); i <= cr * I + (cr - 1); i++) {
                    if (i < 0 || j < 0 || i > L->nr || j > L->nz) continue;
                    int nf = j * fw + i;
                    if (L->A[4][nf] == 0.0) continue;
                    acc += p1d(i, I, cr) * p1d(j, J, cz) * L->res[nf];
                }
            C->b[J * cw + I] = (C->A[4][J * cw + I] != 0.0) ? acc : 0.0;
        }
    vcycle(mg, l + 1);
    for (int j = 0; j <= L->nz; j++)
        for (int i = 0; i <= L->nr; i++) {
            int nf = j * fw + i;
            if (L->A[4][nf] == 0.0) continue;
            double acc = 0.0;
            int I0 = i / cr, J0 = j / cz;
            for (int J = J0 - 1; J <= J0 + 1; J++)
                for (int I = I0 - 1; I <= I0 + 1; I++) {
                    if (I < 0 || J < 0 || I > C->nr || J > C->nz) continue;
                    if (C->A[4][J * cw + I] == 0.0) continue;
                    double p = p1d(i, I, cr) * p1d(j, J, cz);
                    if (p != 0.0) acc += p * C->x[J * cw + I];
                }
            L->x[nf] += acc;
        }
    for (int k = 0; k < MG_NU; k++) smooth(L, 0);
}

static double dot(const double* a, const double* b, int n) {
    double s = 0.0;
    for (int i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

/* residual of K phi = Q at unknown nodes, phi holding the Dirichlet values;
   also the norm of the right-hand side with the Dirichlet lift */
static void full_residual(const orc_sim* s, const double* ar, const double* az, const double* Q,
                          const double* phi, double* r, double* bnorm2) {
    int nr = s->nr, nz = s->nz, w = nr + 1;
    double bb = 0.0;
    for (int j = 0; j <= nz; j++)
        for (int i = 0; i <= nr; i++) {
            int n = j * w + i;
            if (s->node_kind[n] >= 0) { r[n] = 0.0; continue; }
            double Kphi = 0.0, b = Q[n];
            if (i > 0) { Kphi += ar[n - 1] * (phi[n] - phi[n - 1]); if (s->node_kind[n - 1] >= 0) b += ar[n - 1] * phi[n - 1]; }
            if (i < nr) { Kphi += ar[n] * (phi[n] - phi[n + 1]); if (s->node_kind[n + 1] >= 0) b += ar[n] * phi[n + 1]; }
            if (j > 0) { Kphi += az[n - w] * (phi[n] - phi[n - w]); if (s->node_kind[n - w] >= 0) b += az[n - w] * phi[n - w]; }
            if (j < nz) { Kphi += az[n] * (phi[n] - phi[n + w]); if (s->node_kind[n + w] >= 0) b += az[n] * phi[n + w]; }
            r[n] = Q[n] - Kphi;
            bb += b * b;
        }
    *bnorm2 = bb;
}

/* Solve Eq. (1) in finite-volume form, K phi = Q on the unknown nodes, with
   phi = U[e - 1] on driven electrode e and 0 on grounded conductors (Sec. 2:
   metals are equipotential boundaries).  Stops at ||b - K phi|| <= tol ||b||
   [R20].  phi is the warm start on entry. */
int o_solve(orc_sim* s, const double* ar, const double* az, const double* Q, const double* U, double tol,
            double* phi, int* iters, double* relres) {
    int nn = s->nn;
    for (int n = 0; n < nn; n++)
        if (s->node_kind[n] >= 0) phi[n] = (s->node_kind[n] >= 1) ? U[s->node_kind[n] - 1] : 0.0;
    double* r = calloc(nn, sizeof(double));
    double* z = calloc(nn, sizeof(double));
    double* p = calloc(nn, sizeof(double));
    double* q = calloc(nn, sizeof(double));
    double* d = calloc(nn, sizeof(double));
    o_mg mg;
    mg_build(&mg, s, ar, az);
    o_level* L0 = &mg.lv[0];
    int it = 0, status = 0;
    double bb, rel = 0.0;
    for (int restart = 0; restart < 4; restart++) {
        full_residual(s, ar, az, Q, phi, r, &bb);
        double bn = sqrt(bb), rn = sqrt(dot(r, r, nn));
        if (bn == 0.0) { /* no charge and no drive: phi = 0 on the unknowns */
            for (int n = 0; n < nn; n++) if (s->node_kind[n] < 0) phi[n] = 0.0;
            rel = 0.0;
            break;
        }
        rel = rn / bn;
        if (rel <= tol) break;
        memset(d, 0, sizeof(double) * nn);
        memcpy(L0->b, r, sizeof(double) * nn);
        vcycle(&mg, 0);
        memcpy(z, L0->x, sizeof(double) * nn);
        memcpy(p, z, sizeof(double) * nn);
        double rho = dot(r, z, nn);
        while (it < s->cfg.max_iter * 4) {
            lev_apply(L0, p, q);
            double alpha = rho / dot(p, q, nn);
            for (int n = 0; n < nn; n++) { d[n] += alpha * p[n]; r[n] -= alpha * q[n]; }
            it++;
            if (sqrt(dot(r, r, nn)) <= 0.5 * tol * bn) break;
            memcpy(L0->b, r, sizeof(double) * nn);
            vcycle(&mg, 0);
            memcpy(z, L0->x, sizeof(double) * nn);
            double rho2 = dot(r, z, nn);
            double beta = rho2 / rho;
            rho = rho2;
            for (int n = 0; n < nn; n++) p[n] = z[n] + beta * p[n];
        }
        for (int n = 0; n < nn; n++) if (s->node_kind[n] < 0) phi[n] += d[n];
        if (it >= s->cfg.max_iter * 4) status = -3;
    }
    if (rel > tol) {
        full_residual(s, ar, az, Q, phi, r, &bb);
        rel = (bb > 0) ? sqrt(dot(r, r, nn)) / sqrt(bb) : 0.0;
    }
    if (iters) *iters = it;
    if (relres) *relres = rel;
    mg_free(&mg);
    free(r); free(z); free(p); free(q); free(d);
    return (rel <= tol) ? 0 : (status ? status : -3);
}

/* Equivalent capacitance by the energy method (Eqs. 6-7): phi_L solves the
   Laplace problem with the driven electrode at 1 V and every other conductor
   grounded; 1/2 C_eq U^2 = integral of 1/2 eps |E|^2, which in the
   finite-volume form is sum over edges of a (d phi_L)^2.  [R33] with several
   driven electrodes, one Laplace solution per electrode and the capacitance
   matrix C_ef = sum over edges of a (d phi_Le)(d phi_Lf), the bilinear form
   of the same energy (C_ee is each electrode's C_eq).  [R21] the operator
   includes the current chi (vacuum at start), refreshed once per RF period
   (Sec. 2, text after Eq. 4).  Returns C_11. */
double o_laplace(orc_sim* s) {
    double* zero = calloc(s->nn, sizeof(double));
    int it;
    double rel;
    for (int e = 0; e < s->n_el; e++) {
        double U[ORC_MAX_EL] = {0.0};
        U[e] = 1.0;
        o_solve(s, s->ar, s->az, zero, U, 1e-13, s->phiL[e], &it, &rel);
    }
    free(zero);
    int nr = s->nr, nz = s->nz, w = nr + 1;
    for (int e = 0; e < s->n_el; e++)
        for (int f = e; f < s->n_el; f++) {
            const double *a = s->phiL[e], *b = s->phiL[f];
            double C = 0.0;
            for (int j = 0; j <= nz; j++)
                for (int i = 0; i <= nr; i++) {
                    int n = j * w + i;
                    if (i < nr) { double d = a[n] - a[n + 1], g = b[n] - b[n + 1]; C += s->ar[n] * d * g; }
                    if (j < nz) { double d = a[n] - a[n + w], g = b[n] - b[n + w]; C += s->az[n] * d * g; }
                }
            s->Cm[e][f] = C;
            s->Cm[f][e] = C;
        }
    return s->Cm[0][0];
}

double orc_ceq_flux(orc_sim* s) {
    int nr = s->nr, nz = s->nz, w = nr + 1;
    double F = 0.0;
    for (int j = 0; j <= nz; j++)
        for (int i = 0; i <= nr; i++) {
            int n = j * w + i;
            if (s->node_kind[n] != 1) continue;
            const double* L = s->phiL[0];
            if (i > 0) F += s->ar[n - 1] * (L[n] - L[n - 1]);
            if (i < nr) F += s->ar[n] * (L[n] - L[n + 1]);
            if (j > 0) F += s->az[n - w] * (L[n] - L[n - w]);
            if (j < nz) F += s->az[n] * (L[n] - L[n + w]);
        }
    return F;
}

/* [R9] E = -grad phi at nodes: centred differences inside, one-sided on the
   z edges and at r = R, E_r = 0 on the axis. */
void o_efield(orc_sim* s) {
    int nr = s->nr, nz = s->nz, w = nr + 1;
    const double* f = s->phi;
    for (int j = 0; j <= nz; j++)
        for (int i = 0; i <= nr; i++) {
            int n = j * w + i;
            double er, ez;
            if (i == 0) er = 0.0;
            else if (i == nr) er = -(f[n] - f[n - 1]) / s->dr;
            else er = -(f[n + 1] - f[n - 1]) / (2.0 * s->dr);
            if (j == 0) ez = -(f[n + w] - f[n]) / s->dz;
            else if (j == nz) ez = -(f[n] - f[n - w]) / s->dz;
            else ez = -(f[n + w] - f[n - w]) / (2.0 * s->dz);
            s->Er[n] = er;
            s->Ez[n] = ez;
        }
}
