// field.hip -- the implicit field solve on gfx950 (arXiv 2310.04957,
// Sec. 2): assembly of the finite-volume form of Eq. (1) with the implicit
// susceptibility, the equivalent-capacitance electrode voltage and external
// circuit (Eqs. 5, 8-10), FP64 residuals with FP32 (or FP64) multigrid-
// preconditioned CG inside iterative refinement, the per-period Laplace
// solution and energy-method C_eq (Eqs. 6-7), and the node electric field.
// Reductions use fixed-size grids and fixed orders: results are run-to-run
// reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>

#include "pic_internal.h"

namespace pic {

constexpr double kEps0 = 8.8541878128e-12;
// Weights of the two Jacobi sweeps of the multigrid smoother: the degree-2
// Chebyshev polynomial in D^-1 A that is smallest on [1/2, 2], the upper
// three quarters of the spectrum (D^-1 A of the finite-volume operator lies
// in (0, 2)): w_k = 1 / (5/4 + 3/4 cos((2k - 1) pi / 4)).  It damps that part
// to 0.22 per smoothing, against 0.42 for two sweeps of weight 0.7, and
// stays below 1 on (0, 2.5).  Pre-smoothing takes kW1 then kW2,
// post-smoothing kW2 then kW1 (both the same polynomial, so the V-cycle stays
// symmetric).
constexpr double kW1 = 0.5616936, kW2 = 1.3895259;
constexpr int kCheckEvery = 4;   // Krylov iterations between host convergence reads (unguided)

// Tile (or node range) of a block in the tiled and stencil kernels.  The
// hardware deals consecutive blocks round-robin to the eight XCDs, each with
// its own L2; the tiles are handed to the XCDs in contiguous runs instead,
// so that the halo lines neighbouring tiles share are fetched into one L2.
// Partial sums stay indexed by tile, so the results do not change.  (A
// bijection of 0 .. n-1: XCD x takes n/8 tiles, one more if x < n % 8.)
__device__ __forceinline__ int xcd_tile(int b, int n) {
    const int q = n >> 3, r = n & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

// ------------------------------------------------------------ small utils
__global__ void k_fill_u64(unsigned long long* p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}
__global__ void k_fill_f64(double* p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}
void launch_zero_u64(unsigned long long* p, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u64, dim3(512), dim3(256), 0, s, p, n);
}
void launch_zero_f64(double* p, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_f64, dim3(512), dim3(256), 0, s, p, n);
}

template <typename T>
__global__ void k_fill(T* p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = T(0);
}

// block sum of a double into part[blockIdx.x * stride + slot]
__device__ __forceinline__ double block_sum(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
    __syncthreads();
    return t;  // valid in thread 0
}

// block sum of a double returned to every thread (fixed order; up to 1024
// threads, sh: 16 doubles)
__device__ __forceinline__ double block_total(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
    __syncthreads();
    return t;
}

// sum of the n per-block partials a launch left, in every thread of the
// block: the fused Krylov kernels reduce the partials of the launch before
// them themselves instead of in a launch of their own (every block gets the
// same sum, and only one launch computes each scalar)
__device__ __forceinline__ double sum_partials(const double* p, int n, double* sh) {
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += p[i];
    return block_total(v, sh);
}

// --------------------------------------------------------------- assembly
struct AsmArgs {
    const unsigned long long *dep_e, *dep_i, *wallq;
    unsigned long long *next_e, *next_i, *psum_e, *psum_i;
    const double* vol;
    const double* phiL[kMaxEl];
    const int8_t* nk;
    double *chi, *Q, *part;
    double ce, ci, qunit;
    int nn, n_el;
};

// chi_n = 1/2 dt^2 sum_s (q_s^2/m_s) n_s / eps0 (the D1 linearised response),
// Q_n = node charge of the predicted positions plus the dielectric surface
// charge; also the period sums, the clearing of the next deposit buffer and
// the partial sums of Q_P = -sum phi_L Q for each driven electrode
// (part[e kRedBlocks + block]).
__global__ __launch_bounds__(256) void k_assemble(AsmArgs a) {
    __shared__ double sh[4];
    double qp[kMaxEl] = {0.0, 0.0, 0.0, 0.0};
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < a.nn; n += gridDim.x * blockDim.x) {
        long long Ne = (long long)a.dep_e[n], Ni = (long long)a.dep_i[n];
        long long W = (long long)a.wallq[n];
        a.chi[n] = (a.ce * (double)Ne + a.ci * (double)Ni) / a.vol[n];
        double q = a.qunit * (double)(Ni - Ne + W);
        a.Q[n] = q;
        a.psum_e[n] += (unsigned long long)Ne;
        a.psum_i[n] += (unsigned long long)Ni;
        a.next_e[n] = 0ull;
        a.next_i[n] = 0ull;
        if (a.nk[n] < 0)
            for (int e = 0; e < a.n_el; ++e) qp[e] -= a.phiL[e][n] * q;
    }
    for (int e = 0; e < a.n_el; ++e) {
        double t = block_sum(qp[e], sh);
        if (threadIdx.x == 0) a.part[e * kRedBlocks + blockIdx.x] = t;
    }
}

void launch_assemble(pic_handle* h) {
    AsmArgs a;
    int c = h->dep_cur, o = 1 - h->dep_cur;
    a.dep_e = h->dep[c][0]; a.dep_i = h->dep[c][1]; a.wallq = h->wallq;
    a.next_e = h->dep[o][0]; a.next_i = h->dep[o][1];
    a.psum_e = h->psum[0]; a.psum_i = h->psum[1];
    a.vol = h->vol; a.nk = h->node_kind;
    a.n_el = h->n_el;
    for (int e = 0; e < kMaxEl; ++e) a.phiL[e] = h->phiL[e];
    a.chi = h->chi; a.Q = h->Q; a.part = h->part;
    a.ce = h->chi_c[0]; a.ci = h->chi_c[1]; a.qunit = h->qunit; a.nn = h->nn;
    hipLaunchKernelGGL(k_assemble, dim3(kRedBlocks), dim3(256), 0, h->stream, a);
}

// face coefficients a = geometry x eps0 eps_r x (1 + mean chi), FP64 and
// FP32 (the latter divided by eps0)
__global__ __launch_bounds__(256) void k_faces(const double* chi, const double* gr, const double* gz, double* ar,
                                               double* az, float* ar32, float* az32, int nr, int nz) {
    const int w = nr + 1, nn = w * (nz + 1);
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += gridDim.x * blockDim.x) {
        int i = n % w, j = n / w;
        double a1 = (i < nr) ? gr[n] * (1.0 + 0.5 * (chi[n] + chi[n + 1])) : 0.0;
        double a2 = (j < nz) ? gz[n] * (1.0 + 0.5 * (chi[n] + chi[n + w])) : 0.0;
        ar[n] = a1; az[n] = a2;
        ar32[n] = (float)(a1 / kEps0);
        az32[n] = (float)(a2 / kEps0);
    }
}

void launch_faces(pic_handle* h) {
    hipLaunchKernelGGL(k_faces, dim3(1024), dim3(256), 0, h->stream, h->chi, h->gr, h->gz, h->ar, h->az, h->ar32,
                       h->az32, h->nr, h->nz);
}

// ---------------------------------------------------------------- circuit
struct CircEl {
    int kind, substeps;
    double freq, U_amp, U_dc, R_s, C_m1, C_m2, L_m, R_m, C_stray, L_stray, R_stray, C_b, R_b, L_b;
};

struct CircArgs {
    DevScalars* sc;
    const DevCounters* ctr;
    const double* part;
    double *serU, *serI, *serVin, *serI1;   // serU, serI: kMaxEl blocks of spp
    int k, spp, n_el;
    double dt, qunit;
    CircEl ce[kMaxEl];
};

__device__ __forceinline__ double source_v(const CircEl& c, double t) {
    return c.U_amp * sin(2.0 * 3.14159265358979323846 * c.freq * t) + c.U_dc;
}

// y: L-match (Eq. 10) Q1, Q2, I2, Q_ccp, I_stray; series RLC (Eq. 9) Q_b, I_b;
// y[5] the electrode charge of Eq. (8); U_E the electrode voltage.
__device__ void circ_f(const CircEl& a, double U_E, double I_conv, double t, const double* y, double* dy) {
    const double Us = source_v(a, t);
    for (int k = 0; k < 6; ++k) dy[k] = 0.0;
    if (a.kind == PIC_LMATCH) {
        const double Um1 = (y[0] - y[1]) / a.C_m1;
        dy[0] = (Us - Um1) / a.R_s;
        dy[1] = y[2];
        dy[2] = (Um1 - U_E - y[1] / a.C_m2 - y[2] * a.R_m) / a.L_m;
        dy[3] = y[2] - y[4];
        dy[4] = (U_E - (y[1] - y[3]) / a.C_stray - y[4] * a.R_stray) / a.L_stray;
        dy[5] = dy[3] + I_conv;
    } else if (a.kind == PIC_SERIES_RLC) {
        dy[0] = y[1];
        dy[1] = (Us - U_E - y[0] / a.C_b - y[1] * a.R_b) / a.L_b;
        dy[5] = y[1] + I_conv;
    }
}

// element powers (Eq. 13 integrands): source, R_s, R_m or R_b, stray, load
// U_E I_ccp.
__device__ void circ_p(const CircEl& a, double U_E, double t, const double* y, double* p) {
    const double Us = source_v(a, t);
    for (int k = 0; k < 5; ++k) p[k] = 0.0;
    if (a.kind == PIC_LMATCH) {
        const double I1 = (Us - (y[0] - y[1]) / a.C_m1) / a.R_s;
        p[0] = Us * I1;
        p[1] = a.R_s * I1 * I1;
        p[2] = a.R_m * y[2] * y[2];
        p[3] = a.R_stray * y[4] * y[4];
        p[4] = U_E * (y[2] - y[4]);
    } else if (a.kind == PIC_SERIES_RLC) {
        p[0] = Us * y[1];
        p[2] = a.R_b * y[1] * y[1];
        p[4] = U_E * y[1];
    }
}

// Electrode voltages at time t for circuit states Y: Q = C U + Q_P, so an
// ideal source fixes its electrode's voltage and the other electrodes solve
// C_NN U_N = Q_N - Q_P,N - C_NK U_K.  Gaussian elimination over all NE
// electrodes with an ideal source's row replaced by U_e = U_s(t), which is
// the same system (one electrode: U = (Q - Q_P) / C_eq); NE is a
// compile-time count so every array stays in registers.
template <int NE>
__device__ __forceinline__ void volts(const CircArgs& a, const double (*C)[kMaxEl], const double* QP, double t,
                                      const double (*Y)[6], double* U) {
    double A[NE][NE], b[NE];
#pragma unroll
    for (int r = 0; r < NE; ++r) {
        const bool ideal = a.ce[r].kind == PIC_IDEAL_SOURCE;
        b[r] = ideal ? source_v(a.ce[r], t) : Y[r][5] - QP[r];
#pragma unroll
        for (int q = 0; q < NE; ++q) A[r][q] = ideal ? (r == q ? 1.0 : 0.0) : C[r][q];
    }
#pragma unroll
    for (int p = 0; p < NE; ++p)
#pragma unroll
        for (int r = p + 1; r < NE; ++r) {
            const double m = A[r][p] / A[p][p];
#pragma unroll
            for (int q = p; q < NE; ++q) A[r][q] -= m * A[p][q];
            b[r] -= m * b[p];
        }
#pragma unroll
    for (int r = NE - 1; r >= 0; --r) {
        double x = b[r];
#pragma unroll
        for (int q = r + 1; q < NE; ++q) x -= A[r][q] * U[q];
        U[r] = x / A[r][r];
    }
}

// One circuit step (Sec. 2, Eqs. 8-10): the induced charges Q_P from the
// assembly's partial sums, the convective currents from the absorbed-charge
// counters, then RK4 of all circuits together (substeps: the largest of the
// circuits'), electrode 1's element energies by the trapezoid rule, and the
// voltage series.  One block; thread 0 integrates.
template <int NE>
__global__ __launch_bounds__(256) void k_circuit(CircArgs a) {
    __shared__ double sh[kRedBlocks];
    __shared__ double sQP[kMaxEl];
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) sh[i] = a.part[e * kRedBlocks + i];
        __syncthreads();
        for (int o = kRedBlocks / 2; o > 0; o >>= 1) {
            for (int i = threadIdx.x; i < o; i += blockDim.x) sh[i] += sh[i + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) sQP[e] = sh[0];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    DevScalars* s = a.sc;
    double QP[NE], Iconv[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        const int sl = slot_of(e + 1);
        const long long pc = (long long)a.ctr->absorbed[1][sl] - (long long)a.ctr->absorbed[0][sl];
        Iconv[e] = ((double)pc - s->el_prev[e]) * a.qunit / a.dt;
        s->el_prev[e] = (double)pc;
        QP[e] = sQP[e];
        s->Q_P[e] = QP[e];
    }
    const double t0 = s->t, t1 = t0 + a.dt;
    const double U0 = s->U_E[0];
    // the capacitance matrix and the energy sums in registers for the whole
    // integration (the same operations in the same order as on the scalars,
    // without a dependent memory access per stage)
    double Cm[kMaxEl][kMaxEl], en[5];
#pragma unroll
    for (int e = 0; e < NE; ++e)
#pragma unroll
        for (int f = 0; f < NE; ++f) Cm[e][f] = s->Cm[e][f];
#pragma unroll
    for (int k = 0; k < 5; ++k) en[k] = s->energy[k];
    double Y[NE][6], U[NE], q0[NE];
    int M = 0;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
#pragma unroll
        for (int k = 0; k < 5; ++k) Y[e][k] = s->circ[e][k];
        Y[e][5] = s->Q_E[e];
        q0[e] = a.ce[e].kind == PIC_LMATCH ? Y[e][3] : Y[e][0];
        if (a.ce[e].kind != PIC_IDEAL_SOURCE) {
            const int ms = a.ce[e].substeps > 0 ? a.ce[e].substeps : 1;
            if (ms > M) M = ms;
        }
    }
    const double q1 = Y[0][0];
    if (M > 0) {
        const double hh = a.dt / M;
        const bool pe = a.ce[0].kind != PIC_IDEAL_SOURCE;
        double pa[5], pb[5];
        if (pe) {
            volts<NE>(a, Cm, QP, t0, Y, U);
            circ_p(a.ce[0], U[0], t0, Y[0], pa);
        }
        for (int m = 0; m < M; ++m) {
            const double t = t0 + m * hh;
            double k1[NE][6], k2[NE][6], k3[NE][6], k4[NE][6], yt[NE][6];
            volts<NE>(a, Cm, QP, t, Y, U);
#pragma unroll
            for (int e = 0; e < NE; ++e) circ_f(a.ce[e], U[e], Iconv[e], t, Y[e], k1[e]);
#pragma unroll
            for (int e = 0; e < NE; ++e)
#pragma unroll
                for (int k = 0; k < 6; ++k) yt[e][k] = Y[e][k] + 0.5 * hh * k1[e][k];
            volts<NE>(a, Cm, QP, t + 0.5 * hh, yt, U);
#pragma unroll
            for (int e = 0; e < NE; ++e) circ_f(a.ce[e], U[e], Iconv[e], t + 0.5 * hh, yt[e], k2[e]);
#pragma unroll
            for (int e = 0; e < NE; ++e)
#pragma unroll
                for (int k = 0; k < 6; ++k) yt[e][k] = Y[e][k] + 0.5 * hh * k2[e][k];
            volts<NE>(a, Cm, QP, t + 0.5 * hh, yt, U);
#pragma unroll
            for (int e = 0; e < NE; ++e) circ_f(a.ce[e], U[e], Iconv[e], t + 0.5 * hh, yt[e], k3[e]);
#pragma unroll
            for (int e = 0; e < NE; ++e)
#pragma unroll
                for (int k = 0; k < 6; ++k) yt[e][k] = Y[e][k] + hh * k3[e][k];
            volts<NE>(a, Cm, QP, t + hh, yt, U);
#pragma unroll
            for (int e = 0; e < NE; ++e) circ_f(a.ce[e], U[e], Iconv[e], t + hh, yt[e], k4[e]);
#pragma unroll
            for (int e = 0; e < NE; ++e)
                if (a.ce[e].kind != PIC_IDEAL_SOURCE)
#pragma unroll
                    for (int k = 0; k < 6; ++k)
                        Y[e][k] += hh / 6.0 * (k1[e][k] + 2.0 * k2[e][k] + 2.0 * k3[e][k] + k4[e][k]);
            if (pe) {
                volts<NE>(a, Cm, QP, t + hh, Y, U);
                circ_p(a.ce[0], U[0], t + hh, Y[0], pb);
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    en[k] += 0.5 * hh * (pa[k] + pb[k]);
                    pa[k] = pb[k];
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) s->energy[k] = en[k];
    volts<NE>(a, Cm, QP, t1, Y, U);
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        if (a.ce[e].kind == PIC_IDEAL_SOURCE) {
            // the charge that holds the source voltage: Q = C U + Q_P
            double q = 0.0;
#pragma unroll
            for (int f = 0; f < NE; ++f) q += Cm[e][f] * U[f];
            q += QP[e];
            s->I_ccp[e] = (q - s->Q_E[e]) / a.dt - Iconv[e];
            s->Q_E[e] = q;
        } else {
#pragma unroll
            for (int k = 0; k < 5; ++k) s->circ[e][k] = Y[e][k];
            s->Q_E[e] = Y[e][5];
            s->I_ccp[e] = ((a.ce[e].kind == PIC_LMATCH ? Y[e][3] : Y[e][0]) - q0[e]) / a.dt;
        }
        s->U_E[e] = U[e];
    }
    // electrode 1: source-side samples (the matching network's input voltage
    // across C_m1 and the source current, or the source voltage and I_b) and,
    // for an ideal source, its energy
    const CircEl& c0 = a.ce[0];
    if (c0.kind == PIC_IDEAL_SOURCE) {
        const double e = a.dt * 0.5 * (U0 + U[0]) * s->I_ccp[0];
        s->energy[0] += e;
        s->energy[4] += e;
        a.serVin[a.k] = U[0];
        a.serI1[a.k] = s->I_ccp[0];
    } else if (c0.kind == PIC_LMATCH) {
        a.serVin[a.k] = (Y[0][0] - Y[0][1]) / c0.C_m1;
        a.serI1[a.k] = (Y[0][0] - q1) / a.dt;
    } else {
        a.serVin[a.k] = source_v(c0, t1);
        a.serI1[a.k] = s->I_ccp[0];
    }
    s->t = t1;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        a.serU[e * a.spp + a.k] = s->U_E[e];
        a.serI[e * a.spp + a.k] = s->I_ccp[e];
    }
}

static CircEl circ_el(const pic_circuit& c) {
    CircEl e;
    e.kind = c.kind; e.substeps = c.substeps;
    e.freq = c.freq; e.U_amp = c.U_amp; e.U_dc = c.U_dc; e.R_s = c.R_s; e.C_m1 = c.C_m1; e.C_m2 = c.C_m2;
    e.L_m = c.L_m; e.R_m = c.R_m; e.C_stray = c.C_stray; e.L_stray = c.L_stray; e.R_stray = c.R_stray;
    e.C_b = c.C_b; e.R_b = c.R_b; e.L_b = c.L_b;
    return e;
}

void launch_circuit(pic_handle* h) {
    CircArgs a;
    a.sc = h->sc; a.ctr = h->ctr; a.part = h->part; a.serU = h->serU; a.serI = h->serI;
    a.serVin = h->serVin; a.serI1 = h->serI1;
    a.spp = h->cfg.run.steps_per_period;
    a.k = (int)(h->step % a.spp);
    a.dt = h->dt; a.qunit = h->qunit;
    a.n_el = h->n_el;
    for (int e = 0; e < h->n_el; ++e) a.ce[e] = circ_el(e == 0 ? h->cfg.circ : h->cfg.circ_el[e - 1]);
    switch (h->n_el) {
    case 1: hipLaunchKernelGGL(k_circuit<1>, dim3(1), dim3(256), 0, h->stream, a); break;
    case 2: hipLaunchKernelGGL(k_circuit<2>, dim3(1), dim3(256), 0, h->stream, a); break;
    case 3: hipLaunchKernelGGL(k_circuit<3>, dim3(1), dim3(256), 0, h->stream, a); break;
    default: hipLaunchKernelGGL(k_circuit<4>, dim3(1), dim3(256), 0, h->stream, a); break;
    }
}

// ---------------------------------------------------------- FP64 residual
// Dirichlet value of a conductor node: U[e - 1] on driven electrode e, 0 on ground
__device__ __forceinline__ double dir_val(int8_t k, const double* U) { return k >= 1 ? U[k - 1] : 0.0; }

// r = Q - K phi on unknown nodes, Dirichlet neighbours at their conductor
// value; partial sums of r.r and of b.b (b = Q + Dirichlet lift)
__global__ __launch_bounds__(256) void k_resid64(const double* ar, const double* az, const int8_t* nk,
                                                 const double* Q, const double* phi, const double* Up, double* r,
                                                 double* part, int nr, int nz, const DevScalars* s) {
    __shared__ double sh[4];
    if (s->outer_done) return;
    const int w = nr + 1, nn = w * (nz + 1);
    double U[kMaxEl];
    for (int e = 0; e < kMaxEl; ++e) U[e] = Up[e];
    double rr = 0.0, bb = 0.0;
    const int lb = xcd_tile(blockIdx.x, gridDim.x);
    for (int n = lb * blockDim.x + threadIdx.x; n < nn; n += gridDim.x * blockDim.x) {
        const int8_t k0 = nk[n];
        if (k0 >= 0) { r[n] = 0.0; continue; }
        const int i = n % w, j = n / w;
        const double pn = phi[n];
        const double q = Q ? Q[n] : 0.0;
        double Kp = 0.0, b = q;
        if (i > 0) { int m = n - 1; int8_t km = nk[m]; double v = km >= 0 ? dir_val(km, U) : phi[m];
                     Kp += ar[m] * (pn - v); if (km >= 0) b += ar[m] * v; }
        if (i < nr) { int m = n + 1; int8_t km = nk[m]; double v = km >= 0 ? dir_val(km, U) : phi[m];
                      Kp += ar[n] * (pn - v); if (km >= 0) b += ar[n] * v; }
        if (j > 0) { int m = n - w; int8_t km = nk[m]; double v = km >= 0 ? dir_val(km, U) : phi[m];
                     Kp += az[m] * (pn - v); if (km >= 0) b += az[m] * v; }
        if (j < nz) { int m = n + w; int8_t km = nk[m]; double v = km >= 0 ? dir_val(km, U) : phi[m];
                      Kp += az[n] * (pn - v); if (km >= 0) b += az[n] * v; }
        const double res = q - Kp;
        r[n] = res;
        rr += res * res;
        bb += b * b;
    }
    double t1 = block_sum(rr, sh);
    double t2 = block_sum(bb, sh);
    if (threadIdx.x == 0) { part[2 * lb] = t1; part[2 * lb + 1] = t2; }
}

// final sums; decides the outer convergence and the inner target
__global__ __launch_bounds__(256) void k_reduce_resid(const double* part, DevScalars* s, const DevCounters* ctr,
                                                      double tol, int fp64, int dev, double inner_tol, int max_outer) {
    __shared__ double a[kRedBlocks], b[kRedBlocks];
    if (s->outer_done) return;
    for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) { a[i] = part[2 * i]; b[i] = part[2 * i + 1]; }
    __syncthreads();
    for (int o = kRedBlocks / 2; o > 0; o >>= 1) {
        for (int i = threadIdx.x; i < o; i += blockDim.x) { a[i] += a[i + o]; b[i] += b[i + o]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double rr = a[0], bb = b[0];
        s->rr0 = rr;
        s->bb = bb;
        s->nonfinite = !(isfinite(rr) && isfinite(bb));
        s->relres = (bb > 0.0) ? sqrt(rr / bb) : 0.0;
        s->scale = (rr > 0.0) ? 1.0 / sqrt(rr) : 0.0;
        // inner target on r.r: FP64 -> the final tolerance (with margin),
        // FP32 on the normalised residual -> set by the caller
        s->target = fp64 ? 0.25 * tol * tol * bb : s->target;
        s->cap_err = ctr->err;
        if (dev) {
            // the solve ends here, or the next FP32 pass reduces its residual
            // by inner_tol, or by no more than the tolerance still needs
            // (with a factor 2 margin)
            const double rel = s->relres;
            if (s->nonfinite || rel <= tol || s->outer >= max_outer) {
                s->outer_done = 1;
            } else {
                const double want = fmax(inner_tol, 0.5 * tol / rel);
                s->target = want * want;
            }
            s->outer += 1;
        }
    }
}

// start and end of a field solve: no pass is finished and none counted yet
__global__ void k_begin_solve(DevScalars* s) {
    s->outer_done = 0;
    s->outer = 0;
    s->iters_total = 0;
    for (int k = 0; k < 4; ++k) s->its_pass[k] = 0;
}

// ------------------------------------------------------ Krylov kernels (T)
template <typename T>
__global__ __launch_bounds__(256) void k_scale_to(const double* r64, T* r, T* x, const DevScalars* s, int nn) {
    if (s->outer_done) return;
    const double sc = s->scale;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += gridDim.x * blockDim.x) {
        r[n] = (T)(r64[n] * sc);
        x[n] = T(0);
    }
}

// level-0 operator (5-point) on unknown nodes; neighbours that are
// conductors carry zero correction
template <typename T>
__device__ __forceinline__ T apply0(const T* ar, const T* az, const int8_t* nk, const T* x, int n, int i, int j,
                                    int nr, int nz, int w, T& diag) {
    T d = T(0), off = T(0);
    if (i > 0) { T a = ar[n - 1]; d += a; if (nk[n - 1] < 0) off += a * x[n - 1]; }
    if (i < nr) { T a = ar[n]; d += a; if (nk[n + 1] < 0) off += a * x[n + 1]; }
    if (j > 0) { T a = az[n - w]; d += a; if (nk[n - w] < 0) off += a * x[n - w]; }
    if (j < nz) { T a = az[n]; d += a; if (nk[n + w] < 0) off += a * x[n + w]; }
    diag = d;
    return d * x[n] - off;
}

template <typename T>
__global__ __launch_bounds__(256) void k_spmv_dot(const T* ar, const T* az, const int8_t* nk, const T* p, T* q,
                                                  double* part, const DevScalars* s, int nr, int nz) {
    __shared__ double sh[4];
    if (s->done) return;
    const int w = nr + 1, nn = w * (nz + 1);
    double acc = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += gridDim.x * blockDim.x) {
        if (nk[n] >= 0) { q[n] = T(0); continue; }
        T d;
        T v = apply0(ar, az, nk, p, n, n % w, n / w, nr, nz, w, d);
        q[n] = v;
        acc += (double)p[n] * (double)v;
    }
    double t = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

template <typename T>
__global__ __launch_bounds__(256) void k_dot(const T* a, const T* b, double* part, const DevScalars* s, int nn) {
    __shared__ double sh[4];
    if (s->done) return;
    double acc = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += gridDim.x * blockDim.x)
        acc += (double)a[n] * (double)b[n];
    double t = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

template <typename T>
__global__ __launch_bounds__(256) void k_update_xr(T* x, T* r, const T* p, const T* q, double* part,
                                                   const DevScalars* s, int nn) {
    __shared__ double sh[4];
    if (s->done) return;
    const T al = (T)s->alpha;
    double acc = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += gridDim.x * blockDim.x) {
        x[n] += al * p[n];
        T rn = r[n] - al * q[n];
        r[n] = rn;
        acc += (double)rn * (double)rn;
    }
    double t = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

template <typename T>
__global__ __launch_bounds__(256) void k_update_p(T* p, const T* z, const DevScalars* s, int nn) {
    if (s->done) return;
    const T be = (T)s->beta;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += gridDim.x * blockDim.x) p[n] = z[n] + be * p[n];
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy(T* dst, const T* src, const DevScalars* s, int nn) {
    if (s->done) return;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += gridDim.x * blockDim.x) dst[n] = src[n];
}

// what = 0: rz from the partials (start of CG); 1: alpha = rz / pq;
// 2: r.r against the target (sets done); 3: beta = rz_new / rz
__global__ __launch_bounds__(256) void k_reduce(const double* part, DevScalars* s, int what) {
    __shared__ double a[kRedBlocks];
    if (s->done && what != 0) return;
    for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) a[i] = part[i];
    __syncthreads();
    for (int o = kRedBlocks / 2; o > 0; o >>= 1) {
        for (int i = threadIdx.x; i < o; i += blockDim.x) a[i] += a[i + o];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double v = a[0];
    if (what == 0) {
        s->rz = v;
        s->done = !(v > 0.0);
        s->iters = 0;
    } else if (what == 1) {
        s->pq = v;
        if (!(v > 0.0) || !isfinite(v)) { s->done = 1; s->nonfinite = !isfinite(v); }
        else s->alpha = s->rz / v;
    } else if (what == 2) {
        s->rr = v;
        s->iters += 1;
        if (!isfinite(v)) { s->done = 1; s->nonfinite = 1; }
        else if (v <= s->target) s->done = 1;
    } else {
        s->rz_new = v;
        s->beta = v / s->rz;
        s->rz = v;
    }
}

// (a Krylov solve of a finished refinement starts as done)
__global__ void k_begin_cg(DevScalars* s) { s->done = s->outer_done; s->iters = 0; s->fallback = 0; }

// flexible CG: z.r and z.q of the new preconditioned residual in one pass
__global__ __launch_bounds__(256) void k_dot2(const float* z, const float* r, const float* q, double* part,
                                              const DevScalars* s, int nn) {
    __shared__ double sh[4];
    if (s->done) return;
    double a = 0.0, b = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += gridDim.x * blockDim.x) {
        a += (double)z[n] * (double)r[n];
        b += (double)z[n] * (double)q[n];
    }
    double t1 = block_sum(a, sh);
    double t2 = block_sum(b, sh);
    if (threadIdx.x == 0) { part[blockIdx.x] = t1; part[kRedBlocks + blockIdx.x] = t2; }
}

// beta = -(z.q)/(p.q) keeps the new direction A-conjugate to the last one
// (flexible CG with one stored direction); the preconditioner must keep
// z.r > 0, else the solve is handed to multigrid
__global__ __launch_bounds__(256) void k_reduce_fcg(const double* part, DevScalars* s) {
    __shared__ double a[kRedBlocks], b[kRedBlocks];
    if (s->done) return;
    for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) { a[i] = part[i]; b[i] = part[kRedBlocks + i]; }
    __syncthreads();
    for (int o = kRedBlocks / 2; o > 0; o >>= 1) {
        for (int i = threadIdx.x; i < o; i += blockDim.x) { a[i] += a[i + o]; b[i] += b[i + o]; }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double zr = a[0], zq = b[0];
    if (!(zr > 0.0) || !isfinite(zr) || !isfinite(zq)) { s->fallback = 1; s->done = 1; return; }
    s->rz = zr;
    s->beta = -zq / s->pq;
}

__global__ void k_fcg_start(DevScalars* s) {
    if (!(s->rz > 0.0) || !isfinite(s->rz)) { s->fallback = 1; s->done = 1; }
}

// Fused preconditioned CG (multigrid preconditioner).  One iteration is
// k_cg_dir (with the multigrid kernels below), k_cg_step and the V-cycle:
// k_cg_dir sums the r.z partials the last V-cycle left, forms the direction
// p = z + beta p_old (beta = 0 on the first) into the other direction
// buffer, q = K p and the p.q partials; k_cg_step sums those, alpha =
// rz / pq, x += alpha p, r -= alpha q and the r.r partials, which the
// V-cycle's first launch tests against the target.
constexpr int kCgThreads = 512;

template <typename T>
__global__ __launch_bounds__(kCgThreads) void k_cg_step(T* x, T* r, const T* p, const T* q, const double* pqp,
                                                        int npq, double* rrp, DevScalars* s, int nn) {
    __shared__ double sh[16];
    if (s->done) return;
    const double pq = sum_partials(pqp, npq, sh);
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) { s->pq = pq; s->done = 1; s->nonfinite = !isfinite(pq); }
        return;
    }
    const double rz = s->rz_new, alpha = rz / pq;
    const T al = (T)alpha;
    double acc = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += gridDim.x * blockDim.x) {
        x[n] += al * p[n];
        const T rn = r[n] - al * q[n];
        r[n] = rn;
        acc += (double)rn * (double)rn;
    }
    const double t = block_total(acc, sh);
    if (threadIdx.x == 0) rrp[blockIdx.x] = t;
    if (blockIdx.x == 0 && threadIdx.x == 0) { s->pq = pq; s->alpha = alpha; s->rz = rz; }
}

// ------------------------------------------------------------- multigrid
// level 0: residual on the 5-point operator
template <typename T>
__global__ __launch_bounds__(256) void k_res0(const T* ar, const T* az, const int8_t* nk, const T* x, const T* b,
                                              T* res, const DevScalars* s, int nr, int nz) {
    if (s->done) return;
    const int w = nr + 1, nn = w * (nz + 1);
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += gridDim.x * blockDim.x) {
        if (nk[n] >= 0) { res[n] = T(0); continue; }
        T d;
        res[n] = b[n] - apply0(ar, az, nk, x, n, n % w, n / w, nr, nz, w, d);
    }
}

struct Sten {
    const void* A[9];
};

// The passes of the levels >= 1 inside the tail kernel, as block-stride
// loops.  Every load of a node's update is issued before any test on the
// loaded values (a pass then costs one memory round trip per node); values
// at inactive nodes are zero, and so are stencil entries towards them and
// towards off-grid nodes.
template <typename T>
__device__ __forceinline__ void jac9_range(const Sten& S, const T* xin, const T* b, T* xout, int nr, int nz, int first,
                                           int start, int stride, double om) {
    const int w = nr + 1, nn = w * (nz + 1);
    const T* D = (const T*)S.A[4];
    for (int n = start; n < nn; n += stride) {
        const T d0 = D[n], bn = b[n];
        if (first) {
            xout[n] = d0 == T(0) ? T(0) : (T)om * bn / d0;
            continue;
        }
        const int i = n % w, j = n / w;
        T c[9], v[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const int i2 = i + k % 3 - 1, j2 = j + k / 3 - 1;
            const bool ok = i2 >= 0 && j2 >= 0 && i2 <= nr && j2 <= nz;
            c[k] = ok ? ((const T*)S.A[k])[n] : T(0);
            v[k] = ok ? xin[n + (k / 3 - 1) * w + (k % 3 - 1)] : T(0);
        }
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < 9; ++k) acc += c[k] * v[k];
        xout[n] = d0 == T(0) ? T(0) : v[4] + (T)om * (bn - acc) / d0;
    }
}

template <typename T>
__device__ __forceinline__ void res9_range(const Sten& S, const T* x, const T* b, T* res, int nr, int nz, int start,
                                           int stride) {
    const int w = nr + 1, nn = w * (nz + 1);
    for (int n = start; n < nn; n += stride) {
        const int i = n % w, j = n / w;
        const T bn = b[n];
        T c[9], v[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const int i2 = i + k % 3 - 1, j2 = j + k / 3 - 1;
            const bool ok = i2 >= 0 && j2 >= 0 && i2 <= nr && j2 <= nz;
            c[k] = ok ? ((const T*)S.A[k])[n] : T(0);
            v[k] = ok ? x[n + (k / 3 - 1) * w + (k % 3 - 1)] : T(0);
        }
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < 9; ++k) acc += c[k] * v[k];
        res[n] = c[4] == T(0) ? T(0) : bn - acc;
    }
}

// bilinear prolongation weight of coarse node I for fine node i (coarsening
// factor c), zero outside its support
__device__ __forceinline__ float pw1(int i, int I, int c) {
    if (c == 1) return i == I ? 1.0f : 0.0f;
    int d = i - 2 * I;
    return d == 0 ? 1.0f : ((d == 1 || d == -1) ? 0.5f : 0.0f);
}

// prolongation weight of coarse node I for fine node i (coarsening factor
// c, |i - c I| <= c - 1): 1 on the injected node, 1/2 beside it
__device__ __forceinline__ float pwt(int i, int I, int c) { return i == c * I ? 1.0f : 0.5f; }

// b_c = P^T res_f (the residual is zero on inactive fine nodes); coarse
// nodes inactive when their diagonal is zero
template <typename T>
__device__ __forceinline__ void restrict_range(const T* res, int fnr, int fnz, T* bc, const T* Dc, int cnr, int cnz,
                                               int cr, int cz, int start, int stride) {
    const int fw = fnr + 1, cw = cnr + 1, cn = cw * (cnz + 1);
    for (int N = start; N < cn; N += stride) {
        const int I = N % cw, J = N / cw;
        const T dc = Dc[N];
        T v[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int j = cz * J + a - 1, i = cr * I + q - 1;
                const bool ok = a - 1 >= 1 - cz && a - 1 <= cz - 1 && q - 1 >= 1 - cr && q - 1 <= cr - 1 && i >= 0 &&
                                j >= 0 && i <= fnr && j <= fnz;
                v[a][q] = ok ? res[j * fw + i] : T(0);
            }
        T acc = T(0);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int j = cz * J + a - 1, i = cr * I + q - 1;
                if (a - 1 < 1 - cz || a - 1 > cz - 1 || q - 1 < 1 - cr || q - 1 > cr - 1) continue;
                if (i < 0 || j < 0 || i > fnr || j > fnz) continue;
                acc += (T)(pwt(i, I, cr) * pwt(j, J, cz)) * v[a][q];
            }
        bc[N] = dc == T(0) ? T(0) : acc;
    }
}

// y_f += P y_c on active fine nodes (the coarse correction is zero on
// inactive coarse nodes)
template <typename T>
__device__ __forceinline__ void prolong_range(T* yf, const T* Df, int fnr, int fnz, const T* yc, int cnr, int cnz,
                                              int cr, int cz, int start, int stride) {
    const int fw = fnr + 1, cw = cnr + 1, fn = fw * (fnz + 1);
    for (int n = start; n < fn; n += stride) {
        const int i = n % fw, j = n / fw;
        const int Ia = i / cr, Ib = (i + cr - 1) / cr, Ja = j / cz, Jb = (j + cz - 1) / cz;
        const T df = Df[n];
        const T y00 = yc[Ja * cw + Ia];
        const T y01 = Ib <= cnr ? yc[Ja * cw + Ib] : T(0);
        const T y10 = Jb <= cnz ? yc[Jb * cw + Ia] : T(0);
        const T y11 = (Ib <= cnr && Jb <= cnz) ? yc[Jb * cw + Ib] : T(0);
        const T wgt = (T)((Ia == Ib ? 1.0f : 0.5f) * (Ja == Jb ? 1.0f : 0.5f));
        T acc = wgt * y00;
        if (Ib != Ia) acc += wgt * y01;
        if (Jb != Ja) {
            acc += wgt * y10;
            if (Ib != Ia) acc += wgt * y11;
        }
        if (df != T(0)) yf[n] += acc;
    }
}

// coarsest level: y = A^-1 b with the precomputed dense inverse (stored
// exactly symmetric); one block.  A wavefront takes a row: its lanes take
// every 64th column and the row sum is a fixed butterfly over the lanes.
// sb: kMaxCoarse entries of shared memory.
template <typename T>
__device__ __forceinline__ void coarse_block(const T* b, T* y, const int* cmap, const int* clist, const T* inv, int nc,
                                             int cn, T* sb) {
    for (int k = threadIdx.x; k < nc; k += blockDim.x) sb[k] = b[clist[k]];
    for (int n = threadIdx.x; n < cn; n += blockDim.x)
        if (cmap[n] < 0) y[n] = T(0);
    __syncthreads();
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    for (int r = threadIdx.x >> 6; r < nc; r += nw) {
        T acc = T(0);
        for (int c = lane; c < nc; c += 64) acc += inv[r * nc + c] * sb[c];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (lane == 0) y[clist[r]] = acc;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_coarse(const T* b, T* y, const int* cmap, const int* clist, const T* inv,
                                                int nc, int cn, const DevScalars* s) {
    __shared__ T sb[kMaxCoarse];
    if (s->done) return;
    coarse_block(b, y, cmap, clist, inv, nc, cn, sb);
}

// The coarse end of the V-cycle, from the first level of at most
// kTailNodes nodes down to the dense solve, in one block: the same steps as
// the kernels above, in the same order, each a block-stride loop followed
// by a block barrier (on these small levels a kernel launch per step costs
// more than the step).
constexpr int kTailNodes = 2200;
constexpr int kMaxTail = 8;
template <typename T>
struct TailLevel {
    Sten S;
    T *x, *y, *b, *res;
    const T* D;
    int nr, nz, cr, cz;
};
template <typename T>
struct TailArgs {
    TailLevel<T> L[kMaxTail];
    int n;                        // levels; the last one is solved densely
    const int* cmap;
    const T* inv;
    int nc;
    const DevScalars* s;
};

template <typename T>
__global__ __launch_bounds__(1024) void k_tail(TailArgs<T> a) {
    __shared__ T sb[kMaxCoarse];
    if (a.s->done) return;
    const int t0 = threadIdx.x, st = blockDim.x;
    const int last = a.n - 1;
    for (int l = 0; l < last; ++l) {
        const TailLevel<T>& L = a.L[l];
        const TailLevel<T>& C = a.L[l + 1];
        jac9_range(L.S, L.x, L.b, L.x, L.nr, L.nz, 1, t0, st, kW1);
        __syncthreads();
        jac9_range(L.S, L.x, L.b, L.y, L.nr, L.nz, 0, t0, st, kW2);
        __syncthreads();
        res9_range(L.S, L.y, L.b, L.res, L.nr, L.nz, t0, st);
        __syncthreads();
        restrict_range((const T*)L.res, L.nr, L.nz, C.b, C.D, C.nr, C.nz, L.cr, L.cz, t0, st);
        __syncthreads();
    }
    {
        const TailLevel<T>& C = a.L[last];
        const int cn = (C.nr + 1) * (C.nz + 1);
        coarse_block((const T*)C.b, C.y, a.cmap, a.cmap + cn, a.inv, a.nc, cn, sb);
        __syncthreads();
    }
    for (int l = last - 1; l >= 0; --l) {
        const TailLevel<T>& L = a.L[l];
        const TailLevel<T>& C = a.L[l + 1];
        prolong_range(L.y, L.D, L.nr, L.nz, (const T*)C.y, C.nr, C.nz, L.cr, L.cz, t0, st);
        __syncthreads();
        jac9_range(L.S, L.y, L.b, L.x, L.nr, L.nz, 0, t0, st, kW2);
        __syncthreads();
        jac9_range(L.S, L.x, L.b, L.y, L.nr, L.nz, 0, t0, st, kW1);
        __syncthreads();
    }
}

// The same tail with its levels resident in LDS: one launch stages the
// stencils of the smoothed levels and the first level's right-hand side
// (one batch of loads per level), every pass then reads and writes LDS
// (the pass functions above take generic pointers), and only the first
// level's result goes back to memory.  Layout in the dynamic LDS, per
// smoothed level l from off[l]: A[0..8], b, x, y, res (nn_l each); the
// coarsest level's b and y from off[last].  A tail level has at most
// kTailNodes <= 3 x 1024 nodes.
struct TailLds {
    int off[kMaxTail];
    int bytes;
};

template <typename T>
__global__ __launch_bounds__(1024) void k_tail_lds(TailArgs<T> a, TailLds o) {
    extern __shared__ unsigned char tail_dyn[];
    __shared__ T sb[kMaxCoarse];
    if (a.s->done) return;
    T* lds = reinterpret_cast<T*>(tail_dyn);
    const int t0 = threadIdx.x, st = blockDim.x;
    const int last = a.n - 1;
    for (int l = 0; l < last; ++l) {
        const TailLevel<T>& G = a.L[l];
        const int nn = (G.nr + 1) * (G.nz + 1);
        T* base = lds + o.off[l];
        T v[10][3];
#pragma unroll
        for (int k = 0; k < 10; ++k)
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const int n = t0 + u * 1024;
                const T* src = k < 9 ? (const T*)G.S.A[k] : (const T*)G.b;
                v[k][u] = (n < nn && (k < 9 || l == 0)) ? src[n] : T(0);
            }
#pragma unroll
        for (int k = 0; k < 10; ++k)
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const int n = t0 + u * 1024;
                if (n < nn && (k < 9 || l == 0)) base[k * nn + n] = v[k][u];
            }
    }
    __syncthreads();
    auto lev = [&](int l, Sten& S, T*& b, T*& x, T*& y, T*& res) {
        const int nn = (a.L[l].nr + 1) * (a.L[l].nz + 1);
        T* base = lds + o.off[l];
        for (int k = 0; k < 9; ++k) S.A[k] = base + k * nn;
        b = base + 9 * nn;
        x = b + nn;
        y = x + nn;
        res = y + nn;
    };
    for (int l = 0; l < last; ++l) {
        const TailLevel<T>& L = a.L[l];
        const TailLevel<T>& C = a.L[l + 1];
        Sten S;
        T *b, *x, *y, *res;
        lev(l, S, b, x, y, res);
        T* bc;
        const T* Dc;
        if (l + 1 < last) {
            Sten SC;
            T *xc, *yc, *rc;
            lev(l + 1, SC, bc, xc, yc, rc);
            Dc = (const T*)SC.A[4];
        } else {
            bc = lds + o.off[last];
            Dc = C.D;
        }
        jac9_range(S, (const T*)x, (const T*)b, x, L.nr, L.nz, 1, t0, st, kW1);
        __syncthreads();
        jac9_range(S, (const T*)x, (const T*)b, y, L.nr, L.nz, 0, t0, st, kW2);
        __syncthreads();
        res9_range(S, (const T*)y, (const T*)b, res, L.nr, L.nz, t0, st);
        __syncthreads();
        restrict_range((const T*)res, L.nr, L.nz, bc, Dc, C.nr, C.nz, L.cr, L.cz, t0, st);
        __syncthreads();
    }
    {
        const TailLevel<T>& C = a.L[last];
        const int cn = (C.nr + 1) * (C.nz + 1);
        T* bc = lds + o.off[last];
        coarse_block((const T*)bc, bc + cn, a.cmap, a.cmap + cn, a.inv, a.nc, cn, sb);
        __syncthreads();
    }
    for (int l = last - 1; l >= 0; --l) {
        const TailLevel<T>& L = a.L[l];
        const TailLevel<T>& C = a.L[l + 1];
        Sten S;
        T *b, *x, *y, *res;
        lev(l, S, b, x, y, res);
        const T* yc;
        if (l + 1 < last) {
            Sten SC;
            T *bc2, *xc, *ycc, *rc;
            lev(l + 1, SC, bc2, xc, ycc, rc);
            yc = ycc;
        } else {
            yc = lds + o.off[last] + (C.nr + 1) * (C.nz + 1);
        }
        prolong_range(y, (const T*)S.A[4], L.nr, L.nz, yc, C.nr, C.nz, L.cr, L.cz, t0, st);
        __syncthreads();
        jac9_range(S, (const T*)y, (const T*)b, x, L.nr, L.nz, 0, t0, st, kW2);
        __syncthreads();
        jac9_range(S, (const T*)x, (const T*)b, l == 0 ? a.L[0].y : y, L.nr, L.nz, 0, t0, st, kW1);
        __syncthreads();
    }
}

// ------------------------------------------- fused V-cycle level kernels
// A level above the tail takes two launches per V-cycle: the down pass
// (both pre-smoothing sweeps from a zero guess, the residual and its
// restriction to the coarse right-hand side) and the up pass (prolongation
// of the coarse correction and both post-smoothing sweeps).  A block owns a
// tile of TX x TY fine nodes.  It first copies everything it reads (right-
// hand side, stencil or face coefficients, node activity, the iterate and
// the coarse correction), on the tile and the halo its sweeps need, into
// LDS in one batch of independent loads, then runs the sweeps there: the
// iterates on the halo are recomputed instead of exchanged.  Per node the
// arithmetic is that of the one-sweep-per-launch steps above (jac0/jac9,
// res0/res9, restrict, prolong).  Off-grid, conductor and inactive nodes
// hold zero in LDS, and so do the face coefficients of faces that do not
// exist, so the sums need no bounds tests (a zero term changes no sum).
template <typename T>
struct MgArgs {
    Sten S;                      // levels >= 1
    const T* ar;                 // level 0: face coefficients and node kinds
    const T* az;
    const int8_t* nk;
    const T* b;                  // the level's right-hand side
    const T* yin;                // up pass: the pre-smoothed iterate
    T* yout;                     // down pass: the pre-smoothed iterate; up pass: the level's result
    T* bc;                       // down pass: the coarse right-hand side
    const T* yc;                 // up pass: the coarse correction (zero on inactive nodes)
    const T* Dc;                 // down pass: coarse diagonal (zero: inactive)
    int nr, nz, cnr, cnz, cr, cz, tiles_r;
    const DevScalars* s;
    // preconditioned CG (level 0 only; null when unused): the down pass
    // first sums the r.r partials of the update before it and ends the
    // solve at the target; the up pass leaves per-block partials of r.z
    // (r = b, z = the result)
    const double* chk;
    int nchk;
    double* rzp;
};

// tile shape and threads per block: 32 x 32 nodes and 512 threads in FP32,
// 16 x 16 and 256 in FP64 (whose LDS arrays and registers are twice as
// large).  The kernels take the tile's width and height as parameters;
// 64 x 32 tiles (longer staged rows) measured no faster over a step.
template <typename T>
struct MgShape {
    static constexpr int SQ = sizeof(T) == 4 ? 32 : 16;   // tile edge
    static constexpr int NT = sizeof(T) == 4 ? 512 : 256;
};

#define MG_FOR(U) _Pragma("unroll") for (int u_ = 0; u_ < (U); ++u_)

// The stencil of node n = (i, j) on a level >= 1.  The Galerkin operator is
// symmetric: the entry towards neighbour m = n + off_k equals the entry of m
// back towards n, A_k[n] = A_{8-k}[m], so entries 0..3 are read from the
// neighbours' entries 8..5 and only the arrays 4..8 are streamed (20 of 36
// bytes per node; each level's operator is then exactly symmetric).
// Entries towards nodes off the grid are zero.
template <typename T>
__device__ __forceinline__ void stencil_sym(const Sten& S, int n, int i, int j, int nr, int nz, int w, bool in,
                                            T* c) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int di = k % 3 - 1, dj = k / 3 - 1;
        if (k >= 4) {
            c[k] = in ? ((const T*)S.A[k])[n] : T(0);
        } else {
            const bool ok = in && i + di >= 0 && j + dj >= 0 && i + di <= nr && j + dj <= nz;
            c[k] = ok ? ((const T*)S.A[8 - k])[n + dj * w + di] : T(0);
        }
    }
}

// Down pass.  Local coordinates have the origin (i0 - 4, j0 - 4) and row
// stride S = TX + 6 (SY = TY + 6 rows); regions, per coordinate: faces
// [0, S) (level 0), first iterate and right-hand side [1, S), smoothed
// iterate [2, S - 1), residual [3, S - 2), owned nodes [4, S - 2).  The residual region is what the tile's coarse
// nodes restrict from (one node left of the tile when coarsening by 2).
// Each thread takes the same nodes of the smoothed-iterate region in the
// second sweep and in the residual, so on levels >= 1 it keeps their
// stencils in registers.
template <typename T, bool L0, int TX, int TY>
__global__ __launch_bounds__(MgShape<T>::NT) void k_mg_down(MgArgs<T> a) {
    constexpr int NT = MgShape<T>::NT;
    constexpr int S = TX + 6, SY = TY + 6, N = S * SY, U = (N + NT - 1) / NT;
    constexpr int YW = TX + 3, NY = YW * (TY + 3), UY = (NY + NT - 1) / NT;
    constexpr int UC = (TX * TY + NT - 1) / NT;
    __shared__ T sf[2][L0 ? N : 1];              // level 0: face coefficients ar, az
    __shared__ T sd[L0 ? 1 : N];                 // levels >= 1: diagonal
    __shared__ T sb[N], sx[N], sy[N];            // sx holds the residual after the second sweep
    __shared__ int8_t sk[L0 ? N : 1];
    if (a.s->done) return;
    if (L0 && a.chk) {
        // r.r of the new residual against the target (every block decides
        // alike; block 0 records it)
        __shared__ double sh[16];
        const double rr = sum_partials(a.chk, a.nchk, sh);
        const bool fin = isfinite(rr), done = !fin || rr <= a.s->target;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            DevScalars* sw = const_cast<DevScalars*>(a.s);
            sw->rr = rr;
            sw->iters += 1;
            if (done) { sw->done = 1; sw->nonfinite = !fin; }
        }
        if (done) return;
    }
    const int w = a.nr + 1, cw = a.cnr + 1;
    const int tb = xcd_tile(blockIdx.x, gridDim.x);
    const int i0 = (tb % a.tiles_r) * TX, j0 = (tb / a.tiles_r) * TY;
    const int oi = i0 - 4, oj = j0 - 4;
    const int hr = a.cr - 1, hz = a.cz - 1;
    const int CI = TX / a.cr, CJ = TY / a.cz, I0 = i0 / a.cr, J0 = j0 / a.cz;
    T cf[UY][L0 ? 1 : 9];
    T dc[UC];
    // stage: everything the block reads, in one batch of loads
    {
        T vb[U], vf[U][L0 ? 2 : 1];
        int8_t vk[U];
        MG_FOR(U) {
            const int t = threadIdx.x + u_ * NT;
            const int li = t % S, lj = t / S, i = oi + li, j = oj + lj;
            const bool in = t < N && i >= 0 && j >= 0 && i <= a.nr && j <= a.nz;
            const bool px = in && li >= 1 && lj >= 1;
            const int n = j * w + i;
            vb[u_] = px ? a.b[n] : T(0);
            if (L0) {
                vk[u_] = px ? (int8_t)(a.nk[n] < 0) : (int8_t)0;
                vf[u_][0] = (in && i < a.nr) ? a.ar[n] : T(0);
                vf[u_][1] = (in && j < a.nz) ? a.az[n] : T(0);
            } else {
                vf[u_][0] = px ? ((const T*)a.S.A[4])[n] : T(0);
            }
        }
        if (!L0) {
            MG_FOR(UY) {
                const int ty = threadIdx.x + u_ * NT;
                const int i = oi + 2 + ty % YW, j = oj + 2 + ty / YW;
                const bool in = ty < NY && i >= 0 && j >= 0 && i <= a.nr && j <= a.nz;
                stencil_sym<T>(a.S, j * w + i, i, j, a.nr, a.nz, w, in, cf[u_]);
            }
        }
#pragma unroll
        for (int u = 0; u < UC; ++u) {
            const int tc = threadIdx.x + u * NT;
            const int I = I0 + tc % CI, J = J0 + tc / CI;
            dc[u] = (tc < CI * CJ && I <= a.cnr && J <= a.cnz) ? a.Dc[J * cw + I] : T(0);
        }
        MG_FOR(U) {
            const int t = threadIdx.x + u_ * NT;
            if (t < N) {
                sb[t] = vb[u_];
                if (L0) {
                    sk[t] = vk[u_];
                    sf[0][t] = vf[u_][0];
                    sf[1][t] = vf[u_][1];
                } else {
                    sd[t] = vf[u_][0];
                }
            }
        }
    }
    __syncthreads();
    // level 0: (A v)(t) from the faces in LDS; d receives the diagonal
    auto apply0s = [&](const T* v, int t, T& d) -> T {
        const T fl = sf[0][t - 1], fr = sf[0][t], fd = sf[1][t - S], fu = sf[1][t];
        T dd = T(0), off = T(0);
        dd += fl; off += fl * v[t - 1];
        dd += fr; off += fr * v[t + 1];
        dd += fd; off += fd * v[t - S];
        dd += fu; off += fu * v[t + S];
        d = dd;
        return dd * v[t] - off;
    };
    auto apply9r = [&](const T* v, int t, const T* c) -> T {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < 9; ++k) acc += c[k] * v[t + (k / 3 - 1) * S + (k % 3 - 1)];
        return acc;
    };
    // first iterate x = w b / d
    MG_FOR(U) {
        const int t = threadIdx.x + u_ * NT;
        const int li = t % S, lj = t / S;
        if (t < N && li >= 1 && lj >= 1) {
            T v = T(0);
            if (L0) {
                if (sk[t]) v = (T)kW1 * sb[t] / (sf[0][t - 1] + sf[0][t] + sf[1][t - S] + sf[1][t]);
            } else {
                if (sd[t] != T(0)) v = (T)kW1 * sb[t] / sd[t];
            }
            sx[t] = v;
        }
    }
    __syncthreads();
    // second sweep; the owned nodes go out
    MG_FOR(UY) {
        const int ty = threadIdx.x + u_ * NT;
        const int li = 2 + ty % YW, lj = 2 + ty / YW, t = lj * S + li;
        if (ty < NY) {
            T v = T(0);
            if (L0 ? sk[t] != 0 : sd[t] != T(0)) {
                T d, ax;
                if (L0) ax = apply0s(sx, t, d);
                else { ax = apply9r(sx, t, cf[u_]); d = cf[u_][4]; }
                v = sx[t] + (T)kW2 * (sb[t] - ax) / d;
            }
            sy[t] = v;
            const int i = oi + li, j = oj + lj;
            if (li >= 4 && lj >= 4 && li < S - 2 && lj < SY - 2 && i <= a.nr && j <= a.nz) a.yout[j * w + i] = v;
        }
    }
    __syncthreads();
    // residual (into sx, whose first iterate is no longer read)
    MG_FOR(UY) {
        const int ty = threadIdx.x + u_ * NT;
        const int li = 2 + ty % YW, lj = 2 + ty / YW, t = lj * S + li;
        if (ty < NY && li >= 3 && lj >= 3 && li < S - 2 && lj < SY - 2) {
            T v = T(0);
            if (L0 ? sk[t] != 0 : sd[t] != T(0)) {
                T d;
                v = sb[t] - (L0 ? apply0s(sy, t, d) : apply9r(sy, t, cf[u_]));
            }
            sx[t] = v;
        }
    }
    __syncthreads();
    // b_c = P^T res on the tile's coarse nodes
#pragma unroll
    for (int u = 0; u < UC; ++u) {
        const int tc = threadIdx.x + u * NT;
        const int I = I0 + tc % CI, J = J0 + tc / CI;
        if (tc >= CI * CJ || I > a.cnr || J > a.cnz) continue;
        T acc = T(0);
        if (dc[u] != T(0)) {
            for (int j = a.cz * J - hz; j <= a.cz * J + hz; ++j) {
                if (j < 0 || j > a.nz) continue;
                for (int i = a.cr * I - hr; i <= a.cr * I + hr; ++i) {
                    if (i < 0 || i > a.nr) continue;
                    acc += (T)(pwt(i, I, a.cr) * pwt(j, J, a.cz)) * sx[(j - oj) * S + (i - oi)];
                }
            }
        }
        a.bc[J * cw + I] = acc;
    }
}

// Up pass.  Local coordinates have the origin (i0 - 2, j0 - 2) and row
// stride S = TX + 4 (SY = TY + 4 rows); regions, per coordinate:
// prolongated iterate [0, S), first post-smoothing sweep [1, S - 1), owned
// nodes [2, S - 2).  The coarse
// correction is staged on coarse nodes from (i0 - 2) / cr - 1.  Each thread
// takes the same nodes of the sweep region in both sweeps and keeps their
// right-hand side and stencil (level 0: face coefficients) in registers.
template <typename T, bool L0, int TX, int TY>
__global__ __launch_bounds__(MgShape<T>::NT) void k_mg_up(MgArgs<T> a) {
    constexpr int NT = MgShape<T>::NT;
    constexpr int S = TX + 4, SY = TY + 4, N = S * SY, U = (N + NT - 1) / NT;
    constexpr int XW = TX + 2, NX = XW * (TY + 2), UX = (NX + NT - 1) / NT;
    constexpr int CWM = TX + 7, NC = CWM * (TY + 7), UC = (NC + NT - 1) / NT;   // coarsening by 1 is the widest
    constexpr int NCF = L0 ? 4 : 9;
    __shared__ T sp[N], sx[N], sc[NC];
    __shared__ int8_t sk[N];                     // activity
    if (a.s->done) return;
    const int w = a.nr + 1, cw = a.cnr + 1;
    const int tb = xcd_tile(blockIdx.x, gridDim.x);
    const int i0 = (tb % a.tiles_r) * TX, j0 = (tb / a.tiles_r) * TY;
    const int oi = i0 - 2, oj = j0 - 2;
    const int ci = (i0 - 2) / a.cr - 1, cj = (j0 - 2) / a.cz - 1;    // exact: i0 - 2 is even
    const int CW = (TX + 4) / a.cr + 3, CH = (TY + 4) / a.cz + 3;
    T cf[UX][NCF], cb[UX];
    {
        T vy[U];
        int8_t vk[U];
        MG_FOR(U) {
            const int t = threadIdx.x + u_ * NT;
            const int li = t % S, lj = t / S, i = oi + li, j = oj + lj;
            const bool in = t < N && i >= 0 && j >= 0 && i <= a.nr && j <= a.nz;
            const int n = j * w + i;
            vy[u_] = in ? a.yin[n] : T(0);
            if (L0) vk[u_] = in ? (int8_t)(a.nk[n] < 0) : (int8_t)0;
            else vk[u_] = (in && ((const T*)a.S.A[4])[n] != T(0)) ? (int8_t)1 : (int8_t)0;
        }
        MG_FOR(UX) {
            const int tx = threadIdx.x + u_ * NT;
            const int i = oi + 1 + tx % XW, j = oj + 1 + tx / XW;
            const bool in = tx < NX && i >= 0 && j >= 0 && i <= a.nr && j <= a.nz;
            const int n = j * w + i;
            cb[u_] = in ? a.b[n] : T(0);
            if (L0) {
                cf[u_][0] = (in && i > 0) ? a.ar[n - 1] : T(0);
                cf[u_][1] = (in && i < a.nr) ? a.ar[n] : T(0);
                cf[u_][2] = (in && j > 0) ? a.az[n - w] : T(0);
                cf[u_][3] = (in && j < a.nz) ? a.az[n] : T(0);
            } else {
                stencil_sym<T>(a.S, n, i, j, a.nr, a.nz, w, in, cf[u_]);
            }
        }
        T vc[UC];
#pragma unroll
        for (int u = 0; u < UC; ++u) {
            const int t = threadIdx.x + u * NT;
            const int li = t % CWM, lj = t / CWM, I = ci + li, J = cj + lj;
            const bool in = t < NC && li < CW && lj < CH && I >= 0 && J >= 0 && I <= a.cnr && J <= a.cnz;
            vc[u] = in ? a.yc[J * cw + I] : T(0);
        }
        MG_FOR(U) {
            const int t = threadIdx.x + u_ * NT;
            if (t < N) { sp[t] = vy[u_]; sk[t] = vk[u_]; }
        }
#pragma unroll
        for (int u = 0; u < UC; ++u) {
            const int t = threadIdx.x + u * NT;
            if (t < NC) sc[t] = vc[u];
        }
    }
    __syncthreads();
    // (A v)(t) with the stencil c of the node; d receives the diagonal
    auto apply = [&](const T* v, int t, const T* c, T& d) -> T {
        if (L0) {
            T dd = T(0), off = T(0);
            dd += c[0]; off += c[0] * v[t - 1];
            dd += c[1]; off += c[1] * v[t + 1];
            dd += c[2]; off += c[2] * v[t - S];
            dd += c[3]; off += c[3] * v[t + S];
            d = dd;
            return dd * v[t] - off;
        }
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < 9; ++k) acc += c[k] * v[t + (k / 3 - 1) * S + (k % 3 - 1)];
        d = c[4];
        return acc;
    };
    // y += P y_c on active nodes (the coarse correction is zero on inactive
    // coarse nodes)
    MG_FOR(U) {
        const int t = threadIdx.x + u_ * NT;
        if (t < N && sk[t]) {
            const int i = oi + t % S, j = oj + t / S;
            const int Ia = i / a.cr, Ib = (i + a.cr - 1) / a.cr, Ja = j / a.cz, Jb = (j + a.cz - 1) / a.cz;
            const float wa = Ia == Ib ? 1.0f : 0.5f, wb = Ja == Jb ? 1.0f : 0.5f;
            const T* c0 = sc + (Ja - cj) * CWM - ci;
            const T* c1 = sc + (Jb - cj) * CWM - ci;
            T acc = (T)(wa * wb) * c0[Ia];
            if (Ib != Ia) acc += (T)(wa * wb) * c0[Ib];
            if (Jb != Ja) {
                acc += (T)(wa * wb) * c1[Ia];
                if (Ib != Ia) acc += (T)(wa * wb) * c1[Ib];
            }
            sp[t] += acc;
        }
    }
    __syncthreads();
    MG_FOR(UX) {
        const int tx = threadIdx.x + u_ * NT;
        const int t = (1 + tx / XW) * S + 1 + tx % XW;
        if (tx < NX) {
            T v = T(0);
            if (sk[t]) {
                T d;
                const T ax = apply(sp, t, cf[u_], d);
                v = sp[t] + (T)kW2 * (cb[u_] - ax) / d;
            }
            sx[t] = v;
        }
    }
    __syncthreads();
    double rz = 0.0;
    MG_FOR(UX) {
        const int tx = threadIdx.x + u_ * NT;
        const int li = 1 + tx % XW, lj = 1 + tx / XW, t = lj * S + li, i = oi + li, j = oj + lj;
        if (tx < NX && li >= 2 && lj >= 2 && li < S - 2 && lj < SY - 2 && i <= a.nr && j <= a.nz) {
            T v = T(0);
            if (sk[t]) {
                T d;
                const T ax = apply(sx, t, cf[u_], d);
                v = sx[t] + (T)kW1 * (cb[u_] - ax) / d;
            }
            a.yout[j * w + i] = v;
            rz += (double)cb[u_] * (double)v;
        }
    }
    if (L0 && a.rzp) {
        __shared__ double sh[16];
        const double t = block_total(rz, sh);
        if (threadIdx.x == 0) a.rzp[tb] = t;
    }
}
// First kernel of a fused CG iteration, on the multigrid's level-0 tiles:
// the direction p = z + beta p_old (beta = rz / rz_old from the r.z partials
// of the last V-cycle; p = z on the first iteration) on the tile and one
// node around it in LDS, then q = K p, p and q on the tile, and the
// tile's partial of p.q.
template <typename T, int TX, int TY>
__global__ __launch_bounds__(MgShape<T>::NT) void k_cg_dir(const T* ar, const T* az, const int8_t* nk, const T* z,
                                                           const T* pold, T* p, T* q, const double* rzp, int nrz,
                                                           double* pqp, DevScalars* s, int first, int nr, int nz,
                                                           int tiles_r) {
    constexpr int NT = MgShape<T>::NT;
    constexpr int S = TX + 2, N = S * (TY + 2), U = (N + NT - 1) / NT, UO = (TX * TY + NT - 1) / NT;
    __shared__ T sp[N];
    __shared__ double sh[16];
    if (s->done) return;
    const double rz = sum_partials(rzp, nrz, sh);
    if (first && !(rz > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) { s->rz_new = rz; s->done = 1; }
        return;
    }
    const T be = first ? T(0) : (T)(rz / s->rz);
    const int w = nr + 1;
    const int tb = xcd_tile(blockIdx.x, gridDim.x);
    const int i0 = (tb % tiles_r) * TX, j0 = (tb / tiles_r) * TY;
    const int oi = i0 - 1, oj = j0 - 1;
    T vz[U], vp[U];
    MG_FOR(U) {
        const int t = threadIdx.x + u_ * NT;
        const int i = oi + t % S, j = oj + t / S;
        const bool in = t < N && i >= 0 && j >= 0 && i <= nr && j <= nz;
        vz[u_] = in ? z[j * w + i] : T(0);
        vp[u_] = (in && !first) ? pold[j * w + i] : T(0);
    }
    T fl[UO], fr[UO], fd[UO], fu[UO];
    int8_t k0[UO];
    MG_FOR(UO) {
        const int to = threadIdx.x + u_ * NT;
        const int i = i0 + to % TX, j = j0 + to / TX, n = j * w + i;
        const bool in = to < TX * TY && i <= nr && j <= nz;
        k0[u_] = in ? nk[n] : (int8_t)1;
        fl[u_] = (in && i > 0) ? ar[n - 1] : T(0);
        fr[u_] = (in && i < nr) ? ar[n] : T(0);
        fd[u_] = (in && j > 0) ? az[n - w] : T(0);
        fu[u_] = (in && j < nz) ? az[n] : T(0);
    }
    MG_FOR(U) {
        const int t = threadIdx.x + u_ * NT;
        if (t < N) sp[t] = first ? vz[u_] : vz[u_] + be * vp[u_];
    }
    __syncthreads();
    double acc = 0.0;
    MG_FOR(UO) {
        const int to = threadIdx.x + u_ * NT;
        const int li = to % TX, lj = to / TX, i = i0 + li, j = j0 + lj, n = j * w + i;
        if (to < TX * TY && i <= nr && j <= nz) {
            const int t = (lj + 1) * S + li + 1;
            const T p0 = sp[t];
            T v = T(0);
            if (k0[u_] < 0) {
                // the 5-point operator; conductor neighbours hold zero
                T d = T(0), off = T(0);
                d += fl[u_]; off += fl[u_] * sp[t - 1];
                d += fr[u_]; off += fr[u_] * sp[t + 1];
                d += fd[u_]; off += fd[u_] * sp[t - S];
                d += fu[u_]; off += fu[u_] * sp[t + S];
                v = d * p0 - off;
            }
            p[n] = p0;
            q[n] = v;
            acc += (double)p0 * (double)v;
        }
    }
    const double t = block_total(acc, sh);
    if (threadIdx.x == 0) pqp[tb] = t;
    if (blockIdx.x == 0 && threadIdx.x == 0) s->rz_new = rz;
}

#undef MG_FOR

// ------------------------------------------------- multigrid construction
// Galerkin product A_c = P^T A_f P, one coarse node per thread.  A coarse
// node is active only if the fine node it injects into is active, which
// keeps P of full column rank and A_c positive definite.
__device__ __forceinline__ double fine_coef0(const double* ar, const double* az, const int8_t* nk, int n, int i, int j,
                                             int nr, int nz, int w, int k) {
    if (nk[n] >= 0) return 0.0;
    switch (k) {
    case 4: {
        double d = 0.0;
        if (i > 0) d += ar[n - 1];
        if (i < nr) d += ar[n];
        if (j > 0) d += az[n - w];
        if (j < nz) d += az[n];
        return d;
    }
    case 3: return (i > 0 && nk[n - 1] < 0) ? -ar[n - 1] : 0.0;
    case 5: return (i < nr && nk[n + 1] < 0) ? -ar[n] : 0.0;
    case 1: return (j > 0 && nk[n - w] < 0) ? -az[n - w] : 0.0;
    case 7: return (j < nz && nk[n + w] < 0) ? -az[n] : 0.0;
    default: return 0.0;
    }
}

struct RapArgs {
    const double* ar;
    const double* az;
    const int8_t* nk;   // non-null: the fine level is level 0
    const double* Af[9];
    double* Ac[9];
    int fnr, fnz, cnr, cnz, cr, cz;
};

__device__ __forceinline__ bool fine_active(const RapArgs& a, int nf) {
    return a.nk ? (a.nk[nf] < 0) : (a.Af[4][nf] != 0.0);
}

__global__ __launch_bounds__(256) void k_rap(RapArgs a) {
    const int fw = a.fnr + 1, cw = a.cnr + 1, cn = cw * (a.cnz + 1);
    for (int N = blockIdx.x * blockDim.x + threadIdx.x; N < cn; N += gridDim.x * blockDim.x) {
        const int I = N % cw, J = N / cw;
        double acc[9];
        for (int k = 0; k < 9; ++k) acc[k] = 0.0;
        if (fine_active(a, (a.cz * J) * fw + a.cr * I)) {
            for (int j = a.cz * J - (a.cz - 1); j <= a.cz * J + (a.cz - 1); ++j) {
                if (j < 0 || j > a.fnz) continue;
                for (int i = a.cr * I - (a.cr - 1); i <= a.cr * I + (a.cr - 1); ++i) {
                    if (i < 0 || i > a.fnr) continue;
                    const int nf = j * fw + i;
                    if (!fine_active(a, nf)) continue;
                    const double p1 = (double)(pw1(i, I, a.cr) * pw1(j, J, a.cz));
                    if (p1 == 0.0) continue;
                    for (int k = 0; k < 9; ++k) {
                        const int di = k % 3 - 1, dj = k / 3 - 1;
                        const int i2 = i + di, j2 = j + dj;
                        if (i2 < 0 || j2 < 0 || i2 > a.fnr || j2 > a.fnz) continue;
                        const double v = a.nk ? fine_coef0(a.ar, a.az, a.nk, nf, i, j, a.fnr, a.fnz, fw, k)
                                              : a.Af[k][nf];
                        if (v == 0.0) continue;
                        const int nf2 = j2 * fw + i2;
                        if (!fine_active(a, nf2)) continue;
                        for (int k2 = 0; k2 < 9; ++k2) {
                            const int I2 = I + k2 % 3 - 1, J2 = J + k2 / 3 - 1;
                            if (I2 < 0 || J2 < 0 || I2 > a.cnr || J2 > a.cnz) continue;
                            if (!fine_active(a, (a.cz * J2) * fw + a.cr * I2)) continue;
                            const double p2 = (double)(pw1(i2, I2, a.cr) * pw1(j2, J2, a.cz));
                            if (p2 != 0.0) acc[k2] += p1 * v * p2;
                        }
                    }
                }
            }
        }
        for (int k = 0; k < 9; ++k) a.Ac[k][N] = acc[k];
    }
}

__global__ __launch_bounds__(256) void k_to32(const double* a, float* b, int n, double scale) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) b[i] = (float)(a[i] * scale);
}

// dense matrix of the coarsest operator over its active nodes
__global__ __launch_bounds__(256) void k_coarse_dense(Sten S, const int* cmap, double* M, int nc, int nr, int nz) {
    const int w = nr + 1, cn = w * (nz + 1);
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nc * nc; t += gridDim.x * blockDim.x) M[t] = 0.0;
    __syncthreads();
    for (int n = threadIdx.x; n < cn; n += blockDim.x) {
        const int a = cmap[n];
        if (a < 0) continue;
        const int i = n % w, j = n / w;
        for (int k = 0; k < 9; ++k) {
            const int i2 = i + k % 3 - 1, j2 = j + k / 3 - 1;
            if (i2 < 0 || j2 < 0 || i2 > nr || j2 > nz) continue;
            const int b = cmap[j2 * w + i2];
            if (b < 0) continue;
            M[a * nc + b] += ((const double*)S.A[k])[n];
        }
    }
}

// in-place Gauss-Jordan inverse of an SPD matrix (no pivoting), one block
__global__ __launch_bounds__(1024) void k_invert(double* M, int n) {
    __shared__ double rowk[kMaxCoarse], colk[kMaxCoarse];
    for (int k = 0; k < n; ++k) {
        __syncthreads();
        const double piv = M[k * n + k];
        for (int c = threadIdx.x; c < n; c += blockDim.x) {
            rowk[c] = (c == k) ? 1.0 / piv : M[k * n + c] / piv;
            colk[c] = M[c * n + k];
        }
        __syncthreads();
        for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
            const int r = t / n, c = t % n;
            if (r == k) continue;
            const double f = colk[r];
            M[t] = (c == k) ? -f * rowk[k] : M[t] - f * rowk[c];
        }
        __syncthreads();
        for (int c = threadIdx.x; c < n; c += blockDim.x) M[k * n + c] = rowk[c];
    }
}

// the inverse of a symmetric matrix, made exactly symmetric (the mean of
// the two rounded triangles), one block
__global__ __launch_bounds__(1024) void k_symmetrize(double* M, int n) {
    for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
        const int r = t / n, c = t % n;
        if (r < c) {
            const double v = 0.5 * (M[r * n + c] + M[c * n + r]);
            M[r * n + c] = v;
            M[c * n + r] = v;
        }
    }
}

// largest dynamic LDS the resident tail may take: the device's limit per
// block less the static arrays, once the kernels are allowed to use it
static int tail_lds_limit() {
    int dev = 0, lim = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 0;
    lim -= (int)(kMaxCoarse * sizeof(double)) + 1024;
    if (lim <= 0 ||
        hipFuncSetAttribute((const void*)k_tail_lds<float>, hipFuncAttributeMaxDynamicSharedMemorySize, lim) !=
            hipSuccess ||
        hipFuncSetAttribute((const void*)k_tail_lds<double>, hipFuncAttributeMaxDynamicSharedMemorySize, lim) !=
            hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return lim;
}

void mg_rebuild(pic_handle* h) {
    hipStream_t st = h->stream;
    if (h->tail_lds_max < 0) h->tail_lds_max = tail_lds_limit();
    for (int l = 0; l + 1 < h->nlev; ++l) {
        Level& F = h->lv[l];
        Level& C = h->lv[l + 1];
        RapArgs a;
        a.ar = h->ar; a.az = h->az;
        a.nk = (l == 0) ? h->node_kind : nullptr;
        for (int k = 0; k < 9; ++k) { a.Af[k] = F.A64[k]; a.Ac[k] = C.A64[k]; }
        a.fnr = F.nr; a.fnz = F.nz; a.cnr = C.nr; a.cnz = C.nz; a.cr = F.cr; a.cz = F.cz;
        hipLaunchKernelGGL(k_rap, dim3((C.nn + 255) / 256), dim3(256), 0, st, a);
        for (int k = 0; k < 9; ++k)
            hipLaunchKernelGGL(k_to32, dim3((C.nn + 255) / 256), dim3(256), 0, st, (const double*)C.A64[k], C.A32[k],
                               C.nn, 1.0 / kEps0);
    }
    Level& L = h->lv[h->nlev - 1];
    if (h->ncoarse > 0) {
        Sten S;
        for (int k = 0; k < 9; ++k) S.A[k] = L.A64[k];
        if (h->nlev == 1) {
            // a single level: the coarse matrix is the level-0 operator (test-sized grids only)
        }
        hipLaunchKernelGGL(k_coarse_dense, dim3(1), dim3(256), 0, st, S, h->cmap, h->cinv64, h->ncoarse, L.nr, L.nz);
        hipLaunchKernelGGL(k_invert, dim3(1), dim3(1024), 0, st, h->cinv64, h->ncoarse);
        hipLaunchKernelGGL(k_symmetrize, dim3(1), dim3(1024), 0, st, h->cinv64, h->ncoarse);
        hipLaunchKernelGGL(k_to32, dim3(64), dim3(256), 0, st, (const double*)h->cinv64, h->cinv32,
                           h->ncoarse * h->ncoarse, kEps0);
    }
}

template <typename T>
struct VecSet;
template <>
struct VecSet<double> {
    static double* x(Level& L) { return L.x64; }
    static double* y(Level& L) { return L.y64; }
    static double* b(Level& L) { return L.b64; }
    static double* res(Level& L) { return L.res64; }
    static Sten sten(Level& L) { Sten S; for (int k = 0; k < 9; ++k) S.A[k] = L.A64[k]; return S; }
    static const double* diag(Level& L) { return L.A64[4]; }
    static const double* ar(pic_handle* h) { return h->ar; }
    static const double* az(pic_handle* h) { return h->az; }
    static const double* cinv(pic_handle* h) { return h->cinv64; }
};
template <>
struct VecSet<float> {
    static float* x(Level& L) { return L.x32; }
    static float* y(Level& L) { return L.y32; }
    static float* b(Level& L) { return L.b32; }
    static float* res(Level& L) { return L.res32; }
    static Sten sten(Level& L) { Sten S; for (int k = 0; k < 9; ++k) S.A[k] = L.A32[k]; return S; }
    static const float* diag(Level& L) { return L.A32[4]; }
    static const float* ar(pic_handle* h) { return h->ar32; }
    static const float* az(pic_handle* h) { return h->az32; }
    static const float* cinv(pic_handle* h) { return h->cinv32; }
};

static inline dim3 grid_for(int n) { return dim3(std::min(8192, (n + 255) / 256)); }

// copy the device scalars to their pinned host mirror and wait for them
static bool read_scalars(pic_handle* h) {
    return hipMemcpyAsync(h->h_sc, h->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, h->stream) == hipSuccess &&
           hipStreamSynchronize(h->stream) == hipSuccess;
}

// symmetric V(2,2) cycle: on level l, y = M_l b (b in the level's b buffer;
// level 0 takes b0 and writes y0).  A preconditioned-CG caller passes a
// hook at level 0: the r.r partials its first launch tests for convergence,
// and where the up pass leaves the r.z partials (one per level-0 tile).
struct CgHook {
    const double* chk;
    int nchk;
    double* rzp;
};

template <typename T>
static void vcycle(pic_handle* h, int l, const T* b0, T* y0, const CgHook* hook = nullptr) {
    using V = VecSet<T>;
    hipStream_t st = h->stream;
    Level& L = h->lv[l];
    const DevScalars* s = h->sc;
    const T* b = (l == 0) ? b0 : V::b(L);
    T* y = (l == 0) ? y0 : V::y(L);
    T* x = V::x(L);
    if (l >= 1 && l < h->nlev - 1 && L.nn <= kTailNodes && h->nlev - l <= kMaxTail) {
        TailArgs<T> ta;
        ta.n = h->nlev - l;
        for (int k = 0; k < ta.n; ++k) {
            Level& M = h->lv[l + k];
            TailLevel<T>& t = ta.L[k];
            t.S = V::sten(M);
            t.x = V::x(M); t.y = V::y(M); t.b = V::b(M); t.res = V::res(M);
            t.D = V::diag(M);
            t.nr = M.nr; t.nz = M.nz; t.cr = M.cr; t.cz = M.cz;
        }
        ta.cmap = h->cmap;
        ta.inv = V::cinv(h);
        ta.nc = h->ncoarse;
        ta.s = s;
        TailLds o;
        int off = 0;
        for (int k = 0; k < ta.n; ++k) {
            o.off[k] = off;
            const int nn = (ta.L[k].nr + 1) * (ta.L[k].nz + 1);
            off += (k + 1 < ta.n ? 13 : 2) * nn;
        }
        o.bytes = off * (int)sizeof(T);
        if (o.bytes <= h->tail_lds_max) {
            hipLaunchKernelGGL(k_tail_lds<T>, dim3(1), dim3(1024), o.bytes, st, ta, o);
            return;
        }
        hipLaunchKernelGGL(k_tail<T>, dim3(1), dim3(1024), 0, st, ta);
        return;
    }
    if (l == h->nlev - 1) {
        // (level 0 always has a coarser level: a grid too small to coarsen
        // gets an identity level)
        hipLaunchKernelGGL(k_coarse<T>, dim3(1), dim3(256), 0, st, b, y, h->cmap, h->cmap + L.nn, V::cinv(h),
                           h->ncoarse, L.nn, s);
        return;
    }
    Level& C = h->lv[l + 1];
    MgArgs<T> a;
    a.S = V::sten(L);
    a.ar = V::ar(h);
    a.az = V::az(h);
    a.nk = (l == 0) ? h->node_kind : nullptr;
    a.b = b;
    a.yin = nullptr;
    a.yout = x;            // the pre-smoothed iterate
    a.bc = V::b(C);
    a.yc = nullptr;
    a.Dc = V::diag(C);
    a.nr = L.nr; a.nz = L.nz; a.cnr = C.nr; a.cnz = C.nz; a.cr = L.cr; a.cz = L.cz;
    constexpr int SQ = MgShape<T>::SQ;
    const dim3 nt(MgShape<T>::NT);
    a.tiles_r = (L.nr + SQ) / SQ;
    a.s = s;
    a.chk = (l == 0 && hook) ? hook->chk : nullptr;
    a.nchk = (l == 0 && hook) ? hook->nchk : 0;
    a.rzp = (l == 0 && hook) ? hook->rzp : nullptr;
    const dim3 tiles(a.tiles_r * ((L.nz + SQ) / SQ));
    if (l == 0) hipLaunchKernelGGL((k_mg_down<T, true, SQ, SQ>), tiles, nt, 0, st, a);
    else hipLaunchKernelGGL((k_mg_down<T, false, SQ, SQ>), tiles, nt, 0, st, a);
    vcycle<T>(h, l + 1, nullptr, nullptr);
    a.yin = x;
    a.yout = y;
    a.bc = nullptr;
    a.yc = V::y(C);
    a.chk = nullptr;
    if (l == 0) hipLaunchKernelGGL((k_mg_up<T, true, SQ, SQ>), tiles, nt, 0, st, a);
    else hipLaunchKernelGGL((k_mg_up<T, false, SQ, SQ>), tiles, nt, 0, st, a);
}

// preconditioned CG on the level-0 operator; r is overwritten, x receives
// the correction.  Returns the iteration count.
template <typename T>
static void precondition(pic_handle* h, int ident, const T* r, T* z) {
    if (ident)
        hipLaunchKernelGGL(k_copy<T>, grid_for(h->nn), dim3(256), 0, h->stream, z, r, (const DevScalars*)h->sc, h->nn);
    else
        vcycle<T>(h, 0, r, z);
}

// harvest hook of an FP64 solve: iterate k, after the V-cycle z = M r that
// the learned preconditioner also applies before the network, gives the
// pair (res = r - K z, e = x* - (x_k + z)) of the error the V-cycle leaves;
// it is kept in pair slot (n_pairs + k) of the ring.  The level-0
// multigrid residual vector is free between V-cycles and holds res.
template <typename T>
static void harvest_iterate(pic_handle*, int, const T*, const T*, const T*) {}
template <>
void harvest_iterate<double>(pic_handle* h, int k, const double* r, const double* x, const double* z) {
    if (!h->harvesting || k >= h->harvest_limit) return;
    Level& L = h->lv[0];
    hipStream_t st = h->stream;
    const DevScalars* s = h->sc;
    hipLaunchKernelGGL(k_res0<double>, grid_for(L.nn), dim3(256), 0, st, (const double*)h->ar, (const double*)h->az,
                       (const int8_t*)h->node_kind, z, r, L.res64, s, L.nr, L.nz);
    const int slot = (int)((h->net.n_pairs + k) % h->net.cap_pairs);
    unet::harvest_iter(h->net, slot, L.res64, x, z, h->chi, h->node_kind, h->hx64 + (size_t)k * h->nn,
                       &h->sc->done, h->w, h->nn, st);
}

// Capture what `body` launches on the handle's stream into an executable
// graph: the launches go to a private stream in capture mode (nothing
// runs), which stands in for the handle's stream meanwhile.  False if the
// runtime refuses any part; the caller then launches eagerly.
template <class F>
static bool capture_graph(pic_handle* h, hipGraphExec_t* out, F&& body) {
    *out = nullptr;
    if (!h->cap_stream && hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    hipStream_t keep = h->stream;
    h->stream = h->cap_stream;
    bool ok = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
    hipGraph_t g = nullptr;
    if (ok) {
        body();
        ok = hipStreamEndCapture(h->cap_stream, &g) == hipSuccess && g != nullptr;
    }
    h->stream = keep;
    if (ok) ok = hipGraphInstantiate(out, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    if (!ok) {
        *out = nullptr;
        (void)hipGetLastError();
    }
    return ok;
}

// preconditioned CG with the multigrid preconditioner in fused launches
// (k_cg_dir, k_cg_step, V-cycle); r is overwritten, x receives the
// correction.  The second direction buffer is the level-0 y vector, which
// the V-cycle leaves unused.  Returns the iteration count.
template <typename T>
static int pcg_mg(pic_handle* h, T* r, T* x, T* z, T* p, T* q, int max_iter, int* err, int first_check,
                  bool x_zero, bool host_check = true) {
    using V = VecSet<T>;
    hipStream_t st = h->stream;
    const int nn = h->nn;
    DevScalars* s = h->sc;
    T* pb[2] = {p, V::y(h->lv[0])};
    double* rzp = h->cgpart;
    double* pqp = h->cgpart + h->cgpart_n;
    double* rrp = pqp + h->cgpart_n;
    // r.z partials: one per level-0 tile of the V-cycle's up pass; p.q
    // partials: one per tile of k_cg_dir (the same tiles)
    constexpr int SQ = MgShape<T>::SQ;
    const int tiles_r0 = (h->nr + SQ) / SQ;
    const int tiles0 = tiles_r0 * ((h->nz + SQ) / SQ), nrz = tiles0;
    if (!x_zero) hipLaunchKernelGGL(k_fill<T>, grid_for(nn), dim3(256), 0, st, x, nn);
    // the launches of the start and of iteration `it`, on h->stream
    auto start = [&]() {
        hipLaunchKernelGGL(k_begin_cg, dim3(1), dim3(1), 0, h->stream, s);
        CgHook hook{nullptr, 0, rzp};
        vcycle<T>(h, 0, r, z, &hook);
    };
    auto iteration = [&](int it) {
        T* pn = pb[it & 1];
        const T* po = pb[(it + 1) & 1];
        hipLaunchKernelGGL((k_cg_dir<T, SQ, SQ>), dim3(tiles0), dim3(MgShape<T>::NT), 0, h->stream, V::ar(h), V::az(h),
                           h->node_kind, (const T*)z, po, pn, q, (const double*)rzp, nrz, pqp, s, it == 0 ? 1 : 0,
                           h->nr, h->nz, tiles_r0);
        hipLaunchKernelGGL(k_cg_step<T>, dim3(kCgBlocks), dim3(kCgThreads), 0, h->stream, x, r, (const T*)pn,
                           (const T*)q, (const double*)pqp, tiles0, rrp, s, nn);
        CgHook hook{rrp, kCgBlocks, rzp};
        vcycle<T>(h, 0, r, z, &hook);
    };
    // graphs: the launches only read the handle's fixed buffers, so the
    // graphs captured at the first solve serve every later one (a harvested
    // solve adds launches of its own and runs without them)
    const int pi = sizeof(T) == 4 ? 0 : 1;
    const bool want = h->cfg.solver.graphs != 0 && !h->harvesting;
    if (want && !h->cg_graph_tried[pi]) {
        h->cg_graph_tried[pi] = true;
        hipGraphExec_t* g = h->cg_graph[pi];
        bool ok = capture_graph(h, &g[0], start);
        ok = ok && capture_graph(h, &g[1], [&] { iteration(0); });
        ok = ok && capture_graph(h, &g[2], [&] { iteration(1); });
        ok = ok && capture_graph(h, &g[3], [&] { iteration(2); });
        if (!ok)
            for (int v = 0; v < 4; ++v)
                if (g[v]) { (void)hipGraphExecDestroy(g[v]); g[v] = nullptr; }
        h->cg_graph_ok[pi] = ok;
    }
    const bool use = want && h->cg_graph_ok[pi];
    if (use) {
        if (hipGraphLaunch(h->cg_graph[pi][0], st) != hipSuccess) { *err = PIC_E_HIP; return 0; }
    } else {
        start();
    }
    harvest_iterate<T>(h, 0, r, x, (const T*)z);
    int it = 0;
    for (; it < max_iter; ++it) {
        if (use) {
            if (hipGraphLaunch(h->cg_graph[pi][it == 0 ? 1 : (it & 1) ? 2 : 3], st) != hipSuccess) {
                *err = PIC_E_HIP;
                return it;
            }
        } else {
            iteration(it);
        }
        harvest_iterate<T>(h, it + 1, r, x, (const T*)z);
        // the host reads the convergence flag first after first_check
        // iterations (what the same solve needed last time), then after
        // every iteration: iterations launched after convergence return at
        // once but still cost their launches.  Without host checks the
        // max_iter iterations are launched and the device stops itself.
        if (host_check && (it + 1 >= first_check || it + 1 == max_iter)) {
            if (!read_scalars(h)) { *err = PIC_E_HIP; return it; }
            if (h->h_sc->done) break;
        }
    }
    if (!host_check) return 0;
    if (it == 0 && !read_scalars(h)) { *err = PIC_E_HIP; return it; }
    if (h->h_sc->nonfinite) *err = PIC_E_NONFINITE;
    return h->h_sc->iters;
}

// preconditioned CG with separate launches for every vector operation and
// reduction (the identity preconditioner: plain CG)
template <typename T>
static int pcg(pic_handle* h, T* r, T* x, T* z, T* p, T* q, int max_iter, int* err, int ident = 0,
               int first_check = kCheckEvery, bool x_zero = false, bool host_check = true) {
    if (!ident) return pcg_mg<T>(h, r, x, z, p, q, max_iter, err, first_check, x_zero, host_check);
    using V = VecSet<T>;
    hipStream_t st = h->stream;
    const int nn = h->nn;
    DevScalars* s = h->sc;
    hipLaunchKernelGGL(k_begin_cg, dim3(1), dim3(1), 0, st, s);
    hipLaunchKernelGGL(k_fill<T>, grid_for(nn), dim3(256), 0, st, x, nn);
    precondition<T>(h, ident, r, z);
    harvest_iterate<T>(h, 0, r, x, (const T*)z);
    hipLaunchKernelGGL(k_copy<T>, grid_for(nn), dim3(256), 0, st, p, (const T*)z, s, nn);
    hipLaunchKernelGGL(k_dot<T>, dim3(kRedBlocks), dim3(256), 0, st, (const T*)r, (const T*)z, h->part, s, nn);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, st, (const double*)h->part, s, 0);
    int it = 0;
    for (; it < max_iter; ++it) {
        hipLaunchKernelGGL(k_spmv_dot<T>, dim3(kRedBlocks), dim3(256), 0, st, V::ar(h), V::az(h), h->node_kind,
                           (const T*)p, q, h->part, s, h->nr, h->nz);
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, st, (const double*)h->part, s, 1);
        hipLaunchKernelGGL(k_update_xr<T>, dim3(kRedBlocks), dim3(256), 0, st, x, r, (const T*)p, (const T*)q,
                           h->part, s, nn);
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, st, (const double*)h->part, s, 2);
        precondition<T>(h, ident, r, z);
        harvest_iterate<T>(h, it + 1, r, x, (const T*)z);
        hipLaunchKernelGGL(k_dot<T>, dim3(kRedBlocks), dim3(256), 0, st, (const T*)r, (const T*)z, h->part, s, nn);
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, st, (const double*)h->part, s, 3);
        hipLaunchKernelGGL(k_update_p<T>, grid_for(nn), dim3(256), 0, st, p, (const T*)z, s, nn);
        // the host reads the convergence flag first after first_check
        // iterations (what the same solve needed last time), then after
        // every iteration: iterations launched after convergence return at
        // once but still cost their launches
        if (it + 1 >= first_check || it + 1 == max_iter) {
            if (!read_scalars(h)) { *err = PIC_E_HIP; return it; }
            if (h->h_sc->done) break;
        }
    }
    // (the scalars were read after the last iteration launched, unless
    // max_iter is 0)
    if (it == 0 && !read_scalars(h)) { *err = PIC_E_HIP; return it; }
    if (h->h_sc->nonfinite) *err = PIC_E_NONFINITE;
    return h->h_sc->iters;
}

// learned preconditioner, one application z = P(r): the multigrid V-cycle
// z = M r, then the network's output v for the residual the V-cycle leaves,
// res = r - K z, as a one-dimensional Galerkin correction z += c v with
// c = (v.res)/(v.K v) (c = 0 if v.K v is not positive).  The correction
// minimises the energy-norm error of z along v, so the step is never worse
// than the V-cycle alone; the network supplies only a direction, so it is
// trained on unit-RMS pairs (reading R28).
__global__ __launch_bounds__(256) void k_spmv_dot2(const float* ar, const float* az, const int8_t* nk,
                                                   const float* v, const float* res, float* q, double* part,
                                                   const DevScalars* s, int nr, int nz) {
    __shared__ double sh[4];
    if (s->done) return;
    const int w = nr + 1, nn = w * (nz + 1);
    double a = 0.0, b = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += gridDim.x * blockDim.x) {
        if (nk[n] >= 0) { q[n] = 0.0f; continue; }
        float d;
        const float av = apply0(ar, az, nk, v, n, n % w, n / w, nr, nz, w, d);
        q[n] = av;
        a += (double)v[n] * (double)av;
        b += (double)v[n] * (double)res[n];
    }
    double t1 = block_sum(a, sh);
    double t2 = block_sum(b, sh);
    if (threadIdx.x == 0) { part[blockIdx.x] = t1; part[kRedBlocks + blockIdx.x] = t2; }
}

// what = 0: rr_net = sum of part; 1: c_net from (v.Av, v.res)
__global__ __launch_bounds__(256) void k_reduce_net(const double* part, DevScalars* s, int what) {
    __shared__ double a[kRedBlocks], b[kRedBlocks];
    if (s->done) return;
    for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) {
        a[i] = part[i];
        b[i] = what ? part[kRedBlocks + i] : 0.0;
    }
    __syncthreads();
    for (int o = kRedBlocks / 2; o > 0; o >>= 1) {
        for (int i = threadIdx.x; i < o; i += blockDim.x) { a[i] += a[i + o]; b[i] += b[i + o]; }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    if (what == 0) {
        s->rr_net = a[0] > 0.0 ? a[0] : 1.0;
    } else {
        const double vav = a[0], vr = b[0];
        s->c_net = (vav > 0.0 && isfinite(vav) && isfinite(vr)) ? vr / vav : 0.0;
    }
}

__global__ __launch_bounds__(256) void k_axpy_net(float* z, const float* v, const DevScalars* s, int nn) {
    if (s->done) return;
    const float c = (float)s->c_net;
    if (c == 0.0f) return;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += gridDim.x * blockDim.x) z[n] += c * v[n];
}

static void unet_apply(pic_handle* h, const float* r, float* z) {
    unet::Net& n = h->net;
    Level& L = h->lv[0];
    hipStream_t st = h->stream;
    DevScalars* s = h->sc;
    const float* ar = h->ar32;
    const float* az = h->az32;
    const int8_t* nk = h->node_kind;
    const int nn = h->nn;
    vcycle<float>(h, 0, r, z);
    // after the V-cycle the level-0 work vectors are free: res, the network
    // direction v (in x) and K v (in y)
    float* res = L.res32;
    float* v = L.x32;
    float* q = L.y32;
    hipLaunchKernelGGL(k_res0<float>, grid_for(nn), dim3(256), 0, st, ar, az, nk, (const float*)z, r, res,
                       (const DevScalars*)s, h->nr, h->nz);
    hipLaunchKernelGGL(k_dot<float>, dim3(kRedBlocks), dim3(256), 0, st, (const float*)res, (const float*)res, h->part,
                       (const DevScalars*)s, nn);
    hipLaunchKernelGGL(k_reduce_net, dim3(1), dim3(256), 0, st, (const double*)h->part, s, 0);
    unet::input_from_r32(n, res, &s->rr_net, h->chi, nk, h->w, (double)h->img_free, st);
    unet::forward(n, 1, st);
    unet::out_to_z(n, &s->rr_net, nk, v, h->w, nn, st);
    hipLaunchKernelGGL(k_spmv_dot2, dim3(kRedBlocks), dim3(256), 0, st, ar, az, nk, (const float*)v,
                       (const float*)res, q, h->part, (const DevScalars*)s, h->nr, h->nz);
    hipLaunchKernelGGL(k_reduce_net, dim3(1), dim3(256), 0, st, (const double*)h->part, s, 1);
    hipLaunchKernelGGL(k_axpy_net, grid_for(nn), dim3(256), 0, st, z, (const float*)v, (const DevScalars*)s, nn);
    h->unet_apps++;
}

// Flexible CG (FP32) on the normalised residual with the network as the
// preconditioner.  r is overwritten, x receives the correction.  Returns
// the iteration count; sets DevScalars::fallback when the network output
// stops being a descent direction.  The host reads the state after every
// iteration: one network evaluation outweighs the read by far.
static int fpcg(pic_handle* h, float* r, float* x, float* z, float* p, float* q, int max_iter, int* err) {
    hipStream_t st = h->stream;
    const int nn = h->nn;
    DevScalars* s = h->sc;
    hipLaunchKernelGGL(k_begin_cg, dim3(1), dim3(1), 0, st, s);
    hipLaunchKernelGGL(k_fill<float>, grid_for(nn), dim3(256), 0, st, x, nn);
    unet_apply(h, r, z);
    hipLaunchKernelGGL(k_copy<float>, grid_for(nn), dim3(256), 0, st, p, (const float*)z, s, nn);
    hipLaunchKernelGGL(k_dot<float>, dim3(kRedBlocks), dim3(256), 0, st, (const float*)r, (const float*)z, h->part, s,
                       nn);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, st, (const double*)h->part, s, 0);
    hipLaunchKernelGGL(k_fcg_start, dim3(1), dim3(1), 0, st, s);
    for (int it = 0; it < max_iter; ++it) {
        hipLaunchKernelGGL(k_spmv_dot<float>, dim3(kRedBlocks), dim3(256), 0, st, (const float*)h->ar32,
                           (const float*)h->az32, (const int8_t*)h->node_kind, (const float*)p, q, h->part,
                           (const DevScalars*)s, h->nr, h->nz);
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, st, (const double*)h->part, s, 1);
        hipLaunchKernelGGL(k_update_xr<float>, dim3(kRedBlocks), dim3(256), 0, st, x, r, (const float*)p,
                           (const float*)q, h->part, (const DevScalars*)s, nn);
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, st, (const double*)h->part, s, 2);
        if (!read_scalars(h)) { *err = PIC_E_HIP; return it; }
        if (h->h_sc->done) break;
        unet_apply(h, r, z);
        hipLaunchKernelGGL(k_dot2, dim3(kRedBlocks), dim3(256), 0, st, (const float*)z, (const float*)r,
                           (const float*)q, h->part, (const DevScalars*)s, nn);
        hipLaunchKernelGGL(k_reduce_fcg, dim3(1), dim3(256), 0, st, (const double*)h->part, s);
        hipLaunchKernelGGL(k_update_p<float>, grid_for(nn), dim3(256), 0, st, p, (const float*)z,
                           (const DevScalars*)s, nn);
    }
    if (!read_scalars(h)) { *err = PIC_E_HIP; return 0; }
    if (h->h_sc->nonfinite) *err = PIC_E_NONFINITE;
    if (!h->h_sc->done) h->h_sc->fallback = 1;   // out of iterations
    return h->h_sc->iters;
}

template <typename T>
__global__ __launch_bounds__(256) void k_add_phi(double* phi, const T* x, const int8_t* nk, DevScalars* s, int nn,
                                                 int scaled) {
    // FP32 inner: x solves (K/eps0) x = r / ||r||, so K^-1 r = x ||r|| / eps0
    if (s->outer_done) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // the pass's Krylov iterations
        s->its_pass[min(max(s->outer - 1, 0), 3)] = s->iters;
        s->iters_total += s->iters;
    }
    const double f = scaled ? (1.0 / s->scale) / kEps0 : 1.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += gridDim.x * blockDim.x)
        if (nk[n] < 0) phi[n] += f * (double)x[n];
}

// initial guess of the next solve on unknown nodes, extrapolated in time
// from the last solutions: quadratic (3 phi - 3 phi_prev + phi_prev2) once
// two earlier ones are known, linear (2 phi - phi_prev) with one, none
// without; the history moves one step back
__global__ __launch_bounds__(256) void k_extrapolate(double* phi, double* prev, double* prev2, const int8_t* nk, int nn,
                                                     int have) {
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += gridDim.x * blockDim.x) {
        if (nk[n] >= 0) continue;
        const double t = phi[n], p1 = prev[n];
        if (have >= 2) phi[n] = 3.0 * (t - p1) + prev2[n];
        else if (have == 1) phi[n] = 2.0 * t - p1;
        prev2[n] = p1;
        prev[n] = t;
    }
}

void launch_extrapolate(pic_handle* h) {
    hipLaunchKernelGGL(k_extrapolate, grid_for(h->nn), dim3(256), 0, h->stream, h->phi, h->phi_prev, h->phi_prev2,
                       (const int8_t*)h->node_kind, h->nn, h->have_prev);
    h->have_prev = std::min(h->have_prev + 1, 2);
}

__global__ __launch_bounds__(256) void k_set_dirichlet(double* phi, const int8_t* nk, const double* Up, int nn,
                                                       DevScalars* s) {
    // (the solve is over: later Krylov solves start unfinished)
    if (blockIdx.x == 0 && threadIdx.x == 0) s->outer_done = 0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += gridDim.x * blockDim.x)
        if (nk[n] >= 0) phi[n] = nk[n] >= 1 ? Up[nk[n] - 1] : 0.0;
}

__global__ void k_set_target(DevScalars* s, double v) { s->target = v; }

int field_solve(pic_handle* h, double* phi, const double* Q, const double* Up, double tol, int method,
                int32_t* iters_out, double* relres_out) {
    hipStream_t st = h->stream;
    const int nn = h->nn;
    // a harvested solve runs FP64 MG-PCG and keeps its first Krylov iterates
    // (residual r_k, error x* - x_k of the first outer pass) as training pairs
    const bool harvest = h->harvest_now && h->unet_on && Q != nullptr && h->net.cap_pairs > 0;
    if (harvest) method = PIC_SOLVE_MGPCG_FP64;
    const int fp64 = (method == PIC_SOLVE_MGPCG_FP64);
    const int max_outer = fp64 ? 4 : 30;
    const double inner_tol = h->cfg.solver.inner_tol > 0 ? h->cfg.solver.inner_tol : 1e-4;
    // FP32 multigrid refinement runs with its control on the device: each
    // residual reduction ends the solve or sets the next pass's target, and
    // every launch after the end returns at once.  The host launches, ahead
    // of its first read, the passes the last solve needed, each with the
    // Krylov iterations that pass took then (a pass cut short leaves more to
    // the next), and continues pass by pass (reading after each) only if the
    // solve is not finished.
    const bool dev = method == PIC_SOLVE_IR_MG;
    int harvested = 0;
    int total = 0, outer = 0, err = 0;
    double rel = 0.0;
    hipLaunchKernelGGL(k_begin_solve, dim3(1), dim3(1), 0, st, h->sc);
    auto residual = [&]() {
        hipLaunchKernelGGL(k_resid64, dim3(kRedBlocks), dim3(256), 0, st, (const double*)h->ar, (const double*)h->az,
                           (const int8_t*)h->node_kind, Q, (const double*)phi, Up, h->r64, h->part, h->nr, h->nz,
                           (const DevScalars*)h->sc);
        hipLaunchKernelGGL(k_reduce_resid, dim3(1), dim3(256), 0, st, (const double*)h->part, h->sc,
                           (const DevCounters*)h->ctr, tol, fp64, dev ? 1 : 0, inner_tol, max_outer);
    };
    // one FP32 pass of refinement: scaled residual, inner solve, update
    auto pass32 = [&](int max_iter, int first_check, bool host_check) {
        hipLaunchKernelGGL(k_scale_to<float>, grid_for(nn), dim3(256), 0, st, (const double*)h->r64, h->r32, h->x32,
                           (const DevScalars*)h->sc, nn);
        const int its = pcg<float>(h, h->r32, h->x32, h->z32, h->p32, h->q32, max_iter, &err,
                                   method == PIC_SOLVE_IR_CG ? 1 : 0, first_check, true, host_check);
        hipLaunchKernelGGL(k_add_phi<float>, grid_for(nn), dim3(256), 0, st, phi, (const float*)h->x32,
                           (const int8_t*)h->node_kind, h->sc, nn, 1);
        return its;
    };
    const int spec = dev ? h->ir_passes : 0;
    for (int k = 0; k < spec; ++k) {
        residual();
        pass32(std::min(h->cfg.solver.max_iter, h->cg_guess[0][std::min(k, 3)]), 0, false);
    }
    for (outer = spec;; ++outer) {
        residual();
        if (!read_scalars(h)) return PIC_E_HIP;
        rel = h->h_sc->relres;
        if (h->h_sc->nonfinite) { err = PIC_E_NONFINITE; break; }
        if (dev ? h->h_sc->outer_done != 0 : (rel <= tol || outer >= max_outer)) break;
        if (fp64) {
            h->harvesting = harvest && outer == 0;
            h->harvest_limit = std::min(unet::kHarvestPerSolve, h->net.cap_pairs);
            int& guess = h->cg_guess[1][std::min(outer, 3)];
            const int its = pcg<double>(h, h->r64, h->x64, h->z64, h->p64, h->q64, h->cfg.solver.max_iter, &err, 0,
                                        guess);
            guess = std::max(1, its);
            total += its;
            if (h->harvesting && !err && its > 0) {
                // iterates 0 .. its-2: the last two are too close to x* for
                // x* - x_k to be an accurate error
                harvested = std::min(std::max(its - 1, 1), h->harvest_limit);
                for (int k = 0; k < harvested; ++k)
                    unet::pair_finish(h->net, (int)((h->net.n_pairs + k) % h->net.cap_pairs), h->x64,
                                      h->hx64 + (size_t)k * nn, h->node_kind, h->w, (double)h->img_free, h->part, st);
            }
            h->harvesting = false;
            hipLaunchKernelGGL(k_add_phi<double>, grid_for(nn), dim3(256), 0, st, phi, (const double*)h->x64,
                               (const int8_t*)h->node_kind, h->sc, nn, 0);
        } else if (dev) {
            // (the reduction has set the target)
            pass32(h->cfg.solver.max_iter, h->cg_guess[0][std::min(outer, 3)], true);
        } else {
            // the inner solve reduces its residual by inner_tol, or by no more
            // than the outer tolerance still needs (with a factor 2 margin)
            const double want = std::max(inner_tol, 0.5 * tol / rel);
            hipLaunchKernelGGL(k_set_target, dim3(1), dim3(1), 0, st, h->sc, want * want);
            if (method == PIC_SOLVE_IR_UNET && h->unet_off) method = PIC_SOLVE_IR_MG;
            if (method == PIC_SOLVE_IR_UNET) {
                hipLaunchKernelGGL(k_scale_to<float>, grid_for(nn), dim3(256), 0, st, (const double*)h->r64, h->r32,
                                   h->x32, (const DevScalars*)h->sc, nn);
                // the network may take at most twice (plus two) the iterations
                // multigrid needed for this pass last time; a network that
                // cannot keep up gives the solve back to multigrid, and one
                // that fails three solves in a row is switched off until new
                // parameters are set or trained
                const int mg = h->cg_guess[0][std::min(outer, 3)];
                const int cap = mg > 0 ? std::min(h->cfg.solver.max_iter, 2 * mg + 2) : h->cfg.solver.max_iter;
                total += fpcg(h, h->r32, h->x32, h->z32, h->p32, h->q32, cap, &err);
                // the correction found so far is kept; multigrid finishes the solve
                if (h->h_sc->fallback) {
                    method = PIC_SOLVE_IR_MG;
                    h->unet_fallbacks++;
                    if (++h->unet_strikes >= 3) h->unet_off = true;
                } else {
                    h->unet_strikes = 0;
                }
                hipLaunchKernelGGL(k_add_phi<float>, grid_for(nn), dim3(256), 0, st, phi, (const float*)h->x32,
                                   (const int8_t*)h->node_kind, h->sc, nn, 1);
            } else {
                int& guess = h->cg_guess[0][std::min(outer, 3)];
                const int its = pass32(h->cfg.solver.max_iter, guess, true);
                guess = std::max(1, its);
                total += its;
            }
        }
        if (err) break;
    }
    if (dev) {
        // what the device did: passes, iterations in all and per pass (the
        // guesses of the next solve)
        const DevScalars& hs = *h->h_sc;
        outer = std::max(hs.outer - 1, 0);
        total = hs.iters_total;
        for (int k = 0; k < std::min(outer, 4); ++k) h->cg_guess[0][k] = std::max(1, hs.its_pass[k]);
        h->ir_passes = err ? 0 : outer;
    }
    hipLaunchKernelGGL(k_set_dirichlet, grid_for(nn), dim3(256), 0, st, phi, (const int8_t*)h->node_kind, Up, nn,
                       h->sc);
    if (harvested > 0 && !err && rel <= tol) h->net.n_pairs += harvested;
    h->solver_outer = outer;
    if (iters_out) *iters_out = total;
    if (relres_out) *relres_out = rel;
    if (err) return err;
    return rel <= tol ? PIC_OK : PIC_E_SOLVER;
}

// ---------------------------------------------------- Laplace and C_eq
// partial sums of the energy bilinear form sum over edges a (d f)(d g)
__global__ __launch_bounds__(256) void k_ceq_part(const double* ar, const double* az, const double* f,
                                                  const double* g, double* part, int nr, int nz) {
    __shared__ double sh[4];
    const int w = nr + 1, nn = w * (nz + 1);
    double acc = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += gridDim.x * blockDim.x) {
        const int i = n % w, j = n / w;
        if (i < nr) { double d = f[n] - f[n + 1], d2 = g[n] - g[n + 1]; acc += ar[n] * d * d2; }
        if (j < nz) { double d = f[n] - f[n + w], d2 = g[n] - g[n + w]; acc += az[n] * d * d2; }
    }
    double t = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_ceq_final(const double* part, DevScalars* s, int e, int f) {
    __shared__ double a[kRedBlocks];
    for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) a[i] = part[i];
    __syncthreads();
    for (int o = kRedBlocks / 2; o > 0; o >>= 1) {
        for (int i = threadIdx.x; i < o; i += blockDim.x) a[i] += a[i + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        s->Cm[e][f] = a[0];
        s->Cm[f][e] = a[0];
    }
}

// Once per RF period (Sec. 2, text after Eq. 4): rebuild the multigrid
// hierarchy for the current operator, solve the Laplace problem of each
// driven electrode (it at 1 V, every other conductor at 0), and the
// capacitance matrix C_ef = sum over edges of a (d phi_Le)(d phi_Lf), the
// field energy's bilinear form (C_11 = C_eq of Eqs. 6-7).
constexpr double kLaplaceAccept = 1e-9;

int refresh_laplace(pic_handle* h) {
    mg_rebuild(h);
    for (int e = 0; e < h->n_el; ++e) {
        int32_t it;
        double rel;
        int rc = field_solve(h, h->phiL[e], nullptr, h->sc->unit[e], 1e-12, PIC_SOLVE_MGPCG_FP64, &it, &rel);
        // the solve asks for 1e-12 and accepts reaching 1e-9 within its
        // iteration limit: C_eq is quadratic in phi_L, its error stays below
        // 1e-9 relative; a Laplace solve that stops above that is an error
        if (rc == PIC_E_SOLVER && rel <= kLaplaceAccept) rc = PIC_OK;
        if (rc != PIC_OK) return rc;
    }
    for (int e = 0; e < h->n_el; ++e)
        for (int f = e; f < h->n_el; ++f) {
            hipLaunchKernelGGL(k_ceq_part, dim3(kRedBlocks), dim3(256), 0, h->stream, (const double*)h->ar,
                               (const double*)h->az, (const double*)h->phiL[e], (const double*)h->phiL[f], h->part,
                               h->nr, h->nz);
            hipLaunchKernelGGL(k_ceq_final, dim3(1), dim3(256), 0, h->stream, (const double*)h->part, h->sc, e, f);
        }
    return PIC_OK;
}

// -------------------------------------------------------------- E field
// E = -grad phi at nodes: centred inside, one-sided on the z edges and at
// r = R, E_r = 0 on the axis.
__global__ __launch_bounds__(256) void k_efield(const double* phi, float2* E, int nr, int nz, double inv_dr,
                                                double inv_dz) {
    const int w = nr + 1, nn = w * (nz + 1);
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += gridDim.x * blockDim.x) {
        const int i = n % w, j = n / w;
        double er, ez;
        if (i == 0) er = 0.0;
        else if (i == nr) er = -(phi[n] - phi[n - 1]) * inv_dr;
        else er = -(phi[n + 1] - phi[n - 1]) * 0.5 * inv_dr;
        if (j == 0) ez = -(phi[n + w] - phi[n]) * inv_dz;
        else if (j == nz) ez = -(phi[n] - phi[n - w]) * inv_dz;
        else ez = -(phi[n + w] - phi[n - w]) * 0.5 * inv_dz;
        E[n] = make_float2((float)er, (float)ez);
    }
}

void launch_efield(pic_handle* h) {
    hipLaunchKernelGGL(k_efield, dim3(1024), dim3(256), 0, h->stream, (const double*)h->phi, h->E, h->nr, h->nz,
                       1.0 / h->dr, 1.0 / h->dz);
}

struct RollArgs {
    unsigned long long *pe, *pi, *le, *li;
    const double *sU, *sI, *sV, *s1;
    double *lU, *lI, *lV, *l1;
    DevScalars* sc;
    int nn, spp;
};

__global__ __launch_bounds__(256) void k_period_roll(RollArgs a) {
    const int total = a.nn > a.spp ? a.nn : a.spp;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < total; n += gridDim.x * blockDim.x) {
        if (n < a.nn) {
            a.le[n] = a.pe[n]; a.li[n] = a.pi[n];
            a.pe[n] = 0ull; a.pi[n] = 0ull;
        }
        if (n < a.spp) {
            for (int e = 0; e < kMaxEl; ++e) {
                a.lU[e * a.spp + n] = a.sU[e * a.spp + n];
                a.lI[e * a.spp + n] = a.sI[e * a.spp + n];
            }
            a.lV[n] = a.sV[n];
            a.l1[n] = a.s1[n];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < 5) {
        a.sc->last_energy[threadIdx.x] = a.sc->energy[threadIdx.x];
        a.sc->energy[threadIdx.x] = 0.0;
    }
}

void launch_period_roll(pic_handle* h) {
    RollArgs a;
    a.pe = h->psum[0]; a.pi = h->psum[1]; a.le = h->plast[0]; a.li = h->plast[1];
    a.sU = h->serU; a.sI = h->serI; a.sV = h->serVin; a.s1 = h->serI1;
    a.lU = h->lastU; a.lI = h->lastI; a.lV = h->lastVin; a.l1 = h->lastI1;
    a.sc = h->sc; a.nn = h->nn; a.spp = h->cfg.run.steps_per_period;
    hipLaunchKernelGGL(k_period_roll, dim3(1024), dim3(256), 0, h->stream, a);
}

}  // namespace pic
