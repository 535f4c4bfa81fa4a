// pic_device.h -- device-side building blocks of the r-z implicit PIC/MCC
// hot path for gfx950 (arXiv 2310.04957, Sec. 2): fixed-point locate and
// cylindrical-volume deposit weights, the D1 direct-implicit push in local
// (r, theta, z) frames, Philox4x32-10 streams and the null-collision e-Ar /
// Ar+-Ar kinematics.  All particle arithmetic is FP32 except the integer
// deposit definition, which is exact FP64 + int64 by construction.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr int kFBits = 20;        // fraction bits of a fixed-point position (per cell)
constexpr int kKBits = 32;        // fraction bits of a deposited weight
constexpr int kTileShift = 4;     // sort / LDS tiles of 16 x 16 cells
constexpr int kTile = 1 << kTileShift;
constexpr int kVacWords = 256;    // bitmap of all-vacuum tiles: the first 32 kVacWords tiles
constexpr uint32_t kDeadKey = 0xFFFFFFFFu;

// Geometry as the particle kernels see it.
struct Geo {
    int nr, nz, w;                // cells, nodes per row = nr + 1
    double R, Z, Sr, Sz;          // Sr = 2^F / dr, Sz = 2^F / dz
    float inv_dr, inv_dz;
    const double* invd;           // 2^-2F / (2i + 1), i < nr
    const uint8_t* cell_kind;     // 0 vacuum, 1 dielectric, 2 + id conductor
    const uint32_t* vac_tiles;    // bit t: every cell of tile t is vacuum (tiles < 32 kVacWords)
    int ntr;                      // tiles per row
    const int8_t* node_kind;      // -1 unknown, >= 0 conductor id
    int edge_bc[3];               // r=R, z=0, z=Z
};

struct Loc {
    int inside, edge, i, j;
    uint32_t fr, fz;
};

// Fixed-point position q = floor((double)x * 2^F / dx): cell q >> F,
// fraction q & (2^F - 1).  Outside when !(r < R), !(z > 0), !(z < Z) or
// the cell index leaves the grid; `edge` then names the edge crossed.
// Grids have at most 4096 cells a side, so q < 2^32.
// Written without branches: the products are clamped into the range of the
// conversion, which changes nothing for a position inside the domain.
__device__ __forceinline__ Loc locate(float r, float z, const Geo& g) {
    const double rd = (double)r, zd = (double)z;
    const bool okr = rd < g.R, okz0 = zd > 0.0, okz1 = zd < g.Z;
    const uint32_t qr = (uint32_t)floor(fmin(fmax(rd * g.Sr, 0.0), 4294967295.0));
    const uint32_t qz = (uint32_t)floor(fmin(fmax(zd * g.Sz, 0.0), 4294967295.0));
    const int i = (int)(qr >> kFBits), j = (int)(qz >> kFBits);
    const bool oki = i < g.nr, okj = j < g.nz;
    Loc L;
    L.inside = (okr && okz0 && okz1 && oki && okj) ? 1 : 0;
    L.edge = !okr ? 0 : !okz0 ? 1 : !okz1 ? 2 : !oki ? 0 : 2;
    L.i = L.inside ? i : 0;
    L.j = L.inside ? j : 0;
    L.fr = L.inside ? (qr & ((1u << kFBits) - 1u)) : 0u;
    L.fz = L.inside ? (qz & ((1u << kFBits) - 1u)) : 0u;
    return L;
}

// Integer node shares of a particle of relative weight W, in units of
// 2^-K: radial weight to node i+1 is the volume fraction
// (r^2 - r_i^2)/(r_{i+1}^2 - r_i^2) = (2 i f + f^2)/(2i + 1), axial weights
// linear.  Every product is rounded separately (no contraction), so the
// result is the same on any IEEE machine.  Order: (i,j) (i+1,j) (i,j+1)
// (i+1,j+1); the four sum to floor(W 2^K) exactly.
// invd_i = 2^-2F / (2i + 1) for the particle's column i.
__device__ __forceinline__ void node_shares(const Loc& L, double W, double invd_i, int64_t c[4]) {
#pragma clang fp contract(off)
    const uint64_t nrr = (((uint64_t)(2u * (uint32_t)L.i) * (uint64_t)L.fr) << kFBits) + (uint64_t)L.fr * (uint64_t)L.fr;
    double wr = (double)nrr * invd_i;
    double wrb = 1.0 - wr;
    double wz = (double)L.fz * 0x1p-20;
    double wzb = (double)((1u << kFBits) - L.fz) * 0x1p-20;
    double t;
    t = W * wr; t = t * wz; t = t * 0x1p32;
    int64_t c11 = (int64_t)floor(t);
    t = W * wr; t = t * wzb; t = t * 0x1p32;
    int64_t c10 = (int64_t)floor(t);
    t = W * wrb; t = t * wz; t = t * 0x1p32;
    int64_t c01 = (int64_t)floor(t);
    t = W * 0x1p32;
    int64_t tot = (int64_t)floor(t);
    c[0] = tot - c11 - c10 - c01;
    c[1] = c10;
    c[2] = c01;
    c[3] = c11;
}

__device__ __forceinline__ int64_t total_share(double W) {
#pragma clang fp contract(off)
    double t = W * 0x1p32;
    return (int64_t)floor(t);
}

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11).
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
    // opaque to loop-invariant motion: the twenty round keys are rebuilt
    // with scalar adds at every call instead of occupying scalar registers
    asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        c = make_uint4(n0, (uint32_t)p1, n2, (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// uniform in (0,1), exactly representable: ((x >> 9) + 1/2) 2^-23
__device__ __forceinline__ float u01(uint32_t x) { return ((float)(x >> 9) + 0.5f) * 0x1p-23f; }

enum { kPurposeLoad = 0, kPurposeMcc = 1, kPurposeDecide = 2 };

// The null-collision decision of slot p comes from word (p >> 6) & 3 of the
// draw at this counter: one Philox block serves four slots 64 apart, i.e.
// four consecutive 64-slot rounds of one wavefront.
__device__ __forceinline__ uint32_t decision_ctr(uint32_t p) { return (p & 63u) | ((p >> 8) << 6); }

__device__ __forceinline__ uint4 draw(uint32_t slot, uint32_t step, uint32_t purpose, int sp, uint32_t k,
                                      uint32_t key0, uint32_t key1) {
    return philox4x32_10(make_uint4(slot, step, purpose * 2u + (uint32_t)sp, k), key0, key1);
}

// ------------------------------------------------------------ D1 push
// Particle state between steps: predicted position (r~, z~), the explicit
// velocity v* and the averaged acceleration a_bar, all in the local
// (r, theta, z) frame of the particle.
struct P9 {
    float r, z, vr, vt, vz, ar, at, az, w;
};

// Storage of one species: 36 bytes a slot in three arrays, a = (r~, z~,
// v*_r, v*_theta), b = (v*_z, a_bar_r, a_bar_theta, a_bar_z) and the
// weight w.  A slot read out of order (a sort being applied, splitting)
// touches three memory lines instead of nine; in-order reads and writes
// are 16-byte vector accesses.  Slot indices are 32-bit.
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct Species {
    f32x4* a;
    f32x4* b;
    float* w;
};

__device__ __forceinline__ P9 load9(const Species& S, uint32_t p) {
    const f32x4 x = S.a[p], y = S.b[p];
    P9 s;
    s.r = x.x; s.z = x.y; s.vr = x.z; s.vt = x.w;
    s.vz = y.x; s.ar = y.y; s.at = y.z; s.az = y.w;
    s.w = S.w[p];
    return s;
}

__device__ __forceinline__ f32x4 group_a(const P9& s) { return f32x4{s.r, s.z, s.vr, s.vt}; }
__device__ __forceinline__ f32x4 group_b(const P9& s) { return f32x4{s.vz, s.ar, s.at, s.az}; }

// all nine values (the weight too)
__device__ __forceinline__ void store9(const Species& S, uint32_t p, const P9& s) {
    S.a[p] = group_a(s);
    S.b[p] = group_b(s);
    S.w[p] = s.w;
}

// correct: a = (q/m) E(x~); x = x~ + dt^2/2 a; v = v* + dt/2 a;
// a_bar = (a_bar + a)/2; crossing the axis reflects r, v_r, v_t, a_r, a_t.
__device__ __forceinline__ void d1_correct(P9& p, float Er, float Ez, float qm, float dt) {
    float ar = qm * Er, az = qm * Ez;
    float h2 = 0.5f * dt * dt, h = 0.5f * dt;
    p.r = p.r + h2 * ar;
    p.z = p.z + h2 * az;
    p.vr = p.vr + h * ar;
    p.vz = p.vz + h * az;
    p.ar = 0.5f * (p.ar + ar);
    p.at = 0.5f * p.at;
    p.az = 0.5f * (p.az + az);
    if (p.r < 0.0f) {
        p.r = -p.r;
        p.vr = -p.vr; p.vt = -p.vt;
        p.ar = -p.ar; p.at = -p.at;
    }
}

// predict: v* = v + dt/2 a_bar; straight Cartesian move; rotate v* and
// a_bar into the new local frame.
__device__ __forceinline__ void d1_predict(P9& p, float dt) {
    float h = 0.5f * dt;
    float vr = p.vr + h * p.ar, vt = p.vt + h * p.at, vz = p.vz + h * p.az;
    float X = p.r + dt * vr, Y = dt * vt;
    // |(X, Y)| and the rotation from one reciprocal square root; below
    // 2^-50 m the particle is taken to sit on the axis
    const float rr = X * X + Y * Y;
    float rn = 0.0f, c = 1.0f, s = 0.0f;
    if (rr > 0x1p-100f) {
        const float inv = __builtin_amdgcn_rsqf(rr);
        rn = rr * inv;
        c = X * inv;
        s = Y * inv;
    }
    p.r = rn;
    p.z = p.z + dt * vz;
    p.vr = c * vr + s * vt;
    p.vt = -s * vr + c * vt;
    p.vz = vz;
    float ar = p.ar, at = p.at;
    p.ar = c * ar + s * at;
    p.at = -s * ar + c * at;
}

// Gather of E at a position with the cylindrical-volume weights (FP32):
// the cell (i, j) and the weights of its nodes (i,j) (i+1,j) (i,j+1)
// (i+1,j+1).
struct EW {
    int i, j;
    float a0, a1, a2, a3;
};

__device__ __forceinline__ EW e_weights(const Geo& g, float r, float z) {
    EW e;
    const float x = r * g.inv_dr, y = z * g.inv_dz;
    e.i = min(max((int)x, 0), g.nr - 1);
    e.j = min(max((int)y, 0), g.nz - 1);
    const float f = fminf(fmaxf(x - (float)e.i, 0.0f), 1.0f);
    const float gz = fminf(fmaxf(y - (float)e.j, 0.0f), 1.0f);
    const float fi = (float)e.i;
    const float wr = f * (2.0f * fi + f) * __builtin_amdgcn_rcpf(2.0f * fi + 1.0f);
    e.a0 = (1.0f - wr) * (1.0f - gz);
    e.a1 = wr * (1.0f - gz);
    e.a2 = (1.0f - wr) * gz;
    e.a3 = wr * gz;
    return e;
}

__device__ __forceinline__ void e_combine(const EW& e, float2 e00, float2 e10, float2 e01, float2 e11, float& Er,
                                          float& Ez) {
    Er = e.a0 * e00.x + e.a1 * e10.x + e.a2 * e01.x + e.a3 * e11.x;
    Ez = e.a0 * e00.y + e.a1 * e10.y + e.a2 * e01.y + e.a3 * e11.y;
}

// E from the global node grid
__device__ __forceinline__ void gather_E(const float2* __restrict__ E, const Geo& g, float r, float z,
                                         float& Er, float& Ez) {
    const EW e = e_weights(g, r, z);
    const int n00 = e.j * g.w + e.i;
    e_combine(e, E[n00], E[n00 + 1], E[n00 + g.w], E[n00 + g.w + 1], Er, Ez);
}

// --------------------------------------------------------------- MCC (FP32)
struct Mcc {
    float n_gas, nu_max, vth_gas, half_m_over_e, two_e_over_m, m_ratio2; // m_ratio2 = 2 m_e / M
    uint32_t thresh;
};

__device__ __forceinline__ void xsec_e(float eps, float& el, float& ex, float& io) {
    el = 1.0e-19f / sqrtf(1.0f + eps * 0.1f);
    float xe = eps * (1.0f / 11.5f), xi = eps * (1.0f / 15.76f);
    ex = (eps > 11.5f) ? 2.7e-20f * logf(xe) / xe : 0.0f;
    io = (eps > 15.76f) ? 8.0e-20f * logf(xi) / xi : 0.0f;
}

__device__ __forceinline__ float e_cos_chi(float eps, float u) {
    if (eps < 1e-6f) return 1.0f - 2.0f * u;
    float c = (2.0f + eps - 2.0f * powf(1.0f + eps, u)) / eps;
    return fminf(1.0f, fmaxf(-1.0f, c));
}

// turn unit vector d by polar angle chi (cos cchi) and azimuth 2 pi t
__device__ __forceinline__ void rotate_dir(float& u, float& v, float& w, float cchi, float t) {
    float schi = sqrtf(fmaxf(0.0f, 1.0f - cchi * cchi));
    float sp, cp;
    sincospif(2.0f * t, &sp, &cp);
    float st = sqrtf(u * u + v * v);
    if (st > 1e-12f) {
        float inv = 1.0f / st;
        float nu = u * cchi + schi * (u * w * cp - v * sp) * inv;
        float nv = v * cchi + schi * (v * w * cp + u * sp) * inv;
        float nw = w * cchi - st * schi * cp;
        u = nu; v = nv; w = nw;
    } else {
        u = schi * cp;
        v = schi * sp;
        w = (w >= 0.0f ? 1.0f : -1.0f) * cchi;
    }
}

__device__ __forceinline__ void maxwell3(uint4 y, float vth, float& a, float& b, float& c) {
    float m0 = sqrtf(-2.0f * logf(u01(y.x))), m1 = sqrtf(-2.0f * logf(u01(y.z)));
    float s0, c0, s1, c1;
    sincospif(2.0f * u01(y.y), &s0, &c0);
    sincospif(2.0f * u01(y.w), &s1, &c1);
    a = vth * m0 * c0;
    b = vth * m0 * s0;
    c = vth * m1 * c1;
}

// Outcome codes: 0 elastic / isotropic, 1 excitation / charge exchange,
// 2 ionisation, 3 null.  x is the slot's first collision draw of this step
// (its first word is unused: the decision has its own draw).
__device__ __forceinline__ int collide(int sp, uint4 x, float& vr, float& vt, float& vz, const Mcc& m,
                                      uint32_t slot, uint32_t step, uint32_t key0, uint32_t key1,
                                      float* born6, unsigned int* viol) {
    float u1 = u01(x.y), u2 = u01(x.z), u3 = u01(x.w);
    float R = u1 * m.nu_max;
    if (sp == 0) {
        float v2 = vr * vr + vt * vt + vz * vz;
        float vm = sqrtf(v2);
        if (!(vm > 0.0f)) return 3;
        float eps = m.half_m_over_e * v2;
        float el, ex, io;
        xsec_e(eps, el, ex, io);
        float k = m.n_gas * vm;
        float n_el = k * el, n_ex = k * ex, n_io = k * io;
        float inv = 1.0f / vm;
        float du = vr * inv, dv = vt * inv, dw = vz * inv;
        // the scattered electron of every process: scattering energy e_s
        // (elastic: eps; excitation: eps - 11.5 eV; ionisation: what the
        // ejected electron leaves), then one deflection for all three
        int proc;
        float e_s;
        if (R < n_el) {
            proc = 0;
            e_s = eps;
        } else if (R < n_el + n_ex) {
            proc = 1;
            e_s = eps - 11.5f;
        } else if (R < n_el + n_ex + n_io) {
            proc = 2;
            uint4 y = draw(slot, step, kPurposeMcc, sp, 1, key0, key1);
            uint4 z4 = draw(slot, step, kPurposeMcc, sp, 2, key0, key1);
            float e1 = eps - 15.76f;
            float eej = 10.0f * tanf(u01(y.x) * atanf(e1 * (1.0f / 20.0f)));
            e_s = fmaxf(e1 - eej, 0.0f);
            float bu = du, bv = dv, bw = dw;
            rotate_dir(bu, bv, bw, e_cos_chi(eej, u01(y.y)), u01(y.z));
            float s2 = sqrtf(m.two_e_over_m * eej);
            born6[0] = s2 * bu; born6[1] = s2 * bv; born6[2] = s2 * bw;
            maxwell3(z4, m.vth_gas, born6[3], born6[4], born6[5]);
        } else {
            return 3;
        }
        const float cc = e_cos_chi(e_s, u2);
        const float e_out = proc == 0 ? eps * (1.0f - m.m_ratio2 * (1.0f - cc)) : fmaxf(e_s, 0.0f);
        rotate_dir(du, dv, dw, cc, u3);
        float s = sqrtf(m.two_e_over_m * e_out);
        vr = s * du; vt = s * dv; vz = s * dw;
        return proc;
    }
    // Ar+ on Ar: partner from the gas Maxwellian, relative velocity g
    uint4 y = draw(slot, step, kPurposeMcc, sp, 1, key0, key1);
    float nr_, nt_, nz_;
    maxwell3(y, m.vth_gas, nr_, nt_, nz_);
    float gr = vr - nr_, gt = vt - nt_, gz = vz - nz_;
    float gm = sqrtf(gr * gr + gt * gt + gz * gz);
    float n_iso = m.n_gas * 5.0e-19f * gm, n_cx = n_iso;
    float tot = n_iso + n_cx;
    if (tot > m.nu_max) {
        atomicAdd(viol, 1u);
        float f = m.nu_max / tot;
        n_iso *= f;
        n_cx *= f;
    }
    if (R < n_iso && gm > 0.0f) {
        float cc = sqrtf(1.0f - u2);
        float inv = 1.0f / gm;
        float du = gr * inv, dv = gt * inv, dw = gz * inv;
        rotate_dir(du, dv, dw, cc, u3);
        float gp = gm * cc;
        vr = nr_ + gp * du; vt = nt_ + gp * dv; vz = nz_ + gp * dw;
        return 0;
    }
    if (R < n_iso + n_cx) {
        vr = nr_; vt = nt_; vz = nz_;
        return 1;
    }
    return 3;
}

// staged ionisation birth: parent position and weight, new electron and ion
// velocities
struct Birth {
    float r, z, w, v[6];
};

// sort key of a cell's tile: tile row times kmul plus tile column (kmul at
// least the tiles per row, so keys follow the row-major tile order)
__device__ __forceinline__ uint32_t tile_key(const Loc& L, int kmul) {
    return (uint32_t)((L.j >> kTileShift) * kmul + (L.i >> kTileShift));
}

}  // namespace pic
