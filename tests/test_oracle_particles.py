"""Pins of the oracle's particle part: the fixed-point cylindrical-volume
deposit, the direct-implicit push and the sort key.  Expected values come
from exact rational arithmetic, conserved moments, closed-form orbits or
library routines, not from the oracle's own formulas."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from pic_inputs import random_particles, workload
from pic_inputs.workloads import CIRC_IDEAL, GROUND, NEUMANN, POWERED

K = 2 ** 32
F = 2 ** 20


def _o(nr=32, nz=24, R=0.05, Z=0.0254, edge_bc=(GROUND, POWERED, GROUND), **run):
    g = dict(nr=nr, nz=nz, R=R, Z=Z, regions=[], edge_bc=list(edge_bc))
    r = dict(n_e=0, n_i=0, cap_e=4096, cap_i=4096)
    r.update(run)
    return O.Oracle(workload("pp32x24", geometry=g, run=r), load=False)


def test_deposit_conserves_charge_exactly():
    o = _o()
    p = random_particles(20000, 0.05, 0.0254, seed=5)
    g = o.deposit(p["r"], p["z"], p["w"])
    expect = sum(int(math.floor(float(w) * K)) for w in p["w"].astype(np.float64))
    assert int(g.sum()) == expect


def test_deposit_on_node_goes_to_that_node():
    o = _o()
    dr, dz = 0.05 / 32, 0.0254 / 24
    for (i, j) in [(0, 1), (5, 7), (31, 23), (12, 1)]:
        r, z = i * dr, j * dz
        # exactly representable node positions only: check the fixed point hit
        g = o.deposit([r], [z], [1.0])
        nz_idx = np.flatnonzero(g)
        q = math.floor(r * (F / dr))
        if q % F == 0 and math.floor(z * (F / dz)) % F == 0:
            assert list(nz_idx) == [j * 33 + i] and g[j * 33 + i] == K


def test_deposit_conserves_r2_and_z_moments():
    # r^2 (volume-fraction) radial weights preserve the r^2 moment and linear
    # axial weights the z moment, up to the floor of each node share.
    o = _o()
    dr, dz = 0.05 / 32, 0.0254 / 24
    p = random_particles(5000, 0.05, 0.0254, seed=6)
    g = o.deposit(p["r"], p["z"], p["w"]).reshape(25, 33).astype(np.float64)
    rn = np.arange(33) * dr
    zn = np.arange(25) * dz
    r = p["r"].astype(np.float64)
    z = p["z"].astype(np.float64)
    W = p["w"].astype(np.float64)
    m_r2 = (g * (rn ** 2)[None, :]).sum()
    m_z = (g * zn[:, None]).sum()
    e_r2 = (W * K * r * r).sum()
    e_z = (W * K * z).sum()
    n = len(r)
    # bounds: floor of the four node shares, plus the 2^-20-cell position
    # quantisation (d(r^2) <= 2 r dr 2^-20, dz <= dz 2^-20)
    q_r2 = (W * K * 2 * r * dr / F).sum()
    q_z = (W * K * dz / F).sum()
    assert abs(m_r2 - e_r2) <= 4 * n * 0.05 ** 2 + q_r2 + 1e-12 * e_r2
    assert abs(m_z - e_z) <= 4 * n * 0.0254 + q_z + 1e-12 * e_z
    # a linear (not volume-fraction) radial weight would miss by ~ W 2^K dr^2/4
    assert (W * K * dr * dr / 4).sum() > 100 * (4 * n * 0.05 ** 2 + q_r2)


def test_deposit_matches_exact_rational_weights():
    # brute force on a tiny grid: each node share is the exact rational
    # volume-fraction weight times W 2^K, to within the floor (<= 3 units).
    o = _o(nr=4, nz=3, R=0.004, Z=0.003)
    dr, dz = Fraction(0.004) / 4, Fraction(0.003) / 3
    p = random_particles(40, 0.004, 0.003, seed=9)
    for k in range(40):
        r, z, W = float(p["r"][k]), float(p["z"][k]), float(p["w"][k])
        g = o.deposit([r], [z], [W]).reshape(4, 5)
        fr, fz = Fraction(r) / dr, Fraction(z) / dz
        i, j = int(fr), int(fz)
        ri, ri1, rr = i * dr, (i + 1) * dr, Fraction(r)
        wr = (rr * rr - ri * ri) / (ri1 * ri1 - ri * ri)
        wz = fz - j
        Wf = Fraction(W) * K
        exact = {(i, j): (1 - wr) * (1 - wz) * Wf, (i + 1, j): wr * (1 - wz) * Wf,
                 (i, j + 1): (1 - wr) * wz * Wf, (i + 1, j + 1): wr * wz * Wf}
        for (a, b), v in exact.items():
            # fixed-point quantisation of the position moves weights by <= 2^-20
            assert abs(int(g[b, a]) - v) <= 3 + Wf * Fraction(4, F)


def test_deposit_is_permutation_invariant():
    o = _o()
    p = random_particles(3000, 0.05, 0.0254, seed=11)
    perm = np.random.default_rng(1).permutation(3000)
    g1 = o.deposit(p["r"], p["z"], p["w"])
    g2 = o.deposit(p["r"][perm], p["z"][perm], p["w"][perm])
    assert np.array_equal(g1, g2)


def test_uniform_volume_loading_gives_uniform_density():
    o = _o(nr=8, nz=6, R=0.05, Z=0.03)
    n = 400000
    p = random_particles(n, 0.05, 0.03, seed=12, wmin=1.0, wmax=1.0)
    g = o.deposit(p["r"], p["z"], p["w"]).astype(np.float64) / K
    V = o.grid("VOL")
    dens = g / V * (0.05 ** 2 * math.pi * 0.03) / n
    # every node, including the axis, within 5 sigma of 1
    counts = g
    sig = 1 / np.sqrt(np.maximum(counts, 1))
    assert np.all(np.abs(dens - 1) <= 5 * sig + 1e-3)


# ----------------------------------------------------------------- push
def _p1(r, z, vr, vt, vz, ar=0.0, at=0.0, az=0.0, w=0.0):
    return {k: np.array([v], dtype=np.float64) for k, v in
            zip(O.FIELDS, (r, z, vr, vt, vz, ar, at, az, w))}


def test_field_free_motion_is_a_straight_line_in_3d():
    o = _o()
    dt = 1.0 / (13.56e6 * 200)
    r0, z0, vr, vt, vz = 0.01, 0.01, 3e4, 5e4, -1e4
    p = _p1(r0, z0, vr, vt, vz)
    zero = np.zeros(1)
    for n in range(1, 60):
        p = o.predict(p)
        t = n * dt
        assert abs(p["r"][0] - math.hypot(r0 + vr * t, vt * t)) <= 1e-15
        assert abs(p["z"][0] - (z0 + vz * t)) <= 1e-15
        v2 = p["vr"][0] ** 2 + p["vt"][0] ** 2 + p["vz"][0] ** 2
        assert abs(v2 - (vr * vr + vt * vt + vz * vz)) <= 1e-12 * v2
        p = o.correct(0, p, zero, zero)


def test_straight_line_through_the_axis():
    o = _o()
    dt = 1.0 / (13.56e6 * 200)
    r0, vr = 0.002, -2e5
    p = _p1(r0, 0.01, vr, 0.0, 0.0)
    zero = np.zeros(1)
    for n in range(1, 40):
        p = o.predict(p)
        p = o.correct(0, p, zero, zero)
        assert abs(p["r"][0] - abs(r0 + vr * n * dt)) <= 1e-15
        # inward (v_r < 0) before the crossing, outward after it
        assert p["vr"][0] * (r0 + vr * n * dt) <= 0
        assert abs(abs(p["vr"][0]) - abs(vr)) <= 1e-9 * abs(vr)


def test_uniform_field_gives_exact_parabola_through_the_whole_step():
    # parallel plates, Neumann side wall: phi is exactly linear in z, E_z
    # uniform; a zero-weight electron follows z(t) = z0 + v0 t + a t^2 / 2.
    U = 100.0
    w = workload("pp32x24",
                 geometry=dict(nr=8, nz=16, R=0.05, Z=0.02, regions=[],
                               edge_bc=[NEUMANN, POWERED, GROUND]),
                 circuit=dict(kind=CIRC_IDEAL, U_amp=0.0, U_dc=U),
                 gas=dict(p_Pa=0.0),
                 run=dict(n_e=0, n_i=0, cap_e=16, cap_i=16, sort_every=0))
    o = O.Oracle(w, load=False)
    dt = o.diag().dt
    qm = -1.602176634e-19 / 9.1093837015e-31
    a = qm * U / 0.02
    z0, v0, r0 = 0.012, 3e5, 0.02
    st = _p1(r0, z0 + dt * v0, 0.0, 0.0, v0, 0.0, 0.0, a, 0.0)
    o.set_particles(0, st)
    for n in range(1, 12):
        o.step(1)
        Ez = o.grid("EZ")
        assert np.allclose(Ez, U / 0.02, rtol=1e-9)
        q = o.particles(0)
        t = n * dt
        z_exact_next = z0 + v0 * (t + dt) + 0.5 * a * (t + dt) ** 2
        assert abs(q["z"][0] + 0.5 * a * dt * dt - z_exact_next) <= 1e-12 * abs(z_exact_next)
        assert abs(q["vz"][0] - (v0 + a * t)) <= 1e-9 * abs(v0 + a * t) + 1e-6
        assert q["r"][0] == pytest.approx(r0, abs=1e-15)


def test_tile_keys_and_stable_sort_against_numpy():
    o = _o(nr=64, nz=48)
    p = random_particles(5000, 0.05, 0.0254, seed=13, dead_frac=0.05)
    keys = o.tile_keys(p["r"], p["z"])
    dr, dz = 0.05 / 64, 0.0254 / 48
    alive = p["r"] >= 0
    i = np.floor(p["r"].astype(np.float64) * (F / dr)).astype(np.int64) >> 20
    j = np.floor(p["z"].astype(np.float64) * (F / dz)).astype(np.int64) >> 20
    expect = np.where(alive, (j >> 4) * 4 + (i >> 4), 0xFFFFFFFF).astype(np.uint32)
    assert np.array_equal(keys, expect)
    assert np.array_equal(O.stable_perm(keys), np.argsort(keys, kind="stable"))


def test_energy_moments_single_particle_and_maxwellian():
    """Energy moment (R31): one particle puts c_k floor(16 eps) on its four
    nodes (eps = m v^2 / 2e from its stored velocity); a Maxwellian load at
    T has mean energy 3T/2 within its statistical error."""
    import math
    w = workload("pp32x24", run=dict(n_e=0, n_i=0, cap_e=10, cap_i=10))
    o = O.Oracle(w, load=False)
    me, qe = 9.1093837015e-31, 1.602176634e-19
    v = (3.0e5, -1.0e5, 2.0e5)
    p = {f: np.zeros(1) for f in ("r", "z", "vr", "vt", "vz", "ar", "at", "az", "w")}
    p["r"][0], p["z"][0], p["w"][0] = 0.013, 0.007, 0.75
    p["vr"][0], p["vt"][0], p["vz"][0] = v
    o.set_particles(0, p)
    N, E = o.moments(0)
    eps = 0.5 * me / qe * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2])
    q = math.floor(eps * 16.0)
    dep = o.deposit(p["r"], p["z"], p["w"])
    assert np.array_equal(N, dep)
    assert np.array_equal(E, dep * q)
    # Maxwellian at 2 eV: <eps> = 3 eV
    w2 = workload("pp32x24", run=dict(n_e=20000, n_i=0, cap_e=20000, cap_i=10, Te_eV=2.0))
    o2 = O.Oracle(w2)
    N2, E2 = o2.moments(0)
    mean = E2.sum() / (16.0 * N2.sum())
    # floor(16 eps) loses 1/32 eV on average; 20k particles: sigma ~ 3 eV sqrt(2/3 / 20000)
    assert abs(mean + 1.0 / 32 - 3.0) < 4 * 3.0 * math.sqrt(2.0 / 3.0 / 20000), mean
