"""Pins of the implicit parts of the oracle's step: the D1 averaging of the
acceleration, the susceptibility chi of Eq. (1), the node field E = -grad phi
and the r^2 field gather.  Each expected value comes from a closed form (the
characteristic polynomial of the D1 recurrence, the plasma frequency, the
potential of a uniformly charged cylinder, an exactly interpolated field),
written from the mathematics and not from the oracle's code, and each test
fails on a plausible slip in the oracle (a dropped or mis-weighted average,
a factor 2, a wrong mass or node volume, a sign, linear instead of r^2
weights)."""
import math

import numpy as np

import oracle as O
from pic_inputs import random_particles, workload
from pic_inputs.workloads import GROUND, NEUMANN, POWERED

QE = 1.602176634e-19
ME = 9.1093837015e-31
MAR = 39.948 * 1.66053906660e-27
EPS0 = 8.8541878128e-12


def _o(nr=16, nz=12, R=0.05, Z=0.0254, edge_bc=(GROUND, POWERED, GROUND), **run):
    g = dict(nr=nr, nz=nz, R=R, Z=Z, regions=[], edge_bc=list(edge_bc))
    r = dict(n_e=0, n_i=0, cap_e=16, cap_i=16)
    r.update(run)
    return O.Oracle(workload("pp32x24", geometry=g, run=r), load=False)


def _one(r, z, vr=0.0, vt=0.0, vz=0.0, ar=0.0, at=0.0, az=0.0):
    return {k: np.array([v], dtype=np.float64) for k, v in
            zip(O.FIELDS, (r, z, vr, vt, vz, ar, at, az, 0.0))}


# ------------------------------------------------------------ D1 averaging
def _d1_orbit(o, axis, Omega, x0, v0, abar0, centre, nsteps):
    """Drive one electron through the oracle's correct/predict pair in the
    linear field a = -omega^2 (x - centre) along `axis` (0: r, 1: z).  The
    field is the implicit one, taken at the corrected position:
    x_{n+1} = x~ + dt^2/2 a_{n+1} with a_{n+1} = -omega^2 x_{n+1}, i.e.
    x_{n+1} = x~ / (1 + Omega^2/2).  Returns the corrected displacements."""
    dt = o.diag().dt
    w2 = (Omega / dt) ** 2
    qm = -QE / ME
    key_x, key_v, key_a = (("r", "vr", "ar"), ("z", "vz", "az"))[axis]
    p = _one(0.02, 0.0127)
    p[key_x][0] = centre + x0
    p[key_v][0] = v0
    p[key_a][0] = abar0
    xs = []
    for _ in range(nsteps):
        xt = p[key_x][0] - centre
        a = -w2 * xt / (1.0 + 0.5 * Omega * Omega)
        E = np.array([a / qm])
        zero = np.zeros(1)
        p = o.correct(0, p, E if axis == 0 else zero, zero if axis == 0 else E)
        xs.append(p[key_x][0] - centre)
        p = o.predict(p)
    return np.array(xs)


def _d1_roots(Omega):
    """Roots of the D1 characteristic polynomial.  With
    x_{n+1} - 2 x_n + x_{n-1} = dt^2 abar_n and
    abar_n = (abar_{n-1} + a_{n+1}) / 2, a_{n+1} = -omega^2 x_{n+1},
    eliminating abar gives (2 + Omega^2) x_{n+1} - 5 x_n + 4 x_{n-1} - x_{n-2} = 0."""
    return np.roots([2.0 + Omega * Omega, -5.0, 4.0, -1.0])


def test_d1_linear_field_follows_the_closed_form_roots():
    o = _o()
    dt = o.diag().dt
    for axis in (0, 1):
        for Omega in (0.05, 0.3, 1.0, 4.0):
            amp = 2e-3
            # abar differs from the field's value at the start: the third
            # (memory) root of the scheme is excited
            abar0 = 0.7 * (Omega / dt) ** 2 * amp
            xs = _d1_orbit(o, axis, Omega, amp, 0.3 * amp / dt, abar0, 0.025 if axis == 0 else 0.0127, 40)
            lam = _d1_roots(Omega)
            # amplitudes of the three modes from the first three samples, then
            # every later sample from the closed form x_n = sum c_k lam_k^n
            n = np.arange(len(xs))
            V = lam[None, :] ** n[:, None]
            c = np.linalg.solve(V[:3], xs[:3].astype(complex))
            pred = (V @ c).real
            assert np.max(np.abs(pred - xs)) <= 1e-11 * amp, (axis, Omega)


def test_d1_roots_are_those_of_the_averaged_scheme_not_leapfrog():
    # the averaged scheme damps the oscillation (|lambda| < 1 for every
    # Omega > 0) and its phase per step tends to Omega; plain leapfrog
    # (abar = a) would keep |lambda| = 1 for Omega < 2.  The oracle's orbit
    # decays at the rate of the complex pair.
    o = _o()
    dt = o.diag().dt
    for Omega in (0.1, 0.3, 1.0, 1.9):
        lam = _d1_roots(Omega)
        pair = lam[np.abs(lam.imag) > 0]
        assert len(pair) == 2 and np.all(np.abs(pair) < 1.0)
    for Omega in (0.2, 0.3):
        pair = [x for x in _d1_roots(Omega) if abs(x.imag) > 0]
        xs = _d1_orbit(o, 1, Omega, 1e-3, 0.0, -(Omega / dt) ** 2 * 1e-3, 0.0127, 400)
        # after the memory root (|lambda| ~ 0.5) has died out, successive
        # periods shrink by |lambda_pair|^period
        peaks = np.abs(xs[200:]).max(), np.abs(xs[300:]).max()
        rate = abs(pair[0]) ** 100
        assert abs(peaks[1] / peaks[0] - rate) <= 0.05 * rate
    small = _d1_roots(0.05)
    ph = np.abs(np.angle(small[np.abs(small.imag) > 0]))
    assert np.allclose(ph, 0.05, rtol=5e-3)


def test_d1_large_omega_dt_is_damped_not_unstable():
    # the point of the implicit push: omega dt >> 1 stays bounded and decays
    o = _o()
    dt = o.diag().dt
    xs = _d1_orbit(o, 1, 10.0, 1e-3, 0.0, 0.0, 0.0127, 30)
    assert np.all(np.abs(xs) <= 1e-3) and abs(xs[-1]) < 1e-6


# ------------------------------------------------------------ susceptibility
def _node_volumes(nr, nz, R, Z):
    """Volumes of the r^2-weighted deposit's nodes: the volume a uniform
    density assigns to each node.  Interior column i: pi dz (r_{i+1}^2 -
    r_{i-1}^2)/2; axis: pi dr^2 dz/2; r = R: pi dz (R^2 - r_{N-1}^2)/2;
    halved on the z edges."""
    dr, dz = R / nr, Z / nz
    r = np.arange(nr + 1) * dr
    col = np.empty(nr + 1)
    col[1:nr] = math.pi * (r[2:] ** 2 - r[:-2] ** 2) / 2
    col[0] = math.pi * dr * dr / 2
    col[nr] = math.pi * (R * R - r[nr - 1] ** 2) / 2
    h = np.full(nz + 1, dz)
    h[0] = h[-1] = dz / 2
    return np.outer(h, col).ravel()


def test_chi_is_half_the_squared_plasma_frequency_times_dt_squared():
    nr, nz, R, Z = 16, 12, 0.05, 0.0254
    o = _o(nr, nz, R, Z, n_e=2 ** 30)
    d = o.diag()
    dt, unit = d.dt, d.w_unit * 2.0 ** -32
    V = _node_volumes(nr, nz, R, Z)
    ne, ni = 1.0e15, 3.0e15               # different densities: a swapped mass shows
    Ne = np.rint(ne * V / unit).astype(np.int64)
    Ni = np.rint(ni * V / unit).astype(np.int64)
    assert Ne.min() > 2 ** 40            # integer rounding below 1e-12
    wq = np.zeros(o.nn, dtype=np.int64)
    wq[5] = 12345
    o.set_grid("DEP_E", Ne)
    o.set_grid("DEP_I", Ni)
    o.set_grid("WALLQ", wq)
    o.assemble_now()
    chi = o.grid("CHI")
    wpe2 = ne * QE * QE / (ME * EPS0)
    wpi2 = ni * QE * QE / (MAR * EPS0)
    expect = 0.5 * dt * dt * (wpe2 + wpi2)
    # every node, the axis and the domain edges included
    assert np.max(np.abs(chi - expect)) <= 1e-11 * expect
    # the ion term is visible at this bar (a wrong ion mass fails)
    assert 0.5 * dt * dt * wpi2 > 1e-6 * expect
    Q = o.grid("Q")
    assert np.allclose(Q, QE * unit * (Ni - Ne + wq), rtol=1e-14, atol=0)


def test_uniform_chi_scales_the_cylinder_potential_by_one_over_one_plus_chi():
    # Eq. (1) with a uniform susceptibility: div((1 + chi) eps0 grad phi) =
    # -rho gives phi = rho0 (R^2 - r^2) / (4 eps0 (1 + chi)).  chi comes from
    # a uniform deposit (uniform on every node), so this pins the (1 + chi)
    # of both face coefficients together with the assembly.
    nr, nz, R, Z = 16, 4, 0.05, 0.02
    o = _o(nr, nz, R, Z, edge_bc=(GROUND, NEUMANN, NEUMANN), n_e=2 ** 30)
    unit = o.diag().w_unit * 2.0 ** -32
    V = _node_volumes(nr, nz, R, Z)
    o.set_grid("DEP_E", np.rint(4e15 * V / unit).astype(np.int64))
    o.set_grid("DEP_I", np.zeros(o.nn, dtype=np.int64))
    o.assemble_now()
    chi = o.grid("CHI")
    c = float(chi.mean())
    assert np.max(np.abs(chi - c)) <= 1e-11 * c and c > 0.1
    # control volumes of the finite-volume form of Eq. (1)
    dr, dz = R / nr, Z / nz
    i = np.arange(nr + 1)
    rlo = np.where(i > 0, (i - 0.5) * dr, 0.0)
    rhi = np.where(i < nr, (i + 0.5) * dr, R)
    h = np.full(nz + 1, dz)
    h[0] = h[-1] = dz / 2
    rho0 = 1e-6
    Q = rho0 * np.outer(h, math.pi * (rhi ** 2 - rlo ** 2)).ravel()
    phi, it, rel, rc = o.solve_q(Q, chi, 0.0, tol=1e-14)
    r = np.tile(np.arange(nr + 1) * dr, nz + 1)
    exact = rho0 * (R * R - r * r) / (4 * EPS0 * (1 + c))
    assert rc == 0
    assert np.max(np.abs(phi - exact)) <= 1e-11 * exact.max()


# ------------------------------------------------------------ field and gather
def test_node_field_of_the_uniformly_charged_cylinder():
    # phi = rho0 (R^2 - r^2)/(4 eps0) + g z: E_r = rho0 r / (2 eps0) outward
    # (positive) at every node off the axis and r = R, 0 on the axis;
    # E_z = -g everywhere (one-sided differences on the z edges are exact
    # for a linear potential).
    nr, nz, R, Z = 32, 24, 0.05, 0.0254
    o = _o(nr, nz, R, Z)
    rho0, g = 2e-6, 350.0
    r = np.tile(np.arange(nr + 1) * (R / nr), nz + 1)
    z = np.repeat(np.arange(nz + 1) * (Z / nz), nr + 1)
    o.set_grid("PHI", rho0 * (R * R - r * r) / (4 * EPS0) + g * z)
    o.efield_now()
    Er = o.grid("ER").reshape(nz + 1, nr + 1)
    Ez = o.grid("EZ")
    exact = (rho0 * r / (2 * EPS0)).reshape(nz + 1, nr + 1)
    scale = exact.max()
    assert np.max(np.abs(Er[:, 1:nr] - exact[:, 1:nr])) <= 1e-10 * scale
    assert np.all(Er[:, 1:nr] > 0)
    assert np.all(Er[:, 0] == 0.0)
    assert np.max(np.abs(Ez + g)) <= 1e-9 * g


def test_gather_is_exact_for_a_field_linear_in_r_squared_and_z():
    # The r^2 (volume-fraction) weights interpolate r^2 exactly, the axial
    # ones z exactly: node fields c r^2 + e z and d z + f are gathered as
    # their values at the particle, up to the 2^-20-cell fixed-point position.
    nr, nz, R, Z = 32, 24, 0.05, 0.0254
    o = _o(nr, nz, R, Z)
    dr, dz = R / nr, Z / nz
    cr, er, dzc, fz = 3.0e6, -4.0e3, 7.0e4, 11.0
    rn = np.tile(np.arange(nr + 1) * dr, nz + 1)
    zn = np.repeat(np.arange(nz + 1) * dz, nr + 1)
    o.set_grid("ER", cr * rn * rn + er * zn)
    o.set_grid("EZ", dzc * zn + fz)
    p = random_particles(5000, R, Z, seed=21)
    r, z = p["r"].astype(np.float64), p["z"].astype(np.float64)
    Er, Ez = o.gather(r, z)
    qr = cr * 2 * r * dr * 2.0 ** -20 + abs(er) * dz * 2.0 ** -20
    assert np.all(np.abs(Er - (cr * r * r + er * z)) <= qr + 1e-12 * cr * R * R)
    assert np.all(np.abs(Ez - (dzc * z + fz)) <= dzc * dz * 2.0 ** -20 + 1e-12 * dzc * Z)
    # linear radial weights would be off by cr dr^2 f(1 - f): far above the bar
    f = r / dr - np.floor(r / dr)
    assert np.median(cr * dr * dr * f * (1 - f)) > 1000 * np.median(qr)
