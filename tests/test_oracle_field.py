"""Pins of the oracle's field part: geometry, node volumes, the finite-volume
form of Eq. (1), its solution, and the energy-method equivalent capacitance
(Eqs. 6-7).  Each expected value is a closed form or an independent solver,
never the oracle's own formula retyped."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
from pic_inputs import workload
from pic_inputs.workloads import COND, DIEL, GROUND, NEUMANN, POWERED, gec_geometry

EPS0 = 8.8541878128e-12


def _w(nr, nz, R, Z, regions=(), edge_bc=(GROUND, POWERED, GROUND)):
    g = dict(nr=nr, nz=nz, R=R, Z=Z, regions=list(regions), edge_bc=list(edge_bc))
    return workload("pp32x24", geometry=g, run=dict(n_e=0, n_i=0, cap_e=1, cap_i=1))


def test_total_node_volume_is_cylinder_volume():
    R, Z = 0.05, 0.0254
    o = O.Oracle(_w(32, 24, R, Z), load=False)
    V = o.grid("VOL")
    assert abs(V.sum() - math.pi * R * R * Z) <= 1e-14 * math.pi * R * R * Z


def test_uniform_density_is_uniform_on_nodes_in_expectation():
    # A particle uniform in a cell's volume sends each radial node half of the
    # cell's volume-count with r^2 weights: node volumes must equal the
    # expected share.  Checked by exact quadrature of the weight over the cell
    # (closed form: integral of (r^2-r_i^2)/(r_{i+1}^2-r_i^2) 2 pi r dr).
    R, Z, nr, nz = 0.05, 0.02, 8, 4
    o = O.Oracle(_w(nr, nz, R, Z), load=False)
    V = o.grid("VOL").reshape(nz + 1, nr + 1)
    dr, dz = R / nr, Z / nz
    share = np.zeros(nr + 1)
    for i in range(nr):
        a, b = i * dr, (i + 1) * dr
        cellv = math.pi * (b * b - a * a)
        # integral_a^b (r^2 - a^2)/(b^2 - a^2) 2 pi r dr = pi (b^2 - a^2) / 2
        up = math.pi * ((b ** 4 - a ** 4) / 2 - a * a * (b * b - a * a)) / (b * b - a * a)
        share[i + 1] += up
        share[i] += cellv - up
    interior = share * dz
    assert np.allclose(V[1], interior, rtol=1e-13)
    assert np.allclose(V[0], interior / 2, rtol=1e-13)


def test_node_kinds_parallel_plate_corner_goes_to_ground():
    o = O.Oracle(_w(32, 24, 0.05, 0.0254), load=False)
    nk = o.grid("NODE_KIND").reshape(25, 33)
    assert (nk[0, :32] == POWERED).all()
    assert nk[0, 32] == GROUND            # corner between powered plane and grounded wall
    assert (nk[24, :] == GROUND).all() and (nk[:, 32] == GROUND).all()
    assert (nk[1:24, :32] == -1).all()


def test_gec_geometry_nodes():
    w = workload("gec128x256", run=dict(n_e=0, n_i=0, cap_e=1, cap_i=1))
    o = O.Oracle(w, load=False)
    nk = o.grid("NODE_KIND").reshape(257, 129)
    ck = o.grid("CELL_KIND").reshape(256, 128)
    # powered electrode cells i<64, 160<=j<240; dielectric ring 64<=i<72, j>=160
    assert (ck[160:240, :64] == 2 + POWERED).all()
    assert (ck[160:, 64:72] == 1).all() and (ck[240:, :64] == 1).all()
    assert (ck[:96, :64] == 2 + GROUND).all() and (ck[160:, 72:80] == 2 + GROUND).all()
    # no powered node is a lattice neighbour of a grounded node
    pw = nk == POWERED
    gr = nk == GROUND
    assert not (pw[:, :-1] & gr[:, 1:]).any() and not (pw[:, 1:] & gr[:, :-1]).any()
    assert not (pw[:-1, :] & gr[1:, :]).any() and not (pw[1:, :] & gr[:-1, :]).any()


def _fv_control_volume(nr, nz, R, Z):
    dr, dz = R / nr, Z / nz
    i = np.arange(nr + 1)
    rlo = np.where(i > 0, (i - 0.5) * dr, 0.0)
    rhi = np.where(i < nr, (i + 0.5) * dr, R)
    h = np.full(nz + 1, dz)
    h[0] = h[-1] = dz / 2
    return np.outer(h, math.pi * (rhi ** 2 - rlo ** 2)).ravel()


def test_uniform_charge_cylinder_exact():
    # phi = rho0 (R^2 - r^2) / (4 eps0) with grounded r=R and Neumann z ends is
    # reproduced exactly by the discretisation when Q = rho0 x control volume.
    nr, nz, R, Z = 16, 4, 0.05, 0.02
    o = O.Oracle(_w(nr, nz, R, Z, edge_bc=(GROUND, NEUMANN, NEUMANN)), load=False)
    rho0 = 1e-6
    Q = rho0 * _fv_control_volume(nr, nz, R, Z)
    phi, it, rel, rc = o.solve_q(Q, np.zeros(o.nn), 0.0, tol=1e-14)
    r = (np.arange(nr + 1) * (R / nr))[None, :].repeat(nz + 1, 0).ravel()
    exact = rho0 * (R * R - r * r) / (4 * EPS0)
    assert rc == 0
    assert np.max(np.abs(phi - exact)) <= 1e-12 * exact.max()


def _ceq(nr, nz, R, Z, regions=()):
    o = O.Oracle(_w(nr, nz, R, Z, regions, edge_bc=(NEUMANN, POWERED, GROUND)), load=False)
    return o, o.diag().C_eq


def test_parallel_plate_capacitance_exact():
    R, d = 0.05, 0.0254
    o, C = _ceq(8, 6, R, d)
    assert abs(C - EPS0 * math.pi * R * R / d) <= 1e-13 * C


def test_layered_dielectric_capacitance_exact():
    R, d = 0.05, 0.03
    nz = 12
    d2 = d * 4 / nz                   # dielectric layer on the 4 cells next to z=Z
    regions = [(0.0, 1.0, d - d2, 1.0, DIEL, -1, 4.0)]
    o, C = _ceq(6, nz, R, d, regions)
    exact = EPS0 * math.pi * R * R / ((d - d2) + d2 / 4.0)
    assert abs(C - exact) <= 1e-12 * exact


def test_energy_equals_electrode_flux():
    w = workload("gec128x256", run=dict(n_e=0, n_i=0, cap_e=1, cap_i=1))
    o = O.Oracle(w, load=False)
    C = o.diag().C_eq
    assert abs(C - o.ceq_flux()) <= 1e-9 * C
    assert 50e-12 < C < 500e-12


@pytest.mark.parametrize("n", [16, 32, 64])
def test_coaxial_capacitance_converges(n):
    # powered rod r <= a on the axis, grounded r = R, Neumann z ends:
    # C = 2 pi eps0 L / ln(R/a), second order in h.
    R, L = 0.04, 0.01
    a = R / 4
    regions = [(0.0, a, 0.0, 1.0, COND, POWERED, 1.0)]
    o = O.Oracle(_w(n, 4, R, L, regions, edge_bc=(GROUND, NEUMANN, NEUMANN)), load=False)
    C = o.diag().C_eq
    exact = 2 * math.pi * EPS0 * L / math.log(R / a)
    err = abs(C - exact) / exact
    # midpoint-rule error of sum (dr / r_{i+1/2}) vs ln(R/a): (dr/a)^2 / 24 bound
    h = R / n
    assert err <= 0.5 * (h / a) ** 2


def _assemble_scipy(o):
    """K on the unknown nodes from the oracle's face coefficients, plus b."""
    nr, nz = o.nr, o.nz
    ar, az = o.grid("AR"), o.grid("AZ")
    nk = o.grid("NODE_KIND")
    w = nr + 1
    free = np.flatnonzero(nk < 0)
    idx = -np.ones(o.nn, dtype=np.int64)
    idx[free] = np.arange(len(free))
    rows, cols, vals = [], [], []
    for n in range(o.nn):
        i, j = n % w, n // w
        for m, a in ((n + 1, ar[n] if i < nr else 0.0), (n + w, az[n] if j < nz else 0.0)):
            if a == 0.0:
                continue
            for p, q in ((n, m), (m, n)):
                if idx[p] >= 0:
                    rows.append(idx[p]); cols.append(idx[p]); vals.append(a)
                    if idx[q] >= 0:
                        rows.append(idx[p]); cols.append(idx[q]); vals.append(-a)
    K = sp.csr_matrix((vals, (rows, cols)), shape=(len(free), len(free)))
    return K, free, idx


def test_solver_matches_direct_sparse_solve_with_chi_and_dielectric():
    w = workload("gec128x256", geometry=gec_geometry(1), run=dict(n_e=0, n_i=0, cap_e=1, cap_i=1))
    w["geometry"]["nr"], w["geometry"]["nz"] = 32, 64   # coarse GEC-shaped grid
    o = O.Oracle(w, load=False)
    rng = np.random.default_rng(3)
    chi = rng.uniform(0, 2.0, o.nn)
    Q = rng.normal(0, 1e-13, o.nn)
    U = 37.5
    phi, it, rel, rc = o.solve_q(Q, chi, U, tol=1e-13)
    assert rc == 0 and rel <= 1e-13
    # rebuild K(chi) independently from the geometry-only faces x (1 + mean chi)
    o0 = O.Oracle(w, load=False)
    ar0, az0 = o0.grid("AR"), o0.grid("AZ")     # chi = 0 faces
    nk = o.grid("NODE_KIND")
    nr, nz, W = o.nr, o.nz, o.nr + 1
    ar = ar0 * (1 + 0.5 * (chi + np.roll(chi, -1)))
    az = az0 * (1 + 0.5 * (chi + np.roll(chi, -W)))
    free = np.flatnonzero(nk < 0)
    idx = -np.ones(o.nn, dtype=np.int64)
    idx[free] = np.arange(len(free))
    dir_val = np.where(nk == POWERED, U, 0.0)
    rows, cols, vals = [], [], []
    b = Q[free].copy()
    for n in range(o.nn):
        i, j = n % W, n // W
        for m, a in ((n + 1, ar[n] if i < nr else 0.0), (n + W, az[n] if j < nz else 0.0)):
            if a == 0.0:
                continue
            for p, q in ((n, m), (m, n)):
                if idx[p] < 0:
                    continue
                rows.append(idx[p]); cols.append(idx[p]); vals.append(a)
                if idx[q] >= 0:
                    rows.append(idx[p]); cols.append(idx[q]); vals.append(-a)
                else:
                    b[idx[p]] += a * dir_val[q]
    K = sp.csr_matrix((vals, (rows, cols)), shape=(len(free), len(free)))
    x = spla.spsolve(K.tocsc(), b)
    assert np.max(np.abs(phi[free] - x)) <= 1e-9 * np.max(np.abs(x))
    assert np.allclose(phi[nk == POWERED], U) and np.all(phi[nk == GROUND] == 0.0)


def test_operator_is_symmetric_m_matrix():
    w = workload("gec128x256", run=dict(n_e=0, n_i=0, cap_e=1, cap_i=1))
    w["geometry"]["nr"], w["geometry"]["nz"] = 32, 64
    o = O.Oracle(w, load=False)
    K, free, idx = _assemble_scipy(o)
    assert abs(K - K.T).max() == 0.0
    off = K - sp.diags(K.diagonal())
    assert off.max() <= 0.0
    # row sums >= 0, > 0 somewhere (Dirichlet coupling) => SPD after elimination
    rs = np.asarray(K.sum(axis=1)).ravel()
    assert rs.min() >= -1e-12 * K.diagonal().max() and rs.max() > 0
    ev = spla.eigsh(K, k=1, which="SA", return_eigenvectors=False)
    assert ev[0] > 0
