"""Pins of the oracle with several driven electrodes (reading R33: one Laplace
solution per electrode, the capacitance matrix from the field energy, the
circuits coupled through Q = C U + Q_P).

Expected values: the closed-form capacitance of two plates, the flux form of
the same matrix (a discrete Green identity, computed here from the face
coefficients), linear superposition, exact DFTs of ideal sources, a phasor
solution of a series RLC branch coupled to a second electrode, and exact
integer charge conservation."""
import cmath
import math

import numpy as np
import pytest

import oracle as O
from pic_inputs import workload
from pic_inputs.workloads import CIRC_IDEAL, CIRC_SERIES_RLC, NEUMANN, _circuit

EPS0 = 8.8541878128e-12
K = 2 ** 32


def _fundamental(x, k=1):
    n = len(x)
    return 2.0 / n * np.sum(x * np.exp(-2j * np.pi * k * np.arange(n) / n))


def _vac(w):
    w["run"].update(n_e=0, n_i=0, cap_e=1, cap_i=1)
    return O.Oracle(w, load=False)


def test_two_plates_closed_form():
    """Plates z=0 (electrode 1) and z=Z (electrode 2), Neumann wall: the
    field is exactly linear, C = eps0 pi R^2 / Z [[1, -1], [-1, 1]]."""
    R, Z = 0.05, 0.0254
    w = workload("pp32x24", geometry=dict(regions=[], edge_bc=[NEUMANN, 1, 2]))
    w["circuits_more"] = [_circuit(CIRC_IDEAL)]
    C = _vac(w).capacitance()
    c0 = EPS0 * math.pi * R * R / Z
    assert np.max(np.abs(C - c0 * np.array([[1, -1], [-1, 1]]))) <= 1e-9 * c0


def _flux_matrix(o, m):
    ar, az, nk = o.grid("AR"), o.grid("AZ"), o.grid("NODE_KIND")
    nr, nz = o.nr, o.nz
    w = nr + 1
    F = np.zeros((m, m))
    for f in range(m):
        L = o.phi_laplace(f + 1)
        net = np.zeros(o.nn)
        idx = np.arange(o.nn)
        i, j = idx % w, idx // w
        net[i > 0] += ar[idx[i > 0] - 1] * (L[i > 0] - L[idx[i > 0] - 1])
        net[i < nr] += ar[idx[i < nr]] * (L[i < nr] - L[idx[i < nr] + 1])
        net[j > 0] += az[idx[j > 0] - w] * (L[j > 0] - L[idx[j > 0] - w])
        net[j < nz] += az[idx[j < nz]] * (L[j < nz] - L[idx[j < nz] + w])
        for e in range(m):
            F[e, f] = net[nk == e + 1].sum()
    return F


def test_energy_and_flux_capacitance_agree():
    """The energy bilinear form equals the charge each electrode carries
    (net flux out of its nodes) with another electrode at 1 V; the matrix is
    symmetric positive definite, mutual terms negative, rows dominant."""
    o = _vac(workload("pp32x24x2"))
    C = o.capacitance()
    F = _flux_matrix(o, 2)
    assert np.max(np.abs(F - C)) <= 1e-8 * np.max(np.abs(C))
    assert np.array_equal(C, C.T)
    assert np.all(np.linalg.eigvalsh(C) > 0)
    assert C[0, 1] < 0 and C.sum(axis=1).min() > 0


def test_superposition_of_electrode_potentials():
    o = _vac(workload("pp32x24x2"))
    rng = np.random.default_rng(3)
    nk = o.grid("NODE_KIND")
    Q = rng.normal(size=o.nn) * 1e-15 * (nk < 0)
    chi = np.zeros(o.nn)
    U = (37.0, -12.5)
    phi, it, rel, rc = o.solve_qv(Q, chi, U, tol=1e-13)
    phi0, _, _, rc0 = o.solve_qv(Q, chi, (0.0, 0.0), tol=1e-13)
    assert rc == 0 and rc0 == 0
    expect = phi0 + U[0] * o.phi_laplace(1) + U[1] * o.phi_laplace(2)
    assert np.max(np.abs(phi - expect)) <= 1e-9 * np.max(np.abs(expect))


def test_ideal_sources_hold_the_charge_and_their_harmonics():
    """Two ideal sources in vacuum: Q = C U on both electrodes, U the source
    values; over one period of the 13.56 MHz drive the 27.12 MHz electrode
    shows exactly its amplitude at harmonic 2."""
    o = _vac(workload("pp32x24x2"))
    o.step(200)
    d = o.diag()
    C = o.capacitance()
    U = np.array(d.U_el[:2])
    Q = np.array(d.Q_el[:2])
    assert np.max(np.abs(Q - C @ U)) <= 1e-12 * np.max(np.abs(C @ U)) + 1e-30
    t = d.t
    assert U[0] == pytest.approx(100.0 * math.sin(2 * math.pi * 13.56e6 * t), abs=1e-9)
    assert U[1] == pytest.approx(50.0 * math.sin(2 * math.pi * 27.12e6 * t), abs=1e-9)
    ph = 2 * 2 * math.pi / 200
    X2 = complex(d.hU_re[1][2], d.hU_im[1][2])
    assert abs(X2 - 50.0 * (-1j) * cmath.exp(1j * ph)) <= 1e-9
    assert abs(complex(d.hU_re[1][1], d.hU_im[1][1])) <= 1e-9


def test_series_branch_coupled_to_a_second_electrode_matches_phasor():
    """Electrode 1 behind a series R_b L_b C_b branch (Eq. 9), electrode 2 an
    ideal source at the same frequency: in steady state
    Q1 (1/C11 + 1/C_b + j w R_b - w^2 L_b) = Us1 + C12 U2 / C11 and
    U1 = (Q1 - C12 U2) / C11."""
    w = workload("pp32x24x2", circuit=_circuit(CIRC_SERIES_RLC, U_amp=100.0), run=dict(steps_per_period=400))
    w["circuits_more"] = [_circuit(CIRC_IDEAL, U_amp=60.0)]
    o = _vac(w)
    C = o.capacitance()
    spp = 400
    o.step(20 * spp)
    d = o.diag()
    U1 = complex(d.hU_re[0][1], d.hU_im[0][1])
    om = 2 * math.pi * 13.56e6
    rot = cmath.exp(2j * math.pi / spp)          # samples are taken at t_{n+1}
    Us1, U2 = 100.0 * -1j * rot, 60.0 * -1j * rot
    z = 1 / C[0, 0] + 1 / 5e-9 + 1j * om * 0.5 - om * om * 0.01e-6
    Q1 = (Us1 + C[0, 1] * U2 / C[0, 0]) / z
    expect = (Q1 - C[0, 1] * U2) / C[0, 0]
    assert abs(U1 - expect) <= 2e-5 * abs(expect)


def _charge_total(o):
    d = o.diag()
    tot = 0
    for sp, sgn in ((0, -1), (1, 1)):
        p = o.particles(sp)
        alive = p["r"] >= 0
        parts = sum(int(math.floor(float(w) * K)) for w in p["w"][alive])
        cnt = sum(int(d.absorbed[sp][c]) for c in range(4)) + sum(int(d.absorbed_el[sp][e]) for e in range(1, 4))
        tot += sgn * (parts + cnt)
    return tot


def test_integer_charge_conserved_with_two_electrodes():
    """Particles absorbed on the second electrode are counted there: charge
    in particles plus every conductor and dielectric counter is conserved
    exactly through steps with ionisation."""
    o = O.Oracle(workload("pp32x24x2", run=dict(Te_eV=8.0)))
    q0 = _charge_total(o)
    o.step(60)
    d = o.diag()
    assert d.born > 0
    assert d.absorbed_el[0][1] > 0 or d.absorbed_el[1][1] > 0
    assert _charge_total(o) == q0
