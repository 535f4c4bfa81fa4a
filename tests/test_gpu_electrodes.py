"""GPU parity with several driven electrodes (Sec. 2, one equivalent
capacitance and circuit per electrode; the electrodes couple through the
capacitance matrix).  Tolerances: capacitance matrix and Laplace solutions
1e-9, potentials 1e-6 (solves to 1e-12), circuit voltages and charges of a
vacuum run 1e-9, one step from an identical state as in the single-electrode
parity test, and exact integer charge conservation."""
import math

import numpy as np
import pytest

import oracle as O
from pic_inputs import random_particles, workload
from pic_inputs.workloads import CIRC_IDEAL, CIRC_SERIES_RLC, _circuit

pytestmark = pytest.mark.gpu
K = 2 ** 32


def _pic(w, **kw):
    from paper_2310_04957_amd.pic import Pic
    print(f"[gpu] init {w['geometry']['nr']}x{w['geometry']['nz']} electrodes "
          f"{1 + len(w.get('circuits_more', []))} {kw}", flush=True)
    return Pic(w, **kw)


def _vacuum(name="pp32x24x2", **over):
    w = workload(name, **over)
    w["run"].update(n_e=0, n_i=0, cap_e=1, cap_i=1)
    return w


def test_capacitance_matrix_and_laplace_solutions_match_oracle():
    w = _vacuum()
    g = _pic(w, load=False)
    o = O.Oracle(w, load=False)
    Cg, Co = g.capacitance(), o.capacitance()
    assert Cg.shape == (2, 2)
    assert np.max(np.abs(Cg - Co)) <= 1e-9 * np.max(np.abs(Co))
    assert Cg[0, 1] == Cg[1, 0]
    for e, name in ((1, "PHI_L"), (2, "PHI_L2")):
        a, b = g.grid(name), o.phi_laplace(e)
        assert np.max(np.abs(a - b)) <= 1e-9
    g.close()


def test_solve_with_two_electrode_voltages_matches_oracle():
    w = _vacuum()
    g = _pic(w, load=False)
    o = O.Oracle(w, load=False)
    rng = np.random.default_rng(5)
    nk = o.grid("NODE_KIND")
    Q = rng.normal(size=o.nn) * 1e-15 * (nk < 0)
    chi = np.abs(rng.normal(size=o.nn)) * 0.3
    U = (37.0, -12.5)
    ref, _, _, rco = o.solve_qv(Q, chi, U, tol=1e-12)
    phi, it, rel, rc = g.solve_once_el(Q, chi, U, 1e-12)
    assert rc == 0 and rco == 0
    assert np.max(np.abs(phi - ref)) <= 1e-6 * np.max(np.abs(ref))
    assert np.all(phi[nk == 2] == -12.5) and np.all(phi[nk == 1] == 37.0)
    g.close()


@pytest.mark.parametrize("kind", ["ideal", "series"])
def test_vacuum_circuits_match_oracle(kind):
    """Two periods without plasma: electrode 1 ideal (and electrode 2 at
    twice the frequency) or behind a series branch coupled to an ideal
    electrode 2; voltages, charges, currents and harmonics per electrode."""
    over = {} if kind == "ideal" else dict(circuit=_circuit(CIRC_SERIES_RLC, U_amp=100.0))
    w = _vacuum(**over)
    if kind == "series":
        w["circuits_more"] = [_circuit(CIRC_IDEAL, U_amp=60.0)]
    g = _pic(w, load=False)
    o = O.Oracle(w, load=False)
    g.step(400)
    o.step(400)
    dg, do = g.diag(), o.diag()
    assert dg.n_el == do.n_el == 2
    for f in ("U_el", "Q_el", "I_el"):
        a, b = np.array(getattr(dg, f)[:2]), np.array(getattr(do, f)[:2])
        assert np.max(np.abs(a - b)) <= 1e-9 * (np.max(np.abs(b)) + 1e-30), f
    for f in ("hU_re", "hU_im", "hI_re", "hI_im"):
        a = np.array([getattr(dg, f)[e][:] for e in range(2)])
        b = np.array([getattr(do, f)[e][:] for e in range(2)])
        assert np.max(np.abs(a - b)) <= 1e-9 * (np.max(np.abs(b)) + 1e-30), f
    g.close()


def test_one_step_with_two_electrodes_matches_oracle():
    w = workload("pp32x24x2", run=dict(n_e=0, n_i=0, cap_e=40000, cap_i=40000, sort_every=0))
    w["solver"]["tol"] = 1e-12
    gm = w["geometry"]
    pe = random_particles(20000, gm["R"] * 0.98, gm["Z"], seed=43, vmax=6e5, amax=1e13, wmin=1.0, wmax=1.0,
                          z_lo=0.002, z_hi=0.019)
    pi = random_particles(20000, gm["R"] * 0.98, gm["Z"], seed=44, vmax=3e3, amax=1e9, wmin=1.0, wmax=1.0,
                          z_lo=0.002, z_hi=0.019)
    g = _pic(w, load=False)
    o = O.Oracle(w, load=False)
    for s in (g, o):
        s.set_particles(0, pe)
        s.set_particles(1, pi)
        s.redeposit()
    g.step(1)
    o.step(1)
    dg, do = g.diag(), o.diag()
    assert np.max(np.abs(np.array(dg.U_el[:2]) - np.array(do.U_el[:2]))) <= 1e-9 * 100
    phig, phio = g.grid("PHI"), o.grid("PHI")
    assert np.max(np.abs(phig - phio)) <= 1e-6 * np.max(np.abs(phio))
    for sp in (0, 1):
        a, b = g.particles(sp), o.particles(sp)
        both = (a["r"] >= 0) & (b["r"] >= 0)
        for f in ("r", "z", "vr", "vt", "vz"):
            x, y = a[f][both].astype(np.float64), b[f][both]
            err = np.abs(x - y) / (np.abs(y) + np.max(np.abs(y)) * 1e-3)
            assert np.mean(err > 1e-4) <= 2e-3, (sp, f)
    g.close()


def _charge_total(s):
    d = s.diag()
    tot = 0
    for sp, sgn in ((0, -1), (1, 1)):
        p = s.particles(sp)
        alive = p["r"] >= 0
        parts = sum(int(math.floor(float(w) * K)) for w in np.asarray(p["w"], dtype=np.float64)[alive])
        cnt = sum(int(d.absorbed[sp][c]) for c in range(4)) + sum(int(d.absorbed_el[sp][e]) for e in range(1, 4))
        tot += sgn * (parts + cnt)
    return tot


def test_charge_conserved_with_particles_on_the_second_electrode():
    g = _pic(workload("pp32x24x2", run=dict(Te_eV=8.0)))
    q0 = _charge_total(g)
    g.step(60)
    d = g.diag()
    assert d.born > 0
    assert d.absorbed_el[0][1] > 0 or d.absorbed_el[1][1] > 0
    assert _charge_total(g) == q0
    g.close()
