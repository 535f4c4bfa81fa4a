"""GPU parity of one particle step on the GEC cell at 128 x 256 cells, a grid
far wider than the particle kernel's LDS window, so the step takes both its
window paths (E, cell kinds and deposits in LDS) and its global paths (field
gather, cell-kind reads and deposits in global memory), with particles next
to and inside the electrodes, the grounded shield and the dielectric ring
and cap (Sec. 2: absorption, electrode charge of Eq. 8; dielectric surface
charge, reading R10).

Test 1 makes absorption exact on both sides: the plasma density is so small
that the implicit correction moves no particle by more than a tenth of an
FP64 ulp, so the particles inside non-vacuum cells are absorbed at the same
(FP32) position on both sides, and the vacuum particles are kept far enough
from non-vacuum cells that no one reaches one during the step.  Then the
integer counters per conductor, the dielectric charge grid, the set of
removed slots and the collision counts per process are bit-identical.

Test 2 runs a real discharge field with particles that cross into the walls
during the prediction, where FP32 and FP64 landing points may fall on the
two sides of a cell edge: every disagreement is counted, and the counters
must differ by exactly the charge of the disagreeing particles."""
import numpy as np
import pytest

import oracle as O
from pic_inputs import random_particles, workload
from pic_inputs.workloads import CIRC_IDEAL

pytestmark = pytest.mark.gpu

K32 = 2.0 ** 32


def _pic(w, **kw):
    from paper_2310_04957_amd.pic import Pic
    print(f"[gpu] init {w['geometry']['nr']}x{w['geometry']['nz']} {kw}", flush=True)
    return Pic(w, **kw)


def _charge(wf32):
    """floor(W 2^32) of FP32 weights, as the deposit definition takes them."""
    return np.floor(wf32.astype(np.float64) * K32).astype(np.int64)


def _place(o, w, n_safe, n_wall, seed, vmax, margin):
    """n_safe particles in vacuum cells whose neighbourhood of margin =
    (cells in r, cells in z) is vacuum (so a step of at most that many cells
    stays in vacuum), n_wall particles inside dielectric or conductor
    cells."""
    g = w["geometry"]
    nr, nz, R, Z = g["nr"], g["nz"], g["R"], g["Z"]
    ck = o.grid("CELL_KIND").reshape(nz, nr)
    mr, mz = margin
    pad = np.pad(ck != 0, ((mz, mz), (mr, mr)), constant_values=True)
    bad = np.zeros_like(ck, dtype=bool)
    for dj in range(2 * mz + 1):
        for di in range(2 * mr + 1):
            bad |= pad[dj:dj + nz, di:di + nr]
    rng = np.random.Generator(np.random.PCG64(seed))
    out = {f: [] for f in O.FIELDS}
    for want, ok in ((n_safe, ~bad), (n_wall, ck != 0)):
        got = 0
        while got < want:
            p = random_particles(4 * want, R, Z, seed=int(rng.integers(1 << 30)), vmax=vmax, amax=0.0,
                                 wmin=1.0, wmax=3.0)
            i = np.floor(p["r"].astype(np.float64) / (R / nr)).astype(int).clip(0, nr - 1)
            j = np.floor(p["z"].astype(np.float64) / (Z / nz)).astype(int).clip(0, nz - 1)
            sel = np.flatnonzero(ok[j, i])[:want - got]
            for f in O.FIELDS:
                out[f].append(p[f][sel])
            got += len(sel)
    p = {f: np.concatenate(v) for f, v in out.items()}
    perm = rng.permutation(len(p["r"]))
    return {f: v[perm] for f, v in p.items()}


def _setup(w, pe, pi):
    """The same slots on both sides: the GPU tile-sorts them (so its LDS
    windows follow the particles), the oracle takes the sorted order."""
    g = _pic(w, load=False)
    o = O.Oracle(w, load=False)
    g.set_particles(0, pe)
    g.set_particles(1, pi)
    g.sort_now(0)
    g.sort_now(1)
    for sp in (0, 1):
        o.set_particles(sp, g.particles(sp))
    g.redeposit()
    o.redeposit()
    return g, o


def test_absorption_counters_and_wall_charge_are_bit_exact():
    w = workload("gec128x256", circuit=dict(kind=CIRC_IDEAL, U_amp=0.0, U_dc=0.0),
                 run=dict(n_e=1, n_i=1, cap_e=300000, cap_i=300000, sort_every=0, sort_every_ion=0, n0=1e-12))
    w["gas"]["p_Pa"] *= 10.0          # many colliders (electron collision probability ~0.3)
    o0 = O.Oracle(w, load=False)
    # speed bound: |v| dt <= 0.7 dr and <= 1.4 dz at 1.7e6 m/s per component
    pe = _place(o0, w, 60000, 20000, seed=71, vmax=1.7e6, margin=(1, 2))
    pi = _place(o0, w, 60000, 20000, seed=72, vmax=3e3, margin=(1, 2))
    del o0
    g, o = _setup(w, pe, pi)
    g.step(1)
    o.step(1)
    dg, do = g.diag(), o.diag()
    assert dg.error == 0
    # the field of a 1e-12 m^-3 plasma moves nothing: positions of the
    # survivors are the predicted ones of the same start on both sides
    for sp in (0, 1):
        a, b = g.particles(sp), o.particles(sp)
        assert len(a["r"]) == len(b["r"]), sp
        dead_g, dead_o = a["r"] < 0, b["r"] < 0
        assert np.array_equal(dead_g, dead_o), (sp, int((dead_g != dead_o).sum()))
        assert list(dg.absorbed[sp]) == list(do.absorbed[sp]), sp
        assert list(dg.absorbed_el[sp]) == list(do.absorbed_el[sp]), sp
        assert list(dg.coll[sp]) == list(do.coll[sp]), sp
        assert dg.absorbed[sp][3] > 0 and dg.absorbed[sp][0] > 0 and dg.absorbed[sp][1] > 0
    assert np.array_equal(g.grid("WALLQ"), o.grid("WALLQ"))
    assert np.abs(g.grid("WALLQ")).sum() > 0
    assert dg.born == do.born and dg.born > 20
    assert dg.n_alive[0] == do.n_alive[0] and dg.n_alive[1] == do.n_alive[1]
    # the deposit the step left is the exact definition of the positions it
    # predicted, and some of it went through the global fallback
    for sp, name in ((0, "DEP_E"), (1, "DEP_I")):
        p = g.particles(sp)
        ref = o.deposit(p["r"].astype(np.float64), p["z"].astype(np.float64), p["w"].astype(np.float64))
        assert np.array_equal(g.grid(name), ref), name
    live = int(dg.n_alive[0] + dg.n_alive[1])
    assert 0 < dg.deposit_fallback < live, (dg.deposit_fallback, live)
    g.close()


def test_one_step_with_wall_crossings_counts_every_disagreement():
    w = workload("gec128x256", run=dict(n_e=80000, n_i=80000, cap_e=300000, cap_i=300000, sort_every=0,
                                        sort_every_ion=0, n0=1e13))
    w["solver"]["tol"] = 1e-12
    gm = w["geometry"]
    o0 = O.Oracle(w, load=False)
    # electrons up to ~80 eV: they cross one to two cells per step, into the
    # electrodes, the dielectric and the domain edges
    pe = _place(o0, w, 80000, 0, seed=81, vmax=3e6, margin=(0, 0))
    pi = _place(o0, w, 80000, 0, seed=82, vmax=2e4, margin=(0, 0))
    del o0
    g, o = _setup(w, pe, pi)
    g.step(1)
    o.step(1)
    dg, do = g.diag(), o.diag()
    assert dg.error == 0
    phig, phio = g.grid("PHI"), o.grid("PHI")
    assert np.max(np.abs(phig - phio)) <= 1e-6 * np.max(np.abs(phio))
    assert dg.born == do.born
    flips_total = 0
    for sp in (0, 1):
        a, b = g.particles(sp), o.particles(sp)
        n = len(a["r"])
        assert n == len(b["r"])
        W = _charge(a["w"])          # weights never change in a step
        dead_g, dead_o = a["r"] < 0, b["r"] < 0
        only_g, only_o = dead_g & ~dead_o, dead_o & ~dead_g
        flips = int(only_g.sum() + only_o.sum())
        flips_total += flips
        # a disagreement is a landing point within FP32 rounding of a cell
        # edge or the domain boundary: rare
        assert flips <= 1e-3 * n, (sp, flips)
        # total absorbed charge: exactly the charge of the disagreeing slots
        tot_g, tot_o = sum(dg.absorbed[sp]), sum(do.absorbed[sp])
        assert tot_g - tot_o == int(W[only_g].sum() - W[only_o].sum()), sp
        assert sum(dg.absorbed[sp][k] for k in range(4)) > 0
        # per counter: the disagreeing slots plus the rounding of the landing
        # point's node shares for the dielectric hits (<= 64 units of 2^-20
        # cell per node and particle)
        flip_q = int(W[only_g | only_o].sum())
        diel = max(dg.absorbed[sp][3], do.absorbed[sp][3]) / (2 * K32) + 1
        for k in range(4):
            assert abs(dg.absorbed[sp][k] - do.absorbed[sp][k]) <= flip_q + diel * 3 * 64 * 4096, (sp, k)
        # survivors: FP32 push of the same state; a real collision whose
        # process selection flips is the only way to differ by more than
        # rounding, and process flips show in the per-process counts
        both = ~dead_g & ~dead_o
        bad = np.zeros(n, dtype=bool)
        for f in ("r", "z", "vr", "vt", "vz"):
            x, y = a[f].astype(np.float64), b[f]
            err = np.abs(x - y) / (np.abs(y) + np.max(np.abs(y[both])) * 1e-3)
            bad |= both & (err > 1e-4)
        dcoll = sum(abs(dg.coll[sp][k] - do.coll[sp][k]) for k in range(4))
        # a slot removed on one side only before its collision test changes
        # the collider total by one
        assert abs(sum(dg.coll[sp]) - sum(do.coll[sp])) <= flips, sp
        print(f"[gpu] species {sp}: {flips} fate flips, {int(bad.sum())} survivors off by > 1e-4, "
              f"per-process collision differences {dcoll}", flush=True)
        assert int(bad.sum()) <= dcoll + 2, (sp, int(bad.sum()), dcoll)
    print(f"[gpu] wall-crossing step: {flips_total} fate disagreements", flush=True)
    g.close()


def test_births_that_do_not_fit_stop_the_run():
    """Capacity overflow: the births that did not fit are dropped in that
    step; the next step returns PIC_E_CAPACITY before moving a particle and
    every later call refuses.  Forced from the host by a capacity barely
    above the initial count, with ionising electrons."""
    from paper_2310_04957_amd.pic import PicError
    w = workload("pp32x24", run=dict(n_e=0, n_i=0, cap_e=20010, cap_i=20010, sort_every=0))
    w["gas"]["p_Pa"] *= 10.0
    gm = w["geometry"]
    pe = random_particles(20000, gm["R"] * 0.98, gm["Z"], seed=91, vmax=6e6, amax=0.0, wmin=1.0, wmax=1.0,
                          z_lo=0.002, z_hi=0.023)
    pi = random_particles(20000, gm["R"] * 0.98, gm["Z"], seed=92, vmax=3e3, amax=0.0, wmin=1.0, wmax=1.0,
                          z_lo=0.002, z_hi=0.023)
    g = _pic(w, load=False)
    g.set_particles(0, pe)
    g.set_particles(1, pi)
    g.redeposit()
    g.step(1)                             # the overflowing step itself completes
    before = g.particles(0)
    with pytest.raises(PicError) as e:
        g.step(1)
    assert e.value.code == -2
    after = g.particles(0)
    for f in before:
        assert np.array_equal(before[f], after[f]), f    # nothing moved
    with pytest.raises(PicError) as e:
        g.step(3)
    assert e.value.code == -2
    assert g.diag().error == -2
    g.close()


def test_laplace_refresh_that_does_not_converge_is_an_error():
    """The per-period Laplace solve (C_eq, Eqs. 6-7) must converge; forced
    from the host with one Krylov iteration per solve and a loose tolerance
    for the step's own solve."""
    from paper_2310_04957_amd.pic import PicError
    from pic_inputs.workloads import SOLVE_MGPCG_FP64
    w = workload("gec128x256", run=dict(n_e=5000, n_i=5000, cap_e=20000, cap_i=20000, steps_per_period=20))
    w["geometry"]["nr"], w["geometry"]["nz"] = 64, 128
    g = _pic(w)
    g.step(5)
    g.set_solver(method=SOLVE_MGPCG_FP64, tol=0.5, max_iter=1)
    with pytest.raises(PicError) as e:
        g.step(15)                        # the period ends at step 20
    assert e.value.code == -3
    g.close()


def test_matching_design_matches_oracle():
    """Sec. 3: C_m1 and C_m2 of the L-network that match the vacuum C_eq of
    the cell.  The GEC stand-in's C_eq (about 117 pF) needs a larger L_m
    than the paper's 0.85 uH: with it no such network exists on either side.
    The design of the GPU's C_eq equals the oracle's design of its own, and
    after applying it the GPU's circuit runs the oracle's circuit with the
    designed elements (electrical characterisation to 1e-7)."""
    from paper_2310_04957_amd.pic import PicError
    w = workload("gec128x256", run=dict(n_e=0, n_i=0, cap_e=16, cap_i=16, steps_per_period=100))
    w["geometry"]["nr"], w["geometry"]["nz"] = 64, 128
    g = _pic(w, load=False)
    o = O.Oracle(w, load=False)
    with pytest.raises(PicError) as e:
        g.match_design()
    assert e.value.code == -1
    with pytest.raises(ValueError):
        O.match_design(w, o.diag().C_eq)
    g.close()
    w["circuit"]["L_m"] = 2.5e-6
    g = _pic(w, load=False)
    Ceq_g = g.diag().C_eq
    Cg = g.match_design()
    Co = O.match_design(w, o.diag().C_eq)
    assert abs(Cg[0] - Co[0]) <= 1e-9 * Co[0] and abs(Cg[1] - Co[1]) <= 1e-9 * Co[1]
    assert g.match_design(apply=True) == Cg
    g.step(200)
    d = g.diag()
    wd = dict(w, circuit=dict(w["circuit"], C_m1=Cg[0], C_m2=Cg[1]))
    U, I, e = O.circuit_vacuum(wd, Ceq_g, 200, chars=True)
    assert abs(d.U_E - U[-1]) <= 1e-7 * np.max(np.abs(U))
    sc = max(abs(complex(e["Z_load_re"], e["Z_load_im"])), 1.0)
    assert abs(d.Z_load_re - e["Z_load_re"]) <= 1e-7 * sc and abs(d.Z_load_im - e["Z_load_im"]) <= 1e-7 * sc
    assert abs(d.gamma_abs - e["gamma"]) <= 1e-7
    g.close()
