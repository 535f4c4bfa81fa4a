"""GPU parity of the HIP path against the FP64 CPU oracle, through the C ABI.

Bit-exact: fixed-point deposits (of any particle set, and of the positions
the fused step itself predicted), tile keys and sort permutations.
Tolerances: potential per solve 1e-6 relative (both solves to 1e-12), C_eq
1e-9, the electrode voltage of a step 1e-9, particle state after one step at
FP32 rounding."""
import math
import sys

import numpy as np
import pytest

import oracle as O
from pic_inputs import random_particles, workload
from pic_inputs.workloads import SOLVE_IR_MG, SOLVE_MGPCG_FP64

pytestmark = pytest.mark.gpu


def _pic(w, **kw):
    from paper_2310_04957_amd.pic import Pic
    print(f"[gpu] init {w['geometry']['nr']}x{w['geometry']['nz']} {kw}", flush=True)
    return Pic(w, **kw)


def _small_gec(nr=64, nz=128, n=20000, **run):
    r = dict(n_e=n, n_i=n, cap_e=4 * n, cap_i=4 * n)
    r.update(run)
    w = workload("gec128x256", run=r)
    w["geometry"]["nr"], w["geometry"]["nz"] = nr, nz
    return w


def _f64(p):
    return {k: np.asarray(v, dtype=np.float64) for k, v in p.items()}


@pytest.mark.parametrize("case", ["pp", "gec"])
def test_deposit_bit_exact_for_random_particles(case):
    w = workload("pp32x24", run=dict(n_e=0, n_i=0, cap_e=70000, cap_i=70000)) if case == "pp" else \
        _small_gec(n=0, cap_e=70000, cap_i=70000)
    g = w["geometry"]
    g_ = _pic(w, load=False)
    o = O.Oracle(w, load=False)
    p = random_particles(65537, g["R"], g["Z"], seed=21, dead_frac=0.02)   # several chunks + a ragged tail
    q = random_particles(1000, g["R"], g["Z"], seed=22, wmin=0.0, wmax=900.0)
    g_.set_particles(0, p)
    g_.set_particles(1, q)
    g_.redeposit()
    for name, pp in (("DEP_E", p), ("DEP_I", q)):
        ref = o.deposit(pp["r"].astype(np.float64), pp["z"].astype(np.float64), pp["w"].astype(np.float64))
        assert np.array_equal(g_.grid(name), ref), name
    # empty species
    g_.set_particles(1, {f: np.zeros(0, np.float32) for f in p})
    g_.redeposit()
    assert not g_.grid("DEP_I").any()
    g_.close()


def test_fused_step_deposit_and_charge_are_bit_exact():
    # the deposit the fused kernel leaves (LDS windows + global fallback) is
    # the exact definition applied to the positions it predicted
    w = _small_gec(n=30000, Te_eV=5.0, sort_every=3)
    g = _pic(w)
    g.step(7)
    d = g.diag()
    assert d.error == 0
    o = O.Oracle(w, load=False)
    total = 0
    for sp, name in ((0, "DEP_E"), (1, "DEP_I")):
        p = g.particles(sp)
        ref = o.deposit(p["r"].astype(np.float64), p["z"].astype(np.float64), p["w"].astype(np.float64))
        got = g.grid(name)
        assert np.array_equal(got, ref), name
        alive = p["r"] >= 0
        sgn = -1 if sp == 0 else 1
        total += sgn * (sum(int(math.floor(float(x) * 2 ** 32)) for x in p["w"][alive]) +
                        sum(int(d.absorbed[sp][c]) for c in range(4)))
    # integer charge: identical to the initial load (births are neutral pairs)
    g2 = _pic(w)
    d2 = g2.diag()
    t0 = 0
    for sp in (0, 1):
        p = g2.particles(sp)
        alive = p["r"] >= 0
        t0 += (-1 if sp == 0 else 1) * (sum(int(math.floor(float(x) * 2 ** 32)) for x in p["w"][alive]) +
                                        sum(int(d2.absorbed[sp][c]) for c in range(4)))
    assert total == t0
    assert int(g.grid("WALLQ").sum()) == int(d.absorbed[1][3]) - int(d.absorbed[0][3])
    g.close(); g2.close()


@pytest.mark.parametrize("nr", [64, 48, 16])
def test_sort_permutation_matches_stable_sort(nr):
    """Tile keys ty kmul + tx: 64 cells wide is 4 tiles per row (kmul = 4,
    column and row digit passes), 48 is 3 (kmul = 4 > 3: keys skip a value
    per row), 16 is one (kmul = 1, a single 8-bit digit pass)."""
    w = _small_gec(nr=nr, n=0, cap_e=50000, cap_i=50000)
    gm = w["geometry"]
    g = _pic(w, load=False)
    o = O.Oracle(w, load=False)
    p = random_particles(40000, gm["R"], gm["Z"], seed=31, dead_frac=0.1)
    # positions inside conductors are keyed like any other (only r < 0 is dead)
    g.set_particles(0, p)
    perm = g.sort_now(0)
    keys = o.tile_keys(p["r"].astype(np.float64), p["z"].astype(np.float64))
    ref = O.stable_perm(keys)
    alive = int((keys != 0xFFFFFFFF).sum())
    q = g.particles(0)
    assert len(q["r"]) == alive
    assert np.array_equal(perm[:alive], ref[:alive])
    for f in p:
        assert np.array_equal(q[f], p[f][ref[:alive]]), f
    g.close()


@pytest.mark.parametrize("size", [(64, 128), (512, 1024), (1024, 2048)])
@pytest.mark.parametrize("method", [SOLVE_MGPCG_FP64, SOLVE_IR_MG])
def test_field_solve_matches_oracle(method, size):
    """The GEC cell from a coarse grid up to the full 1024 x 2048 one, where
    the multigrid hierarchy runs its fine levels over thousands of blocks
    and its coarse levels in the fused tail kernel."""
    w = _small_gec(nr=size[0], nz=size[1], n=0, cap_e=16, cap_i=16)
    g = _pic(w, load=False, method=method)
    o = O.Oracle(w, load=False)
    rng = np.random.default_rng(7)
    chi = rng.uniform(0, 3.0, o.nn)
    Q = rng.normal(0, 3e-14, o.nn)
    U = 123.0
    ref, _, rel_o, rc_o = o.solve_q(Q, chi, U, tol=1e-12)
    phi, it, rel, rc = g.solve_once(Q, chi, U, tol=1e-12)
    print(f"[gpu] method {method}: iters {it} relres {rel:.2e}", flush=True)
    assert rc == 0 and rel <= 1e-12
    assert np.max(np.abs(phi - ref)) <= 1e-6 * np.max(np.abs(ref))
    # production tolerance: the residual criterion holds
    phi8, it8, rel8, rc8 = g.solve_once(Q, chi, U, tol=1e-8)
    assert rc8 == 0 and rel8 <= 1e-8
    g.close()


def test_device_controlled_refinement_continues_and_skips():
    """FP32 refinement with its control on the device: the host launches,
    ahead of its one read, the passes (and Krylov iterations) the last solve
    needed.  A solve that needs more passes (a tighter tolerance) continues
    pass by pass and reaches it; a solve that needs fewer leaves the extra
    passes to return at once, which changes no bit of its result.  After it
    an FP64 solve (host-controlled) starts unfinished and converges."""
    w = _small_gec(nr=64, nz=128, n=0, cap_e=16, cap_i=16)
    g = _pic(w, load=False, method=SOLVE_IR_MG)
    o = O.Oracle(w, load=False)
    rng = np.random.default_rng(11)
    chi = rng.uniform(0, 3.0, o.nn)
    Q = rng.normal(0, 3e-14, o.nn)
    U = 77.0
    ref, _, _, _ = o.solve_q(Q, chi, U, tol=1e-12)
    scale = np.max(np.abs(ref))
    phi1, it1, rel1, rc1 = g.solve_once(Q, chi, U, tol=1e-8)
    d1 = g.diag()
    assert rc1 == 0 and rel1 <= 1e-8
    phi2, it2, rel2, rc2 = g.solve_once(Q, chi, U, tol=1e-12)
    d2 = g.diag()
    print(f"[gpu] passes {d1.solver_outer} -> {d2.solver_outer}, iters {it1} -> {it2}", flush=True)
    assert rc2 == 0 and rel2 <= 1e-12
    assert d2.solver_outer > d1.solver_outer
    assert np.max(np.abs(phi2 - ref)) <= 1e-6 * scale
    phi3, it3, rel3, rc3 = g.solve_once(Q, chi, U, tol=1e-8)
    d3 = g.diag()
    assert rc3 == 0 and d3.solver_outer == d1.solver_outer and it3 == it1 and rel3 == rel1
    assert np.array_equal(phi3, phi1)
    g.set_solver(method=SOLVE_MGPCG_FP64)
    phi4, it4, rel4, rc4 = g.solve_once(Q, chi, U, tol=1e-12)
    assert rc4 == 0 and rel4 <= 1e-12 and it4 > 0
    assert np.max(np.abs(phi4 - ref)) <= 1e-6 * scale
    g.close()


def test_graph_replay_matches_eager_launches():
    """The fused CG's iterations replayed from HIP graphs (captured once per
    handle) give the same bits as the same kernels launched one by one: a
    12-step discharge on the 64x128 GEC grid (IR solves, each replaying the
    graphs several times between the step's own eager launches and host
    synchronisations) and then repeated FP64 solves from new right-hand
    sides on the same handles."""
    w = _small_gec(n=20000)
    g = _pic(w, graphs=True)
    e = _pic(w, graphs=False)
    for k in range(12):
        g.step(1)
        e.step(1)
        dg, de = g.diag(), e.diag()
        assert dg.error == 0 and de.error == 0
        assert dg.solver_iters == de.solver_iters and dg.solver_relres == de.solver_relres, k
        assert np.array_equal(g.grid("PHI"), e.grid("PHI")), k
    for sp in (0, 1):
        pg, pe = g.particles(sp), e.particles(sp)
        for f in pg:
            assert np.array_equal(pg[f], pe[f]), f
    rng = np.random.default_rng(3)
    for k in range(4):
        Q = rng.normal(0, 3e-14, g.nn)
        chi = rng.uniform(0, 3.0, g.nn)
        for h in (g, e):
            h.set_solver(method=SOLVE_MGPCG_FP64)
        a = g.solve_once(Q, chi, 50.0 * (k + 1), tol=1e-10)
        b = e.solve_once(Q, chi, 50.0 * (k + 1), tol=1e-10)
        assert a[3] == 0 and b[3] == 0 and a[1] == b[1], k
        assert np.array_equal(a[0], b[0]), k
    g.close()
    e.close()


def test_equivalent_capacitance_matches_oracle():
    for w in (workload("pp32x24", run=dict(n_e=0, n_i=0, cap_e=1, cap_i=1)), _small_gec(n=0)):
        g = _pic(w, load=False)
        o = O.Oracle(w, load=False)
        cg, co = g.diag().C_eq, o.diag().C_eq
        assert abs(cg - co) <= 1e-9 * co, (cg, co)
        assert np.max(np.abs(g.grid("PHI_L") - o.grid("PHI_L"))) <= 1e-8
        g.close()


def test_loader_matches_oracle_load():
    w = workload("pp32x24")
    g = _pic(w)
    o = O.Oracle(w)
    for sp in (0, 1):
        pg, po = g.particles(sp), o.particles(sp)
        assert len(pg["r"]) == len(po["r"])
        alive = (pg["r"] >= 0) & (po["r"] >= 0)
        assert (alive == (po["r"] >= 0)).mean() > 0.999
        for f in ("r", "z", "vr", "vt", "vz"):
            a, b = pg[f][alive].astype(np.float64), po[f][alive]
            scale = np.max(np.abs(b)) + 1e-30
            assert np.max(np.abs(a - b)) <= 2e-6 * scale, f
    assert g.diag().n_slots[0] == o.diag().n_slots[0]
    g.close()


def test_step_applying_a_sort_equals_sort_then_step():
    """A deferred sort is applied by the next particle step, which reads each
    new slot through the permutation; births of that step are appended in
    parent-slot order.  Bit for bit the same as sorting at once and stepping
    (every particle array, deposits, counters), with ionising electrons so
    that births occur."""
    w = workload("pp32x24", run=dict(n_e=0, n_i=0, cap_e=60000, cap_i=60000, sort_every=1, sort_every_ion=1))
    w["solver"]["tol"] = 1e-12
    gm = w["geometry"]
    pe = random_particles(30000, gm["R"] * 0.98, gm["Z"], seed=51, vmax=6e6, amax=1e13, wmin=1.0, wmax=1.0,
                          z_lo=0.002, z_hi=0.023, dead_frac=0.05)
    pi = random_particles(30000, gm["R"] * 0.98, gm["Z"], seed=52, vmax=3e3, amax=1e9, wmin=1.0, wmax=1.0,
                          z_lo=0.002, z_hi=0.023, dead_frac=0.05)
    wb = workload("pp32x24", run=dict(w["run"], sort_every=0, sort_every_ion=0))
    wb["solver"]["tol"] = 1e-12
    ga = _pic(w, load=False)
    gb = _pic(wb, load=False)
    for g in (ga, gb):
        g.set_particles(0, pe)
        g.set_particles(1, pi)
        g.redeposit()
    ga.step(1)            # sorts both species at the end (applied by the next step)
    gb.step(1)
    gb.sort_now(0)
    gb.sort_now(1)
    ga.step(1)            # applies the sort; sorts again at the end
    gb.step(1)
    gb.sort_now(0)
    gb.sort_now(1)
    da, db = ga.diag(), gb.diag()
    assert da.error == 0 and db.error == 0
    assert da.born == db.born and da.born > 50
    for sp in (0, 1):
        a, b = ga.particles(sp), gb.particles(sp)
        assert len(a["r"]) == len(b["r"])
        for f in a:
            assert np.array_equal(a[f].view(np.uint32), b[f].view(np.uint32)), (sp, f)
    for name in ("DEP_E", "DEP_I", "WALLQ", "PHI"):
        assert np.array_equal(ga.grid(name), gb.grid(name)), name
    assert [list(x) for x in da.absorbed] == [list(x) for x in db.absorbed]
    ga.close(); gb.close()


def test_sort_keyed_by_the_step_orders_births_and_split_copies():
    """The electron keys of a sort that ends a step come from that step's
    particle kernel; the slots appended after it (births, then split copies)
    get theirs from the key pass.  After such a sort, with ionising electrons
    and splitting on: every slot below the count holds a live particle, the
    tile keys (the oracle's) do not decrease, and the live count and total
    weight are those before the sort plus the copies."""
    from fractions import Fraction
    w = workload("pp32x24", run=dict(n_e=0, n_i=0, cap_e=120000, cap_i=60000, sort_every=1, sort_every_ion=0,
                                     split=1))
    gm = w["geometry"]
    pe = random_particles(30000, gm["R"] * 0.98, gm["Z"], seed=61, vmax=6e6, amax=1e13, wmin=1.0, wmax=3.0,
                          z_lo=0.002, z_hi=0.023, dead_frac=0.05)
    pi = random_particles(30000, gm["R"] * 0.98, gm["Z"], seed=62, vmax=3e3, amax=1e9, wmin=1.0, wmax=1.0,
                          z_lo=0.002, z_hi=0.023, dead_frac=0.05)
    wb = workload("pp32x24", run=dict(w["run"], sort_every=0, split=0))
    ga, gb = _pic(w, load=False), _pic(wb, load=False)
    for g in (ga, gb):
        g.set_particles(0, pe)
        g.set_particles(1, pi)
        g.redeposit()
    ga.step(1)
    gb.step(1)
    da, db = ga.diag(), gb.diag()
    assert da.error == 0 and db.error == 0
    assert da.born == db.born and da.born > 50
    assert da.split_added[0] > 0
    o = O.Oracle(w, load=False)
    a, b = ga.particles(0), gb.particles(0)
    assert np.all(a["r"] >= 0), "a dead slot below the count after the sort"
    live_b = b["r"] >= 0
    assert len(a["r"]) == int(live_b.sum()) + da.split_added[0]
    keys = o.tile_keys(a["r"].astype(np.float64), a["z"].astype(np.float64))
    assert np.all(np.diff(keys.astype(np.int64)) >= 0), "tile keys decrease"
    sa = sum(Fraction(float(x)) for x in a["w"])
    sb = sum(Fraction(float(x)) for x in b["w"][live_b])
    assert sa == sb
    ga.close(); gb.close()


@pytest.mark.parametrize("gas_factor,vmax_e", [(1, 6e5), (10, 6e5), (40, 6e5), (1, 6e6)])
def test_one_step_matches_oracle_given_identical_state(gas_factor, vmax_e):
    """gas_factor scales the pressure: at 10x (collision probability 0.57
    for electrons) and 40x (0.97) most lanes of a round of 64 particles
    collide.  Electrons up to 6e6 m/s (about 100 eV) ionise: the births are
    appended in parent order and compared slot by slot."""
    w = workload("pp32x24", run=dict(n_e=0, n_i=0, cap_e=40000, cap_i=40000, sort_every=0))
    w["gas"]["p_Pa"] *= gas_factor
    w["solver"]["tol"] = 1e-12
    gm = w["geometry"]
    pe = random_particles(20000, gm["R"] * 0.98, gm["Z"], seed=41, vmax=vmax_e, amax=1e13, wmin=1.0, wmax=1.0,
                          z_lo=0.002, z_hi=0.023)
    pi = random_particles(20000, gm["R"] * 0.98, gm["Z"], seed=42, vmax=3e3, amax=1e9, wmin=1.0, wmax=1.0,
                          z_lo=0.002, z_hi=0.023)
    g = _pic(w, load=False)
    o = O.Oracle(w, load=False)
    for s in (g, o):
        s.set_particles(0, pe)
        s.set_particles(1, pi)
        s.redeposit()
    g.step(1)
    o.step(1)
    dg, do = g.diag(), o.diag()
    assert abs(dg.U_E - do.U_E) <= 1e-9 * 100
    phig, phio = g.grid("PHI"), o.grid("PHI")
    assert np.max(np.abs(phig - phio)) <= 1e-6 * np.max(np.abs(phio))
    for sp in (0, 1):
        a, b = g.particles(sp), o.particles(sp)
        assert len(a["r"]) == len(b["r"])
        both = (a["r"] >= 0) & (b["r"] >= 0)
        assert (a["r"] >= 0).sum() == pytest.approx((b["r"] >= 0).sum(), abs=3)
        for f in ("r", "z", "vr", "vt", "vz"):
            x, y = a[f][both].astype(np.float64), b[f][both]
            err = np.abs(x - y) / (np.abs(y) + np.max(np.abs(y)) * 1e-3)
            # FP32 push; a handful of process-selection flips allowed
            assert np.mean(err > 1e-4) <= 2e-3, (sp, f)
        assert dg.coll[sp][0] + dg.coll[sp][1] + dg.coll[sp][2] + dg.coll[sp][3] == \
            do.coll[sp][0] + do.coll[sp][1] + do.coll[sp][2] + do.coll[sp][3]
    if vmax_e > 1e6:
        assert dg.born > 100 and dg.born == do.born
    assert dg.error == 0
    g.close()


@pytest.mark.parametrize("kind", ["lmatch", "series"])
def test_electrical_characterisation_matches_oracle(kind):
    """Eqs. 11-14 over the last RF period without plasma (deterministic FP64
    circuit on both sides): impedances, |Gamma| and element powers agree
    to 1e-7 relative (C_eq itself agrees to 1e-9)."""
    from pic_inputs.workloads import CIRC_LMATCH, CIRC_SERIES_RLC
    circ = dict(kind=CIRC_LMATCH, U_amp=77.0, C_m1=2335.51e-12, C_m2=215.62e-12) if kind == "lmatch" else \
        dict(kind=CIRC_SERIES_RLC, U_amp=100.0)
    w = workload("pp32x24", circuit=circ, run=dict(n_e=0, n_i=0, cap_e=1, cap_i=1, steps_per_period=200))
    g = _pic(w, load=False)
    o = O.Oracle(w, load=False)
    g.step(400)
    o.step(400)
    d = g.diag()
    e = O.elec_dict(o.diag().elec)
    assert d.periods_done == 2
    pairs = [("Z_ccp_re", "Z_ccp_re"), ("Z_ccp_im", "Z_ccp_im"), ("Z_load_re", "Z_load_re"),
             ("Z_load_im", "Z_load_im"), ("gamma_abs", "gamma"), ("P_source", "P_source"), ("P_Rs", "P_Rs"),
             ("P_imn", "P_IMN"), ("P_stray", "P_stray"), ("P_ccp", "P_ccp"), ("P_forward", "P_forward"),
             ("P_ref", "P_ref")]
    scale = {"Z": max(abs(complex(e["Z_ccp_re"], e["Z_ccp_im"])), abs(complex(e["Z_load_re"], e["Z_load_im"]))),
             "P": max(abs(e["P_source"]), 1e-30), "g": 1.0}
    for a, b in pairs:
        sc = scale["Z" if a.startswith("Z") else ("g" if a.startswith("gamma") else "P")]
        assert abs(getattr(d, a) - e[b]) <= 1e-7 * sc, (a, getattr(d, a), e[b])
    g.close()


@pytest.mark.parametrize("sp", [0, 1])
def test_energy_moments_bit_exact(sp):
    """Energy moments (T_e maps): integer node sums of the weight shares and
    of shares x floor(16 eps / eV) equal the oracle's bit for bit."""
    w = _small_gec(n=0, cap_e=70000, cap_i=70000)
    g = w["geometry"]
    gp = _pic(w, load=False)
    o = O.Oracle(w, load=False)
    vmax = 3e6 if sp == 0 else 3e3
    p = random_particles(65537, g["R"], g["Z"], seed=31 + sp, vmax=vmax, dead_frac=0.02)
    gp.set_particles(sp, p)
    o.set_particles(sp, _f64(p))
    N, E = gp.moments(sp)
    No, Eo = o.moments(sp)
    assert np.array_equal(N, No)
    assert np.array_equal(E, Eo)
    assert E.sum() > 0
    gp.close()


@pytest.mark.parametrize("sp", [0, 1])
def test_split_bit_exact(sp):
    """Particle splitting (Sec. 3): the same copies, weights and slot order as
    the oracle, bit for bit, over several chunks with a ragged tail, dead
    slots and particles outside the domain."""
    w = _small_gec(n=0, cap_e=120000, cap_i=120000)
    w["run"]["n_e"], w["run"]["n_i"] = 20000, 10000   # the loading weights (not loaded)
    g = w["geometry"]
    gp = _pic(w, load=False)
    o = O.Oracle(w, load=False)
    p = random_particles(30001, g["R"], g["Z"], seed=41 + sp, wmin=0.01, wmax=8.0, dead_frac=0.03)
    p["z"][::97] = np.float32(g["Z"] * 1.01)          # outside: never split
    gp.set_particles(sp, p)
    o.set_particles(sp, _f64(p))
    ag = gp.split_now(sp)
    ao = o.split_now(sp)
    assert ag == ao and ag > 1000
    qg, qo = gp.particles(sp), o.particles(sp)
    for f in qg:
        oo = qo[f].astype(np.float32)
        assert np.array_equal(oo.astype(np.float64), qo[f]), f   # oracle values are FP32 values
        assert np.array_equal(qg[f].view(np.uint32), oo.view(np.uint32)), f
    assert gp.diag().split_added[sp] == ag
    gp.close()


def test_cell_weighted_load_matches_oracle():
    """Unequal-weight load: same cells, positions to FP32 rounding, weights
    the FP32 of the oracle's."""
    w = workload("pp32x24", run=dict(weights=1))
    g = _pic(w)
    o = O.Oracle(w)
    for sp in (0, 1):
        pg, po = g.particles(sp), o.particles(sp)
        assert len(pg["r"]) == len(po["r"])
        alive = (pg["r"] >= 0) & (po["r"] >= 0)
        assert (alive == (po["r"] >= 0)).mean() > 0.999
        for f in ("r", "z", "vr", "vt", "vz"):
            a, b = pg[f][alive].astype(np.float64), po[f][alive]
            assert np.max(np.abs(a - b)) <= 2e-6 * (np.max(np.abs(b)) + 1e-30), f
        assert np.array_equal(pg["w"][alive], po["w"][alive].astype(np.float32))
    g.close()


def test_step_splits_at_the_sort_and_keeps_the_charge():
    """Two identical GPU runs, one with splitting: at the first electron
    sort the split run has split_added more electrons and the same total
    weight (as exact sums of FP32 weights)."""
    from fractions import Fraction
    w = workload("pp32x24", run=dict(n_e=8000, n_i=8000, cap_e=60000, cap_i=60000, sort_every=3,
                                     sort_every_ion=3))
    wa = workload("pp32x24", run=dict(w["run"], split=1))
    a, b = _pic(wa), _pic(w)
    a.step(3)
    b.step(3)
    da, db = a.diag(), b.diag()
    assert da.split_added[0] > 0
    assert da.n_alive[0] == db.n_alive[0] + da.split_added[0]
    pa, pb = a.particles(0), b.particles(0)
    sa = sum(Fraction(float(x)) for x in pa["w"][pa["r"] >= 0])
    sb = sum(Fraction(float(x)) for x in pb["w"][pb["r"] >= 0])
    assert sa == sb
    a.close()
    b.close()


def test_births_across_staging_segments_match_oracle():
    """More than a million electron slots (two segments of 1024 staging rows
    of the birth scan) with ionising electrons, so one segment holds more
    than 1024 births: the births are appended in parent-slot order, the same
    slots as the oracle's, with the same states to FP32 rounding."""
    n = 1_150_000
    w = workload("pp32x24", run=dict(n_e=0, n_i=0, cap_e=n + 200000, cap_i=n + 200000, sort_every=0,
                                     sort_every_ion=0))
    w["solver"]["tol"] = 1e-12
    gm = w["geometry"]
    pe = random_particles(n, gm["R"] * 0.98, gm["Z"], seed=111, vmax=6e6, amax=0.0, wmin=1.0, wmax=1.0,
                          z_lo=0.002, z_hi=0.023)
    pi = random_particles(n, gm["R"] * 0.98, gm["Z"], seed=112, vmax=3e3, amax=0.0, wmin=1.0, wmax=1.0,
                          z_lo=0.002, z_hi=0.023)
    g = _pic(w, load=False)
    o = O.Oracle(w, load=False)
    for s in (g, o):
        s.set_particles(0, pe)
        s.set_particles(1, pi)
        s.redeposit()
    g.step(1)
    o.step(1)
    dg, do = g.diag(), o.diag()
    assert dg.error == 0
    print(f"[gpu] births {dg.born} (oracle {do.born})", flush=True)
    assert dg.born == do.born and dg.born > 2048
    for sp in (0, 1):
        a, b = g.particles(sp), o.particles(sp)
        assert len(a["r"]) == len(b["r"]) == n + dg.born
        new = slice(n, n + dg.born)
        both = (a["r"][new] >= 0) & (b["r"][new] >= 0)
        assert both.mean() > 0.99
        for f in ("r", "z", "vr", "vt", "vz", "w"):
            x, y = a[f][new][both].astype(np.float64), b[f][new][both]
            err = np.abs(x - y) / (np.abs(y) + np.max(np.abs(y)) * 1e-3)
            assert np.mean(err > 1e-4) <= 1e-3, (sp, f)
    g.close()
