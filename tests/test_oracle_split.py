"""Pins of the oracle's particle splitting and unequal-weight load (reading
R32 of Sec. 3: split heavy particles near the axis against on-axis heating).

Expected values come from the closed form of the reference weight on a
uniform-vacuum grid, exact rational sums, hand-chosen weight ratios and the
identity of the copies, not from the oracle's own formulas."""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from pic_inputs import random_particles, workload
from pic_inputs.workloads import GROUND, POWERED

R, Z, NR, NZ = 0.05, 0.0254, 32, 24
FIELDS = ("r", "z", "vr", "vt", "vz", "ar", "at", "az", "w")


def _o(n_e=1000, n_i=500, cap=20000, load=False, **run):
    g = dict(nr=NR, nz=NZ, R=R, Z=Z, regions=[], edge_bc=[GROUND, POWERED, GROUND])
    r = dict(n_e=n_e, n_i=n_i, cap_e=cap, cap_i=cap)
    r.update(run)
    return O.Oracle(workload("pp32x24", geometry=g, run=r), load=load)


def test_reference_weight_closed_form():
    """All-vacuum grid: V_i = pi dz dr^2 (2i+1) and the mean cell volume is
    pi R^2 Z / (nr nz), so w_ref(i) = W_s (2i + 1) / nr with W_e = 1 and
    W_i = n_e / n_i; the column weights of all cells sum to nr nz W_s."""
    o = _o(n_e=1000, n_i=500)
    for sp, Ws in ((0, 1.0), (1, 2.0)):
        t = np.array([o.split_target(sp, i) for i in range(NR)])
        expect = Ws * (2 * np.arange(NR) + 1) / NR
        assert np.max(np.abs(t / expect - 1.0)) < 1e-13
        assert abs(t.sum() * NZ / (NR * NZ * Ws) - 1.0) < 1e-13


def _column_particles(cols, ratios, sp, o, dead=(), outside=()):
    """One particle per entry at the centre of column i with weight
    ratio * w_ref(i) (float32), distinct velocities."""
    n = len(cols)
    dr = R / NR
    p = {f: np.zeros(n, dtype=np.float32) for f in FIELDS}
    for k, (i, q) in enumerate(zip(cols, ratios)):
        p["r"][k] = np.float32((i + 0.5) * dr)
        p["z"][k] = np.float32(Z * (0.2 + 0.6 * k / n))
        p["w"][k] = np.float32(q * o.split_target(sp, i))
        p["vr"][k], p["vt"][k], p["vz"][k] = 1e5 + k, -2e5 + 3 * k, 7e4 - k
        p["ar"][k], p["at"][k], p["az"][k] = 1e12 * k, -3e11, 5e11 + k
    for k in dead:
        p["r"][k] = -1.0
    for k in outside:
        p["z"][k] = np.float32(Z * 1.5)
    return p


def test_split_rule_by_weight_ratio():
    """Copies k = 2^m with m the largest such that w >= 2^m w_ref, at most 8;
    dead and outside particles never split; copies follow the last slot in
    parent order."""
    o = _o()
    cols = [3, 3, 10, 10, 0, 31, 7, 7, 5, 5, 12]
    ratios = [1.0, 1.999, 2.0, 3.9, 4.0, 7.5, 8.0, 1000.0, 100.0, 100.0, 0.25]
    kexp = [1, 1, 2, 2, 4, 4, 8, 8, 1, 1, 1]
    p = _column_particles(cols, ratios, 0, o, dead=(8,), outside=(9,))
    o.set_particles(0, p)
    added = o.split_now(0)
    assert added == sum(k - 1 for k in kexp)
    q = o.particles(0)
    n = len(cols)
    assert len(q["r"]) == n + added
    tail = n
    for k in range(n):
        kk = kexp[k]
        assert q["w"][k] == np.float64(p["w"][k]) / kk
        for c in range(kk - 1):
            for f in FIELDS:
                assert q[f][tail] == q[f][k], (k, c, f)
            tail += 1
        for f in FIELDS[:8]:
            assert q[f][k] == np.float64(p[f][k])


def test_split_conserves_charge_momentum_energy_exactly():
    o = _o()
    p = random_particles(3000, R, Z * 0.999, seed=11, wmin=0.01, wmax=0.6)
    o.set_particles(0, p)
    w0 = p["w"].astype(np.float64)
    added = o.split_now(0)
    q = o.particles(0)
    n = len(w0)
    assert added > 0 and len(q["r"]) == n + added

    def total(arr_w, arr_v=None):
        if arr_v is None:
            return sum(Fraction(float(x)) for x in arr_w)
        return sum(Fraction(float(x)) * Fraction(float(v)) for x, v in zip(arr_w, arr_v))

    assert total(q["w"]) == total(w0)
    for f in ("vr", "vt", "vz"):
        assert total(q["w"], q[f]) == total(w0, p[f].astype(np.float64))
    e0 = sum(Fraction(float(w)) * (Fraction(float(a)) ** 2 + Fraction(float(b)) ** 2 + Fraction(float(c)) ** 2)
             for w, a, b, c in zip(w0, p["vr"], p["vt"], p["vz"]))
    e1 = sum(Fraction(float(w)) * (Fraction(float(a)) ** 2 + Fraction(float(b)) ** 2 + Fraction(float(c)) ** 2)
             for w, a, b, c in zip(q["w"], q["vr"], q["vt"], q["vz"]))
    assert e0 == e1


def test_split_keeps_deposited_charge_and_leaves_no_heavy_particle():
    o = _o()
    p = random_particles(4000, R, Z * 0.999, seed=12, wmin=0.02, wmax=0.4)
    o.set_particles(0, p)
    g0 = o.deposit(p["r"], p["z"], p["w"])
    o.split_now(0)
    q = o.particles(0)
    g1 = o.deposit(q["r"], q["z"], q["w"])
    assert int(g1.sum()) == int(g0.sum())
    # after one pass every particle is lighter than two reference weights,
    # unless its parent was at least 16 of them (three doublings at most)
    dr = R / NR
    for k in range(len(q["r"])):
        i = min(int(q["r"][k] / dr), NR - 1)
        t = np.float32(o.split_target(0, i))
        if np.float32(q["w"][k]) >= 2 * t:
            assert np.float32(q["w"][k]) * 8 >= 16 * t


def test_split_that_does_not_fit_changes_nothing():
    o = _o(cap=3010)
    p = random_particles(3000, R, Z * 0.999, seed=13, wmin=0.3, wmax=0.6)
    o.set_particles(0, p)
    with pytest.raises(RuntimeError):
        o.split_now(0)
    q = o.particles(0)
    assert len(q["r"]) == 3000
    for f in FIELDS:
        assert np.array_equal(q[f], p[f].astype(np.float64))


def test_cell_weighted_load_is_uniform_per_cell_and_in_density():
    """Unequal-weight load: every vacuum cell equally likely, each particle
    weighted w_ref of its column; counts per cell follow one multinomial
    (chi-square within 6 sigma of its mean) and the total weight matches
    N W_s within 5 standard deviations."""
    N = 120_000
    o = _o(n_e=N, n_i=N // 2, cap=N, load=True, weights=1)
    q = o.particles(0)
    q = {f: v[q["r"] >= 0] for f, v in q.items()}
    n = len(q["r"])
    assert n > 0.99 * N   # the first prediction removed a few at the walls
    dr, dz = R / NR, Z / NZ
    i = np.minimum((q["r"] / dr).astype(int), NR - 1)
    j = np.minimum((q["z"] / dz).astype(int), NZ - 1)
    t = np.array([o.split_target(0, c) for c in range(NR)])
    # the stored positions are the first predicted ones (a fraction of a
    # cell from the loaded ones): the weight is its column's or a neighbour's
    col = np.searchsorted(t, q["w"])
    assert np.array_equal(t[col], q["w"])
    assert np.max(np.abs(col - i)) <= 1
    counts = np.bincount(j * NR + i, minlength=NR * NZ)
    m = NR * NZ
    chi2 = float(((counts - n / m) ** 2 / (n / m)).sum())
    assert abs(chi2 - (m - 1)) < 6 * np.sqrt(2 * (m - 1))
    sd = np.sqrt(n) * np.std(t)
    assert abs(q["w"].sum() - n * 1.0) < 5 * sd + 1e-9


def test_step_splits_at_the_sort_and_keeps_the_charge():
    """Two identical runs, one with splitting: the state is the same until
    the first electron sort; there the split run has split_added more
    electrons and exactly the same total charge."""
    w = dict(n_e=4000, n_i=4000, cap=40000, load=True, sort_every=3, sort_every_ion=3)
    a = _o(split=1, **w)
    b = _o(split=0, **w)
    a.step(3)
    b.step(3)
    da, db = a.diag(), b.diag()
    assert da.split_added[0] > 0
    assert da.n_alive[0] == db.n_alive[0] + da.split_added[0]
    pa, pb = a.particles(0), b.particles(0)
    sa = sum(Fraction(float(x)) for x in pa["w"][pa["r"] >= 0])
    sb = sum(Fraction(float(x)) for x in pb["w"][pb["r"] >= 0])
    assert sa == sb
