"""Pins of the oracle's random streams and null-collision MCC (Vahedi &
Surendra 1995, cited in the collision paragraph of Sec. 2): Philox against
numpy's Philox4x64, collision rates on monoenergetic beams (n_g sigma v),
closed-form distributions of the scattering formulas, energy bookkeeping."""
import math

import numpy as np
import pytest
from scipy import optimize, stats

import oracle as O
from pic_inputs import workload

QE, ME, MAR = 1.602176634e-19, 9.1093837015e-31, 39.948 * 1.66053906660e-27


def test_philox4x64_round_structure_matches_numpy():
    # numpy's Philox is Philox4x64-10 and increments the counter before use.
    for key in ([0, 0], [123456789, 987654321], [2 ** 64 - 1, 5]):
        for c0 in (0, 7, 2 ** 40):
            bg = np.random.Philox(counter=np.array([c0, 0, 0, 0], dtype=np.uint64),
                                  key=np.array(key, dtype=np.uint64))
            ref = bg.random_raw(4)
            mine = O.philox4x64([c0 + 1, 0, 0, 0], key)
            assert [int(x) for x in mine] == [int(x) for x in ref]


def test_philox4x32_uniform_and_decorrelated():
    n = 1 << 15
    out = np.array([O.philox4x32([k, 3, 2, 0], [1, 0]) for k in range(n)], dtype=np.uint64)
    for c in range(4):
        h, _ = np.histogram(out[:, c] >> 24, bins=256, range=(0, 256))
        chi2 = ((h - n / 256) ** 2 / (n / 256)).sum()
        assert stats.chi2.sf(chi2, 255) > 1e-4
    u = out.astype(np.float64) / 2 ** 32
    cc = np.corrcoef(u[:-1, 0], u[1:, 0])[0, 1]
    assert abs(cc) < 5 / math.sqrt(n)
    # different words of one call are uncorrelated too
    assert abs(np.corrcoef(u[:, 0], u[:, 1])[0, 1]) < 5 / math.sqrt(n)


def test_cross_section_closed_forms():
    el, ex, io = O.xsec_e(0.0)
    assert el == pytest.approx(1e-19) and ex == 0.0 and io == 0.0
    assert O.xsec_e(11.49)[1] == 0.0 and O.xsec_e(15.75)[2] == 0.0
    # ln(x)/x peaks at x = e with value 1/e
    assert O.xsec_e(11.5 * math.e)[1] == pytest.approx(2.7e-20 / math.e, rel=1e-12)
    assert O.xsec_e(15.76 * math.e)[2] == pytest.approx(8e-20 / math.e, rel=1e-12)
    assert O.xsec_e(10.0)[0] == pytest.approx(1e-19 / math.sqrt(2), rel=1e-14)


def _oracle(p_mtorr=20.0, T_gas=300.0):
    w = workload("pp32x24", gas=dict(p_Pa=p_mtorr * 133.322368e-3, T_K=T_gas),
                 run=dict(n_e=0, n_i=0, cap_e=1, cap_i=1))
    return O.Oracle(w, load=False)


def test_nu_max_bounds_the_total_rate_and_is_tight():
    o = _oracle()
    d = o.diag()
    ng = d.n_gas
    assert ng == pytest.approx(20 * 133.322368e-3 / (1.380649e-23 * 300), rel=1e-14)

    def sv(logeps):
        eps = 10 ** logeps
        return -sum(O.xsec_e(eps)) * math.sqrt(2 * QE * eps / ME)
    best = optimize.minimize_scalar(sv, bounds=(0, 4), method="bounded", options=dict(xatol=1e-10))
    assert d.nu_max[0] >= -best.fun * ng
    assert d.nu_max[0] <= 1.0011 * -best.fun * ng
    P = -math.expm1(-d.nu_max[0] * d.dt)
    assert d.thresh[0] == math.floor(P * 2 ** 32)


@pytest.mark.parametrize("eps", [5.0, 30.0, 120.0])
def test_monoenergetic_electron_beam_rates(eps):
    o = _oracle()
    d = o.diag()
    n = 400_000
    v = math.sqrt(2 * QE * eps / ME)
    vel = np.tile([0.0, 0.0, v], (n, 1))
    _, proc, _ = o.mcc(0, vel, 0, 17)
    pcoll = d.thresh[0] / 2 ** 32
    sig = O.xsec_e(eps)
    for k in range(3):
        p = pcoll * d.n_gas * sig[k] * v / d.nu_max[0]
        cnt = int((proc == k).sum())
        assert abs(cnt - n * p) <= 5 * math.sqrt(n * p * (1 - p)) + 1
    p_any = pcoll
    assert abs(int((proc >= 0).sum()) - n * p_any) <= 5 * math.sqrt(n * p_any) + 1


def test_monoenergetic_ion_beam_rates():
    o = _oracle(T_gas=1e-6)   # neutrals at rest: relative speed = ion speed
    d = o.diag()
    n = 400_000
    g = 2e4
    vel = np.tile([g, 0.0, 0.0], (n, 1))
    _, proc, _ = o.mcc(1, vel, 0, 3)
    pcoll = d.thresh[1] / 2 ** 32
    p = pcoll * d.n_gas * 5e-19 * g / d.nu_max[1]
    for k in (0, 1):
        cnt = int((proc == k).sum())
        assert abs(cnt - n * p) <= 5 * math.sqrt(n * p) + 1


def _many_collisions(o, sp, v3, proc_want, n=300_000):
    vel = np.tile(v3, (n, 1))
    out, proc, b = o.mcc(sp, vel, 0, 5)
    sel = proc == proc_want
    return vel[sel], out[sel], b[sel]


def test_elastic_angle_cdf_and_energy_loss():
    o = _oracle(p_mtorr=2000)   # high pressure: more collisions per draw
    eps = 40.0
    v = math.sqrt(2 * QE * eps / ME)
    vin, vout, _ = _many_collisions(o, 0, [v, 0.0, 0.0], 0)
    assert len(vin) > 2000
    c = (vout[:, 0]) / np.linalg.norm(vout, axis=1)
    # F(c) = 1 - ln(1 + eps (1 - c)/2) / ln(1 + eps)
    cdf = lambda x: 1 - np.log1p(eps * (1 - x) / 2) / math.log1p(eps)
    assert stats.kstest(c, cdf).pvalue > 1e-4
    e2 = 0.5 * ME * (vout ** 2).sum(1) / QE
    assert np.allclose(e2, eps * (1 - 2 * ME / MAR * (1 - c)), rtol=1e-10)


def test_excitation_and_ionisation_energy_bookkeeping():
    o = _oracle(p_mtorr=2000)
    eps = 60.0
    v = math.sqrt(2 * QE * eps / ME)
    _, vout, _ = _many_collisions(o, 0, [0.0, v, 0.0], 1)
    e2 = 0.5 * ME * (vout ** 2).sum(1) / QE
    assert len(e2) > 100 and np.allclose(e2, eps - 11.5, rtol=1e-12)
    _, vout, b = _many_collisions(o, 0, [0.0, v, 0.0], 2)
    esc = 0.5 * ME * (vout ** 2).sum(1) / QE
    eej = 0.5 * ME * (b[:, :3] ** 2).sum(1) / QE
    assert len(esc) > 100 and np.allclose(esc + eej, eps - 15.76, rtol=1e-12)
    # ejected energy: u = atan(e_ej / B) / atan((e - 15.76) / 2B) is uniform
    u = np.arctan(eej / 10.0) / math.atan((eps - 15.76) / 20.0)
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    # new ions are Maxwellian at the gas temperature
    vth2 = 1.380649e-23 * 300 / MAR
    vi = b[:, 3:]
    assert abs(vi.var(0).mean() / vth2 - 1) < 6 * math.sqrt(2 / (3 * len(vi)))


def test_ion_isotropic_and_charge_exchange():
    o = _oracle(p_mtorr=2000, T_gas=1e-6)
    g = 3e4
    vin, vout, _ = _many_collisions(o, 1, [0.0, 0.0, g], 0)
    # cos chi = sqrt(1 - u), |g'| = |g| cos chi  =>  (|v'|/|v|)^2 = 1 - u uniform
    x = (vout ** 2).sum(1) / g ** 2
    assert len(x) > 1000 and stats.kstest(x, "uniform").pvalue > 1e-4
    cosl = vout[:, 2] / np.linalg.norm(vout, axis=1)
    # neutrals at 1e-6 K move ~0.01 m/s: direction error ~1e-6 rad
    assert np.max(np.abs(cosl ** 2 - x)) <= 1e-5
    _, vout, _ = _many_collisions(o, 1, [0.0, 0.0, g], 1)
    assert len(vout) > 1000 and np.abs(vout).max() < 1.0   # neutral velocity ~ 0 at 1e-6 K
    o2 = _oracle(p_mtorr=2000, T_gas=300.0)
    _, vout, _ = _many_collisions(o2, 1, [0.0, 0.0, g], 1)
    vth2 = 1.380649e-23 * 300 / MAR
    assert abs(vout.var(0).mean() / vth2 - 1) < 6 * math.sqrt(2 / (3 * len(vout)))
    assert np.abs(vout.mean(0)).max() < 6 * math.sqrt(vth2 / len(vout))
