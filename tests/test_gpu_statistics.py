"""Statistical parity of long GPU runs against the FP64 oracle.

The GPU path and the oracle run the same algorithm on the same Philox
streams, but FP32 particle arithmetic against FP64 makes trajectories part
ways within a few hundred steps, after which the GPU run is one more sample
of the discharge.  So the GPU run (seed 1) is compared with an ensemble of
oracle runs that differ only in the seed.  For every compared quantity q
(period-averaged electron and ion inventories, 4x4-node block inventories,
harmonics 1..5 of the electrode current and voltage, the CCP and load
impedances and the source and plasma powers of Eqs. 11-14):

    |q_gpu - mean(q_oracle)| <= max(1% of |mean(q_oracle)|, 3 sigma sqrt(1 + 1/S))

with sigma the seed-to-seed standard deviation of S oracle runs: the 1%
bar wherever the discharge's own statistical noise is below it, the noise
floor where it is not.  Block and harmonic tests also bound the fraction of
entries outside the bar (a few are expected at 3 sigma across many entries).

The first test shows the 1% bar itself: with eight runs on each side,
200k + 200k particles and five RF periods averaged, the discharge's noise
floor drops to about half a percent, and the ensemble means must agree to
1% in the aggregate block densities and in each current harmonic.
"""
import numpy as np
import pytest

from oracle.ensemble import ensemble
from pic_inputs import workload

pytestmark = pytest.mark.gpu

SEEDS = [1, 2, 3, 4, 5, 6]


def _gpu_run(w, steps):
    from paper_2310_04957_amd.pic import Pic
    print(f"[gpu] statistics run {w['geometry']['nr']}x{w['geometry']['nz']} {steps} steps", flush=True)
    g = Pic(w)
    g.step(steps)
    d, grids = g.diag(grids=True)
    out = dict(n_e=grids["n_e"], n_i=grids["n_i"],
               harm_U=np.array(d.harm_U_re[:]) + 1j * np.array(d.harm_U_im[:]),
               harm_I=np.array(d.harm_I_re[:]) + 1j * np.array(d.harm_I_im[:]),
               periods_done=d.periods_done,
               elec=np.array([d.Z_ccp_re, d.Z_ccp_im, d.Z_load_re, d.Z_load_im, d.gamma_abs, d.P_source, d.P_Rs,
                              d.P_imn, d.P_stray, d.P_ccp, d.P_forward, d.P_ref]))
    g.close()
    return out


def _blocks(n, vol, nr, nz, b=4):
    """Particles (n V) summed over b x b node blocks."""
    a = (n * vol).reshape(nz + 1, nr + 1)
    H, W = (nz + 1) // b * b, (nr + 1) // b * b
    return a[:H, :W].reshape(H // b, b, W // b, b).sum(axis=(1, 3)).ravel()


def _check(name, gpu, ens, max_frac_out=0.0):
    ens = np.asarray(ens)
    S = ens.shape[0]
    mean = ens.mean(axis=0)
    sigma = np.sqrt((np.abs(ens - mean) ** 2).sum(axis=0) / (S - 1))
    bar = np.maximum(0.01 * np.abs(mean), 3.0 * sigma * np.sqrt(1.0 + 1.0 / S))
    dev = np.abs(np.asarray(gpu) - mean)
    out = dev > bar
    ratio = np.max(dev / np.maximum(bar, 1e-300))
    print(f"[gpu] {name}: worst |gpu - mean| / bar = {ratio:.2f}, outside {int(out.sum())} of {out.size}",
          flush=True)
    assert out.sum() <= max_frac_out * out.size, name


def _compare(w, steps):
    nr, nz = w["geometry"]["nr"], w["geometry"]["nz"]
    ens = ensemble(w, steps, SEEDS)
    gpu = _gpu_run(w, steps)
    assert gpu["periods_done"] == ens[0]["periods_done"] >= 1
    vol = ens[0]["vol"]
    for sp in ("n_e", "n_i"):
        _check(f"{sp} inventory", [(gpu[sp] * vol).sum()], [[(e[sp] * vol).sum()] for e in ens])
        _check(f"{sp} 4x4 blocks", _blocks(gpu[sp], vol, nr, nz),
               [_blocks(e[sp], vol, nr, nz) for e in ens], max_frac_out=0.1)
    for h in ("harm_I", "harm_U"):
        _check(f"{h} 1..5", gpu[h][1:6], [e[h][1:6] for e in ens], max_frac_out=0.2)
    # electrical characterisation (Eqs. 11-14): Z_ccp, Z_load, source and plasma power
    pick = [0, 1, 2, 3, 5, 9]
    _check("Z_ccp, Z_load, P_source, P_ccp", gpu["elec"][pick], [e["elec"][pick] for e in ens], max_frac_out=0.2)


def _gpu_mean(w, steps, periods, seeds):
    """Mean over GPU runs with the given seeds of the densities and
    harmonics averaged over the last `periods` RF periods."""
    import copy
    from paper_2310_04957_amd.pic import Pic
    spp = w["run"]["steps_per_period"]
    runs = []
    for s in seeds:
        ws = copy.deepcopy(w)
        ws["run"]["seed"] = s
        print(f"[gpu] mean run seed {s}", flush=True)
        g = Pic(ws)
        g.step(steps - (periods - 1) * spp)
        acc = None
        for k in range(periods):
            if k:
                g.step(spp)
            d, grids = g.diag(grids=True)
            cur = dict(n_e=grids["n_e"], n_i=grids["n_i"],
                       harm_I=np.array(d.harm_I_re[:]) + 1j * np.array(d.harm_I_im[:]))
            acc = cur if acc is None else {q: acc[q] + cur[q] for q in acc}
        assert d.error == 0
        runs.append({q: v / periods for q, v in acc.items()})
        g.close()
    return {q: np.mean([r[q] for r in runs], axis=0) for q in runs[0]}


@pytest.mark.timeout(900)
def test_parallel_plate_means_within_one_percent():
    """Ensemble agreement within 1%: eight GPU runs against eight oracle runs
    (seeds 1..8) of the 32x24 parallel-plate discharge with 200k + 200k
    particles, 2000 steps, densities and current harmonics averaged over the
    last five RF periods.  The ensemble means differ by at most 1%: the L2
    norm over 4x4-node blocks of the density difference, relative to the
    oracle's, and every current harmonic 1..5 relative to |I_1|.  The
    oracle's own noise floor (its two half-ensembles' difference, scaled to
    ensembles of eight) is printed beside each."""
    n, steps, periods, seeds = 200_000, 2000, 5, list(range(1, 9))
    w = workload("pp32x24", run=dict(n_e=n, n_i=n, cap_e=4 * n, cap_i=4 * n))
    nr, nz = w["geometry"]["nr"], w["geometry"]["nz"]
    ens = ensemble(w, steps, seeds, periods=periods)
    gpu = _gpu_mean(w, steps, periods, seeds)
    vol = ens[0]["vol"]
    half = len(seeds) // 2
    for sp in ("n_e", "n_i"):
        B = np.array([_blocks(e[sp], vol, nr, nz) for e in ens])
        mo = B.mean(axis=0)
        rel = np.linalg.norm(_blocks(gpu[sp], vol, nr, nz) - mo) / np.linalg.norm(mo)
        floor = np.linalg.norm(B[:half].mean(0) - B[half:].mean(0)) / np.linalg.norm(mo) / np.sqrt(2.0)
        print(f"[gpu] {sp} 4x4 blocks, last {periods} periods: GPU vs oracle {100 * rel:.2f}% "
              f"(oracle noise floor {100 * floor:.2f}%)", flush=True)
        assert rel <= 0.01, sp
    H = np.array([e["harm_I"] for e in ens])
    ho = H.mean(axis=0)
    dev = np.abs(gpu["harm_I"][1:6] - ho[1:6]) / abs(ho[1])
    floor = np.abs(H[:half, 1:6].mean(0) - H[half:, 1:6].mean(0)) / abs(ho[1]) / np.sqrt(2.0)
    print(f"[gpu] current harmonics 1..5 / |I_1|: GPU vs oracle {np.round(100 * dev, 3)}% "
          f"(noise floor {np.round(100 * floor, 3)}%)", flush=True)
    assert np.all(dev <= 0.01)


@pytest.mark.timeout(600)
def test_parallel_plate_ten_periods_match_oracle_statistics():
    """The 32x24 parallel-plate discharge (20k + 20k, 100 V, 20 mTorr),
    2000 steps = 10 RF periods."""
    w = workload("pp32x24")
    _compare(w, w["run"]["steps"])


@pytest.mark.timeout(600)
def test_gec_cell_with_matching_network_matches_oracle_statistics():
    """The GEC-shaped cell with the L-type matching network on a 64x128
    grid, 50k + 50k particles, 2 RF periods (800 steps)."""
    n = 50000
    w = workload("gec128x256", run=dict(n_e=n, n_i=n, cap_e=4 * n, cap_i=4 * n))
    w["geometry"]["nr"], w["geometry"]["nz"] = 64, 128
    _compare(w, 800)
