"""The allocation-free entry point pic_moments_noalloc against pic_moments
(the same energy-moment grids, bit for bit: integer node sums), through the
C ABI: two calls in a row on one GPU, the second on a smaller grid, and a
grid beyond the fixed scratch rejected with PIC_E_TOOBIG."""
import numpy as np
import pytest

from pic_inputs import workload

pytestmark = pytest.mark.gpu


def _pic(w, **kw):
    from paper_2310_04957_amd.pic import Pic
    print(f"[gpu] init {w['geometry']['nr']}x{w['geometry']['nz']} {kw}", flush=True)
    return Pic(w, **kw)


def _gec(nr, nz, n):
    w = workload("gec128x256", run=dict(n_e=n, n_i=n, cap_e=2 * n + 16, cap_i=2 * n + 16, sort_every=3))
    w["geometry"]["nr"], w["geometry"]["nz"] = nr, nz
    return w


def test_noalloc_moments_equal_moments_on_two_calls_the_second_smaller():
    big = _pic(_gec(256, 512, 400000))
    big.step(4)                 # a deferred sort is pending: both calls apply it first
    for sp in (0, 1):
        N0, E0 = big.moments_noalloc(sp)
        N1, E1 = big.moments(sp)
        assert np.array_equal(N0, N1) and np.array_equal(E0, E1), sp
        assert N1.sum() > 0 and E1.sum() > 0
    big.close()
    small = _pic(workload("pp32x24", run=dict(n_e=20000, n_i=20000, cap_e=40000, cap_i=40000)))
    small.step(3)
    for sp in (0, 1):
        N0, E0 = small.moments_noalloc(sp)
        N1, E1 = small.moments(sp)
        assert np.array_equal(N0, N1) and np.array_equal(E0, E1), sp
        assert N1.sum() > 0
    small.close()


def test_noalloc_rejects_a_grid_beyond_its_scratch():
    from paper_2310_04957_amd.pic import PIC_NOALLOC_MAX_NODES, PicError
    w = workload("gec128x256", run=dict(n_e=0, n_i=0, cap_e=16, cap_i=16))
    w["geometry"]["nr"], w["geometry"]["nz"] = 2048, 1026
    assert 2049 * 1027 > PIC_NOALLOC_MAX_NODES
    g = _pic(w, load=False)
    with pytest.raises(PicError) as e:
        g.moments_noalloc(0)
    assert e.value.code == -9
    g.close()
