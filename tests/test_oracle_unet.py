"""Pins of the U-net oracle: central finite differences of the loss for every
parameter group (8 channels, 32x64 image), convolution against scipy's
correlate, pooling/upsampling adjointness, and bfloat16 rounding against
torch's bfloat16 conversion."""
import numpy as np
import pytest
import torch
from scipy import ndimage

from oracle import unet as U


def test_conv3x3_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(12, 10, 3))
    w = rng.normal(size=(9, 4, 3))
    b = rng.normal(size=4)
    y = U.conv3x3(x, w, b)
    for co in range(4):
        ref = np.full((12, 10), b[co])
        for ci in range(3):
            k = w[:, co, ci].reshape(3, 3)    # tap (dy+1, dx+1)
            ref += ndimage.correlate(x[:, :, ci], k, mode="constant", cval=0.0)
        assert np.allclose(y[:, :, co], ref, atol=1e-12)


def test_pool_and_upsample_are_adjoint_to_their_backward():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(8, 6, 3))
    y = rng.normal(size=(4, 3, 3))
    assert np.isclose((U.pool2(x) * y).sum(), (x * U.pool2_backward(y)).sum())
    assert np.isclose((U.up2(y) * x).sum(), (y * U.up2_backward(x)).sum())


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.normal(size=1000) * 10.0 ** rng.integers(-8, 8, 1000),
                        [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -0.0, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(U.bf16(x), ref)


def test_gradient_matches_central_finite_differences():
    rng = np.random.default_rng(3)
    H, W, C = 32, 64, 8
    p = U.init_params(C=C, seed=4)
    for k in p:
        if k.endswith(".b"):
            p[k] = rng.normal(0, 0.05, p[k].shape)
    x = rng.normal(size=(H, W, 3))
    mask = (rng.random((H, W)) > 0.2).astype(float)
    target = rng.normal(size=(H, W))

    def L(pp):
        out, _ = U.forward(pp, x)
        return U.loss_and_grad_out(out, target, mask)[0]

    out, cache = U.forward(p, x)
    _, dout = U.loss_and_grad_out(out, target, mask)
    g = U.backward(p, cache, dout)
    h = 1e-6
    for name in ["enc1a.w", "enc2b.w", "mid5a.w", "dec4a.w", "dec1b.w", "dec1a.b", "enc3a.b", "out.w", "out.b"]:
        flat = p[name].reshape(-1)
        idx = rng.choice(flat.size, size=min(6, flat.size), replace=False)
        for i in idx:
            save = flat[i]
            flat[i] = save + h
            lp = L(p)
            flat[i] = save - h
            lm = L(p)
            flat[i] = save
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-7, (name, i, fd, an)


def test_adam_first_step_moves_by_lr():
    p = {"a": np.array([1.0, -2.0])}
    g = {"a": np.array([0.5, -3.0])}
    st = {}
    U.adam_step(p, g, st, lr=0.1)
    # first Adam step: m_hat = g, v_hat = g^2 -> update lr * sign(g) (eps aside)
    assert np.allclose(p["a"], [0.9, -1.9], atol=1e-6)


def test_parameter_count():
    p = U.init_params()
    n = sum(v.size for v in p.values())
    assert 150_000 < n < 250_000


def test_bf16_storage_backward_stays_close_to_exact():
    """Rounding the stored data gradients to bfloat16 perturbs each parameter
    gradient by a few bfloat16 ulps at most (relative L2 per tensor)."""
    rng = np.random.default_rng(5)
    H, W, C = 32, 32, 8
    p = U.init_params(C=C, seed=6)
    x = U.bf16(rng.normal(size=(H, W, 3)))
    mask = (rng.random((H, W)) > 0.2).astype(float)
    target = rng.normal(size=(H, W))
    out, cache = U.forward(p, x, round_bf16=True)
    _, dout = U.loss_and_grad_out(out, target, mask)
    g0 = U.backward(p, cache, dout)
    g1 = U.backward(p, cache, dout, round_bf16=True)
    for k in g0:
        err = np.linalg.norm(g1[k] - g0[k]) / max(np.linalg.norm(g0[k]), 1e-30)
        assert err < 2e-2, (k, err)
    assert np.array_equal(g1["out.w"], g0["out.w"])


def test_flatten_round_trip_and_count():
    p = U.init_params(seed=7)
    v = U.flatten(p)
    q = U.unflatten(v)
    assert all(np.array_equal(p[k], q[k]) for k in p)
    # enc1a: 9*32*3 + 32 first, then enc1b starts
    assert np.array_equal(v[:9 * 32 * 3], p["enc1a.w"].ravel())
    assert np.array_equal(v[9 * 32 * 3:9 * 32 * 3 + 32], p["enc1a.b"])
