"""FP64 reference of the learned preconditioner: a 5-level convolutional
U-net on the r-z node image, its backward pass, the loss and Adam.

TEST INFRASTRUCTURE ONLY (parity reference for the HIP training and
inference kernels).  Plain numpy, FP64, written for reading: every 3x3
convolution is the explicit sum over its nine taps.

The network (a learned approximation of K^-1 used as the preconditioner of
flexible CG for Eq. 1):
  input  3 channels: normalised residual r/||r||, susceptibility chi, and the
         mask of unknown nodes; image rows are z, columns are r
  encoder level l = 1..4: conv3x3 + ReLU, conv3x3 + ReLU (-> skip_l), 2x2 average pool
  bottom level 5:         conv3x3 + ReLU, conv3x3 + ReLU
  decoder level l = 4..1: nearest x2 upsample, concat [up, skip_l],
                          conv3x3 + ReLU, conv3x3 + ReLU
  output: 1x1 conv 32 -> 1 (no activation)
Every conv3x3 has C channels out (C = 32 by default), zero padding.
Loss: mean over unknown nodes of (out - target)^2 [R24].
"""
import numpy as np

TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]   # tap index t = (dy+1)*3 + (dx+1)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def layer_specs(C=32, cin=3, levels=5):
    """(name, cin, cout) of every 3x3 convolution, in forward order."""
    specs = []
    c = cin
    for l in range(1, levels):
        specs += [(f"enc{l}a", c, C), (f"enc{l}b", C, C)]
        c = C
    specs += [(f"mid{levels}a", C, C), (f"mid{levels}b", C, C)]
    for l in range(levels - 1, 0, -1):
        specs += [(f"dec{l}a", 2 * C, C), (f"dec{l}b", C, C)]
    return specs


def init_params(C=32, cin=3, levels=5, seed=0):
    """He-normal weights W[t][co][ci] for tap t, zero biases; output 1x1."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, ci, co in layer_specs(C, cin, levels):
        p[name + ".w"] = rng.normal(0, np.sqrt(2.0 / (9 * ci)), (9, co, ci))
        p[name + ".b"] = np.zeros(co)
    p["out.w"] = rng.normal(0, np.sqrt(1.0 / C), C)
    p["out.b"] = np.zeros(1)
    return p


def conv3x3(x, w, b):
    """x[H][W][ci], w[9][co][ci], b[co] -> y[H][W][co]; zero padding."""
    H, W, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (0, 0)))
    y = np.zeros((H, W, w.shape[1])) + b
    for t, (dy, dx) in enumerate(TAPS):
        y += xp[1 + dy:1 + dy + H, 1 + dx:1 + dx + W, :] @ w[t].T
    return y


def conv3x3_backward(x, w, dy):
    """Gradients of y = conv3x3(x, w, b): dx, dw, db."""
    H, W, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (0, 0)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for t, (oy, ox) in enumerate(TAPS):
        xs = xp[1 + oy:1 + oy + H, 1 + ox:1 + ox + W, :]
        dw[t] = np.einsum("hwo,hwi->oi", dy, xs)
        dxp[1 + oy:1 + oy + H, 1 + ox:1 + ox + W, :] += dy @ w[t]
    return dxp[1:H + 1, 1:W + 1, :], dw, dy.sum(axis=(0, 1))


def pool2(x):
    H, W, C = x.shape
    return x.reshape(H // 2, 2, W // 2, 2, C).mean(axis=(1, 3))


def pool2_backward(dy):
    return np.repeat(np.repeat(dy, 2, axis=0), 2, axis=1) / 4.0


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=0), 2, axis=1)


def up2_backward(dy):
    H, W, C = dy.shape
    return dy.reshape(H // 2, 2, W // 2, 2, C).sum(axis=(1, 3))


def forward(p, x, levels=5, round_bf16=False):
    """Forward pass; returns the output image [H][W] and a cache for backward.
    With round_bf16, every stored activation is rounded to bfloat16 (the
    storage precision of the GPU kernels) and weights are used as given."""
    rnd = bf16 if round_bf16 else (lambda a: a)
    cache = {"x": x}
    h = x
    skips = []
    for l in range(1, levels):
        for s in "ab":
            name = f"enc{l}{s}"
            cache[name + ".in"] = h
            h = rnd(np.maximum(conv3x3(h, p[name + ".w"], p[name + ".b"]), 0.0))
            cache[name + ".out"] = h
        skips.append(h)
        h = rnd(pool2(h))
    for s in "ab":
        name = f"mid{levels}{s}"
        cache[name + ".in"] = h
        h = rnd(np.maximum(conv3x3(h, p[name + ".w"], p[name + ".b"]), 0.0))
        cache[name + ".out"] = h
    for l in range(levels - 1, 0, -1):
        h = np.concatenate([up2(h), skips[l - 1]], axis=2)
        for s in "ab":
            name = f"dec{l}{s}"
            cache[name + ".in"] = h
            h = rnd(np.maximum(conv3x3(h, p[name + ".w"], p[name + ".b"]), 0.0))
            cache[name + ".out"] = h
    cache["last"] = h
    out = h @ p["out.w"] + p["out.b"][0]
    return out, cache


def loss_and_grad_out(out, target, mask):
    """MSE over the unknown nodes and its gradient with respect to `out`."""
    n = mask.sum()
    d = (out - target) * mask
    return (d * d).sum() / n, 2.0 * d / n


def backward(p, cache, dout, levels=5, round_bf16=False):
    """Gradients of every parameter given dL/d(out).  With round_bf16, every
    stored activation gradient (the data gradients between layers) is rounded
    to bfloat16, the storage precision of the GPU kernels; parameter
    gradients stay exact sums."""
    rnd = bf16 if round_bf16 else (lambda a: a)
    g = {}
    g["out.w"] = np.einsum("hw,hwc->c", dout, cache["last"])
    g["out.b"] = np.array([dout.sum()])
    dh = rnd(dout[:, :, None] * p["out.w"][None, None, :])
    C = p["out.w"].shape[0]
    dskips = {}
    for l in range(1, levels):
        for s in "ba":
            name = f"dec{l}{s}"
            dpre = dh * (cache[name + ".out"] > 0)
            dh, g[name + ".w"], g[name + ".b"] = conv3x3_backward(cache[name + ".in"], p[name + ".w"], dpre)
            dh = rnd(dh)
        dskips[l] = dh[:, :, C:]
        dh = rnd(up2_backward(dh[:, :, :C]))
    for s in "ba":
        name = f"mid{levels}{s}"
        dpre = dh * (cache[name + ".out"] > 0)
        dh, g[name + ".w"], g[name + ".b"] = conv3x3_backward(cache[name + ".in"], p[name + ".w"], dpre)
        dh = rnd(dh)
    for l in range(levels - 1, 0, -1):
        dh = rnd(pool2_backward(dh) + dskips[l])
        for s in "ba":
            name = f"enc{l}{s}"
            dpre = dh * (cache[name + ".out"] > 0)
            dh, g[name + ".w"], g[name + ".b"] = conv3x3_backward(cache[name + ".in"], p[name + ".w"], dpre)
            dh = rnd(dh)
    return g


def adam_step(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma & Ba 2015) with bias correction, in place on p."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m." + k, np.zeros_like(p[k]))
        v = state.setdefault("v." + k, np.zeros_like(p[k]))
        m[:] = b1 * m + (1 - b1) * g[k]
        v[:] = b2 * v + (1 - b2) * g[k] * g[k]
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def flatten(p, levels=5):
    """Parameters in the flat order of the GPU library: per 3x3 convolution
    w[9][cout][cin] then b[cout], in forward order; then out.w, out.b."""
    parts = []
    for name, _, _ in layer_specs(p["out.w"].shape[0], p["enc1a.w"].shape[2], levels):
        parts += [p[name + ".w"].ravel(), p[name + ".b"].ravel()]
    parts += [p["out.w"].ravel(), p["out.b"].ravel()]
    return np.concatenate(parts)


def unflatten(v, C=32, cin=3, levels=5):
    """Inverse of flatten."""
    p, o = {}, 0
    for name, ci, co in layer_specs(C, cin, levels):
        p[name + ".w"] = np.asarray(v[o:o + 9 * co * ci], dtype=np.float64).reshape(9, co, ci)
        o += 9 * co * ci
        p[name + ".b"] = np.asarray(v[o:o + co], dtype=np.float64)
        o += co
    p["out.w"] = np.asarray(v[o:o + C], dtype=np.float64)
    p["out.b"] = np.asarray(v[o + C:o + C + 1], dtype=np.float64)
    assert o + C + 1 == len(v)
    return p
