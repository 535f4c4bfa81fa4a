"""Seeded random particle sets for parity tests.

Values are drawn with numpy's PCG64 from a seed; they are rounded to FP32
(the particle-state precision of the hot path) so that the oracle (which
widens them to FP64 exactly) and the GPU see bit-identical inputs.
"""
import numpy as np

FIELDS = ("r", "z", "vr", "vt", "vz", "ar", "at", "az", "w")


def random_particles(n, R, Z, seed, vmax=1e6, amax=1e15, wmin=0.5, wmax=2.0,
                     r_lo=0.0, r_hi=None, z_lo=0.0, z_hi=None, dead_frac=0.0):
    """n particles, positions uniform in volume inside [r_lo,r_hi]x[z_lo,z_hi],
    velocities uniform in [-vmax, vmax], accelerations uniform in
    [-amax, amax], relative weights uniform in [wmin, wmax].  A fraction
    ``dead_frac`` gets r = -1 (a dead slot)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r_hi = R if r_hi is None else r_hi
    z_hi = Z if z_hi is None else z_hi
    u = rng.random(n)
    r = np.sqrt(r_lo ** 2 + u * (r_hi ** 2 - r_lo ** 2))
    z = z_lo + rng.random(n) * (z_hi - z_lo)
    out = dict(
        r=r, z=z,
        vr=rng.uniform(-vmax, vmax, n), vt=rng.uniform(-vmax, vmax, n),
        vz=rng.uniform(-vmax, vmax, n),
        ar=rng.uniform(-amax, amax, n), at=rng.uniform(-amax, amax, n),
        az=rng.uniform(-amax, amax, n),
        w=rng.uniform(wmin, wmax, n),
    )
    out = {k: v.astype(np.float32) for k, v in out.items()}
    # keep rounded positions strictly inside the requested box
    out["r"] = np.minimum(out["r"], np.nextafter(np.float32(r_hi), np.float32(0)))
    out["z"] = np.clip(out["z"], np.nextafter(np.float32(z_lo), np.float32(1)),
                       np.nextafter(np.float32(z_hi), np.float32(0)))
    if dead_frac > 0:
        dead = rng.random(n) < dead_frac
        out["r"][dead] = np.float32(-1.0)
    return out
