"""Synthetic workloads shaped after the paper's GEC reference cell.

The paper's runs (Sec. 2, reactor-geometry and circuit paragraphs; Sec. 3,
first paragraph) use a 200x200-cell GEC cell whose drawing (Fig. 1) is not
available, argon cross-section tables that are not available either, and give
no timings.  These workloads are the synthetic stand-ins the method is
measured on.  Every value is plain data; the unit conversions below (mTorr to
Pa, kelvin to eV) are input preparation, not part of the method.

Geometry convention (shared by both implementations): a list of rectangles in
metres ``(r0, r1, z0, z1, kind, cond_id, eps_r)``; a cell takes the last
rectangle that contains its centre; ``kind`` is 0 vacuum, 1 dielectric,
2 conductor; ``cond_id`` 0 is ground, 1 the RF-driven electrode (2, 3, 4
further driven electrodes, whose circuits the optional list
``circuits_more`` gives in order).  ``edge_bc`` gives the conductor id of
the r=R, z=0 and z=Z domain edges, or -1 for a Neumann (symmetry) edge.  The
r=0 edge is the axis.
"""
import copy

MTORR_PA = 133.322368e-3          # 1 mTorr in Pa
KB_OVER_E = 1.380649e-23 / 1.602176634e-19   # kelvin -> eV

VACUUM, DIEL, COND = 0, 1, 2
GROUND, POWERED = 0, 1
NEUMANN = -1

CIRC_IDEAL, CIRC_SERIES_RLC, CIRC_LMATCH = 0, 1, 2
SOLVE_MGPCG_FP64, SOLVE_IR_MG, SOLVE_IR_UNET = 0, 1, 2


def parallel_plate_geometry(nr=32, nz=24, R=0.05, Z=0.0254):
    """Powered plate at z=0, grounded plate at z=Z and grounded wall at r=R."""
    return dict(nr=nr, nz=nz, R=R, Z=Z, regions=[],
                edge_bc=[GROUND, POWERED, GROUND])


def disk_electrode_geometry(nr=32, nz=24, R=0.05, Z=0.0254):
    """Parallel plate with a second driven electrode: powered plate at z=0
    (electrode 1), a disk electrode 2 of radius R/2 one cell thick, two cells
    below the grounded top wall, grounded wall at r=R."""
    dz = Z / nz
    return dict(nr=nr, nz=nz, R=R, Z=Z,
                regions=[(0.0, R / 2, Z - 3 * dz, Z - 2 * dz, COND, 2, 1.0)],
                edge_bc=[GROUND, POWERED, GROUND])


def gec_geometry(refine=1, driven_lower=False):
    """GEC-cell-shaped domain on a 128x256 base grid (refine=1), 512x1024
    (refine=4) or 1024x2048 (refine=8).  With driven_lower the lower
    electrode is a second driven electrode (conductor id 2), lifted one base
    cell off the grounded bottom wall.

    Domain r in [0, 10.16] cm, z in [0, 10.16] cm.  All features lie on
    base-grid edges (base cell 5.08/64 cm in r, 2.54/64 cm in z), so every
    refinement sees the same geometry.
      * grounded lower electrode   r <= 5.08,            z <= 3.81
      * powered upper electrode    r <= 5.08,   6.35 <= z <= 9.525  (gap 2.54)
      * dielectric ring (eps_r 4)  5.08 <= r <= 5.715,  z >= 6.35
      * dielectric cap  (eps_r 4)  r <= 5.715,          z >= 9.525
      * grounded shield            5.715 <= r <= 6.35,  z >= 6.35
      * grounded outer wall r=R and grounded top and bottom walls.
    """
    cm = 1e-2
    R = Z = 10.16 * cm
    big = 1.0
    regions = [
        (5.08 * cm, 5.715 * cm, 6.35 * cm, big, DIEL, -1, 4.0),       # ring
        (0.0, 5.715 * cm, 9.525 * cm, big, DIEL, -1, 4.0),            # cap
        (0.0, 5.08 * cm, 2.54 / 64 * cm if driven_lower else 0.0, 3.81 * cm, COND,
         2 if driven_lower else GROUND, 1.0),                         # lower electrode
        (0.0, 5.08 * cm, 6.35 * cm, 9.525 * cm, COND, POWERED, 1.0),  # powered electrode
        (5.715 * cm, 6.35 * cm, 6.35 * cm, big, COND, GROUND, 1.0),   # shield
    ]
    return dict(nr=128 * refine, nz=256 * refine, R=R, Z=Z, regions=regions,
                edge_bc=[GROUND, GROUND, GROUND])


def _circuit(kind=CIRC_IDEAL, **kw):
    c = dict(kind=kind, freq=13.56e6, U_amp=0.0, U_dc=0.0, R_s=50.0,
             C_m1=0.0, C_m2=0.0, L_m=0.85e-6, R_m=0.5,
             C_stray=10e-12, L_stray=0.01e-6, R_stray=0.5,
             C_b=5e-9, R_b=0.5, L_b=0.01e-6, substeps=8)
    c.update(kw)
    return c


def _lmatch(U_amp):
    # L-type network: C_m1 is the shunt capacitor, C_m2 the series capacitor.
    # Drive level "100 W" read as the power available into 50 ohm:
    # U_s = sqrt(8 * 50 * 100) = 200 V amplitude.
    return _circuit(CIRC_LMATCH, U_amp=U_amp, C_m1=200e-12, C_m2=500e-12)


WORKLOADS = {
    # Plain method, parallel-plate cylinder, 32x24 cells, 20k + 20k particles.
    "pp32x24": dict(
        geometry=parallel_plate_geometry(),
        circuit=_circuit(CIRC_IDEAL, U_amp=100.0),
        gas=dict(p_Pa=20 * MTORR_PA, T_K=300.0),
        run=dict(n_e=20_000, n_i=20_000, cap_e=80_000, cap_i=80_000,
                 n0=1e14, Te_eV=2.0, Ti_eV=0.026, steps_per_period=200,
                 seed=1, sort_every=20, sort_every_ion=20, steps=2000),
        solver=dict(method=SOLVE_MGPCG_FP64, tol=1e-8, max_iter=200),
    ),
    # Two driven electrodes (dual frequency): the plate at 13.56 MHz, a disk
    # electrode at 27.12 MHz.
    "pp32x24x2": dict(
        geometry=disk_electrode_geometry(),
        circuit=_circuit(CIRC_IDEAL, U_amp=100.0),
        circuits_more=[_circuit(CIRC_IDEAL, freq=27.12e6, U_amp=50.0)],
        gas=dict(p_Pa=20 * MTORR_PA, T_K=300.0),
        run=dict(n_e=20_000, n_i=20_000, cap_e=80_000, cap_i=80_000,
                 n0=1e14, Te_eV=2.0, Ti_eV=0.026, steps_per_period=200,
                 seed=1, sort_every=20, sort_every_ion=20, steps=2000),
        solver=dict(method=SOLVE_MGPCG_FP64, tol=1e-8, max_iter=200),
    ),
    # GEC-shaped cell, 128x256, 4M + 4M particles, L-match, plain FP64 MG-PCG.
    "gec128x256": dict(
        geometry=gec_geometry(1),
        circuit=_lmatch(200.0),
        gas=dict(p_Pa=10 * MTORR_PA, T_K=300.0),
        run=dict(n_e=4_000_000, n_i=4_000_000, cap_e=6_000_000, cap_i=6_000_000,
                 n0=1e14, Te_eV=30000 * KB_OVER_E, Ti_eV=300 * KB_OVER_E,
                 steps_per_period=400, seed=1, sort_every=4, sort_every_ion=20, steps=8000),
        solver=dict(method=SOLVE_MGPCG_FP64, tol=1e-8, max_iter=200),
    ),
    # Precision study, 512x1024, 64M + 64M (one sweep point: 20 mTorr, 150 V).
    "gec512x1024": dict(
        geometry=gec_geometry(4),
        circuit=_lmatch(150.0),
        gas=dict(p_Pa=20 * MTORR_PA, T_K=300.0),
        run=dict(n_e=64_000_000, n_i=64_000_000, cap_e=160_000_000, cap_i=160_000_000,
                 n0=1e14, Te_eV=30000 * KB_OVER_E, Ti_eV=300 * KB_OVER_E,
                 steps_per_period=400, seed=1, sort_every=4, sort_every_ion=20, steps=1600),
        solver=dict(method=SOLVE_IR_MG, tol=1e-8, max_iter=200),
    ),
    # Full scale, 1024x2048, 200M + 200M, 300 V with the matching network.
    "gec1024x2048": dict(
        geometry=gec_geometry(8),
        circuit=_lmatch(300.0),
        gas=dict(p_Pa=10 * MTORR_PA, T_K=300.0),
        run=dict(n_e=200_000_000, n_i=200_000_000, cap_e=240_000_000, cap_i=240_000_000,
                 n0=1e14, Te_eV=30000 * KB_OVER_E, Ti_eV=300 * KB_OVER_E,
                 steps_per_period=400, seed=1, sort_every=4, sort_every_ion=20, steps=20000),
        solver=dict(method=SOLVE_IR_MG, tol=1e-8, max_iter=200),
    ),
}

# The sweep of the precision study: (pressure mTorr, source amplitude V).
GEC512_SWEEP = [(5, 50), (20, 150), (50, 300), (5, 300), (50, 50)]


def workload(name, **overrides):
    """A deep copy of a named workload, with nested overrides, e.g.
    ``workload("gec128x256", run={"n_e": 1000, "n_i": 1000})``."""
    w = copy.deepcopy(WORKLOADS[name])
    for k, v in overrides.items():
        if isinstance(v, dict):
            w[k].update(v)
        else:
            w[k] = v
    return w
