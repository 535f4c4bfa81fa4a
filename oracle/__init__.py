"""Python (ctypes) wrapper of the plain FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg.  It never imports the HIP package; both take
their configuration from the plain-data workloads in ``pic_inputs``.
"""
import ctypes as C
import os

import numpy as np

from .build import LIB, build

FIELDS = ("r", "z", "vr", "vt", "vz", "ar", "at", "az", "w")
G = dict(DEP_E=0, DEP_I=1, PHI=2, ER=3, EZ=4, CHI=5, WALLQ=6, NODE_KIND=7, CELL_KIND=8,
         VOL=9, PHI_L=10, Q=11, AR=12, AZ=13, NE_AVG=14, NI_AVG=15)
MAX_REGIONS = 32
MAX_EL = 4
CIRC_FIELDS = ("freq", "U_amp", "U_dc", "R_s", "C_m1", "C_m2", "L_m", "R_m", "C_stray", "L_stray", "R_stray",
               "C_b", "R_b", "L_b")


class Region(C.Structure):
    _fields_ = [("r0", C.c_double), ("r1", C.c_double), ("z0", C.c_double), ("z1", C.c_double),
                ("kind", C.c_int32), ("cond_id", C.c_int32), ("eps_r", C.c_double)]


class Circ(C.Structure):
    _fields_ = [("kind", C.c_int32), ("substeps", C.c_int32)] + [(f, C.c_double) for f in CIRC_FIELDS]


class Config(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nz", C.c_int32), ("R", C.c_double), ("Z", C.c_double),
                ("n_regions", C.c_int32), ("edge_bc", C.c_int32 * 3),
                ("regions", Region * MAX_REGIONS),
                ("circ_kind", C.c_int32), ("substeps", C.c_int32),
                ("freq", C.c_double), ("U_amp", C.c_double), ("U_dc", C.c_double), ("R_s", C.c_double),
                ("C_m1", C.c_double), ("C_m2", C.c_double), ("L_m", C.c_double), ("R_m", C.c_double),
                ("C_stray", C.c_double), ("L_stray", C.c_double), ("R_stray", C.c_double),
                ("C_b", C.c_double), ("R_b", C.c_double), ("L_b", C.c_double),
                ("p_Pa", C.c_double), ("T_gas_K", C.c_double),
                ("n_e", C.c_int64), ("n_i", C.c_int64), ("cap_e", C.c_int64), ("cap_i", C.c_int64),
                ("n0", C.c_double), ("Te_eV", C.c_double), ("Ti_eV", C.c_double),
                ("steps_per_period", C.c_int32), ("sort_every", C.c_int32), ("sort_every_ion", C.c_int32),
                ("seed", C.c_uint64), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("load", C.c_int32), ("weights", C.c_int32), ("split", C.c_int32),
                ("n_el", C.c_int32), ("circ_el", Circ * (MAX_EL - 1))]


class Diag(C.Structure):
    _fields_ = [("t", C.c_double), ("U_E", C.c_double), ("Q_E", C.c_double), ("C_eq", C.c_double),
                ("Q_P", C.c_double), ("I_ccp", C.c_double), ("dt", C.c_double), ("w_unit", C.c_double),
                ("n_gas", C.c_double), ("circ", C.c_double * 5), ("nu_max", C.c_double * 2),
                ("thresh", C.c_uint32 * 2), ("step", C.c_int64), ("periods_done", C.c_int64),
                ("n_slots", C.c_int64 * 2), ("n_alive", C.c_int64 * 2),
                ("absorbed", (C.c_int64 * 4) * 2), ("born", C.c_int64), ("coll", (C.c_int64 * 4) * 2),
                ("numax_violations", C.c_int64), ("solver_iters", C.c_int64),
                ("solver_relres", C.c_double),
                ("harm_U_re", C.c_double * 6), ("harm_U_im", C.c_double * 6),
                ("harm_I_re", C.c_double * 6), ("harm_I_im", C.c_double * 6), ("elec", C.c_double * 12),
                ("split_added", C.c_int64 * 2),
                ("n_el", C.c_int32), ("U_el", C.c_double * MAX_EL), ("Q_el", C.c_double * MAX_EL),
                ("QP_el", C.c_double * MAX_EL), ("I_el", C.c_double * MAX_EL),
                ("C_el", C.c_double * (MAX_EL * MAX_EL)),
                ("hU_re", (C.c_double * 6) * MAX_EL), ("hU_im", (C.c_double * 6) * MAX_EL),
                ("hI_re", (C.c_double * 6) * MAX_EL), ("hI_im", (C.c_double * 6) * MAX_EL),
                ("absorbed_el", (C.c_int64 * MAX_EL) * 2)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(Config), C.POINTER(P)]
        L.orc_destroy.argtypes = [P]
        L.orc_step.argtypes = [P, C.c_int32]
        L.orc_diag_get.argtypes = [P, C.POINTER(Diag)]
        L.orc_series.argtypes = [P, C.c_int32, P, P]
        L.orc_num_slots.argtypes = [P, C.c_int32]
        L.orc_num_slots.restype = C.c_int64
        L.orc_get_particles.argtypes = [P, C.c_int32, P]
        L.orc_set_particles.argtypes = [P, C.c_int32, C.c_int64, P]
        L.orc_redeposit.argtypes = [P]
        L.orc_get_grid.argtypes = [P, C.c_int32, P]
        L.orc_set_grid.argtypes = [P, C.c_int32, P]
        L.orc_set_state.argtypes = [P, P]
        L.orc_solve_q.argtypes = [P, P, P, C.c_double, C.c_double, P, C.POINTER(C.c_int32),
                                  C.POINTER(C.c_double)]
        L.orc_refresh_laplace.argtypes = [P]
        L.orc_refresh_laplace.restype = C.c_double
        L.orc_ceq_flux.argtypes = [P]
        L.orc_ceq_flux.restype = C.c_double
        L.orc_deposit.argtypes = [P, C.c_int64, P, P, P, P]
        L.orc_tile_keys.argtypes = [P, C.c_int64, P, P, P]
        L.orc_stable_perm.argtypes = [C.c_int64, P, P]
        L.orc_predict.argtypes = [P, C.c_int64, P]
        L.orc_correct.argtypes = [P, C.c_int32, C.c_int64, P, P, P]
        L.orc_mcc.argtypes = [P, C.c_int32, C.c_int64, P, C.c_uint32, C.c_uint32, P, P]
        L.orc_philox4x32.argtypes = [P, P, P]
        L.orc_philox4x64.argtypes = [P, P, P]
        L.orc_xsec_e.argtypes = [C.c_double, P]
        L.orc_circuit_vacuum.argtypes = [C.POINTER(Config), C.c_double, C.c_int64, P, P, P]
        L.orc_moments.argtypes = [P, C.c_int, P, P]
        L.orc_reflection.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, P]
        L.orc_split_now.argtypes = [P, C.c_int32, C.POINTER(C.c_int64)]
        L.orc_solve_qv.argtypes = [P, P, P, P, C.c_double, P, C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.orc_get_phiL.argtypes = [P, C.c_int32, P]
        L.orc_split_target.argtypes = [P, C.c_int32, C.c_int32]
        L.orc_split_target.restype = C.c_double
        L.orc_match_design.argtypes = [C.POINTER(Config), C.c_double, P]
        L.orc_assemble_now.argtypes = [P]
        L.orc_efield_now.argtypes = [P]
        L.orc_gather.argtypes = [P, C.c_int64, P, P, P, P]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def make_config(w, load=True):
    """Marshal a workload dict (see pic_inputs.workloads) into the oracle's struct."""
    g, c, gas, run, sol = w["geometry"], w["circuit"], w["gas"], w["run"], w["solver"]
    cfg = Config()
    cfg.nr, cfg.nz, cfg.R, cfg.Z = g["nr"], g["nz"], g["R"], g["Z"]
    regs = g["regions"]
    if len(regs) > MAX_REGIONS:
        raise ValueError("too many regions")
    cfg.n_regions = len(regs)
    for k, e in enumerate(g["edge_bc"]):
        cfg.edge_bc[k] = e
    for k, (r0, r1, z0, z1, kind, cid, eps) in enumerate(regs):
        cfg.regions[k] = Region(r0, r1, z0, z1, kind, cid, eps)
    cfg.circ_kind = c["kind"]
    cfg.substeps = c["substeps"]
    for f in ("freq", "U_amp", "U_dc", "R_s", "C_m1", "C_m2", "L_m", "R_m", "C_stray", "L_stray",
              "R_stray", "C_b", "R_b", "L_b"):
        setattr(cfg, f, c[f])
    cfg.p_Pa, cfg.T_gas_K = gas["p_Pa"], gas["T_K"]
    for f in ("n_e", "n_i", "cap_e", "cap_i", "n0", "Te_eV", "Ti_eV", "steps_per_period",
              "sort_every", "sort_every_ion", "seed"):
        setattr(cfg, f, run[f])
    cfg.tol, cfg.max_iter = sol["tol"], sol["max_iter"]
    cfg.load = 1 if load else 0
    cfg.weights = run.get("weights", 0)
    cfg.split = run.get("split", 0)
    more = w.get("circuits_more", [])
    if len(more) > MAX_EL - 1:
        raise ValueError("too many driven electrodes")
    cfg.n_el = 1 + len(more)
    for e, ce in enumerate(more):
        cfg.circ_el[e].kind, cfg.circ_el[e].substeps = ce["kind"], ce["substeps"]
        for f in CIRC_FIELDS:
            setattr(cfg.circ_el[e], f, ce[f])
    return cfg


class Oracle:
    """One oracle simulation (plain FP64 CPU)."""

    def __init__(self, w, load=True):
        self.w = w
        self.cfg = make_config(w, load)
        self.h = C.c_void_p()
        rc = lib().orc_create(C.byref(self.cfg), C.byref(self.h))
        if rc != 0:
            raise RuntimeError(f"orc_create failed ({rc})")
        g = w["geometry"]
        self.nr, self.nz = g["nr"], g["nz"]
        self.nn = (self.nr + 1) * (self.nz + 1)
        self.spp = w["run"]["steps_per_period"]

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def step(self, n=1):
        rc = lib().orc_step(self.h, n)
        if rc != 0:
            raise RuntimeError(f"orc_step failed ({rc})")

    def diag(self):
        d = Diag()
        lib().orc_diag_get(self.h, C.byref(d))
        return d

    def series(self, last=True):
        U = np.zeros(self.spp)
        I = np.zeros(self.spp)
        lib().orc_series(self.h, 1 if last else 0, _ptr(U), _ptr(I))
        return U, I

    def particles(self, sp):
        n = lib().orc_num_slots(self.h, sp)
        a = np.zeros(9 * max(n, 1))
        lib().orc_get_particles(self.h, sp, _ptr(a))
        return {f: a[k * n:(k + 1) * n].copy() for k, f in enumerate(FIELDS)}

    def set_particles(self, sp, p):
        n = len(p["r"])
        a = np.concatenate([np.asarray(p[f], dtype=np.float64) for f in FIELDS]) if n else np.zeros(9)
        rc = lib().orc_set_particles(self.h, sp, n, _ptr(a))
        if rc != 0:
            raise RuntimeError("set_particles failed")

    def redeposit(self):
        lib().orc_redeposit(self.h)

    def grid(self, name):
        which = G[name]
        if name == "CELL_KIND":
            a = np.zeros(self.nr * self.nz, dtype=np.int32)
        elif name == "NODE_KIND":
            a = np.zeros(self.nn, dtype=np.int32)
        elif name in ("DEP_E", "DEP_I", "WALLQ"):
            a = np.zeros(self.nn, dtype=np.int64)
        else:
            a = np.zeros(self.nn, dtype=np.float64)
        lib().orc_get_grid(self.h, which, _ptr(a))
        return a

    def set_grid(self, name, a):
        dt = np.int64 if name in ("DEP_E", "DEP_I", "WALLQ") else np.float64
        a = np.ascontiguousarray(a, dtype=dt)
        if lib().orc_set_grid(self.h, G[name], _ptr(a)) != 0:
            raise ValueError(name)

    def set_state(self, t, Q_E, U_E, circ, C_eq):
        st = np.array([t, Q_E, U_E] + list(circ) + [C_eq], dtype=np.float64)
        lib().orc_set_state(self.h, _ptr(st))

    def assemble_now(self):
        """CHI and Q grids from the deposit grids as they stand (Eq. 1)."""
        lib().orc_assemble_now(self.h)

    def efield_now(self):
        """ER and EZ grids from the PHI grid as it stands (reading R9)."""
        lib().orc_efield_now(self.h)

    def gather(self, r, z):
        """(E_r, E_z) the particle step gathers at the given positions."""
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.ascontiguousarray(z, dtype=np.float64)
        Er = np.zeros(len(r))
        Ez = np.zeros(len(r))
        lib().orc_gather(self.h, len(r), _ptr(r), _ptr(z), _ptr(Er), _ptr(Ez))
        return Er, Ez

    def solve_q(self, Q, chi, U_E, tol=1e-12, phi0=None):
        Q = np.ascontiguousarray(Q, dtype=np.float64)
        chi = np.ascontiguousarray(chi, dtype=np.float64)
        phi = np.zeros(self.nn) if phi0 is None else np.array(phi0, dtype=np.float64)
        it = C.c_int32()
        rel = C.c_double()
        rc = lib().orc_solve_q(self.h, _ptr(Q), _ptr(chi), U_E, tol, _ptr(phi), C.byref(it), C.byref(rel))
        return phi, it.value, rel.value, rc

    def solve_qv(self, Q, chi, U, tol=1e-12, phi0=None):
        """One solve with driven electrode e at U[e - 1] (reading R33)."""
        Q = np.ascontiguousarray(Q, dtype=np.float64)
        chi = np.ascontiguousarray(chi, dtype=np.float64)
        Uv = np.zeros(MAX_EL)
        Uv[:len(U)] = U
        phi = np.zeros(self.nn) if phi0 is None else np.array(phi0, dtype=np.float64)
        it = C.c_int32()
        rel = C.c_double()
        rc = lib().orc_solve_qv(self.h, _ptr(Q), _ptr(chi), _ptr(Uv), tol, _ptr(phi), C.byref(it), C.byref(rel))
        return phi, it.value, rel.value, rc

    def phi_laplace(self, e):
        """Laplace solution of driven electrode e (1-based) at 1 V, the others grounded."""
        a = np.zeros(self.nn)
        if lib().orc_get_phiL(self.h, e, _ptr(a)) != 0:
            raise ValueError(e)
        return a

    def capacitance(self):
        """n_el x n_el capacitance matrix (reading R33)."""
        d = self.diag()
        m = d.n_el
        return np.array(d.C_el[:]).reshape(MAX_EL, MAX_EL)[:m, :m]

    def refresh_laplace(self):
        return lib().orc_refresh_laplace(self.h)

    def ceq_flux(self):
        return lib().orc_ceq_flux(self.h)

    def deposit(self, r, z, w):
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.ascontiguousarray(z, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        g = np.zeros(self.nn, dtype=np.int64)
        lib().orc_deposit(self.h, len(r), _ptr(r), _ptr(z), _ptr(w), _ptr(g))
        return g

    def moments(self, sp):
        """(N, E) int64 node grids: weight shares and shares x floor(16 eps/eV)."""
        N = np.zeros(self.nn, dtype=np.int64)
        E = np.zeros(self.nn, dtype=np.int64)
        lib().orc_moments(self.h, sp, _ptr(N), _ptr(E))
        return N, E

    def split_now(self, sp):
        """One splitting pass over species sp (reading R32); returns the copies added."""
        added = C.c_int64()
        rc = lib().orc_split_now(self.h, sp, C.byref(added))
        if rc != 0:
            raise RuntimeError(f"orc_split_now failed ({rc})")
        return added.value

    def split_target(self, sp, i):
        """Reference weight of cell column i (units of w_unit), reading R32."""
        return lib().orc_split_target(self.h, sp, i)

    def tile_keys(self, r, z):
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.ascontiguousarray(z, dtype=np.float64)
        k = np.zeros(len(r), dtype=np.uint32)
        lib().orc_tile_keys(self.h, len(r), _ptr(r), _ptr(z), _ptr(k))
        return k

    def predict(self, p):
        n = len(p["r"])
        a = np.concatenate([np.asarray(p[f], dtype=np.float64) for f in FIELDS])
        lib().orc_predict(self.h, n, _ptr(a))
        return {f: a[k * n:(k + 1) * n].copy() for k, f in enumerate(FIELDS)}

    def correct(self, sp, p, Er, Ez):
        n = len(p["r"])
        a = np.concatenate([np.asarray(p[f], dtype=np.float64) for f in FIELDS])
        Er = np.ascontiguousarray(Er, dtype=np.float64)
        Ez = np.ascontiguousarray(Ez, dtype=np.float64)
        lib().orc_correct(self.h, sp, n, _ptr(a), _ptr(Er), _ptr(Ez))
        return {f: a[k * n:(k + 1) * n].copy() for k, f in enumerate(FIELDS)}

    def mcc(self, sp, v, slot0, step):
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3).copy()
        n = v.shape[0]
        proc = np.zeros(n, dtype=np.int32)
        b = np.zeros((n, 6))
        lib().orc_mcc(self.h, sp, n, _ptr(v), slot0, step, _ptr(proc), _ptr(b))
        return v, proc, b


def stable_perm(keys):
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    perm = np.zeros(len(keys), dtype=np.int64)
    lib().orc_stable_perm(len(keys), _ptr(keys), _ptr(perm))
    return perm


def philox4x32(ctr, key):
    c = np.array(ctr, dtype=np.uint32)
    k = np.array(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32(_ptr(c), _ptr(k), _ptr(o))
    return o


def philox4x64(ctr, key):
    c = np.array(ctr, dtype=np.uint64)
    k = np.array(key, dtype=np.uint64)
    o = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64(_ptr(c), _ptr(k), _ptr(o))
    return o


def xsec_e(eps):
    o = np.zeros(3)
    lib().orc_xsec_e(eps, _ptr(o))
    return o


ELEC = ("Z_ccp_re", "Z_ccp_im", "Z_load_re", "Z_load_im", "gamma", "P_source", "P_Rs", "P_IMN", "P_stray",
        "P_ccp", "P_forward", "P_ref")


def elec_dict(a):
    """The 12 electrical-characterisation numbers as a dict (Eqs. 11-14)."""
    return dict(zip(ELEC, [float(v) for v in a]))


def reflection(Z_load, R_s, P_source, P_Rs):
    """|Gamma| (Eq. 12), P_forward and P_ref (Eq. 14)."""
    out = np.zeros(3)
    lib().orc_reflection(Z_load.real, Z_load.imag, R_s, P_source, P_Rs, _ptr(out))
    return tuple(float(v) for v in out)


def match_design(w, C_eq):
    """(C_m1, C_m2) of the workload's L-network matching the load C_eq (Sec. 3)."""
    cfg = make_config(w, load=False)
    out = np.zeros(2)
    rc = lib().orc_match_design(C.byref(cfg), C_eq, _ptr(out))
    if rc != 0:
        raise ValueError("no matching network for this load")
    return float(out[0]), float(out[1])


def circuit_vacuum(w, C_eq, nsteps, chars=False):
    """The circuit alone with a fixed C_eq: U_E and I series, and with
    chars the electrical characterisation of the last period."""
    cfg = make_config(w, load=False)
    U = np.zeros(nsteps)
    I = np.zeros(nsteps)
    e = np.zeros(12)
    lib().orc_circuit_vacuum(C.byref(cfg), C_eq, nsteps, _ptr(U), _ptr(I), _ptr(e))
    return (U, I, elec_dict(e)) if chars else (U, I)
