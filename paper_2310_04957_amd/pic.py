"""Thin Python binding of the C ABI in include/pic.h (argument marshalling only).

Every step of the method runs in the HIP kernels of libpic.so.  PyTorch
supplies the device workspace and the stream.  There is no CPU fallback: if
the library or a gfx950 device is missing, construction raises.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

ABI_VERSION = 2
MAX_REGIONS = 32
FIELDS = ("r", "z", "vr", "vt", "vz", "ar", "at", "az", "w")
SOLVE_MGPCG_FP64, SOLVE_IR_MG, SOLVE_IR_UNET, SOLVE_IR_CG = 0, 1, 2, 3
WEIGHTS_EQUAL, WEIGHTS_CELL = 0, 1
GRIDS = dict(DEP_E=0, DEP_I=1, PHI=2, ER=3, EZ=4, CHI=5, WALLQ=6, PHI_L=10, Q=11, AR=12, AZ=13,
             PHI_L2=14, PHI_L3=15, PHI_L4=16)
MAX_EL = 4
PIC_NOALLOC_MAX_NODES = 1025 * 2049     # nodes of the allocation-free entry points
ERRORS = {0: "ok", -1: "PIC_E_CONFIG", -2: "PIC_E_CAPACITY", -3: "PIC_E_SOLVER", -4: "PIC_E_HIP",
          -5: "PIC_E_NONFINITE", -6: "PIC_E_STATE", -7: "PIC_E_ARG", -8: "PIC_E_NODEVICE", -9: "PIC_E_TOOBIG"}


class PicError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({code})")
        self.code = code


class Region(C.Structure):
    _fields_ = [("r0", C.c_double), ("r1", C.c_double), ("z0", C.c_double), ("z1", C.c_double),
                ("kind", C.c_int32), ("cond_id", C.c_int32), ("eps_r", C.c_double)]


class Geometry(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nz", C.c_int32), ("R", C.c_double), ("Z", C.c_double),
                ("n_regions", C.c_int32), ("edge_bc", C.c_int32 * 3), ("regions", Region * MAX_REGIONS)]


class Circuit(C.Structure):
    _fields_ = [("kind", C.c_int32), ("substeps", C.c_int32)] + [
        (f, C.c_double) for f in ("freq", "U_amp", "U_dc", "R_s", "C_m1", "C_m2", "L_m", "R_m", "C_stray",
                                  "L_stray", "R_stray", "C_b", "R_b", "L_b")]


class Gas(C.Structure):
    _fields_ = [("p_Pa", C.c_double), ("T_gas_K", C.c_double)]


class Run(C.Structure):
    _fields_ = [("n_e", C.c_int64), ("n_i", C.c_int64), ("cap_e", C.c_int64), ("cap_i", C.c_int64),
                ("n0", C.c_double), ("Te_eV", C.c_double), ("Ti_eV", C.c_double),
                ("steps_per_period", C.c_int32), ("sort_every", C.c_int32), ("sort_every_ion", C.c_int32),
                ("seed", C.c_uint64),
                ("load", C.c_int32), ("timing", C.c_int32), ("weights", C.c_int32), ("split", C.c_int32)]


class Solver(C.Structure):
    _fields_ = [("method", C.c_int32), ("tol", C.c_double), ("max_iter", C.c_int32), ("inner_tol", C.c_double),
                ("unet_batch", C.c_int32), ("unet_pairs", C.c_int32), ("graphs", C.c_int32)]


class Config(C.Structure):
    _fields_ = [("abi_version", C.c_int32), ("geom", Geometry), ("circ", Circuit), ("gas", Gas), ("run", Run),
                ("solver", Solver), ("n_el", C.c_int32), ("circ_el", Circuit * (MAX_EL - 1))]


class Diag(C.Structure):
    _fields_ = [(f, C.c_double) for f in ("t", "U_E", "Q_E", "C_eq", "Q_P", "I_ccp", "dt", "w_unit", "n_gas")] + [
        ("circ", C.c_double * 5), ("nu_max", C.c_double * 2), ("thresh", C.c_uint32 * 2),
        ("step", C.c_int64), ("periods_done", C.c_int64), ("n_slots", C.c_int64 * 2), ("n_alive", C.c_int64 * 2),
        ("absorbed", (C.c_int64 * 4) * 2), ("born", C.c_int64), ("coll", (C.c_int64 * 4) * 2),
        ("numax_violations", C.c_int64), ("solver_iters", C.c_int64), ("solver_outer", C.c_int64),
        ("solver_relres", C.c_double),
        ("harm_U_re", C.c_double * 6), ("harm_U_im", C.c_double * 6),
        ("harm_I_re", C.c_double * 6), ("harm_I_im", C.c_double * 6),
        ("ms_particles", C.c_double * 2), ("ms_births", C.c_double), ("ms_sort", C.c_double),
        ("ms_field", C.c_double), ("ms_refresh", C.c_double),
        ("timed_steps", C.c_int64), ("deposit_fallback", C.c_int64), ("error", C.c_int32),
        ("unet_pairs", C.c_int64), ("unet_fallbacks", C.c_int64), ("unet_applications", C.c_int64)] + [
        (f, C.c_double) for f in ("Z_ccp_re", "Z_ccp_im", "Z_load_re", "Z_load_im", "gamma_abs", "P_source",
                                  "P_Rs", "P_imn", "P_stray", "P_ccp", "P_forward", "P_ref")] + [
        ("split_added", C.c_int64 * 2),
        ("n_el", C.c_int32), ("U_el", C.c_double * MAX_EL), ("Q_el", C.c_double * MAX_EL),
        ("QP_el", C.c_double * MAX_EL), ("I_el", C.c_double * MAX_EL), ("C_el", C.c_double * (MAX_EL * MAX_EL)),
        ("hU_re", (C.c_double * 6) * MAX_EL), ("hU_im", (C.c_double * 6) * MAX_EL),
        ("hI_re", (C.c_double * 6) * MAX_EL), ("hI_im", (C.c_double * 6) * MAX_EL),
        ("absorbed_el", (C.c_int64 * MAX_EL) * 2), ("unet_disabled", C.c_int32), ("capacity_bits", C.c_int32)]


class DiagBuffers(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in ("n_e", "n_i", "phi", "U_E", "I_ccp")]


_lib = None


def lib():
    """Load libpic.so; raise if it was not built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2310_04957_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.pic_workspace_size.argtypes = [C.POINTER(Config), C.POINTER(C.c_size_t)]
        L.pic_init.argtypes = [C.POINTER(Config), P, C.c_size_t, P, C.POINTER(P)]
        L.pic_step.argtypes = [P, C.c_int32]
        L.pic_diag.argtypes = [P, C.POINTER(Diag), C.POINTER(DiagBuffers)]
        L.pic_reset_timers.argtypes = [P]
        L.pic_free.argtypes = [P]
        L.pic_strerror.argtypes = [C.c_int]
        L.pic_strerror.restype = C.c_char_p
        L.pic_get_particles.argtypes = [P, C.c_int32, P, C.POINTER(C.c_int64)]
        L.pic_set_particles.argtypes = [P, C.c_int32, P, C.c_int64]
        L.pic_get_grid.argtypes = [P, C.c_int32, P]
        L.pic_set_grid.argtypes = [P, C.c_int32, P]
        L.pic_redeposit.argtypes = [P]
        L.pic_sort_now.argtypes = [P, C.c_int32, P]
        L.pic_split_now.argtypes = [P, C.c_int32, C.POINTER(C.c_int64)]
        L.pic_solve_once_el.argtypes = [P, P, P, P, C.c_double, P, C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.pic_solve_once.argtypes = [P, P, P, C.c_double, C.c_double, P, C.POINTER(C.c_int32),
                                     C.POINTER(C.c_double)]
        L.pic_set_state.argtypes = [P, P]
        L.pic_match_design.argtypes = [P, C.c_int32, P]
        L.pic_set_solver.argtypes = [P, C.POINTER(Solver)]
        L.pic_moments.argtypes = [P, C.c_int32, P, P]
        L.pic_moments_noalloc.argtypes = [P, C.c_int32, P, P]
        L.pic_unet_num_params.argtypes = [P, C.POINTER(C.c_int64)]
        L.pic_unet_set_params.argtypes = [P, P, C.c_int64]
        L.pic_unet_get_params.argtypes = [P, P, C.c_int64]
        L.pic_unet_forward.argtypes = [P, P, C.c_int32, P]
        L.pic_unet_grads.argtypes = [P, P, P, P, C.c_int32, P, C.POINTER(C.c_double)]
        L.pic_unet_harvest.argtypes = [P, C.c_int32]
        L.pic_unet_get_pair.argtypes = [P, C.c_int32, P, P, P, P]
        L.pic_unet_put_pair.argtypes = [P, C.c_int32, P, P, P]
        L.pic_unet_train.argtypes = [P, C.c_int32, C.c_int32, C.c_double, C.c_uint64, P]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _check(rc, where):
    if rc != 0:
        raise PicError(rc, where)


def make_config(w, load=True, timing=False, method=None, inner_tol=1e-4, unet_batch=0, unet_pairs=0,
                graphs=False):
    """Marshal a workload dict (pic_inputs.workloads) into pic_config."""
    g, c, gas, run, sol = w["geometry"], w["circuit"], w["gas"], w["run"], w["solver"]
    cfg = Config()
    cfg.abi_version = ABI_VERSION
    cfg.geom.nr, cfg.geom.nz, cfg.geom.R, cfg.geom.Z = g["nr"], g["nz"], g["R"], g["Z"]
    if len(g["regions"]) > MAX_REGIONS:
        raise ValueError("too many regions")
    cfg.geom.n_regions = len(g["regions"])
    for k, e in enumerate(g["edge_bc"]):
        cfg.geom.edge_bc[k] = e
    for k, (r0, r1, z0, z1, kind, cid, eps) in enumerate(g["regions"]):
        cfg.geom.regions[k] = Region(r0, r1, z0, z1, kind, cid, eps)
    cfg.circ.kind, cfg.circ.substeps = c["kind"], c["substeps"]
    for f in ("freq", "U_amp", "U_dc", "R_s", "C_m1", "C_m2", "L_m", "R_m", "C_stray", "L_stray", "R_stray",
              "C_b", "R_b", "L_b"):
        setattr(cfg.circ, f, c[f])
    cfg.gas.p_Pa, cfg.gas.T_gas_K = gas["p_Pa"], gas["T_K"]
    for f in ("n_e", "n_i", "cap_e", "cap_i", "n0", "Te_eV", "Ti_eV", "steps_per_period", "sort_every",
              "sort_every_ion", "seed"):
        setattr(cfg.run, f, run[f])
    cfg.run.load = 1 if load else 0
    cfg.run.timing = 1 if timing else 0
    cfg.run.weights = run.get("weights", 0)
    cfg.run.split = run.get("split", 0)
    cfg.solver.method = sol["method"] if method is None else method
    cfg.solver.tol, cfg.solver.max_iter = sol["tol"], sol["max_iter"]
    cfg.solver.inner_tol = inner_tol
    cfg.solver.unet_batch = unet_batch
    cfg.solver.unet_pairs = unet_pairs
    cfg.solver.graphs = 1 if graphs else 0
    more = w.get("circuits_more", [])
    if len(more) > MAX_EL - 1:
        raise ValueError("too many driven electrodes")
    cfg.n_el = 1 + len(more)
    for e, ce in enumerate(more):
        cfg.circ_el[e].kind, cfg.circ_el[e].substeps = ce["kind"], ce["substeps"]
        for f in ("freq", "U_amp", "U_dc", "R_s", "C_m1", "C_m2", "L_m", "R_m", "C_stray", "L_stray", "R_stray",
                  "C_b", "R_b", "L_b"):
            setattr(cfg.circ_el[e], f, ce[f])
    return cfg


def workspace_bytes(cfg):
    n = C.c_size_t()
    _check(lib().pic_workspace_size(C.byref(cfg), C.byref(n)), "pic_workspace_size")
    return n.value


class Pic:
    """One simulation on the current HIP device and stream."""

    def __init__(self, w, load=True, timing=False, method=None, inner_tol=1e-4, device="cuda:0", unet_batch=0,
                 unet_pairs=0, graphs=False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP path has no CPU fallback")
        self.w = w
        self.cfg = make_config(w, load, timing, method, inner_tol, unet_batch, unet_pairs, graphs)
        L = lib()
        nbytes = workspace_bytes(self.cfg)
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.h = C.c_void_p()
        _check(L.pic_init(C.byref(self.cfg), C.c_void_p(self.ws.data_ptr()), nbytes + 256,
                          C.c_void_p(self.stream.cuda_stream), C.byref(self.h)), "pic_init")
        g = w["geometry"]
        self.nr, self.nz = g["nr"], g["nz"]
        self.nn = (self.nr + 1) * (self.nz + 1)
        self.spp = w["run"]["steps_per_period"]
        self.cap = (w["run"]["cap_e"], w["run"]["cap_i"])

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().pic_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        _check(lib().pic_step(self.h, n), "pic_step")

    def diag(self, grids=False):
        d = Diag()
        bufs = None
        out = {}
        if grids:
            out = dict(n_e=np.zeros(self.nn), n_i=np.zeros(self.nn), phi=np.zeros(self.nn),
                       U_E=np.zeros(self.spp), I_ccp=np.zeros(self.spp))
            bufs = DiagBuffers(*[_ptr(out[k]).value for k in ("n_e", "n_i", "phi", "U_E", "I_ccp")])
        _check(lib().pic_diag(self.h, C.byref(d), C.byref(bufs) if bufs is not None else None), "pic_diag")
        return (d, out) if grids else d

    def reset_timers(self):
        _check(lib().pic_reset_timers(self.h), "pic_reset_timers")

    def particles(self, sp):
        cap = self.cap[sp]
        a = np.zeros(9 * max(cap, 1), dtype=np.float32)
        n = C.c_int64()
        _check(lib().pic_get_particles(self.h, sp, _ptr(a), C.byref(n)), "pic_get_particles")
        n = n.value
        return {f: a[k * cap:k * cap + n].copy() for k, f in enumerate(FIELDS)}

    def set_particles(self, sp, p):
        n = len(p["r"])
        a = np.concatenate([np.asarray(p[f], dtype=np.float32) for f in FIELDS]) if n else np.zeros(9, np.float32)
        _check(lib().pic_set_particles(self.h, sp, _ptr(a), n), "pic_set_particles")

    def grid(self, name):
        if name in ("DEP_E", "DEP_I", "WALLQ"):
            a = np.zeros(self.nn, dtype=np.int64)
        elif name in ("ER", "EZ"):
            a = np.zeros(self.nn, dtype=np.float32)
        else:
            a = np.zeros(self.nn, dtype=np.float64)
        _check(lib().pic_get_grid(self.h, GRIDS[name], _ptr(a)), "pic_get_grid")
        return a

    def set_grid(self, name, a):
        dt = np.int64 if name in ("DEP_E", "DEP_I", "WALLQ") else np.float64
        a = np.ascontiguousarray(a, dtype=dt)
        _check(lib().pic_set_grid(self.h, GRIDS[name], _ptr(a)), "pic_set_grid")

    def redeposit(self):
        _check(lib().pic_redeposit(self.h), "pic_redeposit")

    def sort_now(self, sp):
        perm = np.zeros(max(self.cap[sp], 1), dtype=np.int64)
        _check(lib().pic_sort_now(self.h, sp, _ptr(perm)), "pic_sort_now")
        return perm

    def split_now(self, sp):
        """One particle-splitting pass over species sp; returns the copies added."""
        added = C.c_int64()
        _check(lib().pic_split_now(self.h, sp, C.byref(added)), "pic_split_now")
        return added.value

    def solve_once(self, Q, chi, U_E, tol, phi0=None):
        Q = np.ascontiguousarray(Q, dtype=np.float64)
        chi = np.ascontiguousarray(chi, dtype=np.float64)
        phi = np.zeros(self.nn) if phi0 is None else np.array(phi0, dtype=np.float64)
        it = C.c_int32()
        rel = C.c_double()
        rc = lib().pic_solve_once(self.h, _ptr(Q), _ptr(chi), U_E, tol, _ptr(phi), C.byref(it), C.byref(rel))
        return phi, it.value, rel.value, rc

    def solve_once_el(self, Q, chi, U, tol, phi0=None):
        """One solve with driven electrode e at U[e - 1]."""
        Q = np.ascontiguousarray(Q, dtype=np.float64)
        chi = np.ascontiguousarray(chi, dtype=np.float64)
        Uv = np.zeros(MAX_EL)
        Uv[:len(U)] = U
        phi = np.zeros(self.nn) if phi0 is None else np.array(phi0, dtype=np.float64)
        it = C.c_int32()
        rel = C.c_double()
        rc = lib().pic_solve_once_el(self.h, _ptr(Q), _ptr(chi), _ptr(Uv), tol, _ptr(phi), C.byref(it),
                                     C.byref(rel))
        return phi, it.value, rel.value, rc

    def capacitance(self):
        """n_el x n_el capacitance matrix of the driven electrodes (F)."""
        d = self.diag()
        return np.array(d.C_el[:]).reshape(MAX_EL, MAX_EL)[:d.n_el, :d.n_el]

    def match_design(self, apply=False):
        """(C_m1, C_m2) of electrode 1's L-network matching the current C_eq (Sec. 3)."""
        out = np.zeros(2)
        _check(lib().pic_match_design(self.h, 1 if apply else 0, _ptr(out)), "pic_match_design")
        return float(out[0]), float(out[1])

    def set_state(self, t, Q_E, U_E, circ, C_eq):
        st = np.array([t, Q_E, U_E] + list(circ) + [C_eq], dtype=np.float64)
        _check(lib().pic_set_state(self.h, _ptr(st)), "pic_set_state")

    def moments(self, sp):
        """(N, E) int64 node grids; mean energy E / (16 N) eV."""
        N = np.zeros(self.nn, dtype=np.int64)
        E = np.zeros(self.nn, dtype=np.int64)
        _check(lib().pic_moments(self.h, sp, _ptr(N), _ptr(E)), "pic_moments")
        return N, E

    def moments_noalloc(self, sp):
        """pic_moments through the allocation-free entry point (fixed scratch)."""
        N = np.zeros(self.nn, dtype=np.int64)
        E = np.zeros(self.nn, dtype=np.int64)
        _check(lib().pic_moments_noalloc(self.h, sp, _ptr(N), _ptr(E)), "pic_moments_noalloc")
        return N, E

    def set_solver(self, method=None, tol=None, max_iter=None, inner_tol=None, graphs=None):
        s = Solver()
        C.pointer(s)[0] = self.cfg.solver
        if graphs is not None:
            s.graphs = 1 if graphs else 0
        if method is not None:
            s.method = method
        if tol is not None:
            s.tol = tol
        if max_iter is not None:
            s.max_iter = max_iter
        if inner_tol is not None:
            s.inner_tol = inner_tol
        _check(lib().pic_set_solver(self.h, C.byref(s)), "pic_set_solver")
        self.cfg.solver = s

    # ---- learned preconditioner (image: nz rows by nr columns)
    def unet_num_params(self):
        n = C.c_int64()
        _check(lib().pic_unet_num_params(self.h, C.byref(n)), "pic_unet_num_params")
        return n.value

    def unet_set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        _check(lib().pic_unet_set_params(self.h, _ptr(p), p.size), "pic_unet_set_params")

    def unet_params(self):
        p = np.zeros(self.unet_num_params(), dtype=np.float32)
        _check(lib().pic_unet_get_params(self.h, _ptr(p), p.size), "pic_unet_get_params")
        return p

    def unet_forward(self, in3):
        in3 = np.ascontiguousarray(in3, dtype=np.float32)
        B = in3.shape[0]
        out = np.zeros((B, self.nz, self.nr), dtype=np.float32)
        _check(lib().pic_unet_forward(self.h, _ptr(in3), B, _ptr(out)), "pic_unet_forward")
        return out

    def unet_grads(self, in3, target, mask):
        in3 = np.ascontiguousarray(in3, dtype=np.float32)
        target = np.ascontiguousarray(target, dtype=np.float32)
        mask = np.ascontiguousarray(mask, dtype=np.float32)
        g = np.zeros(self.unet_num_params(), dtype=np.float32)
        loss = C.c_double()
        _check(lib().pic_unet_grads(self.h, _ptr(in3), _ptr(target), _ptr(mask), in3.shape[0], _ptr(g),
                                    C.byref(loss)), "pic_unet_grads")
        return g, loss.value

    def unet_harvest(self, every):
        _check(lib().pic_unet_harvest(self.h, every), "pic_unet_harvest")

    def unet_pair(self, slot):
        a = [np.zeros((self.nz, self.nr), dtype=np.float32) for _ in range(4)]
        _check(lib().pic_unet_get_pair(self.h, slot, *[_ptr(x) for x in a]), "pic_unet_get_pair")
        return dict(zip(("r", "e", "chi", "mask"), a))

    def unet_put_pair(self, slot, r, e, chi):
        a = [np.ascontiguousarray(x, dtype=np.float32) for x in (r, e, chi)]
        for x in a:
            if x.shape != (self.nz, self.nr):
                raise ValueError("pair images are nz x nr")
        _check(lib().pic_unet_put_pair(self.h, slot, *[_ptr(x) for x in a]), "pic_unet_put_pair")

    def unet_train(self, steps, batch, lr, seed=1):
        curve = np.zeros(max(steps, 1))
        _check(lib().pic_unet_train(self.h, steps, batch, lr, seed, _ptr(curve)), "pic_unet_train")
        return curve[:steps]
