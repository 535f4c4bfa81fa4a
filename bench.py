"""Benchmark of the hot path on one MI355X.

One step = the whole time step of the method (assembly of Eq. 1, circuit,
implicit field solve, the fused particle loop for both species, births,
periodic sort, per-period Laplace refresh).  Prints one JSON line.

  value          whole-job particle-steps/s over the timed region
  roofline       fused particle kernel (gather, correct, absorb, MCC, predict,
                 deposit): 68 algorithmic bytes per particle-step against the
                 8 TB/s HBM peak, timed with HIP events on the library's stream
  cpu_baseline   the FP64 oracle on a bounded sample of the same workload
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PER_PARTICLE_STEP = 68.0   # read r z vr vt vz ar at az w, write all but w (FP32)
HBM_PEAK_GBS = 8000.0
# HBM bytes per particle-step of k_particles by the rocprofv3 FETCH_SIZE and
# WRITE_SIZE counters (scaled by a plain-copy calibration: fetch x2, write
# x1) over the first 9 steps after the load (two electron sort cycles, no
# ion sort).  The counters include lines served by the 256 MB last-level
# cache.  A workload is left out (traffic null) whenever the kernel changes,
# until it is measured again.
MEASURED_BYTES_PER_PARTICLE_STEP = {"gec1024x2048": 87.0}


def cpu_baseline(name, sample_particles, steps):
    import oracle as O
    from pic_inputs import workload
    w = workload(name, run=dict(n_e=sample_particles, n_i=sample_particles,
                                cap_e=2 * sample_particles, cap_i=2 * sample_particles))
    o = O.Oracle(w)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    d = o.diag()
    n = int(d.n_alive[0] + d.n_alive[1])
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(value=2 * sample_particles * steps / dt, unit="particle-steps/s", cores=1, kind="oracle",
                host_cores=os.cpu_count(), cpu_model=cpu_model,
                sample=f"{name} geometry and circuit, {sample_particles} e + {sample_particles} Ar+ "
                       f"(uniform load), {steps} whole steps single-threaded FP64 incl. field solve; "
                       f"{dt:.1f} s, {n} alive at end",
                seconds=dt)


def unet_flops(H, W, C=32, cin_pad=16, levels=5):
    """FLOPs of one U-net forward on an H x W image (3x3 convolutions as the
    kernels run them: the first layer on 16 padded input channels)."""
    f = 0.0
    for l in range(levels):
        px = (H >> l) * (W >> l)
        if l < levels - 1:
            f += 2 * 9 * px * ((cin_pad if l == 0 else C) * C + C * C)     # encoder a, b
            f += 2 * 9 * px * (2 * C * C + C * C)                          # decoder a (concat), b
        else:
            f += 2 * 9 * px * 2 * C * C                                    # bottom a, b
    return f + 2 * H * W * C                                               # 1x1 output


def learned_vs_plain(sim, args, w):
    """Field-solve ms per step on the same discharge: plain FP64 MG-PCG,
    FP32-inner mixed precision MG-PCG, and flexible CG preconditioned by the
    U-net after training it on pairs harvested from this run."""
    import torch
    from paper_2310_04957_amd.pic import SOLVE_IR_MG, SOLVE_IR_UNET, SOLVE_MGPCG_FP64
    sim.unet_harvest(1)
    sim.step(args.learned_harvest_steps)
    sim.unet_harvest(0)
    pairs = int(sim.diag().unet_pairs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    curve = sim.unet_train(args.learned_train_steps, args.learned_batch, 1e-3, seed=1)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    res = {}
    for m, name in ((SOLVE_MGPCG_FP64, "plain_fp64_mgpcg"), (SOLVE_IR_MG, "mixed_ir_mgpcg"),
                    (SOLVE_IR_UNET, "learned_ir_unet_fpcg")):
        sim.set_solver(method=m)
        sim.step(1)
        d0 = sim.diag()
        sim.reset_timers()
        its = []
        for _ in range(args.learned_solve_steps):
            sim.step(1)
            d = sim.diag()
            its.append(int(d.solver_iters))
        res[name] = {"ms_per_step": d.ms_field / args.learned_solve_steps, "inner_iters": its,
                     "fallbacks": int(d.unet_fallbacks - d0.unet_fallbacks),
                     "unet_applications": int(d.unet_applications - d0.unet_applications)}
    sim.set_solver(method=SOLVE_IR_MG)
    H, W = w["geometry"]["nz"], w["geometry"]["nr"]
    lr = res["learned_ir_unet_fpcg"]
    return {
        **res,
        "faster_than_plain": lr["ms_per_step"] < res["plain_fp64_mgpcg"]["ms_per_step"],
        "training": {"pairs": pairs, "steps": args.learned_train_steps, "batch": args.learned_batch,
                     "seconds": t_train, "loss_first": float(curve[:5].mean()), "loss_last": float(curve[-20:].mean())},
        "unet_gflop_per_application": unet_flops(H, W) / 1e9,
        "image": f"{H}x{W}",
    }


def c4_protocol(args):
    """The learned preconditioner's protocol on the 512 x 1024 GEC discharge
    (64M + 64M particles): pairs harvested from FP64 MG-PCG solves of runs
    with seeds 1..16 (the five points of the pressure / voltage sweep in
    turn), one network trained on all of them with the library's kernels,
    then evaluated on seeds 17..20 inside flexible CG against plain FP64
    MG-PCG and FP32-inner MG-PCG: inner iterations from the same warm starts
    (solve_once, FP64 residual 1e-8), and field-solve ms per step and
    fallbacks over steps of the running discharge."""
    import numpy as np
    import torch
    from paper_2310_04957_amd.pic import Pic, SOLVE_IR_MG, SOLVE_IR_UNET, SOLVE_MGPCG_FP64
    from pic_inputs import workload
    from pic_inputs.workloads import GEC512_SWEEP, MTORR_PA, _lmatch

    def discharge(seed, **kw):
        p_mtorr, U = GEC512_SWEEP[(seed - 1) % len(GEC512_SWEEP)]
        w = workload("gec512x1024")
        w["gas"]["p_Pa"] = p_mtorr * MTORR_PA
        w["circuit"] = _lmatch(float(U))
        w["run"]["seed"] = seed
        # room for the discharges of the sweep that ionise fastest (at 50
        # mTorr and 300 V the ions grow from 64M to about 150M in 550 steps)
        w["run"]["cap_e"] = w["run"]["cap_i"] = 240_000_000
        print(f"[c4] seed {seed}: {p_mtorr} mTorr, {U} V", file=sys.stderr, flush=True)
        return w, Pic(w, method=SOLVE_IR_MG, timing=True, **kw)

    t_start = time.perf_counter()
    pairs = []
    for seed in range(1, args.c4_train_seeds + 1):
        w, sim = discharge(seed, unet_batch=1, unet_pairs=args.c4_pairs_per_seed)
        sim.step(args.c4_warmup)
        sim.unet_harvest(args.c4_every)
        for _ in range(0, args.c4_harvest_steps, 20):
            sim.step(20)
        sim.unet_harvest(0)
        got = min(int(sim.diag().unet_pairs), args.c4_pairs_per_seed)
        for k in range(got):
            pr = sim.unet_pair(k)
            pairs.append((pr["r"], pr["e"], pr["chi"]))
        sim.close()
        print(f"[c4] seed {seed}: {got} pairs ({len(pairs)} in all)", file=sys.stderr, flush=True)
    t_harvest = time.perf_counter() - t_start

    wt = workload("gec512x1024")
    wt["run"].update(n_e=0, n_i=0, cap_e=1, cap_i=1)
    trainer = Pic(wt, load=False, method=SOLVE_IR_MG, unet_batch=args.c4_batch, unet_pairs=len(pairs))
    for k, (r, e, chi) in enumerate(pairs):
        trainer.unet_put_pair(k, r, e, chi)
    del pairs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    curve = trainer.unet_train(args.c4_train_steps, args.c4_batch, args.c4_lr, seed=1)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    params = trainer.unet_params()
    n_pairs = int(trainer.diag().unet_pairs)
    trainer.close()
    print(f"[c4] trained {args.c4_train_steps} steps on {n_pairs} pairs in {t_train:.1f} s: "
          f"loss {curve[:20].mean():.3f} -> {curve[-100:].mean():.3f}", file=sys.stderr, flush=True)
    if args.c4_save:
        params.astype(np.float32).tofile(args.c4_save)

    methods = ((SOLVE_MGPCG_FP64, "plain_fp64_mgpcg"), (SOLVE_IR_MG, "mixed_ir_mgpcg"),
               (SOLVE_IR_UNET, "learned_ir_unet_fpcg"))
    tol = 1e-8
    evals = []
    for seed in range(args.c4_train_seeds + 1, args.c4_train_seeds + 1 + args.c4_eval_seeds):
        w, sim = discharge(seed, unet_batch=1, unet_pairs=0)
        sim.unet_set_params(params)
        sim.step(args.c4_warmup)
        # the same warm starts for every method: a step's Q, chi and U_E,
        # started from the previous step's solution
        res = {"seed": seed, "point": GEC512_SWEEP[(seed - 1) % len(GEC512_SWEEP)]}
        its = {name: [] for _, name in methods}
        phi_n1 = sim.grid("PHI")
        for _ in range(args.c4_problems):
            phi_n0 = phi_n1
            sim.step(1)
            phi_n1 = sim.grid("PHI")
            Q, chi, U = sim.grid("Q"), sim.grid("CHI"), sim.diag().U_E
            for m, name in methods:
                sim.set_solver(method=m)
                _, it, rel, rc = sim.solve_once(Q, chi, U, tol, phi_n0)
                its[name].append(int(it) if rc == 0 and rel <= tol else -1)
            sim.set_solver(method=SOLVE_IR_MG)
            sim.step(args.c4_problem_gap - 1)
            phi_n1 = sim.grid("PHI")
        res["inner_iters_same_start"] = its
        for m, name in methods:
            sim.set_solver(method=m)
            sim.step(1)
            d0 = sim.diag()
            sim.reset_timers()
            steps_its = []
            for _ in range(args.c4_steps):
                sim.step(1)
                steps_its.append(int(sim.diag().solver_iters))
            d = sim.diag()
            res[name] = {"field_ms_per_step": d.ms_field / args.c4_steps, "inner_iters": steps_its,
                         "fallbacks": int(d.unet_fallbacks - d0.unet_fallbacks),
                         "unet_applications": int(d.unet_applications - d0.unet_applications),
                         "relres_last": d.solver_relres, "network_switched_off": int(d.unet_disabled)}
        sim.close()
        evals.append(res)
        print(f"[c4] eval seed {seed}: " + ", ".join(
            f"{name} {res[name]['field_ms_per_step']:.3f} ms/step its {sum(its[name])}" for _, name in methods),
              file=sys.stderr, flush=True)

    def mean(name, key):
        return float(np.mean([e[name][key] for e in evals]))
    summary = {name: {"field_ms_per_step": mean(name, "field_ms_per_step"),
                      "inner_iters_same_start_total": int(sum(sum(e["inner_iters_same_start"][name]) for e in evals)),
                      "fallbacks": int(sum(e[name]["fallbacks"] for e in evals))} for _, name in methods}
    return {
        "grid": "512x1024", "particles": "64M + 64M", "train_seeds": list(range(1, args.c4_train_seeds + 1)),
        "eval_seeds": [e["seed"] for e in evals], "pairs": n_pairs, "harvest_seconds": t_harvest,
        "training": {"steps": args.c4_train_steps, "batch": args.c4_batch, "lr": args.c4_lr, "seconds": t_train,
                     "loss_first": float(curve[:20].mean()), "loss_last": float(curve[-100:].mean())},
        "summary": summary,
        "faster_than_plain": summary["learned_ir_unet_fpcg"]["field_ms_per_step"] <
        summary["plain_fp64_mgpcg"]["field_ms_per_step"],
        "evaluation": evals,
    }


def electrodes_pass(args):
    """Cost of a second driven electrode on the same grid without particles:
    the lower GEC electrode driven (ideal, 2 MHz) besides the upper one.  One
    RF period of steps each; field-solve ms per step and the once-per-period
    refresh (one Laplace solve per electrode and the capacitance matrix)."""
    import torch
    from paper_2310_04957_amd.pic import Pic
    from pic_inputs import workload
    from pic_inputs.workloads import CIRC_IDEAL, _circuit, gec_geometry
    w0 = workload(args.workload)
    refine = w0["geometry"]["nr"] // 128
    res = {"grid": f"{w0['geometry']['nr']}x{w0['geometry']['nz']}", "particles": 0}
    for n_el in (1, 2):
        w = workload(args.workload)
        w["run"].update(n_e=0, n_i=0, cap_e=1, cap_i=1)
        if n_el == 2:
            w["geometry"] = gec_geometry(refine, driven_lower=True)
            w["circuits_more"] = [_circuit(CIRC_IDEAL, freq=2e6, U_amp=100.0)]
        sim = Pic(w, load=False, timing=True)
        spp = w["run"]["steps_per_period"]
        sim.reset_timers()
        sim.step(spp)
        torch.cuda.synchronize()
        d = sim.diag()
        res[str(n_el)] = {"field_ms_per_step": d.ms_field / spp, "refresh_ms": d.ms_refresh,
                          "capacitance_pF": [[round(x * 1e12, 4) for x in row] for row in sim.capacitance()]}
        sim.close()
    return res


def precision_study(periods=4):
    """The 512x1024 precision study: for each (pressure, source amplitude)
    point, the same discharge (64M + 64M particles) run `periods` RF periods
    with the FP32-inner IR solve (seed 1) and with all-FP64 MG-PCG (seeds 1
    and 2).  The IR-vs-FP64 difference of the last period's averaged
    densities and of the electrode current and voltage harmonics 1..5 is
    reported beside the seed-to-seed difference of the FP64 runs (the
    discharge's own statistical noise).  The push is FP32 in all three runs;
    its error against an FP64 push is measured by the one-step and
    statistical parity tests against the oracle."""
    import numpy as np
    import torch
    from paper_2310_04957_amd.pic import Pic, SOLVE_IR_MG, SOLVE_MGPCG_FP64
    from pic_inputs import workload
    from pic_inputs.workloads import GEC512_SWEEP, MTORR_PA, _lmatch

    def run(p_mtorr, U, method, seed):
        w = workload("gec512x1024")
        w["gas"]["p_Pa"] = p_mtorr * MTORR_PA
        w["circuit"] = _lmatch(float(U))
        w["run"]["seed"] = seed
        spp = w["run"]["steps_per_period"]
        print(f"[bench] precision study {p_mtorr} mTorr {U} V method {method} seed {seed}",
              file=sys.stderr, flush=True)
        sim = Pic(w, method=method, timing=True)
        sim.reset_timers()
        sim.step(periods * spp)
        torch.cuda.synchronize()
        d, g = sim.diag(grids=True)
        out = dict(n_e=g["n_e"], n_i=g["n_i"],
                   hI=np.array(d.harm_I_re[:]) + 1j * np.array(d.harm_I_im[:]),
                   hU=np.array(d.harm_U_re[:]) + 1j * np.array(d.harm_U_im[:]),
                   field_ms=d.ms_field / (periods * spp), nr=w["geometry"]["nr"], nz=w["geometry"]["nz"])
        sim.close()
        return out

    def blocks(n, nr, nz, b=16):
        a = n.reshape(nz + 1, nr + 1)
        H, W = (nz + 1) // b * b, (nr + 1) // b * b
        return a[:H, :W].reshape(H // b, b, W // b, b).sum(axis=(1, 3)).ravel()

    def diff(a, b):
        r = {}
        for sp in ("n_e", "n_i"):
            r[sp + "_total"] = abs(a[sp].sum() - b[sp].sum()) / b[sp].sum()
            ba, bb = blocks(a[sp], a["nr"], a["nz"]), blocks(b[sp], b["nr"], b["nz"])
            m = bb > 1e-3 * bb.max()
            r[sp + "_16x16_blocks_rms"] = float(np.sqrt(np.mean(((ba[m] - bb[m]) / bb[m]) ** 2)))
        for h in ("hI", "hU"):
            r[h + "_1_5"] = [float(abs(a[h][k] - b[h][k]) / abs(b[h][k])) for k in range(1, 6)]
        return {k: (round(v, 5) if isinstance(v, float) else [round(x, 5) for x in v]) for k, v in r.items()}

    res = []
    for p_mtorr, U in GEC512_SWEEP:
        try:
            ir = run(p_mtorr, U, SOLVE_IR_MG, 1)
            f1 = run(p_mtorr, U, SOLVE_MGPCG_FP64, 1)
            f2 = run(p_mtorr, U, SOLVE_MGPCG_FP64, 2)
        except RuntimeError as e:
            res.append({"p_mTorr": p_mtorr, "U_s": U, "error": str(e)})
            continue
        res.append({"p_mTorr": p_mtorr, "U_s": U, "ir_vs_fp64": diff(ir, f1), "fp64_seed2_vs_seed1": diff(f2, f1),
                    "field_ms_per_step": {"ir": round(ir["field_ms"], 3), "fp64": round(f1["field_ms"], 3)}})
    return {"grid": "512x1024", "particles": "64M + 64M", "periods": periods, "points": res}


def split_pass(sim):
    """One particle-splitting pass per species on the discharge as it stands
    (equal loading weights: particles near the axis are heavier than the
    reference weight of their column), timed by the wall clock around the
    synchronous call."""
    res = {}
    for sp, name in ((0, "e"), (1, "i")):
        n0 = sim.diag().n_slots[sp]
        t0 = time.perf_counter()
        try:
            added = sim.split_now(sp)
        except Exception as e:  # the copies do not fit: reported, nothing changed
            res[name] = {"error": str(e), "slots": int(n0), "capacity": int(sim.cap[sp]),
                         "note": "the copies would not fit in the slot capacity; nothing was changed"}
            continue
        ms = 1e3 * (time.perf_counter() - t0)
        res[name] = {"ms": ms, "slots": int(n0), "copies": int(added),
                     "slots_per_s": n0 / (ms * 1e-3) if ms > 0 else None}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400,
                    help="timed steps (default: one RF period of the workload)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="gec1024x2048")
    ap.add_argument("--method", default="ir", choices=["ir", "mgpcg"])
    ap.add_argument("--cpu-sample", type=int, default=1_000_000)
    ap.add_argument("--cpu-steps", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sort-every", type=int, default=None)
    ap.add_argument("--sort-every-ion", type=int, default=None)
    ap.add_argument("--inner-tol", type=float, default=1e-4,
                    help="relative residual reduction of each FP32 inner solve of the field solve")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-vs-plain field-solve comparison")
    ap.add_argument("--learned-harvest-steps", type=int, default=24)
    ap.add_argument("--learned-train-steps", type=int, default=150)
    ap.add_argument("--learned-batch", type=int, default=4)
    ap.add_argument("--learned-solve-steps", type=int, default=3)
    ap.add_argument("--precision-study", action="store_true",
                    help="also run the 512x1024 precision study (IR vs all-FP64 solve, seed noise floor)")
    ap.add_argument("--no-electrodes-pass", action="store_true",
                    help="skip timing the field solve and refresh with one and two driven electrodes")
    ap.add_argument("--no-split-pass", action="store_true",
                    help="skip timing one particle-splitting pass per species after the run")
    ap.add_argument("--c4", action="store_true",
                    help="only run the learned preconditioner's train/evaluate protocol on 512x1024 (seeds 1-16 / 17-20)")
    ap.add_argument("--no-c4", action="store_true",
                    help="skip the learned preconditioner's 512x1024 train/evaluate protocol after the timed run")
    ap.add_argument("--c4-train-seeds", type=int, default=16)
    ap.add_argument("--c4-eval-seeds", type=int, default=4)
    ap.add_argument("--c4-warmup", type=int, default=300)
    ap.add_argument("--c4-every", type=int, default=4)
    ap.add_argument("--c4-harvest-steps", type=int, default=200)
    ap.add_argument("--c4-pairs-per-seed", type=int, default=200)
    ap.add_argument("--c4-train-steps", type=int, default=3000)
    ap.add_argument("--c4-batch", type=int, default=8)
    ap.add_argument("--c4-lr", type=float, default=1e-3)
    ap.add_argument("--c4-problems", type=int, default=4)
    ap.add_argument("--c4-problem-gap", type=int, default=20)
    ap.add_argument("--c4-steps", type=int, default=40)
    ap.add_argument("--c4-save", default="")
    ap.add_argument("--unet-forwards", type=int, default=0,
                    help="only run this many U-net forwards (batch 1, no particles) on the workload's node image")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain FP32 copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy_mib:
        import torch
        n = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.add(src, 0.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": 4 * n, "bytes_written": 4 * n, "launches": 3}))
        return
    if args.unet_forwards:
        # the learned preconditioner's forward pass alone, for the kernel
        # trace and counters of its convolutions at full resolution
        import numpy as np
        import torch
        from paper_2310_04957_amd.pic import Pic
        from pic_inputs import workload
        from pic_inputs.workloads import SOLVE_IR_MG
        w = workload(args.workload, run={"n_e": 0, "n_i": 0, "cap_e": 16, "cap_i": 16})
        g = Pic(w, load=False, method=SOLVE_IR_MG, unet_batch=1, unet_pairs=0)
        nr, nz = w["geometry"]["nr"], w["geometry"]["nz"]
        x = np.random.default_rng(1).normal(size=(1, nz, nr, 3)).astype(np.float32)
        g.unet_forward(x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.unet_forwards):
            out = g.unet_forward(x)
        wall = time.perf_counter() - t0
        g.close()
        print(json.dumps({"unet_forwards": args.unet_forwards, "image": [nz, nr],
                          "ms_per_forward_with_copies": 1e3 * wall / args.unet_forwards,
                          "mean_abs_out": float(np.abs(out).mean())}))
        return
    if args.c4:
        print(json.dumps({"c4": c4_protocol(args)}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; multi-GPU runs are not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2310_04957_amd.pic import Pic
    from pic_inputs import workload
    from pic_inputs.workloads import SOLVE_IR_MG, SOLVE_MGPCG_FP64

    w = workload(args.workload)
    if args.sort_every is not None:
        w["run"]["sort_every"] = args.sort_every
    if args.sort_every_ion is not None:
        w["run"]["sort_every_ion"] = args.sort_every_ion
    method = SOLVE_IR_MG if args.method == "ir" else SOLVE_MGPCG_FP64
    print(f"[bench] init {args.workload} method={args.method}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    learned = not args.no_learned
    sim = Pic(w, timing=True, method=method, inner_tol=args.inner_tol, unet_batch=args.learned_batch if learned else 0,
              unet_pairs=512 if learned else 0)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    print(f"[bench] init done in {t_init:.1f} s; warmup {args.warmup}", file=sys.stderr, flush=True)
    sim.step(args.warmup)
    sim.reset_timers()
    d0 = sim.diag()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    d = sim.diag()
    print(f"[bench] timed {args.steps} steps in {wall:.3f} s", file=sys.stderr, flush=True)

    # particle-steps in the timed region: slots are processed each step;
    # use the mean of the live counts at both ends
    n_start = d0.n_alive[0] + d0.n_alive[1]
    n_end = d.n_alive[0] + d.n_alive[1]
    n_mean = 0.5 * (n_start + n_end)
    ps = n_mean * args.steps
    ms_part = d.ms_particles[0] + d.ms_particles[1]
    # a step right after a sort also reads the permutation (4 B) and writes w
    # (4 B) for that species (the sort at the end of step s moves the
    # particles during step s + 1)
    def sorted_steps(every):
        return sum(1 for s_ in range(args.warmup, args.warmup + args.steps) if every > 0 and s_ > 0 and s_ % every == 0)
    extra = 8.0 * (d0.n_alive[0] * sorted_steps(w["run"]["sort_every"]) +
                   d0.n_alive[1] * sorted_steps(w["run"]["sort_every_ion"]))
    part_bytes = BYTES_PER_PARTICLE_STEP * ps + extra
    achieved = part_bytes / (ms_part * 1e-3) / 1e9 if ms_part > 0 else 0.0
    out = {
        "metric": "particle-steps/s (push+deposit+MCC) + field-solve ms/step, learned vs plain PCG",
        "value": ps / wall,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": f"{w['geometry']['nr']}x{w['geometry']['nz']}",
                   "particles": int(n_start), "solver": args.method, "sort_every": w["run"]["sort_every"],
                   "sort_every_ion": w["run"]["sort_every_ion"], "steps_per_period": w["run"]["steps_per_period"]},
        "particle_loop_particle_steps_per_s": ps / (ms_part * 1e-3) if ms_part > 0 else None,
        "field_solve_ms_per_step": d.ms_field / max(args.steps, 1),
        "phase_ms_per_step": {"particles_e": d.ms_particles[0] / args.steps, "particles_i": d.ms_particles[1] / args.steps,
                              "births": d.ms_births / args.steps, "sort": d.ms_sort / args.steps,
                              "field": d.ms_field / args.steps, "refresh": d.ms_refresh / args.steps},
        "solver_iters_last": int(d.solver_iters), "solver_relres_last": d.solver_relres,
        "deposit_fallback_per_step": (d.deposit_fallback - d0.deposit_fallback) / args.steps,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (MEASURED_BYTES_PER_PARTICLE_STEP[args.workload] * ps / (2 * args.steps) / 1e9
                                 if args.workload in MEASURED_BYTES_PER_PARTICLE_STEP else None),
                     "traffic_unit": "GB per launch (HBM, rocprofv3 counters)",
                     "algorithmic_gb_per_launch": part_bytes / (2 * args.steps) / 1e9,
                     "kernel": "k_particles", "bytes_per_unit": BYTES_PER_PARTICLE_STEP,
                     "bytes_after_sort": "+8 per particle on the step after its species' sort",
                     "unit_of_work": "particle-step"},
    }
    if learned:
        print("[bench] learned vs plain field solve", file=sys.stderr, flush=True)
        out["field_solve_learned_vs_plain"] = learned_vs_plain(sim, args, w)
    if not args.no_split_pass:
        print("[bench] particle-splitting pass", file=sys.stderr, flush=True)
        out["split_pass"] = split_pass(sim)
    sim.close()
    if not args.no_electrodes_pass and args.workload.startswith("gec"):
        print("[bench] driven electrodes", file=sys.stderr, flush=True)
        out["electrodes_pass"] = electrodes_pass(args)
    if not args.no_c4:
        print("[bench] learned preconditioner protocol (512x1024)", file=sys.stderr, flush=True)
        try:
            out["learned_preconditioner_512x1024"] = c4_protocol(args)
        except Exception as e:  # reported, the timed result stands
            out["learned_preconditioner_512x1024"] = {"error": str(e)}
    if args.precision_study:
        out["precision_study"] = precision_study()
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_sample, args.cpu_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
