"""Seed ensembles of the FP64 oracle, run in parallel child processes.

TEST INFRASTRUCTURE ONLY: the statistical parity tests compare a GPU run
with the spread of oracle runs that differ only in the Philox seed.  Each
run is a fresh interpreter (python -m oracle.ensemble) that never touches a
GPU and writes its results to an .npz file.
"""
import copy
import json
import os
import subprocess
import sys
import tempfile

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(w, steps, periods=1):
    """One oracle run of `steps` steps; returns the RF-period-averaged
    densities and the harmonics 0..5 of U_E and I, each averaged over the
    last `periods` complete periods, the node volumes, and the last
    period's counts and characterisation."""
    from oracle import Oracle
    o = Oracle(w)
    spp = w["run"]["steps_per_period"]
    o.step(steps - (periods - 1) * spp)
    acc = None
    for k in range(periods):
        if k:
            o.step(spp)
        d = o.diag()
        cur = dict(n_e=o.grid("NE_AVG"), n_i=o.grid("NI_AVG"),
                   harm_U=np.array(d.harm_U_re[:]) + 1j * np.array(d.harm_U_im[:]),
                   harm_I=np.array(d.harm_I_re[:]) + 1j * np.array(d.harm_I_im[:]))
        acc = cur if acc is None else {q: acc[q] + cur[q] for q in acc}
    out = {q: v / periods for q, v in acc.items()}
    out.update(vol=o.grid("VOL"), n_alive=np.array(d.n_alive[:]), periods_done=np.array(d.periods_done),
               elec=np.array(d.elec[:]))
    return out


def ensemble(w, steps, seeds, workers=8, periods=1):
    """run() for each seed (the workload's run.seed replaced), at most
    `workers` child processes at a time."""
    out = {}
    with tempfile.TemporaryDirectory() as tmp:
        pending = list(seeds)
        running = []
        while pending or running:
            while pending and len(running) < workers:
                s = pending.pop(0)
                ws = copy.deepcopy(w)
                ws["run"]["seed"] = int(s)
                path = os.path.join(tmp, f"seed{s}.npz")
                cmd = [sys.executable, "-m", "oracle.ensemble", json.dumps(ws), str(steps), path, str(periods)]
                running.append((s, path, subprocess.Popen(cmd, cwd=ROOT)))
            s, path, p = running.pop(0)
            if p.wait() != 0:
                raise RuntimeError(f"oracle run for seed {s} failed ({p.returncode})")
            with np.load(path) as z:
                out[s] = {k: z[k] for k in z.files}
    return [out[s] for s in seeds]


if __name__ == "__main__":
    w, steps, path = json.loads(sys.argv[1]), int(sys.argv[2]), sys.argv[3]
    periods = int(sys.argv[4]) if len(sys.argv) > 4 else 1
    np.savez(path, **run(w, steps, periods))
