"""Writes fk4_ens_smallest_at_apd.csv: activation times and APD90 of the FP64 oracle on the
smallest tissue of the 96-tissue FK4 ensemble workload (workloads.FK4_ENSEMBLE: its own
side, diffusion tensor, fibre angle, time constants and S1-S2 stimuli), the full 20,000
steps of 0.05 ms, threshold u = 0.5, at 3,000 voxels drawn with a fixed seed.  Calls only
the oracle and the seeded input generator.

    python tests/golden/make_fk4_tissue_maps.py      (about a minute on 8 cores)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1605_06015_amd import workloads as WL  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fk4_ens_smallest_at_apd.csv")
NSAMPLE = 3000
SAMPLE_SEED = 77


def smallest_tissue():
    c = WL.FK4_ENSEMBLE
    w = WL.fk4_ensemble(n=c["n"], side_lo=c["side_lo"], side_hi=c["side_hi"], seed=c["seed"],
                        h=c["h"], Dpar=c["Dpar"], aniso=c["aniso"], spread=c["spread"],
                        s1_amp=c["s1_amp"], s1_ms=c["s1_ms"], apd_est_ms=c["apd_est_ms"],
                        cv_est_mm_ms=c["cv_est_mm_ms"])
    return int(np.argmin(w["nx"])), w, c


def main():
    i, w, c = smallest_tissue()
    s = int(w["nx"][i])
    mask = np.ones((1, s, s), np.uint8)
    fib = np.zeros((1, s, s, 3))
    fib[..., 0] = np.cos(w["angle"][i])
    fib[..., 1] = np.sin(w["angle"][i])
    o = O.Sim(mask, c["h"], fib, w["Dpar"][i], w["Dperp"][i], O.MODEL_FK4, list(w["params"][i]), c["dt"])
    for v, val in enumerate(WL.FK4_INITIAL):
        o.state[v] = val
    for (k, x0, x1, y0, y1, amp, t0, dur) in w["stims"]:
        if k == i:
            reg = np.zeros_like(mask)
            reg[0, y0:y1, x0:x1] = 1
            o.stimuli.append(O.Stimulus(reg, amp, int(round(t0 / c["dt"])), int(round(dur / c["dt"]))))
    o.start_recording(c["theta"])
    for k in range(0, c["steps"], 5000):
        o.step(5000)
        print(f"step {k + 5000} / {c['steps']}", flush=True)
    pick = np.sort(np.random.default_rng(SAMPLE_SEED).choice(s * s, NSAMPLE, replace=False))
    with open(OUT, "w") as f:
        f.write(f"# FP64 oracle, FK4 ensemble tissue {i} ({s}x{s}, workloads.FK4_ENSEMBLE), "
                f"{c['steps']} steps: voxel index y*side+x, activation time (ms), APD90 (ms); nan = not reached\n")
        f.write("idx,at,apd90\n")
        for t in pick:
            f.write(f"{int(t)},{o.rec.at[t]:.9g},{o.rec.apd[t]:.9g}\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
