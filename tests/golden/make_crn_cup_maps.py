"""Writes crn_cup128_at_apd.csv: activation times and APD90 of the FP64 oracle on the
3D CRN workload (128x128x64 ellipsoidal cup, 35% active, rotating fibres, dt 0.01 ms,
2 ms 40 pA/pF apex stimulus, 500 ms, threshold -40 mV) at 4,000 tissue voxels drawn with
a fixed seed.  Calls only the oracle and the seeded input generator.

    python tests/golden/make_crn_cup_maps.py      (about 10-20 minutes on 8 cores)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1605_06015_amd import workloads as WL  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "crn_cup128_at_apd.csv")
NSAMPLE = 4000
SAMPLE_SEED = 123


def main():
    c = WL.CRN_3D
    g = WL.crn_cup(c["nx"], c["ny"], c["nz"], seed=c["seed"], active=c["active"], h=c["h"])
    s = O.Sim(g["mask"], c["h"], g["fibre"], c["Dpar"], c["Dperp"], O.MODEL_CRN, [], c["dt"])
    s.state[:] = g["state"]
    s.stimuli.append(O.Stimulus(g["stim"], c["stim_amp"], 0, int(round(c["stim_ms"] / c["dt"]))))
    s.start_recording(c["theta"])
    nsteps = int(round(c["t_end"] / c["dt"]))
    for k in range(0, nsteps, 5000):
        s.step(min(5000, nsteps - k))
        print(f"step {min(k + 5000, nsteps)} / {nsteps}", flush=True)
    act = s.act
    pick = np.sort(np.random.default_rng(SAMPLE_SEED).choice(act.size, NSAMPLE, replace=False))
    with open(OUT, "w") as f:
        f.write("# FP64 oracle, CRN cup 128x128x64 (workloads.CRN_3D), 500 ms: box index, "
                "activation time (ms), APD90 (ms); nan = not reached\n")
        f.write("idx,at,apd90\n")
        for t in pick:
            f.write(f"{int(act[t])},{s.rec.at[t]:.9g},{s.rec.apd[t]:.9g}\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
