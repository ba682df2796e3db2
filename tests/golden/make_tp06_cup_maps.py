"""Writes tp06_cup64_at_apd.csv: activation times and APD90 of the FP64 oracle on a TP06
tissue (64x64x32 ellipsoidal cup, 35% active, rotating fibres, h 0.25 mm, dt 0.02 ms,
D 0.3/0.03 mm^2/ms, 2 ms 60 pA/pF apex stimulus, published epicardial initial state,
500 ms, threshold -40 mV) at 4,000 tissue voxels drawn with a fixed seed.  Calls only the
oracle and the seeded input generator.

    python tests/golden/make_tp06_cup_maps.py      (a few minutes on 8 cores)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1605_06015_amd import workloads as WL  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tp06_cup64_at_apd.csv")
NX, NY, NZ, SEED, H, DT = 64, 64, 32, 5, 0.25, 0.02
NSAMPLE = 4000
SAMPLE_SEED = 321


def main():
    g = WL.tp06_cup(NX, NY, NZ, seed=SEED, h=H)
    s = O.Sim(g["mask"], H, g["fibre"], 0.3, 0.03, O.MODEL_TP06, [], DT)
    s.state[:] = g["state"]
    s.stimuli.append(O.Stimulus(g["stim"], 60.0, 0, int(round(2.0 / DT))))
    s.start_recording(-40.0)
    nsteps = int(round(500.0 / DT))
    for k in range(0, nsteps, 2500):
        s.step(min(2500, nsteps - k))
        print(f"step {min(k + 2500, nsteps)} / {nsteps}", flush=True)
    act = s.act
    pick = np.sort(np.random.default_rng(SAMPLE_SEED).choice(act.size, NSAMPLE, replace=False))
    with open(OUT, "w") as f:
        f.write(f"# FP64 oracle, TP06 cup {NX}x{NY}x{NZ} (workloads.tp06_cup, seed {SEED}), h {H} mm, "
                f"dt {DT} ms, 500 ms: box index, activation time (ms), APD90 (ms); nan = not reached\n")
        f.write("idx,at,apd90\n")
        for t in pick:
            f.write(f"{int(act[t])},{s.rec.at[t]:.9g},{s.rec.apd[t]:.9g}\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
