"""Writes tp06_cup128_at_apd.csv: activation times and APD90 of the FP64 oracle on the TP06
cup of the benchmark's surrogate comparison (128x128x64 ellipsoidal cup, 35% active,
geometry seed 1, rotating fibres, h 0.25 mm, dt 0.02 ms, D 0.3/0.03 mm^2/ms, 2 ms
60 pA/pF apex stimulus, published epicardial initial state, 500 ms, threshold -40 mV) at
4,000 tissue voxels drawn with a fixed seed.  Calls only the oracle and the seeded input
generator.

    python tests/golden/make_tp06_cup128_maps.py [threads]     (about 30 minutes on 8 cores)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1605_06015_amd import workloads as WL  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tp06_cup128_at_apd.csv")
NX, NY, NZ, SEED, ACTIVE, H, DT = 128, 128, 64, 1, 0.35, 0.25, 0.02
DPAR, DPERP, AMP, DUR, THETA, T_END = 0.3, 0.03, 60.0, 2.0, -40.0, 500.0
NSAMPLE = 4000
SAMPLE_SEED = 456


def main():
    nthreads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    g = WL.tp06_cup(NX, NY, NZ, seed=SEED, active=ACTIVE, h=H)
    s = O.Sim(g["mask"], H, g["fibre"], DPAR, DPERP, O.MODEL_TP06, [], DT, nthreads=nthreads)
    s.state[:] = g["state"]
    s.stimuli.append(O.Stimulus(g["stim"], AMP, 0, int(round(DUR / DT))))
    s.start_recording(THETA)
    nsteps = int(round(T_END / DT))
    for k in range(0, nsteps, 1000):
        s.step(min(1000, nsteps - k))
        print(f"step {min(k + 1000, nsteps)} / {nsteps}", flush=True)
    act = s.act
    pick = np.sort(np.random.default_rng(SAMPLE_SEED).choice(act.size, NSAMPLE, replace=False))
    with open(OUT, "w") as f:
        f.write(f"# FP64 oracle, TP06 cup {NX}x{NY}x{NZ} (workloads.tp06_cup, seed {SEED}, active "
                f"{ACTIVE}), h {H} mm, dt {DT} ms, {T_END:.0f} ms: box index, activation time (ms), "
                f"APD90 (ms); nan = not reached\n")
        f.write("idx,at,apd90\n")
        for t in pick:
            f.write(f"{int(act[t])},{s.rec.at[t]:.9g},{s.rec.apd[t]:.9g}\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
