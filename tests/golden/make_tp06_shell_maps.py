"""Writes the stored FP64 oracle results of the TP06 S1-S2 protocol on the down-scaled
double shell (workloads.TP06_3D_SMALL: 128x128x96 box at h 0.2 mm, 25% active, fibres
rotating through each wall, dt 0.02 ms, S1 on a y-strip at 0 ms, S2 on the upper half at
310 ms, 600 ms, threshold -40 mV):

  tp06_shell128_at_apd.csv     activation time and APD90 (first action potential) at
                               4,000 tissue voxels drawn with a fixed seed;
  tp06_shell128_traces.npz     V at 1,000 of those voxels every 2 ms (float32), and the
                               pseudo-ECG at the workload's eight electrodes every 10 ms.

Calls only the oracle and the seeded input generator.

    python tests/golden/make_tp06_shell_maps.py [threads]     (about 15 minutes on 8 cores)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1605_06015_amd import workloads as WL  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "tp06_shell128_at_apd.csv")
OUT_T = os.path.join(HERE, "tp06_shell128_traces.npz")
NSAMPLE, NTRACE = 4000, 1000
SAMPLE_SEED = 321
V_EVERY, ECG_EVERY = 100, 500      # steps (2 ms, 10 ms)


def main():
    nthreads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    c = WL.TP06_3D_SMALL
    g = WL.tp06_biv(c["nx"], c["ny"], c["nz"], c["h"], c["seed"], c["active"], c["s1_strip"])
    s = O.Sim(g["mask"], c["h"], g["fibre"], c["Dpar"], c["Dperp"], O.MODEL_TP06, [], c["dt"],
              nthreads=nthreads)
    for v, val in enumerate(WL.TP06_INITIAL):
        s.state[v][g["mask"] == 1] = val
    s.stimuli.append(O.Stimulus(g["s1"], c["s1_amp"], 0, int(round(c["s1_ms"] / c["dt"]))))
    s.stimuli.append(O.Stimulus(g["s2"], c["s2_amp"], int(round(c["s2_t"] / c["dt"])),
                                int(round(c["s2_ms"] / c["dt"]))))
    s.start_recording(c["theta"])
    act = s.act
    pick = np.sort(np.random.default_rng(SAMPLE_SEED).choice(act.size, NSAMPLE, replace=False))
    tpick = pick[:: NSAMPLE // NTRACE]
    nsteps = int(round(c["t_end"] / c["dt"]))
    V, ecg = [], []
    for k in range(nsteps // V_EVERY):
        s.step(V_EVERY)
        V.append(s.state[0].ravel()[act[tpick]].astype(np.float32))
        if s.n % ECG_EVERY == 0:
            ecg.append(O.pseudo_ecg(g["mask"], c["h"], g["fibre"], c["Dpar"], c["Dperp"],
                                    s.state[0], g["electrodes"]))
        if (k + 1) % 25 == 0:
            print(f"step {s.n} / {nsteps}", flush=True)
    with open(OUT, "w") as f:
        f.write("# FP64 oracle, TP06 S1-S2 on the 128x128x96 double shell (workloads.TP06_3D_SMALL), "
                "600 ms: box index, activation time (ms), APD90 (ms) of the first action "
                "potential; nan = not reached\n")
        f.write("idx,at,apd90\n")
        for t in pick:
            f.write(f"{int(act[t])},{s.rec.at[t]:.9g},{s.rec.apd[t]:.9g}\n")
    np.savez_compressed(OUT_T, idx=act[tpick].astype(np.int64),
                        t_ms=np.arange(1, len(V) + 1) * V_EVERY * c["dt"], V=np.array(V),
                        ecg_t_ms=np.arange(1, len(ecg) + 1) * ECG_EVERY * c["dt"], ecg=np.array(ecg))
    print("wrote", OUT, OUT_T)


if __name__ == "__main__":
    main()
