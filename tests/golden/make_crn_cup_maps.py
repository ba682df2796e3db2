"""Writes the stored FP64 oracle results of the 3D CRN workload (128x128x64 ellipsoidal
cup, 35% active, rotating fibres, dt 0.01 ms, 2 ms 40 pA/pF apex stimulus, 500 ms,
threshold -40 mV) at 4,000 tissue voxels drawn with a fixed seed:

  crn_cup128_at_apd.csv     activation time and APD90 of each sampled voxel;
  crn_cup128_v_traces.npz   V of each sampled voxel every 1 ms (t = 1, 2, ..., 500 ms),
                            stored as float32 (resolution ~1e-5 mV, far below the
                            0.5 mV bar it is compared at).

Calls only the oracle and the seeded input generator.

    python tests/golden/make_crn_cup_maps.py [threads]     (about 40 minutes on 8 cores)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1605_06015_amd import workloads as WL  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "crn_cup128_at_apd.csv")
OUT_V = os.path.join(HERE, "crn_cup128_v_traces.npz")
NSAMPLE = 4000
SAMPLE_SEED = 123
EVERY = 100          # steps between stored V samples (1 ms)


def main():
    nthreads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    c = WL.CRN_3D
    g = WL.crn_cup(c["nx"], c["ny"], c["nz"], seed=c["seed"], active=c["active"], h=c["h"])
    s = O.Sim(g["mask"], c["h"], g["fibre"], c["Dpar"], c["Dperp"], O.MODEL_CRN, [], c["dt"],
              nthreads=nthreads)
    s.state[:] = g["state"]
    s.stimuli.append(O.Stimulus(g["stim"], c["stim_amp"], 0, int(round(c["stim_ms"] / c["dt"]))))
    s.start_recording(c["theta"])
    act = s.act
    pick = np.sort(np.random.default_rng(SAMPLE_SEED).choice(act.size, NSAMPLE, replace=False))
    box = act[pick]
    nsteps = int(round(c["t_end"] / c["dt"]))
    traces = np.zeros((nsteps // EVERY, NSAMPLE), np.float32)
    for k in range(nsteps // EVERY):
        s.step(EVERY)
        traces[k] = s.state[0].ravel()[box]
        if (k + 1) % 50 == 0:
            print(f"step {(k + 1) * EVERY} / {nsteps}", flush=True)
    with open(OUT, "w") as f:
        f.write("# FP64 oracle, CRN cup 128x128x64 (workloads.CRN_3D), 500 ms: box index, "
                "activation time (ms), APD90 (ms); nan = not reached\n")
        f.write("idx,at,apd90\n")
        for t in pick:
            f.write(f"{int(act[t])},{s.rec.at[t]:.9g},{s.rec.apd[t]:.9g}\n")
    t_ms = (np.arange(1, nsteps // EVERY + 1) * EVERY * c["dt"]).astype(np.float64)
    np.savez_compressed(OUT_V, idx=box.astype(np.int64), t_ms=t_ms, V=traces)
    print("wrote", OUT, OUT_V)


if __name__ == "__main__":
    main()
