"""Host-side checks of the benchmark script and the stored reference data (no GPU)."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1605_06015_amd import workloads as WL  # noqa: E402


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_counter_summary_is_consistent():
    """The committed counter file of the headline kernel: taken on the current kernel
    sources (else the benchmark line drops its traffic and VALU figures), bytes add up,
    the traffic is within 10% of the bytes the library's layout moves (and not below the
    algorithmic floor), and the VALU mix is complete: its classes fit in the total and the
    issue slots the kernel used are at least the floor of its mix."""
    d = json.load(open(os.path.join(ROOT, "profiles", "step_crn_cup128_fp32_traffic.json")))
    assert d["source_hash"] == bench.source_hash()
    assert d["bytes_per_launch"] == d["bytes_read"] + d["bytes_written"]
    layout = bench.CRN_LAYOUT_BYTES_PER_VOXEL * 367000
    assert 0.9 * layout <= d["bytes_per_launch"] <= 1.1 * layout
    assert d["bytes_per_launch"] >= bench.CRN_BYTES_PER_VOXEL * 367000
    n, tr, fma = d["valu_insts_per_launch"], d["valu_trans_per_launch"], d["valu_fma_per_launch"]
    assert d["waves_per_launch"] > 0 and 0 < tr and 0 < fma and tr + fma < n
    assert bench.valu_floor_slots(d) <= d["valu_slots_used_per_launch"] <= n + tr


def test_valu_slot_model():
    """Issue-slot costs: a 2-source instruction half a slot, a 3-source FMA one, a
    transcendental two; the chip's 1,024 SIMDs issue 614.4 G slots/s at 2.4 GHz."""
    assert bench.VALU_SLOT_PEAK_G == 614.4
    only = lambda n, tr=0, fma=0: bench.valu_floor_slots(
        {"valu_insts_per_launch": n, "valu_trans_per_launch": tr, "valu_fma_per_launch": fma})
    assert only(100) == 50 and only(100, tr=100) == 200 and only(100, fma=100) == 100
    assert only(10, tr=2, fma=3) == 2 * 2 + 3 + 0.5 * 5


def test_golden_maps_match_the_workload():
    """The stored oracle maps belong to the current CRN cup: every sampled index is a
    tissue voxel of the generator's mask, the sample is the file's 4,000 distinct voxels,
    and the activation times grow with distance from the stimulated apex."""
    d = np.loadtxt(bench.GOLDEN_MAPS, delimiter=",", skiprows=2)
    idx, at, apd = d[:, 0].astype(np.int64), d[:, 1], d[:, 2]
    assert len(idx) == 4000 and len(np.unique(idx)) == 4000
    c = WL.CRN_3D
    g = WL.crn_cup(c["nx"], c["ny"], c["nz"], seed=c["seed"], active=c["active"], h=c["h"])
    assert np.all(g["mask"].ravel()[idx] == 1)
    assert np.all(np.isfinite(at)) and np.all(np.isfinite(apd))
    z, y, x = np.unravel_index(idx, g["mask"].shape)
    stim = np.argwhere(g["stim"] == 1).mean(axis=0)
    dist = np.sqrt((z - stim[0]) ** 2 + (y - stim[1]) ** 2 + (x - stim[2]) ** 2)
    assert np.corrcoef(dist, at)[0, 1] > 0.8


@pytest.mark.parametrize("name,shape,seed", [("tp06_cup64_at_apd.csv", (64, 64, 32), 5),
                                              ("tp06_cup128_at_apd.csv", (128, 128, 64), 1)])
def test_tp06_golden_maps_match_the_workload(name, shape, seed):
    """The stored TP06 oracle maps belong to the current TP06 cups (the 64x64x32 test cup
    and the 128x128x64 cup of the benchmark's surrogate comparison)."""
    path = os.path.join(ROOT, "tests", "golden", name)
    d = np.loadtxt(path, delimiter=",", skiprows=2)
    idx, at = d[:, 0].astype(np.int64), d[:, 1]
    assert len(idx) == 4000 and len(np.unique(idx)) == 4000
    g = WL.tp06_cup(*shape, seed=seed, active=0.35, h=0.25)
    assert np.all(g["mask"].ravel()[idx] == 1)
    z, y, x = np.unravel_index(idx, g["mask"].shape)
    stim = np.argwhere(g["stim"] == 1).mean(axis=0)
    dist = np.sqrt((z - stim[0]) ** 2 + (y - stim[1]) ** 2 + (x - stim[2]) ** 2)
    assert np.corrcoef(dist, at)[0, 1] > 0.8


def test_fk4_golden_maps_match_the_workload():
    """The stored FK4 maps belong to the smallest tissue of the current ensemble workload,
    and its S1 wave (from the left columns) activates voxels later further right."""
    path = os.path.join(ROOT, "tests", "golden", "fk4_ens_smallest_at_apd.csv")
    head = open(path).readline()
    d = np.loadtxt(path, delimiter=",", skiprows=2)
    idx, at = d[:, 0].astype(np.int64), d[:, 1]
    c = WL.FK4_ENSEMBLE
    w = WL.fk4_ensemble(n=c["n"], side_lo=c["side_lo"], side_hi=c["side_hi"], seed=c["seed"],
                        h=c["h"], Dpar=c["Dpar"], aniso=c["aniso"], spread=c["spread"],
                        s1_amp=c["s1_amp"], s1_ms=c["s1_ms"], apd_est_ms=c["apd_est_ms"],
                        cv_est_mm_ms=c["cv_est_mm_ms"])
    i = int(np.argmin(w["nx"]))
    s = int(w["nx"][i])
    assert f"tissue {i} ({s}x{s}" in head
    assert len(np.unique(idx)) == len(idx) == 3000 and idx.max() < s * s
    assert np.corrcoef(idx % s, at)[0, 1] > 0.5
