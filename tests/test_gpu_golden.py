"""The 3D CRN workload (128x128x64 cup, 35% active, rotating fibres) run for its full
500 ms in the benchmark's launch configuration, against activation times and APD90
that the FP64 oracle wrote for 4,000 seeded tissue voxels (tests/golden/
crn_cup128_at_apd.csv, made by make_crn_cup_maps.py beside it).

FP64: activation times and APD90 within 2e-6 ms: the file holds 9 significant digits
(at most 5e-7 ms of rounding for an APD90 near 300 ms), and the 1e-10 relative state bar
moves a threshold crossing far less than that.
FP32: the same voxels activate; activation times within 1 dt (0.01 ms); APD90 within
2 ms.  The APD bound follows from the voltage bar: at the 90% repolarisation level
(about -68 mV) the CRN membrane potential of a single FP64 oracle cell falls at
0.26 mV/ms, so a 0.5 mV voltage error moves that crossing by about 2 ms."""
import os

import numpy as np
import pytest

from paper_1605_06015_amd import workloads as WL

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "crn_cup128_at_apd.csv")
TRACES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "crn_cup128_v_traces.npz")


def load_traces():
    d = np.load(TRACES)
    return d["idx"], d["t_ms"], d["V"].astype(np.float64)


def load_golden():
    d = np.loadtxt(GOLDEN, delimiter=",", skiprows=2)
    return d[:, 0].astype(np.int64), d[:, 1], d[:, 2]


def run_headline(prec, traces=None):
    """The workload for 500 ms; with traces = (box indices, every), also V at those
    voxels after every `every` steps (read on the device, gathered there)."""
    import torch
    from paper_1605_06015_amd import bbx as B
    c = WL.CRN_3D
    g = WL.crn_cup(c["nx"], c["ny"], c["nz"], seed=c["seed"], active=c["active"], h=c["h"])
    grid = B.Grid(g["mask"], c["h"], g["fibre"], c["Dpar"], c["Dperp"], prec)
    grid.model(B.BBX_MODEL_CRN, [], c["dt"])
    for v in range(21):
        grid.set(v, g["state"][v])
    grid.stimulus(g["stim"], c["stim_amp"], 0.0, c["stim_ms"])
    grid.record(c["theta"])
    n = int(round(c["t_end"] / c["dt"]))
    V = []
    if traces is None:
        for _ in range(10):
            grid.step(n // 10)
    else:
        idx, every = traces
        buf = torch.empty(g["mask"].size, dtype=torch.float64, device="cuda")
        sel = torch.from_numpy(idx).cuda()
        for _ in range(n // every):
            grid.step(every)
            B.bbx_readout(grid.handle, B.BBX_READ_VAR, 0, None, buf.data_ptr(), buf.numel() * 8, 1)
            V.append(buf[sel].cpu().numpy())
    assert grid.read(B.BBX_READ_STEP) == n
    return (grid.read(B.BBX_READ_ACT_TIME).ravel(), grid.read(B.BBX_READ_APD90).ravel(),
            g["mask"].ravel(), np.array(V))


@pytest.mark.parametrize("prec", [1, 0])
def test_crn_headline_500ms_against_oracle_maps(prec):
    """Activation times and APD90 at 4,000 voxels, and V at the same voxels every 1 ms
    (the oracle's V stored as float32: 1e-5 mV resolution).  FP64: |dV| <= 1e-4 mV;
    FP32: |dV| <= 0.5 mV at every sample, the headline metric's voltage bar."""
    idx, at_o, apd_o = load_golden()
    tidx, t_ms, V_o = load_traces()
    every = int(round((t_ms[1] - t_ms[0]) / WL.CRN_3D["dt"]))
    at, apd, mask, V_g = run_headline(prec, (tidx, every))
    assert V_g.shape == V_o.shape
    dV = np.abs(V_g - V_o)
    worst = np.unravel_index(np.argmax(dV), dV.shape)
    print(f"prec {prec}: max |dV| over {dV.size} samples {dV.max():.3g} mV at t = "
          f"{t_ms[worst[0]]:.0f} ms (V_oracle {V_o[worst]:.2f} mV), mean {dV.mean():.3g} mV")
    assert dV.max() <= (1e-4 if prec == 1 else 0.5), dV.max()
    assert np.all(mask[idx] == 1)
    assert np.isfinite(at_o).mean() > 0.9                  # the wave covers the cup
    assert np.isfinite(apd_o).mean() > 0.9                 # and it repolarises
    at_g, apd_g = at[idx], apd[idx]
    assert np.array_equal(np.isnan(at_g), np.isnan(at_o))
    assert np.array_equal(np.isnan(apd_g), np.isnan(apd_o))
    fa, fp = np.isfinite(at_o), np.isfinite(apd_o)
    dat = np.abs(at_g[fa] - at_o[fa]).max()
    dapd = np.abs(apd_g[fp] - apd_o[fp]).max()
    print(f"prec {prec}: max |dAT| {dat:.3g} ms, max |dAPD90| {dapd:.3g} ms, "
          f"AT range {at_o[fa].min():.2f}-{at_o[fa].max():.2f} ms, "
          f"APD90 range {apd_o[fp].min():.1f}-{apd_o[fp].max():.1f} ms")
    if prec == 1:
        assert dat <= 2e-6 and dapd <= 2e-6, (dat, dapd)
    else:
        assert dat <= WL.CRN_3D["dt"] + 1e-9, dat
        assert dapd <= 2.0, dapd


def test_crn_headline_500ms_tabulated_against_oracle_maps():
    """The FP32 step with the CRN voltage terms read from a table (spacing 0.05 mV, the
    benchmark's tabulated run) over the same 500 ms: activation times within 1 dt and APD90
    within 2 ms of the untabulated FP64 oracle's maps, same activated voxels."""
    from paper_1605_06015_amd import bbx as B
    idx, at_o, apd_o = load_golden()
    c = WL.CRN_3D
    g = WL.crn_cup(c["nx"], c["ny"], c["nz"], seed=c["seed"], active=c["active"], h=c["h"])
    grid = B.Grid(g["mask"], c["h"], g["fibre"], c["Dpar"], c["Dperp"], B.BBX_FP32)
    grid.model(B.BBX_MODEL_CRN, [], c["dt"])
    grid.tabulate(0.05)
    for v in range(21):
        grid.set(v, g["state"][v])
    grid.stimulus(g["stim"], c["stim_amp"], 0.0, c["stim_ms"])
    grid.record(c["theta"])
    grid.step(int(round(c["t_end"] / c["dt"])))
    at = grid.read(B.BBX_READ_ACT_TIME).ravel()[idx]
    apd = grid.read(B.BBX_READ_APD90).ravel()[idx]
    assert np.array_equal(np.isnan(at), np.isnan(at_o))
    fa, fp = np.isfinite(at_o), np.isfinite(apd_o)
    dat = np.abs(at[fa] - at_o[fa]).max()
    dapd = np.abs(apd[fp] - apd_o[fp]).max()
    print(f"tabulated: max |dAT| {dat:.3g} ms, max |dAPD90| {dapd:.3g} ms")
    assert dat <= c["dt"] + 1e-9 and dapd <= 2.0, (dat, dapd)


TP06_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tp06_cup64_at_apd.csv")


# (box, geometry seed, stored maps): the small test cup, and the cup of the benchmark's
# TP06 surrogate comparison
TP06_CUPS = {"cup64": ((64, 64, 32), 5, TP06_GOLDEN),
             "cup128": ((128, 128, 64), 1, os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                        "golden", "tp06_cup128_at_apd.csv"))}


@pytest.mark.parametrize("cup", ["cup64", "cup128"])
@pytest.mark.parametrize("prec", [1, 0])
def test_tp06_cup_500ms_against_oracle_maps(prec, cup):
    """TP06 on a 64x64x32 cup, and on the 128x128x64 cup of the benchmark's TP06 surrogate
    comparison, for 500 ms (dt 0.02 ms) against the FP64 oracle's activation times and
    APD90 at 4,000 seeded tissue voxels (tests/golden/tp06_cup64_at_apd.csv and
    tp06_cup128_at_apd.csv, made by make_tp06_cup_maps.py and make_tp06_cup128_maps.py).
    FP64 to the file's 9 significant digits (2e-6 ms).  FP32: same activated voxels,
    activation times within 1 dt, APD90 within 0.5 ms: at the 90% level a single FP64
    oracle cell repolarises at 2.1 mV/ms, so the 0.5 mV bar moves the crossing by about
    0.24 ms; the bound leaves room for slopes down to 1 mV/ms in tissue."""
    from paper_1605_06015_amd import bbx as B
    (nx, ny, nz), seed, path = TP06_CUPS[cup]
    d = np.loadtxt(path, delimiter=",", skiprows=2)
    idx, at_o, apd_o = d[:, 0].astype(np.int64), d[:, 1], d[:, 2]
    g = WL.tp06_cup(nx, ny, nz, seed=seed, active=0.35, h=0.25)
    grid = B.Grid(g["mask"], 0.25, g["fibre"], 0.3, 0.03, prec)
    grid.model(B.BBX_MODEL_TP06, [], 0.02)
    for v in range(19):
        grid.set(v, g["state"][v])
    grid.stimulus(g["stim"], 60.0, 0.0, 2.0)
    grid.record(-40.0)
    grid.step(25000)
    at = grid.read(B.BBX_READ_ACT_TIME).ravel()[idx]
    apd = grid.read(B.BBX_READ_APD90).ravel()[idx]
    assert np.array_equal(np.isnan(at), np.isnan(at_o))
    assert np.array_equal(np.isnan(apd), np.isnan(apd_o))
    fa, fp = np.isfinite(at_o), np.isfinite(apd_o)
    assert fa.mean() > 0.9 and fp.mean() > 0.9
    dat = np.abs(at[fa] - at_o[fa]).max()
    dapd = np.abs(apd[fp] - apd_o[fp]).max()
    print(f"tp06 {cup} prec {prec}: max |dAT| {dat:.3g} ms, max |dAPD90| {dapd:.3g} ms")
    if prec == 1:
        assert dat <= 2e-6 and dapd <= 2e-6, (dat, dapd)
    else:
        assert dat <= 0.02 + 1e-9 and dapd <= 0.5, (dat, dapd)


FK4_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fk4_ens_smallest_at_apd.csv")


def test_fk4_ensemble_full_protocol_against_oracle_maps():
    """The 96-tissue FK4 ensemble run as the benchmark runs it (tuned tile, graph replay in
    chunks of 1,000 steps, FP32, the whole 20,000-step S1-S2 protocol): the smallest tissue's
    activation times (threshold 0.5) and APD90 against the FP64 oracle's at 3,000 seeded
    voxels (tests/golden/fk4_ens_smallest_at_apd.csv, made by make_fk4_tissue_maps.py).
    Bars: same activated voxels, activation times within 1 dt (0.05 ms), APD90 within 0.75 ms
    (the 0.0075 bar on u over the 0.020/ms slope of u at the 90% level of a single FP64
    oracle cell is 0.37 ms)."""
    import torch
    import bench
    from paper_1605_06015_amd import bbx as B
    d = np.loadtxt(FK4_GOLDEN, delimiter=",", skiprows=2)
    idx, at_o, apd_o = d[:, 0].astype(np.int64), d[:, 1], d[:, 2]
    e, w, c = bench.ensemble_workload(torch.cuda.current_stream())
    i = int(np.argmin(w["nx"]))
    e.tune(20)
    e.graph(1000)
    e.step(c["steps"])
    at = e.read(B.BBX_READ_ACT_TIME, i).ravel()[idx]
    apd = e.read(B.BBX_READ_APD90, i).ravel()[idx]
    e.close()
    assert np.array_equal(np.isnan(at), np.isnan(at_o))
    fa, fp = np.isfinite(at_o), np.isfinite(apd_o)
    assert fa.all() and fp.mean() > 0.9
    dat = np.abs(at[fa] - at_o[fa]).max()
    dapd = np.abs(apd[fp] - apd_o[fp]).max()
    print(f"fk4 ensemble tissue {i}: max |dAT| {dat:.3g} ms, max |dAPD90| {dapd:.3g} ms")
    assert dat <= c["dt"] + 1e-9 and dapd <= 0.75, (dat, dapd)


SHELL_MAPS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tp06_shell128_at_apd.csv")
SHELL_TRACES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tp06_shell128_traces.npz")


@pytest.mark.parametrize("prec", [1, 0])
def test_tp06_shell_s1s2_protocol_against_oracle(prec):
    """The TP06 S1-S2 protocol on the down-scaled double shell (128x128x96, 600 ms; the
    S2 wave meets refractory tissue and dies out) against the FP64 oracle's stored
    results (tests/golden/tp06_shell128_*, made by make_tp06_shell_maps.py): first
    activation times and APD90 at 4,000 voxels, V at 1,000 voxels every 2 ms, and the
    pseudo-ECG at eight electrodes every 10 ms.
    FP64: AT / APD90 within 2e-6 ms, |dV| <= 1e-4 mV (float32 storage), ECG within
    1e-7 of its largest magnitude.  FP32: AT within 1 dt, APD90 within 0.5 ms (voxels whose
    S1 beat repolarised before S2), |dV| <= 0.5 mV at every sample, ECG within 1e-2 of its
    largest magnitude."""
    import torch
    from paper_1605_06015_amd import bbx as B
    c = WL.TP06_3D_SMALL
    d = np.loadtxt(SHELL_MAPS, delimiter=",", skiprows=2)
    idx, at_o, apd_o = d[:, 0].astype(np.int64), d[:, 1], d[:, 2]
    tr = np.load(SHELL_TRACES)
    tidx, V_o, ecg_o = tr["idx"], tr["V"].astype(np.float64), tr["ecg"]
    every = int(round((tr["t_ms"][1] - tr["t_ms"][0]) / c["dt"]))
    ecg_every = int(round((tr["ecg_t_ms"][1] - tr["ecg_t_ms"][0]) / c["dt"]))
    g3 = WL.tp06_biv(c["nx"], c["ny"], c["nz"], c["h"], c["seed"], c["active"], c["s1_strip"])
    grid = B.Grid(g3["mask"], c["h"], g3["fibre"], c["Dpar"], c["Dperp"], prec)
    grid.model(B.BBX_MODEL_TP06, [], c["dt"])
    for v, val in enumerate(WL.TP06_INITIAL):
        grid.fill(v, val)
    grid.stimulus(g3["s1"], c["s1_amp"], 0.0, c["s1_ms"])
    grid.stimulus(g3["s2"], c["s2_amp"], c["s2_t"], c["s2_ms"])
    grid.record(c["theta"])
    grid.ecg(g3["electrodes"], every=ecg_every, max_samples=1000)
    buf = torch.empty(g3["mask"].size, dtype=torch.float64, device="cuda")
    sel = torch.from_numpy(tidx).cuda()
    Vg = []
    for _ in range(V_o.shape[0]):
        grid.step(every)
        B.bbx_readout(grid.handle, B.BBX_READ_VAR, 0, None, buf.data_ptr(), buf.numel() * 8, 1)
        Vg.append(buf[sel].cpu().numpy())
    Vg = np.array(Vg)
    ecg = grid.ecg_series()
    at = grid.read(B.BBX_READ_ACT_TIME).ravel()[idx]
    apd = grid.read(B.BBX_READ_APD90).ravel()[idx]
    assert np.isfinite(at_o).mean() > 0.9
    assert np.array_equal(np.isnan(at), np.isnan(at_o))
    assert np.array_equal(np.isnan(apd), np.isnan(apd_o))
    fa, fp = np.isfinite(at_o), np.isfinite(apd_o)
    # APD90 of the S1 beat is well defined where that beat has repolarised before S2 (2 ms
    # margin); a voxel still near its 90% level when S2 arrives may cross it before or
    # after its second upstroke, a difference a rounding of V can decide
    s1 = fp & (at_o + apd_o < c["s2_t"] - 2.0)
    dat, dapd = np.abs(at[fa] - at_o[fa]).max(), np.abs(apd[s1] - apd_o[s1]).max()
    dapd_all = np.abs(apd[fp] - apd_o[fp])
    dV = np.abs(Vg - V_o)
    assert ecg.shape == ecg_o.shape, (ecg.shape, ecg_o.shape)
    decg = np.abs(ecg - ecg_o).max() / np.abs(ecg_o).max()
    # the S2 response: part of the traced voxels activate a second time after 310 ms
    late = (tr["t_ms"] > c["s2_t"])[:, None] & (V_o > -40.0)
    print(f"prec {prec}: |dAT| {dat:.3g} ms, |dAPD90| {dapd:.3g} ms on {int(s1.sum())} voxels repolarised "
          f"before S2 (all {fp.sum()}: max {dapd_all.max():.3g}, > 0.5 ms at {(dapd_all > 0.5).sum()}), "
          f"|dV| max {dV.max():.3g} mV, ECG rel {decg:.3g}; voxels re-excited by S2: "
          f"{int(late.any(axis=0).sum())}")
    assert s1.sum() > 0.35 * fp.sum()                  # 1,745 of 4,000 in the stored run
    assert late.any(axis=0).sum() > 0
    if prec == 1:
        assert dat <= 2e-6 and dapd <= 2e-6 and dV.max() <= 1e-4 and decg <= 1e-7
    else:
        assert dat <= c["dt"] + 1e-9 and dapd <= 0.5 and dV.max() <= 0.5 and decg <= 1e-2
