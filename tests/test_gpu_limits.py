"""A box at the library's size limit: 1290^3 = 2,146,689,000 voxels, just under the
2^31 - 1 that box indices may reach.  Two small tissue blobs sit at opposite corners (the
far one holds the largest box indices).  Each tissue voxel's update reads only its own
neighbourhood, so after the same FP32 run every value equals, bit for bit, that of the
same blob simulated alone in a box of its own size (the blob boxes themselves are
checked against the oracle by the other parity tests).  This checks every box index,
neighbour offset and box-layout readout near the limit without an oracle run over
2 G voxels."""
import numpy as np
import pytest

from paper_1605_06015_amd import workloads as WL

pytestmark = pytest.mark.gpu

N = 1290
H, D, DT, STEPS = 0.5, 1.0, 0.01, 300
BARKLEY = [0.75, 0.02, 0.02]


def setup_grid(B, mask, stim):
    g = B.Grid(mask, H, None, D, D, B.BBX_FP32)
    g.model(B.BBX_MODEL_BARKLEY, BARKLEY, DT)
    g.fill(0, 0.0)
    g.fill(1, 0.0)
    g.stimulus(stim, 1.0, 0.0, 1.0)
    return g


def test_box_at_index_limit_matches_blob_boxes():
    import torch
    from paper_1605_06015_amd import bbx as B
    assert N ** 3 <= 2 ** 31 - 1
    blobs = [WL.random_blob_mask(14, 11, 9, seed=4), WL.random_blob_mask(12, 13, 10, seed=6)]
    where = [tuple(slice(N - s, N) for s in blobs[0].shape),        # far corner
             tuple(slice(0, s) for s in blobs[1].shape)]            # origin corner
    stims = []
    for m in blobs:
        st = np.zeros_like(m)
        st[:, :, :4] = m[:, :, :4]                                  # the low-x end of each blob
        stims.append(st)

    small = []
    for m, st in zip(blobs, stims):
        g = setup_grid(B, m, st)
        g.step(STEPS)
        small.append((g.get(0), g.get(1)))
        assert np.nanmax(small[-1][0][m == 1]) > 0.5                # the blob is excited
        g.close()

    mask = np.zeros((N, N, N), np.uint8)
    stim = np.zeros((N, N, N), np.uint8)
    for m, st, w in zip(blobs, stims, where):
        mask[w] = m
        stim[w] = st
    print("limit box: creating", flush=True)
    big = setup_grid(B, mask, stim)
    del stim
    assert big.nact == sum(int(m.sum()) for m in blobs)
    big.step(STEPS)
    print("limit box: stepped", flush=True)
    out = torch.empty(N ** 3, dtype=torch.float64, device="cuda")
    for var in (0, 1):
        B.bbx_readout(big.handle, B.BBX_READ_VAR, var, None, out.data_ptr(), out.numel() * 8, 1)
        torch.cuda.synchronize()
        for (m, w, (u, v)) in zip(blobs, where, small):
            z, y, x = np.nonzero(m)
            flat = ((z + w[0].start) * N + (y + w[1].start)) * N + (x + w[2].start)
            got = out[torch.from_numpy(flat).to("cuda")].cpu().numpy()
            want = (u if var == 0 else v)[m == 1]
            assert np.array_equal(got, want), (var, np.abs(got - want).max())
    del out
    big.close()


def test_ensemble_at_voxel_limit_last_tissue_matches_alone():
    """Two 46340 x 23170 tissues and a small 9 x 7 one after them: 2,147,395,663 voxels in
    total, just under the 2^31 limit, so the small tissue holds the largest voxel offsets.
    FP32 Barkley, a stimulus on the small tissue, 100 steps: its values equal, bit for bit,
    those of the same tissue alone in an ensemble of one."""
    from paper_1605_06015_amd import bbx as B
    nx, ny = [46340, 46340, 9], [23170, 23170, 7]
    assert sum(a * b for a, b in zip(nx, ny)) < 2 ** 31

    def run(nxs, nys):
        k = len(nxs)
        e = B.Ensemble(nxs, nys, H, [D] * k, [0.5 * D] * k, [0.3] * k, B.BBX_MODEL_BARKLEY,
                       BARKLEY * k, DT, B.BBX_FP32)
        e.stimulus(k - 1, 0, 3, 0, 7, 1.0, 0.0, 1.0)
        e.step(100)
        out = [e.get(k - 1, v) for v in range(2)]
        e.close()
        return out

    alone = run(nx[2:], ny[2:])
    assert alone[0].max() > 0.5
    print("ensemble at the limit: running", flush=True)
    full = run(nx, ny)
    for v in range(2):
        assert np.array_equal(full[v], alone[v]), v


@pytest.mark.parametrize("aniso", ["random", "rotating", False])
def test_dense_box_beyond_cache_streaming_kernels_sampled(aniso):
    """A dense 512x512x264 box (277 MB of V in FP32, above the 256 MB Infinity Cache, so
    the streaming instantiations of the z-marching kernels run: the LDS ring with rotating
    fibres, the register march when isotropic), pure diffusion of a smooth field for 3
    steps: 32 sampled voxels match the FP64 oracle run on 9^3 crops around them (a value
    after 3 steps depends only on voxels within 3 of it, plus the fibres one further); the
    same run continued to step 30 matches it on 12 voxels (corners included) on 63^3 crops
    within 5e-4 (measured at most 4.9e-5)."""
    from oracle import oracle as O
    from paper_1605_06015_amd import bbx as B
    nx, ny, nz, h, dt, Dpar, Dperp = 512, 512, 264, 0.25, 0.01, 0.3, 0.03
    assert nx * ny * nz * 4 > 256 * 1024 * 1024
    mask, fib = WL.full_box_rotating(nx, ny, nz)
    if not aniso:
        fib = None
    elif aniso == "random":
        # fibres varying in every direction: the tensor-gradient coefficients the kernel
        # rebuilds are nonzero everywhere (rotating in z alone they vanish)
        fib = WL.random_fibres(mask.shape, seed=17)
    z, y, x = np.ogrid[0:nz, 0:ny, 0:nx]
    V = -60.0 + 20.0 * np.sin(0.05 * x + 0.3) * np.cos(0.07 * y) + 10.0 * np.sin(0.11 * z)
    g = B.Grid(mask, h, fib, Dpar, Dperp, B.BBX_FP32)
    g.model(B.BBX_MODEL_NONE, [], dt)
    g.set(0, V)
    Vb = np.broadcast_to(V, (nz, ny, nx))

    def check(got, picks, nsteps, tol):
        r = nsteps + 1
        for c in picks:
            sl = tuple(slice(max(0, c[i] - r), min((nz, ny, nx)[i], c[i] + r + 1)) for i in range(3))
            cm = np.ascontiguousarray(mask[sl])
            cf = None if fib is None else np.ascontiguousarray(fib[sl])
            s = O.Sim(cm, h, cf, Dpar, Dperp, O.MODEL_NONE, [], dt)
            s.state[0] = Vb[sl]
            s.step(nsteps)
            loc = tuple(int(c[i] - sl[i].start) for i in range(3))
            want = s.state[0][loc]
            assert abs(got[tuple(c)] - want) <= tol, (nsteps, tuple(c), got[tuple(c)], want)

    g.step(3)
    got = g.get(0)
    rng = np.random.default_rng(3)
    picks = np.stack([rng.integers(0, nz, 32), rng.integers(0, ny, 32), rng.integers(0, nx, 32)], 1)
    picks[:4] = [[0, 0, 0], [nz - 1, ny - 1, nx - 1], [nz // 2, 0, nx - 1], [nz - 1, ny // 2, 0]]
    check(got, picks, 3, 1e-4)
    del got
    g.step(27)
    got = g.get(0)
    g.close()
    picks = np.stack([rng.integers(0, nz, 12), rng.integers(0, ny, 12), rng.integers(0, nx, 12)], 1)
    picks[:2] = [[0, 0, 0], [nz - 1, ny - 1, nx - 1]]
    check(got, picks, 30, 5e-4)
