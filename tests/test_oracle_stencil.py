"""Pins of the oracle's stencil ("Monodomain diffusion and boundary conditions",
eqs (Lu), (nonflux), (sigma) and the weight formulas) against what mathematics
fixes: polynomial exactness, second-order consistency with variable fibres,
zero row sums, symmetry and conservation for uniform tensors on any mask,
lattice symmetries, and the Gaussian closed form of the diffusion equation."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1605_06015_amd import workloads as WL


def tensor(f, Dpar, Dperp):
    f = np.asarray(f, float) / np.linalg.norm(f)
    return Dperp * np.eye(3) + (Dpar - Dperp) * np.outer(f, f)


def coords(shape, h):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x * h, y * h, z * h


def test_row_sums_zero_any_mask_and_fibres():
    mask = WL.random_blob_mask(12, 10, 9, seed=3, frac=0.55)
    fib = WL.random_fibres(mask.shape, seed=4)
    act, W = O.weights(mask, 0.3, fib, 1.3, 0.2)
    assert np.abs(W.sum(axis=1)).max() < 1e-12 * np.abs(W).max()
    Lc = O.apply_L(mask, act, W, np.full(mask.shape, 2.5))
    assert np.abs(Lc).max() == 0.0


def test_weights_vanish_towards_void_and_corners():
    mask = WL.random_blob_mask(10, 9, 8, seed=5, frac=0.5)
    fib = WL.random_fibres(mask.shape, seed=6)
    act, W = O.weights(mask, 0.5, fib, 1.0, 0.1)
    nz, ny, nx = mask.shape
    pad = np.pad(mask, 1)
    for a, p in enumerate(act):
        x, y, z = p % nx, (p // nx) % ny, p // (nx * ny)
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    qi = (dz + 1) * 9 + (dy + 1) * 3 + dx + 1
                    if qi == 13:
                        continue
                    if abs(dx) + abs(dy) + abs(dz) == 3 or pad[z + dz + 1, y + dy + 1, x + dx + 1] == 0:
                        assert W[a, qi] == 0.0


@pytest.mark.parametrize("fdir", [(1, 0, 0), (1, 2, 0.5), (-0.3, 0.8, 1.1)])
def test_quadratic_exactness_uniform_tensor(fdir):
    """For uniform D: L x_j = 0, L x_j^2 = 2 D_jj, L x_j x_k = 2 D_jk at interior voxels."""
    shape, h = (7, 8, 9), 0.37
    mask = np.ones(shape, np.uint8)
    fib = np.broadcast_to(np.asarray(fdir, float), shape + (3,)).copy()
    Dpar, Dperp = 1.7, 0.4
    D = tensor(fdir, Dpar, Dperp)
    act, W = O.weights(mask, h, fib, Dpar, Dperp)
    X = coords(shape, h)
    nz, ny, nx = shape
    z, y, x = act // (nx * ny), (act // nx) % ny, act % nx
    interior = (x > 0) & (x < nx - 1) & (y > 0) & (y < ny - 1) & (z > 0) & (z < nz - 1)
    for j in range(3):
        L1 = O.apply_L(mask, act, W, X[j])
        assert np.abs(L1[interior]).max() < 1e-11
        for k in range(3):
            Lq = O.apply_L(mask, act, W, X[j] * X[k])
            np.testing.assert_allclose(Lq[interior], 2 * D[j, k], rtol=0, atol=1e-10)


def _manufactured(h, kap=(0.7, 0.5)):
    """Variable fibres f(x,y) = (cos t, sin t cos s, sin t sin s), t = k1 x + .3, s = k2 y + .2;
    u = sin(x) cos(y) exp(z/2).  Returns the interior max error of L u."""
    n = int(round(3.0 / h)) + 1
    shape = (n, n, n)
    mask = np.ones(shape, np.uint8)
    x, y, z = coords(shape, h)
    Dpar, Dperp = 1.0, 0.15

    def fib(x, y):
        t = kap[0] * x + 0.3
        s = kap[1] * y + 0.2
        return np.stack([np.cos(t), np.sin(t) * np.cos(s), np.sin(t) * np.sin(s)], -1)

    def Dfun(x, y):
        f = fib(x, y)
        return Dperp * np.eye(3) + (Dpar - Dperp) * f[..., :, None] * f[..., None, :]

    act, W = O.weights(mask, h, fib(x, y), Dpar, Dperp)
    u = np.sin(x) * np.cos(y) * np.exp(0.5 * z)
    Lu = O.apply_L(mask, act, W, u)
    # exact: sum_jk D_jk u_jk + sum_k (sum_j d_j D_jk) u_k, derivatives of D by a
    # 4th-order central difference of the analytic tensor (error ~1e-12).
    xs, ys, zs = x.ravel()[act], y.ravel()[act], z.ravel()[act]
    D = Dfun(xs, ys)
    d = 1e-3

    def dd(fun, e):
        return (-fun(2 * e) + 8 * fun(e) - 8 * fun(-e) + fun(-2 * e)) / (12 * d)

    dDx = dd(lambda s: Dfun(xs + s * d, ys), 1)
    dDy = dd(lambda s: Dfun(xs, ys + s * d), 1)
    divD = dDx[:, 0, :] + dDy[:, 1, :]          # sum_j d_j D_jk (D independent of z)
    e = np.exp(0.5 * zs)
    ux = np.cos(xs) * np.cos(ys) * e
    uy = -np.sin(xs) * np.sin(ys) * e
    uz = 0.5 * np.sin(xs) * np.cos(ys) * e
    H = np.empty((xs.size, 3, 3))
    H[:, 0, 0] = -np.sin(xs) * np.cos(ys) * e
    H[:, 1, 1] = -np.sin(xs) * np.cos(ys) * e
    H[:, 2, 2] = 0.25 * np.sin(xs) * np.cos(ys) * e
    H[:, 0, 1] = H[:, 1, 0] = -np.cos(xs) * np.sin(ys) * e
    H[:, 0, 2] = H[:, 2, 0] = 0.5 * np.cos(xs) * np.cos(ys) * e
    H[:, 1, 2] = H[:, 2, 1] = -0.5 * np.sin(xs) * np.sin(ys) * e
    exact = (D * H).sum(axis=(1, 2)) + divD[:, 0] * ux + divD[:, 1] * uy + divD[:, 2] * uz
    nx = n
    xi, yi, zi = act % nx, (act // nx) % nx, act // (nx * nx)
    inner = (xi > 1) & (xi < n - 2) & (yi > 1) & (yi < n - 2) & (zi > 1) & (zi < n - 2)
    return np.abs(Lu - exact)[inner].max()


def test_variable_fibres_second_order():
    e1 = _manufactured(0.2)
    e2 = _manufactured(0.1)
    assert e2 < 2e-2
    assert 3.3 < e1 / e2 < 4.8, (e1, e2)


@pytest.mark.parametrize("fdir", [(1, 0, 0), (0.6, 0.8, 0.0), (1, -1, 2)])
def test_uniform_tensor_symmetric_and_conservative_on_any_mask(fdir):
    mask = WL.random_blob_mask(14, 12, 10, seed=7, frac=0.6)
    fib = np.broadcast_to(np.asarray(fdir, float), mask.shape + (3,)).copy()
    act, W = O.weights(mask, 0.25, fib, 0.3, 0.03)
    nz, ny, nx = mask.shape
    pos = {int(p): a for a, p in enumerate(act)}
    for a, p in enumerate(act):
        x, y, z = p % nx, (p // nx) % ny, p // (nx * ny)
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    qi = (dz + 1) * 9 + (dy + 1) * 3 + dx + 1
                    if qi == 13 or W[a, qi] == 0.0:
                        continue
                    b = pos[int(p + dx + nx * (dy + ny * dz))]
                    back = (-dz + 1) * 9 + (-dy + 1) * 3 + (-dx + 1)
                    assert abs(W[a, qi] - W[b, back]) < 1e-12 * abs(W[a, qi])
    u = np.random.default_rng(0).standard_normal(mask.shape)
    Lu = O.apply_L(mask, act, W, u)
    assert abs(Lu.sum()) < 1e-12 * np.abs(Lu).sum()


def test_lattice_symmetry_isotropic():
    mask = WL.random_blob_mask(11, 11, 6, seed=9, frac=0.6)
    u = np.random.default_rng(1).standard_normal(mask.shape)
    act, W = O.weights(mask, 0.2, None, 0.5, 0.5)
    Lu = np.zeros(mask.size)
    Lu[act] = O.apply_L(mask, act, W, u)
    Lu = Lu.reshape(mask.shape)
    for op in (lambda a: np.rot90(a, 1, axes=(1, 2)), lambda a: a[:, :, ::-1],
               lambda a: a[::-1], lambda a: np.swapaxes(a, 1, 2)):
        m2, u2 = np.ascontiguousarray(op(mask)), np.ascontiguousarray(op(u))
        act2, W2 = O.weights(m2, 0.2, None, 0.5, 0.5)
        L2 = np.zeros(m2.size)
        L2[act2] = O.apply_L(m2, act2, W2, u2)
        np.testing.assert_allclose(L2.reshape(m2.shape), op(Lu), rtol=0, atol=1e-12)


def _gaussian_error(h, fdir=(np.cos(0.5), np.sin(0.5), 0.0), Dpar=1.0, Dperp=0.25):
    L = 6.4
    n = int(round(L / h))
    mask = np.ones((1, n, n), np.uint8)
    fib = np.broadcast_to(np.asarray(fdir, float), mask.shape + (3,)).copy()
    D = tensor(fdir, Dpar, Dperp)[:2, :2]
    s0, T = 0.5, 0.1
    dt = h * h / 16.0
    nsteps = int(round(T / dt))
    dt = T / nsteps
    x, y, _ = coords(mask.shape, h)
    c = 0.5 * (n - 1) * h
    X = np.stack([x[0] - c, y[0] - c], -1)

    def exact(t):
        S = s0 ** 2 * np.eye(2) + 2 * t * D
        Si = np.linalg.inv(S)
        q = np.einsum("...i,ij,...j->...", X, Si, X)
        return s0 ** 2 / np.sqrt(np.linalg.det(S)) * np.exp(-0.5 * q)

    sim = O.Sim(mask, h, fib, Dpar, Dperp, O.MODEL_NONE, [], dt)
    sim.set_state(0, exact(0.0)[None])
    sim.step(nsteps)
    return np.abs(sim.state[0, 0] - exact(T)).max()


def test_gaussian_closed_form_anisotropic():
    e1 = _gaussian_error(0.2)
    e2 = _gaussian_error(0.1)
    assert e2 < 5e-3
    assert 3.0 < e1 / e2 < 5.0, (e1, e2)


def test_zero_fibre_rejected():
    mask = np.ones((2, 2, 2), np.uint8)
    fib = np.ones((2, 2, 2, 3))
    fib[1, 1, 0] = 0.0
    with pytest.raises(ValueError):
        O.weights(mask, 0.1, fib, 1.0, 0.1)
    fib2 = fib.copy()
    mask[1, 1, 0] = 0          # void voxels' fibres are ignored
    O.weights(mask, 0.1, fib2, 1.0, 0.1)
