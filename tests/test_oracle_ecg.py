"""Pins of the oracle's pseudo-ECG, phi(x_e) = h^3 sum_p (L V)_p / |x_p - x_e|:
the monopole vanishes for a uniform tensor (L has zero column sums), and the far
field of a linear ramp on a full box is the dipole given in closed form by
summation by parts over the stencil's links."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1605_06015_amd import workloads as WL


def unit(v):
    v = np.asarray(v, float)
    return v / np.linalg.norm(v)


def test_monopole_vanishes_for_uniform_tensor():
    mask = WL.random_blob_mask(14, 12, 9, seed=2)
    f = unit([0.6, -0.3, 0.74])
    fib = np.broadcast_to(f, mask.shape + (3,)).copy()
    rng = np.random.default_rng(0)
    V = rng.standard_normal(mask.shape)
    h = 0.25
    act, W = O.weights(mask, h, fib, 0.3, 0.04)
    LV = O.apply_L(mask, act, W, V)
    scale = h ** 3 * np.abs(LV).sum()
    for d in ([1, 0, 0], [0.3, -0.8, 0.5]):
        R = 1e9
        phi = O.pseudo_ecg(mask, h, fib, 0.3, 0.04, V, [R * unit(d)])
        assert abs(R * phi[0]) <= 1e-7 * scale


def test_linear_ramp_dipole_closed_form():
    """V = a . x on a full nx x ny x nz box, uniform D: summation by parts over the links
    gives sum_p x_p (L V)_p = -sum_links W_q (q h)(q h . a), so at a far electrode R u,
    R^2 phi -> h^3 u . M with M that sum."""
    nx, ny, nz, h = 7, 6, 5, 0.2
    Dpar, Dperp = 0.3, 0.05
    f = unit([0.5, 0.7, -0.2])
    D = Dperp * np.eye(3) + (Dpar - Dperp) * np.outer(f, f)
    a = np.array([0.7, -1.1, 0.4])
    mask = np.ones((nz, ny, nx), np.uint8)
    fib = np.broadcast_to(f, mask.shape + (3,)).copy()
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    V = h * (a[0] * x + a[1] * y + a[2] * z)
    n = np.array([nx, ny, nz])
    M = np.zeros(3)
    for q in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1),
              (0, 1, 1), (0, 1, -1)]:
        q = np.array(q)
        nz_ = np.flatnonzero(q)
        if nz_.size == 1:
            w = D[nz_[0], nz_[0]] / h ** 2
        else:
            j, k = nz_
            w = np.sign(q[j] * q[k]) * D[j, k] / (2 * h ** 2)
        links = np.prod(n - np.abs(q))
        M -= w * links * (q * h) * np.dot(q * h, a)
    for d in ([1, 0, 0], [0, 1, 0], [0.2, 0.5, -0.9]):
        u = unit(d)
        R = 1e6
        phi = O.pseudo_ecg(mask, h, fib, Dpar, Dperp, V, [R * u])[0]
        want = h ** 3 * np.dot(u, M)
        assert abs(R * R * phi - want) <= 1e-5 * np.abs(M).max() * h ** 3


def test_chunking_does_not_change_the_sum():
    mask = WL.random_blob_mask(9, 8, 7, seed=5)
    fib = WL.random_fibres(mask.shape, seed=6)
    V = np.random.default_rng(1).standard_normal(mask.shape)
    E = [[-1.0, 0.5, 0.3], [3.0, 4.0, 5.5]]
    a = O.pseudo_ecg(mask, 0.3, fib, 0.2, 0.05, V, E)
    b = O.pseudo_ecg(mask, 0.3, fib, 0.2, 0.05, V, E, chunk=17)
    np.testing.assert_allclose(a, b, rtol=1e-12)
