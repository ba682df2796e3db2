"""Pins of the oracle's phase-singularity finder (the `singz` device: intersections of
isolines of two fields in z cross-sections, the isoline pieces in each cell from
linear interpolation): exact points for linear fields, symmetry, masking, the saddle
rule, and second-order convergence of the point for smooth fields."""
import numpy as np
import pytest

from oracle import oracle as O


def grid(nx, ny, nz):
    return np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")


@pytest.mark.parametrize("a,b,c,d", [(1.0, 0.0, 0.0, 1.0), (1.0, 0.5, -0.3, 1.0),
                                     (-0.2, 1.3, 0.9, 0.4)])
def test_linear_fields_exact_point_per_plane(a, b, c, d):
    """Linear fields are reproduced exactly by the interpolation: one point per plane at
    the fields' common zero (x0, y0), whatever the (non-singular) mixing."""
    nz, ny, nx, h = 4, 21, 25, 0.3
    z, y, x = grid(nx, ny, nz)
    x0, y0 = 9.37, 12.61
    u = a * (x - x0) + b * (y - y0)
    v = c * (x - x0) + d * (y - y0)
    st, pts = O.tips(np.ones((nz, ny, nx), np.uint8), h, u, 0.0, v, 0.0)
    assert st[0] == nz
    assert np.allclose(pts[:, 0], h * x0, atol=1e-12) and np.allclose(pts[:, 1], h * y0, atol=1e-12)
    assert np.allclose(pts[:, 2], h * np.arange(nz))
    assert np.allclose(st[1:4], [h * x0, h * y0, h * (nz - 1) / 2])
    assert np.allclose(st[4:6], 0.0, atol=1e-9)
    assert abs(st[6] - h * np.std(np.arange(nz))) < 1e-12
    # levels: u = 1.5 and v = -2 moves the point to the solution of the shifted system
    st2, pts2 = O.tips(np.ones((nz, ny, nx), np.uint8), h, u, 1.5, v, -2.0)
    sol = np.linalg.solve([[a, b], [c, d]], [1.5, -2.0]) + [x0, y0]
    assert np.allclose(pts2[0, :2], h * sol, atol=1e-12)


def test_swapping_fields_gives_same_points():
    rng = np.random.default_rng(1)
    nz, ny, nx = 2, 30, 30
    u = rng.standard_normal((nz, ny, nx))
    v = rng.standard_normal((nz, ny, nx))
    m = np.ones((nz, ny, nx), np.uint8)
    s1, p1 = O.tips(m, 1.0, u, 0.1, v, -0.2)
    s2, p2 = O.tips(m, 1.0, v, -0.2, u, 0.1)
    assert s1[0] == s2[0] > 10
    k1 = np.lexsort(p1.T[::-1])
    k2 = np.lexsort(p2.T[::-1])
    assert np.allclose(p1[k1], p2[k2], atol=1e-12)
    assert np.allclose(s1, s2, rtol=1e-12, atol=1e-12)


def test_cells_with_a_void_corner_are_skipped():
    nz, ny, nx = 1, 10, 10
    z, y, x = grid(nx, ny, nz)
    u, v = x - 4.5, y - 5.5
    m = np.ones((nz, ny, nx), np.uint8)
    assert O.tips(m, 1.0, u, 0.0, v, 0.0)[0][0] == 1
    m[0, 6, 5] = 0          # a corner of the cell holding the point
    assert O.tips(m, 1.0, u, 0.0, v, 0.0)[0][0] == 0


def test_saddle_pairing_rule():
    """One cell, u with a saddle (corners 00, 11 above, 10, 01 below, centre on the
    level: counts as above) and v = x - y (its isoline the cell's diagonal).  The u
    segments then cut off corners 10 and 01 and miss the diagonal; with u negated they
    cut off 00 and 11 and cross it twice, at (1/4, 1/4) and (3/4, 3/4)."""
    m = np.ones((1, 2, 2), np.uint8)
    u = np.array([[[1.0, -1.0], [-1.0, 1.0]]])
    z, y, x = grid(2, 2, 1)
    v = (x - y).astype(float)
    st, _ = O.tips(m, 1.0, u, 0.0, v, 0.0)
    assert st[0] == 0
    st, pts = O.tips(m, 1.0, -u, 0.0, v, 0.0)
    assert st[0] == 2
    assert np.allclose(np.sort(pts[:, 0]), [0.25, 0.75]) and np.allclose(pts[:, 0], pts[:, 1])


def test_second_order_convergence_smooth_fields():
    """Smooth nonlinear fields with the common zero (a, b): the point's error under grid
    refinement falls at second order (the interpolation is exact to first order).  The
    zero sits at the same relative position (0.37, 0.61) inside its cell at every
    resolution, so that the error constant does not change with the refinement."""
    errs = []
    for n in (24, 48, 96, 192):
        h = 6.0 / n
        a, b = h * (n // 2 + 0.37), h * (n // 2 + 0.61)
        X = np.arange(n) * h
        XX, YY = np.meshgrid(X, X, indexing="xy")
        dx, dy = XX - a, YY - b
        u = (dx + 0.4 * dy * dy + 0.3 * dx * dy)[None]
        v = (dy - 0.5 * dx * dx + 0.2 * dx * dy)[None]
        st, pts = O.tips(np.ones((1, n, n), np.uint8), h, u, 0.0, v, 0.0)
        assert st[0] >= 1            # the fields have a second common zero farther out
        errs.append(np.hypot(pts[:, 0] - a, pts[:, 1] - b).min())
    errs = np.array(errs)
    order = np.log2(errs[:-1] / errs[1:])
    print("errors", errs, "orders", order)
    assert np.all(order > 1.6) and np.all(order < 2.6)
