"""Pins of the oracle's line probes (Sec. 3.1): trilinear interpolation
between cell centres over the fluid cells around a point."""
import math
from types import SimpleNamespace

import numpy as np
import pytest

from oracle import oracle as O


def _case(n, h, solid=None, dim=3):
    return SimpleNamespace(n=n, h=h, dim=dim, solid=solid)


def _linear(n, h, coef):
    nx, ny, nz = n
    x = (np.arange(nx) + 0.5) * h[0]
    y = (np.arange(ny) + 0.5) * h[1]
    z = (np.arange(nz) + 0.5) * h[2]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return coef[0] + coef[1] * X + coef[2] * Y + coef[3] * Z


def _fields(n, h, rng):
    names = ("u", "v", "w", "T", "k", "omega")
    coefs = {nm: rng.normal(size=4) for nm in names}
    return {nm: _linear(n, h, coefs[nm]) for nm in names}, coefs


def test_linear_fields_are_reproduced_exactly():
    """Trilinear interpolation is exact for fields linear in x, y, z: T, k and
    omega at interior points equal the linear function, V the magnitude of
    the three linear components."""
    rng = np.random.default_rng(3)
    n, h = (7, 5, 6), (0.1, 0.2, 0.15)
    f, co = _fields(n, h, rng)
    L = [n[d] * h[d] for d in range(3)]
    pts = np.column_stack([rng.uniform(0.5 * h[d], L[d] - 0.5 * h[d], 40) for d in range(3)])
    out = O.line_probe(_case(n, h), f, pts)
    lin = lambda c, p: c[0] + c[1] * p[:, 0] + c[2] * p[:, 1] + c[3] * p[:, 2]
    V = np.sqrt(lin(co["u"], pts) ** 2 + lin(co["v"], pts) ** 2 + lin(co["w"], pts) ** 2)
    np.testing.assert_allclose(out[:, 0], V, rtol=1e-12, atol=1e-12)
    for col, nm in ((1, "T"), (2, "k"), (3, "omega")):
        np.testing.assert_allclose(out[:, col], lin(co[nm], pts), rtol=1e-12, atol=1e-12)


def test_cell_centres_return_cell_values():
    rng = np.random.default_rng(4)
    n, h = (4, 3, 5), (0.3, 0.2, 0.1)
    f = {nm: rng.normal(size=n[::-1]) for nm in ("u", "v", "w", "T", "k", "omega")}
    ijk = [(0, 0, 0), (3, 2, 4), (1, 2, 3), (2, 0, 1)]
    pts = np.array([[(i + 0.5) * h[0], (j + 0.5) * h[1], (k + 0.5) * h[2]] for i, j, k in ijk])
    out = O.line_probe(_case(n, h), f, pts)
    for q, (i, j, k) in enumerate(ijk):
        # (x / h - 1/2 lands on i up to rounding)
        assert out[q, 1] == pytest.approx(f["T"][k, j, i], rel=1e-13, abs=1e-15)
        assert out[q, 3] == pytest.approx(f["omega"][k, j, i], rel=1e-13, abs=1e-15)
        assert out[q, 0] == pytest.approx(math.sqrt(sum(f[c][k, j, i] ** 2 for c in "uvw")),
                                          rel=1e-13)


def test_points_outside_the_centres_are_clamped():
    """Between the wall and the first cell centre the probe takes the value at
    the nearest point of the box of centres."""
    n, h = (3, 3, 3), (1.0, 1.0, 1.0)
    f, co = _fields(n, h, np.random.default_rng(5))
    inside = O.line_probe(_case(n, h), f, [[0.5, 1.5, 2.5]])
    edge = O.line_probe(_case(n, h), f, [[0.0, 1.5, 3.0]])
    np.testing.assert_array_equal(inside, edge)


def test_solid_corners_are_left_out_and_weights_renormalised():
    """A point among eight cells of which some are solid: the fluid cells all
    hold the value c, so the renormalised average is c whatever the weights;
    with every corner solid the probe is NaN."""
    n, h = (2, 2, 2), (1.0, 1.0, 1.0)
    solid = np.zeros((2, 2, 2), np.uint8)
    solid[0, 0, 0] = solid[1, 1, 0] = 1
    f = {nm: np.where(solid == 0, 2.5, 1e6) for nm in ("u", "v", "w", "T", "k", "omega")}
    out = O.line_probe(_case(n, h, solid), f, [[0.8, 1.1, 0.7], [0.6, 0.6, 0.6]])
    np.testing.assert_allclose(out[:, 1:], 2.5, rtol=1e-15)
    np.testing.assert_allclose(out[:, 0], 2.5 * math.sqrt(3), rtol=1e-15)
    all_solid = O.line_probe(_case(n, h, np.ones((2, 2, 2), np.uint8)), f, [[1.0, 1.0, 1.0]])
    assert np.isnan(all_solid).all()


def test_renormalisation_matches_hand_weights():
    """One solid corner of eight: the value is the weighted mean of the other
    seven with the trilinear weights divided by their sum (hand-computed)."""
    n, h = (2, 2, 2), (1.0, 1.0, 1.0)
    solid = np.zeros((2, 2, 2), np.uint8)
    solid[1, 1, 1] = 1
    vals = np.arange(8, dtype=float).reshape(2, 2, 2)  # [k][j][i] = 4k + 2j + i
    f = {nm: vals for nm in ("u", "v", "w", "T", "k", "omega")}
    x = np.array([0.75, 0.9, 0.6])  # t = (0.25, 0.4, 0.1)
    t = x - 0.5
    num = den = 0.0
    for k in range(2):
        for j in range(2):
            for i in range(2):
                if (i, j, k) == (1, 1, 1):
                    continue
                wt = (t[0] if i else 1 - t[0]) * (t[1] if j else 1 - t[1]) * (t[2] if k else 1 - t[2])
                num += wt * (4 * k + 2 * j + i)
                den += wt
    out = O.line_probe(_case(n, h, solid), f, [x])
    assert out[0, 1] == pytest.approx(num / den, rel=1e-14)


def test_two_dimensional_grids_ignore_z():
    n, h = (5, 4, 1), (0.1, 0.1, 1.0)
    f, co = _fields(n, h, np.random.default_rng(6))
    a = O.line_probe(_case(n, h, dim=2), f, [[0.23, 0.17, 0.0]])
    b = O.line_probe(_case(n, h, dim=2), f, [[0.23, 0.17, 9.0]])
    np.testing.assert_array_equal(a, b)
    assert a[0, 1] == pytest.approx(co["T"][0] + co["T"][1] * 0.23 + co["T"][2] * 0.17
                                    + co["T"][3] * 0.5, rel=1e-12)
