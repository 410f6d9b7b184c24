"""Pins of the oracle's implicit-surface initial values (Sec. 2.2, Fig. 4).

- the cylinder and the box equal the input generators' independent numpy
  signed distances bit for bit;
- the sphere and the box are signed distances: against brute-force distances
  to densely sampled surface points (within the sampling error), negative
  inside, -r at the centre;
- the ellipsoid is the quadratic form of the paper's ellipsoid listing;
- union, intersection and difference are min, max and max(v, -s) of the
  separate shapes.
"""
import math

import numpy as np
import pytest

from paper_2507_11542_amd import inputs

GRID2 = ((41, 37), (-3.0, -2.5), (3.0, 2.5), (False, False))
GRID3 = ((23, 21, 19), (-2.0, -2.0, -2.0), (2.0, 2.0, 2.0), (False, False, True))


def _coords(grid):
    return np.meshgrid(*inputs.node_coords(*grid), indexing="ij")


def test_cylinder_and_box_equal_the_generators(orc):
    n, lo, hi, per = GRID3
    cyl = orc.shapes(n, lo, hi, per, [dict(kind="cylinder", axes=(0, 1), radius=1.1)])
    assert np.array_equal(cyl, inputs.sdf_cylinder(n, lo, hi, per, 1.1, (0, 1)))
    box = orc.shapes(n, lo, hi, per, [dict(kind="box", axes=(0, 2), center=(0.3, 0.0, -0.2),
                                           size=(0.7, 0.0, 0.4))])
    ref = inputs.sdf_box(n, lo, hi, per, (0.3, -0.2), (0.7, 0.4), (0, 2))
    assert np.array_equal(box, ref)


def _brute_distance(pts, surf):
    d = np.sqrt(((pts[:, None, :] - surf[None, :, :]) ** 2).sum(-1))
    return d.min(axis=1)


def test_sphere_is_a_signed_distance(orc):
    n, lo, hi, per = GRID2
    c, r = (0.4, -0.3), 1.3
    v = orc.shapes(n, lo, hi, per, [dict(kind="sphere", center=c, radius=r)])
    X, Y = _coords(GRID2)
    th = np.linspace(0, 2 * math.pi, 20000, endpoint=False)
    surf = np.stack([c[0] + r * np.cos(th), c[1] + r * np.sin(th)], axis=1)
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    dist = _brute_distance(pts, surf)
    inside = (X.ravel() - c[0]) ** 2 + (Y.ravel() - c[1]) ** 2 < r * r
    signed = np.where(inside, -dist, dist)
    assert np.abs(v.ravel() - signed).max() < 2e-4  # half the sample spacing


def test_box_is_a_signed_distance(orc):
    n, lo, hi, per = GRID2
    c, h = (-0.2, 0.35), (1.1, 0.6)
    v = orc.shapes(n, lo, hi, per, [dict(kind="box", center=c, size=h)])
    X, Y = _coords(GRID2)
    m = 4000
    xs = np.linspace(c[0] - h[0], c[0] + h[0], m)
    ys = np.linspace(c[1] - h[1], c[1] + h[1], m)
    surf = np.concatenate([
        np.stack([xs, np.full(m, c[1] - h[1])], 1), np.stack([xs, np.full(m, c[1] + h[1])], 1),
        np.stack([np.full(m, c[0] - h[0]), ys], 1), np.stack([np.full(m, c[0] + h[0]), ys], 1)])
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    dist = np.concatenate([_brute_distance(pts[i:i + 200], surf)
                           for i in range(0, len(pts), 200)])
    inside = (np.abs(X.ravel() - c[0]) < h[0]) & (np.abs(Y.ravel() - c[1]) < h[1])
    signed = np.where(inside, -dist, dist)
    assert np.abs(v.ravel() - signed).max() < 1e-3


def test_sphere_centre_and_lipschitz(orc):
    n, lo, hi, per = (21, 21, 21), (-1.0,) * 3, (1.0,) * 3, (False,) * 3
    v = orc.shapes(n, lo, hi, per, [dict(kind="sphere", radius=0.5)])
    assert v[10, 10, 10] == -0.5
    dx = 0.1
    for ax in range(3):
        assert np.abs(np.diff(v, axis=ax)).max() <= dx * (1 + 1e-12)


def test_ellipsoid_is_the_listing_form(orc):
    """The ellipsoid listing: x^2 + 4 y^2 (+ 9 z^2 in 3-D) minus the radius."""
    n, lo, hi, per = GRID3
    v = orc.shapes(n, lo, hi, per, [dict(kind="ellipsoid", size=(1.0, 4.0, 9.0), radius=2.0)])
    X, Y, Z = _coords(GRID3)
    assert np.abs(v - (X ** 2 + 4.0 * Y ** 2 + 9.0 * Z ** 2 - 2.0)).max() < 1e-13


@pytest.mark.parametrize("op,combine", [("union", np.minimum), ("intersect", np.maximum),
                                        ("subtract", lambda a, b: np.maximum(a, -b))])
def test_boolean_operations(orc, op, combine):
    n, lo, hi, per = GRID2
    a = dict(kind="sphere", center=(-0.8, 0.0), radius=1.0)
    b = dict(kind="box", center=(0.7, 0.2), size=(0.9, 0.5), op=op)
    va = orc.shapes(n, lo, hi, per, [a])
    vb = orc.shapes(n, lo, hi, per, [b])
    vab = orc.shapes(n, lo, hi, per, [a, b])
    assert np.array_equal(vab, combine(va, vb))
