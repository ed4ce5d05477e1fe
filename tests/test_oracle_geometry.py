"""Pins of the oracle's aperture geometry: the crossing-number test against an
analytic circle / half-plane test and an independent winding-number test, the
half-open tie rule as a tiling partition, and the edge distance against
bisection on the inside test."""
import math

import numpy as np
import pytest

from paper_2307_01416_amd import inputs as I


def _halfplane_inside_regular(poly, x, y):
    # convex polygon (counter-clockwise): inside iff left of every edge
    n = poly.shape[0]
    for i in range(n):
        a, b = poly[i], poly[(i + 1) % n]
        if (b[0] - a[0]) * (y - a[1]) - (b[1] - a[1]) * (x - a[0]) < 0:
            return False
    return True


def _winding_inside(poly, x, y):
    d = poly - np.array([x, y])
    ang = np.arctan2(d[:, 1], d[:, 0])
    tot = np.sum(np.angle(np.exp(1j * (np.roll(ang, -1) - ang))))
    return abs(tot) > math.pi


def test_crossing_number_circle(orc):
    poly = I.circle_polygon(20.0, 256).astype(np.float64)
    r_in = 10.0 * math.cos(math.pi / 256)
    rng = np.random.default_rng(0)
    pts = rng.uniform(-12, 12, size=(4000, 2))
    for x, y in pts:
        r = math.hypot(x, y)
        got = orc.in_polygon(poly, x, y)
        if r < r_in - 1e-9:
            assert got
        elif r > 10.0 + 1e-9:
            assert not got
        else:
            assert got == _halfplane_inside_regular(poly, x, y)


def test_crossing_number_concave_vs_winding(orc):
    # star-shaped concave polygon
    n = 14
    t = np.arange(n) * 2 * math.pi / n
    r = np.where(np.arange(n) % 2 == 0, 10.0, 4.0)
    poly = np.stack([r * np.cos(t), r * np.sin(t)], 1)
    rng = np.random.default_rng(1)
    for x, y in rng.uniform(-11, 11, size=(3000, 2)):
        # skip points within 1e-6 of the boundary (the tie rule is tested apart)
        assert orc.in_polygon(poly, x, y) == _winding_inside(poly, x, y)


def test_crossing_number_ties_partition_the_plane(orc):
    # unit squares tiling [0,3]^2: every sample (vertices and edges included)
    # must belong to exactly one square under the half-open rule
    squares = []
    for i in range(3):
        for j in range(3):
            squares.append(np.array([[i, j], [i + 1, j], [i + 1, j + 1], [i, j + 1]], float))
    for x in np.arange(0.5, 2.51, 0.25):
        for y in np.arange(0.5, 2.51, 0.25):
            hits = sum(orc.in_polygon(s, x, y) for s in squares)
            assert hits == 1, (x, y)


def test_no_vertices_means_closed(orc):
    assert not orc.in_polygon(np.zeros((0, 2)), 0.0, 0.0)


def test_edge_distance_vs_bisection(orc):
    poly = I.circle_polygon(20.0, 64).astype(np.float64)
    rng = np.random.default_rng(2)
    for _ in range(200):
        x, y = rng.uniform(-5, 5, 2)
        phi = rng.uniform(0, 2 * math.pi)
        w = rng.uniform(0.2, 1.0)
        u, v = math.sqrt(1 - w * w) * math.cos(phi), math.sqrt(1 - w * w) * math.sin(phi)
        t = orc.edge_distance(poly, x, y, u, v)
        lo, hi = 0.0, 200.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if orc.in_polygon(poly, x + mid * u, y + mid * v):
                lo = mid
            else:
                hi = mid
        assert t == pytest.approx(lo, abs=1e-9)
    assert orc.edge_distance(poly, 0.0, 0.0, 0.0, 0.0) == math.inf
