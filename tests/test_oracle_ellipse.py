"""Pins of the oracle's exact ellipse-cell area (the solid fraction of an
elliptical particle, Sec. 3.2) and of its readings for ellipses: the band of
the circumscribed disk, cells wholly inside the inscribed disk.

The area is an exact column integral (the chord of a rotated ellipse has a
linear centre and a square-root half-width).  It is pinned by what fixes it
independently: with equal semi-axes it is the disk's area, computed by a
different formula; over the whole grid the areas add up to pi a b; brute
force by point sampling; the ellipse's symmetries (a half turn, swapping the
axes with a quarter turn, turning the whole picture by 90 degrees); and the
band and inside readings bound it.
"""
import math

import numpy as np
import pytest


def boundary_cells(X, Y, a, b, th, rng, n):
    """n random cells crossed by the ellipse's boundary."""
    c, s = math.cos(th), math.sin(th)
    out = []
    while len(out) < n:
        phi = rng.uniform(0, 2 * math.pi)
        u, v = a * math.cos(phi), b * math.sin(phi)
        px, py = X + c * u - s * v, Y + s * u + c * v
        out.append((math.floor(px), math.floor(py)))
    return out


def test_equal_axes_give_the_disk_area(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(1)
    worst = 0.0
    for _ in range(300):
        R = rng.uniform(0.6, 20.0)
        X, Y = rng.uniform(30, 31), rng.uniform(30, 31)
        th = rng.uniform(0, 2 * math.pi)
        for i, j in boundary_cells(X, Y, R, R, 0.0, rng, 4):
            e = O.ellipse_cell_area(X, Y, R, R, th, i, j)
            d = O.disk_cell_area(X, Y, R, i, j)
            worst = max(worst, abs(e - d))
    assert worst < 1e-13, worst


@pytest.mark.parametrize("seed", range(6))
def test_areas_add_up_to_pi_a_b(oracle_mod, seed):
    O = oracle_mod
    rng = np.random.default_rng(100 + seed)
    a = rng.uniform(2.0, 14.0)
    b = a * rng.uniform(0.2, 0.95)
    th = rng.uniform(0, 2 * math.pi)
    X, Y = rng.uniform(20, 21), rng.uniform(20, 21)
    lo, hi = int(X - a) - 2, int(X + a) + 3
    tot = sum(O.ellipse_cell_area(X, Y, a, b, th, i, j)
              for i in range(lo, hi) for j in range(int(Y - a) - 2,
                                                     int(Y + a) + 3))
    assert abs(tot - math.pi * a * b) < 1e-12 * math.pi * a * b, tot


def test_point_sampling(oracle_mod):
    """Midpoint sampling on a 1200 x 1200 grid per cell agrees within the
    sampling error (about the boundary's length in the cell over N)."""
    O = oracle_mod
    rng = np.random.default_rng(7)
    N = 1200
    g = (np.arange(N) + 0.5) / N
    gx, gy = np.meshgrid(g, g)
    worst = 0.0
    for _ in range(12):
        a = rng.uniform(1.5, 12.0)
        b = a * rng.uniform(0.25, 0.9)
        th = rng.uniform(0, 2 * math.pi)
        X, Y = rng.uniform(10, 11), rng.uniform(10, 11)
        c, s = math.cos(th), math.sin(th)
        for i, j in boundary_cells(X, Y, a, b, th, rng, 3):
            dx, dy = i + gx - X, j + gy - Y
            u, v = c * dx + s * dy, -s * dx + c * dy
            inside = (u / a) ** 2 + (v / b) ** 2 < 1.0
            exact = O.ellipse_cell_area(X, Y, a, b, th, i, j)
            worst = max(worst, abs(inside.mean() - exact))
    assert worst < 3.0 / N, worst


def test_symmetries(oracle_mod):
    """A half turn changes nothing; (a, b, theta) is (b, a, theta + pi/2);
    turning the whole picture by 90 degrees about the origin maps cell
    (i, j) to (-j - 1, i) and the centre (X, Y) to (-Y, X)."""
    O = oracle_mod
    rng = np.random.default_rng(3)
    w1 = w2 = w3 = 0.0
    for _ in range(60):
        a = rng.uniform(1.0, 15.0)
        b = a * rng.uniform(0.2, 0.95)
        th = rng.uniform(0, 2 * math.pi)
        X, Y = rng.uniform(40, 41), rng.uniform(40, 41)
        for i, j in boundary_cells(X, Y, a, b, th, rng, 4):
            A0 = O.ellipse_cell_area(X, Y, a, b, th, i, j)
            w1 = max(w1, abs(A0 - O.ellipse_cell_area(X, Y, a, b, th + math.pi,
                                                      i, j)))
            w2 = max(w2, abs(A0 - O.ellipse_cell_area(X, Y, b, a,
                                                      th + math.pi / 2, i, j)))
            w3 = max(w3, abs(A0 - O.ellipse_cell_area(-Y, X, a, b,
                                                      th + math.pi / 2,
                                                      -j - 1, i)))
    assert w1 < 1e-13 and w2 < 1e-13 and w3 < 1e-13, (w1, w2, w3)


def test_band_and_inside_readings_bound_the_area(oracle_mod):
    """Outside the circumscribed disk's band the area is zero; inside the
    inscribed disk it is one."""
    O = oracle_mod
    rng = np.random.default_rng(5)
    for _ in range(20):
        a = rng.uniform(2.0, 12.0)
        b = a * rng.uniform(0.3, 0.9)
        th = rng.uniform(0, 2 * math.pi)
        X, Y = rng.uniform(20, 21), rng.uniform(20, 21)
        for i in range(int(X - a) - 3, int(X + a) + 4):
            for j in range(int(Y - a) - 3, int(Y + a) + 4):
                A = O.ellipse_cell_area(X, Y, a, b, th, i, j)
                if not O.cell_in_band(X, Y, a, i, j):
                    assert A == 0.0
                if O.cell_inside(X, Y, b, i, j):
                    assert abs(A - 1.0) < 1e-14
