"""Deformation factor of a drop from an order-parameter field.

TEST INFRASTRUCTURE ONLY (part of the oracle): plain numpy, used by the tests
to measure the oracle's fields and to check the library's own deformation
diagnostic.  Shares nothing with the HIP library.

Sec. 4.4 defines the deformation factor D = (r_par - r_perp) / (r_par +
r_perp) from the drop's radii parallel and perpendicular to the applied
field.  Here the field is along y.  The radii are measured on the lines
through the drop's centroid: r_par is half the distance between the two
w = 1/2 crossings of the indicator w along the y line, r_perp the same along
the x line.  The centroid is the w-weighted mean position of the nodes with
w > 0; the lines generally fall between lattice rows and columns, so w on
them is interpolated linearly (bilinearly in 3-D) from the neighbouring
nodes, and each crossing is located by linear interpolation between the last
node value >= 1/2 and the first one below it, scanning outward from the node
nearest the centroid.

Axes are periodic except y, which is bounded when `walls` is set (a scan
that reaches a wall finds no crossing and returns nan).
"""
from __future__ import annotations

import math

import numpy as np


def centroid(w: np.ndarray):
    """w-weighted mean position (weights max(w, 0)) of a [ny, nx] or
    [nz, ny, nx] field, returned as (x, y) or (x, y, z)."""
    wp = np.maximum(np.asarray(w, np.float64), 0.0)
    tot = wp.sum()
    grids = np.indices(wp.shape, dtype=np.float64)
    # indices() gives (y, x) or (z, y, x)
    c = [float((g * wp).sum() / tot) for g in grids]
    return tuple(reversed(c))


def _line(w, axis, at):
    """Values of w along the lattice axis `axis` (0 x, 1 y, 2 z) through the
    point `at` (x, y[, z]), interpolated in the other axes (periodic
    wrap)."""
    dim = w.ndim
    arr = np.moveaxis(w, dim - 1 - axis, 0)  # scan axis first
    others = [a for a in range(dim) if a != axis]  # remaining lattice axes
    out = np.zeros(arr.shape[0])
    # the remaining array axes are the remaining lattice axes in descending order
    rest_axes = sorted(others, reverse=True)
    idx0, frac = [], []
    for a in rest_axes:
        n = w.shape[dim - 1 - a]
        f = math.floor(at[a])
        idx0.append((int(f) % n, (int(f) + 1) % n))
        frac.append(at[a] - f)
    for corner in range(1 << len(rest_axes)):
        wt = 1.0
        sel = []
        for k in range(len(rest_axes)):
            bit = (corner >> k) & 1
            wt *= frac[k] if bit else 1.0 - frac[k]
            sel.append(idx0[k][bit])
        out = out + wt * arr[(slice(None),) + tuple(sel)]
    return out


def _half_width(v, start, periodic):
    """Half the distance between the w = 1/2 crossings of the 1-D profile v
    on both sides of index `start` (nan if v[start] < 1/2 or a bounded scan
    runs out)."""
    n = len(v)
    if v[start] < 0.5:
        return math.nan
    ends = []
    for step in (1, -1):
        i, found = start, None
        for _ in range(n):
            j = i + step
            if not periodic and (j < 0 or j >= n):
                break
            a, b = v[i % n], v[j % n]
            if b < 0.5:
                found = i + step * (a - 0.5) / (a - b)
                break
            i = j
        if found is None:
            return math.nan
        ends.append(found)
    return 0.5 * (ends[0] - ends[1])


def contour_deformation(w: np.ndarray, walls: bool = False):
    """Sec. 4.4 deformation factor of the drop whose indicator is w (field
    along y).  Returns (D, r_par, r_perp)."""
    w = np.asarray(w, np.float64)
    c = centroid(w)
    r = []
    for axis in (1, 0):  # along the field (y), then across it (x)
        v = _line(w, axis, c)
        start = int(math.floor(c[axis] + 0.5)) % len(v)
        r.append(_half_width(v, start, periodic=not (walls and axis == 1)))
    rpar, rperp = r  # in 3-D the perpendicular line is the x line
    return (rpar - rperp) / (rpar + rperp), rpar, rperp


def moment_deformation(w: np.ndarray):
    """Second-moment form: (sqrt(I_par) - sqrt(I_perp)) / (sqrt(I_par) +
    sqrt(I_perp)) with I_par, I_perp the w-weighted variances along y and x
    (equal to the contour form for a sharp ellipse)."""
    w = np.asarray(w, np.float64)
    grids = np.indices(w.shape, dtype=np.float64)
    tot = w.sum()
    gy, gx = grids[-2], grids[-1]
    ybar, xbar = (gy * w).sum() / tot, (gx * w).sum() / tot
    ipar = ((gy - ybar) ** 2 * w).sum() / tot
    iper = ((gx - xbar) ** 2 * w).sum() / tot
    a, b = math.sqrt(ipar), math.sqrt(iper)
    return (a - b) / (a + b)
