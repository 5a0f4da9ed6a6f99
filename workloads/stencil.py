"""Stencil inputs: grids with a fixed Dirichlet ring, and weight boxes.

Grid convention (full extents include the ring): a 2D grid has shape
``(ny, nx)`` and a 3D grid ``(nz, ny, nx)``, x fastest.  The ring of width
``r`` (the stencil radius) is never updated; configurations set it to zero.

Weights are a dense ``(2r+1)^d`` box indexed ``[dz][dy][dx]`` (2D: ``[dy][dx]``)
with offsets ``-r..r``; an entry of zero marks an unused point.  Eq. 2 of the
paper names the 2D 5-point weights N (j+1), S (j-1), C, W (i-1), E (i+1) with
i along x and j along y, i.e. ``w[1+1][1]`` is N, ``w[1][1+1]`` is E.
"""
import numpy as np

STENCIL_KINDS = ("2d5pt", "2d9pt", "3d7pt")
# the rest of the 2D suite of tab:domain: stars of radius 2, 3, 4 and the
# radius-2 box
WIDE_KINDS = ("2ds9pt", "2d13pt", "2d17pt", "2d25pt")
_WIDE = {"2ds9pt": (2, False), "2d13pt": (3, False), "2d17pt": (4, False), "2d25pt": (2, True)}
# and of its 3D suite
WIDE3_KINDS = ("3d13pt", "3d17pt", "3d27pt", "poisson")
_WIDE3 = {"3d13pt": 2, "3d17pt": 1, "3d27pt": 1, "poisson": 1}


def stencil_radius(kind):
    """Radius of a named stencil."""
    if kind in _WIDE:
        return _WIDE[kind][0]
    if kind in _WIDE3:
        return _WIDE3[kind]
    if kind in STENCIL_KINDS:
        return 1
    raise ValueError(f"unknown stencil kind {kind!r}")


def stencil_weights(kind, dtype=np.float64):
    """Weight box of the benchmark stencils.

    2d5pt: centre and four neighbours 0.2 each (Eq. 2 with C=N=S=W=E=0.2).
    2d9pt: the radius-1 box, uniform 1/9 (tab:domain "2d9pt", order 1, 18 FLOPs).
    3d7pt: centre 0.4, six face neighbours 0.1 (tab:domain "3d7pt", 14 FLOPs).
    2ds9pt, 2d13pt, 2d17pt: the stars of radius 2, 3, 4 (centre and r cells
    along each axis direction; tab:domain orders 2, 3, 4 and 18, 26, 34
    FLOPs), 2d25pt: the 5x5 box (order 2, 50 FLOPs).  The paper names the
    patterns only; their weights here are uniform over the footprint (they
    sum to one, as the 2d9pt box's do).
    3d13pt: the radius-2 3D star (order 2, 26 FLOPs); 3d27pt: the 3x3x3 box
    (54 FLOPs); poisson: the 19 points of that box that are not corners (38
    FLOPs); 3d17pt (order 1, 34 FLOPs: 17 points of the 3x3x3 box, which no
    union of the box's symmetry classes gives): the 3x3 box of the centre
    plane and the four points (+-1, 0), (0, +-1) of each neighbouring plane.
    Uniform weights as above.
    """
    if kind in _WIDE3:
        d = np.indices((5, 5, 5) if kind == "3d13pt" else (3, 3, 3)) - (2 if kind == "3d13pt" else 1)
        az, ay, ax = np.abs(d)
        nz = (az > 0).astype(int) + (ay > 0) + (ax > 0)
        if kind == "3d13pt":
            m = nz <= 1
        elif kind == "3d27pt":
            m = np.ones_like(nz, dtype=bool)
        elif kind == "poisson":
            m = nz <= 2
        else:
            m = (az == 0) | ((nz == 2) & (az == 1))
        return np.where(m, 1.0 / m.sum(), 0.0).astype(dtype)
    if kind in _WIDE:
        r, box = _WIDE[kind]
        n = 2 * r + 1
        if box:
            w = np.full((n, n), 1.0 / (n * n))
        else:
            w = np.zeros((n, n))
            w[r, :] = 1.0 / (4 * r + 1)
            w[:, r] = 1.0 / (4 * r + 1)
        return w.astype(dtype)
    if kind == "2d5pt":
        w = np.zeros((3, 3))
        w[1, 1] = 0.2
        w[0, 1] = w[2, 1] = w[1, 0] = w[1, 2] = 0.2
    elif kind == "2d9pt":
        w = np.full((3, 3), 1.0 / 9.0)
    elif kind == "3d7pt":
        w = np.zeros((3, 3, 3))
        w[1, 1, 1] = 0.4
        w[0, 1, 1] = w[2, 1, 1] = 0.1
        w[1, 0, 1] = w[1, 2, 1] = 0.1
        w[1, 1, 0] = w[1, 1, 2] = 0.1
    else:
        raise ValueError(f"unknown stencil kind {kind!r}")
    return w.astype(dtype)


def interior_slices(ndim, r=1):
    return tuple(slice(r, -r) for _ in range(ndim))


def stencil_grid(shape, seed=0, dtype=np.float64, r=1, ring_value=0.0):
    """Grid of full extents ``shape`` whose interior is U[0,1) from ``seed``.

    The interior values are drawn in float64 in row-major order and then
    rounded to ``dtype``; the ring holds ``ring_value``.
    """
    shape = tuple(int(s) for s in shape)
    if any(s < 2 * r + 1 for s in shape):
        raise ValueError("every extent must exceed the ring on both sides")
    rng = np.random.default_rng(seed)
    g = np.full(shape, ring_value, dtype=np.float64)
    inner = tuple(s - 2 * r for s in shape)
    g[interior_slices(len(shape), r)] = rng.random(inner)
    return g.astype(dtype)
