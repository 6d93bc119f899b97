"""Exact-rational rasterizer used to pin the oracle on tiny meshes.

A voxel centre p belongs to a tetrahedron when the point p + (e, e^2, e^3),
with e = 2^-60, has strictly positive barycentric coordinates.  The
coordinates are solved with Cramer's rule in ``fractions.Fraction``, so this
shares no formulation with the oracle's integer plane tests: it checks the
tie rule by its geometric meaning (a symbolic perturbation of the point),
not by the lexicographic normal test.

e = 2^-60 is small enough: snapped vertices have 10 fractional bits, so a
non-zero barycentric numerator is at least 2^-30 in absolute value while the
perturbation moves it by less than 2^-8 * 2^-30.
"""
from fractions import Fraction

import numpy as np

EPS = Fraction(1, 2 ** 60)


def snap(x):
    return Fraction(int(np.rint(np.float64(np.float32(x)) * 1024.0)), 1024)


def _det3(a, b, c):
    return (a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0])
            + a[2] * (b[0] * c[1] - b[1] * c[0]))


def barycentric(verts, p):
    """Exact barycentric coordinates of p in the tet (Cramer's rule)."""
    v0 = verts[0]
    cols = [[verts[i][k] - v0[k] for k in range(3)] for i in (1, 2, 3)]
    rhs = [p[k] - v0[k] for k in range(3)]
    D = _det3(*cols)
    if D == 0:
        return None
    l1 = _det3(rhs, cols[1], cols[2]) / D
    l2 = _det3(cols[0], rhs, cols[2]) / D
    l3 = _det3(cols[0], cols[1], rhs) / D
    return [1 - l1 - l2 - l3, l1, l2, l3]


def tet_voxels(verts_f, dims):
    """Sorted flat voxel indices whose perturbed centre is strictly inside."""
    verts = [[snap(c) for c in v] for v in np.asarray(verts_f, dtype=np.float64).reshape(4, 3)]
    nx, ny, nz = dims
    lo = [max(0, int(np.ceil(float(min(v[a] for v in verts))))) for a in range(3)]
    hi = [min(n - 1, int(np.floor(float(max(v[a] for v in verts))))) for a, n in
          zip(range(3), dims)]
    out = []
    for z in range(lo[2], hi[2] + 1):
        for y in range(lo[1], hi[1] + 1):
            for x in range(lo[0], hi[0] + 1):
                p = (x + EPS, y + EPS ** 2, z + EPS ** 3)
                lam = barycentric(verts, p)
                if lam is not None and all(l > 0 for l in lam):
                    out.append((z * ny + y) * nx + x)
    return sorted(out)
