"""Oracle: the discrete operator A = -L on a uniform cell-centred grid (test infrastructure).

Follows the paper's Sec. "Spatially Adaptive Discretizations" restricted to one level:
L = D G, where G takes the difference of neighbouring cell values across each face
divided by the spacing (same-level face gradient) and D sums the outward face fluxes
divided by the spacing (eq. def_discr_div).  The domain is periodic in x and y and has
no-slip walls (homogeneous Dirichlet, Sec. 2 steady Stokes with u = 0 on the boundary)
on the faces z = 0 and z = nz*h.  Reading taken here: the wall lies on cell faces and the
missing neighbour is an antisymmetric ghost (value -c), so the wall-face gradient is
(-c - c)/h.  The unknown ordering is lexicographic with x fastest:
index = x + nx*(y + ny*z).

A is symmetric positive definite; the target law of the sampler is N(A^-1 b, kT A^-1).
"""
import numpy as np
import scipy.sparse as sp


def cell_index(x, y, z, nx, ny):
    return x + nx * (y + ny * z)


def assemble_A(nx, ny, nz, h=1.0):
    """A = -L = -(D G) as a CSR matrix, built face by face from the flux form.

    For every cell m and each of its six faces the outward flux is
    (c_nbr - c_m)/h on an interior (or periodic) face and (-c_m - c_m)/h on a wall
    face; (L c)_m is the sum of the outward fluxes divided by h.
    """
    n = nx * ny * nz
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x = x.ravel(); y = y.ravel(); z = z.ravel()
    m = cell_index(x, y, z, nx, ny)
    rows, cols, vals = [], [], []
    inv_h2 = 1.0 / (h * h)
    for axis, sgn in ((0, 1), (0, -1), (1, 1), (1, -1), (2, 1), (2, -1)):
        xn, yn, zn = x.copy(), y.copy(), z.copy()
        if axis == 0:
            xn = (x + sgn) % nx
        elif axis == 1:
            yn = (y + sgn) % ny
        else:
            zn = z + sgn
        if axis < 2:
            interior = np.ones(n, dtype=bool)
        else:
            interior = (zn >= 0) & (zn < nz)
        # interior face:  -(L c)_m gets  +c_m/h^2 - c_nbr/h^2
        mi = m[interior]
        nb = cell_index(xn[interior], yn[interior], zn[interior], nx, ny)
        rows += [mi, mi]
        cols += [mi, nb]
        vals += [np.full(mi.size, inv_h2), np.full(mi.size, -inv_h2)]
        # wall face: flux (-c - c)/h, so -(L c)_m gets +2 c_m/h^2
        mw = m[~interior]
        rows.append(mw); cols.append(mw); vals.append(np.full(mw.size, 2.0 * inv_h2))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.eliminate_zeros()
    return A


def apply_A(x, nx, ny, nz, h=1.0):
    """A x for a field x[nz, ny, nx] (same operator, written as a stencil on arrays)."""
    x = np.asarray(x, dtype=np.float64).reshape(nz, ny, nx)
    out = 6.0 * x
    out -= np.roll(x, 1, axis=2) + np.roll(x, -1, axis=2)
    out -= np.roll(x, 1, axis=1) + np.roll(x, -1, axis=1)
    zp = np.zeros_like(x)
    zp[:-1] = x[1:]
    zp[-1] = -x[-1]          # ghost above the top wall
    zm = np.zeros_like(x)
    zm[1:] = x[:-1]
    zm[0] = -x[0]            # ghost below the bottom wall
    out -= zp + zm
    return (out / (h * h)).ravel()
