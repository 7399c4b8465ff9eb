"""Oracle: single-cell evaluators of the uniform-grid steps (test infrastructure).

For grids too large to assemble (the 512 x 512 x 256 single-instance grid has 67 M unknowns)
the parity tests compare the GPU at sampled cells.  These functions compute, cell by cell and
from the definitions, what one step gives at a cell:

* ``row_A``: the row of A = -L (Sec. "Spatially Adaptive Discretizations", L = D G with the
  same-level face gradient; periodic x and y, no-slip walls on the z faces through the
  antisymmetric ghost), built face by face from the flux form.
* ``heat_bath_at``: one colour pass of the stochastic Gauss-Seidel (heat-bath) smoother at the
  given cells (Sec. "Stochastic Iterative Methods": each site is redrawn from its conditional
  law given the others, mean (b_i - sum_{j != i} A_ij x_j)/A_ii and variance kT/A_ii), with the
  noise of the counter-based stream (fine level: site = lexicographic index >> 1).
* ``restrict_residual_at``: b_c = P^T (b - A x) at given coarse cells (Alg. 3; unscaled
  transpose of trilinear prolongation, Sec. "Stochastic Multigrid Methods").
* ``prolong_at``: (P e) at given fine cells.

The 1D prolongation weights come from ``oracle.transfer.prolong_1d``; nothing is shared with
the GPU path.  Fields are natural-layout arrays [nz, ny, nx] (x fastest).
"""
import numpy as np

from .philox import normals
from .transfer import prolong_1d

KIND_SMOOTH = 0


def _unravel(i, nx, ny):
    return i % nx, (i // nx) % ny, i // (nx * ny)


def row_A(nx, ny, nz, i, h=1.0):
    """(columns, values) of row i of A, one face at a time: an interior or periodic face adds
    +1/h^2 to the diagonal and -1/h^2 to the neighbour; a wall face adds +2/h^2 to the
    diagonal (flux (-c - c)/h against the antisymmetric ghost)."""
    x, y, z = _unravel(int(i), nx, ny)
    ih2 = 1.0 / (h * h)
    cols = {int(i): 0.0}
    for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        zn = z + dz
        if not 0 <= zn < nz:
            cols[int(i)] += 2.0 * ih2
            continue
        j = (x + dx) % nx + nx * ((y + dy) % ny + ny * zn)
        cols[int(i)] += ih2
        cols[j] = cols.get(j, 0.0) - ih2
    keys = sorted(cols)
    vals = np.array([cols[k] for k in keys])
    return np.array(keys, dtype=np.int64), vals


def heat_bath_at(x, b, cells, colour, seed, cycle, slot, comp=0, kT=1.0, h=1.0, noise=True):
    """Values of `cells` (all of colour (x+y+z)%2 == colour) after one heat-bath pass of that
    colour on level 0; x, b: [nz, ny, nx] (b None = 0)."""
    nz, ny, nx = x.shape
    xf = x.ravel()
    bf = None if b is None else b.ravel()
    out = np.empty(len(cells))
    diag = np.empty(len(cells))
    for k, i in enumerate(cells):
        cx, cy, cz = _unravel(int(i), nx, ny)
        assert (cx + cy + cz) % 2 == colour
        cols, vals = row_A(nx, ny, nz, i, h)
        diag[k] = vals[cols == i][0]
        off = cols != i
        out[k] = ((0.0 if bf is None else bf[i]) - np.dot(vals[off], xf[cols[off]])) / diag[k]
    if noise:
        sites = np.asarray(cells, dtype=np.int64) >> 1
        n = normals(seed, cycle, 0, slot, colour, comp, KIND_SMOOTH, sites)
        out += np.sqrt(kT / diag) * n
    return out


def _weights_1d(nc, periodic, J):
    """(fine indices, weights) of column J of the 1D prolongation (nf = 2 nc)."""
    col = prolong_1d(nc, periodic).tocsc()[:, J]
    return col.indices, col.data


def restrict_residual_at(x, b, coarse_cells, h=1.0):
    """(P^T (b - A x)) at the given coarse cells (coarse grid nx/2 x ny/2 x nz/2)."""
    nz, ny, nx = x.shape
    ncx, ncy, ncz = nx // 2, ny // 2, nz // 2
    xf = x.ravel()
    bf = None if b is None else b.ravel()
    out = np.empty(len(coarse_cells))
    for k, I in enumerate(coarse_cells):
        X, Y, Z = _unravel(int(I), ncx, ncy)
        ix, wx = _weights_1d(ncx, True, X)
        iy, wy = _weights_1d(ncy, True, Y)
        iz, wz = _weights_1d(ncz, False, Z)
        acc = 0.0
        for a, fz in zip(wz, iz):
            for bb, fy in zip(wy, iy):
                for c, fx in zip(wx, ix):
                    i = fx + nx * (fy + ny * fz)
                    cols, vals = row_A(nx, ny, nz, i, h)
                    r = (0.0 if bf is None else bf[i]) - np.dot(vals, xf[cols])
                    acc += a * bb * c * r
        out[k] = acc
    return out


def prolong_at(e, fine_dims, fine_cells):
    """(P e) at the given fine cells; e: coarse field [nz/2, ny/2, nx/2]."""
    nx, ny, nz = fine_dims
    ncx, ncy, ncz = nx // 2, ny // 2, nz // 2
    ef = e.ravel()
    Px = prolong_1d(ncx, True).tocsr()
    Py = prolong_1d(ncy, True).tocsr()
    Pz = prolong_1d(ncz, False).tocsr()
    out = np.empty(len(fine_cells))
    for k, i in enumerate(fine_cells):
        fx, fy, fz = _unravel(int(i), nx, ny)
        acc = 0.0
        rz, ry, rx = Pz[fz], Py[fy], Px[fx]
        for a, Z in zip(rz.data, rz.indices):
            for bb, Y in zip(ry.data, ry.indices):
                for c, X in zip(rx.data, rx.indices):
                    acc += a * bb * c * ef[X + ncx * (Y + ncy * Z)]
        out[k] = acc
    return out


def sample_cells(nx, ny, nz, n, seed, colour=None):
    """n cells spread over the grid plus every corner-, edge- and wall-type cell class (the
    walls z = 0 and z = nz-1, the periodic seams x, y in {0, n-1}); with `colour`, only cells
    of that colour.  Test-side helper (no arithmetic of the method)."""
    rng = np.random.default_rng(seed)
    pts = set()
    for z in (0, 1, nz // 2, nz - 2, nz - 1):
        for y in (0, 1, ny // 2, ny - 1):
            for x in (0, 1, nx // 2, nx - 2, nx - 1):
                pts.add((x % nx, y % ny, z % nz))
    while len(pts) < n:
        pts.add((int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))))
    cells = []
    for x, y, z in sorted(pts):
        if colour is not None and (x + y + z) % 2 != colour:
            x = (x + 1) % nx
        cells.append(x + nx * (y + ny * z))
    return np.unique(np.array(cells, dtype=np.int64))
