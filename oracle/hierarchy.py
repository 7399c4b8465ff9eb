"""Oracle: level plan, Galerkin coarse operators and colour classes (test infrastructure).

Galerkin operators (Sec. "Stochastic Multigrid Methods", energy E(v) = 1/2 v^T A v - v^T b
and A^(l) = I^T A I):  A_{l+1} = P_l^T A_l P_l, computed here as explicit sparse triple
products of the 3D matrices.

Level plan (the paper is silent; reading documented with the package):
* level 0 can smooth (red-black point heat bath) when nx and ny are even;
* a level l >= 1 can smooth (2x2x2 block heat bath, 8 block colours) when its periodic
  extents are multiples of 4 and nz_l is even;
* level l is coarsened (every extent halved) when it can smooth, all extents are even,
  and either the requested level count is not yet reached or, in automatic mode, the
  level still has more than ``coarsest_max`` unknowns.  The last level is the coarsest.

Colour classes:
* level 0: red = (x+y+z) even, black = odd.  No two cells of one colour are coupled by
  the 7-point operator (checked).
* levels >= 1: blocks B = (bx,by,bz) of 2x2x2 cells, colour (bx%2) + 2(by%2) + 4(bz%2),
  cells inside a block in the order dx + 2dy + 4dz.  No two blocks of one colour are
  coupled by the Galerkin operator (checked), which makes each colour pass an exact
  draw from the conditional law of its blocks.
"""
import numpy as np
import scipy.sparse as sp

from .operator import assemble_A
from .transfer import prolong_3d


def can_smooth(level, dims):
    nx, ny, nz = dims
    if level == 0:
        return nx % 2 == 0 and ny % 2 == 0
    return nx % 4 == 0 and ny % 4 == 0 and nz % 2 == 0


def plan_levels(nx, ny, nz, levels=0, coarsest_max=512):
    dims = [(nx, ny, nz)]
    while True:
        l = len(dims) - 1
        d = dims[-1]
        halvable = all(v % 2 == 0 for v in d)
        if levels > 0:
            want = len(dims) < levels
        else:
            want = d[0] * d[1] * d[2] > coarsest_max
        if want and can_smooth(l, d) and halvable:
            dims.append((d[0] // 2, d[1] // 2, d[2] // 2))
        else:
            break
    if levels > 0 and len(dims) != levels:
        raise ValueError("grid %s cannot be coarsened to %d levels" % ((nx, ny, nz), levels))
    return dims


def red_black_sets(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    colour = ((x + y + z) % 2).ravel()
    idx = np.arange(nx * ny * nz)
    return [idx[colour == 0], idx[colour == 1]]


def block_sets(nx, ny, nz):
    """For each of the 8 block colours: (block ids [nb], cell indices [nb, 8])."""
    nbx, nby, nbz = nx // 2, ny // 2, nz // 2
    bz, by, bx = np.meshgrid(np.arange(nbz), np.arange(nby), np.arange(nbx), indexing="ij")
    bx = bx.ravel(); by = by.ravel(); bz = bz.ravel()
    bid = bx + nbx * (by + nby * bz)
    colour = (bx % 2) + 2 * (by % 2) + 4 * (bz % 2)
    out = []
    for c in range(8):
        sel = colour == c
        cells = np.empty((sel.sum(), 8), dtype=np.int64)
        for k in range(8):
            dx, dy, dz = k & 1, (k >> 1) & 1, (k >> 2) & 1
            cells[:, k] = (2 * bx[sel] + dx) + nx * ((2 * by[sel] + dy) + ny * (2 * bz[sel] + dz))
        out.append((bid[sel], cells))
    return out


class Level:
    pass


def build_hierarchy(nx, ny, nz, h=1.0, levels=0, coarsest_max=512):
    """List of Level objects, finest first, each with dims, A, and P (to the next finer)."""
    dims = plan_levels(nx, ny, nz, levels, coarsest_max)
    out = []
    A = assemble_A(nx, ny, nz, h)
    for l, d in enumerate(dims):
        L = Level()
        L.index = l
        L.dims = d
        L.n = d[0] * d[1] * d[2]
        L.A = A
        L.coarsest = (l == len(dims) - 1)
        out.append(L)
        if not L.coarsest:
            c = dims[l + 1]
            P = prolong_3d(c[0], c[1], c[2])
            L.P = P                      # maps level l+1 -> level l
            A = (P.T @ A @ P).tocsr()
            A.sum_duplicates()
    return out
