"""Oracle: trilinear prolongation and its adjoint restriction (test infrastructure).

Sec. "Stochastic Multigrid Methods": the prolongation from level l-1 to level l is
trilinear interpolation and the restriction is its transpose (eq.
restr_prolong_variation), with no 1/8 scaling -- the variational (Galerkin) structure
is what keeps the target law invariant.

On cell centres, with the coarse cell J covering fine cells 2J and 2J+1, the fine centre
2J sits a quarter coarse spacing from coarse centre J and three quarters from J-1, so
fine 2J = 3/4 c_J + 1/4 c_{J-1} and fine 2J+1 = 3/4 c_J + 1/4 c_{J+1}.  Periodic axes
wrap; at a no-slip wall the missing coarse neighbour is the antisymmetric ghost -c_J,
so the fine cell next to the wall receives (3/4 - 1/4) c_J = 1/2 c_J.
"""
import numpy as np
import scipy.sparse as sp


def prolong_1d(nc, periodic):
    """1D prolongation matrix of shape (2*nc, nc)."""
    nf = 2 * nc
    rows, cols, vals = [], [], []
    for J in range(nc):
        for i, other in ((2 * J, J - 1), (2 * J + 1, J + 1)):
            rows.append(i); cols.append(J); vals.append(0.75)
            if periodic:
                rows.append(i); cols.append(other % nc); vals.append(0.25)
            elif 0 <= other < nc:
                rows.append(i); cols.append(other); vals.append(0.25)
            else:
                # ghost across the wall carries -c_J
                rows.append(i); cols.append(J); vals.append(-0.25)
    P = sp.coo_matrix((vals, (rows, cols)), shape=(nf, nc)).tocsr()
    P.sum_duplicates()
    return P


def prolong_3d(ncx, ncy, ncz):
    """P = Pz (x) Py (x) Px for lexicographic ordering with x fastest."""
    Px = prolong_1d(ncx, periodic=True)
    Py = prolong_1d(ncy, periodic=True)
    Pz = prolong_1d(ncz, periodic=False)
    return sp.kron(Pz, sp.kron(Py, Px, format="csr"), format="csr")
