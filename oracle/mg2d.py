"""Oracle: the two-dimensional wall-bounded sampler (test infrastructure).

The paper compares its multigrid sampler with stochastic Gauss-Seidel on two- and
three-dimensional meshes (Sec. "Performance of the Stochastic Samplers in Practice").  This is
the 2D form of the uniform-grid method: cells (x, z) of width h on nx x nz, periodic in x, no-slip
walls on the faces z = 0 and z = nz h (antisymmetric ghost), A = -L the 5-point operator built
face by face from the flux form (Sec. "Spatially Adaptive Discretizations", one level).

* Level plan: level 0 smooths when nx is even (red-black point heat bath, colour (x + z) % 2);
  a level l >= 1 smooths when nx_l % 4 == 0 and nz_l is even (2 x 2 block heat bath, block
  colour (bx % 2) + 2 (bz % 2), cells in a block ordered dx + 2 dz: the Galerkin stencils reach
  two cells, so blocks of one colour are uncoupled); coarsen (halve both extents) while a level
  smooths and the requested depth (or, automatically, more than coarsest_max unknowns) asks for
  it.
* Transfers: bilinear P = P_z (x) P_x from ``oracle.transfer.prolong_1d`` (3/4, 1/4 weights,
  the wall ghost -c), R = P^T, Galerkin A_{l+1} = P^T A_l P as sparse products.
* Smoothers, coarsest draw and V-cycle exactly as in ``oracle.mg`` (Alg. 3), with noise sites:
  level 0 site = (x + nx z) >> 1; block levels site = 4 block + in-block index; coarsest
  site = row.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .philox import PhiloxNoise, KIND_SMOOTH, KIND_COARSEST
from .transfer import prolong_1d


def assemble_A2(nx, nz, h=1.0):
    """A = -L on the 2D grid: each of the four faces of a cell adds 1/h^2 to its diagonal and
    -1/h^2 to the neighbour (periodic in x), or 2/h^2 to the diagonal on a wall face."""
    n = nx * nz
    z, x = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
    x = x.ravel()
    z = z.ravel()
    m = x + nx * z
    ih2 = 1.0 / (h * h)
    rows, cols, vals = [], [], []
    for dx, dz in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        xn, zn = (x + dx) % nx, z + dz
        inside = (zn >= 0) & (zn < nz)
        mi = m[inside]
        rows += [mi, mi]
        cols += [mi, xn[inside] + nx * zn[inside]]
        vals += [np.full(mi.size, ih2), np.full(mi.size, -ih2)]
        mw = m[~inside]
        rows.append(mw)
        cols.append(mw)
        vals.append(np.full(mw.size, 2.0 * ih2))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.eliminate_zeros()
    return A


def eigenvalues_2d(nx, nz, h=1.0):
    """Closed-form spectrum (4/h^2)[sin^2(pi j / nx) + sin^2(pi m / (2 nz))]."""
    j = np.arange(nx)
    m = np.arange(1, nz + 1)
    return np.sort((4.0 / h ** 2 * (np.sin(np.pi * j / nx)[None, :] ** 2
                                    + np.sin(np.pi * m / (2 * nz))[:, None] ** 2)).ravel())


def can_smooth(level, nx, nz):
    if level == 0:
        return nx % 2 == 0
    return nx % 4 == 0 and nz % 2 == 0


def plan_levels(nx, nz, levels=0, coarsest_max=512):
    dims = [(nx, nz)]
    while True:
        l = len(dims) - 1
        cx, cz = dims[-1]
        want = len(dims) < levels if levels > 0 else cx * cz > coarsest_max
        if want and can_smooth(l, cx, cz) and cx % 2 == 0 and cz % 2 == 0:
            dims.append((cx // 2, cz // 2))
        else:
            break
    if levels > 0 and len(dims) != levels:
        raise ValueError("grid %s cannot be coarsened to %d levels" % ((nx, nz), levels))
    return dims


class _Level:
    pass


class StochasticMG2D:
    def __init__(self, nx, nz, h=1.0, kT=1.0, levels=0, nu1=2, nu2=2, coarsest_max=512,
                 coarsest="cholesky"):
        self.h, self.kT = float(h), float(kT)
        self.nu1, self.nu2 = int(nu1), int(nu2)
        self.coarsest_mode = coarsest
        dims = plan_levels(nx, nz, levels, coarsest_max)
        A = assemble_A2(nx, nz, h)
        self.levels = []
        for l, (cx, cz) in enumerate(dims):
            L = _Level()
            L.index, L.dims, L.n, L.A = l, (cx, cz), cx * cz, A
            L.coarsest = l == len(dims) - 1
            if not L.coarsest:
                fx, fz = dims[l + 1]
                L.P = sp.kron(prolong_1d(fz, periodic=False), prolong_1d(fx, periodic=True),
                              format="csr")
                A = (L.P.T @ A @ L.P).tocsr()
                A.sum_duplicates()
            self.levels.append(L)
        for L in self.levels:
            if L.coarsest and coarsest == "cholesky":
                L.kind = "chol"
                L.chol = np.linalg.cholesky(L.A.toarray())
            elif not can_smooth(L.index, *L.dims):
                raise ValueError("level %d %s cannot be smoothed" % (L.index, L.dims))
            elif L.index == 0:
                self._setup_point(L)
            else:
                self._setup_block(L)

    def _setup_point(self, L):
        L.kind = "point"
        nx, nz = L.dims
        z, x = np.meshgrid(np.arange(nz), np.arange(nx), indexing="ij")
        colour = ((x + z) % 2).ravel()
        idx = np.arange(L.n)
        L.sets = [idx[colour == 0], idx[colour == 1]]
        L.diag = L.A.diagonal()
        L.sub = []
        for c in range(2):
            S, rest = L.sets[c], L.sets[1 - c]
            ASS = L.A[S][:, S]
            assert abs(ASS - sp.diags(ASS.diagonal())).max() == 0.0  # same colour uncoupled
            L.sub.append(L.A[S][:, rest].tocsr())

    def _setup_block(self, L):
        L.kind = "block"
        nx, nz = L.dims
        nbx = nx // 2
        bz, bx = np.meshgrid(np.arange(nz // 2), np.arange(nbx), indexing="ij")
        bx = bx.ravel()
        bz = bz.ravel()
        bid = bx + nbx * bz
        colour = (bx % 2) + 2 * (bz % 2)
        L.blocks = []
        for c in range(4):
            sel = colour == c
            cells = np.empty((sel.sum(), 4), dtype=np.int64)
            for k in range(4):
                cells[:, k] = (2 * bx[sel] + (k & 1)) + nx * (2 * bz[sel] + (k >> 1))
            flat = cells.ravel()
            mask = np.ones(L.n, dtype=bool)
            mask[flat] = False
            rest = np.nonzero(mask)[0]
            ASS = L.A[flat][:, flat].tocoo()
            assert np.all(ASS.row // 4 == ASS.col // 4)  # blocks of one colour uncoupled
            nb = cells.shape[0]
            ABB = np.zeros((nb, 4, 4))
            ABB[ASS.row // 4, ASS.row % 4, ASS.col % 4] = ASS.data
            L.blocks.append(dict(bid=bid[sel], cells=cells, rest=rest,
                                 sub=L.A[flat][:, rest].tocsr(), ABB=ABB,
                                 chol=np.linalg.cholesky(ABB)))

    def _point_pass(self, L, x, b, colour, noise, tag):
        S, rest = L.sets[colour], L.sets[1 - colour]
        d = L.diag[S]
        x[S] = (b[S] - L.sub[colour] @ x[rest]) / d
        if noise is not None:
            cycle, slot, comp = tag
            n = noise.draw(cycle, L.index, slot, colour, comp, KIND_SMOOTH, S >> 1)
            x[S] += np.sqrt(self.kT / d) * n

    def _block_pass(self, L, x, b, colour, noise, tag):
        blk = L.blocks[colour]
        cells = blk["cells"]
        nb = cells.shape[0]
        rhs = b[cells] - (blk["sub"] @ x[blk["rest"]]).reshape(nb, 4)
        new = np.linalg.solve(blk["ABB"], rhs[..., None])[..., 0]
        if noise is not None:
            cycle, slot, comp = tag
            sites = (4 * blk["bid"][:, None] + np.arange(4)[None, :]).ravel()
            n = noise.draw(cycle, L.index, slot, colour, comp, KIND_SMOOTH, sites).reshape(nb, 4)
            LT = np.transpose(blk["chol"], (0, 2, 1))
            new += np.sqrt(self.kT) * np.linalg.solve(LT, n[..., None])[..., 0]
        x[cells] = new

    def smooth(self, L, x, b, slot, post, noise, tag):
        ncol = 2 if L.kind == "point" else 4
        order = range(ncol - 1, -1, -1) if post else range(ncol)
        for colour in order:
            if L.kind == "point":
                self._point_pass(L, x, b, colour, noise, (tag[0], slot, tag[1]))
            else:
                self._block_pass(L, x, b, colour, noise, (tag[0], slot, tag[1]))

    def coarsest_step(self, L, b, noise, tag):
        v = sla.cho_solve((L.chol, True), b)
        if noise is not None:
            cycle, comp = tag
            n = noise.draw(cycle, L.index, 0, 0, comp, KIND_COARSEST, np.arange(L.n))
            v = v + np.sqrt(self.kT) * sla.solve_triangular(L.chol.T, n, lower=False)
        return v

    def vcycle(self, x, b, noise=None, cycle=0, comp=0, level=0):
        L = self.levels[level]
        x = np.array(x, dtype=np.float64, copy=True)
        b = np.asarray(b, dtype=np.float64)
        tag = (cycle, comp)
        if L.coarsest and self.coarsest_mode == "cholesky":
            return self.coarsest_step(L, b, noise, tag)
        for s in range(self.nu1):
            self.smooth(L, x, b, s, False, noise, tag)
        if not L.coarsest:
            bc = L.P.T @ (b - L.A @ x)
            x += L.P @ self.vcycle(np.zeros(bc.size), bc, noise, cycle, comp, level + 1)
        for s in range(self.nu2):
            self.smooth(L, x, b, self.nu1 + s, True, noise, tag)
        return x

    def sample_chain(self, n, seed, first_cycle=0, ncomp=1, stride=1):
        N = self.levels[0].n
        x = np.zeros((ncomp, N))
        noise = PhiloxNoise(seed)
        zero = np.zeros(N)
        out = np.empty((n, ncomp, N))
        cyc = first_cycle
        for i in range(n):
            for _ in range(stride):
                for c in range(ncomp):
                    x[c] = self.vcycle(x[c], zero, noise, cyc, c)
                cyc += 1
            out[i] = x
        return out, x


def mode_vector_2d(nx, nz, a, m):
    """Real eigenvector e_a(x) w_m(z) of A (e_a as in the 3D observables; w_m the normalised
    cell-centred sine)."""
    i = np.arange(nx)
    if a == 0:
        ex = np.full(nx, 1.0 / np.sqrt(nx))
    elif a == nx - 1:
        ex = (-1.0) ** i / np.sqrt(nx)
    else:
        j = (a + 1) // 2
        ex = np.sqrt(2.0 / nx) * (np.cos(2 * np.pi * j * i / nx) if a % 2 else
                                  np.sin(2 * np.pi * j * i / nx))
    w = np.sin(np.pi * m * (np.arange(nz) + 0.5) / nz)
    w /= np.linalg.norm(w)
    return np.kron(w, ex)
