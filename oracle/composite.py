"""Oracle: spatially adaptive composite grid, its operator and the stochastic FAC cycle
(TEST INFRASTRUCTURE ONLY: used by tests/, smoke() and the CPU baseline, never by the
product path).

Mesh (Sec. "Spatially Adaptive Discretizations", nested structured meshes, neighbours at
most one level apart): a base grid of nx x ny x nz cells of width h, periodic in x and y
with no-slip walls at z = 0 and z = nz*h, and one box of base cells [x0,x1) x [y0,y1) x
[z0,z1) refined by two (cells of width h/2).  The partition is the base cells outside the
box ("coarse") plus the fine cells of the box.

Operator L = D G (eq. def_L) from the flux form:
* D (eq. def_discr_div): the sum over the faces of a partition cell of the outward normal
  face gradient, divided by the cell width; on a coarse face that borders fine cells the
  face value is the mean of the fine face values (eq. def_discr_grad_last), which makes
  the scheme conservative.
* G on a face between cells of one level (eq. def_discr_grad0): difference of the two cell
  values divided by the width.
* G on a coarse-fine face (eq. def_discr_grad): the paper gives the 2D cluster A, B, C; the
  3D reading taken here averages the FOUR fine cells B, C, D, E that touch the coarse face
  of cell A, over the distance 3/4 of the coarse width from A's centre to the plane of the
  fine centres.  Every one of the four fine cells uses that same face gradient.
* Walls (homogeneous Dirichlet on cell faces, both levels): antisymmetric ghost, face
  gradient (-c - c)/width.

With M = diag(cell volumes), S = M L is symmetric, so L^-1 (kT M^-1) = kT S^-1 is
symmetric (the property the paper states for this discretization).  The sampling
precision is A = -S / h^3: on coarse cells the rows of A are those of -L (the uniform-grid
operator of the rest of the package); fine rows are -L/8.  Target: N(A^-1 b, kT A^-1),
i.e. C = -2 L^-1 Ccal with Ccal = (kT/2) h^3 M^-1 (equipartition per unit volume).

Composite unknown ordering: coarse cells in base natural order (x fastest), covered base
cells skipped, then the fine cells in the box's natural order (fx fastest).

FAC cycle (Algs. 1-3 with the variational property of Sec. "Stochastic Multigrid
Methods"): the coarse space of the composite mesh is the whole base grid, mapped onto the
composite unknowns by P (identity on coarse cells, trilinear interpolation onto fine
cells, walls by the antisymmetric ghost).  Its operator is the Galerkin product
A_0 = P^T A P, and the base hierarchy below it uses trilinear transfers and Galerkin
products as well.  Reading of Alg. 1 (its residual sign is taken so that the correction
solves A q = b - A v): one cycle is
    b_0 = P^T (b - A x);  y = V-cycle_0(0, b_0);  x += P y;  nu composite sweeps,
with the base V-cycle (Alg. 3, mu1/mu2 sweeps, exact coarsest draw) run by the uniform
oracle's machinery on the Galerkin operators.  Every base level is smoothed by the 2x2x2
block heat bath (its operators are not 7-point near the box).

Composite sweep: a point heat bath (stochastic Gauss-Seidel site update) over twelve
classes of mutually uncoupled cells, in this order:
  0, 1   coarse cells with (x+y+z) % 2 == 0, 1
  2, 3   fine cells off the interface layer with (fx+fy+fz) % 2 == 0, 1
  4..11  fine cells of the interface layer (a face on the box boundary towards coarse
         cells) with parity class (fx%2) + 2 (fy%2) + 4 (fz%2) == class - 4
(the four fine cells of a coarse-fine face are coupled to each other, so the layer needs
the eight parity classes).

Noise streams (shared counter convention of the package, see oracle.philox): composite
passes draw from (level 0, slot = sweep, colour = class, kind KIND_COMPOSITE); the site of a
cell is its natural index in its own array (base grid for coarse cells, box for fine cells),
halved (index >> 1) in the four parity classes 0..3: a parity class holds one cell of every
pair (2q, 2q + 1) of its array (nx and the fine extents are even), so the halved indices are
distinct and consecutive cells of the class share a Philox call; the base hierarchy draws with kind KIND_FAC_BASE (block levels) and
KIND_FAC_COARSEST (coarsest), level = base level index, sites as in oracle.mg.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .mg import StochasticMG
from .hierarchy import Level
from .philox import KIND_SMOOTH, KIND_COARSEST
from .transfer import prolong_3d

KIND_COMPOSITE = 2
KIND_FAC_BASE = 3
KIND_FAC_COARSEST = 4
N_CLASSES = 12


class CompositeGrid:
    """Base grid plus one refined box (None = no refinement)."""

    def __init__(self, nx, ny, nz, box=None, h=1.0):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.h = float(h)
        nb = self.nx * self.ny * self.nz
        self.nbase = nb
        covered = np.zeros((self.nz, self.ny, self.nx), dtype=bool)
        if box is None:
            self.box = None
            self.fx = self.fy = self.fz = 0
        else:
            x0, x1, y0, y1, z0, z1 = (int(v) for v in box)
            if not (0 <= x0 < x1 <= self.nx and 0 <= y0 < y1 <= self.ny and
                    0 <= z0 < z1 <= self.nz):
                raise ValueError("box outside the grid")
            self.box = (x0, x1, y0, y1, z0, z1)
            self.fx, self.fy, self.fz = 2 * (x1 - x0), 2 * (y1 - y0), 2 * (z1 - z0)
            covered[z0:z1, y0:y1, x0:x1] = True
        self.covered = covered.ravel()
        self.coarse_id = np.full(nb, -1, dtype=np.int64)
        self.coarse_cells = np.flatnonzero(~self.covered)
        self.coarse_id[self.coarse_cells] = np.arange(self.coarse_cells.size)
        self.nc = self.coarse_cells.size
        self.nf = self.fx * self.fy * self.fz
        self.n = self.nc + self.nf
        self.A = self._assemble()

    # ------------------------------------------------------------- indexing
    def base_index(self, x, y, z):
        return x + self.nx * (y + self.ny * z)

    def fine_index(self, i, j, k):
        """Composite index of fine cell (i, j, k) in box coordinates."""
        return self.nc + i + self.fx * (j + self.fy * k)

    def fine_parent(self, i, j, k):
        x0, _, y0, _, z0, _ = self.box
        return x0 + i // 2, y0 + j // 2, z0 + k // 2

    def split(self, v):
        """Composite vector -> (coarse field [nz,ny,nx] with zeros on covered cells, fine
        field [fz,fy,fx])."""
        v = np.asarray(v, dtype=np.float64)
        c = np.zeros(self.nbase)
        c[self.coarse_cells] = v[:self.nc]
        return (c.reshape(self.nz, self.ny, self.nx),
                v[self.nc:].reshape(self.fz, self.fy, self.fx))

    def join(self, c, f):
        c = np.asarray(c, dtype=np.float64).ravel()
        f = np.asarray(f, dtype=np.float64).ravel()
        return np.concatenate([c[self.coarse_cells], f])

    # ------------------------------------------------------------- operator
    def _faces(self):
        """All faces of the partition as (kind, data) records:
        ('same', m, l, area, dist)   two cells of one level
        ('wall', m, area, dist)      a cell face on a wall (ghost -c at distance dist)
        ('cf', a, [g0..g3], area)    coarse cell a, the four fine cells of its face
        """
        h, hf = self.h, 0.5 * self.h
        out = []
        nx, ny, nz = self.nx, self.ny, self.nz
        cov = self.covered.reshape(nz, ny, nx)
        # coarse cells: faces towards +x, +y, +z (each interior face once), walls
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    if cov[z, y, x]:
                        continue
                    m = self.coarse_id[self.base_index(x, y, z)]
                    for axis in range(3):
                        for sgn in (1, -1):
                            q = [x, y, z]
                            q[axis] += sgn
                            if axis == 2 and not 0 <= q[2] < nz:
                                out.append(("wall", m, h * h, h))
                                continue
                            q[0] %= nx
                            q[1] %= ny
                            if not cov[q[2], q[1], q[0]]:
                                if sgn == 1:
                                    l = self.coarse_id[self.base_index(*q)]
                                    out.append(("same", m, l, h * h, h))
                                continue
                            # coarse-fine face: the four children of the covered cell q
                            # that touch the shared face
                            out.append(("cf", m, self._face_children(q, axis, -sgn), h * h))
        if self.box is None:
            return out
        fx, fy, fz = self.fx, self.fy, self.fz
        full_x = self.box[1] - self.box[0] == nx
        full_y = self.box[3] - self.box[2] == ny
        for k in range(fz):
            for j in range(fy):
                for i in range(fx):
                    m = self.fine_index(i, j, k)
                    for axis, n_ax, full in ((0, fx, full_x), (1, fy, full_y)):
                        q = [i, j, k]
                        q[axis] += 1
                        if q[axis] < n_ax:
                            out.append(("same", m, self.fine_index(*q), hf * hf, hf))
                        elif full:
                            q[axis] = 0
                            out.append(("same", m, self.fine_index(*q), hf * hf, hf))
                    if k + 1 < fz:
                        out.append(("same", m, self.fine_index(i, j, k + 1), hf * hf, hf))
                    z_abs = 2 * self.box[4] + k
                    if z_abs == 0 or z_abs == 2 * nz - 1:
                        out.append(("wall", m, hf * hf, hf))
        return out

    def _face_children(self, q, axis, side):
        """Composite ids of the four fine children of covered base cell q lying on the face
        of q in direction `side` (+1/-1) along `axis`."""
        x0, _, y0, _, z0, _ = self.box
        base = [2 * (q[0] - x0), 2 * (q[1] - y0), 2 * (q[2] - z0)]
        kids = []
        for a in (0, 1):
            for b in (0, 1):
                c = list(base)
                c[axis] += 1 if side > 0 else 0
                t = [ax for ax in range(3) if ax != axis]
                c[t[0]] += a
                c[t[1]] += b
                kids.append(self.fine_index(*c))
        return kids

    def _assemble(self):
        """S = M L face by face; returns A = -S / h^3 (CSR).  Also keeps S and the volumes."""
        rows, cols, vals = [], [], []

        def add(r, c, v):
            rows.append(r); cols.append(c); vals.append(v)

        for f in self._faces():
            if f[0] == "same":
                _, m, l, area, dist = f
                w = area / dist                      # flux area * (c_l - c_m) / dist
                add(m, m, -w); add(m, l, w); add(l, l, -w); add(l, m, w)
            elif f[0] == "wall":
                _, m, area, dist = f
                add(m, m, -2.0 * area / dist)       # area * (-c - c) / dist
            else:
                _, a, kids, area = f
                dist = 0.75 * self.h
                # coarse face gradient G = (mean(kids) - c_a) / dist; A receives area * G,
                # each child (a quarter of the area) loses area/4 * G
                w = area / dist
                add(a, a, -w)
                for g in kids:
                    add(a, g, 0.25 * w)
                    add(g, a, 0.25 * w)
                    for g2 in kids:
                        add(g, g2, -0.0625 * w)
        S = sp.coo_matrix((vals, (rows, cols)), shape=(self.n, self.n)).tocsr()
        S.sum_duplicates()
        self.S = S
        vol = np.full(self.n, self.h ** 3)
        vol[self.nc:] = (0.5 * self.h) ** 3
        self.vol = vol
        A = (-S / self.h ** 3).tocsr()
        A.eliminate_zeros()
        return A

    def laplacian(self):
        """L = M^-1 S (non-symmetric on a composite mesh)."""
        return (sp.diags(1.0 / self.vol) @ self.S).tocsr()

    def face_energy(self, c):
        """-c^T S c written as the sum over faces of area * (face gradient)^2 * distance,
        evaluated from the geometry (walls: the ghost carries half of its face)."""
        c = np.asarray(c, dtype=np.float64)
        e = 0.0
        for f in self._faces():
            if f[0] == "same":
                _, m, l, area, dist = f
                e += area / dist * (c[l] - c[m]) ** 2
            elif f[0] == "wall":
                _, m, area, dist = f
                e += 0.5 * area / dist * (2.0 * c[m]) ** 2
            else:
                _, a, kids, area = f
                g = (np.mean(c[kids]) - c[a]) / (0.75 * self.h)
                e += area * g * g * (0.75 * self.h)
        return e

    # ------------------------------------------------------------- transfers
    def prolong_base(self):
        """P: base grid (natural order, nbase) -> composite unknowns (n)."""
        rows, cols, vals = [], [], []
        for r, b in enumerate(self.coarse_cells):
            rows.append(r); cols.append(b); vals.append(1.0)
        if self.box is not None:
            x0, _, y0, _, z0, _ = self.box

            def w1d(p, n, periodic):
                J = p >> 1
                other = J - 1 if p % 2 == 0 else J + 1
                out = [(J, 0.75)]
                if periodic:
                    out.append((other % n, 0.25))
                elif 0 <= other < n:
                    out.append((other, 0.25))
                else:
                    out.append((J, -0.25))
                return out

            for k in range(self.fz):
                wz = w1d(2 * z0 + k, self.nz, False)
                for j in range(self.fy):
                    wy = w1d(2 * y0 + j, self.ny, True)
                    for i in range(self.fx):
                        wx = w1d(2 * x0 + i, self.nx, True)
                        r = self.fine_index(i, j, k)
                        for (Z, a) in wz:
                            for (Y, b) in wy:
                                for (X, c) in wx:
                                    rows.append(r); cols.append(self.base_index(X, Y, Z))
                                    vals.append(a * b * c)
        P = sp.coo_matrix((vals, (rows, cols)), shape=(self.n, self.nbase)).tocsr()
        P.sum_duplicates()
        return P

    # ------------------------------------------------------------- sweep classes
    def classes(self):
        """The twelve point classes of a composite sweep: list of (composite ids, noise sites)."""
        out = []
        cx = self.coarse_cells % self.nx
        cy = (self.coarse_cells // self.nx) % self.ny
        cz = self.coarse_cells // (self.nx * self.ny)
        par = (cx + cy + cz) % 2
        ids = np.arange(self.nc)
        for c in range(2):
            sel = par == c
            out.append((ids[sel], self.coarse_cells[sel] >> 1))
        if self.box is None:
            for _ in range(10):
                out.append((np.zeros(0, np.int64), np.zeros(0, np.int64)))
            return out
        k, j, i = np.meshgrid(np.arange(self.fz), np.arange(self.fy), np.arange(self.fx),
                              indexing="ij")
        i = i.ravel(); j = j.ravel(); k = k.ravel()
        loc = i + self.fx * (j + self.fy * k)
        layer = self.layer_mask(i, j, k)
        for c in range(2):
            sel = (~layer) & ((i + j + k) % 2 == c)
            out.append((self.nc + loc[sel], loc[sel] >> 1))
        pc = (i % 2) + 2 * (j % 2) + 4 * (k % 2)
        for p in range(8):
            sel = layer & (pc == p)
            out.append((self.nc + loc[sel], loc[sel]))
        return out

    def layer_mask(self, i, j, k):
        """Fine cells with a face on the box boundary towards coarse cells."""
        x0, x1, y0, y1, z0, z1 = self.box
        m = np.zeros(np.shape(i), dtype=bool)
        if x1 - x0 < self.nx:
            m |= (i == 0) | (i == self.fx - 1)
        if y1 - y0 < self.ny:
            m |= (j == 0) | (j == self.fy - 1)
        if z0 > 0:
            m |= k == 0
        if z1 < self.nz:
            m |= k == self.fz - 1
        return m


def base_plan(nx, ny, nz, levels=0, coarsest_max=512):
    """Base levels of the FAC coarse space: coarsen (halve every extent) while the level can
    be block-smoothed (nx, ny multiples of 4, nz even) and, in automatic mode, has more than
    coarsest_max cells; the last level is drawn exactly."""
    dims = [(nx, ny, nz)]
    while True:
        d = dims[-1]
        smoothable = d[0] % 4 == 0 and d[1] % 4 == 0 and d[2] % 2 == 0
        want = len(dims) < levels if levels > 0 else d[0] * d[1] * d[2] > coarsest_max
        if want and smoothable:
            dims.append((d[0] // 2, d[1] // 2, d[2] // 2))
        else:
            break
    if levels > 0 and len(dims) != levels:
        raise ValueError("base grid cannot be coarsened to %d levels" % levels)
    return dims


class _KindMap:
    """Passes the base hierarchy's draws to the noise source under the FAC kinds."""

    def __init__(self, inner):
        self.inner = inner

    def draw(self, cycle, level, slot, colour, comp, kind, sites):
        k = KIND_FAC_BASE if kind == KIND_SMOOTH else KIND_FAC_COARSEST
        return self.inner.draw(cycle, level, slot, colour, comp, k, sites)


class FACSampler:
    """Stochastic FAC cycle and deterministic FAC solve on a CompositeGrid."""

    def __init__(self, grid, kT=1.0, nu=2, mu1=2, mu2=2, levels=0, coarsest_max=512,
                 gs_only=False):
        """gs_only: the cycle is the nu composite sweeps alone (stochastic Gauss-Seidel on the
        composite mesh, Sec. "Stochastic Iterative Methods"), for the comparison of the two
        samplers."""
        self.g = grid
        self.gs_only = bool(gs_only)
        self.kT = float(kT)
        self.nu = int(nu)
        self.A = grid.A
        self.P = grid.prolong_base()
        A0 = (self.P.T @ self.A @ self.P).tocsr()
        A0.sum_duplicates()
        dims = base_plan(grid.nx, grid.ny, grid.nz, levels, coarsest_max)
        self.base = self._base_mg(A0, dims, mu1, mu2)
        self.cls = grid.classes()
        self.diag = self.A.diagonal()
        self.sub = []
        for ids, _ in self.cls:
            rest = np.setdiff1d(np.arange(grid.n), ids)
            ASS = self.A[ids][:, ids]
            off = ASS - sp.diags(ASS.diagonal())
            assert abs(off).sum() == 0.0, "composite sweep class is coupled"
            self.sub.append((rest, self.A[ids][:, rest].tocsr()))

    def _base_mg(self, A0, dims, mu1, mu2):
        mg = StochasticMG.__new__(StochasticMG)
        mg.dims0 = dims[0]
        mg.h = self.g.h
        mg.kT = self.kT
        mg.nu1, mg.nu2 = int(mu1), int(mu2)
        mg.coarsest_mode = "cholesky"
        mg.levels = []
        A = A0
        for l, d in enumerate(dims):
            L = Level()
            L.index = l
            L.dims = d
            L.n = d[0] * d[1] * d[2]
            L.A = A
            L.coarsest = l == len(dims) - 1
            mg.levels.append(L)
            if not L.coarsest:
                c = dims[l + 1]
                L.P = prolong_3d(*c)
                A = (L.P.T @ A @ L.P).tocsr()
                A.sum_duplicates()
        for L in mg.levels:
            if L.coarsest:
                L.chol = np.linalg.cholesky(L.A.toarray())
            else:
                mg._setup_block(L)
        return mg

    def class_pass(self, x, b, c, slot, noise, cycle, comp=0):
        """Heat bath of class c in place: x_i = (b_i - sum_j A_ij x_j)/A_ii + sqrt(kT/A_ii) n_i."""
        ids, sites = self.cls[c]
        if ids.size == 0:
            return
        rest, sub = self.sub[c]
        d = self.diag[ids]
        x[ids] = (b[ids] - sub @ x[rest]) / d
        if noise is not None:
            n = noise.draw(cycle, 0, slot, c, comp, KIND_COMPOSITE, sites)
            x[ids] += np.sqrt(self.kT / d) * n

    def sweep(self, x, b, slot, noise, cycle, comp):
        for c in range(len(self.cls)):
            self.class_pass(x, b, c, slot, noise, cycle, comp)

    def cycle(self, x, b, noise=None, cycle=0, comp=0):
        """One FAC cycle (returns the new iterate; x is not modified)."""
        x = np.array(x, dtype=np.float64, copy=True)
        b = np.asarray(b, dtype=np.float64)
        if not self.gs_only:
            b0 = self.P.T @ (b - self.A @ x)
            nz = None if noise is None else _KindMap(noise)
            y = self.base.vcycle(np.zeros(b0.size), b0, nz, cycle, comp, 0)
            x += self.P @ y
        for s in range(self.nu):
            self.sweep(x, b, s, noise, cycle, comp)
        return x

    def solve(self, f, rtol=1e-10, max_cycles=100):
        f = np.asarray(f, dtype=np.float64)
        u = np.zeros_like(f)
        fn = np.linalg.norm(f)
        if fn == 0.0:
            return u, 0, 0.0
        relres, k = 1.0, 0
        while k < max_cycles:
            u = self.cycle(u, f)
            k += 1
            relres = np.linalg.norm(f - self.A @ u) / fn
            if relres <= rtol:
                break
        return u, k, relres

    def affine_map(self):
        """(T, G) with one cycle (b = 0) equal to x -> T x + G n, n every normal it draws."""
        from .analysis import _RecordingNoise, _InjectedNoise
        N = self.g.n
        zero = np.zeros(N)
        rec = _RecordingNoise()
        self.cycle(zero, zero, rec)
        T = np.empty((N, N))
        for i in range(N):
            e = np.zeros(N)
            e[i] = 1.0
            T[:, i] = self.cycle(e, zero)
        G = np.empty((N, rec.count))
        for k in range(rec.count):
            v = np.zeros(rec.count)
            v[k] = 1.0
            G[:, k] = self.cycle(zero, zero, _InjectedNoise(v))
        return T, G


def row_of(nx, ny, nz, box, h, kind, idx):
    """Row of A for one composite cell, from the face rules alone (no assembly), for sampled
    checks on grids too large to assemble here.  kind 'c': base cell index idx (uncovered);
    kind 'f': fine cell index idx in the box.  Returns {('c', base index) or ('f', fine
    index): coefficient}."""
    x0, x1, y0, y1, z0, z1 = box
    fx, fy, fz = 2 * (x1 - x0), 2 * (y1 - y0), 2 * (z1 - z0)
    ih2 = 1.0 / (h * h)
    out = {}

    def add(key, v):
        out[key] = out.get(key, 0.0) + v * ih2

    def cov(x, y, z):
        return x0 <= x < x1 and y0 <= y < y1 and z0 <= z < z1

    def fkey(i, j, k):
        return ("f", i + fx * (j + fy * k))

    if kind == "c":
        x, y, z = idx % nx, (idx // nx) % ny, idx // (nx * ny)
        me = ("c", idx)
        for axis in range(3):
            for sgn in (1, -1):
                q = [x, y, z]
                q[axis] += sgn
                if axis == 2 and not 0 <= q[2] < nz:
                    add(me, 2.0)                     # wall face: ghost -c at distance h
                    continue
                q[0] %= nx
                q[1] %= ny
                if cov(*q):
                    # coarse-fine face: gradient (mean of 4 fine - c) / (3h/4) on area h^2
                    base = [2 * (q[0] - x0), 2 * (q[1] - y0), 2 * (q[2] - z0)]
                    base[axis] += 1 if sgn < 0 else 0
                    t = [a for a in range(3) if a != axis]
                    add(me, 4.0 / 3.0)
                    for a in (0, 1):
                        for b in (0, 1):
                            c = list(base)
                            c[t[0]] += a
                            c[t[1]] += b
                            add(fkey(*c), -1.0 / 3.0)
                else:
                    add(me, 1.0)
                    add(("c", q[0] + nx * (q[1] + ny * q[2])), -1.0)
        return out
    i, j, k = idx % fx, (idx // fx) % fy, idx // (fx * fy)
    me = ("f", idx)
    ext = (fx, fy, fz)
    for axis in range(3):
        for sgn in (1, -1):
            p = [i, j, k]
            p[axis] += sgn
            if 0 <= p[axis] < ext[axis]:
                add(me, 0.5)                         # fine face: area h^2/4, distance h/2
                add(fkey(*p), -0.5)
                continue
            A = [x0 + i // 2, y0 + j // 2, z0 + k // 2]
            A[axis] += sgn
            if axis == 2 and not 0 <= A[2] < nz:
                add(me, 1.0)                         # fine wall face
                continue
            A[0] %= nx
            A[1] %= ny
            # this cell's share (a quarter of the coarse face) of the coarse-fine gradient
            add(("c", A[0] + nx * (A[1] + ny * A[2])), -1.0 / 3.0)
            t = [a for a in range(3) if a != axis]
            for a in (0, 1):
                for b in (0, 1):
                    c = [i, j, k]
                    c[t[0]] = (c[t[0]] // 2) * 2 + a
                    c[t[1]] = (c[t[1]] // 2) * 2 + b
                    add(fkey(*c), 1.0 / 12.0)
    return out
