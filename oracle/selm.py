"""Oracle: SELM hydrodynamic coupling on the wall-bounded grid (test infrastructure).

Plain dense/sparse FP64 statement of Sec. "Stochastic Eulerian-Lagrangian Method for
Fluid-Structure Interactions", Sec. "Discretization of SELM Hydrodynamic Coupling Tensor",
Sec. "Generation of the Stochastic Driving Fields Accounting for Thermal Fluctuations" and the
algorithm "Stochastic Dynamics of Elastic Structures with Hydrodynamic Coupling".

Fluid: three cell-centred velocity components on the nx x ny x nz grid of width h, periodic in
x and y, no-slip walls on the z faces; each component has the scalar operator A = -L_h of
``oracle.operator`` (antisymmetric wall ghost), and the viscous operator of the steady Stokes
equations is L = mu L_h on each component, i.e. L^-1 = -(1/mu) A^-1.

Readings taken where the paper leaves the construction open:

* Discrete projection.  The paper asks for a symmetric projection that commutes with L.
  Here D = sum_c delta_c applied to component c along axis c, with delta_x, delta_y the periodic
  forward differences ((u[i+1] - u[i])/h) and delta_z = a_z^{1/2}, the symmetric square root of
  the 1D wall operator a_z (the z part of A = a_x + a_y + a_z).  Then D D^T = A exactly, and
  P = I - D^T A^-1 D is symmetric, idempotent, annihilates gradients D^T p, satisfies D P = 0
  and commutes with L (each delta_c commutes with A).  Applying P takes one scalar solve with A
  (the deterministic multigrid solve).  On a collocated grid with walls no local z-difference
  gives both symmetry and commutation; the square root does.
* Coupling.  Gamma interpolates each velocity component at a structure point X with Peskin's
  4-point function phi (the immersed-boundary kernel of the Stochastic Immersed Boundary
  Method the paper names): weight phi((x_i - X)/h) phi((y_j - Y)/h) phi((z_k - Z)/h) at the cell
  centre ((i + 1/2) h, ...); cells beyond a wall are the antisymmetric ghosts of their mirror
  cells (u = 0 on the wall), so their weight enters the mirror cell with a minus sign.
  Lambda = alpha Gamma^T with alpha = 1/h^3 (spreading a force into a force density).
* H = -Gamma P L^-1 P Lambda = (alpha/mu) Gamma P A^-1 P Gamma^T (eq. H_selm_discr) and the
  driving field g = K xi, K = sqrt(2 kT alpha) Gamma P, xi ~ N(0, A^-1 / mu) (eqs.
  G_special_form and g_gen_xi with Lambda = alpha Gamma^T), so that <g g^T> = 2 kT H.
* Time stepping (the algorithm's step 4): Euler-Maruyama, X' = X + dt H(X) F(X) + sqrt(dt) g
  with one independent g per step.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operator import assemble_A


# ---------------------------------------------------------------- 1D pieces and the projection
def wall_operator_1d(nz, h=1.0):
    """a_z: the 1D cell-centred -d^2/dz^2 with antisymmetric ghosts at both walls (dense)."""
    a = np.zeros((nz, nz))
    for k in range(nz):
        a[k, k] = 2.0 + (k == 0) + (k == nz - 1)
        if k > 0:
            a[k, k - 1] = -1.0
        if k < nz - 1:
            a[k, k + 1] = -1.0
    return a / (h * h)


def sqrt_wall_operator(nz, h=1.0):
    """a_z^{1/2}: the symmetric positive square root, from a dense symmetric eigensolver."""
    lam, V = np.linalg.eigh(wall_operator_1d(nz, h))
    return (V * np.sqrt(lam)) @ V.T


def forward_difference(n, h=1.0):
    """Periodic (u[i+1] - u[i]) / h as an n x n sparse matrix."""
    I = sp.identity(n, format="csr")
    S = sp.csr_matrix((np.ones(n), (np.arange(n), (np.arange(n) + 1) % n)), shape=(n, n))
    return (S - I) / h


def divergence_matrix(nx, ny, nz, h=1.0):
    """D (N x 3N) acting on (u_x, u_y, u_z), each natural layout (x fastest)."""
    Ix, Iy, Iz = (sp.identity(n, format="csr") for n in (nx, ny, nz))
    dx = sp.kron(Iz, sp.kron(Iy, forward_difference(nx, h)))
    dy = sp.kron(Iz, sp.kron(forward_difference(ny, h), Ix))
    dz = sp.kron(sp.csr_matrix(sqrt_wall_operator(nz, h)), sp.kron(Iy, Ix))
    return sp.hstack([dx, dy, dz]).tocsr()


def apply_projection(u, nx, ny, nz, h=1.0, A=None, D=None):
    """P u = u - D^T A^-1 D u for u of length 3N (one sparse direct solve)."""
    A = assemble_A(nx, ny, nz, h) if A is None else A
    D = divergence_matrix(nx, ny, nz, h) if D is None else D
    p = spla.spsolve(A.tocsc(), D @ u)
    return u - D.T @ p


def projection_matrix(nx, ny, nz, h=1.0):
    """Dense P (tiny grids)."""
    A = assemble_A(nx, ny, nz, h).toarray()
    D = divergence_matrix(nx, ny, nz, h).toarray()
    return np.eye(D.shape[1]) - D.T @ np.linalg.solve(A, D)


# ---------------------------------------------------------------- the coupling Gamma
def peskin4(r):
    """Peskin's 4-point immersed-boundary function phi(r) (support |r| < 2)."""
    r = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(r)
    a = r < 1.0
    b = (r >= 1.0) & (r < 2.0)
    out[a] = (3.0 - 2.0 * r[a] + np.sqrt(1.0 + 4.0 * r[a] - 4.0 * r[a] ** 2)) / 8.0
    out[b] = (5.0 - 2.0 * r[b] - np.sqrt(-7.0 + 12.0 * r[b] - 4.0 * r[b] ** 2)) / 8.0
    return out


def interpolation_weights(X, nx, ny, nz, h=1.0):
    """Sparse W (M x N): (W u)[k] = sum_cells phi phi phi u, ghosts beyond the walls folded
    onto their mirror cells with a minus sign.  X: (M, 3) positions, 0 < Z < nz h."""
    X = np.asarray(X, dtype=np.float64).reshape(-1, 3)
    rows, cols, vals = [], [], []
    for k, (px, py, pz) in enumerate(X):
        assert 0.0 < pz < nz * h
        ix0 = int(np.floor(px / h - 0.5)) - 1
        iy0 = int(np.floor(py / h - 0.5)) - 1
        iz0 = int(np.floor(pz / h - 0.5)) - 1
        for dz in range(4):
            kz = iz0 + dz
            wz = float(peskin4((kz + 0.5) - pz / h))
            sign = 1.0
            if kz < 0:
                kz, sign = -1 - kz, -1.0
            elif kz >= nz:
                kz, sign = 2 * nz - 1 - kz, -1.0
            for dy in range(4):
                jy = iy0 + dy
                wy = float(peskin4((jy + 0.5) - py / h))
                for dx in range(4):
                    jx = ix0 + dx
                    wx = float(peskin4((jx + 0.5) - px / h))
                    rows.append(k)
                    cols.append((jx % nx) + nx * ((jy % ny) + ny * kz))
                    vals.append(sign * wx * wy * wz)
    W = sp.coo_matrix((vals, (rows, cols)), shape=(X.shape[0], nx * ny * nz)).tocsr()
    W.sum_duplicates()
    return W


def gamma_matrix(X, nx, ny, nz, h=1.0):
    """Gamma (3M x 3N): component c of point k from component c of the field; rows ordered
    (point, component) as X (M, 3) flattens, columns (component, cell)."""
    W = interpolation_weights(X, nx, ny, nz, h).tocoo()
    M = W.shape[0]
    N = nx * ny * nz
    rows, cols, vals = [], [], []
    for c in range(3):
        rows.append(3 * W.row + c)
        cols.append(c * N + W.col)
        vals.append(W.data)
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(3 * M, 3 * N)).tocsr()


# ---------------------------------------------------------------- H, g and the dynamics
class SELM:
    """The discrete SELM coupling of structure points to the wall-bounded Stokes fluid."""

    def __init__(self, nx, ny, nz, h=1.0, mu=1.0, kT=1.0):
        self.dims = (nx, ny, nz)
        self.h, self.mu, self.kT = float(h), float(mu), float(kT)
        self.alpha = 1.0 / h ** 3
        self.N = nx * ny * nz
        self.A = assemble_A(nx, ny, nz, h).tocsc()
        self.D = divergence_matrix(nx, ny, nz, h)
        self._lu = spla.splu(self.A)

    def project(self, u):
        p = self._lu.solve(self.D @ u)
        return u - self.D.T @ p

    def solve_velocity(self, f):
        """u = -L^-1 f = A^-1 f / mu for each component of f (length 3N)."""
        N = self.N
        return np.concatenate([self._lu.solve(f[c * N:(c + 1) * N]) for c in range(3)]) / self.mu

    def mobility(self, X, F):
        """V = H F = -Gamma P L^-1 P Lambda F (eq. H_selm_discr), F: (M, 3)."""
        G = gamma_matrix(X, *self.dims, self.h)
        f = self.alpha * (G.T @ np.asarray(F, dtype=np.float64).ravel())
        u = self.project(self.solve_velocity(self.project(f)))
        return (G @ u).reshape(-1, 3)

    def mobility_matrix(self, X):
        """Dense H (3M x 3M)."""
        M = np.asarray(X).reshape(-1, 3).shape[0]
        H = np.empty((3 * M, 3 * M))
        for j in range(3 * M):
            e = np.zeros(3 * M)
            e[j] = 1.0
            H[:, j] = self.mobility(X, e.reshape(-1, 3)).ravel()
        return H

    def drive(self, X, xi):
        """g = K xi with K = sqrt(2 kT alpha) Gamma P (eq. g_gen_xi), xi of length 3N with
        covariance A^-1 / mu."""
        G = gamma_matrix(X, *self.dims, self.h)
        return (np.sqrt(2.0 * self.kT * self.alpha) * (G @ self.project(xi))).reshape(-1, 3)

    def em_step(self, X, F, dt, g):
        """Euler-Maruyama step of dX/dt = H F + g: X + dt H F + sqrt(dt) g."""
        X = np.asarray(X, dtype=np.float64).reshape(-1, 3)
        return X + dt * self.mobility(X, F) + np.sqrt(dt) * np.asarray(g).reshape(-1, 3)


def xi_covariance(nx, ny, nz, h=1.0, mu=1.0):
    """Cov(xi) = -L^-1 = A^-1 / mu on each of the three components (dense, block diagonal)."""
    Ai = np.linalg.inv(assemble_A(nx, ny, nz, h).toarray()) / mu
    return sla.block_diag(Ai, Ai, Ai)
