"""Oracle: stochastic multigrid sampler and deterministic multigrid solve (test infrastructure).

Written from the paper's Sec. "Stochastic Iterative Methods" and "Stochastic Multigrid
Methods":

* Smoother: stochastic Gauss-Seidel with R = (D - L)^-1 U and noise factor
  Q = (D - L)^-1 D^{1/2} (eqs. R_GS and def_Q_GS).  For a single site this is the heat
  bath: x_i <- (b_i - sum_{j != i} A_ij x_j) / A_ii + sqrt(kT / A_ii) n_i.  A colour
  class of mutually uncoupled sites is updated at once; on Galerkin levels the sites are
  2x2x2 blocks drawn from their exact 8-variable conditional law
  x_B <- A_BB^-1 (b_B - A_{B,rest} x_rest) + sqrt(kT) L_BB^-T n_B  with A_BB = L_BB L_BB^T.
  Pre-sweeps visit the colours in increasing order, post-sweeps in decreasing order.
* V-cycle (Alg. 3): mu1 pre-sweeps; b^(l+1) = P^T (b^(l) - A^(l) v^(l)) (the residual of
  the current level); v^(l+1) = 0; recurse; v^(l) += P v^(l+1); mu2 post-sweeps.  At the
  coarsest level the default is an exact draw from the level's law,
  v = A_c^-1 b_c + sqrt(kT) L_c^-T n (dense Cholesky); the paper's literal reading
  (smoothing only) is available as coarsest="smooth".
* Target: density proportional to exp(-(1/2 x^T A x - x^T b)/kT), i.e. N(A^-1 b, kT A^-1).
  Sampling uses b = 0.  With the noise switched off the same cycle is the deterministic
  multigrid iteration whose fixed point is A^-1 b (stationary mean (I - R)^-1 s).
* Solve: u_0 = 0, u <- V-cycle(u, f) until ||f - A u||_2 <= rtol ||f||_2.

Noise enters only through ``noise.draw(cycle, level, slot, colour, comp, kind, sites)``
so that tests can inject arbitrary vectors (affine-map extraction).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .hierarchy import build_hierarchy, red_black_sets, block_sets, can_smooth
from .philox import PhiloxNoise, KIND_SMOOTH, KIND_COARSEST


class StochasticMG:
    def __init__(self, nx, ny, nz, h=1.0, kT=1.0, levels=0, nu1=2, nu2=2,
                 coarsest_max=512, coarsest="cholesky"):
        self.dims0 = (nx, ny, nz)
        self.h = float(h)
        self.kT = float(kT)
        self.nu1 = int(nu1)
        self.nu2 = int(nu2)
        self.coarsest_mode = coarsest
        self.levels = build_hierarchy(nx, ny, nz, h, levels, coarsest_max)
        for L in self.levels:
            if L.coarsest and coarsest == "cholesky":
                Ad = L.A.toarray()
                L.chol = np.linalg.cholesky(Ad)          # lower, Ad = L L^T
                continue
            if not can_smooth(L.index, L.dims):
                raise ValueError("level %d %s cannot be smoothed" % (L.index, L.dims))
            if L.index == 0:
                self._setup_point(L)
            else:
                self._setup_block(L)

    # ---------------------------------------------------------------- set-up
    def _setup_point(self, L):
        L.kind = "point"
        L.sets = red_black_sets(*L.dims)
        L.diag = L.A.diagonal()
        L.sub = []
        for c in range(2):
            S, rest = L.sets[c], L.sets[1 - c]
            ASS = L.A[S][:, S]
            off = ASS - sp.diags(ASS.diagonal())
            assert abs(off).sum() == 0.0, "red-black colour class is coupled"
            L.sub.append(L.A[S][:, rest].tocsr())

    def _setup_block(self, L):
        L.kind = "block"
        L.blocks = []
        n = L.n
        for c, (bid, cells) in enumerate(block_sets(*L.dims)):
            flat = cells.ravel()
            rest = np.setdiff1d(np.arange(n), flat)
            ASS = L.A[flat][:, flat].tocoo()
            nb = cells.shape[0]
            assert np.all(ASS.row // 8 == ASS.col // 8), "block colour class is coupled"
            ABB = np.zeros((nb, 8, 8))
            ABB[ASS.row // 8, ASS.row % 8, ASS.col % 8] = ASS.data
            chol = np.linalg.cholesky(ABB)
            L.blocks.append(dict(bid=bid, cells=cells, rest=rest,
                                 sub=L.A[flat][:, rest].tocsr(), ABB=ABB, chol=chol))

    # ---------------------------------------------------------------- smoothers
    def _point_pass(self, L, x, b, colour, noise, tag):
        S = L.sets[colour]
        rest = L.sets[1 - colour]
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
        rhs = b[cells] - (blk["sub"] @ x[blk["rest"]]).reshape(nb, 8)
        new = np.linalg.solve(blk["ABB"], rhs[..., None])[..., 0]
        if noise is not None:
            cycle, slot, comp = tag
            sites = (8 * blk["bid"][:, None] + np.arange(8)[None, :]).ravel()
            n = noise.draw(cycle, L.index, slot, colour, comp, KIND_SMOOTH, sites).reshape(nb, 8)
            LT = np.transpose(blk["chol"], (0, 2, 1))
            new += np.sqrt(self.kT) * np.linalg.solve(LT, n[..., None])[..., 0]
        x[cells] = new

    def smooth(self, L, x, b, slot, post, noise, tag):
        ncol = 2 if L.kind == "point" else 8
        order = range(ncol - 1, -1, -1) if post else range(ncol)
        for colour in order:
            if L.kind == "point":
                self._point_pass(L, x, b, colour, noise, (tag[0], slot, tag[1]))
            else:
                self._block_pass(L, x, b, colour, noise, (tag[0], slot, tag[1]))

    def coarsest_step(self, L, b, noise, tag):
        """Exact draw v = A_c^-1 b + sqrt(kT) L_c^-T n (noise None: v = A_c^-1 b)."""
        v = sla.cho_solve((L.chol, True), b)
        if noise is not None:
            cycle, comp = tag
            n = noise.draw(cycle, L.index, 0, 0, comp, KIND_COARSEST, np.arange(L.n))
            v = v + np.sqrt(self.kT) * sla.solve_triangular(L.chol.T, n, lower=False)
        return v

    # ---------------------------------------------------------------- cycle
    def vcycle(self, x, b, noise=None, cycle=0, comp=0, level=0):
        """One V-cycle (Alg. 3) at ``level``; returns the new iterate (x is not modified)."""
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
            vc = self.vcycle(np.zeros(bc.size), bc, noise, cycle, comp, level + 1)
            x += L.P @ vc
        for s in range(self.nu2):
            self.smooth(L, x, b, self.nu1 + s, True, noise, tag)
        return x

    # ---------------------------------------------------------------- drivers
    def sample_chain(self, n, seed, first_cycle=0, x0=None, ncomp=1, stride=1, burn_in=0,
                     noise=None):
        """Run burn_in + n*stride cycles with b = 0; return samples [n, ncomp, N] and the state."""
        N = self.levels[0].n
        x = np.zeros((ncomp, N)) if x0 is None else np.array(x0, dtype=np.float64).reshape(ncomp, N)
        noise = PhiloxNoise(seed) if noise is None else noise
        zero = np.zeros(N)
        out = np.empty((n, ncomp, N))
        cyc = first_cycle
        for _ in range(burn_in):
            for c in range(ncomp):
                x[c] = self.vcycle(x[c], zero, noise, cyc, c)
            cyc += 1
        for i in range(n):
            for _ in range(stride):
                for c in range(ncomp):
                    x[c] = self.vcycle(x[c], zero, noise, cyc, c)
                cyc += 1
            out[i] = x
        return out, x

    def solve(self, f, rtol=1e-12, max_cycles=100):
        """Deterministic MG solve A u = f from u = 0; returns (u, cycles, relres)."""
        f = np.asarray(f, dtype=np.float64)
        u = np.zeros_like(f)
        A = self.levels[0].A
        fn = np.linalg.norm(f)
        if fn == 0.0:
            return u, 0, 0.0
        relres = 1.0
        cycles = 0
        while cycles < max_cycles:
            u = self.vcycle(u, f, None)
            cycles += 1
            relres = np.linalg.norm(f - A @ u) / fn
            if relres <= rtol:
                break
        return u, cycles, relres
