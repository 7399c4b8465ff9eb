"""Oracle: effective structure dynamics for a non-symmetric discrete Laplacian (test
infrastructure; only tests, the smoke check and the benchmark's CPU leg use it).

Appendix A removes the fluid from the coupled system by a formal two-time-scale argument.  The
fluid obeys the linear SDE  du = eps^-1 L u dt + f dt + Q dB  with L a (possibly non-symmetric)
discrete Laplacian whose eigenvalues have negative real parts and C the stationary covariance,
tied to the forcing by the Lyapunov relation L C + C L^T = -eps Q Q^T.  The structure moves as
dX = Gamma u dt.  For eps << dt the increments of X have, per unit time,

  mean        a = -eps Gamma L^-1 f,
  covariance  b = -eps alpha Gamma (L^-1 C + C L^-T) Gamma^T,

and with eps -> 1/mu the effective structure dynamics dX = H F dt + R dB use

  H = -(alpha/mu) Gamma L^-1 Gamma^T,    R R^T = -(alpha/mu) Gamma (L^-1 C + C L^-T) Gamma^T.

alpha and mu are scalars here, as in the appendix.  For symmetric L^-1 C the covariance is
-2 (alpha/mu) Gamma L^-1 C Gamma^T.  On the uniform grid L = -A and C = kT I, so R R^T = 2 kT H.
The projection is the identity in these formulas; the wall-bounded projection belongs to the
uniform-grid coupling in ``oracle.selm``.

Readings (the appendix is formal and the text is garbled in places):
* Sign of b.  The appendix's intermediate steps treat the A_2 term as O(eps^2).  But Q Q^T is
  O(1/eps), so A_2 = -eps dt (L^-1 C + C L^-T) to leading order, and I_1 totals
  -eps dt C L^-T.  The full covariance rate is therefore -eps (L^-1 C + C L^-T), which is
  positive semi-definite.  This is the sign of the appendix's final R R^T, and it is the one
  used here.  The tests settle it by quadrature of the exact increment covariance.
* The closed form of J_1.  The appendix writes the integral of e^{rL} C e^{rL^T} over [0, T] as
  (1/2) L^-1 [e^{TL} C e^{TL^T} - C].  That holds only when L commutes with the bracket.  In
  general the integral is the solution Y of L Y + Y L^T = e^{TL} C e^{TL^T} - C.  The leading
  order is unchanged.
* Sampling.  -(L^-1 C + C L^-T) = eps L^-1 Q Q^T L^-T, so one draw of the field noise is
  w = L^-1 Q eta with eta ~ N(0, I), and R = sqrt(alpha eps / mu) Gamma L^-1 Q.  This is
  positive semi-definite by construction; it needs one solve with L per draw, and no
  symmetry of L or of L^-1 C.
* Composite mesh (Sec. "Spatially Adaptive Discretizations"): L = M^-1 S with M the diagonal of
  cell volumes and S = -h^3 A symmetric.  A forcing with per-cell amplitudes Q = diag(q) gives
  w = L^-1 Q eta = S^-1 M (q * eta).  With q^2 = c / volume, L^-1 Q Q^T = c S^-1 is symmetric,
  the stationary covariance is C = -(c/2) S^-1 = (c/2) h^-3 A^-1 (the composite sampler's
  target up to scale) and L^-1 C is symmetric.  Any other q (a uniform q, say) gives a
  non-symmetric L^-1 C, which is the case the appendix addresses.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .philox import normals

KIND_FORCING = 5   # noise stream of the forcing eta (see forcing_noise)


def _dense(M):
    return M.toarray() if sp.issparse(M) else np.asarray(M, dtype=np.float64)


def forcing_from_covariance(L, C, eps=1.0):
    """Q Q^T = -(L C + C L^T) / eps: the forcing that keeps C stationary (Lyapunov relation)."""
    L, C = _dense(L), _dense(C)
    return -(L @ C + C @ L.T) / eps


def covariance_from_forcing(L, QQt, eps=1.0):
    """The stationary covariance C solving (L/eps) C + C (L/eps)^T = -Q Q^T (Bartels-Stewart,
    scipy's continuous Lyapunov solver)."""
    return sla.solve_continuous_lyapunov(_dense(L) / eps, -_dense(QQt))


def drift(L, Gamma, f, eps=1.0):
    """Mean increment per unit time a = -eps Gamma L^-1 f."""
    return -eps * (_dense(Gamma) @ np.linalg.solve(_dense(L), np.asarray(f, dtype=np.float64)))


def increment_covariance_rate(L, C, Gamma, eps=1.0, alpha=1.0):
    """b = -eps alpha Gamma (L^-1 C + C L^-T) Gamma^T (sign as in the appendix's final form)."""
    L, C, G = _dense(L), _dense(C), _dense(Gamma)
    LiC = np.linalg.solve(L, C)
    CLt = np.linalg.solve(L, C.T).T          # C L^-T
    return -eps * alpha * (G @ (LiC + CLt) @ G.T)


def mobility(L, Gamma, alpha=1.0, mu=1.0):
    """H = -(alpha/mu) Gamma L^-1 Gamma^T."""
    G = _dense(Gamma)
    return -(alpha / mu) * (G @ np.linalg.solve(_dense(L), G.T))


def noise_covariance(L, C, Gamma, alpha=1.0, mu=1.0):
    """R R^T = -(alpha/mu) Gamma (L^-1 C + C L^-T) Gamma^T."""
    return increment_covariance_rate(L, C, Gamma, eps=1.0 / mu, alpha=alpha)


def noise_factor(L, Q, Gamma, alpha=1.0, mu=1.0, eps=1.0):
    """R = sqrt(alpha eps / mu) Gamma L^-1 Q (so R R^T equals noise_covariance with the
    stationary C of the forcing Q at this eps)."""
    return np.sqrt(alpha * eps / mu) * (_dense(Gamma) @ np.linalg.solve(_dense(L), _dense(Q)))


# ------------------------------------------------------------- composite mesh, Q = diag(q)
def forcing_noise(seed, sample, nbase, nfine):
    """eta for draw `sample`: the coarse part on the whole base grid (stream colour 0, site =
    base cell index) and the fine part on the box (colour 1, site = fine index), kind
    KIND_FORCING, level 0, slot 0, component 0, counter cycle = sample."""
    ec = normals(seed, sample, 0, 0, 0, 0, KIND_FORCING, np.arange(nbase))
    ef = normals(seed, sample, 0, 0, 1, 0, KIND_FORCING, np.arange(nfine))
    return ec, ef


def forced_field(grid, qc, qf, eta_c, eta_f):
    """w = L^-1 Q eta on a composite grid (oracle.composite.CompositeGrid), Q = diag(q): the
    sparse solve with L = M^-1 S itself.  qc, eta_c: base-grid arrays (covered entries unused);
    qf, eta_f: fine-box arrays.  Returns (wc on the base grid with covered cells 0, wf)."""
    qe = np.concatenate([np.asarray(qc)[grid.coarse_cells] * np.asarray(eta_c)[grid.coarse_cells],
                         np.asarray(qf) * np.asarray(eta_f)])
    w = spla.spsolve(grid.laplacian().tocsc(), qe)
    c, f = grid.split(w)
    return c, f


def forced_covariance(grid, q):
    """Cov(w) = L^-1 Q Q^T L^-T (dense; q over the composite unknowns)."""
    Li = np.linalg.inv(grid.laplacian().toarray())
    return (Li * np.asarray(q) ** 2) @ Li.T
