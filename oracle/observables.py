"""Oracle: scalar observables and moments of the sampled field (test infrastructure).

Sec. "Stochastic Iterative Methods" judges the cost of a sampler by how many iterations
separate effectively independent samples: the lag-k correlation of the emitted fields.  It is
read off scalar observables of each sample.  The observables here are

* projections of x onto eigenvectors of A.  On the uniform grid A is a Kronecker sum of 1D
  operators: the periodic axes are diagonalised by real Fourier vectors and the wall axis
  (antisymmetric ghost cells) by the cell-centred sine vectors sin(pi m (z + 1/2) / nz).  A
  product of one real 1D eigenvector per axis is a real eigenvector of A with the sum of the
  1D eigenvalues;
* the energy E = 1/2 x^T A x of the sample (its expectation is kT N / 2 under the target
  law N(0, kT A^-1));
* per-cell running sums of x and x*x (first and second moments, i.e. the diagonal of the
  sample covariance).

Real 1D periodic basis on n points (n even), index a = 0..n-1:
  a = 0            constant 1/sqrt(n)                        (wave number 0)
  a = 2j - 1       sqrt(2/n) cos(2 pi j i / n), 1 <= j < n/2
  a = 2j           sqrt(2/n) sin(2 pi j i / n), 1 <= j < n/2
  a = n - 1        (-1)^i / sqrt(n)                          (wave number n/2)
with eigenvalue 4 sin^2(pi j / n) / h^2 of the 1D operator -d^2 (three-point, periodic).
Wall axis, m = 1..nz: sin(pi m (z + 1/2) / nz) normalised, eigenvalue 4 sin^2(pi m/(2 nz))/h^2.
"""
import numpy as np

from .operator import apply_A


def periodic_wavenumber(n, a):
    if a == 0:
        return 0
    if a == n - 1:
        return n // 2
    return (a + 1) // 2


def periodic_vector(n, a):
    """Real orthonormal eigenvector a of the periodic 1D second difference on n points."""
    i = np.arange(n, dtype=np.float64)
    if a == 0:
        return np.full(n, 1.0 / np.sqrt(n))
    if a == n - 1:
        return np.where(i % 2 == 0, 1.0, -1.0) / np.sqrt(n)
    j = (a + 1) // 2
    f = np.cos if a % 2 == 1 else np.sin
    return np.sqrt(2.0 / n) * f(2.0 * np.pi * j * i / n)


def wall_vector(nz, m):
    """Orthonormal wall-axis eigenvector m = 1..nz on cell centres."""
    z = np.arange(nz, dtype=np.float64)
    v = np.sin(np.pi * m * (z + 0.5) / nz)
    return v / np.linalg.norm(v)


def mode_eigenvalue(nx, ny, nz, mode, h=1.0):
    a, b, m = mode
    jx = periodic_wavenumber(nx, a)
    jy = periodic_wavenumber(ny, b)
    return (4.0 * np.sin(np.pi * jx / nx) ** 2 + 4.0 * np.sin(np.pi * jy / ny) ** 2
            + 4.0 * np.sin(np.pi * m / (2.0 * nz)) ** 2) / (h * h)


def mode_vector(nx, ny, nz, mode):
    """The eigenvector phi(x, y, z) = e_a(x) e_b(y) w_m(z), flattened with x fastest."""
    a, b, m = mode
    ex = periodic_vector(nx, a)
    ey = periodic_vector(ny, b)
    ez = wall_vector(nz, m)
    return (ez[:, None, None] * ey[None, :, None] * ex[None, None, :]).ravel()


def lowest_modes(nx, ny, nz, K):
    """The K eigenvectors of A with the smallest eigenvalues, as (a, b, m) triples.

    Ties are broken by m, then b, then a.  Eigenvalues are compared after rounding to a grid
    of 2^-30 (in units of 1/h^2) so that equal eigenvalues reached by different sums of the
    1D terms compare equal.  Only a, b < 2K + 2 and m <= K + 1 are enumerated: a mode beyond
    those bounds has at least K modes strictly below it.
    """
    cand = []
    for m in range(1, min(nz, K + 1) + 1):
        for b in range(min(ny, 2 * K + 2)):
            for a in range(min(nx, 2 * K + 2)):
                lam = mode_eigenvalue(nx, ny, nz, (a, b, m))
                cand.append((int(round(lam * 2.0 ** 30)), m, b, a))
    cand.sort()
    return [(a, b, m) for (_, m, b, a) in cand[:K]]


def projections(x, nx, ny, nz, modes):
    """<phi_q, x> for each mode q."""
    x = np.asarray(x, dtype=np.float64).ravel()
    return np.array([np.dot(mode_vector(nx, ny, nz, md), x) for md in modes])


def energy(x, nx, ny, nz, h=1.0):
    """E = 1/2 x^T A x."""
    x = np.asarray(x, dtype=np.float64).ravel()
    return 0.5 * float(np.dot(x, apply_A(x, nx, ny, nz, h)))


def observables(x, nx, ny, nz, modes, h=1.0):
    """[projections onto `modes`..., energy] of one component's field."""
    return np.concatenate([projections(x, nx, ny, nz, modes), [energy(x, nx, ny, nz, h)]])


def moments(samples):
    """(sum of x, sum of x*x) over the leading (sample) axis."""
    s = np.asarray(samples, dtype=np.float64)
    return s.sum(axis=0), (s * s).sum(axis=0)
