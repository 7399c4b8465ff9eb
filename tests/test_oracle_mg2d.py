"""Pins of the 2D wall-bounded oracle (CPU).

* The assembled 5-point operator has the closed-form spectrum (4/h^2)[sin^2(pi j/nx) +
  sin^2(pi m/(2 nz))], and equals the 3D operator of a grid one cell deep in y (whose periodic
  y-neighbour is the cell itself, so the y faces cancel).
* The mode vectors are eigenvectors with those eigenvalues.
* Galerkin operators: the first coarse operator's interior row is the tensor sum of the 1D
  pieces [-1/16, -1/4, 5/8, -1/4, -1/16] and [3/8, 5/4, 3/8] (the 3D hand-derived values).
* The heat-bath pass draws from the exact Gaussian conditional (dense conditioning).
* Exactness: the stationary covariance of the extracted affine map of one cycle equals kT A^-1
  (eq. J = C - R C R^T) to 1e-12, for the multigrid cycle and for the one-level Gauss-Seidel
  chain; the multigrid cycle contracts (spectral radius < 0.15), Gauss-Seidel does not.
* Special cases: the one-level Cholesky hierarchy is an exact draw; the noise-free cycle solves.
"""
import numpy as np
import pytest

from oracle import mg2d
from oracle.analysis import extract_affine_map, stationary_covariance, extract_linear_part
from oracle.operator import assemble_A
from oracle.philox import PhiloxNoise


@pytest.mark.parametrize("dims", [(8, 4), (6, 5), (16, 8)])
def test_operator_spectrum_and_3d_reduction(dims):
    nx, nz = dims
    A = mg2d.assemble_A2(nx, nz, h=0.5).toarray()
    assert np.allclose(np.linalg.eigvalsh(A), mg2d.eigenvalues_2d(nx, nz, 0.5), atol=1e-12)
    A3 = assemble_A(nx, 1, nz, h=0.5).toarray()
    assert np.allclose(A, A3, atol=1e-13)
    for a, m in ((0, 1), (1, 2), (nx - 1, nz), (2, 1)):
        v = mg2d.mode_vector_2d(nx, nz, a, m)
        j = (a + 1) // 2 if a not in (0, nx - 1) else (0 if a == 0 else nx // 2)
        lam = 16.0 * (np.sin(np.pi * j / nx) ** 2 + np.sin(np.pi * m / (2 * nz)) ** 2)
        assert abs(np.linalg.norm(v) - 1.0) < 1e-13 and np.allclose(A @ v, lam * v, atol=1e-12)


def test_galerkin_interior_row():
    mg = mg2d.StochasticMG2D(16, 16, levels=2)
    A1 = mg.levels[1].A.toarray()
    nx = 8
    i = 3 + nx * 4   # interior cell (3, 4)
    row = np.zeros((5, 5))
    for dz in range(-2, 3):
        for dx in range(-2, 3):
            row[dz + 2, dx + 2] = A1[i, (3 + dx) % nx + nx * (4 + dz)]
    a = np.array([-1 / 16, -1 / 4, 5 / 8, -1 / 4, -1 / 16])
    m = np.array([0.0, 3 / 8, 5 / 4, 3 / 8, 0.0])
    assert np.allclose(row, np.outer(a, m) + np.outer(m, a), atol=1e-14)


def test_point_pass_is_gaussian_conditional():
    mg = mg2d.StochasticMG2D(6, 4, kT=0.8, levels=1, coarsest="smooth")
    L = mg.levels[0]
    A = L.A.toarray()
    rng = np.random.default_rng(2)
    x, b = rng.standard_normal(L.n), rng.standard_normal(L.n)
    for colour in (0, 1):
        S, rest = L.sets[colour], L.sets[1 - colour]
        mean = np.linalg.solve(A[np.ix_(S, S)], b[S] - A[np.ix_(S, rest)] @ x[rest])
        y = x.copy()
        mg._point_pass(L, y, b, colour, None, None)
        assert np.allclose(y[S], mean, atol=1e-13) and np.array_equal(y[rest], x[rest])


@pytest.mark.parametrize("kw", [dict(levels=3), dict(levels=2), dict(levels=1, coarsest="smooth")])
def test_cycle_stationary_covariance_is_exact(kw):
    mg = mg2d.StochasticMG2D(8, 8, kT=1.3, **kw)
    T, G = extract_affine_map(mg)
    C = stationary_covariance(T, G @ G.T)
    target = 1.3 * np.linalg.inv(mg.levels[0].A.toarray())
    assert np.max(np.abs(C - target)) <= 1e-12 * np.max(np.abs(target))
    rho = np.max(np.abs(np.linalg.eigvals(T)))
    if kw.get("coarsest") == "smooth":
        assert rho > 0.4
    else:
        assert rho < 0.15


def test_one_level_cholesky_and_solve():
    mg = mg2d.StochasticMG2D(4, 4, kT=1.0, levels=1)
    T, G = extract_affine_map(mg)
    A = mg.levels[0].A.toarray()
    assert np.allclose(T, 0.0, atol=1e-14) and np.allclose(G @ G.T, np.linalg.inv(A), atol=1e-13)
    mg = mg2d.StochasticMG2D(16, 8, levels=3)
    f = np.random.default_rng(4).standard_normal(128)
    u = np.zeros(128)
    for _ in range(14):
        u = mg.vcycle(u, f)
    assert np.linalg.norm(f - mg.levels[0].A @ u) <= 1e-11 * np.linalg.norm(f)
