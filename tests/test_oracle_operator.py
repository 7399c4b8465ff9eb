"""Pins for the oracle's operator, transfers and Galerkin hierarchy (CPU only).

Each check compares the oracle with something the mathematics fixes independently of how
the oracle builds it: a closed-form spectrum, exact reproduction of linear functions by
trilinear interpolation, hand-derived Galerkin coefficients.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.operator import assemble_A, apply_A
from oracle.transfer import prolong_1d, prolong_3d
from oracle.hierarchy import build_hierarchy, plan_levels
from oracle import spectral


@pytest.mark.parametrize("dims", [(8, 8, 8), (6, 4, 5), (4, 6, 2), (4, 4, 1), (2, 4, 3)])
def test_spectrum_closed_form(dims):
    # eigenvalues (4/h^2)[sin^2(pi j/nx) + sin^2(pi k/ny) + sin^2(pi m/(2nz))], m = 1..nz
    nx, ny, nz = dims
    h = 0.5
    A = assemble_A(nx, ny, nz, h).toarray()
    assert np.allclose(A, A.T, atol=0, rtol=0)
    ev = np.sort(np.linalg.eigvalsh(A))
    j, k, m = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(1, nz + 1), indexing="ij")
    cf = 4.0 / h ** 2 * (np.sin(np.pi * j / nx) ** 2 + np.sin(np.pi * k / ny) ** 2
                         + np.sin(np.pi * m / (2 * nz)) ** 2)
    assert np.max(np.abs(ev - np.sort(cf.ravel()))) < 1e-12 * ev.max()
    assert ev.min() > 0.0


def test_diagonal_and_constants():
    nx, ny, nz = 6, 4, 5
    A = assemble_A(nx, ny, nz)
    d = A.diagonal().reshape(nz, ny, nx)
    assert np.all(d[1:-1] == 6.0) and np.all(d[0] == 7.0) and np.all(d[-1] == 7.0)
    r = (A @ np.ones(nx * ny * nz)).reshape(nz, ny, nx)
    assert np.all(r[1:-1] == 0.0)           # constants are harmonic away from the walls
    assert np.all(r[0] == 2.0) and np.all(r[-1] == 2.0)


def test_stencil_form_matches_matrix():
    rng = np.random.default_rng(3)
    x = rng.standard_normal(6 * 4 * 5)
    assert np.max(np.abs(assemble_A(6, 4, 5, 0.3) @ x - apply_A(x, 6, 4, 5, 0.3))) < 1e-10


def test_spectral_solver_against_direct():
    nx, ny, nz = 8, 6, 10
    rng = np.random.default_rng(0)
    f = rng.standard_normal(nx * ny * nz)
    u_dir = spla.spsolve(assemble_A(nx, ny, nz).tocsc(), f)
    u_sp = spectral.solve(f, nx, ny, nz)
    assert np.max(np.abs(u_sp - u_dir)) < 1e-12 * np.max(np.abs(u_dir))


def test_prolongation_reproduces_linear_functions():
    # fine spacing 1: fine centre i at i + 1/2, coarse centre J at 2J + 1
    nc = 6
    s_c = 2.0 * np.arange(nc) + 1.0
    s_f = np.arange(2 * nc) + 0.5
    Pw = prolong_1d(nc, periodic=False).toarray()
    # f(s) = s vanishes on the bottom wall: exact up to and including the bottom wall
    # cell (ghost rule); the top wall cell sees the ghost of a function that does not vanish
    assert np.allclose((Pw @ s_c)[:-1], s_f[:-1], atol=1e-15)
    # f(s) = 2nc - s vanishes on the top wall
    assert np.allclose((Pw @ (2 * nc - s_c))[1:], (2 * nc - s_f)[1:], atol=1e-15)
    Pp = prolong_1d(nc, periodic=True).toarray()
    inner = slice(1, 2 * nc - 1)
    assert np.allclose((Pp @ s_c)[inner], s_f[inner], atol=1e-15)
    assert np.allclose(Pp @ np.ones(nc), 1.0)
    assert np.allclose(Pp.sum(axis=0), 2.0)            # each coarse cell spreads 1/4+3/4+3/4+1/4


def test_prolongation_3d_is_tensor_trilinear():
    P = prolong_3d(2, 3, 2).toarray()
    # fine (x=2, y=2, z=1) = coarse parents x in {1 (3/4), 0 (1/4)}, y in {1, 0}, z in {0 (3/4), 1 (1/4)}
    nxf, nyf = 4, 6
    i = 2 + nxf * (2 + nyf * 1)
    w = {}
    for cx, wx in ((1, .75), (0, .25)):
        for cy, wy in ((1, .75), (0, .25)):
            for cz, wz in ((0, .75), (1, .25)):
                w[cx + 2 * (cy + 3 * cz)] = wx * wy * wz
    expect = np.zeros(12)
    for k, v in w.items():
        expect[k] += v
    assert np.allclose(P[i], expect, atol=0)


def test_galerkin_one_dimensional_pieces():
    # P^T tridiag(-1,2,-1) P and P^T P on a periodic line, hand-derived:
    #   (P^T P)[J,J]   = 2(1/4)^2 + 2(3/4)^2 = 5/4 ; (P^T P)[J,J+1] = 2 (3/4)(1/4) = 3/8
    #   P^T a P        = [-1/16, -1/4, 5/8, -1/4, -1/16]
    nc = 8
    P = prolong_1d(nc, periodic=True).toarray()
    nf = 2 * nc
    a = 2 * np.eye(nf) - np.roll(np.eye(nf), 1, axis=1) - np.roll(np.eye(nf), -1, axis=1)
    m1 = P.T @ P
    a1 = P.T @ a @ P
    J = 4
    assert np.allclose(m1[J, J - 1:J + 2], [3 / 8, 5 / 4, 3 / 8], atol=1e-15)
    assert np.allclose(a1[J, J - 2:J + 3], [-1 / 16, -1 / 4, 5 / 8, -1 / 4, -1 / 16], atol=1e-15)
    assert abs(m1[J, J + 2]) == 0 and abs(a1[J, J + 3]) == 0


def test_galerkin_3d_coefficients():
    H = build_hierarchy(16, 16, 16, levels=3)
    A1 = H[1].A
    i = 3 + 8 * (3 + 8 * 3)
    # interior: 3 * (5/8)(5/4)(5/4) = 375/128
    assert A1[i, i] == pytest.approx(375 / 128, abs=1e-14)
    # wall row: a_z = 7/8, m_z = 7/8 there (P column (1/2, 3/4, 1/4)): 7/8*25/16 + 2*7/8*25/32
    j = 3 + 8 * 3
    assert A1[j, j] == pytest.approx(175 / 64, abs=1e-14)
    assert A1[i].nnz == 81                     # 5x3x3 union of three tensor stencils
    A2 = build_hierarchy(32, 32, 32, levels=3)[2].A
    assert A2[i].nnz == 125                    # from level 2 on the mass pieces are 5 wide
    for L in H:
        assert abs(L.A - L.A.T).max() < 1e-14
    # Galerkin operators of a Kronecker sum: constants still harmonic away from walls
    r = (A1 @ np.ones(8 ** 3)).reshape(8, 8, 8)
    assert np.max(np.abs(r[2:-2])) < 1e-14


def test_level_plan():
    assert plan_levels(16, 16, 16, levels=3) == [(16, 16, 16), (8, 8, 8), (4, 4, 4)]
    assert len(plan_levels(128, 128, 128, levels=6)) == 6
    assert plan_levels(8, 8, 8, levels=3)[-1] == (2, 2, 2)
    d = plan_levels(256, 256, 16, levels=0, coarsest_max=512)
    assert d[-1] == (16, 16, 1)
    assert plan_levels(48, 48, 48, levels=0, coarsest_max=4096)[-1] == (12, 12, 12)
    with pytest.raises(ValueError):
        plan_levels(12, 12, 12, levels=4)
