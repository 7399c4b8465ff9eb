"""Pins for the oracle's composite (spatially adaptive) grid and its FAC cycle (CPU only).

* Special cases: with no refined box the operator is the uniform-grid operator; with the
  box covering the whole domain it is the uniform operator of the fine grid (scaled by the
  fine/coarse volume ratio 1/8).
* Structure: S = M L symmetric (L^-1 times the inverse volume matrix symmetric, the
  property the paper states), A positive definite, rows summing to zero except for the
  wall terms (conservation), and the quadratic form equal to the sum over faces of
  area * gradient^2 * distance.
* Hand-derived interface coefficients of the 3D coarse-fine face (four fine cells, 3/4 of
  the coarse width).
* Consistency: a manufactured solution converges at second order in the RMS norm (an
  interface distance of h/2 instead of 3h/4 falls to about first order and fails).
* Prolongation: the trilinear map reproduces linear fields on fine cells away from walls.
* FAC cycle: the stationary covariance of one stochastic cycle equals kT A^-1 (eq.
  J_eq_C_R through the extracted affine map), its spectral radius is small, and the
  noise-free cycle converges to the direct solution.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.composite import CompositeGrid, FACSampler
from oracle.operator import assemble_A
from oracle.analysis import stationary_covariance


def _centres(g):
    h = g.h
    z, y, x = np.meshgrid(np.arange(g.nz), np.arange(g.ny), np.arange(g.nx), indexing="ij")
    cc = g.coarse_cells
    pc = [(x.ravel()[cc] + 0.5) * h, (y.ravel()[cc] + 0.5) * h, (z.ravel()[cc] + 0.5) * h]
    x0, _, y0, _, z0, _ = g.box
    k, j, i = np.meshgrid(np.arange(g.fz), np.arange(g.fy), np.arange(g.fx), indexing="ij")
    hf = 0.5 * h
    pf = [x0 * h + (i.ravel() + 0.5) * hf, y0 * h + (j.ravel() + 0.5) * hf,
          z0 * h + (k.ravel() + 0.5) * hf]
    return [np.concatenate([a, b]) for a, b in zip(pc, pf)]


def test_no_box_is_uniform_operator():
    g = CompositeGrid(8, 6, 4, None, h=0.7)
    assert abs(g.A - assemble_A(8, 6, 4, 0.7)).max() < 1e-14


def test_full_box_is_uniform_fine_operator():
    g = CompositeGrid(4, 4, 3, (0, 4, 0, 4, 0, 3), h=1.0)
    ref = assemble_A(8, 8, 6, 0.5) / 8.0
    assert abs(g.A - ref).max() < 1e-14


def test_symmetry_definiteness_conservation():
    h = 0.5
    g = CompositeGrid(8, 8, 6, (2, 6, 3, 7, 1, 4), h=h)
    assert abs(g.S - g.S.T).max() == 0.0
    L = g.laplacian().toarray()
    K = np.linalg.inv(L) @ np.diag(1.0 / g.vol)        # L^-1 C with C = M^-1
    assert np.abs(K - K.T).max() < 1e-10 * np.abs(K).max()
    A = g.A.toarray()
    assert np.linalg.eigvalsh(A).min() > 0.0
    # row sums of A: zero except wall faces, +2/h^2 per coarse wall face, +1/h^2 per fine one
    rs = A.sum(axis=1)
    expect = np.zeros(g.n)
    cz = g.coarse_cells // (g.nx * g.ny)
    expect[:g.nc] += 2.0 / h**2 * ((cz == 0).astype(float) + (cz == g.nz - 1))
    k = np.arange(g.nf) // (g.fx * g.fy)
    zabs = 2 * g.box[4] + k
    expect[g.nc:] += 1.0 / h**2 * ((zabs == 0).astype(float) + (zabs == 2 * g.nz - 1))
    assert np.abs(rs - expect).max() < 1e-12 / h**2


def test_energy_is_sum_over_faces():
    g = CompositeGrid(6, 8, 4, (1, 4, 2, 6, 0, 2), h=1.3)
    c = np.random.default_rng(3).standard_normal(g.n)
    quad = float(c @ (g.A @ c)) * g.h**3
    assert abs(quad - g.face_energy(c)) < 1e-12 * abs(quad)


def test_interface_coefficients_by_hand():
    """h = 1.  Coarse A next to the box (one coarse-fine face, interior in z): diagonal
    5 + 4/3, coupling -1/3 to each of the four fine cells.  A fine cell of that face:
    diagonal 5/2 + 1/12, +1/12 to its diagonal partner in the face, 1/12 - 1/2 = -5/12 to
    its two face partners, -1/3 to A."""
    g = CompositeGrid(8, 8, 8, (2, 6, 2, 6, 2, 6))
    A = g.A.toarray()
    a = g.coarse_id[g.base_index(1, 3, 4)]          # west of the box at y=3, z=4
    kids = [g.fine_index(0, j, k) for k in (4, 5) for j in (2, 3)]
    assert A[a, a] == pytest.approx(5.0 + 4.0 / 3.0, abs=1e-14)
    for q in kids:
        assert A[a, q] == pytest.approx(-1.0 / 3.0, abs=1e-14)
    f0 = g.fine_index(0, 2, 4)
    assert A[f0, f0] == pytest.approx(2.5 + 1.0 / 12.0, abs=1e-14)
    assert A[f0, g.fine_index(0, 3, 5)] == pytest.approx(1.0 / 12.0, abs=1e-14)
    assert A[f0, g.fine_index(0, 3, 4)] == pytest.approx(-5.0 / 12.0, abs=1e-14)
    assert A[f0, g.fine_index(0, 2, 5)] == pytest.approx(-5.0 / 12.0, abs=1e-14)
    assert A[f0, g.fine_index(1, 2, 4)] == pytest.approx(-0.5, abs=1e-14)


def test_second_order_convergence():
    """Manufactured u = sin(2 pi x) cos(2 pi y) sin(2 pi z) on [0,1)^2 x [0,1/2] with a box
    over the middle of x, y touching the bottom wall; A u = Mhat (-Lap u)."""
    rms = []
    for n in (8, 16, 32):
        g = CompositeGrid(n, n, n // 2, (n // 4, 3 * n // 4, n // 4, 3 * n // 4, 0, n // 8),
                          h=1.0 / n)
        X, Y, Z = _centres(g)
        u = np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y) * np.sin(2 * np.pi * Z)
        lam = 3 * (2 * np.pi) ** 2
        mhat = np.where(np.arange(g.n) < g.nc, 1.0, 0.125)
        uh = spla.spsolve(g.A.tocsc(), mhat * lam * u)
        rms.append(np.sqrt(np.mean((uh - u) ** 2)))
    assert rms[0] / rms[1] > 3.5 and rms[1] / rms[2] > 3.5, rms


def test_prolongation_reproduces_linear_fields():
    g = CompositeGrid(12, 12, 8, (3, 8, 4, 9, 2, 6), h=1.0)
    P = g.prolong_base()
    z, y, x = np.meshgrid(np.arange(8), np.arange(12), np.arange(12), indexing="ij")
    lin = (0.3 * (x + 0.5) - 0.7 * (y + 0.5) + 1.1 * (z + 0.5)).ravel()
    v = P @ lin
    X, Y, Z = _centres(g)
    assert np.abs(v - (0.3 * X - 0.7 * Y + 1.1 * Z)).max() < 1e-12
    assert np.array_equal(v[:g.nc], lin[g.coarse_cells])


def test_classes_partition_unknowns():
    g = CompositeGrid(8, 8, 8, (2, 6, 2, 6, 2, 6))
    ids = np.concatenate([c[0] for c in g.classes()])
    assert np.array_equal(np.sort(ids), np.arange(g.n))


def test_class_noise_sites_distinct():
    """Every class draws distinct noise sites: the halved indices of the parity classes (one
    cell of each pair (2q, 2q + 1) of its array) and the plain indices of the layer classes;
    consecutive cells of a parity class in a row share a Philox call (sites 2m, 2m + 1)."""
    for box in ((2, 6, 2, 6, 2, 6), (0, 4, 1, 7, 0, 8), (3, 5, 2, 4, 1, 3)):
        g = CompositeGrid(8, 8, 8, box)
        for c, (ids, sites) in enumerate(g.classes()):
            assert np.unique(sites).size == sites.size, (box, c)
        # coarse parity class 0: base cells (x, y, z) and (x + 2, y, z) are halved sites
        # differing by one, so pairs of neighbours along x share a call
        ids, sites = g.classes()[0]
        cells = g.coarse_cells[ids]
        assert np.array_equal(sites, cells >> 1)


def test_fac_cycle_is_exact_and_fast():
    g = CompositeGrid(8, 8, 4, (2, 6, 2, 6, 0, 2))
    kT = 1.3
    fac = FACSampler(g, kT=kT, coarsest_max=64)
    assert [L.dims for L in fac.base.levels] == [(8, 8, 4), (4, 4, 2)]
    T, G = fac.affine_map()
    C = stationary_covariance(T, G @ G.T)
    target = kT * np.linalg.inv(g.A.toarray())
    assert np.abs(C - target).max() < 1e-12 * np.abs(target).max()
    assert max(abs(np.linalg.eigvals(T))) < 0.15


def test_fac_solve_matches_direct():
    g = CompositeGrid(16, 16, 8, (4, 12, 4, 12, 0, 4))
    fac = FACSampler(g, coarsest_max=256)
    f = np.random.default_rng(5).standard_normal(g.n)
    u, k, rel = fac.solve(f, rtol=1e-11)
    assert rel <= 1e-11 and k <= 14
    ref = spla.spsolve(g.A.tocsc(), f)
    assert np.abs(u - ref).max() < 1e-9 * np.abs(ref).max()


def test_row_of_matches_assembly():
    from oracle.composite import row_of
    nx, ny, nz, box, h = 12, 8, 6, (0, 5, 3, 7, 0, 6), 0.8
    g = CompositeGrid(nx, ny, nz, box, h=h)
    A = g.A.toarray()
    for r in range(g.n):
        if r < g.nc:
            row = row_of(nx, ny, nz, box, h, "c", int(g.coarse_cells[r]))
        else:
            row = row_of(nx, ny, nz, box, h, "f", r - g.nc)
        dense = np.zeros(g.n)
        for (kind, q), v in row.items():
            dense[g.coarse_id[q] if kind == "c" else g.nc + q] += v
        assert np.abs(dense - A[r]).max() < 1e-13 * np.abs(A[r]).max()


def test_gauss_seidel_only_composite_chain_is_exact_but_slow():
    """The composite sweeps alone (no coarse correction) also leave kT A^-1 invariant (every
    class pass is an exact conditional draw), but contract far more slowly than the FAC
    cycle: spectral radius 0.78 against 0.105 on this grid."""
    g = CompositeGrid(8, 8, 4, (2, 6, 2, 6, 0, 2))
    gs = FACSampler(g, kT=0.7, coarsest_max=64, gs_only=True)
    T, G = gs.affine_map()
    C = stationary_covariance(T, G @ G.T)
    target = 0.7 * np.linalg.inv(g.A.toarray())
    assert np.abs(C - target).max() < 1e-11 * np.abs(target).max()
    rho_gs = max(abs(np.linalg.eigvals(T)))
    assert 0.7 < rho_gs < 0.85
