"""Pins of the oracle's single-cell evaluators (CPU): each equals, at every cell of small grids
(odd-even extents, both walls, periodic seams), the whole-level oracle step that is pinned
elsewhere -- the assembled A (closed-form spectrum), the heat-bath pass of StochasticMG (Gaussian
conditioning), and the sparse Kronecker prolongation (reproduction of linear fields) -- so a
wrong face, weight, sign or site index in the cell-by-cell form fails here."""
import numpy as np

from oracle import sampled
from oracle.mg import StochasticMG
from oracle.operator import assemble_A
from oracle.philox import PhiloxNoise
from oracle.transfer import prolong_3d

DIMS = [(6, 4, 5), (8, 8, 2), (4, 6, 8)]


def test_row_A_equals_assembled_rows():
    for nx, ny, nz in DIMS:
        A = assemble_A(nx, ny, nz, h=0.7).toarray()
        for i in range(nx * ny * nz):
            cols, vals = sampled.row_A(nx, ny, nz, i, h=0.7)
            row = np.zeros(nx * ny * nz)
            row[cols] = vals
            assert np.allclose(row, A[i], rtol=0, atol=1e-13), (nx, ny, nz, i)


def test_heat_bath_at_equals_point_pass():
    for nx, ny, nz in ((8, 8, 4), (6, 4, 5)):
        mg = StochasticMG(nx, ny, nz, kT=1.3, levels=1, coarsest="smooth")
        L = mg.levels[0]
        rng = np.random.default_rng(5)
        x = rng.standard_normal(L.n)
        b = rng.standard_normal(L.n)
        for colour in (0, 1):
            ref = x.copy()
            mg._point_pass(L, ref, b, colour, PhiloxNoise(17), (3, 2, 1))
            cells = np.array([i for i in range(L.n) if (i % nx + (i // nx) % ny + i // (nx * ny)) % 2 == colour])
            got = sampled.heat_bath_at(x.reshape(nz, ny, nx), b.reshape(nz, ny, nx), cells,
                                       colour, seed=17, cycle=3, slot=2, comp=1, kT=1.3)
            assert np.allclose(got, ref[cells], rtol=0, atol=1e-12), (nx, ny, nz, colour)


def test_restrict_and_prolong_at_equal_sparse_transfers():
    for nx, ny, nz in ((8, 4, 6), (4, 8, 4)):
        P = prolong_3d(nx // 2, ny // 2, nz // 2)
        A = assemble_A(nx, ny, nz)
        rng = np.random.default_rng(9)
        x, b = rng.standard_normal(nx * ny * nz), rng.standard_normal(nx * ny * nz)
        ref = P.T @ (b - A @ x)
        nc = ref.size
        got = sampled.restrict_residual_at(x.reshape(nz, ny, nx), b.reshape(nz, ny, nx),
                                           np.arange(nc))
        assert np.allclose(got, ref, rtol=0, atol=1e-12)
        e = rng.standard_normal(nc)
        got = sampled.prolong_at(e.reshape(nz // 2, ny // 2, nx // 2), (nx, ny, nz),
                                 np.arange(nx * ny * nz))
        assert np.allclose(got, P @ e, rtol=0, atol=1e-13)


def test_sample_cells_cover_walls_and_seams():
    cells = sampled.sample_cells(16, 8, 6, 50, 1, colour=1)
    x, y, z = cells % 16, (cells // 16) % 8, cells // 128
    assert np.all((x + y + z) % 2 == 1)
    assert {0, 5} <= set(z.tolist()) and 0 in y and (0 in x or 15 in x)
