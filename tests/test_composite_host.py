"""Host-side checks of the composite-grid C-ABI (no GPU): the library's plan stores, for every
cell of every base level, the row of the Galerkin operator A_0 = P^T A P, A_{l+1} =
P_l^T A_l P_l that the oracle forms by sparse triple products; invalid geometries are rejected."""
import ctypes

import numpy as np
import pytest

from oracle.composite import CompositeGrid, FACSampler
from paper_1003_2680_amd import abi
from paper_1003_2680_amd import composite as pc

CASES = [
    (8, 8, 4, (2, 6, 2, 6, 0, 2), 64),      # box on the bottom wall
    (16, 16, 8, (4, 12, 3, 11, 1, 5), 64),  # interior box, three base levels
    (16, 12, 8, (0, 6, 5, 12, 0, 8), 64),   # box on the periodic seam and on both walls
    (12, 8, 6, (3, 9, 1, 4, 2, 3), 512),    # one base level: the coarsest is the base grid
]


@pytest.mark.parametrize("case", CASES)
def test_stored_galerkin_rows_match_oracle(case):
    nx, ny, nz, box, cm = case
    hd, info = pc.plan(nx, ny, nz, box, coarsest_max=cm)
    try:
        g = CompositeGrid(nx, ny, nz, box)
        fac = FACSampler(g, coarsest_max=cm)
        assert [tuple(info.dims[l]) for l in range(info.n_levels)] == \
            [L.dims for L in fac.base.levels]
        assert info.unknowns == g.n
        assert info.layer_cells == sum(c[0].size for c in g.classes()[4:])
        for l, L in enumerate(fac.base.levels):
            A = L.A.tocsr()
            for cell in range(L.n):
                t, v = pc.stored_row(hd, l, cell)
                row = np.zeros(L.n)
                np.add.at(row, t, v)
                ref = A[cell].toarray().ravel()
                assert np.abs(row - ref).max() <= 1e-14 * np.abs(ref).max(), (l, cell)
    finally:
        pc.destroy_plan(hd)


@pytest.mark.parametrize("nx,ny,nz,box", [
    (8, 8, 4, (0, 8, 2, 6, 0, 2)),   # spans the periodic x extent
    (8, 8, 4, (2, 6, 2, 6, 3, 5)),   # leaves the grid in z
    (8, 8, 4, (4, 4, 2, 6, 0, 2)),   # empty
    (7, 8, 4, (2, 6, 2, 6, 0, 2)),   # odd nx
])
def test_invalid_geometry_rejected(nx, ny, nz, box):
    with pytest.raises(abi.SMGError) as e:
        pc.plan(nx, ny, nz, box)
    assert e.value.code == abi.SMG_EINVAL


@pytest.mark.parametrize("lanes", [1, 4, -1, 16])
def test_invalid_row_lanes_rejected(lanes):
    with pytest.raises(abi.SMGError) as e:
        pc.plan(8, 8, 4, (2, 6, 2, 6, 0, 2), row_lanes=lanes)
    assert e.value.code == abi.SMG_EINVAL and "row_lanes" in str(e.value)


@pytest.mark.parametrize("lanes", [0, 2, 8])
def test_row_lanes_accepted(lanes):
    hd, info = pc.plan(8, 8, 4, (2, 6, 2, 6, 0, 2), row_lanes=lanes)
    pc.destroy_plan(hd)
    assert info.n_levels >= 1
