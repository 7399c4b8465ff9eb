"""C-ABI host-side checks (no GPU needed).

* the library loads and exports every entry point that include/smg.h declares;
* the planner's level dimensions equal the oracle's;
* the host-built Galerkin tables (1D recurrences, folded by modular indexing) equal the
  oracle's explicit sparse triple products P^T A P, and the block / coarsest factors invert
  the oracle's operators -- two independent constructions of the same operators;
* invalid shapes and parameters are rejected with SMG_EINVAL.
"""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.hierarchy import build_hierarchy, plan_levels, block_sets

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

abi = pytest.importorskip("paper_1003_2680_amd.abi")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(abi.LIB_PATH):
        pytest.fail("libsmg.so is not built (run __graft_entry__.build())")
    return abi.load()


def _create(lib, nx, ny, nz, ncomp=1, levels=0, coarsest_max=512, mode=0, h=1.0, kT=1.0):
    desc = abi.GridDesc(nx, ny, nz, ncomp, h, kT)
    prm = abi.CycleParams(levels, 2, 2, coarsest_max, mode, 0, 1, 0)
    hd = ctypes.c_void_p()
    rc = lib.smg_create_hierarchy(ctypes.byref(desc), ctypes.byref(prm), ctypes.byref(hd))
    return rc, hd


def _info(lib, hd):
    info = abi.Info()
    abi.check(lib.smg_hierarchy_info(hd, ctypes.byref(info)))
    return info


def _table(lib, hd, level, which, count):
    out = np.empty(count)
    abi.check(lib.smg_debug_host_table(hd, level, which, out.ctypes.data_as(ctypes.c_void_p),
                                       count))
    return out


def test_exports_match_header(lib):
    hdr = open(os.path.join(ROOT, "include", "smg.h")).read()
    declared = set(re.findall(r"^(?:int|void|const char\*)\s+(smg\w+)\(", hdr, re.M))
    assert declared, "no declarations parsed"
    assert declared == set(abi.EXPORTED)
    for name in declared:
        assert hasattr(lib, name)


@pytest.mark.parametrize("dims,levels,cmax", [((16, 16, 16), 3, 512), ((128, 128, 128), 6, 512),
                                              ((256, 256, 16), 0, 512), ((48, 48, 48), 0, 4096),
                                              ((12, 8, 6), 0, 64), ((8, 8, 8), 3, 512)])
def test_plan_matches_oracle(lib, dims, levels, cmax):
    rc, hd = _create(lib, *dims, levels=levels, coarsest_max=cmax)
    abi.check(rc)
    try:
        info = _info(lib, hd)
        got = [tuple(info.dims[l]) for l in range(info.n_levels)]
        assert got == plan_levels(*dims, levels=levels, coarsest_max=cmax)
        assert info.state_bytes == 8 * dims[0] * dims[1] * dims[2]
        assert info.workspace_bytes > 0
    finally:
        lib.smg_destroy_hierarchy(hd)


def _matrix_from_table(coef, nx, ny, nz):
    """Sparse operator assembled from [nz][125] row coefficients (wrapping in x and y)."""
    rows, cols, vals = [], [], []
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x = x.ravel(); y = y.ravel(); z = z.ravel()
    i = x + nx * (y + ny * z)
    for oz in range(-2, 3):
        for oy in range(-2, 3):
            for ox in range(-2, 3):
                c = coef.reshape(nz, 125)[z, (oz + 2) * 25 + (oy + 2) * 5 + (ox + 2)]
                zz = z + oz
                ok = (zz >= 0) & (zz < nz) & (c != 0)
                j = (x[ok] + ox) % nx + nx * (((y[ok] + oy) % ny) + ny * zz[ok])
                rows.append(i[ok]); cols.append(j); vals.append(c[ok])
    n = nx * ny * nz
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n)).tocsr()


@pytest.mark.parametrize("dims,levels", [((16, 16, 16), 4), ((16, 16, 8), 3), ((32, 16, 12), 3),
                                         ((8, 8, 8), 3)])
def test_galerkin_tables_match_oracle(lib, dims, levels):
    H = build_hierarchy(*dims, h=0.7, levels=levels)
    rc, hd = _create(lib, *dims, levels=levels, h=0.7, coarsest_max=4096)
    abi.check(rc)
    try:
        for L in H[1:]:
            nx, ny, nz = L.dims
            if L.coarsest:
                n = L.n
                ainv = _table(lib, hd, L.index, 2, n * n).reshape(n, n)
                W = _table(lib, hd, L.index, 3, n * n).reshape(n, n)
                Ad = L.A.toarray()
                assert np.max(np.abs(ainv @ Ad - np.eye(n))) < 1e-10
                assert np.max(np.abs(W.T @ W @ Ad - np.eye(n))) < 1e-10
                assert np.max(np.abs(np.triu(W, 1))) == 0.0
                continue
            coef = _table(lib, hd, L.index, 0, nz * 125)
            A_tab = _matrix_from_table(coef, nx, ny, nz)
            scale = abs(L.A).max()
            assert abs(A_tab - L.A).max() <= 1e-14 * scale
            bf = _table(lib, hd, L.index, 1, (nz // 2) * 192).reshape(nz // 2, 3, 8, 8)
            for c, (bid, cells) in enumerate(block_sets(nx, ny, nz)):
                for k in range(0, len(bid), max(1, len(bid) // 5)):
                    ABB = L.A[cells[k]][:, cells[k]].toarray()
                    bz = cells[k][0] // (nx * ny) // 2
                    Ainv, U = bf[bz, 0], bf[bz, 1]
                    assert np.max(np.abs(bf[bz, 2] - ABB)) <= 1e-14 * np.max(np.abs(ABB))
                    assert np.max(np.abs(Ainv @ ABB - np.eye(8))) < 1e-12
                    assert np.max(np.abs(U @ U.T @ ABB - np.eye(8))) < 1e-12
                    assert np.max(np.abs(np.tril(U, -1))) == 0.0
    finally:
        lib.smg_destroy_hierarchy(hd)


@pytest.mark.parametrize("dims,levels", [((7, 8, 8), 0), ((8, 5, 8), 0), ((12, 12, 12), 4),
                                         ((0, 8, 8), 0)])
def test_invalid_shapes_rejected(lib, dims, levels):
    rc, hd = _create(lib, *dims, levels=levels)
    assert rc == abi.SMG_EINVAL and not hd.value
    assert len(lib.smg_last_error()) > 0


def test_invalid_params_rejected(lib):
    desc = abi.GridDesc(8, 8, 8, 1, 1.0, 1.0)
    hd = ctypes.c_void_p()
    for prm in (abi.CycleParams(0, 2, 2, 0, 0, 0, 1, 0), abi.CycleParams(0, 2, 2, 512, 5, 0, 1, 0),
                abi.CycleParams(0, 2, 2, 512, 0, 0, 0, 0), abi.CycleParams(0, -1, 2, 512, 0, 0, 1, 0),
                abi.CycleParams(0, 2, 2, 8192, 0, 0, 1, 0)):
        assert lib.smg_create_hierarchy(ctypes.byref(desc), ctypes.byref(prm),
                                        ctypes.byref(hd)) == abi.SMG_EINVAL
    # too large a dense coarsest level
    rc, hd = _create(lib, 32, 32, 32, levels=1, coarsest_max=4096)
    assert rc == abi.SMG_EINVAL


def test_boundary_conditions(lib):
    """The wall-bounded channel (periodic x, y; Dirichlet-face z) is accepted spelled out or
    by the zero defaults; every other combination is rejected with SMG_EINVAL."""
    prm = abi.CycleParams(0, 2, 2, 512, 0, 0, 1, 0)
    P, D, DEF = abi.SMG_BC_PERIODIC, abi.SMG_BC_DIRICHLET_FACE, abi.SMG_BC_DEFAULT
    ok = [(DEF, DEF, DEF), (P, P, D), (DEF, P, D), (P, DEF, DEF)]
    bad = [(P, P, P), (D, P, D), (P, D, D), (P, P, 7), (-1, P, D), (D, D, D)]
    for bc, want in [(b, abi.SMG_OK) for b in ok] + [(b, abi.SMG_EINVAL) for b in bad]:
        desc = abi.GridDesc(8, 8, 8, 1, 1.0, 1.0, *bc)
        hd = ctypes.c_void_p()
        rc = lib.smg_create_hierarchy(ctypes.byref(desc), ctypes.byref(prm), ctypes.byref(hd))
        assert rc == want, (bc, rc)
        if rc == abi.SMG_OK:
            lib.smg_destroy_hierarchy(hd)
        else:
            assert "boundary" in lib.smg_last_error().decode()


def test_batch_run_argument_checks(lib):
    """smg_batch_run refuses a repeated hierarchy before any work, reports an unknown op and an
    unbound hierarchy per item (status), and returns the first failing item's code."""
    hs = []
    for dims in ((8, 8, 8), (16, 16, 8)):
        rc, hd = _create(lib, *dims, levels=2)
        abi.check(rc)
        hs.append(hd)
    try:
        items = (abi.BatchItem * 2)()
        for k in range(2):
            items[k].h = hs[0].value
            items[k].op = abi.SMG_OP_SAMPLE
        assert lib.smg_batch_run(items, 2, None) == abi.SMG_EINVAL
        assert b"once" in lib.smg_last_error()
        items[1].h = hs[1].value
        items[1].op = 7
        rc = lib.smg_batch_run(items, 2, None)
        assert items[0].status == abi.SMG_ESTATE and items[1].status == abi.SMG_EINVAL
        assert rc in (abi.SMG_ESTATE, abi.SMG_EINVAL)
        assert lib.smg_batch_run(items, 0, None) == abi.SMG_OK
    finally:
        for hd in hs:
            lib.smg_destroy_hierarchy(hd)


def test_unbound_hierarchy_refuses_work(lib):
    rc, hd = _create(lib, 8, 8, 8, levels=3)
    abi.check(rc)
    try:
        info = abi.SolveInfo()
        rc = lib.smg_solve(hd, ctypes.c_void_p(256), ctypes.c_void_p(512), 1e-8, 5, None,
                           ctypes.byref(info))
        assert rc == abi.SMG_ESTATE
        rc = lib.smg_sample_field(hd, 1, 0, 0, ctypes.c_void_p(256), ctypes.c_void_p(512), 0, None)
        assert rc == abi.SMG_ESTATE
    finally:
        lib.smg_destroy_hierarchy(hd)


def test_refined_precision_plan(lib):
    """SMG_FP32_REFINED needs a smoothed finest level; its plan has the FP64 plan's levels."""
    desc = abi.GridDesc(4, 4, 4, 1, 1.0, 1.0)  # one level, drawn exactly
    prm = abi.CycleParams(1, 2, 2, 512, 0, abi.SMG_FP32_REFINED, 1, 0)
    hd = ctypes.c_void_p()
    assert lib.smg_create_hierarchy(ctypes.byref(desc), ctypes.byref(prm),
                                    ctypes.byref(hd)) == abi.SMG_EINVAL
    assert "FP32" in lib.smg_last_error().decode()
    for dims in ((16, 16, 16), (128, 128, 128)):
        desc = abi.GridDesc(*dims, 3, 1.0, 1.0)
        infos = []
        for prec in (abi.SMG_FP64, abi.SMG_FP32_REFINED):
            prm = abi.CycleParams(0, 2, 2, 512, 0, prec, 1, 0)
            abi.check(lib.smg_create_hierarchy(ctypes.byref(desc), ctypes.byref(prm),
                                               ctypes.byref(hd)))
            infos.append(_info(lib, hd))
            lib.smg_destroy_hierarchy(hd)
        a, b = infos
        assert a.n_levels == b.n_levels and a.state_bytes == b.state_bytes
        assert [tuple(a.dims[l]) for l in range(a.n_levels)] == \
            [tuple(b.dims[l]) for l in range(b.n_levels)]
        assert b.workspace_bytes > 0


@pytest.mark.parametrize("dims,k", [((128, 128, 128), 8), ((16, 16, 8), 32), ((6, 4, 3), 20),
                                    ((256, 256, 64), 12), ((2, 2, 1), 4)])
def test_lowest_modes_match_oracle(lib, dims, k):
    from oracle.observables import lowest_modes
    arr = (ctypes.c_int32 * (3 * k))()
    abi.check(lib.smg_lowest_modes(*dims, k, arr))
    got = [(arr[3 * q], arr[3 * q + 1], arr[3 * q + 2]) for q in range(k)]
    assert got == lowest_modes(*dims, k)


def test_lowest_modes_invalid(lib):
    arr = (ctypes.c_int32 * 3)()
    for args in ((7, 8, 8, 1), (8, 8, 8, 33), (8, 8, 8, -1), (2, 2, 1, 5)):
        assert lib.smg_lowest_modes(*args, arr) == abi.SMG_EINVAL


def test_2d_plan_matches_oracle_levels(lib):
    """The 2D planner takes the oracle's level plan; invalid shapes are refused."""
    from oracle.mg2d import plan_levels
    for (nx, nz, levels, cmax) in ((64, 32, 0, 512), (48, 16, 0, 64), (16, 8, 3, 512),
                                   (12, 6, 0, 4096), (8, 5, 1, 512)):
        d = abi.Desc2D(nx, nz, 1, 1.0, 1.0, levels, 2, 2, cmax, 0, 1)
        hd = ctypes.c_void_p()
        abi.check(lib.smg2d_create(ctypes.byref(d), ctypes.byref(hd)))
        info = abi.Info2D()
        abi.check(lib.smg2d_get_info(hd, ctypes.byref(info)))
        got = [tuple(info.dims[l]) for l in range(info.n_levels)]
        lib.smg2d_destroy(hd)
        assert got == plan_levels(nx, nz, levels, cmax), (nx, nz, got)
    for bad in (abi.Desc2D(7, 8, 1, 1.0, 1.0, 0, 2, 2, 512, 0, 1),
                abi.Desc2D(8, 8, 0, 1.0, 1.0, 0, 2, 2, 512, 0, 1),
                abi.Desc2D(8, 8, 1, 1.0, 1.0, 0, 2, 2, 512, 0, 0),
                abi.Desc2D(12, 12, 1, 1.0, 1.0, 3, 2, 2, 512, 0, 1)):
        hd = ctypes.c_void_p()
        assert lib.smg2d_create(ctypes.byref(bad), ctypes.byref(hd)) == abi.SMG_EINVAL


def test_autotune_depth_candidates_cover_coarsest_sizes():
    """The tuner's depths come from the planner's automatic plans over a sweep of coarsest sizes
    (host planning only), so the exactly drawn coarsest level is tuned through the depth; plans
    that differ only in depth-independent parameters reuse the coarsest factors."""
    import time
    from paper_1003_2680_amd import autotune
    assert autotune.depth_candidates((32, 32, 32)) == [(3, 512), (4, 64), (5, 8)]
    assert autotune.depth_candidates((48, 48, 48), "fp32_refined") == [(3, 1728), (4, 216)]
    t = time.perf_counter()
    assert autotune.depth_candidates((48, 48, 48)) == [(3, 1728), (4, 216)]
    assert time.perf_counter() - t < 1.0   # the 1728-unknown factors come from the cache
