"""The adaptive workload at full size and the covariance of its 16^3-base copy (GPU).

Full size (256x256x128 base, box [64,192)^2 x [0,32) refined by two, 12.06 M unknowns): the
plan's sizes; the GPU residual at sampled cells (interface cells on every box face, edges,
corners, the bottom wall, the periodic seam and random cells) against the oracle's per-cell
rows evaluated from the face rules; the deterministic solve; and equipartition of a sample,
x^T A x / (n kT) = 1 within five standard deviations sqrt(2/n) of the chi-square law.

16^3-base copy (box [4,12)^2 x [0,4), 5888 unknowns): chain covariance against the dense
target kT A^-1 of the oracle's operator -- variances of fixed probe vectors and of every
unknown -- within Monte Carlo error (batch-means estimate of the error of each variance).
"""
import numpy as np
import pytest

from oracle.composite import CompositeGrid, row_of

pytestmark = pytest.mark.gpu

BASE = (256, 256, 128)
BOX = (64, 192, 64, 192, 0, 32)


def _sample_cells(rng):
    nx, ny, nz = BASE
    x0, x1, y0, y1, z0, z1 = BOX
    fx, fy, fz = 2 * (x1 - x0), 2 * (y1 - y0), 2 * (z1 - z0)
    coarse = [(x0 - 1, 100, 10), (x1, 70, 31), (100, y0 - 1, 0), (150, y1, 20), (80, 90, z1),
              (x0 - 1, y0 - 1, z1), (x1, y1, z1), (0, 0, 0), (nx - 1, ny - 1, nz - 1),
              (x0 - 2, 128, 5), (128, 128, z1 + 1)]
    fine = [(0, 5, 3), (fx - 1, 17, 40), (9, 0, 63), (33, fy - 1, 0), (50, 60, fz - 1),
            (0, 0, fz - 1), (fx - 1, fy - 1, 0), (1, 1, 1), (128, 128, 32)]
    cidx = [x + nx * (y + ny * z) for x, y, z in coarse]
    fidx = [i + fx * (j + fy * k) for i, j, k in fine]
    for _ in range(120):
        x, y, z = rng.integers(0, nx), rng.integers(0, ny), rng.integers(0, nz)
        if not (x0 <= x < x1 and y0 <= y < y1 and z0 <= z < z1):
            cidx.append(int(x + nx * (y + ny * z)))
        fidx.append(int(rng.integers(0, fx * fy * fz)))
    return cidx, fidx


def test_full_size_residual_solve_equipartition():
    import torch
    from paper_1003_2680_amd.composite import CompositeSampler
    nx, ny, nz = BASE
    S = CompositeSampler(nx, ny, nz, BOX, kT=1.0)
    assert S.info.unknowns == 12058624
    rng = np.random.default_rng(4)
    xc = rng.standard_normal((nz, ny, nx))
    xf = rng.standard_normal(S.fine_shape)
    bc = rng.standard_normal((nz, ny, nx))
    bf = rng.standard_normal(S.fine_shape)
    d = lambda a: torch.tensor(a, device="cuda")
    rc, rf = S.residual(d(xc), d(xf), d(bc), d(bf))
    rc, rf = rc.cpu().numpy().ravel(), rf.cpu().numpy().ravel()
    xcf, xff, bcf, bff = xc.ravel(), xf.ravel(), bc.ravel(), bf.ravel()
    cidx, fidx = _sample_cells(rng)
    for kind, idxs, bvec, got in (("c", cidx, bcf, rc), ("f", fidx, bff, rf)):
        for q in idxs:
            row = row_of(nx, ny, nz, BOX, 1.0, kind, q)
            ax = sum(v * (xcf[t] if k == "c" else xff[t]) for (k, t), v in row.items())
            ref = bvec[q] - ax
            assert abs(got[q] - ref) <= 1e-12 * max(1.0, abs(ref)), (kind, q)
    # solve
    fc = d(rng.standard_normal((nz, ny, nx)))
    ff = d(rng.standard_normal(S.fine_shape))
    uc, uf, info = S.solve(fc, ff, rtol=1e-10, max_cycles=40)
    assert info.relres <= 1e-10 and info.cycles <= 16 and info.last_ratio < 0.3
    # equipartition of a sample after 12 cycles from zero
    zc, zf = S.zeros()
    S.sample(zc, zf, 12, seed=3)
    r1, r2 = S.residual(zc, zf)
    e = -(zc.reshape(-1) @ r1.reshape(-1) + zf.reshape(-1) @ r2.reshape(-1)).item()
    n = S.info.unknowns
    assert abs(e / n - 1.0) < 5.0 * np.sqrt(2.0 / n)


def test_copy_covariance_against_dense_target():
    import torch
    from paper_1003_2680_amd.composite import CompositeSampler
    kT = 1.0
    base, box = (16, 16, 16), (4, 12, 4, 12, 0, 4)
    g = CompositeGrid(*base, box)
    assert g.n == 5888
    C = kT * np.linalg.inv(g.A.toarray())
    S = CompositeSampler(*base, box, kT=kT)
    # composite ordering on the device: coarse cells (uncovered base cells), then fine cells
    cc = torch.tensor(g.coarse_cells, device="cuda")
    xc, xf = S.zeros()
    S.sample(xc, xf, 20, seed=11)
    N = 6000
    X = torch.empty((N, g.n), dtype=torch.float64, device="cuda")
    for i in range(N):
        S.sample(xc, xf, 1, seed=11, first_cycle=20 + i)
        X[i, :g.nc] = xc.reshape(-1)[cc]
        X[i, g.nc:] = xf.reshape(-1)
    Xh = X.cpu().numpy()
    rng = np.random.default_rng(8)
    probes = [rng.standard_normal(g.n) for _ in range(12)]
    for c in (g.nc // 3, g.nc + 5, g.nc + 1234, g.n - 1):   # single cells incl. the interface
        e = np.zeros(g.n)
        e[c] = 1.0
        probes.append(e)
    nb = 30                                                # batch means over N/nb samples
    for phi in probes:
        y = Xh @ phi
        true = phi @ C @ phi
        sq = (y * y).reshape(nb, -1).mean(axis=1)
        est, se = sq.mean(), sq.std(ddof=1) / np.sqrt(nb)
        assert abs(est - true) < 5.0 * se, (est, true, se)
        assert abs(est / true - 1.0) < 0.1
    var = (Xh * Xh).mean(axis=0)
    ratio = var / np.diag(C)
    assert abs(ratio.mean() - 1.0) < 0.01
    assert np.abs(ratio - 1.0).max() < 0.15
