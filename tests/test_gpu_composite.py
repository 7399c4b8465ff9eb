"""GPU parity of the composite-grid FAC path (through the C-ABI) against the oracle.

Every piece is compared element by element with the oracle on the same seeded inputs and the
same counter-based noise: the composite residual, each of the twelve point classes of a
composite sweep, the block passes of the Galerkin base levels, whole stochastic and
deterministic FAC cycles, a sampling run and the solve.  Cases cover a box on the bottom wall,
an interior box with three base levels, a box on the periodic seam touching both walls
(ny = 12, not a power of two), and a small box in a larger base grid (short rows).  FP64 on both sides; the tolerance (1e-12 relative to the largest oracle value) covers
summation order only.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.composite import CompositeGrid, FACSampler, _KindMap
from oracle.philox import PhiloxNoise

pytestmark = pytest.mark.gpu

CASES = {
    "wall_box": (8, 8, 4, (2, 6, 2, 6, 0, 2), 64),
    "interior_3lev": (16, 16, 8, (4, 12, 3, 11, 1, 5), 64),
    "seam_walls": (16, 12, 8, (0, 6, 5, 12, 0, 8), 64),
    # small box in a larger base grid: most base rows are 7-point (one lane per row)
    "small_box_32": (32, 32, 16, (12, 20, 12, 20, 4, 8), 512),
}
TOL = 1e-12


@pytest.fixture(scope="module")
def setups():
    import torch
    from paper_1003_2680_amd.composite import CompositeSampler
    out = {}
    for name, (nx, ny, nz, box, cm) in CASES.items():
        g = CompositeGrid(nx, ny, nz, box)
        fac = FACSampler(g, kT=0.9, coarsest_max=cm)
        s = CompositeSampler(nx, ny, nz, box, kT=0.9, coarsest_max=cm)
        out[name] = (g, fac, s)
    yield out, torch


def _dev(torch, g, v):
    c, f = g.split(v)
    return (torch.tensor(np.ascontiguousarray(c), device="cuda"),
            torch.tensor(np.ascontiguousarray(f), device="cuda"))


def _host(g, c, f):
    return g.join(c.cpu().numpy(), f.cpu().numpy())


def _close(a, b, scale):
    err = np.abs(a - b).max()
    print("[composite parity] max |gpu - oracle| / max |oracle| = %.3e" % (err / scale),
          flush=True)
    assert err <= TOL * scale, err / scale


@pytest.mark.parametrize("name", list(CASES))
def test_residual(setups, name):
    st, torch = setups
    g, fac, s = st[name]
    rng = np.random.default_rng(11)
    x, b = rng.standard_normal(g.n), rng.standard_normal(g.n)
    xc, xf = _dev(torch, g, x)
    bc, bf = _dev(torch, g, b)
    rc, rf = s.residual(xc, xf, bc, bf)
    torch.cuda.synchronize()
    ref = b - g.A @ x
    _close(_host(g, rc, rf), ref, np.abs(ref).max())
    assert float(rc.reshape(-1)[g.covered].abs().max()) == 0.0


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("cls", range(12))
def test_class_pass(setups, name, cls):
    st, torch = setups
    g, fac, s = st[name]
    rng = np.random.default_rng(100 + cls)
    x, b = rng.standard_normal(g.n), rng.standard_normal(g.n)
    xc, xf = _dev(torch, g, x)
    bc, bf = _dev(torch, g, b)
    s.debug_pass(cls, xc, xf, bc, bf, seed=77, cycle=5, slot=1, noise=True)
    torch.cuda.synchronize()
    ref = x.copy()
    fac.class_pass(ref, b, cls, 1, PhiloxNoise(77), 5)
    _close(_host(g, xc, xf), ref, np.abs(ref).max())


@pytest.mark.parametrize("name", list(CASES))
def test_base_block_passes(setups, name):
    st, torch = setups
    g, fac, s = st[name]
    for l, L in enumerate(fac.base.levels[:-1]):
        for colour in range(8):
            rng = np.random.default_rng(1000 + 10 * l + colour)
            x, b = rng.standard_normal(L.n), rng.standard_normal(L.n)
            xd = torch.tensor(x, device="cuda")
            bd = torch.tensor(b, device="cuda")
            s.debug_base_pass(l, colour, xd, bd, seed=5, cycle=3, slot=2, noise=True)
            torch.cuda.synchronize()
            ref = x.copy()
            fac.base._block_pass(L, ref, b, colour, _KindMap(PhiloxNoise(5)), (3, 2, 0))
            _close(xd.cpu().numpy(), ref, np.abs(ref).max())


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("lanes", [2, 8])
def test_row_lanes_fixed(setups, name, lanes):
    """The long-row block passes and residuals with a fixed lane count per row (a large launch
    takes two lanes, a small one eight): every block pass of every base level, then three
    stochastic cycles with a right-hand side (the base residuals), against the oracle."""
    from paper_1003_2680_amd.composite import CompositeSampler
    st, torch = setups
    g, fac, _ = st[name]
    nx, ny, nz, box, cm = CASES[name]
    print("[gpu-case] composite %s row_lanes=%d" % (name, lanes), flush=True)
    s = CompositeSampler(nx, ny, nz, box, kT=0.9, coarsest_max=cm, row_lanes=lanes)
    for l, L in enumerate(fac.base.levels[:-1]):
        for colour in range(8):
            rng = np.random.default_rng(2000 + 10 * l + colour)
            x, b = rng.standard_normal(L.n), rng.standard_normal(L.n)
            xd = torch.tensor(x, device="cuda")
            bd = torch.tensor(b, device="cuda")
            s.debug_base_pass(l, colour, xd, bd, seed=6, cycle=4, slot=1, noise=True)
            torch.cuda.synchronize()
            ref = x.copy()
            fac.base._block_pass(L, ref, b, colour, _KindMap(PhiloxNoise(6)), (4, 1, 0))
            _close(xd.cpu().numpy(), ref, np.abs(ref).max())
    rng = np.random.default_rng(8)
    x, b = rng.standard_normal(g.n), rng.standard_normal(g.n)
    xc, xf = _dev(torch, g, x)
    bc, bf = _dev(torch, g, b)
    ref = x.copy()
    for cyc in range(3):
        s.cycle(xc, xf, bc, bf, seed=31, cycle=cyc, noise=True)
        ref = fac.cycle(ref, b, PhiloxNoise(31), cyc)
    torch.cuda.synchronize()
    _close(_host(g, xc, xf), ref, np.abs(ref).max())
    s.close()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("with_b", [False, True])
def test_stochastic_cycles(setups, name, with_b):
    st, torch = setups
    g, fac, s = st[name]
    rng = np.random.default_rng(7)
    x = rng.standard_normal(g.n)
    b = rng.standard_normal(g.n) if with_b else np.zeros(g.n)
    xc, xf = _dev(torch, g, x)
    bc, bf = _dev(torch, g, b) if with_b else (None, None)
    ref = x.copy()
    for cyc in range(3):
        s.cycle(xc, xf, bc, bf, seed=2024, cycle=10 + cyc, noise=True)
        ref = fac.cycle(ref, b, PhiloxNoise(2024), 10 + cyc)
    torch.cuda.synchronize()
    _close(_host(g, xc, xf), ref, np.abs(ref).max())


@pytest.mark.parametrize("name", list(CASES))
def test_sample_equals_cycles(setups, name):
    st, torch = setups
    g, fac, s = st[name]
    x0 = np.random.default_rng(3).standard_normal(g.n)
    ac, af = _dev(torch, g, x0)
    bc_, bf_ = _dev(torch, g, x0)
    s.sample(ac, af, 4, seed=99, first_cycle=7)
    for k in range(4):
        s.cycle(bc_, bf_, seed=99, cycle=7 + k, noise=True)
    torch.cuda.synchronize()
    assert np.array_equal(_host(g, ac, af), _host(g, bc_, bf_))


@pytest.mark.parametrize("name", list(CASES))
def test_solve(setups, name):
    st, torch = setups
    g, fac, s = st[name]
    f = np.random.default_rng(21).standard_normal(g.n)
    fc, ff = _dev(torch, g, f)
    uc, uf, info = s.solve(fc, ff, rtol=1e-11, max_cycles=40)
    ref = spla.spsolve(g.A.tocsc(), f)
    assert info.relres <= 1e-11 and info.cycles <= 16
    u = _host(g, uc, uf)
    assert np.abs(u - ref).max() <= 1e-9 * np.abs(ref).max()
    # the deterministic cycle is the oracle's cycle: the same iterate after two cycles
    xc, xf = s.zeros()
    for _ in range(2):
        s.cycle(xc, xf, fc, ff, noise=False)
    ref2 = np.zeros(g.n)
    for _ in range(2):
        ref2 = fac.cycle(ref2, f)
    torch.cuda.synchronize()
    _close(_host(g, xc, xf), ref2, np.abs(ref2).max())


def test_wide_levels_two_lanes_agree_with_eight():
    """A base grid 256 cells wide, so that its Galerkin levels hold whole waves of cells away
    from the periodic seams with one shared row (the residual then reads the row's records as
    wave-uniform values): three stochastic cycles with a right-hand side with two lanes per
    long row against eight lanes per long row (the form the oracle parity above pins), equal up
    to summation order."""
    import torch
    from paper_1003_2680_amd.composite import CompositeSampler
    base, box = (256, 256, 8), (100, 140, 96, 136, 0, 4)
    print("[gpu-case] composite wide levels %s box %s" % (base, box), flush=True)
    res = []
    for lanes in (2, 8):
        s = CompositeSampler(*base, box, kT=0.9, coarsest_max=512, row_lanes=lanes)
        assert s.info.n_levels >= 3 and s.info.dims[1][0] == 128
        rng = np.random.default_rng(12)
        xc = torch.tensor(rng.standard_normal(s.base_shape), device="cuda")
        xf = torch.tensor(rng.standard_normal(s.fine_shape), device="cuda")
        bc = torch.tensor(rng.standard_normal(s.base_shape), device="cuda")
        bf = torch.tensor(rng.standard_normal(s.fine_shape), device="cuda")
        for cyc in range(3):
            s.cycle(xc, xf, bc, bf, seed=17, cycle=cyc, noise=True)
        torch.cuda.synchronize()
        cov = torch.zeros(s.base_shape, dtype=torch.bool, device="cuda")
        cov[box[4]:box[5], box[2]:box[3], box[0]:box[1]] = True
        res.append((xc.masked_fill(cov, 0).cpu().numpy(), xf.cpu().numpy()))
        s.close()
    for a, b in zip(*res):
        assert np.isfinite(a).all()
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
