"""FP32-refined form of the composite FAC cycle (GPU): FP32 sweeps and transfers in the
correction form, FP64 residual, update and coarsest draw, on the same noise streams as the
FP64 form.  Bars: relative RMS against the FP64 GPU form <= 1e-5 and against the oracle
<= 1e-4 after three stochastic cycles (with and without a right-hand side); the refined solve
reaches 1e-10 in FP64 residual; the component entry points refuse the refined form."""
import numpy as np
import pytest

from oracle.composite import CompositeGrid, FACSampler
from oracle.philox import PhiloxNoise

pytestmark = pytest.mark.gpu

CASES = {
    "wall_box": (8, 8, 4, (2, 6, 2, 6, 0, 2), 64),
    "interior_3lev": (16, 16, 8, (4, 12, 3, 11, 1, 5), 64),
    "small_box_32": (32, 32, 16, (12, 20, 12, 20, 4, 8), 512),
}


def _rel_rms(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2)) / np.sqrt(np.mean(b ** 2)))


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("with_b", [False, True])
def test_refined_cycles_track_fp64(name, with_b):
    import torch
    from paper_1003_2680_amd.composite import CompositeSampler
    nx, ny, nz, box, cm = CASES[name]
    print("[gpu-case] refined composite %s with_b=%s" % (name, with_b), flush=True)
    g = CompositeGrid(nx, ny, nz, box)
    fac = FACSampler(g, kT=0.8, coarsest_max=cm)
    s64 = CompositeSampler(nx, ny, nz, box, kT=0.8, coarsest_max=cm)
    s32 = CompositeSampler(nx, ny, nz, box, kT=0.8, coarsest_max=cm, precision="fp32_refined")
    rng = np.random.default_rng(17)
    x = rng.standard_normal(g.n)
    b = rng.standard_normal(g.n) if with_b else np.zeros(g.n)

    def dev(v):
        c, f = g.split(v)
        return (torch.tensor(np.ascontiguousarray(c), device="cuda"),
                torch.tensor(np.ascontiguousarray(f), device="cuda"))

    a64, a32 = dev(x), dev(x)
    bb = dev(b) if with_b else (None, None)
    ref = x.copy()
    for cyc in range(3):
        s64.cycle(*a64, *bb, seed=9, cycle=cyc, noise=True)
        s32.cycle(*a32, *bb, seed=9, cycle=cyc, noise=True)
        ref = fac.cycle(ref, b, PhiloxNoise(9), cyc)
    torch.cuda.synchronize()
    v64 = g.join(a64[0].cpu().numpy(), a64[1].cpu().numpy())
    v32 = g.join(a32[0].cpu().numpy(), a32[1].cpu().numpy())
    assert _rel_rms(v32, v64) <= 1e-5
    assert _rel_rms(v32, ref) <= 1e-4


def test_refined_solve_and_entry_point_guard():
    import torch
    from paper_1003_2680_amd import abi
    from paper_1003_2680_amd.composite import CompositeSampler
    nx, ny, nz, box, cm = CASES["interior_3lev"]
    s32 = CompositeSampler(nx, ny, nz, box, coarsest_max=cm, precision="fp32_refined")
    g = CompositeGrid(nx, ny, nz, box)
    f = np.random.default_rng(2).standard_normal(g.n)
    c, fi = g.split(f)
    fc = torch.tensor(np.ascontiguousarray(c), device="cuda")
    ff = torch.tensor(np.ascontiguousarray(fi), device="cuda")
    uc, uf, info = s32.solve(fc, ff, rtol=1e-10, max_cycles=40)
    assert info.relres <= 1e-10 and info.cycles <= 25
    xc, xf = s32.zeros()
    with pytest.raises(abi.SMGError):
        s32.debug_pass(0, xc, xf)
