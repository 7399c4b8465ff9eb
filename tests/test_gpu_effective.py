"""GPU parity of the composite-mesh field noise w = L^-1 Q eta (Appendix A; C-ABI
smg_composite_forced_field) against the oracle.

* Per draw, on the same Philox eta: the GPU field (a FAC solve of A w = -(volume/h^3) q eta to
  rtol 1e-12) against the oracle's sparse solve with L = M^-1 S itself.  Bar: max |gpu - oracle|
  <= 1e-9 max |oracle| (the solve tolerance times the condition number of these small grids, with
  margin).  Cases: a wall box with random amplitudes, the 16^3-base copy of the adaptive
  workload (box [4, 12)^2 x [0, 4), 5888 unknowns) with uniform q, and the FP32-refined form.
* Covered base cells of the output are exactly 0.
* Statistics: the variance of three fixed projections over 1500 draws matches the oracle's dense
  L^-1 Q Q^T L^-T within 5 standard errors, for a uniform q (a non-symmetric L^-1 C).
* Argument errors are reported (negative n, a misaligned output).
"""
import ctypes

import numpy as np
import pytest

from oracle import effective as eff
from oracle.composite import CompositeGrid

pytestmark = pytest.mark.gpu

CASES = {
    "wall_box_random_q": (8, 8, 4, (2, 6, 2, 6, 0, 2), "random", "fp64"),
    "base16_uniform_q": (16, 16, 16, (4, 12, 4, 12, 0, 4), "ones", "fp64"),
    "wall_box_refined": (8, 8, 4, (2, 6, 2, 6, 0, 2), "random", "fp32_refined"),
}
TOL = 1e-9


def _amplitudes(g, kind, seed=3):
    if kind == "ones":
        return None, None
    rng = np.random.default_rng(seed)
    return (rng.uniform(0.5, 1.5, (g.nz, g.ny, g.nx)),
            rng.uniform(0.5, 1.5, (g.fz, g.fy, g.fx)))


@pytest.mark.parametrize("name", list(CASES))
def test_forced_field_parity(name):
    import torch
    from paper_1003_2680_amd.composite import CompositeSampler
    nx, ny, nz, box, qkind, prec = CASES[name]
    print("[forced field] case %s" % name, flush=True)
    g = CompositeGrid(nx, ny, nz, box)
    s = CompositeSampler(nx, ny, nz, box, precision=prec)
    qc, qf = _amplitudes(g, qkind)
    qc_d = torch.tensor(qc, device="cuda") if qc is not None else None
    qf_d = torch.tensor(qf, device="cuda") if qf is not None else None
    seed, first, n = 9, 5, 3
    wc, wf, infos = s.forced_field(n, seed, first, qc_d, qf_d, rtol=1e-12, max_cycles=60)
    wc, wf = wc.cpu().numpy(), wf.cpu().numpy()
    covered = np.ones(g.nbase, dtype=bool)
    covered[g.coarse_cells] = False
    qch = qc if qc is not None else np.ones((nz, ny, nx))
    qfh = qf if qf is not None else np.ones((g.fz, g.fy, g.fx))
    for i in range(n):
        ec, ef = eff.forcing_noise(seed, first + i, g.nbase, g.nf)
        oc, of = eff.forced_field(g, qch.ravel(), qfh.ravel(), ec, ef)
        ref = g.join(oc, of)
        got = g.join(wc[i], wf[i])
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print("[forced field] %s draw %d: cycles %d, max |gpu - oracle| / max |oracle| = %.3e"
              % (name, i, infos[i].cycles, err), flush=True)
        assert err <= TOL
        assert np.all(wc[i].ravel()[covered] == 0.0)
    s.close()


def test_forced_field_covariance_monte_carlo():
    import torch
    from paper_1003_2680_amd.composite import CompositeSampler
    nx, ny, nz, box = 4, 4, 2, (1, 3, 1, 3, 0, 1)
    g = CompositeGrid(nx, ny, nz, box)
    s = CompositeSampler(nx, ny, nz, box)
    n = 1500
    wc, wf, _ = s.forced_field(n, 21, 0, rtol=1e-11, max_cycles=60)
    W = eff.forced_covariance(g, np.ones(g.n))
    rng = np.random.default_rng(8)
    P = rng.standard_normal((3, g.n))
    wc, wf = wc.cpu().numpy(), wf.cpu().numpy()
    proj = np.array([P @ g.join(wc[i], wf[i]) for i in range(n)])
    var = np.einsum("ij,jk,ik->i", P, W, P)
    emp = (proj ** 2).mean(axis=0)
    print("[forced field] Monte Carlo variances", emp, "exact", var, flush=True)
    assert np.all(np.abs(emp - var) <= 5.0 * var * np.sqrt(2.0 / n))
    s.close()


def test_forced_field_argument_errors():
    import torch
    from paper_1003_2680_amd import abi
    from paper_1003_2680_amd.composite import CompositeSampler
    s = CompositeSampler(8, 8, 4, (2, 6, 2, 6, 0, 2))
    lib = s.lib
    wc = torch.zeros(1024, dtype=torch.float64, device="cuda")
    wf = torch.zeros(1024, dtype=torch.float64, device="cuda")
    P = lambda t, off=0: ctypes.c_void_p(t.data_ptr() + off)
    rc = lib.smg_composite_forced_field(s._h, -1, 0, 0, None, None, P(wc), P(wf), 1e-10, 10,
                                        s._stream(), None)
    assert rc == abi.SMG_EINVAL
    rc = lib.smg_composite_forced_field(s._h, 1, 0, 0, None, None, P(wc, 8), P(wf), 1e-10, 10,
                                        s._stream(), None)
    assert rc == abi.SMG_EINVAL
    # n = 0 is a no-op
    rc = lib.smg_composite_forced_field(s._h, 0, 0, 0, None, None, None, None, 1e-10, 10,
                                        s._stream(), None)
    assert rc == abi.SMG_OK
    s.close()
