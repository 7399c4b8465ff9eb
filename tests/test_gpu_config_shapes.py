"""GPU parity at the shapes of the batched, served and single-grid workloads.

* Batched workload: its tuned configurations (48^3 with 4 levels, 96^3 with 5 levels, V(2,2))
  run through the library's batch call (smg_batch_run, the instances' small levels in one merged
  launch): two stochastic cycles of each instance from the zero start against the oracle on the
  same Philox streams, FP64 (every value, 1e-12 relative to the largest) and FP32-refined
  (1e-4 relative RMS).
* Served workload: the automatic-depth shapes 256x256x16 (coarsest level 16x16x1) and 32x32x128,
  the same bars, and a solve to 1e-10 whose residual is recomputed with the oracle's stencil.
* Single 512x512x256 grid (67 M cells, too large for the oracle to assemble): one level-0 colour
  pass of each colour, the fused residual restriction and the prolongation at sampled cells
  (both walls, the periodic seams, random cells) against the oracle's cell-by-cell evaluators
  (1e-12 relative to the largest sampled value); a solve to 1e-10 with its residual recomputed by
  the oracle's stencil over the whole grid; equipartition x^T A x / (N kT) = 1 within 5 sqrt(2/N)
  after three cycles of the chain (every mode carries kT/2 at stationarity).
"""
import numpy as np
import pytest

from oracle.mg import StochasticMG
from oracle.operator import apply_A
from oracle.philox import PhiloxNoise
from oracle import sampled

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _announce(msg):
    print("[gpu-case] " + msg, flush=True)


def _oracle_cycles(dims, levels, seed, ncyc, coarsest_max=512):
    mg = StochasticMG(*dims, kT=1.0, levels=levels, coarsest_max=coarsest_max)
    zero = np.zeros(mg.levels[0].n)
    x = zero.copy()
    out = []
    for c in range(ncyc):
        x = mg.vcycle(x, zero, PhiloxNoise(seed), c, 0)
        out.append(x.copy())
    return mg, out


def _compare(got, ref, precision, what):
    for c, (g, r) in enumerate(zip(got, ref)):
        if precision == "fp64":
            err = np.max(np.abs(g - r)) / np.max(np.abs(r))
            print("  %s cycle %d max rel %.2e" % (what, c, err), flush=True)
            assert err <= 1e-12, (what, c, err)
        else:
            err = np.linalg.norm(g - r) / np.linalg.norm(r)
            print("  %s cycle %d rel RMS %.2e" % (what, c, err), flush=True)
            assert err <= 1e-4, (what, c, err)


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_batched_tuned_configs_against_oracle(precision):
    from paper_1003_2680_amd.api import Hierarchy, batch_run
    _announce("batched tuned configs 48^3 L4, 96^3 L5 %s" % precision)
    cases = [((48, 48, 48), 4, 1001), ((96, 96, 96), 5, 1002)]
    items = []
    for dims, levels, seed in cases:
        H = Hierarchy(*dims, ncomp=1, levels=levels, precision=precision)
        st = torch.zeros(H.shape, dtype=torch.float64, device="cuda")
        out = torch.empty((2,) + H.shape, dtype=torch.float64, device="cuda")
        items.append({"H": H, "op": "sample", "nchains": 1, "comps_per_chain": 1, "n": 2,
                      "seeds": [seed], "first_cycles": [0], "state": st, "out": out})
    res = batch_run(items)
    torch.cuda.synchronize()
    assert all(s == 0 for s, _ in res)
    for (dims, levels, seed), it in zip(cases, items):
        _, ref = _oracle_cycles(dims, levels, seed, 2)
        got = it["out"].cpu().numpy().reshape(2, -1)
        _compare(got, ref, precision, "%s L%d" % (dims, levels))


@pytest.mark.parametrize("dims", [(256, 256, 16), (32, 32, 128)])
@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_served_shapes_against_oracle(dims, precision):
    from paper_1003_2680_amd.api import Hierarchy
    from paper_1003_2680_amd.inputs import gaussian_field
    _announce("served shape %s auto depth %s" % (dims, precision))
    H = Hierarchy(*dims, ncomp=1, levels=0, coarsest_max=512, precision=precision)
    mg, ref = _oracle_cycles(dims, 0, 777, 2)
    assert [tuple(d) for d in H.level_dims] == [L.dims for L in mg.levels]
    out, _ = H.sample(2, 777)
    torch.cuda.synchronize()
    _compare(out.cpu().numpy().reshape(2, -1), ref, precision, str(dims))
    f = gaussian_field(H.shape, 31)
    u, cycles, relres = H.solve(torch.from_numpy(f).cuda(), rtol=1e-10)
    torch.cuda.synchronize()
    r = f[0].ravel() - apply_A(u.cpu().numpy()[0], *dims)
    assert relres <= 1e-10 and np.linalg.norm(r) / np.linalg.norm(f) <= 1.01e-10
    assert cycles <= 16


BIG = (512, 512, 256)


@pytest.fixture(scope="module")
def big():
    from paper_1003_2680_amd.api import Hierarchy
    H = Hierarchy(*BIG, ncomp=1, levels=0, coarsest_max=512)
    x = np.random.default_rng(12).standard_normal((1,) + BIG[::-1])
    return H, x


@pytest.mark.parametrize("colour", [0, 1])
def test_big_colour_pass_at_sampled_cells(big, colour):
    H, x = big
    _announce("512x512x256 colour pass %d at sampled cells" % colour)
    xd = torch.from_numpy(x).cuda()
    H.debug_smooth(0, colour, xd, seed=41, cycle=9, slot=3)
    got = xd.cpu().numpy()[0].ravel()
    nx, ny, nz = BIG
    cells = sampled.sample_cells(nx, ny, nz, 3000, 2, colour=colour)
    ref = sampled.heat_bath_at(x[0], None, cells, colour, seed=41, cycle=9, slot=3)
    err = np.max(np.abs(got[cells] - ref)) / np.max(np.abs(ref))
    print("  max rel %.2e over %d cells" % (err, len(cells)), flush=True)
    assert err <= 1e-12
    # the other colour is untouched, everywhere
    z, y, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    other = ((xx + y + z) % 2 != colour).ravel()
    assert np.array_equal(got[other], x[0].ravel()[other])


def test_big_transfers_at_sampled_cells(big):
    H, x = big
    _announce("512x512x256 fused restriction and prolongation at sampled cells")
    nx, ny, nz = BIG
    b = np.random.default_rng(13).standard_normal((1,) + BIG[::-1])
    bc = torch.empty((1, nz // 2, ny // 2, nx // 2), dtype=torch.float64, device="cuda")
    H.debug_restrict_residual(0, torch.from_numpy(x).cuda(), torch.from_numpy(b).cuda(), bc)
    got = bc.cpu().numpy()[0].ravel()
    cc = sampled.sample_cells(nx // 2, ny // 2, nz // 2, 400, 3)
    ref = sampled.restrict_residual_at(x[0], b[0], cc)
    err = np.max(np.abs(got[cc] - ref)) / np.max(np.abs(ref))
    print("  restriction max rel %.2e over %d coarse cells" % (err, len(cc)), flush=True)
    assert err <= 1e-12
    e = np.random.default_rng(14).standard_normal((1, nz // 2, ny // 2, nx // 2))
    xd = torch.from_numpy(x).cuda()
    H.debug_prolong_add(0, xd, torch.from_numpy(e).cuda())
    got = xd.cpu().numpy()[0].ravel()
    fc = sampled.sample_cells(nx, ny, nz, 3000, 4)
    ref = x[0].ravel()[fc] + sampled.prolong_at(e[0], BIG, fc)
    err = np.max(np.abs(got[fc] - ref)) / np.max(np.abs(ref))
    print("  prolongation max rel %.2e over %d cells" % (err, len(fc)), flush=True)
    assert err <= 1e-12


def test_big_solve_and_equipartition(big):
    H, _ = big
    _announce("512x512x256 solve and equipartition")
    from paper_1003_2680_amd.inputs import gaussian_field
    f = gaussian_field(H.shape, 15)
    u, cycles, relres = H.solve(torch.from_numpy(f).cuda(), rtol=1e-10)
    torch.cuda.synchronize()
    r = f[0].ravel() - apply_A(u.cpu().numpy()[0], *BIG)
    rel = np.linalg.norm(r) / np.linalg.norm(f)
    print("  solve %d cycles relres %.2e (oracle stencil %.2e)" % (cycles, relres, rel),
          flush=True)
    assert relres <= 1e-10 and rel <= 1.01e-10 and cycles <= 16
    out, _ = H.sample(3, 5)
    torch.cuda.synchronize()
    xs = out[-1, 0].cpu().numpy()
    n = xs.size
    ratio = float(np.dot(xs.ravel(), apply_A(xs, *BIG))) / n
    print("  x^T A x / (N kT) = %.6f (bound %.2e)" % (ratio, 5 * np.sqrt(2.0 / n)), flush=True)
    assert abs(ratio - 1.0) <= 5 * np.sqrt(2.0 / n)
