"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle on identical inputs and
identical Philox streams.

Bar (FP64): max |gpu - oracle| <= 1e-12 * max |oracle| for every compared field -- the
paths differ only in the order of floating-point operations and in the last ulp of the
transcendental functions of Box-Muller.
"""
import numpy as np
import pytest

from oracle.mg import StochasticMG
from oracle.philox import PhiloxNoise
from oracle import spectral
from paper_1003_2680_amd.inputs import gaussian_field, uniform_field

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = 1e-12


def _hier(*args, **kw):
    from paper_1003_2680_amd.api import Hierarchy
    return Hierarchy(*args, **kw)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _relerr(g, o):
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    scale = max(np.max(np.abs(o)), 1e-300)
    return np.max(np.abs(g - o)) / scale


def _announce(msg):
    print("[gpu-case] " + msg, flush=True)


# ----------------------------------------------------------------------------- components
# (10,6,5), (2,4,3): odd colour rows, the generic form; every other case one 16-byte vector per
# thread: (12,8,6), (16,8,6) waves across planes, (24,6,5) row and plane counts not powers of
# two, (4,2,1), (8,4,1) both walls on one plane, (32,32,4) and (64,16,9) every wave in one
# plane, the latter with a ragged last work-group
@pytest.mark.parametrize("dims,ncomp", [((12, 8, 6), 2), ((10, 6, 5), 1), ((4, 2, 1), 1),
                                        ((2, 4, 3), 3), ((16, 8, 6), 2), ((24, 6, 5), 2),
                                        ((8, 4, 1), 1), ((32, 32, 4), 1), ((64, 16, 9), 3)])
@pytest.mark.parametrize("with_b", [False, True])
def test_point_pass(dims, ncomp, with_b):
    _announce("point pass %s ncomp=%d b=%s" % (dims, ncomp, with_b))
    kT = 1.7
    H = _hier(*dims, ncomp=ncomp, kT=kT, levels=1, coarsest="smooth")
    mg = StochasticMG(*dims, kT=kT, levels=1, coarsest="smooth")
    L = mg.levels[0]
    N = L.n
    x0 = uniform_field((ncomp, N), 5)
    b = gaussian_field((ncomp, N), 6) if with_b else np.zeros((ncomp, N))
    seed, cycle, slot = 123456789012345, 77, 3
    for colour in (0, 1):
        xg = _dev(x0.reshape(H.shape))
        H.debug_smooth(0, colour, xg, _dev(b.reshape(H.shape)) if with_b else None,
                       seed=seed, cycle=cycle, slot=slot)
        got = _host(xg).reshape(ncomp, N)
        for c in range(ncomp):
            xo = x0[c].copy()
            mg._point_pass(L, xo, b[c], colour, PhiloxNoise(seed), (cycle, slot, c))
            assert _relerr(got[c], xo) <= RTOL


@pytest.mark.parametrize("dims,levels,level", [((16, 16, 12), 3, 1), ((16, 16, 8), 4, 2),
                                               ((32, 16, 8), 4, 1), ((32, 32, 16), 4, 2)])
@pytest.mark.parametrize("noise", [True, False])
def test_block_pass(dims, levels, level, noise):
    _announce("block pass %s L=%d l=%d noise=%s" % (dims, levels, level, noise))
    kT = 0.8
    ncomp = 2
    H = _hier(*dims, ncomp=ncomp, kT=kT, levels=levels)
    mg = StochasticMG(*dims, kT=kT, levels=levels)
    L = mg.levels[level]
    assert L.kind == "block"
    x0 = uniform_field((ncomp, L.n), 7)
    b = gaussian_field((ncomp, L.n), 8)
    shape = (ncomp,) + tuple(reversed(L.dims))
    seed, cycle, slot = 99, 5, 2
    for colour in (0, 3, 6, 7):
        xg = _dev(x0.reshape(shape))
        H.debug_smooth(level, colour, xg, _dev(b.reshape(shape)), seed=seed, cycle=cycle,
                       slot=slot, noise=noise)
        got = _host(xg).reshape(ncomp, L.n)
        for c in range(ncomp):
            xo = x0[c].copy()
            mg._block_pass(L, xo, b[c], colour, PhiloxNoise(seed) if noise else None,
                           (cycle, slot, c))
            assert _relerr(got[c], xo) <= RTOL


@pytest.mark.parametrize("dims,levels", [((16, 16, 12), 3), ((16, 16, 8), 4), ((12, 8, 6), 2),
                                         ((24, 12, 10), 2)])
def test_transfers(dims, levels):
    _announce("transfers %s L=%d" % (dims, levels))
    ncomp = 2
    H = _hier(*dims, ncomp=ncomp, levels=levels)
    mg = StochasticMG(*dims, levels=levels)
    for l in range(len(mg.levels) - 1):
        L, C = mg.levels[l], mg.levels[l + 1]
        shape = (ncomp,) + tuple(reversed(L.dims))
        cshape = (ncomp,) + tuple(reversed(C.dims))
        x = uniform_field((ncomp, L.n), 10 + l)
        b = gaussian_field((ncomp, L.n), 20 + l)
        e = gaussian_field((ncomp, C.n), 30 + l)
        for use_b in ([False, True] if l == 0 else [True]):
            bc = torch.zeros(cshape, dtype=torch.float64, device="cuda")
            H.debug_restrict_residual(l, _dev(x.reshape(shape)),
                                      _dev(b.reshape(shape)) if use_b else None, bc)
            got = _host(bc).reshape(ncomp, C.n)
            for c in range(ncomp):
                ref = L.P.T @ ((b[c] if use_b else 0.0) - L.A @ x[c])
                assert _relerr(got[c], ref) <= RTOL
        xg = _dev(x.reshape(shape))
        H.debug_prolong_add(l, xg, _dev(e.reshape(cshape)))
        got = _host(xg).reshape(ncomp, L.n)
        for c in range(ncomp):
            assert _relerr(got[c], x[c] + L.P @ e[c]) <= RTOL


# level-0 residual + restriction on grids whose coarse columns and coarse layers are ragged
# (partial tiles in x and y, several z-runs per column with a short last one), with 16 x 8
# coarse tiles (coarse x-extent 24 and 20) and 8 x 8 ones (10)
@pytest.mark.parametrize("dims,levels", [((48, 24, 40), 3), ((20, 12, 36), 2),
                                         ((40, 16, 24), 3)])
def test_restrict_residual0_ragged(dims, levels):
    _announce("restrict_residual0 %s L=%d" % (dims, levels))
    ncomp = 2
    H = _hier(*dims, ncomp=ncomp, levels=levels, coarsest_max=2048)
    mg = StochasticMG(*dims, levels=levels, coarsest_max=2048)
    L, C = mg.levels[0], mg.levels[1]
    shape = (ncomp,) + tuple(reversed(L.dims))
    cshape = (ncomp,) + tuple(reversed(C.dims))
    x = uniform_field((ncomp, L.n), 41)
    b = gaussian_field((ncomp, L.n), 42)
    for use_b in (False, True):
        bc = torch.zeros(cshape, dtype=torch.float64, device="cuda")
        H.debug_restrict_residual(0, _dev(x.reshape(shape)),
                                  _dev(b.reshape(shape)) if use_b else None, bc)
        got = _host(bc).reshape(ncomp, C.n)
        for c in range(ncomp):
            ref = L.P.T @ ((b[c] if use_b else 0.0) - L.A @ x[c])
            assert _relerr(got[c], ref) <= RTOL


@pytest.mark.parametrize("dims,levels", [((16, 16, 16), 3), ((8, 8, 8), 1), ((16, 16, 8), 3),
                                         ((32, 32, 16), 3)])
def test_coarsest(dims, levels):
    _announce("coarsest %s L=%d" % (dims, levels))
    ncomp = 3
    kT = 2.5
    H = _hier(*dims, ncomp=ncomp, kT=kT, levels=levels, coarsest_max=4096)
    mg = StochasticMG(*dims, kT=kT, levels=levels, coarsest_max=4096)
    L = mg.levels[-1]
    shape = (ncomp,) + tuple(reversed(L.dims))
    b = gaussian_field((ncomp, L.n), 3)
    for noise in (False, True):
        xg = torch.zeros(shape, dtype=torch.float64, device="cuda")
        H.debug_coarsest(xg, _dev(b.reshape(shape)), seed=17, cycle=4, noise=noise)
        got = _host(xg).reshape(ncomp, L.n)
        for c in range(ncomp):
            ref = mg.coarsest_step(L, b[c], PhiloxNoise(17) if noise else None, (4, c))
            assert _relerr(got[c], ref) <= RTOL


# ----------------------------------------------------------------------------- whole cycles
def _chain_case(dims, ncomp, levels, n, seed, kT=1.0, coarsest="cholesky", nu=(2, 2),
                first_cycle=0, stride=1, burn_in=0, coarsest_max=512):
    _announce("chain %s ncomp=%d L=%d n=%d seed=%d mode=%s" % (dims, ncomp, levels, n, seed, coarsest))
    H = _hier(*dims, ncomp=ncomp, kT=kT, levels=levels, coarsest=coarsest, nu1=nu[0], nu2=nu[1],
              stride=stride, burn_in=burn_in, coarsest_max=coarsest_max)
    out, state = H.sample(n, seed, first_cycle=first_cycle)
    got = _host(out)
    mg = StochasticMG(*dims, kT=kT, levels=levels, coarsest=coarsest, nu1=nu[0], nu2=nu[1],
                      coarsest_max=coarsest_max)
    ref, ref_state = mg.sample_chain(n, seed, first_cycle=first_cycle, ncomp=ncomp, stride=stride,
                                     burn_in=burn_in)
    got = got.reshape(n, ncomp, -1)
    for i in range(n):
        assert _relerr(got[i], ref[i]) <= RTOL, "sample %d" % i
    assert _relerr(_host(state).reshape(ncomp, -1), ref_state) <= RTOL
    return H


def test_chain_plain_fp64_16cubed_200_cycles():
    """16^3, h = 1, kT = 1, V(2,2), 3 levels, seed 0, 200 cycles from the zero start."""
    _chain_case((16, 16, 16), 1, 3, 200, 0)


@pytest.mark.parametrize("dims,ncomp,levels,coarsest", [
    ((8, 8, 16), 3, 3, "cholesky"), ((12, 8, 6), 2, 2, "cholesky"), ((32, 32, 16), 1, 4, "smooth"),
    ((6, 4, 3), 1, 1, "smooth"), ((4, 4, 4), 2, 1, "cholesky"), ((32, 16, 8), 1, 0, "cholesky"),
    ((4, 2, 2), 1, 2, "cholesky")])
def test_chain_shapes(dims, ncomp, levels, coarsest):
    _chain_case(dims, ncomp, levels, 6, 31, kT=1.3, coarsest=coarsest, coarsest_max=64)


def test_chain_stride_burnin_firstcycle():
    _chain_case((16, 16, 8), 2, 3, 4, 8, stride=3, burn_in=2, first_cycle=11)


def test_chain_nu_variants():
    _chain_case((16, 16, 16), 1, 3, 3, 2, nu=(1, 3))
    _chain_case((16, 16, 16), 1, 3, 3, 2, nu=(3, 0))


def test_chain_resume_bitwise():
    _announce("resume 16x16x8")
    H = _hier(16, 16, 8, ncomp=2, levels=3)
    full, _ = H.sample(6, 9)
    a, st = H.sample(3, 9)
    b, _ = H.sample(3, 9, first_cycle=3, state=st)
    assert torch.equal(full, torch.cat([a, b]))


def test_float32_output_is_cast_of_float64():
    _announce("f32 out")
    H = _hier(16, 16, 8, levels=3)
    a, _ = H.sample(3, 4)
    b, _ = H.sample(3, 4, out_dtype=torch.float32)
    assert torch.equal(a.float(), b)


def test_kT_scaling_on_gpu():
    _announce("kT scaling")
    a, _ = _hier(16, 16, 8, levels=3, kT=1.0).sample(3, 4)
    b, _ = _hier(16, 16, 8, levels=3, kT=4.0).sample(3, 4)
    assert _relerr(_host(b), 2.0 * _host(a)) <= RTOL


# ----------------------------------------------------------------------------- solve
@pytest.mark.parametrize("dims,levels,ncomp", [((16, 16, 16), 3, 1), ((12, 8, 6), 2, 2),
                                               ((8, 8, 8), 1, 1), ((32, 16, 8), 0, 3)])
def test_solve(dims, levels, ncomp):
    _announce("solve %s L=%d ncomp=%d" % (dims, levels, ncomp))
    H = _hier(*dims, ncomp=ncomp, levels=levels, coarsest_max=512)
    mg = StochasticMG(*dims, levels=levels, coarsest_max=512)
    f = gaussian_field(H.shape, 1)
    u, cycles, relres = H.solve(_dev(f), rtol=1e-12, max_cycles=60)
    assert relres <= 1e-12
    got = _host(u).reshape(ncomp, -1)
    for c in range(ncomp):
        ref, rc, rres = mg.solve(f[c].ravel(), rtol=1e-12)
        exact = spectral.solve(f[c], *dims)
        assert _relerr(got[c], exact) <= 1e-10
        if c == 0:
            assert abs(cycles - rc) <= 1
            # same number of cycles: same iterate up to rounding
            if cycles == rc:
                assert _relerr(got[c], ref) <= 1e-10


def test_solve_errors():
    from paper_1003_2680_amd.abi import SMGError, SMG_ENOTCONV, SMG_ENONFINITE
    _announce("solve errors")
    H = _hier(16, 16, 8, levels=3)
    f = gaussian_field(H.shape, 2)
    with pytest.raises(SMGError) as e:
        H.solve(_dev(f), rtol=1e-14, max_cycles=1)
    assert e.value.code == SMG_ENOTCONV
    bad = f.copy()
    bad[0, 1, 2, 3] = np.nan
    with pytest.raises(SMGError) as e:
        H.solve(_dev(bad), rtol=1e-10)
    assert e.value.code == SMG_ENONFINITE
    u, cycles, relres = H.solve(torch.zeros(H.shape, dtype=torch.float64, device="cuda"))
    assert cycles == 0 and relres == 0.0 and float(u.abs().max()) == 0.0


@pytest.mark.parametrize("dims,levels,ncomp", [((32, 32, 16), 4, 2), ((16, 16, 16), 3, 1),
                                               ((64, 32, 32), 0, 1)])
def test_bottom_kernel_matches_per_pass_launches(dims, levels, ncomp):
    """The LDS-resident bottom of the V-cycle and the one-launch-per-pass path agree, and both
    follow the oracle's chain."""
    _announce("bottom on/off %s L=%d" % (dims, levels))
    outs = []
    for use in (True, False):
        H = _hier(*dims, ncomp=ncomp, levels=levels, coarsest_max=64)
        H.set_bottom_kernel(use)
        out, _ = H.sample(3, 21)
        outs.append(_host(out))
    assert _relerr(outs[0], outs[1]) <= 1e-13
    mg = StochasticMG(*dims, levels=levels, coarsest_max=64)
    ref, _ = mg.sample_chain(3, 21, ncomp=ncomp)
    assert _relerr(outs[0].reshape(ref.shape), ref) <= RTOL
    f = gaussian_field((ncomp,) + tuple(reversed(dims)), 3)
    sols = []
    for use in (True, False):
        H = _hier(*dims, ncomp=ncomp, levels=levels, coarsest_max=64)
        H.set_bottom_kernel(use)
        u, cycles, relres = H.solve(_dev(f), rtol=1e-11)
        sols.append(_host(u))
    assert _relerr(sols[0], sols[1]) <= 1e-12


@pytest.mark.gpu
def test_level0_normals_close_to_oracle():
    """With x = 0, b = 0 and kT = 6 h^2 an interior site's update is exactly its normal, so
    the FP64 Box-Muller of the kernels is compared with the oracle's (NumPy log, cos, sin)
    value by value: 1e-14 absolute, far tighter than the field bar (the oracle rounds 2 pi u2,
    worth a few 1e-16 times the radius)."""
    dims = (64, 16, 8)
    _announce("level-0 normals %s" % (dims,))
    H = _hier(*dims, ncomp=1, kT=6.0, levels=1, coarsest="smooth")
    mg = StochasticMG(*dims, kT=6.0, levels=1, coarsest="smooth")
    L = mg.levels[0]
    N = L.n
    nx, ny, nz = dims
    interior = (np.arange(N) // (nx * ny) > 0) & (np.arange(N) // (nx * ny) < nz - 1)
    seed, cycle, slot = 987654321, 5, 1
    for colour in (0, 1):
        xg = torch.zeros(H.shape, dtype=torch.float64, device="cuda")
        H.debug_smooth(0, colour, xg, None, seed=seed, cycle=cycle, slot=slot)
        got = _host(xg).reshape(N)
        ref = np.zeros(N)
        mg._point_pass(L, ref, np.zeros(N), colour, PhiloxNoise(seed), (cycle, slot, 0))
        sel = interior & (ref != 0.0)
        assert sel.sum() == (nz - 2) * nx * ny // 2   # the colour's interior sites
        assert np.max(np.abs(got[sel] - ref[sel])) <= 1e-14
