"""Two block colours per launch (SMG_OPT_BLOCK_PAIRS) against one launch per colour.

The paired launch draws colours c and c ^ 1 of a Galerkin level in turn from one staged tile;
it must give bit for bit the chain of the single-colour passes in order.  Cases: block levels
of x-extent 8 to 128 (four block rows per work-group up to 64 cells, two at 128), a ragged
number of block rows, a level wider than 128 cells (which keeps one launch per colour), the
FP32-refined form, a noise-free solve, and the bottom kernel switched off (every small level's
sweeps as launches).
"""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [
    ((32, 32, 32), dict(levels=3), False),        # level 1: 16^3 as launches (bottom off)
    ((64, 64, 32), dict(levels=4), True),         # level 1: 32 x 32 x 16
    ((128, 128, 32), dict(levels=4), True),       # levels 1, 2: 64 and 32 wide
    ((256, 64, 16), dict(levels=4), True),        # level 1: 128 x 32 x 8 (two rows per group)
    ((48, 40, 24), dict(levels=3), True),         # level 1: 24 x 20 x 12, ragged rows
    ((512, 16, 8), dict(levels=3), True),         # level 1 is 256 wide: one colour per launch
    ((64, 64, 32), dict(levels=4, precision="fp32_refined"), True),
    ((32, 32, 16), dict(levels=3), False),        # bottom off: 16 x 16 x 8 as launches
]


@pytest.mark.parametrize("dims,kw,bottom", CASES)
def test_pairs_equal_single_colour(dims, kw, bottom):
    from paper_1003_2680_amd.api import Hierarchy
    print("[gpu-case] block pairs %s %s bottom=%s" % (dims, kw, bottom), flush=True)
    outs = []
    for pairs in (False, True):
        H = Hierarchy(*dims, ncomp=2, **kw)
        H.set_block_pairs(pairs)
        H.set_bottom_kernel(bottom)
        x, state = H.sample(3, 17, first_cycle=5)
        f = torch.randn(H.shape, dtype=torch.float64, device=H.device,
                        generator=torch.Generator(device=H.device).manual_seed(3))
        u, cycles, _ = H.solve(f, rtol=1e-10, max_cycles=40)
        torch.cuda.synchronize()
        outs.append((x, state, u, cycles))
    (x0, s0, u0, c0), (x1, s1, u1, c1) = outs
    assert torch.equal(x0, x1) and torch.equal(s0, s1)
    assert torch.equal(u0, u1) and c0 == c1
