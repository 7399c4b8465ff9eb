"""The C-ABI batch call smg_batch_run over uneven hierarchies: every item's result equals the
same operation called alone, bit for bit.

Items differ in grid, depth, precision, chain batching and bottom handling: a one-chain FP64
sampler, a batched FP32-refined sampler, a hierarchy whose small levels run one launch per pass
(no merged bottom), a one-level hierarchy drawn exactly, and several hierarchies whose bottoms
share a launch; sampling items run different numbers of cycles (stride, burn-in, n), also in
two staggered stream groups; solve items converge after different numbers of cycles (different
rtol).
"""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _announce(msg):
    print("[gpu-case] " + msg, flush=True)


def _H(dims, **kw):
    from paper_1003_2680_amd.api import Hierarchy
    return Hierarchy(*dims, **kw)


SAMPLE_CASES = [
    # dims, hierarchy kwargs, nchains, cpc, n, bottom kernel
    ((16, 16, 16), dict(ncomp=2, levels=3, kT=1.1), 0, 1, 3, True),
    ((32, 32, 16), dict(ncomp=4, levels=4, precision="fp32_refined"), 2, 2, 2, True),
    ((16, 16, 8), dict(ncomp=1, levels=3, stride=2, burn_in=1), 0, 1, 2, True),
    ((32, 16, 16), dict(ncomp=3, levels=4), 3, 1, 4, False),
    ((8, 8, 8), dict(ncomp=1, levels=1), 0, 1, 2, True),
    ((48, 48, 48), dict(ncomp=2, levels=0, coarsest_max=4096), 2, 1, 1, True),
]


def _items(seed_base, dtype, groups=1):
    items, hs = [], []
    for k, (dims, kw, nch, cpc, n, bottom) in enumerate(SAMPLE_CASES):
        H = _H(dims, **kw)
        H.set_bottom_kernel(bottom)
        H.set_stream_groups(groups)
        st = torch.zeros(H.shape, dtype=torch.float64, device="cuda")
        nact = nch * cpc if nch else H.shape[0]
        st = st[:nact].contiguous()
        out = torch.empty((n, nact) + H.shape[1:], dtype=dtype, device="cuda")
        it = {"H": H, "op": "sample", "nchains": nch, "comps_per_chain": cpc, "n": n,
              "state": st, "out": out, "out_dtype": dtype}
        if nch:
            it["seeds"] = [seed_base + 10 * k + c for c in range(nch)]
            it["first_cycles"] = [3 * c for c in range(nch)]
        else:
            it["seed"], it["first_cycle"] = seed_base + 10 * k, 5
        items.append(it)
        hs.append(H)
    return items


@pytest.mark.parametrize("dtype,groups", [(torch.float64, 1), (torch.float32, 1),
                                          (torch.float64, 2), (torch.float32, 2)])
def test_batch_run_samples_equal_alone(dtype, groups):
    """groups > 1: the items' components in staggered stream groups (each group a share of
    every item, lockstep legs and merged bottoms within the group)."""
    from paper_1003_2680_amd.api import batch_run
    _announce("smg_batch_run samples %s, %d stream group(s)" % (dtype, groups))
    items = _items(300, dtype, groups)
    res = batch_run(items)
    torch.cuda.synchronize()
    assert all(st == 0 for st, _ in res), res
    for k, it in enumerate(items):
        dims, kw, nch, cpc, n, bottom = SAMPLE_CASES[k]
        H = _H(dims, **kw)
        H.set_bottom_kernel(bottom)
        if nch:
            st = torch.zeros((nch * cpc,) + H.shape[1:], dtype=torch.float64, device="cuda")
            out, _, st = H.sample_batch(n, seeds=it["seeds"], first_cycles=it["first_cycles"],
                                        comps_per_chain=cpc, state=st, out_dtype=dtype)
        else:
            out, st = H.sample(n, it["seed"], first_cycle=it["first_cycle"], out_dtype=dtype)
        torch.cuda.synchronize()
        assert torch.equal(out, it["out"]), (k, dims)
        assert torch.equal(st, it["state"]), (k, dims)


def test_batch_run_solves_equal_alone():
    from paper_1003_2680_amd.api import batch_run
    from paper_1003_2680_amd.inputs import gaussian_field
    _announce("smg_batch_run solves")
    cases = [((16, 16, 16), dict(ncomp=2, levels=3), 0, 1, 1e-12),
             ((32, 32, 16), dict(ncomp=4, levels=4, precision="fp32_refined"), 2, 2, 1e-10),
             ((32, 16, 16), dict(ncomp=3, levels=4), 3, 1, 1e-6),
             ((8, 8, 8), dict(ncomp=1, levels=1), 0, 1, 1e-12)]
    items = []
    for k, (dims, kw, nch, cpc, rtol) in enumerate(cases):
        H = _H(dims, **kw)
        f = torch.from_numpy(gaussian_field(H.shape, 70 + k)).cuda()
        items.append({"H": H, "op": "solve", "nchains": nch, "comps_per_chain": cpc, "f": f,
                      "u": torch.empty_like(f), "rtol": rtol, "max_cycles": 60})
    res = batch_run(items)
    torch.cuda.synchronize()
    cycles = []
    for k, ((dims, kw, nch, cpc, rtol), it, (st, infos)) in enumerate(zip(cases, items, res)):
        assert st == 0, (k, st)
        H = _H(dims, **kw)
        if nch:
            u, inf = H.solve_batch(it["f"], nchains=nch, comps_per_chain=cpc, rtol=rtol,
                                   max_cycles=60)
        else:
            u, cyc, rel = H.solve(it["f"], rtol=rtol, max_cycles=60)
            inf = [(cyc, rel, H.last_ratio)]
        assert torch.equal(u, it["u"]), (k, dims)
        assert list(inf) == list(infos), (k, inf, infos)
        cycles.append(inf[0][0])
    assert len(set(cycles)) > 1   # the items stopped after different numbers of cycles


def test_batch_run_rejects_repeated_hierarchy():
    from paper_1003_2680_amd.api import batch_run
    from paper_1003_2680_amd import abi
    _announce("smg_batch_run repeated hierarchy")
    H = _H((16, 16, 8), ncomp=1, levels=3)
    st = torch.zeros(H.shape, dtype=torch.float64, device="cuda")
    it = {"H": H, "op": "sample", "nchains": 0, "n": 0, "state": st, "out": None}
    with pytest.raises(abi.SMGError):
        batch_run([it, dict(it)])
