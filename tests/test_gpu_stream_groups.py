"""Component groups on streams of their own (SMG_OPT_STREAM_GROUPS) against the one-stream call.

A sampling call with G stream groups runs components [i nc / G, (i+1) nc / G) on stream i,
group i starting each cycle after group i - 1 has finished that cycle's down-leg; every
component's kernels are those of the one-stream call, on shifted pointers with the component
offset added to the noise keys, so every output must match bit for bit.

* Batched chains (smg_sample_batch): the emitted fields, the observables, the running moments
  and the final state, over two calls in a row (the second continues the chains from the device
  table).  Cases: the bottom kernel with FP64 sweeps, groups that cut chains apart (5 chains of
  2 components in 2 groups), one component per chain with float32 output, the FP32-refined
  form, the bottom kernel off (every level as launches), a one-level hierarchy (exact draws
  only), more groups than components, and one chain of three components split 1 + 2.
* One chain (smg_sample_field, smg_sample_stats from a nonzero first cycle).
"""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (dims, hierarchy keywords, chains, comps per chain, groups, bottom kernel, out dtype)
CASES = [
    ((64, 64, 32), dict(levels=4), 8, 3, 2, True, torch.float64),
    ((32, 32, 16), dict(levels=3), 5, 2, 2, True, torch.float64),
    ((32, 32, 32), dict(levels=3), 8, 1, 2, True, torch.float32),
    ((64, 64, 32), dict(levels=4, precision="fp32_refined"), 4, 3, 2, True, torch.float64),
    ((32, 32, 16), dict(levels=3), 4, 2, 2, False, torch.float64),
    ((8, 8, 4), dict(levels=1), 6, 1, 2, True, torch.float64),
    ((16, 16, 8), dict(levels=2), 1, 1, 2, True, torch.float64),
    ((64, 64, 32), dict(levels=4), 1, 3, 2, True, torch.float64),
]


def _hier(dims, kw, ncomp, groups, bottom=True):
    from paper_1003_2680_amd.api import Hierarchy
    H = Hierarchy(*dims, ncomp=ncomp, stride=2, burn_in=1, **kw)
    H.set_bottom_kernel(bottom)
    H.set_stream_groups(groups)
    return H


def _run_batch(dims, kw, nch, cpc, groups, bottom, out_dtype):
    H = _hier(dims, kw, nch * cpc, groups, bottom)
    nx, ny, nz = dims
    shape = (nch * cpc, nz, ny, nx)
    state = torch.zeros(shape, dtype=torch.float64, device=H.device)
    res = []
    for call in range(2):
        n = 3 - call
        out = torch.empty((n,) + shape, dtype=out_dtype, device=H.device)
        mom = torch.zeros((2,) + shape, dtype=torch.float64, device=H.device)
        seeds = [11 + 7 * c for c in range(nch)] if call == 0 else None
        firsts = [3 * c for c in range(nch)] if call == 0 else None
        _, obs, _ = H.sample_batch(n, seeds=seeds, first_cycles=firsts, nchains=nch,
                                   comps_per_chain=cpc, state=state, out=out, with_obs=True,
                                   moments=mom)
        torch.cuda.synchronize()
        res += [out.clone(), obs.clone(), mom.clone(), state.clone()]
    H.close()
    return res


@pytest.mark.parametrize("dims,kw,nch,cpc,groups,bottom,out_dtype", CASES)
def test_stream_groups_batch_equal_one_stream(dims, kw, nch, cpc, groups, bottom, out_dtype):
    print("[gpu-case] stream groups %s %s chains=%d cpc=%d groups=%d bottom=%s"
          % (dims, kw, nch, cpc, groups, bottom), flush=True)
    ref = _run_batch(dims, kw, nch, cpc, 1, bottom, out_dtype)
    got = _run_batch(dims, kw, nch, cpc, groups, bottom, out_dtype)
    names = ["out", "obs", "moments", "state"] * 2
    for i, (a, b) in enumerate(zip(ref, got)):
        assert torch.isfinite(a).all()
        assert torch.equal(a, b), "call %d: %s differs" % (i // 4, names[i])
    assert ref[3].abs().max() > 0  # the chains moved


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_stream_groups_one_chain_equal_one_stream(precision):
    dims, kw = (32, 32, 16), dict(levels=3, precision=precision)
    print("[gpu-case] stream groups one chain %s" % precision, flush=True)
    res = []
    for groups in (1, 2):
        H = _hier(dims, kw, 3, groups)
        x, st = H.sample(4, 21, first_cycle=6)
        out = torch.empty_like(x)
        mom = torch.zeros((2,) + H.shape, dtype=torch.float64, device=H.device)
        obs, st2 = H.sample_stats(3, 5, first_cycle=9, out=out[:3], moments=mom)
        torch.cuda.synchronize()
        res.append([x.clone(), st.clone(), obs.clone(), out[:3].clone(), mom.clone(),
                    st2.clone()])
        H.close()
    for a, b in zip(*res):
        assert torch.equal(a, b)


def test_stream_groups_option_range():
    from paper_1003_2680_amd import abi
    H = _hier((16, 16, 8), dict(levels=2), 2, 1)
    for bad in (0, 3, -1):
        rc = H.lib.smg_set_option(H._h, abi.SMG_OPT_STREAM_GROUPS, bad)
        assert rc == abi.SMG_EINVAL
    H.set_stream_groups(2)
    H.close()
