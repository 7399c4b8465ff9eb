"""Allocation-free sampling entry point (smg_sample_field_static) against smg_sample_field.

Called through the C-ABI with ctypes: the static entry point must give the same samples and
final state, bit for bit, as the ordinary entry point on the same hierarchy shape, seed and
cycles; two calls in a row, the second on a smaller grid (the shared device array keeps the
first call's contents), then the first shape again; the ordinary binding of a hierarchy keeps
working after a static call; a hierarchy larger than the array is refused with SMG_ENOMEM
before any device work.
"""
import ctypes

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _announce(msg):
    print("[gpu-case] " + msg, flush=True)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _static_sample(H, n, seed, first_cycle=0, state=None, out_dtype=torch.float64):
    from paper_1003_2680_amd import abi
    lib = abi.load()
    if state is None:
        state = H.new_state()
    out = torch.empty((n,) + H.shape, dtype=out_dtype, device=H.device)
    code = abi.SMG_OUT_F32 if out_dtype == torch.float32 else abi.SMG_OUT_F64
    abi.check(lib.smg_sample_field_static(H._h, int(n), int(seed), int(first_cycle), _ptr(state),
                                          _ptr(out), code, _stream()))
    return out, state


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_static_equals_bound_two_calls(precision):
    from paper_1003_2680_amd.api import Hierarchy
    cases = [((32, 16, 16), 3, 4, 11), ((8, 8, 8), 1, 2, 5), ((32, 16, 16), 3, 3, 12)]
    for dims, ncomp, levels, seed in cases:
        _announce("static sample %s x%d L=%d %s" % (dims, ncomp, levels, precision))
        H = Hierarchy(*dims, ncomp=ncomp, levels=levels, kT=0.7, precision=precision)
        ref, st_ref = H.sample(3, seed, first_cycle=4)
        got, st = _static_sample(H, 3, seed, first_cycle=4)
        torch.cuda.synchronize()
        assert torch.equal(got, ref) and torch.equal(st, st_ref), (dims, precision)
        # the ordinary binding still works after the static call
        again, _ = H.sample(3, seed, first_cycle=4)
        torch.cuda.synchronize()
        assert torch.equal(again, ref)


def test_static_continues_chain_and_float_out():
    from paper_1003_2680_amd.api import Hierarchy
    _announce("static sample continuation, float32 out")
    H = Hierarchy(16, 16, 16, ncomp=2, levels=3)
    ref, _ = H.sample(4, 3)
    a, st = _static_sample(H, 2, 3)
    b, _ = _static_sample(H, 2, 3, first_cycle=2, state=st, out_dtype=torch.float32)
    torch.cuda.synchronize()
    assert torch.equal(a, ref[:2]) and torch.equal(b, ref[2:].float())


def test_static_refuses_oversized_hierarchy():
    from paper_1003_2680_amd import abi
    _announce("static sample size limit")
    lib = abi.load()
    desc = abi.GridDesc(128, 128, 128, 3, 1.0, 1.0, 0, 0, 0)
    prm = abi.CycleParams(6, 2, 2, 512, 0, 0, 1, 0)
    hd = ctypes.c_void_p()
    abi.check(lib.smg_create_hierarchy(ctypes.byref(desc), ctypes.byref(prm), ctypes.byref(hd)))
    try:
        info = abi.Info()
        abi.check(lib.smg_hierarchy_info(hd, ctypes.byref(info)))
        assert info.workspace_bytes > abi.SMG_STATIC_SCRATCH_BYTES
        rc = lib.smg_sample_field_static(hd, 1, 0, 0, ctypes.c_void_p(256), ctypes.c_void_p(512),
                                         0, None)
        assert rc == abi.SMG_ENOMEM and b"static scratch" in lib.smg_last_error()
    finally:
        lib.smg_destroy_hierarchy(hd)
