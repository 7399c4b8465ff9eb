"""Python front end of the composite-grid FAC sampler/solver (C-ABI smg_composite_*).

Argument marshalling only: torch tensors hold the device fields and the workspace, the
current torch stream orders the work, and every step runs in the library's HIP kernels.
A composite field is a pair (coarse, fine): coarse float64 [nz, ny, nx] over the whole base
grid (covered cells ignored), fine float64 [fz, fy, fx] over the refined box.
"""
import ctypes

import numpy as np

from . import abi


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


PRECISIONS = {"fp64": abi.SMG_FP64, "fp32_refined": abi.SMG_FP32_REFINED}


def plan(nx, ny, nz, box, h=1.0, kT=1.0, nu=2, mu1=2, mu2=2, levels=0, coarsest_max=512,
         gs_only=False, precision="fp64", row_lanes=0):
    """Host-only plan: (handle, info).  The caller destroys the handle (destroy_plan)."""
    lib = abi.load()
    desc = abi.CompositeDesc(nx, ny, nz, (ctypes.c_int32 * 6)(*box), h, kT)
    prm = abi.FACParams(nu, mu1, mu2, levels, coarsest_max, int(bool(gs_only)),
                        PRECISIONS[precision], int(row_lanes))
    hd = ctypes.c_void_p()
    abi.check(lib.smg_composite_create(ctypes.byref(desc), ctypes.byref(prm), ctypes.byref(hd)))
    info = abi.CompositeInfo()
    abi.check(lib.smg_composite_get_info(hd, ctypes.byref(info)))
    return hd, info


def destroy_plan(hd):
    abi.load().smg_composite_destroy(hd)


def stored_row(hd, level, cell):
    """Row `cell` of base level `level` as stored by the plan: (targets, values)."""
    lib = abi.load()
    t = (ctypes.c_int64 * 125)()
    v = (ctypes.c_double * 125)()
    c = ctypes.c_int32()
    abi.check(lib.smg_composite_debug_row(hd, int(level), int(cell), t, v, ctypes.byref(c)))
    return np.array(t[:c.value], dtype=np.int64), np.array(v[:c.value])


class CompositeSampler:
    """A planned composite hierarchy bound to a device workspace."""

    def __init__(self, nx, ny, nz, box, h=1.0, kT=1.0, nu=2, mu1=2, mu2=2, levels=0,
                 coarsest_max=512, gs_only=False, precision="fp64", device=None, row_lanes=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no ROCm device: the composite FAC library runs only on the GPU")
        self.torch = torch
        self.lib = abi.load()
        dev = torch.device(device if device is not None else "cuda")
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self._h, self.info = plan(nx, ny, nz, box, h, kT, nu, mu1, mu2, levels, coarsest_max,
                                  gs_only, precision, row_lanes)
        self.precision = precision
        self.base_shape = (nz, ny, nx)
        fd = self.info.fine_dims
        self.fine_shape = (fd[2], fd[1], fd[0])
        self.box = tuple(box)
        with torch.cuda.device(dev):
            self.workspace = torch.empty(max(int(self.info.workspace_bytes), 256),
                                         dtype=torch.uint8, device=dev)
            abi.check(self.lib.smg_composite_bind(self._h, _ptr(self.workspace),
                                                  self.workspace.numel(), self._stream()))

    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def zeros(self):
        t = self.torch
        return (t.zeros(self.base_shape, dtype=t.float64, device=self.device),
                t.zeros(self.fine_shape, dtype=t.float64, device=self.device))

    def _chk(self, *ts):
        for x in ts:
            if x is not None:
                assert x.is_contiguous() and x.dtype == self.torch.float64 and x.device == self.device

    def cycle(self, xc, xf, bc=None, bf=None, seed=0, cycle=0, noise=True):
        self._chk(xc, xf, bc, bf)
        abi.check(self.lib.smg_composite_cycle(self._h, _ptr(xc), _ptr(xf), _ptr(bc), _ptr(bf),
                                               seed, cycle, int(bool(noise)), self._stream()))

    def sample(self, xc, xf, ncycles, seed, first_cycle=0):
        self._chk(xc, xf)
        abi.check(self.lib.smg_composite_sample(self._h, int(ncycles), seed, first_cycle,
                                                _ptr(xc), _ptr(xf), self._stream()))

    def residual(self, xc, xf, bc=None, bf=None):
        rc, rf = self.zeros()
        self._chk(xc, xf, bc, bf)
        abi.check(self.lib.smg_composite_residual(self._h, _ptr(xc), _ptr(xf), _ptr(bc),
                                                  _ptr(bf), _ptr(rc), _ptr(rf), self._stream()))
        return rc, rf

    def solve(self, fc, ff, rtol=1e-10, max_cycles=100):
        uc, uf = self.zeros()
        self._chk(fc, ff)
        si = abi.SolveInfo()
        abi.check(self.lib.smg_composite_solve(self._h, _ptr(fc), _ptr(ff), _ptr(uc), _ptr(uf),
                                               rtol, max_cycles, self._stream(),
                                               ctypes.byref(si)))
        return uc, uf, si

    def forced_field(self, n, seed, first_sample=0, qc=None, qf=None, rtol=1e-10, max_cycles=100):
        """n draws of the field noise w = L^-1 Q eta, Q = diag(q) (q None = 1): returns
        (wc [n, nz, ny, nx], wf [n, fz, fy, fx], list of solve infos)."""
        t = self.torch
        self._chk(qc, qf)
        wc = t.empty((n,) + self.base_shape, dtype=t.float64, device=self.device)
        wf = t.empty((n,) + self.fine_shape, dtype=t.float64, device=self.device)
        infos = (abi.SolveInfo * max(n, 1))()
        abi.check(self.lib.smg_composite_forced_field(self._h, int(n), seed, first_sample,
                                                      _ptr(qc), _ptr(qf), _ptr(wc), _ptr(wf),
                                                      rtol, max_cycles, self._stream(), infos))
        return wc, wf, list(infos)[:n]

    def debug_pass(self, cls, xc, xf, bc=None, bf=None, seed=0, cycle=0, slot=0, noise=True):
        self._chk(xc, xf, bc, bf)
        abi.check(self.lib.smg_composite_debug_pass(self._h, cls, _ptr(xc), _ptr(xf), _ptr(bc),
                                                    _ptr(bf), seed, cycle, slot, int(bool(noise)),
                                                    self._stream()))

    def debug_base_pass(self, level, colour, x, b=None, seed=0, cycle=0, slot=0, noise=True):
        self._chk(x, b)
        abi.check(self.lib.smg_composite_debug_base_pass(self._h, level, colour, _ptr(x), _ptr(b),
                                                         seed, cycle, slot, int(bool(noise)),
                                                         self._stream()))

    def close(self):
        if getattr(self, "_h", None):
            self.lib.smg_composite_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
