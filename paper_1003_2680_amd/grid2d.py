"""Python front end of the two-dimensional wall-bounded sampler (C-ABI smg2d_*): torch tensors
for device memory, the current torch stream for ordering; argument marshalling only."""
import ctypes

import torch

from . import abi


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Hierarchy2D:
    """nx x nz cells (periodic x, no-slip walls in z), ncomp independent chains; fields float64
    [ncomp, nz, nx]."""

    def __init__(self, nx, nz, ncomp=1, h=1.0, kT=1.0, levels=0, nu1=2, nu2=2, coarsest_max=512,
                 coarsest="cholesky", stride=1, device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("no ROCm device: the 2D sampler runs only on the GPU")
        self.lib = abi.load()
        dev = torch.device(device if device is not None else "cuda")
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        mode = {"cholesky": abi.SMG_COARSEST_CHOLESKY, "smooth": abi.SMG_COARSEST_SMOOTH}[coarsest]
        d = abi.Desc2D(nx, nz, ncomp, h, kT, levels, nu1, nu2, coarsest_max, mode, stride)
        hd = ctypes.c_void_p()
        abi.check(self.lib.smg2d_create(ctypes.byref(d), ctypes.byref(hd)))
        self._h = hd
        info = abi.Info2D()
        abi.check(self.lib.smg2d_get_info(self._h, ctypes.byref(info)))
        self.n_levels = info.n_levels
        self.level_dims = [tuple(info.dims[l]) for l in range(info.n_levels)]
        self.shape = (ncomp, nz, nx)
        with torch.cuda.device(dev):
            self.workspace = torch.empty(max(int(info.workspace_bytes), 256), dtype=torch.uint8,
                                         device=dev)
            abi.check(self.lib.smg2d_bind(self._h, _ptr(self.workspace),
                                          self.workspace.numel(), self._stream()))

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def close(self):
        if self._h:
            self.lib.smg2d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_state(self):
        return torch.zeros(self.shape, dtype=torch.float64, device=self.device)

    def sample(self, n, seed, first_cycle=0, state=None):
        """Returns (samples [n, ncomp, nz, nx], state)."""
        state = self.new_state() if state is None else state
        out = torch.empty((max(n, 1),) + self.shape, dtype=torch.float64, device=self.device)
        abi.check(self.lib.smg2d_sample(self._h, int(n), int(seed), int(first_cycle), _ptr(state),
                                        _ptr(out), self._stream()))
        return out[:n], state

    def solve(self, f, rtol=1e-12, max_cycles=100):
        u = torch.empty_like(f)
        info = abi.SolveInfo()
        abi.check(self.lib.smg2d_solve(self._h, _ptr(f), _ptr(u), float(rtol), int(max_cycles),
                                       self._stream(), ctypes.byref(info)))
        return u, info.cycles, info.relres
