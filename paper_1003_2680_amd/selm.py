"""Python front end of the SELM coupling C-ABI (smg_selm_*): torch tensors for device memory,
the current torch stream for ordering.  Argument marshalling only; every step runs in the
library (its sampler, its multigrid solve and its coupling kernels)."""
import ctypes

import torch

from . import abi


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class SELM:
    """Structure points coupled to the wall-bounded Stokes fluid on an nx x ny x nz grid.

    Fields are float64 [3, nz, ny, nx]; positions, forces and velocities float64 [m, 3]."""

    def __init__(self, nx, ny, nz, h=1.0, mu=1.0, kT=1.0, levels=0, stride=2, max_points=64,
                 device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("no ROCm device: the SELM coupling runs only on the GPU")
        self.lib = abi.load()
        dev = torch.device(device if device is not None else "cuda")
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.dims = (nx, ny, nz)
        self.stride = stride
        self.max_points = max_points
        d = abi.SelmDesc(nx, ny, nz, h, mu, kT, levels, stride, max_points)
        hd = ctypes.c_void_p()
        abi.check(self.lib.smg_selm_create(ctypes.byref(d), ctypes.byref(hd)))
        self._h = hd
        info = abi.SelmInfo()
        abi.check(self.lib.smg_selm_get_info(self._h, ctypes.byref(info)))
        self.info = info
        with torch.cuda.device(dev):
            self.workspace = torch.empty(int(info.workspace_bytes), dtype=torch.uint8, device=dev)
            abi.check(self.lib.smg_selm_bind(self._h, _ptr(self.workspace),
                                             self.workspace.numel(), self._stream()))

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def close(self):
        if self._h:
            self.lib.smg_selm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_state(self):
        nx, ny, nz = self.dims
        return torch.zeros((3, nz, ny, nx), dtype=torch.float64, device=self.device)

    def project(self, u, out=None, rtol=1e-12):
        out = torch.empty_like(u) if out is None else out
        abi.check(self.lib.smg_selm_project(self._h, _ptr(u), _ptr(out), float(rtol),
                                            self._stream()))
        return out

    def mobility(self, X, F, rtol=1e-12):
        V = torch.empty_like(F)
        abi.check(self.lib.smg_selm_mobility(self._h, X.shape[0], _ptr(X), _ptr(F), _ptr(V),
                                             float(rtol), self._stream()))
        return V

    def drive(self, X, seed, first_cycle, state, rtol=1e-12):
        g = torch.empty_like(X)
        abi.check(self.lib.smg_selm_drive(self._h, X.shape[0], _ptr(X), int(seed),
                                          int(first_cycle), _ptr(state), _ptr(g), float(rtol),
                                          self._stream()))
        return g

    def step(self, X, F, dt, seed, step, state, rtol=1e-12):
        """X <- X + dt H F + sqrt(dt) g in place."""
        abi.check(self.lib.smg_selm_step(self._h, X.shape[0], _ptr(X), _ptr(F), float(dt),
                                         int(seed), int(step), _ptr(state), float(rtol),
                                         self._stream()))
        return X
