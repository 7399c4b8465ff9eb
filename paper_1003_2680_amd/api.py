"""Python front end of the C-ABI: torch tensors for device memory, the current torch stream
for ordering.  Every step of the computation runs in the library's HIP kernels; this module
only allocates buffers and marshals arguments.
"""
import ctypes

import torch

from . import abi


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def lowest_modes(nx, ny, nz, k):
    """The k eigenvectors of A with the smallest eigenvalues, as (a, b, m) triples (C-ABI
    smg_lowest_modes)."""
    lib = abi.load()
    arr = (ctypes.c_int32 * (3 * max(k, 1)))()
    abi.check(lib.smg_lowest_modes(int(nx), int(ny), int(nz), int(k), arr))
    return [(arr[3 * q], arr[3 * q + 1], arr[3 * q + 2]) for q in range(k)]


def plan_bytes(dims, ncomp, precision="fp64", levels=0, coarsest_max=512):
    """Workspace bytes of a hierarchy (host planning only, no device work)."""
    lib = abi.load()
    desc = abi.GridDesc(dims[0], dims[1], dims[2], ncomp, 1.0, 1.0)
    prec = {"fp64": abi.SMG_FP64, "fp32_refined": abi.SMG_FP32_REFINED}[precision]
    prm = abi.CycleParams(levels, 2, 2, coarsest_max, abi.SMG_COARSEST_CHOLESKY, prec, 1, 0)
    h = ctypes.c_void_p()
    abi.check(lib.smg_create_hierarchy(ctypes.byref(desc), ctypes.byref(prm), ctypes.byref(h)))
    try:
        info = abi.Info()
        abi.check(lib.smg_hierarchy_info(h, ctypes.byref(info)))
        return int(info.workspace_bytes)
    finally:
        lib.smg_destroy_hierarchy(h)


def batch_run(items, device=None):
    """One library call over several hierarchies (C-ABI smg_batch_run): sampling items cycle in
    step, then solve items, with the small levels of all of them in merged launches.

    items: dicts with "H" (a Hierarchy; each at most once), "op" ("sample" or "solve"),
    "nchains" (0: one chain over all components) and "comps_per_chain"; sample items also
    "n", "state", "out" (or None), "out_dtype" (torch dtype), "seed"/"first_cycle" (one chain)
    or "seeds"/"first_cycles" (host lists; None continues the chain table); solve items "f",
    "u", "rtol", "max_cycles".  Returns, per item, (status, [(cycles, relres, last_ratio)])."""
    lib = abi.load()
    n = len(items)
    arr = (abi.BatchItem * max(n, 1))()
    keep = []
    for k, it in enumerate(items):
        H = it["H"]
        e = arr[k]
        e.h = H._h
        e.op = abi.SMG_OP_SAMPLE if it["op"] == "sample" else abi.SMG_OP_SOLVE
        e.nchains = int(it.get("nchains", 0))
        e.comps_per_chain = int(it.get("comps_per_chain", 1))
        if it["op"] == "sample":
            e.n = int(it["n"])
            e.out_dtype = abi.SMG_OUT_F32 if it.get("out_dtype") == torch.float32 else abi.SMG_OUT_F64
            e.seed = int(it.get("seed", 0))
            e.first_cycle = int(it.get("first_cycle", 0))
            if it.get("seeds") is not None:
                sd = (ctypes.c_uint64 * len(it["seeds"]))(*[int(v) for v in it["seeds"]])
                e.seeds = sd
                keep.append(sd)
                if it.get("first_cycles") is not None:
                    fc = (ctypes.c_uint64 * len(it["first_cycles"]))(
                        *[int(v) for v in it["first_cycles"]])
                    e.first_cycles = fc
                    keep.append(fc)
            e.state = it["state"].data_ptr()
            e.out = it["out"].data_ptr() if it.get("out") is not None else None
        else:
            e.f = it["f"].data_ptr()
            e.u = it["u"].data_ptr()
            e.rtol = float(it.get("rtol", 1e-12))
            e.max_cycles = int(it.get("max_cycles", 100))
            inf = (abi.SolveInfo * max(e.nchains, 1))()
            e.infos = inf
            keep.append(inf)
    dev = items[0]["H"].device if items else device
    rc = lib.smg_batch_run(arr, n, _stream(dev))
    out = []
    for k, it in enumerate(items):
        e = arr[k]
        infos = None
        if it["op"] == "solve":
            infos = [(e.infos[i].cycles, e.infos[i].relres, e.infos[i].last_ratio)
                     for i in range(max(e.nchains, 1))]
        out.append((e.status, infos))
    if rc not in (abi.SMG_OK, abi.SMG_ENOTCONV):
        abi.check(rc)
    return out


class Hierarchy:
    """A planned multigrid hierarchy bound to a device workspace.

    Fields are float64 tensors of shape [ncomp, nz, ny, nx] (x fastest).
    """

    def __init__(self, nx, ny, nz, ncomp=1, h=1.0, kT=1.0, levels=0, nu1=2, nu2=2,
                 coarsest_max=512, coarsest="cholesky", precision="fp64", stride=1, burn_in=0,
                 device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("no ROCm device: the stochastic multigrid library runs only on the GPU")
        self.lib = abi.load()
        dev = torch.device(device if device is not None else "cuda")
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.desc = abi.GridDesc(nx, ny, nz, ncomp, h, kT, abi.SMG_BC_PERIODIC,
                                 abi.SMG_BC_PERIODIC, abi.SMG_BC_DIRICHLET_FACE)
        mode = {"cholesky": abi.SMG_COARSEST_CHOLESKY, "smooth": abi.SMG_COARSEST_SMOOTH}[coarsest]
        prec = {"fp64": abi.SMG_FP64, "fp32_refined": abi.SMG_FP32_REFINED}[precision]
        self.params = abi.CycleParams(levels, nu1, nu2, coarsest_max, mode, prec, stride, burn_in)
        self.shape = (ncomp, nz, ny, nx)
        handle = ctypes.c_void_p()
        abi.check(self.lib.smg_create_hierarchy(ctypes.byref(self.desc), ctypes.byref(self.params),
                                                ctypes.byref(handle)))
        self._h = handle
        info = abi.Info()
        abi.check(self.lib.smg_hierarchy_info(self._h, ctypes.byref(info)))
        self.info = info
        self.n_levels = info.n_levels
        self.level_dims = [tuple(info.dims[l]) for l in range(info.n_levels)]
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(max(int(info.workspace_bytes), 256), dtype=torch.uint8,
                                         device=self.device)
            abi.check(self.lib.smg_bind_workspace(self._h, _ptr(self.workspace),
                                                  self.workspace.numel(), _stream(self.device)))

    def close(self):
        if self._h:
            self.lib.smg_destroy_hierarchy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ main entry points
    def new_state(self):
        return torch.zeros(self.shape, dtype=torch.float64, device=self.device)

    def sample(self, n, seed, first_cycle=0, state=None, out_dtype=torch.float64, out=None):
        """Run the chain; returns (samples [n, ncomp, nz, ny, nx], state).  A caller's `out`
        (float64 or float32, contiguous) decides the type written; out_dtype only sets that of
        a new one."""
        if state is None:
            state = self.new_state()
        self._check_field(state)
        if out is None and n > 0:
            out = torch.empty((n,) + self.shape, dtype=out_dtype, device=self.device)
        code = self._out_code(out, n, self.shape) if out is not None else abi.SMG_OUT_F64
        abi.check(self.lib.smg_sample_field(self._h, int(n), int(seed), int(first_cycle),
                                            _ptr(state), _ptr(out) if n > 0 else None, code,
                                            _stream(self.device)))
        return out, state

    def sample_stats(self, n, seed, modes=None, first_cycle=0, state=None, out=None,
                     out_dtype=torch.float64, moments=None, with_obs=True):
        """Run the chain and take FP64 statistics of every emitted sample.

        modes: (a, b, m) triples (default: the 8 lowest modes of A).  Returns
        (obs [n, ncomp, len(modes) + 1] float64 -- projections then the energy 1/2 x^T A x --
        or None, state).  `moments` ([2, ncomp, nz, ny, nx] float64, caller-zeroed) receives
        running sums of x and x^2; `out` (optional) the samples themselves."""
        if state is None:
            state = self.new_state()
        self._check_field(state)
        if modes is None:
            modes = lowest_modes(self.desc.nx, self.desc.ny, self.desc.nz, 8)
        marr = (ctypes.c_int32 * (3 * max(len(modes), 1)))(*[int(v) for md in modes for v in md])
        obs = None
        if with_obs:
            obs = torch.empty((n, self.shape[0], len(modes) + 1), dtype=torch.float64,
                              device=self.device)
        if moments is not None:
            self._check_moments(moments, self.shape)
        code = self._out_code(out, n, self.shape) if out is not None else abi.SMG_OUT_F64
        abi.check(self.lib.smg_sample_stats(
            self._h, int(n), int(seed), int(first_cycle), _ptr(state),
            _ptr(out) if out is not None else None, code, marr, len(modes),
            _ptr(obs) if obs is not None and n > 0 else None,
            _ptr(moments) if moments is not None else None, _stream(self.device)))
        return obs, state

    # ------------------------------------------------------------------ batched chains
    def _batch_shape(self, nchains, comps_per_chain):
        if comps_per_chain is None:
            comps_per_chain = self.shape[0] // nchains
        nact = nchains * comps_per_chain
        if nchains < 1 or comps_per_chain < 1 or nact > self.shape[0]:
            raise ValueError("nchains * comps_per_chain must be within ncomp")
        return comps_per_chain, (nact,) + self.shape[1:]

    def sample_batch(self, n, seeds=None, first_cycles=None, nchains=None, comps_per_chain=None,
                     state=None, out=None, out_dtype=torch.float64, modes=None, with_obs=False,
                     moments=None, emit=True):
        """Run nchains independent chains (seeds[c], first_cycles[c]) in the same launches.

        seeds=None continues the chains of the previous batched call (nchains required).
        emit=False runs the cycles without writing samples (unless `out` is given); a caller's
        `out` decides the type written (float64 or float32).
        Returns (out [n, nact, nz, ny, nx] or None, obs or None, state [nact, nz, ny, nx])
        with nact = nchains * comps_per_chain."""
        if seeds is not None:
            nchains = len(seeds)
        cpc, fshape = self._batch_shape(nchains, comps_per_chain)
        if state is None:
            state = torch.zeros(fshape, dtype=torch.float64, device=self.device)
        if state.dtype != torch.float64 or tuple(state.shape) != fshape or not state.is_contiguous():
            raise ValueError("state must be a contiguous float64 %s tensor" % (fshape,))
        if out is None and n > 0 and emit and not with_obs and moments is None:
            out = torch.empty((n,) + fshape, dtype=out_dtype, device=self.device)
        if moments is not None:
            self._check_moments(moments, fshape)
        sd = fc = None
        if seeds is not None:
            sd = (ctypes.c_uint64 * nchains)(*[int(v) for v in seeds])
            if first_cycles is not None:
                fc = (ctypes.c_uint64 * nchains)(*[int(v) for v in first_cycles])
        marr, nm, obs = None, 0, None
        if with_obs:
            if modes is None:
                modes = lowest_modes(self.desc.nx, self.desc.ny, self.desc.nz, 8)
            nm = len(modes)
            marr = (ctypes.c_int32 * (3 * max(nm, 1)))(*[int(v) for md in modes for v in md])
            obs = torch.empty((n, fshape[0], nm + 1), dtype=torch.float64, device=self.device)
        code = self._out_code(out, n, fshape) if out is not None else abi.SMG_OUT_F64
        abi.check(self.lib.smg_sample_batch(
            self._h, int(nchains), int(cpc), sd, fc, int(n), _ptr(state),
            _ptr(out) if out is not None else None, code, marr, nm,
            _ptr(obs) if obs is not None and n > 0 else None,
            _ptr(moments) if moments is not None else None, _stream(self.device)))
        return out, obs, state

    def solve_batch(self, f, nchains, comps_per_chain=None, rtol=1e-12, max_cycles=100, u=None,
                    raise_on_notconv=True):
        """Solve every chain's A u = f together; returns (u, [(cycles, relres, last_ratio)])."""
        cpc, fshape = self._batch_shape(nchains, comps_per_chain)
        if f.dtype != torch.float64 or tuple(f.shape) != fshape or not f.is_contiguous():
            raise ValueError("f must be a contiguous float64 %s tensor" % (fshape,))
        if u is None:
            u = torch.empty(fshape, dtype=torch.float64, device=self.device)
        infos = (abi.SolveInfo * nchains)()
        rc = self.lib.smg_solve_batch(self._h, int(nchains), int(cpc), _ptr(f), _ptr(u),
                                      float(rtol), int(max_cycles), _stream(self.device), infos)
        if rc != abi.SMG_ENOTCONV or raise_on_notconv:
            abi.check(rc)
        return u, [(i.cycles, i.relres, i.last_ratio) for i in infos]

    def solve(self, f, rtol=1e-12, max_cycles=100, u=None, raise_on_notconv=True):
        """Solve A u = f from u = 0; returns (u, cycles, relres).  The contraction of the
        last cycle is kept in ``self.last_ratio``."""
        self._check_field(f)
        if u is None:
            u = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        info = abi.SolveInfo()
        rc = self.lib.smg_solve(self._h, _ptr(f), _ptr(u), float(rtol), int(max_cycles),
                                _stream(self.device), ctypes.byref(info))
        if rc != abi.SMG_ENOTCONV or raise_on_notconv:
            abi.check(rc)
        self.last_ratio = info.last_ratio
        return u, info.cycles, info.relres

    # ------------------------------------------------------------------ component entry points
    def debug_smooth(self, level, colour, x, b=None, seed=0, cycle=0, slot=0, noise=True):
        abi.check(self.lib.smg_debug_smooth(self._h, level, colour, _ptr(x), _ptr(b), int(seed),
                                            int(cycle), int(slot), int(bool(noise)),
                                            _stream(self.device)))

    def debug_restrict_residual(self, level, x, b, b_coarse):
        abi.check(self.lib.smg_debug_restrict_residual(self._h, level, _ptr(x), _ptr(b),
                                                       _ptr(b_coarse), _stream(self.device)))

    def debug_prolong_add(self, level, x, e_coarse):
        abi.check(self.lib.smg_debug_prolong_add(self._h, level, _ptr(x), _ptr(e_coarse),
                                                 _stream(self.device)))

    def debug_coarsest(self, x, b, seed=0, cycle=0, noise=True):
        abi.check(self.lib.smg_debug_coarsest(self._h, _ptr(x), _ptr(b), int(seed), int(cycle),
                                              int(bool(noise)), _stream(self.device)))

    def set_bottom_kernel(self, enable):
        """Run the small levels in one LDS-resident launch per cycle (default) or per pass."""
        abi.check(self.lib.smg_set_option(self._h, abi.SMG_OPT_BOTTOM_KERNEL, int(bool(enable))))

    def set_block_tile(self, tile):
        """Tile shape of the Galerkin block passes: "auto", "4x4", "4x2" or "8x4"."""
        code = {"auto": abi.SMG_TILE_AUTO, "4x4": abi.SMG_TILE_4X4, "4x2": abi.SMG_TILE_4X2,
                "8x4": abi.SMG_TILE_8X4}[tile]
        abi.check(self.lib.smg_set_option(self._h, abi.SMG_OPT_BLOCK_TILE, code))

    def set_block_pairs(self, enable):
        """Two block colours per launch on Galerkin levels (default) or one."""
        abi.check(self.lib.smg_set_option(self._h, abi.SMG_OPT_BLOCK_PAIRS, int(bool(enable))))

    def set_stream_groups(self, n):
        """Sampling calls run their components in n staggered groups, each on a stream of its
        own (1, the default: the caller's stream only; at most 2); results are unchanged."""
        abi.check(self.lib.smg_set_option(self._h, abi.SMG_OPT_STREAM_GROUPS, int(n)))

    def kernel_timing(self, enable, kernel="fine_pass"):
        """Bracket every launch of one kernel class with HIP events: "fine_pass" (level-0
        colour pass), "level1_block_pass" or "bottom"."""
        which = {"fine_pass": abi.SMG_TIMED_FINE_PASS,
                 "level1_block_pass": abi.SMG_TIMED_LEVEL1_BLOCK_PASS,
                 "bottom": abi.SMG_TIMED_BOTTOM}[kernel]
        abi.check(self.lib.smg_set_option(self._h, abi.SMG_OPT_TIMED_KERNEL, which))
        abi.check(self.lib.smg_kernel_timing(self._h, int(bool(enable))))

    def kernel_timing_read(self):
        cnt = ctypes.c_int64()
        ms = ctypes.c_double()
        abi.check(self.lib.smg_kernel_timing_read(self._h, ctypes.byref(cnt), ctypes.byref(ms)))
        return cnt.value, ms.value

    def _out_code(self, out, n, fshape):
        """The output dtype code of a caller's `out` ([n] + fshape, float64 or float32,
        contiguous, on this device); the library writes exactly that many elements of that
        type."""
        if out.dtype not in (torch.float64, torch.float32) or not out.is_contiguous() \
                or tuple(out.shape) != (n,) + tuple(fshape) or out.device != self.device:
            raise ValueError("out must be a contiguous float64 or float32 %s tensor on %s"
                             % ((n,) + tuple(fshape), self.device))
        return abi.SMG_OUT_F32 if out.dtype == torch.float32 else abi.SMG_OUT_F64

    def _check_moments(self, moments, fshape):
        if moments.dtype != torch.float64 or tuple(moments.shape) != (2,) + tuple(fshape) \
                or not moments.is_contiguous() or moments.device != self.device:
            raise ValueError("moments must be a contiguous float64 %s tensor on %s"
                             % ((2,) + tuple(fshape), self.device))

    def _check_field(self, t):
        if t.dtype != torch.float64 or tuple(t.shape) != self.shape or not t.is_contiguous() \
                or t.device != self.device:
            raise ValueError("field must be a contiguous float64 %s tensor on %s" %
                             (self.shape, self.device))
