"""Autotuner for the cycle configuration of a grid shape (depth, sweeps, tile shape, bottom).

The paper leaves the V-cycle depth (hence the size of the coarsest, exactly drawn level) and
the sweep counts open; every choice gives an exact
sampler of N(0, kT A^-1) (each move of the cycle is a heat-bath step), so the choice is a
matter of cost.  The cost of one effectively independent sample is

    t_cycle(config) * k_dec(rho(config)),   k_dec = max(1, ceil(ln 0.01 / ln rho)),

with t_cycle measured on the device for the batch the shape will run with, and rho the
contraction of the deterministic cycle of the same configuration (the decorrelation of the
stochastic iteration is governed by the same iteration matrix).  Depth and sweeps are chosen
on this cost; the tile shape of the Galerkin block passes and the LDS-resident bottom launch
change only the work distribution (never a result) and are then chosen on t_cycle alone.

Everything measured runs through the library's kernels; this module only orchestrates.
"""
import ctypes
import math

import torch

from . import abi
from .api import Hierarchy
from .inputs import gaussian_field

NU_CANDIDATES = ((1, 1), (2, 1), (1, 2), (2, 2))
TILES = ("4x4", "4x2", "8x4")


def _k_dec(rho):
    if not (rho > 0.0):
        return 1
    return max(1, math.ceil(math.log(0.01) / math.log(min(rho, 0.999))))


def _cycle_time(H, nchains, cycles, device):
    """Seconds per batched cycle (events on the current stream)."""
    state = torch.zeros((H.shape[0],) + H.shape[1:], dtype=torch.float64, device=device)
    H.sample_batch(2, seeds=list(range(nchains)), comps_per_chain=H.shape[0] // nchains,
                   state=state, emit=False)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(device)
    e0.record()
    H.sample_batch(cycles, nchains=nchains, comps_per_chain=H.shape[0] // nchains, state=state,
                   emit=False)
    e1.record()
    torch.cuda.synchronize(device)
    return e0.elapsed_time(e1) / 1e3 / cycles


def _contraction(dims, levels, nu, precision, device):
    H = Hierarchy(*dims, ncomp=1, levels=levels, nu1=nu[0], nu2=nu[1], precision=precision,
                  device=device)
    f = torch.from_numpy(gaussian_field(H.shape, 11)).to(device)
    H.solve(f, rtol=1e-9, max_cycles=60, raise_on_notconv=False)
    return H.last_ratio


# coarsest sizes whose automatic plans are tried (the exact draw of the coarsest level is dense:
# beyond about 2k unknowns its factors no longer fit the caches and its plan takes seconds)
COARSEST_SIZES = (2048, 1024, 512, 256, 128, 64, 32, 16, 8)


def depth_candidates(dims, precision="fp64"):
    """The depths worth trying and the size of their coarsest level: the automatic plans for
    every coarsest size in COARSEST_SIZES (each stops at the first level with at most that many
    unknowns), so that the coarsest size is tuned through the depth.  Host planning only (the
    library's planner; no device memory).  Returns [(levels, coarsest unknowns)], deepest last."""
    lib = abi.load()
    prec = {"fp64": abi.SMG_FP64, "fp32_refined": abi.SMG_FP32_REFINED}[precision]
    desc = abi.GridDesc(*dims, 1, 1.0, 1.0, abi.SMG_BC_PERIODIC, abi.SMG_BC_PERIODIC,
                        abi.SMG_BC_DIRICHLET_FACE)
    out = {}
    for cm in COARSEST_SIZES:
        prm = abi.CycleParams(0, 2, 2, cm, abi.SMG_COARSEST_CHOLESKY, prec, 1, 0)
        hd = ctypes.c_void_p()
        if lib.smg_create_hierarchy(ctypes.byref(desc), ctypes.byref(prm), ctypes.byref(hd)):
            continue
        info = abi.Info()
        rc = lib.smg_hierarchy_info(hd, ctypes.byref(info))
        lib.smg_destroy_hierarchy(hd)
        if rc:
            continue
        c = info.dims[info.n_levels - 1]
        out.setdefault(info.n_levels, c[0] * c[1] * c[2])
    return sorted(out.items())


def tune(dims, nchains, precision="fp32_refined", cycles=4, device=None):
    """Best configuration for `nchains` batched scalar chains on a grid `dims`.

    Returns a dict: levels, nu1, nu2, tile, bottom, plus the measured t_cycle (s), rho, k_dec
    and cost (s per decorrelated sample of the whole batch) of the choice, and the table of
    every candidate measured."""
    device = torch.device(device if device is not None else "cuda")
    table = []
    best = None
    for levels, coarsest in depth_candidates(dims, precision):
        for nu in NU_CANDIDATES:
            H = Hierarchy(*dims, ncomp=nchains, levels=levels, nu1=nu[0], nu2=nu[1],
                          precision=precision, device=device)
            t = _cycle_time(H, nchains, cycles, device)
            del H
            rho = _contraction(dims, levels, nu, precision, device)
            cost = t * _k_dec(rho)
            row = {"levels": levels, "coarsest": coarsest, "nu1": nu[0], "nu2": nu[1],
                   "tile": "auto", "bottom": True, "t_cycle": t, "rho": rho,
                   "k_dec": _k_dec(rho), "cost": cost}
            table.append(row)
            if best is None or cost < best["cost"]:
                best = dict(row)
    # work distribution only: tile shape and bottom launch on t_cycle
    for tile in TILES:
        for bottom in (True, False):
            H = Hierarchy(*dims, ncomp=nchains, levels=best["levels"], nu1=best["nu1"],
                          nu2=best["nu2"], precision=precision, device=device)
            H.set_block_tile(tile)
            H.set_bottom_kernel(bottom)
            t = _cycle_time(H, nchains, cycles, device)
            del H
            row = dict(best, tile=tile, bottom=bottom, t_cycle=t, cost=t * best["k_dec"])
            table.append(row)
            if row["cost"] < best["cost"]:
                best = dict(row)
    best["table"] = table
    return best


def apply(H, config):
    """Apply the work-distribution part of a tuned configuration to a hierarchy."""
    H.set_block_tile(config.get("tile", "auto"))
    H.set_bottom_kernel(config.get("bottom", True))
