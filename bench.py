"""Benchmark: decorrelated 128^3 field samples/s of the stochastic multigrid sampler on one GPU.

Workload: a 128x128x128 cell-centred grid (h = 1, kT = 1), periodic in x and y with no-slip
walls on the z faces; a 3-component velocity field (three decoupled scalar chains with the
same wall-bounded Laplacian); the 6-level stochastic V(2,2) cycle in FP64 (red-black heat
bath on the fine level, 2x2x2 block heat bath on the Galerkin levels, exact Cholesky draw on
the 4^3 coarsest level).  The chains of seeds 0..CHAINS-1 (--chains, default 8) are batched
into every launch (one hierarchy carrying CHAINS x 3 components; each chain draws exactly what
it draws alone).
k_dec = max(1, ceil(ln 0.01 / ln rho)) with rho the contraction of the cycle measured by the
deterministic solves (the lag-k correlation of the stochastic iteration is R^k applied to the
stationary covariance): k_dec cycles separate nearly independent draws.  One step = one batched
call that advances every chain by SAMPLES_PER_STEP * k_dec cycles and emits a sample every
k_dec cycles -- each emitted sample a decorrelated one -- writing its fields to an output buffer
in HBM and taking their observables (projections on the 8 lowest eigenvectors of A and the
energy 1/2 x^T A x) in the same pass.

value = decorrelated samples/s = emitted samples/s.  The lag-1 correlation of the emitted
observables (the chain's lag-k_dec correlation) is checked against 0.01 within its standard
error.  Also reported: one 3-component chain alone (no batching of chains); the integrated
autocorrelation time of each observable; per-step p50/p99 latency; the whole cycle against the
algorithmic-byte roofline; one FP64 chain on a single 512x512x256 grid, whose fields exceed the
256 MB Infinity Cache (cycles/s and the level-0 pass against HBM); 10 solves to 1e-12 (batched
throughput and single latency); the roofline of the dominant kernel class (per-launch time from
HIP events around each sweep's launches) and of the other; and the CPU oracle on a bounded
sample.

The FP32-refined form of the same workload (FP32 sweeps and transfers, FP64 residual,
correction and coarsest arithmetic) is measured beside it under "fp32_refined", with its
relative RMS difference from the FP64 chain on the same Philox streams.

The spatially adaptive composite workload (256x256x128 base with the box [64,192)^2 x [0,32)
refined by two, 12.06 M unknowns; stochastic FAC cycle, FP64 and FP32-refined) is measured under
"composite": cycles/s, decorrelated samples/s, the solve, equipartition, the live-timed block
pass of its finest base level against HBM, and the oracle's FAC cycle on its 16^3-base copy.

Run: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-refined]
                     [--no-composite]
     python bench.py --composite-only   (the adaptive workload alone)
     python bench.py --batched-only     (the 64-instance batched workload alone)
     python bench.py --copy-calibration   (a plain 1 GiB copy, for counter calibration)
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

def progress(msg):
    """One line per finished stage on stderr (stdout carries only the result line)."""
    print("[bench] %s" % msg, file=sys.stderr, flush=True)


NX = NY = NZ = 128
NCOMP = 3
LEVELS = 6
SAMPLES_PER_STEP = 8
STREAM_GROUPS = 2  # the sampled components run in this many groups, each on a stream of its own
HBM_PEAK_GBS = 8000.0
METRIC = "decorrelated 128³ field samples/s + p99 latency; achieved HBM GB/s"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_128cubed_3comp_fp64.json")
# the sources each timed kernel class is compiled from: a traffic record applies only to them
KERNEL_SOURCES = {
    "fine_pass": ("kernels_fine.hip", "device_common.hpp", "philox.hpp", "kernels.hpp"),
    "fine_pass_fp32": ("kernels_fine.hip", "device_common.hpp", "philox.hpp", "kernels.hpp"),
    "level1_block_pass": ("kernels_gal.hip", "device_common.hpp", "philox.hpp", "kernels.hpp"),
    "composite_base_pass": ("kernels_comp.hip", "composite.hpp", "device_common.hpp",
                            "philox.hpp", "kernels.hpp"),
}


def kernel_source_hash(kind):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, "paper_1003_2680_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kind, chains):
    """HBM bytes per launch of a kernel class from committed rocprofv3 counters, if they were
    taken on the current sources and the same batch; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f).get("kernels", {}).get(kind)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("sources_sha256_16") != kernel_source_hash(kind) \
            or rec.get("chains") != chains:
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(k_dec, cycles=15):
    """The CPU oracle (FP64 NumPy/SciPy, one thread) on a bounded sample of the workload."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle.mg import StochasticMG
    from oracle.philox import PhiloxNoise

    with threadpool_limits(limits=1):
        mg = StochasticMG(NX, NY, NZ, kT=1.0, levels=LEVELS)
        x = np.zeros(NX * NY * NZ)
        zero = np.zeros_like(x)
        noise = PhiloxNoise(0)
        t0 = time.perf_counter()
        for c in range(cycles):
            x = mg.vcycle(x, zero, noise, c, 0)
        dt = (time.perf_counter() - t0) / cycles
    per_field_cycle = dt * NCOMP
    return {"value": round(1.0 / per_field_cycle / k_dec, 6), "unit": "decorrelated samples/s",
            "cores": 1, "kind": "oracle", "host": host_info(),
            "sample": "%d V(2,2) cycles of one component of the 128^3 6-level FP64 chain "
                      "(%.2f s/cycle), scaled to the 3-component field; hierarchy set-up "
                      "excluded; NumPy/SciPy limited to one thread" % (cycles, dt)}


def copy_calibration(mib=1024, reps=5):
    """A plain device copy of known size, for scaling the memory-traffic counters
    (FETCH_SIZE / WRITE_SIZE) of a profiled run to bytes: each copy reads and writes mib MiB."""
    import torch
    torch.cuda.set_device(0)
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read_per_copy": n * 8,
                                           "bytes_written_per_copy": n * 8, "copies": reps}}))


def lag1(obs):
    """Lag-1 autocorrelation of each observable, pooled over components: obs [T, C, Q]."""
    import numpy as np
    o = obs - obs.mean(axis=0, keepdims=True)
    num = (o[:-1] * o[1:]).sum(axis=(0, 1))
    den = (o * o).sum(axis=(0, 1))
    return num / den


def tau_int(obs, c=5.0):
    """Integrated autocorrelation time 1 + 2 sum_k rho(k) of each observable (pooled over
    components), summed up to the first lag k >= c tau(k) (Sokal's self-consistent window)."""
    import numpy as np
    o = obs - obs.mean(axis=0, keepdims=True)
    den = (o * o).sum(axis=(0, 1))
    T = o.shape[0]
    taus = []
    for q in range(o.shape[2]):
        tau = 1.0
        for k in range(1, T // 2):
            rho = float((o[:-k, :, q] * o[k:, :, q]).sum() / den[q])
            tau += 2.0 * rho
            if k >= c * tau:
                break
        taus.append(tau)
    return np.array(taus)


def host_info():
    """The host cores the CPU baseline ran on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model,
            "threads_used": 1, "blas": "NumPy/SciPy BLAS limited to one thread"}


def run_batch(H, nchains, steps, warmup, spp, out):
    """Warm-up, then `steps` timed steps; each step is one batched call that advances every
    chain by spp cycles, emits their fields into `out` and takes the observables of every
    emitted field.  Returns (ms per step by wall clock, per-step latencies in ms, observables
    of the timed steps [steps*spp, nact, Q])."""
    import numpy as np
    import torch
    stream = torch.cuda.current_stream()
    state = torch.zeros((nchains * NCOMP, NZ, NY, NX), dtype=torch.float64, device=out.device)
    H.sample_batch(0, seeds=list(range(nchains)), comps_per_chain=NCOMP, state=state)
    for _ in range(warmup):
        H.sample_batch(spp, nchains=nchains, comps_per_chain=NCOMP, state=state, out=out,
                       with_obs=True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    obs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(stream)
        _, ob, _ = H.sample_batch(spp, nchains=nchains, comps_per_chain=NCOMP, state=state,
                                  out=out, with_obs=True)
        ev[k][1].record(stream)
        obs.append(ob)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    return wall * 1e3 / max(steps, 1), lat, torch.cat(obs).cpu().numpy(), state


def time_solves(Hsingle, Hbatch, fs, rtol):
    """Latency of one 3-component solve (and the contraction it measures), and the throughput
    of all the right-hand sides solved as one batch."""
    import torch
    u = torch.empty_like(fs[0])
    Hsingle.solve(fs[0], rtol=rtol, u=u)  # warm-up
    ratios, cyc = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in fs:
        _, c, _ = Hsingle.solve(f, rtol=rtol, u=u)
        cyc.append(c)
        ratios.append(Hsingle.last_ratio)
    torch.cuda.synchronize()
    single_s = (time.perf_counter() - t0) / len(fs)
    fb = torch.cat(fs).contiguous()
    Hbatch.solve_batch(fb, nchains=len(fs), comps_per_chain=NCOMP, rtol=rtol)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, infos = Hbatch.solve_batch(fb, nchains=len(fs), comps_per_chain=NCOMP, rtol=rtol)
    torch.cuda.synchronize()
    batch_s = time.perf_counter() - t0
    return single_s, batch_s, ratios, cyc


def measure_solves(precision, fs, rtol=1e-12):
    """Latency of one 3-component solve and the batched throughput of all right-hand sides;
    the contraction each solve measures."""
    import numpy as np
    import torch
    from paper_1003_2680_amd.api import Hierarchy
    Hs = Hierarchy(NX, NY, NZ, ncomp=NCOMP, kT=1.0, levels=LEVELS, precision=precision)
    Hb = Hierarchy(NX, NY, NZ, ncomp=NCOMP * len(fs), kT=1.0, levels=LEVELS,
                   precision=precision)
    single_s, batch_s, ratios, cyc = time_solves(Hs, Hb, fs, rtol)
    del Hs, Hb
    torch.cuda.empty_cache()
    return {"solve_single_s": single_s, "solve_batch_s": batch_s, "rho": max(ratios),
            "solve_cycles": float(np.mean(cyc))}


def measure(precision, args, dev, stride, chains, steps, timing=True,
            stream_groups=STREAM_GROUPS):
    """Sampling (and per-launch kernel times) of one precision mode: `chains` chains of the
    3-component field batched, one emitted sample every `stride` cycles."""
    import torch
    from paper_1003_2680_amd.api import Hierarchy

    C = chains
    H = Hierarchy(NX, NY, NZ, ncomp=NCOMP * C, kT=1.0, levels=LEVELS, nu1=2, nu2=2,
                  precision=precision, stride=stride, burn_in=0)
    H.set_stream_groups(stream_groups)
    out = torch.empty((SAMPLES_PER_STEP, NCOMP * C, NZ, NY, NX), dtype=torch.float64,
                      device=dev)
    ms, lat, obs, state = run_batch(H, C, steps, args.warmup, SAMPLES_PER_STEP, out)
    res = {"ms_per_step": ms, "lat": lat, "obs": obs}
    if timing:
        # per-launch kernel times: HIP events bracketing each sweep's colour passes (or the
        # bottom launch) on the batch's stream, over the same number of further steps (the
        # FP32-refined form: its FP32 level-0 colour pass only)
        cyc_timed = steps * SAMPLES_PER_STEP * stride
        kern = {}
        names = ("fine_pass", "level1_block_pass", "bottom") if precision == "fp64" \
            else ("fine_pass",)
        for name in names:
            H.kernel_timing(True, name)
            torch.cuda.synchronize()
            for _ in range(steps):
                H.sample_batch(SAMPLES_PER_STEP, nchains=C, comps_per_chain=NCOMP,
                               state=state, out=out)
            torch.cuda.synchronize()
            n_l, k_ms = H.kernel_timing_read()
            H.kernel_timing(False, name)
            kern[name] = {"launches": n_l, "avg_launch_s": k_ms / 1e3 / max(n_l, 1),
                          "per_cycle_s": k_ms / 1e3 / cyc_timed}
            if name == "level1_block_pass":
                # one or two colours per launch: 8 colour passes per sweep, 4 sweeps per cycle
                kern[name]["colours_per_launch"] = max(1, round(cyc_timed * 32 / max(n_l, 1)))
        res["kern"] = kern
    del H, out, state
    torch.cuda.empty_cache()
    return res


def measure_hbm_point(dev, dims=(512, 512, 256), cycles=10):
    """One FP64 chain on a single 512x512x256 grid (537 MB per field, beyond the 256 MB
    Infinity Cache): cycles/s of the 7-level V(2,2) cycle and the level-0 colour pass
    against the HBM roofline (8 B per cell per pass)."""
    import torch
    from paper_1003_2680_amd.api import Hierarchy
    nx, ny, nz = dims
    H = Hierarchy(nx, ny, nz, ncomp=1, kT=1.0, levels=0, nu1=2, nu2=2)
    state = torch.zeros(H.shape, dtype=torch.float64, device=dev)
    H.sample_batch(0, seeds=[0], comps_per_chain=1, state=state)
    H.sample_batch(2, nchains=1, comps_per_chain=1, state=state, emit=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H.sample_batch(cycles, nchains=1, comps_per_chain=1, state=state, emit=False)
    torch.cuda.synchronize()
    cyc_s = (time.perf_counter() - t0) / cycles
    H.kernel_timing(True, "fine_pass")
    H.sample_batch(cycles, nchains=1, comps_per_chain=1, state=state, emit=False)
    torch.cuda.synchronize()
    n_l, k_ms = H.kernel_timing_read()
    H.kernel_timing(False, "fine_pass")
    avg = k_ms / 1e3 / max(n_l, 1)
    nbytes = nx * ny * nz * 8
    ach = nbytes / avg / 1e9
    levels = H.n_levels
    del H, state
    torch.cuda.empty_cache()
    return {"workload": "%dx%dx%d, 1 component, FP64, auto depth (coarsest <= 512 unknowns), "
                        "V(2,2)" % dims,
            "levels": levels, "cycles_per_s": round(1.0 / cyc_s, 2),
            "ms_per_cycle": round(cyc_s * 1e3, 3),
            "fine_pass": {"avg_launch_us": round(avg * 1e6, 2),
                          "algorithmic_bytes_per_launch": nbytes,
                          "achieved_GBs": round(ach, 1), "frac_of_8TBs": round(ach / HBM_PEAK_GBS, 4)}}


COMP_BASE = (256, 256, 128)
COMP_BOX = (64, 192, 64, 192, 0, 32)
# sweeps of the FAC cycle: the contraction is set by the composite sweeps (nu) -- base V-cycles
# V(2,2) and V(1,0) give the same rate -- so the bench runs nu = 3 with one base pre-sweep
COMP_NU, COMP_MU1, COMP_MU2 = 3, 1, 0
# automatic base depth: coarsen while a level has more than 512 cells (8x8x4 drawn exactly)
COMP_COARSEST = 512


def composite_cpu_baseline(seconds=10.0):
    """The oracle's FAC cycle (oracle.composite, unmodified) on the 16^3-base copy of the
    adaptive workload (box [4,12)^2 x [0,4), 5888 unknowns): unknown-cycles/s on the host."""
    import numpy as np
    import threadpoolctl
    from oracle.composite import CompositeGrid, FACSampler
    from oracle.philox import PhiloxNoise
    g = CompositeGrid(16, 16, 16, (4, 12, 4, 12, 0, 4))
    fac = FACSampler(g, kT=1.0, nu=COMP_NU, mu1=COMP_MU1, mu2=COMP_MU2)
    x = np.zeros(g.n)
    zero = np.zeros(g.n)
    noise = PhiloxNoise(0)
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        x = fac.cycle(x, zero, noise, n)
        n += 1
    dt = time.perf_counter() - t0
    info = threadpoolctl.threadpool_info()
    cores = max([i.get("num_threads", 1) for i in info] + [1])
    return {"value": round(g.n * n / dt, 1), "unit": "unknown-cycles/s", "cores": cores,
            "kind": "oracle",
            "sample": "%d stochastic FAC cycles of the oracle on the 16^3-base copy (%d unknowns), "
                      "%.1f s; NumPy/SciPy sparse, BLAS threads as listed" % (n, g.n, dt)}


def measure_composite(dev, cycles=20, with_cpu=True):
    """Spatially adaptive composite grid: 256x256x128 base, box [64,192)^2 x [0,32) refined by
    two (12.06 M unknowns), stochastic FAC cycle (COMP_NU composite sweeps, base V-cycle
    V(COMP_MU1, COMP_MU2)), FP64."""
    import numpy as np
    import torch
    from paper_1003_2680_amd.composite import CompositeSampler
    from paper_1003_2680_amd.inputs import gaussian_field
    t0 = time.perf_counter()
    S = CompositeSampler(*COMP_BASE, COMP_BOX, kT=1.0, nu=COMP_NU, mu1=COMP_MU1, mu2=COMP_MU2,
                         coarsest_max=COMP_COARSEST)
    plan_s = time.perf_counter() - t0
    info = S.info
    xc, xf = S.zeros()
    S.sample(xc, xf, 5, seed=0, first_cycle=0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    S.sample(xc, xf, cycles, seed=0, first_cycle=5)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / cycles
    rc, rf = S.residual(xc, xf)
    energy = -(xc.reshape(-1) @ rc.reshape(-1) + xf.reshape(-1) @ rf.reshape(-1)).item()
    n = int(info.unknowns)
    fc = torch.from_numpy(gaussian_field(S.base_shape, 7)).to(dev)
    ff = torch.from_numpy(gaussian_field(S.fine_shape, 8)).to(dev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, _, si = S.solve(fc, ff, rtol=1e-10, max_cycles=60)
    solve_s = time.perf_counter() - t1
    rho = max(float(si.last_ratio), 1e-3)
    k_dec = max(1, math.ceil(math.log(0.01) / math.log(rho)))
    # dominant kernel: the block colour pass of the finest base level (A_0 = P^T A P on
    # 256x256x128), timed live on the stream it runs on
    nb = info.dims[0][0] * info.dims[0][1] * info.dims[0][2]
    x0 = torch.from_numpy(gaussian_field((nb,), 9)).to(dev)
    b0 = torch.from_numpy(gaussian_field((nb,), 10)).to(dev)
    S.debug_base_pass(0, 0, x0, b0, seed=1, cycle=0)
    reps = 10
    torch.cuda.synchronize()
    e0.record()
    for r in range(reps):
        for c in range(8):
            S.debug_base_pass(0, c, x0, b0, seed=1, cycle=r, slot=0)
    e1.record()
    torch.cuda.synchronize()
    avg_s = e0.elapsed_time(e1) / 1e3 / (8 * reps)
    # algorithmic bytes of one colour pass: x of the three neighbouring block colours (3/8 of
    # the level), b and x of this colour's cells (read b, write x: 2/8), 8 B per value
    nbytes = nb * 8 * 5 // 8
    ach = nbytes / avg_s / 1e9
    # the field noise of Appendix A, w = L^-1 Q eta with q = 1 (a draw: the Philox forcing, then
    # a FAC solve of A w = -(volume / h^3) q eta from zero to rtol 1e-8)
    S.forced_field(1, 11, 0, rtol=1e-8, max_cycles=60)
    torch.cuda.synchronize()
    n_draws = 4
    t2 = time.perf_counter()
    _, _, finfos = S.forced_field(n_draws, 11, 1, rtol=1e-8, max_cycles=60)
    torch.cuda.synchronize()
    draw_s = (time.perf_counter() - t2) / n_draws
    forced = {"rtol": 1e-8, "ms_per_draw": round(draw_s * 1e3, 3),
              "draws_per_s": round(1.0 / draw_s, 2),
              "cycles_per_draw": round(sum(i.cycles for i in finfos) / n_draws, 2),
              "q": "1 on every cell (L^-1 C not symmetric: the composite mesh's L = M^-1 S)"}
    out = {
        "workload": "adaptive composite grid: 256x256x128 base (periodic x,y; no-slip z walls) "
                    "with the box [64,192)^2 x [0,32) refined by two; FAC cycle nu=%d, base "
                    "V(%d,%d) on Galerkin levels, exact coarsest (<= %d unknowns); FP64" % (
                        COMP_NU, COMP_MU1, COMP_MU2, COMP_COARSEST),
        "unknowns": n, "base_levels": [list(info.dims[l]) for l in range(info.n_levels)],
        "distinct_rows_per_level": list(info.stencils[:info.n_levels]),
        "plan_s": round(plan_s, 2),
        "ms_per_cycle": round(ms, 3), "cycles_per_s": round(1e3 / ms, 2),
        "unknown_cycles_per_s": float("%.4e" % (n * 1e3 / ms)),
        "rho_solve": round(rho, 4), "k_dec": k_dec,
        "decorrelated_samples_per_s": round(1e3 / ms / k_dec, 3),
        "solve_ms": round(solve_s * 1e3, 2), "solve_cycles": int(si.cycles),
        "solve_relres": float("%.3e" % si.relres),
        "energy_over_n_kT": round(energy / n, 5),
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("composite_base_pass", 1),
                     "kernel": "k_gblock_pass (block colour pass, finest base level)",
                     "avg_launch_us": round(avg_s * 1e6, 2),
                     "algorithmic_bytes_per_launch": nbytes},
        "forced_field": forced,
    }
    del S, xc, xf, rc, rf, x0, b0
    torch.cuda.empty_cache()
    # FP32-refined form of the same cycle (FP32 sweeps and transfers, FP64 residual, update and
    # coarsest draw), same noise streams; its error against the FP64 form after two cycles
    S64 = CompositeSampler(*COMP_BASE, COMP_BOX, kT=1.0, nu=COMP_NU, mu1=COMP_MU1, mu2=COMP_MU2,
                           coarsest_max=COMP_COARSEST)
    a, af = S64.zeros()
    S64.sample(a, af, 2, seed=0)
    del S64
    S32 = CompositeSampler(*COMP_BASE, COMP_BOX, kT=1.0, nu=COMP_NU, mu1=COMP_MU1, mu2=COMP_MU2,
                           coarsest_max=COMP_COARSEST, precision="fp32_refined")
    b_, bf_ = S32.zeros()
    S32.sample(b_, bf_, 2, seed=0)
    num = ((a - b_).square().sum() + (af - bf_).square().sum()).item()
    den = (a.square().sum() + af.square().sum()).item()
    del a, af
    S32.sample(b_, bf_, 3, seed=0, first_cycle=2)
    torch.cuda.synchronize()
    e0.record()
    S32.sample(b_, bf_, cycles, seed=0, first_cycle=5)
    e1.record()
    torch.cuda.synchronize()
    ms32 = e0.elapsed_time(e1) / cycles
    _, _, si32 = S32.solve(fc, ff, rtol=1e-10, max_cycles=60)
    rho32 = max(float(si32.last_ratio), 1e-3)
    k32 = max(1, math.ceil(math.log(0.01) / math.log(rho32)))
    out["fp32_refined"] = {"ms_per_cycle": round(ms32, 3), "cycles_per_s": round(1e3 / ms32, 2),
                           "rho_solve": round(rho32, 4), "k_dec": k32,
                           "decorrelated_samples_per_s": round(1e3 / ms32 / k32, 3),
                           "solve_cycles": int(si32.cycles),
                           "rel_rms_vs_fp64_2_cycles": float("%.3e" % math.sqrt(num / den))}
    del S32, b_, bf_, fc, ff
    torch.cuda.empty_cache()
    if with_cpu:
        out["cpu_baseline"] = composite_cpu_baseline()
    return out


def measure_batched(dev, n_instances=64, n_samples=100):
    """64 uneven instances ({32,48,64,96}^3 drawn by seed), tuned per grid: 100 samples
    (float32, in HBM) and one solve to 1e-10 per instance.  The FP32-refined form through the
    library's batch call (cycles in step, the small levels of all instances in merged
    launches), eager and as one replayed graph; the same through one stream per grid group;
    the batched plain FP64 form at the same configuration and solve tolerance; and the
    refined form's error against FP64 on the same streams."""
    import numpy as np
    import torch
    from paper_1003_2680_amd.api import Hierarchy
    from paper_1003_2680_amd.batch import BatchRunner, Instance
    from paper_1003_2680_amd.inputs import batched_sizes, gaussian_field_device

    sizes = batched_sizes(n_instances)
    insts = [Instance((e, e, e), seed=1000 + i) for i, e in enumerate(sizes)]

    def timed_sample(R, emit=True):
        R.start()
        R.sample(2, emit=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = R.sample(n_samples, out_dtype=torch.float32, emit=emit)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        del outs
        return dt

    def timed_solve(R):
        fs = {i: gaussian_field_device(inst.dims[::-1], 2000 + i, dev)
              for i, inst in enumerate(insts)}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        us, infos = R.solve(fs, rtol=1e-10)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        cyc = max(v[0] for v in infos.values())
        del us, fs
        return dt, cyc

    t0 = time.perf_counter()
    R = BatchRunner(insts, precision="fp32_refined", tune=True, device=dev,
                    stream_groups=STREAM_GROUPS)
    tune_s = time.perf_counter() - t0
    configs = R.configs
    sample_s = timed_sample(R)
    R.capture(n_samples)
    R.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    R.replay()
    torch.cuda.synchronize()
    graph_s = time.perf_counter() - t0
    solve_s, solve_cyc = timed_solve(R)
    cells = R.cells()
    del R
    torch.cuda.empty_cache()
    Rs = BatchRunner(insts, precision="fp32_refined", configs=configs, device=dev,
                     engine="streams")
    streams_s = timed_sample(Rs)
    del Rs
    torch.cuda.empty_cache()
    R64 = BatchRunner(insts, precision="fp64", configs=configs, device=dev,
                      stream_groups=STREAM_GROUPS)
    fp64_s = timed_sample(R64)
    fp64_solve_s, fp64_solve_cyc = timed_solve(R64)
    del R64
    torch.cuda.empty_cache()
    cfgs = {"%dx%dx%d" % d: {k: (round(v, 6) if isinstance(v, float) else v)
                             for k, v in c.items() if k != "table"}
            for d, c in configs.items()}
    # plain FP64 form, one instance at a time (10 cycles each, scaled to n_samples cycles)
    plain_s = 0.0
    err = {}
    for e in sorted(set(sizes)):
        H = Hierarchy(e, e, e, ncomp=1, levels=0)
        st = H.new_state()
        o = torch.empty((10,) + H.shape, dtype=torch.float64, device=dev)
        H.sample(2, 1, state=st, out=o[:2])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H.sample(10, 1, first_cycle=2, state=st, out=o)
        torch.cuda.synchronize()
        per_cycle = (time.perf_counter() - t0) / 10
        plain_s += per_cycle * n_samples * sizes.count(e)
        # refined vs FP64 error on the same Philox stream (2 cycles from zero), same config
        H32 = Hierarchy(e, e, e, ncomp=1, levels=0, precision="fp32_refined")
        a, _ = Hierarchy(e, e, e, ncomp=1, levels=0).sample(2, 5)
        b, _ = H32.sample(2, 5)
        err["%d^3" % e] = float("%.3e" % float(((a - b).norm() / a.norm()).item()))
        del H, H32, a, b, o, st
    torch.cuda.empty_cache()
    # algorithmic bytes per cell-cycle of the sample cycle: ~106 (FP32-refined) and ~108.6
    # (FP64) bytes per cell
    def roof(seconds, bpc):
        ach = cells * n_samples * bpc / seconds / 1e9
        return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "bytes_per_cell_cycle": bpc}
    return {"workload": "%d instances, grids {32,48,64,96}^3 drawn by seed 2026, scalar, "
                        "tuned per grid" % n_instances,
            "cells": cells, "groups": len(cfgs), "configs": cfgs,
            "tune_s": round(tune_s, 2),
            "fp32_refined": {
                "engine": "smg_batch_run (%d staggered stream groups, merged bottom launches "
                          "within a group)" % STREAM_GROUPS,
                "instance_samples_per_s": round(n_instances * n_samples / sample_s, 1),
                "sample_s": round(sample_s, 4),
                "graph_replay_cycles_s": round(graph_s, 4),
                "per_group_streams_sample_s": round(streams_s, 4),
                "solve_all_s": round(solve_s, 4), "solve_cycles_max": solve_cyc,
                "roofline": roof(sample_s, 106.0),
                "roofline_graph": roof(graph_s, 106.0)},
            "fp64": {
                "engine": "smg_batch_run (%d staggered stream groups, merged bottom launches "
                          "within a group)" % STREAM_GROUPS,
                "instance_samples_per_s": round(n_instances * n_samples / fp64_s, 1),
                "sample_s": round(fp64_s, 4),
                "solve_all_s": round(fp64_solve_s, 4), "solve_cycles_max": fp64_solve_cyc,
                "roofline": roof(fp64_s, 108.6)},
            "equal_accuracy": "both solve to 1e-10; samples of the refined form differ from the "
                              "FP64 form on the same streams by the relative RMS below",
            "plain_fp64_sequential_s_est": round(plain_s, 3),
            "speedup_refined_vs_plain_fp64_sequential": round(plain_s / sample_s, 2),
            "refined_rel_rms_vs_fp64_2_cycles": err}


def measure_selm(dev, dims=(128, 128, 128), m=64, steps=10):
    """SELM coupling on the 128^3 channel with m structure points (Peskin 4-point coupling,
    projection through the multigrid solve): mobility H F, driving field g (the stochastic
    multigrid chain, stride 2) and Euler-Maruyama steps of a harmonic bead chain."""
    import numpy as np
    import torch
    from paper_1003_2680_amd.selm import SELM
    S = SELM(*dims, mu=1.0, kT=1.0, stride=2, max_points=m, device=dev)
    rng = np.random.default_rng(8)
    X0 = np.column_stack([rng.uniform(0, dims[0], m), rng.uniform(0, dims[1], m),
                          rng.uniform(4.0, dims[2] - 4.0, m)])
    X = torch.from_numpy(X0).to(dev)
    x0 = X.clone()
    F = torch.from_numpy(rng.standard_normal((m, 3))).to(dev)
    state = S.new_state()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_mob = timed(lambda: S.mobility(X, F, rtol=1e-10), 3)
    cyc = [0]

    def drv():
        S.drive(X, 5, cyc[0], state, rtol=1e-10)
        cyc[0] += 2
    t_drv = timed(drv, 3)
    k = [0]

    def stp():
        S.step(X, -1.0 * (X - x0), 0.5, 7, k[0], state, rtol=1e-10)
        k[0] += 1
    t_step = timed(stp, steps)
    del S, state
    torch.cuda.empty_cache()
    return {"workload": "SELM coupling: %dx%dx%d wall-bounded channel, 3-component Stokes "
                        "velocity, %d structure points, FP64, solves to 1e-10" % (dims + (m,)),
            "mobility_ms": round(t_mob * 1e3, 3), "drive_ms": round(t_drv * 1e3, 3),
            "em_step_ms": round(t_step * 1e3, 3), "em_steps_per_s": round(1.0 / t_step, 2)}


def measure_serving(dev, stride, rate=200.0, n=300):
    """Poisson arrivals (seed 7) of sample (k ~ U{1..16}, stride = burn-in = k_dec) and solve
    (1e-10) requests on grids nx = ny in {32..256}, nz in {16..128}, FP32-refined, 32 GB HBM
    budget, 16 chain slots per pool."""
    import numpy as np
    import torch
    from paper_1003_2680_amd.inputs import gaussian_field_device
    from paper_1003_2680_amd.serve import Server, make_requests, simulate

    srv = Server(budget_bytes=32 << 30, slots=16, stride=stride, precision="fp32_refined",
                 device=dev)
    reqs = make_requests(n, rate, seed=7)
    ok, wall, lat = simulate(srv, reqs, lambda r: gaussian_field_device(r.dims[::-1], r.seed, dev),
                             timeout=150.0)
    errors = sum(1 for r in srv.done if r.error)
    pools = len(srv.pools) + srv.evictions
    srv.shutdown()
    torch.cuda.empty_cache()
    return {"rate_req_s": rate, "requests": n, "completed": len(lat), "errors": errors,
            "all_completed": bool(ok), "throughput_req_s": round(len(lat) / wall, 2),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
            "pools_created": pools, "evictions": srv.evictions,
            "latency_from": "scheduled Poisson arrival",
            "max_submit_lag_ms": round(srv.max_submit_lag * 1e3, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=125)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--solves", type=int, default=10)
    ap.add_argument("--chains", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-refined", action="store_true",
                    help="skip the FP32-refined measurement")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 64-instance batched measurement")
    ap.add_argument("--no-hbm-point", action="store_true",
                    help="skip the single 512x512x256 grid (beyond the Infinity Cache)")
    ap.add_argument("--no-selm", action="store_true",
                    help="skip the SELM coupling leg")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving-loop measurement")
    ap.add_argument("--no-composite", action="store_true",
                    help="skip the adaptive composite-grid leg")
    ap.add_argument("--composite-only", action="store_true",
                    help="only run the adaptive composite-grid leg (prints its object)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only run the 64-instance batched leg (prints its object)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the sampler chains (128^3, 3 components) "
              "are single-device jobs here; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.batched_only:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"batched": measure_batched(torch.device("cuda", 0))}), flush=True)
        return
    if args.composite_only:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"composite": measure_composite(torch.device("cuda", 0),
                                                         with_cpu=not args.no_cpu_baseline)}),
              flush=True)
        return

    import numpy as np
    import torch
    from paper_1003_2680_amd.api import Hierarchy
    from paper_1003_2680_amd.inputs import gaussian_field

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    C = max(1, args.chains)
    shape = (NCOMP, NZ, NY, NX)
    fs = [torch.from_numpy(gaussian_field(shape, 100 + i)).to(dev)
          for i in range(max(args.solves, 1))]

    # the contraction of the cycle, measured by the deterministic solves, fixes the stride of
    # decorrelated samples: the lag-k correlation of the chain is R^k applied to its stationary
    # covariance, so k_dec = ceil(ln 0.01 / ln rho) cycles separate nearly independent draws
    s64 = measure_solves("fp64", fs)
    rho_solve = s64["rho"]
    k_dec = max(1, math.ceil(math.log(0.01) / math.log(rho_solve)))
    r64 = measure("fp64", args, dev, k_dec, C, args.steps)
    r64.update(s64)
    progress("fp64 sampling, kernel timing and solves done")
    # every emitted sample is k_dec cycles after the previous one: its observables' lag-1
    # correlation is the chain's lag-k_dec correlation, which must be below 0.01 up to the
    # estimate's standard error
    rho_obs = lag1(r64["obs"])
    n_obs = r64["obs"].shape[0] * r64["obs"].shape[1]
    se_obs = 1.0 / math.sqrt(n_obs)
    decor = {"lag": k_dec, "max_abs_lag_corr": round(float(np.max(np.abs(rho_obs))), 4),
             "bound": 0.01, "standard_error": round(se_obs, 4),
             "ok": bool(float(np.max(np.abs(rho_obs))) <= 0.01 + 3.0 * se_obs)}
    value = C * SAMPLES_PER_STEP / (r64["ms_per_step"] / 1e3)
    samples_per_s = value
    cycles_per_s = value * k_dec / C
    # one chain: its three components stay on one stream (splitting them measured no faster)
    r1 = measure("fp64", args, dev, k_dec, 1, max(10, args.steps // 4), timing=False,
                 stream_groups=1)
    progress("single 3-component chain done")

    N0 = NX * NY * NZ
    N1 = N0 // 8
    nact = NCOMP * C
    kern = r64["kern"]

    def roof(k, name, nbytes, traffic=None):
        ach = nbytes / k["avg_launch_s"] / 1e9
        return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": name,
                "avg_launch_us": round(k["avg_launch_s"] * 1e6, 3),
                "launches_timed": int(k["launches"]), "algorithmic_bytes_per_launch": nbytes,
                "us_per_cycle": round(k["per_cycle_s"] * 1e6, 1)}

    # level-0 colour pass (b = 0): read the other colour, write this colour, 8 B per value
    fine = roof(kern["fine_pass"], "k_rb_pass (level-0 colour pass, 128^3)", nact * N0 * 8)
    fine["traffic"] = measured_traffic("fine_pass", C)
    # level-1 block colour pass: read x of the whole level, b and the noise of this colour's
    # cells, write x of this colour's cells: N1 * 8 B * (1 + 3/8) per colour; a launch of two
    # colours (k_block_pair) reads x once and b, noise and writes for both: N1 * 8 B * (1 + 6/8)
    cpl = kern["level1_block_pass"].get("colours_per_launch", 1)
    if cpl == 2:
        blk = roof(kern["level1_block_pass"],
                   "k_block_pair (two level-1 block colour passes per launch, 64^3)",
                   nact * N1 * 8 * 14 // 8)
    else:
        blk = roof(kern["level1_block_pass"], "k_block_tile (level-1 block colour pass, 64^3)",
                   nact * N1 * 8 * 11 // 8)
    blk["traffic"] = measured_traffic("level1_block_pass", C)
    # the dominant kernel class by GPU time per cycle carries `roofline`
    dominant = max((fine, blk), key=lambda r: r["us_per_cycle"])
    other = blk if dominant is fine else fine
    lat = r64["lat"]
    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "decorrelated samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(r64["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "128x128x128 wall-bounded cell-centred Laplacian (periodic x,y; "
                               "no-slip z walls), 3-component field, 6-level stochastic "
                               "V(2,2) cycle, FP64; the chains of seeds 0..%d batched into "
                               "every launch, in %d groups on streams of their own"
                               % (C - 1, STREAM_GROUPS),
                   "grid": [NX, NY, NZ], "ncomp": NCOMP, "levels": LEVELS, "nu": [2, 2],
                   "chains": C, "stream_groups": STREAM_GROUPS,
                   "samples_per_step": C * SAMPLES_PER_STEP, "k_dec": k_dec,
                   "cycles_per_step": SAMPLES_PER_STEP * k_dec},
        "samples_per_s": round(samples_per_s, 2),
        "emission": "one sample per chain every k_dec cycles (each emitted sample is a "
                    "decorrelated one); value = emitted samples/s",
        "cycles_per_s_3comp": round(cycles_per_s, 2),
        "p50_ms": round(float(np.percentile(lat, 50)), 4),
        "p99_ms": round(float(np.percentile(lat, 99)), 4),
        "rho_solve": round(rho_solve, 5),
        "decorrelation_check": decor,
        "obs_lag1_of_emitted": [round(float(v), 4) for v in rho_obs],
        "tau_int_obs_emitted": [round(float(v), 3) for v in tau_int(r64["obs"])],
        "single_instance": {
            "workload": "one chain of the 3-component 128^3 field (no batching of chains)",
            "value": round(SAMPLES_PER_STEP / (r1["ms_per_step"] / 1e3), 3),
            "ms_per_step": round(r1["ms_per_step"], 4),
            "p99_ms": round(float(np.percentile(r1["lat"], 99)), 4)},
        "cycle_roofline": {
            "bound": "hbm", "bytes_per_component_cycle": round(108.6 * N0),
            "achieved": round(cycles_per_s * C * NCOMP * 108.6 * N0 / 1e9, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(cycles_per_s * C * NCOMP * 108.6 * N0 / 1e9 / HBM_PEAK_GBS, 4),
            "model": "read and write x once per sweep on every level, b where present, the "
                     "level-0 transfers (108.6 N bytes per FP64 component-cycle); emission "
                     "time included"},
        "solves_per_s": round(len(fs) / r64["solve_batch_s"], 3),
        "solve_ms_single": round(r64["solve_single_s"] * 1e3, 3),
        "solve_cycles": round(r64["solve_cycles"], 2),
        "roofline": dominant,
        "roofline_other": other,
        "bottom_kernel": {"kernel": "k_bottom (LDS-resident levels 16^3..4^3, one work-group "
                                    "per component)",
                          "avg_launch_us": round(kern["bottom"]["avg_launch_s"] * 1e6, 1),
                          "us_per_cycle": round(kern["bottom"]["per_cycle_s"] * 1e6, 1)},
    }

    # ---- FP32-refined form of the same workload (same streams, same k_dec)
    if not args.no_refined:
        H64 = Hierarchy(NX, NY, NZ, ncomp=NCOMP, kT=1.0, levels=LEVELS)
        H32 = Hierarchy(NX, NY, NZ, ncomp=NCOMP, kT=1.0, levels=LEVELS, precision="fp32_refined")
        a, _ = H64.sample(2, seed=0)
        b, _ = H32.sample(2, seed=0)
        rel_rms = float(((a - b).norm() / a.norm()).item())
        del H64, H32, a, b
        torch.cuda.empty_cache()
        r32 = measure("fp32_refined", args, dev, k_dec, C, args.steps)
        r32.update(measure_solves("fp32_refined", fs))
        progress("fp32-refined form done")
        r_sps = C * SAMPLES_PER_STEP / (r32["ms_per_step"] / 1e3)
        line["fp32_refined"] = {
            "value": round(r_sps, 3), "samples_per_s": round(r_sps, 2),
            "ms_per_step": round(r32["ms_per_step"], 4),
            "p50_ms": round(float(np.percentile(r32["lat"], 50)), 4),
            "p99_ms": round(float(np.percentile(r32["lat"], 99)), 4),
            "solves_per_s": round(len(fs) / r32["solve_batch_s"], 3),
            "solve_ms_single": round(r32["solve_single_s"] * 1e3, 3),
            "solve_cycles": round(r32["solve_cycles"], 2),
            "rho_solve": round(r32["rho"], 5),
            "obs_lag1_of_emitted_max": round(float(np.max(np.abs(lag1(r32["obs"])))), 4),
            "rel_rms_vs_fp64_2_cycles": float("%.3e" % rel_rms)}
        # the FP32 level-0 colour pass of the inner cycle (b = the FP32 residual): read the
        # other colour and this colour's b, write this colour, 4 B per value
        line["fp32_refined"]["roofline"] = roof(
            r32["kern"]["fine_pass"], "k_rb_pass (FP32 level-0 colour pass, 128^3, with b)",
            nact * N0 * 4 * 3 // 2, measured_traffic("fine_pass_fp32", C))

    if not args.no_hbm_point:
        line["hbm_point"] = measure_hbm_point(dev)
        progress("512x512x256 HBM point done")
    if not args.no_composite:
        line["composite"] = measure_composite(dev, with_cpu=not args.no_cpu_baseline)
        progress("adaptive composite grid done")
    if not args.no_batched:
        line["batched"] = measure_batched(dev)
        progress("batched instances done")
    if not args.no_selm:
        line["selm"] = measure_selm(dev)
        progress("SELM coupling done")
    if not args.no_serving:
        line["serving"] = measure_serving(dev, stride=k_dec)
        progress("serving done")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(k_dec)
        progress("cpu baseline done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
