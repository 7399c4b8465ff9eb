"""Benchmark: decorrelated 128^3 field samples/s of the stochastic multigrid sampler on one GPU.

Workload: a 128x128x128 cell-centred grid (h = 1, kT = 1), periodic in x and y with no-slip
walls on the z faces; a 3-component velocity field (three decoupled scalar chains with the
same wall-bounded Laplacian); the 6-level stochastic V(2,2) cycle in FP64 (red-black heat
bath on the fine level, 2x2x2 block heat bath on the Galerkin levels, exact Cholesky draw on
the 4^3 coarsest level).  The chains of seeds 0..CHAINS-1 run concurrently, one hierarchy
and one HIP stream each (the small coarse levels of one chain overlap the bandwidth-bound fine
sweeps of another).  One step = one smg_sample_field call per chain that runs
SAMPLES_PER_STEP cycles and writes every cycle's 3-component field to an output buffer in HBM.

value = decorrelated samples/s = emitted samples/s / k_dec with
k_dec = max(1, ceil(ln 0.01 / ln rho)), rho the measured contraction of the deterministic
cycle (the paper ties the decorrelation of the stochastic iteration to the deterministic
convergence rate: the lag-k correlation is R^k applied to the initial covariance).
Also reported: per-step p50/p99 latency, 10 solves to 1e-12 (solves/s), the roofline of the
fine colour-pass kernel, and the CPU oracle on a bounded sample of the same workload.

The FP32-refined form of the same workload (FP32 sweeps and transfers, FP64 residual,
correction and coarsest arithmetic) is measured beside it under "fp32_refined", with its
relative RMS difference from the FP64 chain on the same Philox streams.

Run: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-refined]
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

NX = NY = NZ = 128
NCOMP = 3
LEVELS = 6
SAMPLES_PER_STEP = 8
HBM_PEAK_GBS = 8000.0
METRIC = "decorrelated 128³ field samples/s + p99 latency; achieved HBM GB/s"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rb_pass_128cubed_3comp_traffic.json")


def kernel_source_hash():
    with open(os.path.join(ROOT, "paper_1003_2680_amd", "csrc", "kernels_fine.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(bytes_per_launch):
    """HBM bytes per fine colour-pass launch from committed rocprofv3 counters, if they were
    taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernels_hip_sha256_16") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(k_dec, cycles=3):
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
            "cores": 1, "kind": "oracle",
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


def run_chains(Hs, states, outs, streams, steps, warmup, first_cycle, samples_per_step):
    """Warm-up, then `steps` timed steps of every chain on its own stream.  Returns
    (ms per step by wall clock, per-step latencies in ms, next cycle)."""
    import numpy as np
    import torch
    stream = torch.cuda.current_stream()

    def step(first):
        for i, H in enumerate(Hs):
            streams[i].wait_stream(stream)
            with torch.cuda.stream(streams[i]):
                H.sample(samples_per_step, seed=i, first_cycle=first, state=states[i],
                         out=outs[i])
        for i in range(len(Hs)):
            stream.wait_stream(streams[i])

    cycle = first_cycle
    for _ in range(warmup):
        step(cycle)
        cycle += samples_per_step
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(stream)
        step(cycle)
        ev[k][1].record(stream)
        cycle += samples_per_step
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    return wall * 1e3 / max(steps, 1), lat, cycle


def time_solves(H, fs, u, rtol):
    import torch
    H.solve(fs[0], rtol=rtol, u=u)  # warm-up
    ratios, cyc = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in fs:
        _, c, _ = H.solve(f, rtol=rtol, u=u)
        cyc.append(c)
        ratios.append(H.last_ratio)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / len(fs), ratios, cyc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--solves", type=int, default=10)
    ap.add_argument("--chains", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-refined", action="store_true",
                    help="skip the FP32-refined measurement")
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
    u = torch.empty(shape, dtype=torch.float64, device=dev)
    streams = [torch.cuda.Stream(device=dev) for _ in range(C)]

    # ---- FP64: deterministic contraction -> k_dec; solves/s; sampling
    Hs = [Hierarchy(NX, NY, NZ, ncomp=NCOMP, kT=1.0, levels=LEVELS, nu1=2, nu2=2)
          for _ in range(C)]
    H = Hs[0]
    solve_s, ratios, cyc = time_solves(H, fs, u, 1e-12)
    rho = max(ratios)
    k_dec = max(1, math.ceil(math.log(0.01) / math.log(rho)))
    states = [h.new_state() for h in Hs]
    outs = [torch.empty((SAMPLES_PER_STEP,) + shape, dtype=torch.float64, device=dev)
            for _ in range(C)]
    ms_per_step, lat, cycle = run_chains(Hs, states, outs, streams, args.steps, args.warmup, 0,
                                         SAMPLES_PER_STEP)

    # ---- per-launch kernel times: HIP events (on the chain's own stream) around every launch
    # of one kernel class while chain 0 runs alone (the same steps again, so that a launch's
    # time is not shared with other chains)
    def timed(kernel):
        nonlocal cycle
        H.kernel_timing(True, kernel)
        torch.cuda.synchronize()
        for k in range(args.steps):
            H.sample(SAMPLES_PER_STEP, seed=0, first_cycle=cycle, state=states[0], out=outs[0])
            cycle += SAMPLES_PER_STEP
        torch.cuda.synchronize()
        n_launch, k_ms = H.kernel_timing_read()
        H.kernel_timing(False, kernel)
        return n_launch, k_ms / 1e3 / max(n_launch, 1)

    N0 = NX * NY * NZ
    N1 = N0 // 8
    cyc_timed = args.steps * SAMPLES_PER_STEP
    kern = {}
    # level-0 colour pass (b = 0): read the other colour, write this colour, 8 B per value
    n_l, t_l = timed("fine_pass")
    kern["fine_pass"] = {"kernel": "k_rb_pass (level-0 colour pass, 128^3)", "launches": n_l,
                         "avg_launch_s": t_l, "bytes": NCOMP * N0 * 8,
                         "per_cycle_s": t_l * n_l / cyc_timed}
    # level-1 block colour pass: read x of the whole level, b and the noise of this colour's
    # cells, write x of this colour's cells: N1 * 8 B * (1 + 3/8)
    n_l, t_l = timed("level1_block_pass")
    kern["level1_block_pass"] = {"kernel": "k_block_tile (level-1 block colour pass, 64^3)",
                                 "launches": n_l, "avg_launch_s": t_l,
                                 "bytes": NCOMP * N1 * 8 * 11 // 8,
                                 "per_cycle_s": t_l * n_l / cyc_timed}
    n_l, t_l = timed("bottom")
    kern["bottom"] = {"kernel": "k_bottom (LDS-resident levels 16^3..4^3, one work-group per "
                                "component)", "launches": n_l, "avg_launch_s": t_l,
                      "per_cycle_s": t_l * n_l / cyc_timed}

    def roof(k, traffic=None):
        ach = k["bytes"] / k["avg_launch_s"] / 1e9
        return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": k["kernel"],
                "avg_launch_us": round(k["avg_launch_s"] * 1e6, 3),
                "launches_timed": int(k["launches"]), "algorithmic_bytes_per_launch": k["bytes"],
                "us_per_cycle": round(k["per_cycle_s"] * 1e6, 1)}

    samples_per_s = C * SAMPLES_PER_STEP / (ms_per_step / 1e3)
    value = samples_per_s / k_dec
    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "decorrelated samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "128x128x128 wall-bounded cell-centred Laplacian (periodic x,y; "
                               "no-slip z walls), 3-component field, 6-level stochastic "
                               "V(2,2) cycle, FP64, chains of seeds 0..%d run concurrently" % (C - 1),
                   "grid": [NX, NY, NZ], "ncomp": NCOMP, "levels": LEVELS, "nu": [2, 2],
                   "chains": C, "samples_per_step": C * SAMPLES_PER_STEP, "k_dec": k_dec},
        "samples_per_s": round(samples_per_s, 2),
        "p50_ms": round(float(np.percentile(lat, 50)), 4),
        "p99_ms": round(float(np.percentile(lat, 99)), 4),
        "rho": round(rho, 5),
        "solves_per_s": round(1.0 / solve_s, 3),
        "solve_cycles": int(round(float(np.mean(cyc)))),
        # dominant kernel class by GPU time per cycle (rocprofv3: k_block_tile); the
        # LDS-resident bottom launch has no HBM roofline (its fields never leave LDS)
        "roofline": roof(kern["level1_block_pass"]),
        "roofline_fine_pass": roof(kern["fine_pass"],
                                   measured_traffic(kern["fine_pass"]["bytes"])),
        "bottom_kernel": {"kernel": kern["bottom"]["kernel"],
                          "avg_launch_us": round(kern["bottom"]["avg_launch_s"] * 1e6, 1),
                          "us_per_cycle": round(kern["bottom"]["per_cycle_s"] * 1e6, 1)},
    }
    del Hs, H, states, outs
    torch.cuda.empty_cache()

    # ---- FP32-refined form of the same workload (same streams, same k_dec)
    if not args.no_refined:
        Rs = [Hierarchy(NX, NY, NZ, ncomp=NCOMP, kT=1.0, levels=LEVELS, nu1=2, nu2=2,
                        precision="fp32_refined") for _ in range(C)]
        r_solve_s, r_ratios, r_cyc = time_solves(Rs[0], fs, u, 1e-12)
        # error against the FP64 chain on the same Philox streams (2 cycles from zero)
        H64 = Hierarchy(NX, NY, NZ, ncomp=NCOMP, kT=1.0, levels=LEVELS)
        a, _ = H64.sample(2, seed=0)
        b, _ = Rs[0].sample(2, seed=0)
        rel_rms = float(((a - b).norm() / a.norm()).item())
        del H64, a, b
        r_states = [h.new_state() for h in Rs]
        r_outs = [torch.empty((SAMPLES_PER_STEP,) + shape, dtype=torch.float64, device=dev)
                  for _ in range(C)]
        r_ms, r_lat, _ = run_chains(Rs, r_states, r_outs, streams, args.steps, args.warmup, 0,
                                    SAMPLES_PER_STEP)
        r_sps = C * SAMPLES_PER_STEP / (r_ms / 1e3)
        line["fp32_refined"] = {
            "value": round(r_sps / k_dec, 3), "samples_per_s": round(r_sps, 2),
            "ms_per_step": round(r_ms, 4),
            "p50_ms": round(float(np.percentile(r_lat, 50)), 4),
            "p99_ms": round(float(np.percentile(r_lat, 99)), 4),
            "solves_per_s": round(1.0 / r_solve_s, 3),
            "solve_cycles": int(round(float(np.mean(r_cyc)))),
            "rho": round(max(r_ratios), 5),
            "rel_rms_vs_fp64_2_cycles": float("%.3e" % rel_rms)}
        del Rs, r_states, r_outs
        torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(k_dec)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
