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

Run: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--solves", type=int, default=10)
    ap.add_argument("--chains", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the sampler chains (128^3, 3 components) "
              "are single-device jobs here; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1003_2680_amd.api import Hierarchy
    from paper_1003_2680_amd.inputs import gaussian_field

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    C = max(1, args.chains)
    Hs = [Hierarchy(NX, NY, NZ, ncomp=NCOMP, kT=1.0, levels=LEVELS, nu1=2, nu2=2)
          for _ in range(C)]
    H = Hs[0]
    states = [h.new_state() for h in Hs]
    outs = [torch.empty((SAMPLES_PER_STEP,) + H.shape, dtype=torch.float64, device=dev)
            for _ in range(C)]
    streams = [torch.cuda.Stream(device=dev) for _ in range(C)]
    stream = torch.cuda.current_stream()

    def step(first):
        for i in range(C):
            streams[i].wait_stream(stream)
            with torch.cuda.stream(streams[i]):
                Hs[i].sample(SAMPLES_PER_STEP, seed=i, first_cycle=first, state=states[i],
                             out=outs[i])
        for i in range(C):
            stream.wait_stream(streams[i])

    # ---- deterministic contraction -> k_dec; solves/s
    fs = [torch.from_numpy(gaussian_field(H.shape, 100 + i)).to(dev) for i in range(args.solves)]
    u = torch.empty(H.shape, dtype=torch.float64, device=dev)
    H.solve(fs[0], rtol=1e-12, u=u)            # warm-up
    ratios, cyc = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in fs:
        _, c, rr = H.solve(f, rtol=1e-12, u=u)
        cyc.append(c)
        ratios.append(H.last_ratio)
    torch.cuda.synchronize()
    solve_s = (time.perf_counter() - t0) / len(fs)
    rho = max(ratios)
    k_dec = max(1, math.ceil(math.log(0.01) / math.log(rho)))

    # ---- sampling: warm-up, then exactly K timed steps
    cycle = 0
    for _ in range(args.warmup):
        step(cycle)
        cycle += SAMPLES_PER_STEP
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        step(cycle)
        ev[k][1].record(stream)
        cycle += SAMPLES_PER_STEP
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    ms_per_step = wall * 1e3 / args.steps

    # ---- fine colour-pass kernel: HIP events around every launch of chain 0 running alone
    # (the same steps again, so that the per-launch time is not shared with other chains)
    H.kernel_timing(True)
    torch.cuda.synchronize()
    for k in range(args.steps):
        H.sample(SAMPLES_PER_STEP, seed=0, first_cycle=cycle, state=states[0], out=outs[0])
        cycle += SAMPLES_PER_STEP
    torch.cuda.synchronize()
    n_launch, k_ms = H.kernel_timing_read()
    H.kernel_timing(False)
    avg_launch_s = k_ms / 1e3 / max(n_launch, 1)
    # algorithmic bytes of one colour pass over the 3 components (b = 0): read the other
    # colour (N/2 values) and write this colour (N/2 values), 8 bytes each
    bytes_per_launch = NCOMP * NX * NY * NZ * 8
    achieved = bytes_per_launch / avg_launch_s / 1e9
    traffic = measured_traffic(bytes_per_launch)

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
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "k_rb_pass (fine colour pass)",
                     "avg_launch_us": round(avg_launch_s * 1e6, 3),
                     "launches_timed": int(n_launch),
                     "algorithmic_bytes_per_launch": bytes_per_launch},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(k_dec)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
