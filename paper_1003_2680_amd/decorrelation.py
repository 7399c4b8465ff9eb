"""Decorrelation of the stochastic multigrid chain against the plain stochastic Gauss-Seidel
sampler, as the grid grows (Sec. "Stochastic Iterative Methods" and the paper's comparison of
the two samplers, on 3D grids, on 2D grids and on adaptive composite grids).

Both chains run in the library: the multigrid chain is the V(nu1, nu2) cycle; the
Gauss-Seidel chain is the same hierarchy reduced to one level whose "coarsest" step is nu1 +
nu2 red-black heat-bath sweeps (no coarse correction).  Each emitted cycle's observables --
projections onto the lowest eigenvectors of A and the energy -- come from the library's fused
statistics; this module only estimates lag-k autocorrelations and integrated autocorrelation
times from them (host arithmetic on the observable series, not on any field).
"""
import json
import time

import numpy as np
import torch

from .api import Hierarchy, lowest_modes


def make_chain(dims, kind, nchains=8, kT=1.0, nu=(2, 2), burn_in=0, device=None):
    """'mg': the multigrid cycle (automatic depth); 'gs': one level, heat-bath sweeps only.
    The hierarchy's components are independent chains (the component enters the counters)."""
    if kind == "mg":
        return Hierarchy(*dims, ncomp=nchains, kT=kT, levels=0, nu1=nu[0], nu2=nu[1],
                         burn_in=burn_in, device=device)
    if kind == "gs":
        return Hierarchy(*dims, ncomp=nchains, kT=kT, levels=1, coarsest="smooth",
                         nu1=nu[0], nu2=nu[1], burn_in=burn_in, device=device)
    raise ValueError("kind must be 'mg' or 'gs'")


def make_chain_2d(dims, kind, nchains=8, kT=1.0, nu=(2, 2), stride=1, device=None):
    """The 2D grid (nx, nz): 'mg' the multigrid cycle (automatic depth, coarsest <= 512
    unknowns), 'gs' one level of heat-bath sweeps only; a sample every `stride` cycles."""
    from .grid2d import Hierarchy2D
    nx, nz = dims
    if kind == "mg":
        return Hierarchy2D(nx, nz, ncomp=nchains, kT=kT, levels=0, nu1=nu[0], nu2=nu[1],
                           stride=stride, device=device)
    if kind == "gs":
        return Hierarchy2D(nx, nz, ncomp=nchains, kT=kT, levels=1, coarsest="smooth",
                           nu1=nu[0], nu2=nu[1], stride=stride, device=device)
    raise ValueError("kind must be 'mg' or 'gs'")


def mode_vectors_2d(dims, modes, device):
    """Real eigenvectors e_a(x) w_m(z) of the 2D operator (e_a as for the 3D observables, w_m the
    normalised cell-centred sine), [len(modes), nz * nx] float64."""
    nx, nz = dims
    i = torch.arange(nx, dtype=torch.float64, device=device)
    zc = torch.arange(nz, dtype=torch.float64, device=device) + 0.5
    vecs = []
    for a, m in modes:
        if a == 0:
            ex = torch.full((nx,), 1.0 / np.sqrt(nx), dtype=torch.float64, device=device)
        elif a == nx - 1:
            ex = torch.where(i.remainder(2) == 0, 1.0, -1.0) / np.sqrt(nx)
        else:
            j = (a + 1) // 2
            ang = 2.0 * np.pi * j * i / nx
            ex = np.sqrt(2.0 / nx) * (torch.cos(ang) if a % 2 else torch.sin(ang))
        w = torch.sin(np.pi * m * zc / nz)
        w = w / torch.linalg.norm(w)
        vecs.append(torch.outer(w, ex).reshape(-1))
    return torch.stack(vecs)


def projections_2d(samples, dims, modes):
    """Projections of 2D samples [n, nchains, nz, nx] on the given modes: [n, nchains, Q]
    (observables of the study; not part of the sampler)."""
    V = mode_vectors_2d(dims, modes, samples.device)
    n, c = samples.shape[:2]
    return (samples.reshape(n * c, -1) @ V.T).reshape(n, c, -1)


def study_2d(sizes=((32, 32), (64, 64), (128, 128)), nchains=8, n_mg=2000,
             gs_cycles_per_tau=100, device=None, seed=0):
    """The 2D form of the comparison: per (grid, sampler) the lag-1 correlation (per cycle) and
    tau_int (in cycles) of the lowest mode, cycles/s and the cost of one decorrelated sample.
    The Gauss-Seidel chains emit every tau_guess/10 cycles (tau_guess from the lowest
    eigenvalue) and run about gs_cycles_per_tau times tau_guess after ten of them of burn-in."""
    rows = []
    for dims in sizes:
        nz = dims[1]
        lam = 4.0 * np.sin(np.pi / (2 * nz)) ** 2
        tau_guess = max(2.0, 2.0 / (4 * lam / 3.0))
        for kind in ("mg", "gs"):
            stride = 1 if kind == "mg" else max(1, int(tau_guess / 10))
            H = make_chain_2d(dims, kind, nchains=nchains, stride=stride, device=device)
            if kind == "mg":
                burn, n = 20, n_mg
            else:
                burn = int(10 * tau_guess / stride) + 1
                n = int(max(1000, gs_cycles_per_tau * tau_guess / stride))
            _, st = H.sample(burn, seed)
            torch.cuda.synchronize(H.device)
            t0 = time.perf_counter()
            xs, _ = H.sample(n, seed, first_cycle=burn * stride, state=st)
            torch.cuda.synchronize(H.device)
            dt = time.perf_counter() - t0
            obs = projections_2d(xs, dims, [(0, 1), (1, 1)]).cpu().numpy()
            del xs
            rho_emit = float(autocorrelation(obs, 1)[1][0])
            tau = float(tau_int(obs)[0]) * stride
            cyc_s = n * stride / dt
            rows.append({"grid": list(dims), "sampler": kind, "cycles": n * stride,
                         "stride": stride,
                         "rho1_lowest_mode": round(rho_emit ** (1.0 / stride)
                                                   if rho_emit > 0 else rho_emit, 4),
                         "tau_int_lowest_mode": round(tau, 2),
                         "cycles_per_s": round(cyc_s, 1),
                         "s_per_decorrelated_sample": round(tau / cyc_s, 6)})
            print(json.dumps(rows[-1]), flush=True)
            del H
            torch.cuda.empty_cache()
    return rows


def observables(H, n, seed=0, modes=None):
    """n emitted cycles after the hierarchy's burn-in, from the zero state:
    [n, nchains, len(modes) + 1] (float64, host)."""
    dims = (H.desc.nx, H.desc.ny, H.desc.nz)
    if modes is None:
        modes = lowest_modes(*dims, 4)
    obs, _ = H.sample_stats(n, seed, modes=modes)
    torch.cuda.synchronize(H.device)
    return obs.cpu().numpy()


def autocorrelation(obs, max_lag):
    """Lag-k autocorrelation of each observable pooled over chains: [max_lag + 1, Q]."""
    o = obs - obs.mean(axis=0, keepdims=True)
    den = (o * o).sum(axis=(0, 1))
    T = o.shape[0]
    return np.stack([(o[:T - k] * o[k:]).sum(axis=(0, 1)) / den for k in range(max_lag + 1)])


def tau_int(obs, c=5.0):
    """1 + 2 sum_k rho(k) per observable, up to the first lag k >= c tau(k) (Sokal)."""
    o = obs - obs.mean(axis=0, keepdims=True)
    den = (o * o).sum(axis=(0, 1))
    T = o.shape[0]
    taus = []
    for q in range(o.shape[2]):
        tau = 1.0
        for k in range(1, T // 2):
            tau += 2.0 * float((o[:T - k, :, q] * o[k:, :, q]).sum() / den[q])
            if k >= c * tau:
                break
        taus.append(tau)
    return np.array(taus)


def study(sizes=((16, 16, 16), (32, 32, 32), (64, 64, 64)), nchains=8, n_mg=2000,
          gs_cycles_per_tau=200, device=None, seed=0):
    """One row per (grid, sampler): lag-1 correlation and tau_int of the lowest mode and the
    energy, cycles/s, and the cost of one decorrelated sample in cycles and in seconds.  The
    Gauss-Seidel chains run for about gs_cycles_per_tau times their expected tau (a first
    estimate from the grid's lowest eigenvalue) after a burn-in of ten of them."""
    rows = []
    for dims in sizes:
        nz = dims[2]
        # lowest mode's heat-bath contraction per sweep ~ 1 - lambda_min / 3 (red-black)
        lam = 4.0 * np.sin(np.pi / (2 * nz)) ** 2
        tau_guess = max(2.0, 2.0 / (4 * lam / 3.0))
        for kind in ("mg", "gs"):
            n = n_mg if kind == "mg" else int(gs_cycles_per_tau * tau_guess)
            burn = 20 if kind == "mg" else int(10 * tau_guess)
            H = make_chain(dims, kind, nchains=nchains, burn_in=burn, device=device)
            torch.cuda.synchronize(H.device)
            t0 = time.perf_counter()
            obs = observables(H, n, seed=seed)
            secs = time.perf_counter() - t0
            tau = tau_int(obs)
            rho1 = autocorrelation(obs, 1)[1]
            rate = (n + burn) / secs
            k_tau = max(tau[0], tau[-1])
            rows.append({"grid": list(dims), "sampler": kind, "levels": H.n_levels,
                         "cycles": n, "chains": nchains,
                         "lag1_lowest_mode": round(float(rho1[0]), 4),
                         "lag1_energy": round(float(rho1[-1]), 4),
                         "tau_int_lowest_mode": round(float(tau[0]), 2),
                         "tau_int_energy": round(float(tau[-1]), 2),
                         "cycles_per_s": round(rate, 1),
                         "seconds_per_decorrelated_sample": float("%.4g" % (k_tau / rate))})
            print(json.dumps(rows[-1]), flush=True)
            del H
            torch.cuda.empty_cache()
    return rows


def composite_weights(S):
    """Observable of the composite-grid study: the volume-weighted lowest wall mode
    sin(pi z / (nz h)) over the composite unknowns (a smooth field, slowest to relax under
    Gauss-Seidel), as (coarse weights with zeros on covered cells, fine weights)."""
    nz, ny, nx = S.base_shape
    fz, fy, fx = S.fine_shape
    x0, x1, y0, y1, z0, z1 = S.box
    zc = np.sin(np.pi * (np.arange(nz) + 0.5) / nz)
    wc = np.broadcast_to(zc[:, None, None], (nz, ny, nx)).copy()
    wc[z0:z1, y0:y1, x0:x1] = 0.0
    zf = np.sin(np.pi * (z0 + (np.arange(fz) + 0.5) / 2.0) / nz) / 8.0
    wf = np.broadcast_to(zf[:, None, None], (fz, fy, fx)).copy()
    return (torch.tensor(wc, device=S.device), torch.tensor(wf, device=S.device))


def composite_study(edges=(16, 32, 64), n_mg=4000, gs_cycles_per_tau=100, nu=2, seed=0):
    """The paper's comparison on an adaptive mesh: base e x e x e/2 with the box
    [e/4, 3e/4)^2 x [0, e/8) refined by two (the shape of the full adaptive workload), the FAC
    chain (nu composite sweeps after a V(2,2) base cycle) against the Gauss-Seidel-only chain
    (the same nu composite sweeps per cycle, no coarse correction).  One row per (grid,
    sampler): lag-1 correlation and tau_int of the observable, cycles/s and seconds per
    decorrelated sample."""
    from .composite import CompositeSampler
    rows = []
    for e in edges:
        base = (e, e, e // 2)
        box = (e // 4, 3 * e // 4, e // 4, 3 * e // 4, 0, max(1, e // 8))
        lam = 4.0 * np.sin(np.pi / (2 * base[2])) ** 2
        tau_guess = max(2.0, 3.0 / lam)
        for kind in ("mg", "gs"):
            gs = kind == "gs"
            n = int(gs_cycles_per_tau * tau_guess) if gs else n_mg
            burn = int(10 * tau_guess) if gs else 20
            S = CompositeSampler(*base, box, nu=nu, gs_only=gs)
            wc, wf = composite_weights(S)
            xc, xf = S.zeros()
            S.sample(xc, xf, burn, seed=seed)
            y = torch.empty(n, dtype=torch.float64, device=S.device)
            torch.cuda.synchronize(S.device)
            t0 = time.perf_counter()
            for t in range(n):
                S.sample(xc, xf, 1, seed=seed, first_cycle=burn + t)
                y[t] = (xc * wc).sum() + (xf * wf).sum()
            torch.cuda.synchronize(S.device)
            secs = time.perf_counter() - t0
            obs = y.cpu().numpy().reshape(n, 1, 1)
            tau = float(tau_int(obs)[0])
            rho1 = float(autocorrelation(obs, 1)[1][0])
            rate = n / secs
            rows.append({"base": list(base), "box": list(box), "unknowns": int(S.info.unknowns),
                         "sampler": "fac" if not gs else "gauss-seidel", "nu": nu,
                         "cycles": n, "lag1": round(rho1, 4), "tau_int": round(tau, 2),
                         "cycles_per_s": round(rate, 1),
                         "seconds_per_decorrelated_sample": float("%.4g" % (max(tau, 1.0) /
                                                                            rate))})
            print(json.dumps(rows[-1]), flush=True)
            del S
            torch.cuda.empty_cache()
    return rows


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="multigrid vs Gauss-Seidel decorrelation study")
    ap.add_argument("--sizes", default="16,32,64", help="cubic grid edges")
    ap.add_argument("--chains", type=int, default=8)
    ap.add_argument("--mg-cycles", type=int, default=2000)
    ap.add_argument("--gs-cycles-per-tau", type=int, default=200)
    ap.add_argument("--composite", action="store_true",
                    help="run the comparison on adaptive composite grids (base e x e x e/2)")
    ap.add_argument("--two-d", action="store_true",
                    help="run the comparison on square 2D grids e x e (periodic x, walls in z)")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    if args.two_d:
        study_2d(tuple((int(e), int(e)) for e in args.sizes.split(",")), nchains=args.chains,
                 n_mg=args.mg_cycles, gs_cycles_per_tau=args.gs_cycles_per_tau,
                 device=torch.device("cuda", 0))
        return
    if args.composite:
        composite_study(tuple(int(e) for e in args.sizes.split(",")), n_mg=args.mg_cycles,
                        gs_cycles_per_tau=args.gs_cycles_per_tau)
        return
    sizes = [(int(e), int(e), int(e)) for e in args.sizes.split(",")]
    study(sizes, nchains=args.chains, n_mg=args.mg_cycles,
          gs_cycles_per_tau=args.gs_cycles_per_tau, device=torch.device("cuda", 0))


if __name__ == "__main__":
    main()
