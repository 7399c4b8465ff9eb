"""Many independent instances of uneven grid sizes on one GPU.

Instances with the same grid and cycle configuration form a group: one hierarchy whose
components are the group's chains, so every launch of the cycle covers all of them (each
chain draws exactly what it draws alone: seeds and cycle counters are per chain).  With the
default engine ("library") every call goes to the library's batch entry point, which steps all
groups through their cycles together on one stream and runs the small levels of every group
(the LDS-resident bottom of each V-cycle) in merged launches; the whole sampling call can be
captured once as a HIP graph and replayed (the chain tables on the device advance with every
replay).  The "streams" engine runs each group's calls on its own HIP stream instead (kept for
comparison).  The cycle configuration of each grid comes from the autotuner (or is given).

Only orchestration lives here; every step runs in the library's kernels.
"""
from collections import OrderedDict

import torch

from .api import Hierarchy, batch_run
from . import autotune


class Instance:
    """One scalar instance: a cubic (or any) grid, its chain seed and first cycle."""

    def __init__(self, dims, seed, first_cycle=0):
        self.dims = tuple(int(d) for d in dims)
        self.seed = int(seed)
        self.first_cycle = int(first_cycle)


class Group:
    def __init__(self, dims, members, config, precision, device):
        self.dims = dims
        self.members = members            # indices into the runner's instance list
        self.config = config
        self.n = len(members)
        self.H = Hierarchy(*dims, ncomp=self.n, levels=config["levels"], nu1=config["nu1"],
                           nu2=config["nu2"], precision=precision, device=device)
        autotune.apply(self.H, config)
        self.stream = torch.cuda.Stream(device=device)
        self.state = torch.zeros(self.H.shape, dtype=torch.float64, device=device)
        self.graphs = []


class BatchRunner:
    """Runs a list of Instances grouped by grid.

    configs: {dims: config} (keys levels, nu1, nu2 and optionally tile, bottom); missing
    grids are tuned with autotune.tune for their group size (tune=True) or get the automatic
    depth with V(2,2).  stream_groups: the library engine's staggered stream groups for eager
    calls (each a share of every grid's instances; 1 = the call's stream only); a captured graph
    takes the one-stream form."""

    def __init__(self, instances, precision="fp32_refined", configs=None, tune=False,
                 device=None, engine="library", stream_groups=1):
        dev = torch.device(device if device is not None else "cuda")
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        if engine not in ("library", "streams"):
            raise ValueError("engine must be 'library' or 'streams'")
        self.engine = engine
        self.graph = None
        self.instances = list(instances)
        self.precision = precision
        by_dims = OrderedDict()
        for i, inst in enumerate(self.instances):
            by_dims.setdefault(inst.dims, []).append(i)
        configs = dict(configs or {})
        self.tuned = {}
        for dims, members in by_dims.items():
            if dims not in configs:
                if tune:
                    configs[dims] = autotune.tune(dims, len(members), precision=precision,
                                                  device=self.device)
                    self.tuned[dims] = configs[dims]
                else:
                    configs[dims] = {"levels": 0, "nu1": 2, "nu2": 2}
        self.groups = [Group(d, m, configs[d], precision, self.device) for d, m in by_dims.items()]
        self.stream_groups = stream_groups
        if engine == "library":
            for g in self.groups:
                g.H.set_stream_groups(stream_groups)
        self.configs = configs
        self._started = False

    def cells(self):
        return sum(g.n * g.dims[0] * g.dims[1] * g.dims[2] for g in self.groups)

    def start(self):
        """(Re)start every chain at its seed and first cycle from the zero state."""
        cur = torch.cuda.current_stream(self.device)
        for g in self.groups:
            g.stream.wait_stream(cur)
            with torch.cuda.stream(g.stream):
                g.state.zero_()
                g.H.sample_batch(0, seeds=[self.instances[i].seed for i in g.members],
                                 first_cycles=[self.instances[i].first_cycle for i in g.members],
                                 comps_per_chain=1, state=g.state)
            cur.wait_stream(g.stream)
        self._started = True

    def sample(self, n, out_dtype=torch.float32, emit=True):
        """Advance every chain by n emitted samples; returns {instance index: tensor
        [n, nz, ny, nx]} (views into the group's output) or {} when emit is False."""
        if not self._started:
            self.start()
        outs = {}
        if self.engine == "library":
            items = []
            for g in self.groups:
                o = None
                if emit:
                    o = torch.empty((n,) + g.H.shape, dtype=out_dtype, device=self.device)
                items.append({"H": g.H, "op": "sample", "nchains": g.n, "comps_per_chain": 1,
                              "n": n, "state": g.state, "out": o, "out_dtype": out_dtype})
                if emit:
                    for k, i in enumerate(g.members):
                        outs[i] = o[:, k]
            self._check(batch_run(items))
            return outs
        cur = torch.cuda.current_stream(self.device)
        for g in self.groups:
            g.stream.wait_stream(cur)
            with torch.cuda.stream(g.stream):
                o = None
                if emit:
                    o = torch.empty((n,) + g.H.shape, dtype=out_dtype, device=self.device)
                g.H.sample_batch(n, nchains=g.n, comps_per_chain=1, state=g.state, out=o,
                                 out_dtype=out_dtype, emit=emit)
            cur.wait_stream(g.stream)
            if emit:
                for k, i in enumerate(g.members):
                    outs[i] = o[:, k]
        return outs

    @staticmethod
    def _check(results):
        bad = [st for st, _ in results if st != 0]
        if bad:
            raise RuntimeError("batch item failed with status %d" % bad[0])

    def capture(self, n):
        """Capture one call that advances every chain by n cycles (no emission) as a HIP graph
        (library engine: one graph of the whole batch; streams engine: one per group);
        replay() then reruns it, continuing every chain."""
        if not self._started:
            self.start()
        torch.cuda.synchronize(self.device)
        if self.engine == "library":
            items = [{"H": g.H, "op": "sample", "nchains": g.n, "comps_per_chain": 1, "n": n,
                      "state": g.state, "out": None} for g in self.groups]
            # captured on a side stream (the chain tables advance on the device per replay), in
            # the one-stream form: a replayed fork / join of stream groups measured slower than
            # the one-stream graph
            side = torch.cuda.Stream(device=self.device)
            graph = torch.cuda.CUDAGraph()
            for g in self.groups:
                g.H.set_stream_groups(1)
            try:
                with torch.cuda.graph(graph, stream=side):
                    self._check(batch_run(items))
            finally:
                for g in self.groups:
                    g.H.set_stream_groups(self.stream_groups)
            self.graph = graph
            return
        for g in self.groups:
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=g.stream):
                g.H.sample_batch(n, nchains=g.n, comps_per_chain=1, state=g.state, emit=False)
            g.graphs = [graph]

    def replay(self):
        if self.engine == "library":
            self.graph.replay()
            return
        cur = torch.cuda.current_stream(self.device)
        for g in self.groups:
            g.stream.wait_stream(cur)
            with torch.cuda.stream(g.stream):
                for graph in g.graphs:
                    graph.replay()
            cur.wait_stream(g.stream)

    def solve(self, fs, rtol=1e-10, max_cycles=100):
        """fs: {instance index: f [nz, ny, nx] float64 on the device}.  Returns
        ({index: u}, {index: (cycles, relres, last_ratio)}).  The groups solve concurrently,
        one host thread and one stream each (a solve reads its residual norms every cycle)."""
        from concurrent.futures import ThreadPoolExecutor
        torch.cuda.synchronize(self.device)
        if self.engine == "library":
            items, us_g = [], []
            for g in self.groups:
                f = torch.stack([fs[i] for i in g.members]).contiguous()
                u = torch.empty_like(f)
                us_g.append(u)
                items.append({"H": g.H, "op": "solve", "nchains": g.n, "comps_per_chain": 1,
                              "f": f, "u": u, "rtol": rtol, "max_cycles": max_cycles})
            res = batch_run(items)
            torch.cuda.synchronize(self.device)
            us, infos = {}, {}
            for g, u, (st, inf) in zip(self.groups, us_g, res):
                if st not in (0, -3):
                    raise RuntimeError("batch solve failed with status %d" % st)
                for k, i in enumerate(g.members):
                    us[i] = u[k]
                    infos[i] = inf[k]
            return us, infos

        def run(g):
            with torch.cuda.device(self.device), torch.cuda.stream(g.stream):
                f = torch.stack([fs[i] for i in g.members]).contiguous()
                return g.H.solve_batch(f, nchains=g.n, comps_per_chain=1, rtol=rtol,
                                       max_cycles=max_cycles)

        with ThreadPoolExecutor(max_workers=len(self.groups)) as ex:
            results = list(ex.map(run, self.groups))
        torch.cuda.synchronize(self.device)
        us, infos = {}, {}
        for g, (u, inf) in zip(self.groups, results):
            for k, i in enumerate(g.members):
                us[i] = u[k]
                infos[i] = inf[k]
        return us, infos
