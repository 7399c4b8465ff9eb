"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

Holds none of the method's arithmetic: only reproducible random right-hand sides and
fields (NumPy's PCG64 generator), and the instance-size draw of the batched workload.
"""
import numpy as np


def gaussian_field(shape, seed):
    """Independent N(0, 1) entries (float64), e.g. a solve right-hand side f ~ N(0, 1)."""
    return np.random.default_rng(seed).standard_normal(shape)


def gaussian_field_device(shape, seed, device):
    """Independent N(0, 1) float64 entries drawn on the device (torch's seeded generator):
    right-hand sides too large to stage from the host at request rate."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return torch.randn(shape, generator=g, dtype=torch.float64, device=device)


def uniform_field(shape, seed, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, shape)


def batched_sizes(n_instances, seed=2026, choices=(32, 48, 64, 96)):
    """Cubic grid edge per instance, drawn uniformly from `choices`."""
    rng = np.random.default_rng(seed)
    return [int(choices[k]) for k in rng.integers(0, len(choices), n_instances)]
