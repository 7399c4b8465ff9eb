"""Pins for the oracle's observables (CPU only).

The mode vectors are checked against the assembled operator itself (A phi = lambda phi,
orthonormality, completeness), the lowest-mode selection against a dense eigensolver, and
the energy against Parseval's identity in the eigenbasis -- none of which reuses the
oracle's own formulas.
"""
import numpy as np
import pytest

from oracle.operator import assemble_A
from oracle import observables as ob


def _all_modes(nx, ny, nz):
    return [(a, b, m) for m in range(1, nz + 1) for b in range(ny) for a in range(nx)]


@pytest.mark.parametrize("dims", [(6, 4, 3), (4, 4, 4), (2, 6, 2), (8, 2, 1)])
def test_modes_are_an_orthonormal_eigenbasis(dims):
    nx, ny, nz = dims
    h = 0.7
    A = assemble_A(nx, ny, nz, h).toarray()
    modes = _all_modes(nx, ny, nz)
    Q = np.stack([ob.mode_vector(nx, ny, nz, md) for md in modes], axis=1)
    assert np.max(np.abs(Q.T @ Q - np.eye(len(modes)))) < 1e-13
    for q, md in enumerate(modes):
        lam = ob.mode_eigenvalue(nx, ny, nz, md, h)
        assert np.max(np.abs(A @ Q[:, q] - lam * Q[:, q])) < 1e-12 * max(lam, 1.0)


@pytest.mark.parametrize("dims,K", [((8, 8, 8), 8), ((6, 4, 3), 20), ((16, 8, 4), 12),
                                    ((4, 4, 16), 9), ((8, 8, 2), 30)])
def test_lowest_modes_match_dense_spectrum(dims, K):
    nx, ny, nz = dims
    A = assemble_A(nx, ny, nz).toarray()
    ev = np.sort(np.linalg.eigvalsh(A))[:K]
    modes = ob.lowest_modes(nx, ny, nz, K)
    assert len(modes) == K and len(set(modes)) == K
    lam = np.array([ob.mode_eigenvalue(nx, ny, nz, md) for md in modes])
    assert np.all(np.diff(lam) >= -1e-12)
    assert np.max(np.abs(lam - ev)) < 1e-12
    # the bounded enumeration selects what a full enumeration would
    full = sorted(_all_modes(nx, ny, nz),
                  key=lambda md: (round(ob.mode_eigenvalue(nx, ny, nz, md) * 2 ** 30),
                                  md[2], md[1], md[0]))
    assert modes == full[:K]


def test_lowest_modes_known_order_128():
    # 128^3: the wall mode m = 1 is lowest, then m = 2 and the first x/y waves with m = 1
    # (4 sin^2(pi/128) vs 4 sin^2(pi/128) + 4 sin^2(pi/256) decides: m = 2 comes first)
    modes = ob.lowest_modes(128, 128, 128, 6)
    assert modes[0] == (0, 0, 1)
    assert modes[1] == (0, 0, 2)
    assert set(modes[2:6]) == {(1, 0, 1), (2, 0, 1), (0, 1, 1), (0, 2, 1)}


@pytest.mark.parametrize("dims", [(6, 4, 3), (8, 8, 4)])
def test_energy_parseval_and_projections(dims):
    nx, ny, nz = dims
    h = 1.3
    rng = np.random.default_rng(4)
    x = rng.standard_normal(nx * ny * nz)
    modes = _all_modes(nx, ny, nz)
    p = ob.projections(x, nx, ny, nz, modes)
    lam = np.array([ob.mode_eigenvalue(nx, ny, nz, md, h) for md in modes])
    assert abs(np.dot(p, p) - np.dot(x, x)) < 1e-12 * np.dot(x, x)
    E = ob.energy(x, nx, ny, nz, h)
    assert abs(E - 0.5 * np.dot(lam, p * p)) < 1e-12 * E
    obs = ob.observables(x, nx, ny, nz, modes[:5], h)
    assert obs.shape == (6,) and obs[-1] == E and np.array_equal(obs[:5], p[:5])


def test_moments():
    s = np.arange(12.0).reshape(3, 4)
    m1, m2 = ob.moments(s)
    assert np.array_equal(m1, [12.0, 15.0, 18.0, 21.0])
    assert np.array_equal(m2, [0 + 16 + 64, 1 + 25 + 81, 4 + 36 + 100, 9 + 49 + 121])
