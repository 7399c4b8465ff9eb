"""Oracle: exact eigen-decomposition of the uniform wall-bounded operator (test infrastructure).

On the uniform grid A = -L is a Kronecker sum of 1D operators.  The periodic axes are
diagonalised by the discrete Fourier transform with eigenvalues (4/h^2) sin^2(pi j/n);
the wall axis with antisymmetric ghosts is diagonalised by sin(pi m (z + 1/2)/nz),
m = 1..nz, with eigenvalues (4/h^2) sin^2(pi m/(2 nz)) (a DST-II basis).  This gives an
independent solver and sampler valid at any size (the paper's point is that such
transforms are unavailable on adaptive meshes; on the uniform box they are an exact
reference).
"""
import numpy as np
import scipy.fft as sfft


def eigenvalues(nx, ny, nz, h=1.0):
    """Array lam[m-1, k, j] for z-mode m = 1..nz, y-mode k, x-mode j."""
    j = np.arange(nx)
    k = np.arange(ny)
    m = np.arange(1, nz + 1)
    lx = 4.0 * np.sin(np.pi * j / nx) ** 2
    ly = 4.0 * np.sin(np.pi * k / ny) ** 2
    lz = 4.0 * np.sin(np.pi * m / (2.0 * nz)) ** 2
    return (lz[:, None, None] + ly[None, :, None] + lx[None, None, :]) / (h * h)


def _forward(x):
    # FFT over x, y; DST-II over z (orthonormal scaling)
    X = sfft.fft2(x, axes=(1, 2), norm="ortho")
    return sfft.dst(X.real, type=2, axis=0, norm="ortho") + 1j * sfft.dst(X.imag, type=2, axis=0, norm="ortho")


def _inverse(X):
    Y = sfft.idst(X.real, type=2, axis=0, norm="ortho") + 1j * sfft.idst(X.imag, type=2, axis=0, norm="ortho")
    return sfft.ifft2(Y, axes=(1, 2), norm="ortho").real


def solve(f, nx, ny, nz, h=1.0):
    """u = A^-1 f for a field f[nz, ny, nx] (or flat)."""
    F = _forward(np.asarray(f, dtype=np.float64).reshape(nz, ny, nx))
    return _inverse(F / eigenvalues(nx, ny, nz, h)).ravel()


def mode_amplitudes(x, nx, ny, nz):
    """Coefficients of x in the orthonormal eigenbasis (complex for the Fourier part)."""
    return _forward(np.asarray(x, dtype=np.float64).reshape(nz, ny, nx))


def z_mode(m, nz):
    """Normalised wall-axis eigenvector m (1-based) on cell centres."""
    z = np.arange(nz)
    v = np.sin(np.pi * m * (z + 0.5) / nz)
    return v / np.linalg.norm(v)
