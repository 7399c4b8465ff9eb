"""Oracle: exactness and decorrelation analysis of the stochastic cycle (test infrastructure).

Sec. "Stochastic Iterative Methods": a linear stochastic iteration Z' = R Z + s + eta with
eta ~ N(0, J) has stationary covariance C solving C = R C R^T + J (eq. C_np1_recur and its
limit J = C - R C R^T), which is unique when the spectral radius of R is below one.  One
stochastic V-cycle is such an affine map x' = T x + G n in the vector n of all normals it
draws.  ``extract_affine_map`` recovers T and G by running the oracle's cycle on basis
vectors with injected noise, and ``stationary_covariance`` solves the discrete Lyapunov
equation so that it can be compared with the target kT A^-1.
"""
import numpy as np
import scipy.linalg as sla


class _RecordingNoise:
    """Counts the normals one cycle draws (in draw order)."""

    def __init__(self):
        self.count = 0

    def draw(self, cycle, level, slot, colour, comp, kind, sites):
        k = len(sites)
        self.count += k
        return np.zeros(k)


class _InjectedNoise:
    """Serves consecutive slices of a fixed vector, in draw order."""

    def __init__(self, vec):
        self.vec = vec
        self.pos = 0

    def draw(self, cycle, level, slot, colour, comp, kind, sites):
        k = len(sites)
        out = self.vec[self.pos:self.pos + k]
        self.pos += k
        return out


def extract_affine_map(mg):
    """Return (T, G) with one cycle (b = 0) equal to x -> T x + G n."""
    N = mg.levels[0].n
    zero = np.zeros(N)
    rec = _RecordingNoise()
    mg.vcycle(zero, zero, rec, 0, 0)
    m = rec.count
    T = np.empty((N, N))
    for i in range(N):
        e = np.zeros(N); e[i] = 1.0
        T[:, i] = mg.vcycle(e, zero, None, 0, 0)
    G = np.empty((N, m))
    for k in range(m):
        v = np.zeros(m); v[k] = 1.0
        G[:, k] = mg.vcycle(zero, zero, _InjectedNoise(v), 0, 0)
    return T, G


def stationary_covariance(T, Sigma):
    """Solve C = T C T^T + Sigma."""
    return sla.solve_discrete_lyapunov(T, Sigma)


def autocorrelation(series, max_lag):
    """Normalised sample autocorrelation of a scalar series for lags 0..max_lag: the lag-k
    sample autocovariance (1/n) sum_t (s_t - mean)(s_{t+k} - mean), with the full-length 1/n
    weight at every lag, divided by the lag-0 value (the estimator of the lag-k correlation
    of Sec. "Stochastic Iterative Methods")."""
    s = np.asarray(series, dtype=np.float64)
    s = s - s.mean()
    var = np.dot(s, s) / s.size
    return np.array([np.dot(s[:s.size - k], s[k:]) / s.size / var for k in range(max_lag + 1)])


def extract_linear_part(mg):
    """T of one cycle x -> T x + G n (b = 0): the cycle applied to the unit vectors, noise off."""
    N = mg.levels[0].n
    zero = np.zeros(N)
    T = np.empty((N, N))
    for i in range(N):
        e = np.zeros(N)
        e[i] = 1.0
        T[:, i] = mg.vcycle(e, zero, None, 0, 0)
    return T


def exact_lag_correlation(T, C, phi, max_lag):
    """Lag-k correlation of the observable phi^T x of the stationary chain x' = T x + G n with
    stationary covariance C: Cov(phi^T x_{t+k}, phi^T x_t) = phi^T T^k C phi, normalised by
    phi^T C phi, for k = 0 .. max_lag (the lag-k correlation of Sec. "Stochastic Iterative
    Methods", R^k applied to the stationary covariance)."""
    v = C @ phi
    den = float(phi @ v)
    out = np.empty(max_lag + 1)
    for k in range(max_lag + 1):
        out[k] = float(phi @ v) / den
        v = T @ v
    return out
