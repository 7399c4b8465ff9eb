"""Pins for the oracle's noise source (CPU only).

* Bitwise agreement with rocRAND's Philox4x32-10 engine, an implementation of the same
  published generator written independently of this project (built here for the host).
* Distributional checks on the Box-Muller normals: moments, a Kolmogorov-Smirnov test,
  and absence of correlation between the two outputs of a call and between streams.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.stats as st

from oracle.philox import philox4x32_10, normals, stream_id, uniforms_from_words

HERE = os.path.dirname(os.path.abspath(__file__))


def _hipcc():
    for p in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if p and os.path.exists(p):
            return p
    return None


@pytest.fixture(scope="module")
def rocrand_words(tmp_path_factory):
    hipcc = _hipcc()
    if hipcc is None or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    out = tmp_path_factory.mktemp("rr") / "rocrand_words"
    src = os.path.join(HERE, "helpers", "rocrand_philox_words.cpp")
    subprocess.run([hipcc, "-O1", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__", "-x", "c++",
                    src, "-o", str(out)], check=True, capture_output=True)

    def run(triples):
        txt = "".join("%d %d %d\n" % t for t in triples)
        res = subprocess.run([str(out)], input=txt, capture_output=True, text=True, check=True)
        return np.array([[int(w) for w in line.split()] for line in res.stdout.strip().splitlines()])

    return run


def test_philox_matches_rocrand(rocrand_words):
    rng = np.random.default_rng(11)
    cases = [(0, 0, 0, 0, 0), (0xFFFFFFFF, 0, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFFFFFFFFFF)]
    for _ in range(200):
        c0 = int(rng.integers(0, 2 ** 32))
        c1 = int(rng.integers(0, 2 ** 30))
        c2 = int(rng.integers(0, 2 ** 32))
        c3 = int(rng.integers(0, 2 ** 32))
        seed = int(rng.integers(0, 2 ** 63)) * 2 + int(rng.integers(0, 2))
        cases.append((c0, c1, c2, c3, seed))
    triples = [(s, c2 | (c3 << 32), 4 * (c0 | (c1 << 32))) for (c0, c1, c2, c3, s) in cases]
    ref = rocrand_words(triples)
    for (c0, c1, c2, c3, s), r in zip(cases, ref):
        w = philox4x32_10(c0, c1, c2, c3, s & 0xFFFFFFFF, s >> 32)
        assert [int(v) for v in w] == list(r)


def test_uniform_map_open_interval():
    lo = uniforms_from_words(np.uint64(0), np.uint64(0))
    hi = uniforms_from_words(np.uint64(0xFFFFFFFF), np.uint64(0xFFFFFFFF))
    # the smallest uniform is 2^-54 > 0, so ln u1 is finite; for the largest word the
    # half-ulp offset rounds away (2^53 - 1/2 is not a double) and u = 1 exactly, which
    # gives a zero radius -- harmless.  Both sides round the same IEEE operations.
    assert lo == 0.5 * 2.0 ** -53 and 0.0 < lo
    assert hi == 1.0


def test_normals_distribution():
    n = 400_000
    z = normals(7, 3, 0, 1, 0, 2, 0, np.arange(n))
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert abs(st.kurtosis(z)) < 5 * np.sqrt(24.0 / n)
    assert st.kstest(z, "norm").pvalue > 1e-4
    even, odd = z[0::2], z[1::2]
    assert abs(np.corrcoef(even, odd)[0, 1]) < 5 / np.sqrt(n / 2)
    other = normals(7, 3, 0, 1, 1, 2, 0, np.arange(n))        # other colour
    assert abs(np.corrcoef(z, other)[0, 1]) < 5 / np.sqrt(n)
    later = normals(7, 4, 0, 1, 0, 2, 0, np.arange(n))        # next cycle
    assert abs(np.corrcoef(z, later)[0, 1]) < 5 / np.sqrt(n)


def test_stream_id_fields_are_disjoint():
    ids = {stream_id(l, s, c, k, kind) for l in range(3) for s in range(4) for c in range(8)
           for k in range(3) for kind in range(2)}
    assert len(ids) == 3 * 4 * 8 * 3 * 2
