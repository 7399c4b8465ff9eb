"""MI355X-native stochastic multigrid sampler/solver (Atzberger, arXiv:1003.2680).

The compute path lives in ``libsmg.so`` (host C++ runtime + gfx950 HIP kernels) behind the
C-ABI declared in ``include/smg.h``.  ``paper_1003_2680_amd.abi`` binds it with ctypes and
``paper_1003_2680_amd.api`` wraps it with torch tensors for device memory and streams.
Importing the package loads nothing; the library is loaded on first use and a missing
build raises immediately (there is no fallback path).
"""

__all__ = ["abi", "api"]
