"""CPU oracle for the stochastic multigrid sampler/solver (Atzberger, arXiv:1003.2680).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It is a plain, slow, FP64 NumPy/SciPy restatement of the method,
written so that each step can be checked against the paper by eye:

* ``operator``  -- the cell-centred discrete Laplacian L = DG with no-slip walls
                   (Sec. "Spatially Adaptive Discretizations", uniform-mesh case).
* ``transfer``  -- trilinear prolongation and its adjoint restriction
                   (Sec. "Stochastic Multigrid Methods", eq. restr_prolong_variation).
* ``hierarchy`` -- Galerkin coarse operators A^(l) = I^T A I and the level plan.
* ``philox``    -- the counter-based noise source n ~ N(0, I) (Philox4x32-10 of
                   Salmon et al., SC'11, plus Box-Muller).
* ``mg``        -- stochastic Gauss-Seidel (heat-bath) smoothers, coarsest exact step,
                   the V-cycle (Alg. 3), the sampling chain and the deterministic solve.
* ``spectral``  -- the exact eigen-decomposition of the uniform wall-bounded operator
                   (FFT in x,y and DST-II in z), used as an independent reference.
* ``analysis``  -- affine-map extraction, the stationary-covariance (Lyapunov) check of
                   eq. J_eq_C_R, autocorrelation estimates.
* ``composite`` -- the spatially adaptive composite grid (one box refined by two): the
                   operator L = DG with the coarse-fine face gradient, the base-to-composite
                   prolongation and the stochastic FAC cycle (Algs. 1-3) with Galerkin
                   base levels.
* ``observables`` -- projections onto eigenvectors of A, the energy 1/2 x^T A x and
                   per-cell moments of the samples (the decorrelation observables).
* ``sampled``   -- the same steps evaluated cell by cell (a row of A, a heat-bath colour
                   pass, the residual restriction, the prolongation) for parity at sampled
                   cells of grids too large to assemble.
* ``selm``      -- the SELM coupling on the uniform grid: projection with D D^T = A,
                   Peskin's 4-point interpolation, mobility and driving field, Euler-Maruyama.
* ``mg2d``      -- the two-dimensional wall-bounded sampler (5-point operator, 2 x 2 blocks).
* ``effective`` -- the effective structure dynamics of Appendix A for a non-symmetric L
                   (drift, mobility, noise covariance, the Lyapunov relation of the forcing)
                   and the composite-mesh field noise w = L^-1 Q eta.

The oracle shares no code with the HIP path; the two meet only on seeded inputs.
"""
