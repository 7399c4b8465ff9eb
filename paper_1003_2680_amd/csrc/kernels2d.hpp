// Launchers of the two-dimensional sampler's kernels (kernels_2d.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"

namespace smg {

// One level of the 2D hierarchy on the device: x stencils s1d = (m_x, a_x) (10 values, offsets
// -2..2), per-row z bands zt[nz][10] = (a_z[z][z-2..z+2], m_z[z][z-2..z+2]) (zero beyond the
// walls), block factors bfac[nz/2][32] = (A_BB^-1, L_BB^-T) row-major 4 x 4 (Galerkin levels).
struct Lev2 {
  int nx, nz;
  const double* s1d;
  const double* zt;
  const double* bfac;
};

// level-0 red-black point heat bath of one colour (b null = 0); noise site = lex >> 1
hipError_t launch2_point_pass(double* x, const double* b, const Lev2& L, int ncomp, int colour,
                              double kT, bool noise, const NoiseArgs& na, hipStream_t s);
// Galerkin-level 2 x 2 block heat bath of one colour (colour = bx%2 + 2 (bz%2)); noise site =
// 4 block + in-block index
hipError_t launch2_block_pass(double* x, const double* b, const Lev2& L, int ncomp, int colour,
                              double kT, bool noise, const NoiseArgs& na, hipStream_t s);
// r = b - A x (b null = 0)
hipError_t launch2_residual(double* r, const double* x, const double* b, const Lev2& L,
                            int ncomp, hipStream_t s);
// b_c = P^T r; x_c = 0 when xc is not null
hipError_t launch2_restrict(double* bc, double* xc, const double* r, int nxf, int nzf, int ncomp,
                            hipStream_t s);
// x += P e
hipError_t launch2_prolong(double* x, const double* e, int nxf, int nzf, int ncomp,
                           hipStream_t s);

}  // namespace smg
