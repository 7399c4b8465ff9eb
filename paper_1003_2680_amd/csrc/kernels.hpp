// Launchers of the HIP kernels (host-callable).  Fields are float64; level 0 of a
// point-smoothed hierarchy is stored split by colour: colour c (cells with (x+y+z)%2 == c)
// occupies [ncomp][nz][ny][nx/2], entry j of row (y,z) being x = 2j + ((y+z+c)&1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"

namespace smg {

hipError_t launch_rb_pass(double* xc, const double* xo, const double* bc, int nx, int ny, int nz,
                          int ncomp, int colour, double h, double kT, bool noise,
                          const NoiseArgs& na, hipStream_t s);
hipError_t launch_residual0(double* r, const double* xr, const double* xb, const double* br,
                            const double* bb, int nx, int ny, int nz, int ncomp, double h,
                            hipStream_t s);
hipError_t launch_residual7_nat(double* r, const double* x, const double* b, int nx, int ny,
                                int nz, int ncomp, double h, hipStream_t s);
hipError_t launch_residual_gal(double* r, const double* x, const double* b, const double* coef,
                               int nx, int ny, int nz, int ncomp, hipStream_t s);
hipError_t launch_restrict(double* bc, const double* r, int nxf, int nyf, int nzf, int ncomp,
                           hipStream_t s);
hipError_t launch_prolong0(double* xr, double* xb, const double* e, int nxf, int nyf, int nzf,
                           int ncomp, hipStream_t s);
hipError_t launch_prolong(double* x, const double* e, int nxf, int nyf, int nzf, int ncomp,
                          hipStream_t s);
hipError_t launch_block_pass(double* x, const double* b, const double* coef, const double* bfac,
                             int nx, int ny, int nz, int ncomp, int colour, bool noise,
                             const NoiseArgs& na, hipStream_t s);
hipError_t launch_coarsest(double* x, const double* b, const double* ainv, const double* w, int n,
                           int ncomp, bool noise, const NoiseArgs& na, hipStream_t s);
hipError_t launch_zero(double* p, int64_t n, hipStream_t s);
hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s);
hipError_t launch_to_split(double* xr, double* xb, const double* nat, int nx, int ny, int nz,
                           int ncomp, hipStream_t s);
hipError_t launch_from_split(void* nat, int out_f32, const double* xr, const double* xb, int nx,
                             int ny, int nz, int ncomp, hipStream_t s);
hipError_t launch_cast(void* dst, int out_f32, const double* src, int64_t n, hipStream_t s);
// sums of squares per component of v[ncomp][n] into out[ncomp] (fixed reduction order)
hipError_t launch_sumsq(double* out, double* part, const double* v, int64_t n, int ncomp,
                        hipStream_t s);

}  // namespace smg
