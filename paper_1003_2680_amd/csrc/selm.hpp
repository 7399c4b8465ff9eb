// Launchers of the SELM coupling kernels (kernels_selm.hip).  Fields: three cell-centred
// velocity components, natural layout [3][nz][ny][nx], float64; S: the nz x nz symmetric square
// root of the 1D wall operator (row-major); X: structure points [m][3] (positions, 0 < z < nz h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smg {

// div = D u = delta_x u_x + delta_y u_y + S u_z  (forward differences in x and y)
hipError_t launch_selm_div(double* div, const double* u, const double* S, int nx, int ny, int nz,
                           double h, hipStream_t s);
// out = u - D^T p
hipError_t launch_selm_grad_sub(double* out, const double* u, const double* p, const double* S,
                                int nx, int ny, int nz, double h, hipStream_t s);
// f += scale * Gamma^T F  (F: [m][3]; f must be initialised by the caller)
hipError_t launch_selm_spread(double* f, const double* X, const double* F, int m, int nx, int ny,
                              int nz, double h, double scale, hipStream_t s);
// V = scale * Gamma u  (V: [m][3])
hipError_t launch_selm_interp(double* V, const double* X, const double* u, int m, int nx, int ny,
                              int nz, double h, double scale, hipStream_t s);
// X += dt V + sqrt(dt) g over n values
hipError_t launch_selm_em(double* X, const double* V, const double* g, int n, double dt,
                          hipStream_t s);

}  // namespace smg
