// SELM coupling kernels (Sec. "Discretization of SELM Hydrodynamic Coupling Tensor"; Sec.
// "Generation of the Stochastic Driving Fields Accounting for Thermal Fluctuations").
//
// Velocity fields are three cell-centred components, natural layout [3][nz][ny][nx].  The
// discrete divergence is D u = delta_x u_x + delta_y u_y + delta_z u_z with delta_x, delta_y the
// periodic forward differences and delta_z = a_z^{1/2} (the symmetric square root of the 1D
// wall operator, a dense nz x nz table S), so that D D^T = A and the projection
// P = I - D^T A^-1 D commutes with the viscous operator.  Gamma interpolates with Peskin's
// 4-point function (cells beyond a no-slip wall are antisymmetric ghosts of their mirrors).
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "selm.hpp"

namespace smg {
namespace {

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + TPB - 1) / TPB); }

// div = D u (one thread per cell; a wave lies in one (y, z) row when nx is a multiple of 64, so
// the row of S it reads is the same for every lane)
__global__ __launch_bounds__(TPB) void k_selm_div(double* __restrict__ div,
                                                   const double* __restrict__ u,
                                                   const double* __restrict__ S, int nx, int ny,
                                                   int nz, double inv_h) {
  const int64_t N = (int64_t)nx * ny * nz;
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= N) return;
  const int x = (int)(i % nx);
  const int64_t row = i / nx;
  const int y = (int)(row % ny);
  const int z = (int)(row / ny);
  const double* ux = u;
  const double* uy = u + N;
  const double* uz = u + 2 * N;
  const int xp = x + 1 == nx ? 0 : x + 1;
  const int yp = y + 1 == ny ? 0 : y + 1;
  const int64_t col = (int64_t)y * nx + x;  // (x, y) column of the z sum
  double d = (ux[row * nx + xp] - ux[i]) * inv_h;
  d += (uy[((int64_t)z * ny + yp) * nx + x] - uy[i]) * inv_h;
  const double* Sz = S + (int64_t)z * nz;
  double acc = 0.0;
  for (int k = 0; k < nz; ++k) acc = fma(Sz[k], uz[(int64_t)k * nx * ny + col], acc);
  div[i] = d + acc;
}

// out = u - D^T p: delta_x^T p = (p[x-1] - p[x]) / h, the same in y, and S p in z (S symmetric)
// (out may be u: each thread reads and writes the same three entries)
__global__ __launch_bounds__(TPB) void k_selm_grad_sub(double* out, const double* u,
                                                        const double* __restrict__ p,
                                                        const double* __restrict__ S, int nx,
                                                        int ny, int nz, double inv_h) {
  const int64_t N = (int64_t)nx * ny * nz;
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= N) return;
  const int x = (int)(i % nx);
  const int64_t row = i / nx;
  const int y = (int)(row % ny);
  const int z = (int)(row / ny);
  const int xm = x == 0 ? nx - 1 : x - 1;
  const int ym = y == 0 ? ny - 1 : y - 1;
  const int64_t col = (int64_t)y * nx + x;
  out[i] = u[i] - (p[row * nx + xm] - p[i]) * inv_h;
  out[N + i] = u[N + i] - (p[((int64_t)z * ny + ym) * nx + x] - p[i]) * inv_h;
  const double* Sz = S + (int64_t)z * nz;
  double acc = 0.0;
  for (int k = 0; k < nz; ++k) acc = fma(Sz[k], p[(int64_t)k * nx * ny + col], acc);
  out[2 * N + i] = u[2 * N + i] - acc;
}

// Peskin's 4-point immersed-boundary function phi(r)
__device__ __forceinline__ double peskin4(double r) {
  r = fabs(r);
  if (r < 1.0) return (3.0 - 2.0 * r + sqrt(1.0 + 4.0 * r - 4.0 * r * r)) * 0.125;
  if (r < 2.0) return (5.0 - 2.0 * r - sqrt(-7.0 + 12.0 * r - 4.0 * r * r)) * 0.125;
  return 0.0;
}

// The stencil cell q = 0..63 of a point (4 x 4 x 4 cells from the first cell whose centre is
// within two widths) and its weight; a cell beyond a wall folds onto its mirror with a minus
// sign (antisymmetric ghost).
struct StencilCell {
  int64_t cell;
  double w;
};
__device__ __forceinline__ StencilCell stencil_cell(const double* __restrict__ X, int k, int q,
                                                    int nx, int ny, int nz, double inv_h) {
  const double px = X[3 * k] * inv_h, py = X[3 * k + 1] * inv_h, pz = X[3 * k + 2] * inv_h;
  const int ix = (int)floor(px - 0.5) - 1 + (q & 3);
  const int iy = (int)floor(py - 0.5) - 1 + ((q >> 2) & 3);
  int iz = (int)floor(pz - 0.5) - 1 + (q >> 4);
  double w = peskin4(ix + 0.5 - px) * peskin4(iy + 0.5 - py) * peskin4(iz + 0.5 - pz);
  if (iz < 0) {
    iz = -1 - iz;
    w = -w;
  } else if (iz >= nz) {
    iz = 2 * nz - 1 - iz;
    w = -w;
  }
  if (iz < 0 || iz >= nz) {  // a point outside the channel: no weight, no access out of range
    iz = 0;
    w = 0.0;
  }
  const int jx = ((ix % nx) + nx) % nx, jy = ((iy % ny) + ny) % ny;
  StencilCell s;
  s.cell = ((int64_t)iz * ny + jy) * nx + jx;
  s.w = w;
  return s;
}

// f += scale * Gamma^T F (one thread per (point, stencil cell); points may share cells, so the
// adds are atomic)
__global__ __launch_bounds__(TPB) void k_selm_spread(double* __restrict__ f,
                                                      const double* __restrict__ X,
                                                      const double* __restrict__ F, int m, int nx,
                                                      int ny, int nz, double inv_h, double scale) {
  const int t = blockIdx.x * TPB + threadIdx.x;
  if (t >= 64 * m) return;
  const int k = t >> 6, q = t & 63;
  const StencilCell s = stencil_cell(X, k, q, nx, ny, nz, inv_h);
  const int64_t N = (int64_t)nx * ny * nz;
  for (int c = 0; c < 3; ++c) atomicAdd(&f[c * N + s.cell], scale * s.w * F[3 * k + c]);
}

// V = scale * Gamma u: one wave per point, lane q = stencil cell, sums by a fixed shuffle tree
__global__ __launch_bounds__(TPB) void k_selm_interp(double* __restrict__ V,
                                                      const double* __restrict__ X,
                                                      const double* __restrict__ u, int m, int nx,
                                                      int ny, int nz, double inv_h, double scale) {
  const int k = (blockIdx.x * TPB + threadIdx.x) >> 6;
  const int q = threadIdx.x & 63;
  if (k >= m) return;
  const StencilCell s = stencil_cell(X, k, q, nx, ny, nz, inv_h);
  const int64_t N = (int64_t)nx * ny * nz;
  double v[3];
  for (int c = 0; c < 3; ++c) v[c] = s.w * u[c * N + s.cell];
  for (int off = 32; off >= 1; off >>= 1)
    for (int c = 0; c < 3; ++c) v[c] += __shfl_xor(v[c], off, 64);
  if (q == 0)
    for (int c = 0; c < 3; ++c) V[3 * k + c] = scale * v[c];
}

// X += dt V + sqrt(dt) g (Euler-Maruyama)
__global__ __launch_bounds__(TPB) void k_selm_em(double* __restrict__ X,
                                                  const double* __restrict__ V,
                                                  const double* __restrict__ g, int n, double dt,
                                                  double sdt) {
  const int i = blockIdx.x * TPB + threadIdx.x;
  if (i < n) X[i] = X[i] + dt * V[i] + sdt * g[i];
}

}  // namespace

hipError_t launch_selm_div(double* div, const double* u, const double* S, int nx, int ny, int nz,
                           double h, hipStream_t s) {
  const int64_t N = (int64_t)nx * ny * nz;
  k_selm_div<<<blocks_for(N), TPB, 0, s>>>(div, u, S, nx, ny, nz, 1.0 / h);
  return hipGetLastError();
}

hipError_t launch_selm_grad_sub(double* out, const double* u, const double* p, const double* S,
                                int nx, int ny, int nz, double h, hipStream_t s) {
  const int64_t N = (int64_t)nx * ny * nz;
  k_selm_grad_sub<<<blocks_for(N), TPB, 0, s>>>(out, u, p, S, nx, ny, nz, 1.0 / h);
  return hipGetLastError();
}

hipError_t launch_selm_spread(double* f, const double* X, const double* F, int m, int nx, int ny,
                              int nz, double h, double scale, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  k_selm_spread<<<blocks_for(64 * (int64_t)m), TPB, 0, s>>>(f, X, F, m, nx, ny, nz, 1.0 / h,
                                                           scale);
  return hipGetLastError();
}

hipError_t launch_selm_interp(double* V, const double* X, const double* u, int m, int nx, int ny,
                              int nz, double h, double scale, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  k_selm_interp<<<blocks_for(64 * (int64_t)m), TPB, 0, s>>>(V, X, u, m, nx, ny, nz, 1.0 / h,
                                                           scale);
  return hipGetLastError();
}

hipError_t launch_selm_em(double* X, const double* V, const double* g, int n, double dt,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_selm_em<<<blocks_for(n), TPB, 0, s>>>(X, V, g, n, dt, sqrt(dt));
  return hipGetLastError();
}

}  // namespace smg
