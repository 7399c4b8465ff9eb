// Kernels of the two-dimensional wall-bounded sampler (cells (x, z), periodic in x, no-slip walls
// on the z faces).  Every level's operator is the tensor sum A = a_z (x) m_x + m_z (x) a_x of
// 1D pieces (Galerkin recurrences; level 0: m = I, a = the 1D three-point operators), applied
// from two uniform 5-entry x stencils and per-row z bands.  Fields: natural layout
// [ncomp][nz][nx], float64.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels2d.hpp"

namespace smg {
namespace {

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + TPB - 1) / TPB); }

// (A x) at cell (x, z): sum over dz of a_z[z][dz] (m_x * x_row) + m_z[z][dz] (a_x * x_row)
__device__ __forceinline__ double apply2(const double* __restrict__ X, const Lev2& L, int x,
                                         int z) {
  double acc = 0.0;
  for (int dz = -2; dz <= 2; ++dz) {
    const int zz = z + dz;
    if (zz < 0 || zz >= L.nz) continue;  // the z band is zero beyond the walls
    const double az = L.zt[z * 10 + dz + 2], mz = L.zt[z * 10 + 5 + dz + 2];
    if (az == 0.0 && mz == 0.0) continue;
    const double* row = X + (int64_t)zz * L.nx;
    double sm = 0.0, sa = 0.0;
    for (int dx = -2; dx <= 2; ++dx) {
      int xx = x + dx;
      xx = xx < 0 ? xx + L.nx : (xx >= L.nx ? xx - L.nx : xx);
      sm = fma(L.s1d[dx + 2], row[xx], sm);
      sa = fma(L.s1d[5 + dx + 2], row[xx], sa);
    }
    acc = fma(az, sm, fma(mz, sa, acc));
  }
  return acc;
}

__device__ __forceinline__ double diag2(const Lev2& L, int z) {
  return L.zt[z * 10 + 2] * L.s1d[2] + L.zt[z * 10 + 7] * L.s1d[7];
}

// Point heat bath of one colour on level 0: thread p serves the Philox call p, i.e. the sites
// 2p and 2p + 1 (site s = lexicographic index >> 1); site s holds one cell of each colour.
template <bool NOISE>
__global__ __launch_bounds__(TPB) void k2_point_pass(double* __restrict__ xg,
                                                      const double* __restrict__ bg, Lev2 L,
                                                      int colour, double sqkT, NoiseArgs na) {
  const uint32_t comp = blockIdx.y;
  const int64_t N = (int64_t)L.nx * L.nz;
  const int64_t p = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (2 * p >= N / 2) return;
  double* X = xg + comp * N;
  const double* B = bg ? bg + comp * N : nullptr;
  double z0 = 0.0, z1 = 0.0;
  if (NOISE) normal_pair(na, na.sid, comp, (uint32_t)p, z0, z1);
  for (int t = 0; t < 2; ++t) {
    const int64_t s = 2 * p + t;
    if (s >= N / 2) break;
    const int z = (int)((2 * s) / L.nx);
    const int64_t lex = 2 * s + ((colour + z) & 1);
    const int x = (int)(lex - (int64_t)z * L.nx);
    const double d = diag2(L, z);
    double v = X[lex] + ((B ? B[lex] : 0.0) - apply2(X, L, x, z)) / d;
    if (NOISE) v = fma(sqkT / sqrt(d), t ? z1 : z0, v);
    X[lex] = v;
  }
}

// 2 x 2 block heat bath of one colour on a Galerkin level: four lanes per block (cell
// k = dx + 2 dz), x_B += A_BB^-1 (b - A x)_B + sqrt(kT) L_BB^-T n_B with the block's factors
// (one pair per block row, [A_BB^-1 | L_BB^-T] row-major 4 x 4 each).
template <bool NOISE>
__global__ __launch_bounds__(TPB) void k2_block_pass(double* __restrict__ xg,
                                                      const double* __restrict__ bg, Lev2 L,
                                                      int colour, double sqkT, NoiseArgs na) {
  const uint32_t comp = blockIdx.y;
  const int64_t N = (int64_t)L.nx * L.nz;
  const int cx = colour & 1, cz = colour >> 1;
  const int nbx = L.nx / 2, nbz = L.nz / 2;
  const int nix = nbx / 2, njz = (nbz + 1 - cz) / 2;
  const int t = blockIdx.x * TPB + threadIdx.x;
  const int k = t & 3;
  const int blk = t >> 2;
  const bool active = blk < nix * njz;
  const int i = active ? blk % nix : 0, j = active ? blk / nix : 0;
  const int bx = 2 * i + cx, bz = 2 * j + cz;
  const int x = 2 * bx + (k & 1), z = 2 * bz + (k >> 1);
  double* X = xg + comp * N;
  double res = 0.0, xk = 0.0;
  if (active) {
    xk = X[(int64_t)z * L.nx + x];
    res = bg[comp * N + (int64_t)z * L.nx + x] - apply2(X, L, x, z);
  }
  const double* F = L.bfac + (int64_t)bz * 32;
  double v = xk;
  for (int q = 0; q < 4; ++q) v = fma(F[k * 4 + q], __shfl(res, q, 4), v);
  if (NOISE) {
    double z0 = 0.0, z1 = 0.0;
    const uint32_t bid = (uint32_t)(bx + nbx * bz);
    normal_pair(na, na.sid, comp, 2 * bid + (uint32_t)(k >> 1), z0, z1);
    const double nk = (k & 1) ? z1 : z0;
    double e = 0.0;
    for (int q = 0; q < 4; ++q) e = fma(F[16 + k * 4 + q], __shfl(nk, q, 4), e);
    v = fma(sqkT, e, v);
  }
  if (active) X[(int64_t)z * L.nx + x] = v;
}

__global__ __launch_bounds__(TPB) void k2_residual(double* __restrict__ r,
                                                    const double* __restrict__ xg,
                                                    const double* __restrict__ bg, Lev2 L) {
  const uint32_t comp = blockIdx.y;
  const int64_t N = (int64_t)L.nx * L.nz;
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= N) return;
  const int x = (int)(i % L.nx), z = (int)(i / L.nx);
  const double bv = bg ? bg[comp * N + i] : 0.0;
  r[comp * N + i] = bv - apply2(xg + comp * N, L, x, z);
}

// b_c = P^T r (bilinear transpose: weights 1/4, 3/4, 3/4, 1/4 per axis; a fine cell next to a
// wall carries 1/2 for its own coarse cell), and x_c = 0
__global__ __launch_bounds__(TPB) void k2_restrict(double* __restrict__ bc,
                                                    double* __restrict__ xc,
                                                    const double* __restrict__ r, int nxf,
                                                    int nzf) {
  const uint32_t comp = blockIdx.y;
  const int nxc = nxf / 2, nzc = nzf / 2;
  const int64_t Nc = (int64_t)nxc * nzc;
  const int64_t I = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (I >= Nc) return;
  const int X = (int)(I % nxc), Z = (int)(I / nxc);
  const double* R = r + comp * (int64_t)nxf * nzf;
  const double w[4] = {0.25, 0.75, 0.75, 0.25};
  double acc = 0.0;
  for (int a = 0; a < 4; ++a) {
    const int fz = 2 * Z - 1 + a;
    if (fz < 0 || fz >= nzf) continue;
    double wz = w[a];
    if ((Z == 0 && fz == 0) || (Z == nzc - 1 && fz == nzf - 1)) wz = 0.5;
    double sx = 0.0;
    for (int c = 0; c < 4; ++c) {
      int fx = 2 * X - 1 + c;
      fx = fx < 0 ? fx + nxf : (fx >= nxf ? fx - nxf : fx);
      sx = fma(w[c], R[(int64_t)fz * nxf + fx], sx);
    }
    acc = fma(wz, sx, acc);
  }
  bc[comp * Nc + I] = acc;
  if (xc) xc[comp * Nc + I] = 0.0;
}

// x += P e (bilinear on cell centres, the wall ghost -c)
__global__ __launch_bounds__(TPB) void k2_prolong(double* __restrict__ xg,
                                                   const double* __restrict__ e, int nxf,
                                                   int nzf) {
  const uint32_t comp = blockIdx.y;
  const int64_t Nf = (int64_t)nxf * nzf;
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= Nf) return;
  const int nxc = nxf / 2, nzc = nzf / 2;
  const int xf = (int)(i % nxf), zf = (int)(i / nxf);
  const int X0 = xf >> 1, Z0 = zf >> 1;
  int X1 = (xf & 1) ? X0 + 1 : X0 - 1;
  X1 = X1 < 0 ? nxc - 1 : (X1 >= nxc ? 0 : X1);
  int Z1 = (zf & 1) ? Z0 + 1 : Z0 - 1;
  double wz0 = 0.75, wz1 = 0.25;
  if (Z1 < 0 || Z1 >= nzc) {
    wz0 = 0.5;
    wz1 = 0.0;
    Z1 = Z0;
  }
  const double* E = e + comp * (int64_t)nxc * nzc;
  const double r0 = 0.75 * E[(int64_t)Z0 * nxc + X0] + 0.25 * E[(int64_t)Z0 * nxc + X1];
  const double r1 = 0.75 * E[(int64_t)Z1 * nxc + X0] + 0.25 * E[(int64_t)Z1 * nxc + X1];
  xg[comp * Nf + i] += wz0 * r0 + wz1 * r1;
}

}  // namespace

hipError_t launch2_point_pass(double* x, const double* b, const Lev2& L, int ncomp, int colour,
                              double kT, bool noise, const NoiseArgs& na, hipStream_t s) {
  const int64_t calls = ((int64_t)L.nx * L.nz / 2 + 1) / 2;
  dim3 grid(blocks_for(calls), ncomp);
  if (noise) k2_point_pass<true><<<grid, TPB, 0, s>>>(x, b, L, colour, sqrt(kT), na);
  else k2_point_pass<false><<<grid, TPB, 0, s>>>(x, b, L, colour, sqrt(kT), na);
  return hipGetLastError();
}

hipError_t launch2_block_pass(double* x, const double* b, const Lev2& L, int ncomp, int colour,
                              double kT, bool noise, const NoiseArgs& na, hipStream_t s) {
  const int nbx = L.nx / 2, nbz = L.nz / 2;
  const int nblk = (nbx / 2) * ((nbz + 1 - (colour >> 1)) / 2);
  dim3 grid(blocks_for(4 * (int64_t)nblk), ncomp);
  if (noise) k2_block_pass<true><<<grid, TPB, 0, s>>>(x, b, L, colour, sqrt(kT), na);
  else k2_block_pass<false><<<grid, TPB, 0, s>>>(x, b, L, colour, sqrt(kT), na);
  return hipGetLastError();
}

hipError_t launch2_residual(double* r, const double* x, const double* b, const Lev2& L,
                            int ncomp, hipStream_t s) {
  dim3 grid(blocks_for((int64_t)L.nx * L.nz), ncomp);
  k2_residual<<<grid, TPB, 0, s>>>(r, x, b, L);
  return hipGetLastError();
}

hipError_t launch2_restrict(double* bc, double* xc, const double* r, int nxf, int nzf, int ncomp,
                            hipStream_t s) {
  dim3 grid(blocks_for((int64_t)(nxf / 2) * (nzf / 2)), ncomp);
  k2_restrict<<<grid, TPB, 0, s>>>(bc, xc, r, nxf, nzf);
  return hipGetLastError();
}

hipError_t launch2_prolong(double* x, const double* e, int nxf, int nzf, int ncomp,
                           hipStream_t s) {
  dim3 grid(blocks_for((int64_t)nxf * nzf), ncomp);
  k2_prolong<<<grid, TPB, 0, s>>>(x, e, nxf, nzf);
  return hipGetLastError();
}

}  // namespace smg
