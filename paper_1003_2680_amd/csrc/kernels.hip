// HIP kernels of the stochastic multigrid cycle (gfx950, wave64).
//
// Fine level (red-black point heat bath, the stochastic Gauss-Seidel smoother of Sec.
// "Stochastic Iterative Methods"): the field is stored split by colour, so one colour pass
// reads only the other colour (plus b) and writes only its own colour.  A heat-bath update
// never reads the old value of the site it replaces, hence a pass streams exactly
// read(other colour) + write(own colour) = w*N/2 + w*N/2 bytes: the minimum traffic of a
// sweep, with no halo recomputation and no ordering between work-groups.
//
// Galerkin levels (2x2x2 block heat bath with 8 block colours): eight lanes own the eight
// cells of a block; each lane forms its row of b_B - A_{B,rest} x_rest from the 5x5x5 row
// coefficients of its z-row, then the lanes exchange the eight values with cross-lane
// shuffles and apply the precomputed A_BB^-1 and L_BB^-T.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "philox.hpp"

namespace smg {
namespace {

constexpr int TPB = 256;

struct Diag3 {
  double inv_d[3];  // h^2 / (6 + walls)
  double sig[3];    // sqrt(kT h^2 / (6 + walls))
};

__device__ __forceinline__ int wrapm(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// ----------------------------------------------------------------------------- fine level
// One colour pass: xc <- (bc + sum(neighbours)/h^2) h^2/(6+walls) + sigma * n.
// Thread q owns colour sites 2q and 2q+1 and one Philox call.
template <bool HAS_B, bool NOISE>
__global__ __launch_bounds__(TPB) void k_rb_pass(double* __restrict__ xc,
                                                  const double* __restrict__ xo,
                                                  const double* __restrict__ bc, int nh, int ny,
                                                  int nz, uint32_t nsite, int colour,
                                                  double inv_h2, Diag3 dg, NoiseArgs na) {
  const uint32_t comp = blockIdx.y;
  const uint32_t q = blockIdx.x * TPB + threadIdx.x;
  const uint32_t p0 = 2u * q;
  if (p0 >= nsite) return;
  const size_t base = (size_t)comp * nsite;
  const double* __restrict__ o = xo + base;
  double z0 = 0.0, z1 = 0.0;
  if (NOISE) normal_pair(na, comp, q, z0, z1);
  const uint32_t plane = (uint32_t)nh * ny;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const uint32_t p = p0 + t;
    if (p >= nsite) break;
    const uint32_t row = p / nh;
    const int j = p - row * nh;
    const int y = row % ny;
    const int z = row / ny;
    const int xs = (y + z + colour) & 1;
    const uint32_t rb = row * nh;
    const int jl = xs ? j : (j == 0 ? nh - 1 : j - 1);
    const int jr = xs ? (j == nh - 1 ? 0 : j + 1) : j;
    double s = o[rb + jl] + o[rb + jr];
    const int yn = (y + 1 == ny) ? 0 : y + 1;
    const int ys = (y == 0) ? ny - 1 : y - 1;
    s += o[((uint32_t)z * ny + yn) * nh + j] + o[((uint32_t)z * ny + ys) * nh + j];
    int nw = 0;
    if (z + 1 < nz) s += o[rb + j + plane]; else ++nw;
    if (z > 0) s += o[rb + j - plane]; else ++nw;
    double v = s * inv_h2;
    if (HAS_B) v += bc[base + p];
    v *= dg.inv_d[nw];
    if (NOISE) v += dg.sig[nw] * (t == 0 ? z0 : z1);
    xc[base + p] = v;
  }
}

__device__ __forceinline__ double split_at(const double* __restrict__ xr,
                                           const double* __restrict__ xb, size_t cbase, int x,
                                           int y, int z, int nh, int ny) {
  const double* a = ((x + y + z) & 1) ? xb : xr;
  return a[cbase + ((size_t)z * ny + y) * nh + (x >> 1)];
}

// r = b - A x on level 0 (split input, natural output).
template <bool HAS_B>
__global__ __launch_bounds__(TPB) void k_residual0(double* __restrict__ r,
                                                    const double* __restrict__ xr,
                                                    const double* __restrict__ xb,
                                                    const double* __restrict__ br,
                                                    const double* __restrict__ bb, int nx, int ny,
                                                    int nz, uint32_t N, double inv_h2) {
  const uint32_t comp = blockIdx.y;
  const uint32_t i = blockIdx.x * TPB + threadIdx.x;
  if (i >= N) return;
  const int x = i % nx;
  const uint32_t row = i / nx;
  const int y = row % ny;
  const int z = row / ny;
  const int nh = nx >> 1;
  const size_t cb = (size_t)comp * (N >> 1);
  double c = split_at(xr, xb, cb, x, y, z, nh, ny);
  double s = split_at(xr, xb, cb, wrapm(x - 1, nx), y, z, nh, ny) +
             split_at(xr, xb, cb, wrapm(x + 1, nx), y, z, nh, ny) +
             split_at(xr, xb, cb, x, wrapm(y - 1, ny), z, nh, ny) +
             split_at(xr, xb, cb, x, wrapm(y + 1, ny), z, nh, ny);
  int nw = 0;
  if (z + 1 < nz) s += split_at(xr, xb, cb, x, y, z + 1, nh, ny); else ++nw;
  if (z > 0) s += split_at(xr, xb, cb, x, y, z - 1, nh, ny); else ++nw;
  double ax = ((6 + nw) * c - s) * inv_h2;
  double bv = HAS_B ? split_at(br, bb, cb, x, y, z, nh, ny) : 0.0;
  r[(size_t)comp * N + i] = bv - ax;
}

// r = b - A x with the 7-point operator on a natural-layout level (b may be null).
__global__ __launch_bounds__(TPB) void k_residual7_nat(double* __restrict__ r,
                                                        const double* __restrict__ xg,
                                                        const double* __restrict__ bg, int nx,
                                                        int ny, int nz, uint32_t N,
                                                        double inv_h2) {
  const uint32_t comp = blockIdx.y;
  const uint32_t i = blockIdx.x * TPB + threadIdx.x;
  if (i >= N) return;
  const double* X = xg + (size_t)comp * N;
  const int x = i % nx;
  const uint32_t row = i / nx;
  const int y = row % ny;
  const int z = row / ny;
  const uint32_t rb = row * nx;
  double s = X[rb + wrapm(x - 1, nx)] + X[rb + wrapm(x + 1, nx)] +
             X[((uint32_t)z * ny + wrapm(y - 1, ny)) * nx + x] +
             X[((uint32_t)z * ny + wrapm(y + 1, ny)) * nx + x];
  int nw = 0;
  if (z + 1 < nz) s += X[i + (uint32_t)nx * ny]; else ++nw;
  if (z > 0) s += X[i - (uint32_t)nx * ny]; else ++nw;
  double ax = ((6 + nw) * X[i] - s) * inv_h2;
  r[(size_t)comp * N + i] = (bg ? bg[(size_t)comp * N + i] : 0.0) - ax;
}

// ----------------------------------------------------------------------------- transfers
__constant__ double kPW[4] = {0.25, 0.75, 0.75, 0.25};

// b_c = P^T r: each coarse cell gathers the 4x4x4 fine window 2J-1..2J+2 per axis with
// weights (1/4, 3/4, 3/4, 1/4); on the wall axis the fine cell next to a wall carries 1/2.
__global__ __launch_bounds__(TPB) void k_restrict(double* __restrict__ bc,
                                                   const double* __restrict__ r, int nxf,
                                                   int nyf, int nzf, uint32_t Nf, uint32_t Nc) {
  const uint32_t comp = blockIdx.y;
  const uint32_t I = blockIdx.x * TPB + threadIdx.x;
  if (I >= Nc) return;
  const int nxc = nxf >> 1, nyc = nyf >> 1, nzc = nzf >> 1;
  const int X = I % nxc;
  const uint32_t row = I / nxc;
  const int Y = row % nyc;
  const int Z = row / nyc;
  const double* R = r + (size_t)comp * Nf;
  double acc = 0.0;
  for (int c = 0; c < 4; ++c) {
    const int zf = 2 * Z - 1 + c;
    if (zf < 0 || zf >= nzf) continue;
    double wz = kPW[c];
    if ((Z == 0 && zf == 0) || (Z == nzc - 1 && zf == nzf - 1)) wz = 0.5;
    for (int b = 0; b < 4; ++b) {
      const int yf = wrapm(2 * Y - 1 + b, nyf);
      const double wzy = wz * kPW[b];
      const double* Rr = R + ((size_t)zf * nyf + yf) * nxf;
      double s = 0.0;
      for (int a = 0; a < 4; ++a) s += kPW[a] * Rr[wrapm(2 * X - 1 + a, nxf)];
      acc += wzy * s;
    }
  }
  bc[(size_t)comp * Nc + I] = acc;
}

// value of P e at fine cell (xf, yf, zf)
__device__ __forceinline__ double prolong_at(const double* __restrict__ E, int xf, int yf, int zf,
                                             int nxc, int nyc, int nzc) {
  const int X0 = xf >> 1, Y0 = yf >> 1, Z0 = zf >> 1;
  const int X1 = wrapm((xf & 1) ? X0 + 1 : X0 - 1, nxc);
  const int Y1 = wrapm((yf & 1) ? Y0 + 1 : Y0 - 1, nyc);
  int Z1 = (zf & 1) ? Z0 + 1 : Z0 - 1;
  double wz0 = 0.75, wz1 = 0.25;
  if (Z1 < 0 || Z1 >= nzc) {  // ghost beyond the wall carries -e
    wz0 = 0.5;
    wz1 = 0.0;
    Z1 = Z0;
  }
  const size_t pz0 = (size_t)Z0 * nyc, pz1 = (size_t)Z1 * nyc;
  auto plane = [&](size_t pz) {
    const double* r0 = E + (pz + Y0) * nxc;
    const double* r1 = E + (pz + Y1) * nxc;
    return 0.75 * (0.75 * r0[X0] + 0.25 * r0[X1]) + 0.25 * (0.75 * r1[X0] + 0.25 * r1[X1]);
  };
  double v = wz0 * plane(pz0);
  if (wz1 != 0.0) v += wz1 * plane(pz1);
  return v;
}

__global__ __launch_bounds__(TPB) void k_prolong(double* __restrict__ x,
                                                  const double* __restrict__ e, int nxf, int nyf,
                                                  int nzf, uint32_t Nf, uint32_t Nc) {
  const uint32_t comp = blockIdx.y;
  const uint32_t i = blockIdx.x * TPB + threadIdx.x;
  if (i >= Nf) return;
  const int xf = i % nxf;
  const uint32_t row = i / nxf;
  const int yf = row % nyf;
  const int zf = row / nyf;
  x[(size_t)comp * Nf + i] +=
      prolong_at(e + (size_t)comp * Nc, xf, yf, zf, nxf >> 1, nyf >> 1, nzf >> 1);
}

// x += P e into the split level-0 storage (grid.z = colour).
__global__ __launch_bounds__(TPB) void k_prolong0(double* __restrict__ xr,
                                                   double* __restrict__ xb,
                                                   const double* __restrict__ e, int nxf,
                                                   int nyf, int nzf, uint32_t nsite,
                                                   uint32_t Nc) {
  const uint32_t comp = blockIdx.y;
  const int colour = blockIdx.z;
  const uint32_t p = blockIdx.x * TPB + threadIdx.x;
  if (p >= nsite) return;
  const int nh = nxf >> 1;
  const uint32_t row = p / nh;
  const int j = p - row * nh;
  const int yf = row % nyf;
  const int zf = row / nyf;
  const int xf = 2 * j + ((yf + zf + colour) & 1);
  double* X = (colour ? xb : xr) + (size_t)comp * nsite;
  X[p] += prolong_at(e + (size_t)comp * Nc, xf, yf, zf, nxf >> 1, nyf >> 1, nzf >> 1);
}

// ----------------------------------------------------------------------------- Galerkin levels
// r = b - A x with the 5x5x5 row coefficients of each z-row.
__global__ __launch_bounds__(TPB) void k_residual_gal(double* __restrict__ r,
                                                       const double* __restrict__ xg,
                                                       const double* __restrict__ bg,
                                                       const double* __restrict__ coef, int nx,
                                                       int ny, int nz, uint32_t N) {
  const uint32_t comp = blockIdx.y;
  const uint32_t i = blockIdx.x * TPB + threadIdx.x;
  if (i >= N) return;
  const double* X = xg + (size_t)comp * N;
  const int x = i % nx;
  const uint32_t row = i / nx;
  const int y = row % ny;
  const int z = row / ny;
  const double* cf = coef + (size_t)z * 125;
  double acc = 0.0;
  for (int oz = -2; oz <= 2; ++oz) {
    const int zz = z + oz;
    if (zz < 0 || zz >= nz) continue;
    for (int oy = -2; oy <= 2; ++oy) {
      const double* Xr = X + ((size_t)zz * ny + wrapm(y + oy, ny)) * nx;
      const double* c = cf + (oz + 2) * 25 + (oy + 2) * 5;
#pragma unroll
      for (int ox = -2; ox <= 2; ++ox) acc += c[ox + 2] * Xr[wrapm(x + ox, nx)];
    }
  }
  r[(size_t)comp * N + i] = bg[(size_t)comp * N + i] - acc;
}

// One block-colour pass: every 2x2x2 block B of colour `colour` is redrawn from its exact
// conditional  x_B = A_BB^-1 (b_B - A_{B,rest} x_rest) + sqrt(kT) L_BB^-T n_B.
template <bool NOISE>
__global__ __launch_bounds__(TPB) void k_block_pass(double* __restrict__ xg,
                                                     const double* __restrict__ bg,
                                                     const double* __restrict__ coef,
                                                     const double* __restrict__ bfac, int nx,
                                                     int ny, int nz, uint32_t N, int colour,
                                                     int nbx2, int nby2, uint32_t total,
                                                     NoiseArgs na) {
  const uint32_t comp = blockIdx.y;
  const uint32_t t = blockIdx.x * TPB + threadIdx.x;
  const bool active = t < total;  // total is a multiple of 8: whole blocks only
  const int k = t & 7;
  const uint32_t blk = active ? (t >> 3) : 0;
  const int i = blk % nbx2;
  const uint32_t rest = blk / nbx2;
  const int j = rest % nby2;
  const int l = rest / nby2;
  const int bx = 2 * i + (colour & 1);
  const int by = 2 * j + ((colour >> 1) & 1);
  const int bz = 2 * l + (colour >> 2);
  const int cx = 2 * bx + (k & 1);
  const int cy = 2 * by + ((k >> 1) & 1);
  const int cz = 2 * bz + (k >> 2);
  double* X = xg + (size_t)comp * N;
  const uint32_t cell = ((uint32_t)cz * ny + cy) * nx + cx;
  double rhs = 0.0;
  if (active) {
    const double* cf = coef + (size_t)cz * 125;
    double acc = 0.0;
    for (int oz = -2; oz <= 2; ++oz) {
      const int zz = cz + oz;
      if (zz < 0 || zz >= nz) continue;
      const bool inz = (zz >> 1) == bz;
      for (int oy = -2; oy <= 2; ++oy) {
        const int yy = wrapm(cy + oy, ny);
        const bool inzy = inz && (yy >> 1) == by;
        const double* Xr = X + ((size_t)zz * ny + yy) * nx;
        const double* c = cf + (oz + 2) * 25 + (oy + 2) * 5;
#pragma unroll
        for (int ox = -2; ox <= 2; ++ox) {
          const int xx = wrapm(cx + ox, nx);
          if (inzy && (xx >> 1) == bx) continue;  // in-block term
          acc += c[ox + 2] * Xr[xx];
        }
      }
    }
    rhs = bg[(size_t)comp * N + cell] - acc;
  }
  double nrm = 0.0;
  if (NOISE) {
    const uint32_t bid = ((uint32_t)bz * (ny >> 1) + by) * (nx >> 1) + bx;
    double z0, z1;
    normal_pair(na, comp, 4u * bid + (k >> 1), z0, z1);
    nrm = (k & 1) ? z1 : z0;
  }
  const double* F = bfac + (size_t)(active ? bz : 0) * 128;
  double v = 0.0, w = 0.0;
#pragma unroll
  for (int jj = 0; jj < 8; ++jj) {
    v += F[k * 8 + jj] * __shfl(rhs, jj, 8);
    if (NOISE) w += F[64 + k * 8 + jj] * __shfl(nrm, jj, 8);
  }
  if (NOISE) v += na.sqkT * w;
  if (active) X[cell] = v;
}

// ----------------------------------------------------------------------------- coarsest level
// x = A_c^-1 b (+ sqrt(kT) L_c^-T n): rows split over work-groups; every work-group stages b
// and the full noise vector in LDS.
template <bool NOISE>
__global__ __launch_bounds__(TPB) void k_coarsest(double* __restrict__ xg,
                                                   const double* __restrict__ bg,
                                                   const double* __restrict__ ainv,
                                                   const double* __restrict__ w, int n,
                                                   NoiseArgs na) {
  extern __shared__ double sh[];
  const uint32_t comp = blockIdx.y;
  const double* B = bg + (size_t)comp * n;
  for (int i = threadIdx.x; i < n; i += TPB) sh[i] = B[i];
  if (NOISE) {
    for (int q = threadIdx.x; 2 * q < n; q += TPB) {
      double z0, z1;
      normal_pair(na, comp, (uint32_t)q, z0, z1);
      sh[n + 2 * q] = z0;
      if (2 * q + 1 < n) sh[n + 2 * q + 1] = z1;
    }
  }
  __syncthreads();
  const int row = blockIdx.x * TPB + threadIdx.x;
  if (row >= n) return;
  double acc = 0.0;
  for (int jj = 0; jj < n; ++jj) acc += ainv[(size_t)jj * n + row] * sh[jj];
  if (NOISE) {
    double an = 0.0;
    for (int jj = row; jj < n; ++jj) an += w[(size_t)jj * n + row] * sh[n + jj];
    acc += na.sqkT * an;
  }
  xg[(size_t)comp * n + row] = acc;
}

// ----------------------------------------------------------------------------- utilities
__global__ __launch_bounds__(TPB) void k_zero(double* __restrict__ p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * TPB) p[i] = 0.0;
}

__global__ __launch_bounds__(TPB) void k_copy(double* __restrict__ d, const double* __restrict__ s,
                                              int64_t n) {
  int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * TPB) d[i] = s[i];
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_cast(T* __restrict__ d, const double* __restrict__ s,
                                              int64_t n) {
  int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * TPB) d[i] = (T)s[i];
}

__global__ __launch_bounds__(TPB) void k_to_split(double* __restrict__ xr,
                                                   double* __restrict__ xb,
                                                   const double* __restrict__ nat, int nx,
                                                   int ny, uint32_t N) {
  const uint32_t comp = blockIdx.y;
  const uint32_t i = blockIdx.x * TPB + threadIdx.x;
  if (i >= N) return;
  const int x = i % nx;
  const uint32_t row = i / nx;
  const int y = row % ny;
  const int z = row / ny;
  double* a = ((x + y + z) & 1) ? xb : xr;
  a[(size_t)comp * (N >> 1) + row * (nx >> 1) + (x >> 1)] = nat[(size_t)comp * N + i];
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_from_split(T* __restrict__ nat,
                                                     const double* __restrict__ xr,
                                                     const double* __restrict__ xb, int nx,
                                                     int ny, uint32_t N) {
  const uint32_t comp = blockIdx.y;
  const uint32_t i = blockIdx.x * TPB + threadIdx.x;
  if (i >= N) return;
  const int x = i % nx;
  const uint32_t row = i / nx;
  const int y = row % ny;
  const int z = row / ny;
  const double* a = ((x + y + z) & 1) ? xb : xr;
  nat[(size_t)comp * N + i] = (T)a[(size_t)comp * (N >> 1) + row * (nx >> 1) + (x >> 1)];
}

// Fixed-order sums of squares: stage 1 writes one partial per 256-element block.
__global__ __launch_bounds__(TPB) void k_sumsq_part(double* __restrict__ part,
                                                     const double* __restrict__ v, int64_t n,
                                                     uint32_t nblk) {
  __shared__ double sh[TPB];
  const uint32_t comp = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  double a = 0.0;
  if (i < n) {
    double t = v[(size_t)comp * n + i];
    a = t * t;
  }
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)comp * nblk + blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(TPB) void k_sumsq_final(double* __restrict__ out,
                                                      const double* __restrict__ part,
                                                      uint32_t nblk) {
  __shared__ double sh[TPB];
  const uint32_t comp = blockIdx.x;
  double a = 0.0;
  for (uint32_t i = threadIdx.x; i < nblk; i += TPB) a += part[(size_t)comp * nblk + i];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[comp] = sh[0];
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + TPB - 1) / TPB); }

inline unsigned grid_stride_blocks(int64_t n) {
  int64_t b = (n + TPB - 1) / TPB;
  return (unsigned)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

}  // namespace

hipError_t launch_rb_pass(double* xc, const double* xo, const double* bc, int nx, int ny, int nz,
                          int ncomp, int colour, double h, double kT, bool noise,
                          const NoiseArgs& na, hipStream_t s) {
  const int nh = nx / 2;
  const uint32_t nsite = (uint32_t)nh * ny * nz;
  Diag3 dg;
  for (int w = 0; w < 3; ++w) {
    dg.inv_d[w] = h * h / (6.0 + w);
    dg.sig[w] = sqrt(kT * h * h / (6.0 + w));
  }
  const double ih2 = 1.0 / (h * h);
  dim3 grid(blocks_for((nsite + 1) / 2), ncomp);
  if (bc) {
    if (noise) k_rb_pass<true, true><<<grid, TPB, 0, s>>>(xc, xo, bc, nh, ny, nz, nsite, colour, ih2, dg, na);
    else k_rb_pass<true, false><<<grid, TPB, 0, s>>>(xc, xo, bc, nh, ny, nz, nsite, colour, ih2, dg, na);
  } else {
    if (noise) k_rb_pass<false, true><<<grid, TPB, 0, s>>>(xc, xo, bc, nh, ny, nz, nsite, colour, ih2, dg, na);
    else k_rb_pass<false, false><<<grid, TPB, 0, s>>>(xc, xo, bc, nh, ny, nz, nsite, colour, ih2, dg, na);
  }
  return hipGetLastError();
}

hipError_t launch_residual0(double* r, const double* xr, const double* xb, const double* br,
                            const double* bb, int nx, int ny, int nz, int ncomp, double h,
                            hipStream_t s) {
  const uint32_t N = (uint32_t)nx * ny * nz;
  dim3 grid(blocks_for(N), ncomp);
  if (br) k_residual0<true><<<grid, TPB, 0, s>>>(r, xr, xb, br, bb, nx, ny, nz, N, 1.0 / (h * h));
  else k_residual0<false><<<grid, TPB, 0, s>>>(r, xr, xb, br, bb, nx, ny, nz, N, 1.0 / (h * h));
  return hipGetLastError();
}

hipError_t launch_residual7_nat(double* r, const double* x, const double* b, int nx, int ny,
                                int nz, int ncomp, double h, hipStream_t s) {
  const uint32_t N = (uint32_t)nx * ny * nz;
  dim3 grid(blocks_for(N), ncomp);
  k_residual7_nat<<<grid, TPB, 0, s>>>(r, x, b, nx, ny, nz, N, 1.0 / (h * h));
  return hipGetLastError();
}

hipError_t launch_residual_gal(double* r, const double* x, const double* b, const double* coef,
                               int nx, int ny, int nz, int ncomp, hipStream_t s) {
  const uint32_t N = (uint32_t)nx * ny * nz;
  dim3 grid(blocks_for(N), ncomp);
  k_residual_gal<<<grid, TPB, 0, s>>>(r, x, b, coef, nx, ny, nz, N);
  return hipGetLastError();
}

hipError_t launch_restrict(double* bc, const double* r, int nxf, int nyf, int nzf, int ncomp,
                           hipStream_t s) {
  const uint32_t Nf = (uint32_t)nxf * nyf * nzf;
  const uint32_t Nc = Nf / 8;
  dim3 grid(blocks_for(Nc), ncomp);
  k_restrict<<<grid, TPB, 0, s>>>(bc, r, nxf, nyf, nzf, Nf, Nc);
  return hipGetLastError();
}

hipError_t launch_prolong0(double* xr, double* xb, const double* e, int nxf, int nyf, int nzf,
                           int ncomp, hipStream_t s) {
  const uint32_t nsite = (uint32_t)(nxf / 2) * nyf * nzf;
  const uint32_t Nc = (uint32_t)(nxf / 2) * (nyf / 2) * (nzf / 2);
  dim3 grid(blocks_for(nsite), ncomp, 2);
  k_prolong0<<<grid, TPB, 0, s>>>(xr, xb, e, nxf, nyf, nzf, nsite, Nc);
  return hipGetLastError();
}

hipError_t launch_prolong(double* x, const double* e, int nxf, int nyf, int nzf, int ncomp,
                          hipStream_t s) {
  const uint32_t Nf = (uint32_t)nxf * nyf * nzf;
  dim3 grid(blocks_for(Nf), ncomp);
  k_prolong<<<grid, TPB, 0, s>>>(x, e, nxf, nyf, nzf, Nf, Nf / 8);
  return hipGetLastError();
}

hipError_t launch_block_pass(double* x, const double* b, const double* coef, const double* bfac,
                             int nx, int ny, int nz, int ncomp, int colour, bool noise,
                             const NoiseArgs& na, hipStream_t s) {
  const int nbx2 = nx / 4, nby2 = ny / 4;
  const int nbz = nz / 2;
  const int nbzc = (nbz + 1 - (colour >> 2)) / 2;
  const uint32_t total = (uint32_t)nbx2 * nby2 * nbzc * 8;
  if (total == 0) return hipSuccess;
  const uint32_t N = (uint32_t)nx * ny * nz;
  dim3 grid(blocks_for(total), ncomp);
  if (noise) k_block_pass<true><<<grid, TPB, 0, s>>>(x, b, coef, bfac, nx, ny, nz, N, colour, nbx2, nby2, total, na);
  else k_block_pass<false><<<grid, TPB, 0, s>>>(x, b, coef, bfac, nx, ny, nz, N, colour, nbx2, nby2, total, na);
  return hipGetLastError();
}

hipError_t launch_coarsest(double* x, const double* b, const double* ainv, const double* w, int n,
                           int ncomp, bool noise, const NoiseArgs& na, hipStream_t s) {
  dim3 grid(blocks_for(n), ncomp);
  size_t lds = (size_t)(noise ? 2 : 1) * n * sizeof(double);
  if (noise) k_coarsest<true><<<grid, TPB, lds, s>>>(x, b, ainv, w, n, na);
  else k_coarsest<false><<<grid, TPB, lds, s>>>(x, b, ainv, w, n, na);
  return hipGetLastError();
}

hipError_t launch_zero(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_zero<<<grid_stride_blocks(n), TPB, 0, s>>>(p, n);
  return hipGetLastError();
}

hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_copy<<<grid_stride_blocks(n), TPB, 0, s>>>(dst, src, n);
  return hipGetLastError();
}

hipError_t launch_cast(void* dst, int out_f32, const double* src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (out_f32) k_cast<float><<<grid_stride_blocks(n), TPB, 0, s>>>((float*)dst, src, n);
  else k_cast<double><<<grid_stride_blocks(n), TPB, 0, s>>>((double*)dst, src, n);
  return hipGetLastError();
}

hipError_t launch_to_split(double* xr, double* xb, const double* nat, int nx, int ny, int nz,
                           int ncomp, hipStream_t s) {
  const uint32_t N = (uint32_t)nx * ny * nz;
  dim3 grid(blocks_for(N), ncomp);
  k_to_split<<<grid, TPB, 0, s>>>(xr, xb, nat, nx, ny, N);
  return hipGetLastError();
}

hipError_t launch_from_split(void* nat, int out_f32, const double* xr, const double* xb, int nx,
                             int ny, int nz, int ncomp, hipStream_t s) {
  const uint32_t N = (uint32_t)nx * ny * nz;
  dim3 grid(blocks_for(N), ncomp);
  if (out_f32) k_from_split<float><<<grid, TPB, 0, s>>>((float*)nat, xr, xb, nx, ny, N);
  else k_from_split<double><<<grid, TPB, 0, s>>>((double*)nat, xr, xb, nx, ny, N);
  return hipGetLastError();
}

hipError_t launch_sumsq(double* out, double* part, const double* v, int64_t n, int ncomp,
                        hipStream_t s) {
  const uint32_t nblk = blocks_for(n);
  k_sumsq_part<<<dim3(nblk, ncomp), TPB, 0, s>>>(part, v, n, nblk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_sumsq_final<<<ncomp, TPB, 0, s>>>(out, part, nblk);
  return hipGetLastError();
}

}  // namespace smg
