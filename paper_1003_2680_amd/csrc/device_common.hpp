// Device helpers shared by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"

namespace smg {

constexpr int TPB = 256;

__device__ __forceinline__ int wrapm(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// padded LDS strides (doubles) of an nx x ny x nz field
__host__ __device__ inline int lds_sy(int nx) { return nx + 2; }
__host__ __device__ inline int lds_sz(int nx, int ny) { return ny * (nx + 2) + 1; }
__host__ __device__ inline int lds_field(int nx, int ny, int nz) { return nz * lds_sz(nx, ny); }

// Quotient and remainder by d, using a shift when d is a power of two (lg2 >= 0).
__device__ __forceinline__ uint32_t udiv(uint32_t a, uint32_t d, int lg2) {
  return lg2 >= 0 ? (a >> lg2) : a / d;
}

// 1D prolongation weights for the fine cells 2J-1, 2J, 2J+1, 2J+2 around coarse cell J.
template <typename T = double>
__device__ __forceinline__ T pw(int i) { return (i == 1 || i == 2) ? T(0.75) : T(0.25); }

// XCD-aware work-group numbering.  The dispatcher deals work-groups to the 8 XCDs round-robin
// by linear id, and each XCD has its own L2.  Renumbering so that XCD k runs the k-th
// contiguous eighth of the grid keeps neighbouring tiles (which share halo rows and planes)
// on one L2.  A bijection on [0, total); the ragged tail beyond a multiple of 8 keeps its ids.
constexpr uint32_t kXcds = 8;
struct Blk3 {
  uint32_t x, y, z;
};
__device__ __forceinline__ Blk3 xcd_block() {
  const uint32_t gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
  const uint32_t total = gx * gy * gz;
  uint32_t lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const uint32_t per = total / kXcds;
  if (lin < per * kXcds) lin = (lin % kXcds) * per + lin / kXcds;
  Blk3 b;
  b.x = lin % gx;
  const uint32_t r = lin / gx;
  b.y = r % gy;
  b.z = r / gy;
  return b;
}

// q = v / d, r = v % d for v >= 0 and a wave-uniform d > 0: a shift and a mask when d is a power
// of two (the usual level extents), else the division.
__device__ __forceinline__ void divmod_uniform(int v, int d, int& q, int& r) {
  if ((d & (d - 1)) == 0) {
    const int lg = __builtin_ctz((unsigned)d);
    q = v >> lg;
    r = v & (d - 1);
  } else {
    q = v / d;
    r = v - q * d;
  }
}

// Periodic index of a staged halo position: v mod n for -n <= v < 2n.  A tile that overhangs
// a small level may stage positions further out; no cell inside the level reads them (a
// stencil reaches at most two cells, and n >= 4), so they are clamped into range instead of
// reduced by a division.
__device__ __forceinline__ int wrap_near(int v, int n) {
  if (v < 0) v += n;
  if (v >= n) v -= n;
  return v < n ? v : n - 1;
}

// (A x) at cell (cx, cy, cz) of a Galerkin level.  The Galerkin operator of the wall-bounded
// Laplacian is a Kronecker sum, A = a_z (x) m_y (x) m_x + m_z (x) (a_y (x) m_x + m_y (x) a_x),
// with 5-point periodic 1D stencils s1d = (m_x, a_x, m_y, a_y) (offsets -2..2, uniform over
// the level) and the wall-axis rows zt[cz] = (a_z[cz][cz+dz], m_z[cz][cz+dz]).  Each row of a
// plane is reduced with m_x and a_x, then the plane with m_y and a_y: 65 FMAs per plane.
// Rows beyond a wall have zero z-factors; their loads are clamped into the grid so the
// accumulation is branch-free.
// Fields are addressed as X[z*sz + y*sy + x]; global fields use sy = nx, sz = nx*ny, LDS copies
// use padded strides (sy = 2 mod 4, sz = 1 mod 4 doubles) so that the 64 lanes of a wave --
// 8 blocks x 8 cells -- spread evenly over the LDS banks.
template <typename T>
__device__ __forceinline__ T gal_plane(const T* __restrict__ P, int sy, const int* xs,
                                       const int* ys, const T* s1d, T& p1) {
  T q0[5], q1[5];
#pragma unroll
  for (int dy = 0; dy < 5; ++dy) {
    const T* row = P + (size_t)ys[dy] * sy;
    T sm = 0, sa = 0;
#pragma unroll
    for (int dx = 0; dx < 5; ++dx) {
      const T v = row[xs[dx]];
      sm = fma(s1d[dx], v, sm);
      sa = fma(s1d[5 + dx], v, sa);
    }
    q0[dy] = sm;
    q1[dy] = sa;
  }
  T p0 = 0, pa = 0, pb = 0;
#pragma unroll
  for (int dy = 0; dy < 5; ++dy) {
    p0 = fma(s1d[10 + dy], q0[dy], p0);
    pa = fma(s1d[15 + dy], q0[dy], pa);
    pb = fma(s1d[10 + dy], q1[dy], pb);
  }
  p1 = pa + pb;
  return p0;
}

// v of the lane two apart in the same quad (lane ^ 2) by one DPP move per 32-bit half.
__device__ __forceinline__ double dpp_xor2(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)u, 0x4E, 0xf, 0xf, false);  // quad_perm [2,3,0,1]
  const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), 0x4E, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float dpp_xor2(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xf, 0xf, false));
}

// The in-plane sums of gal_plane for the two cells (x, y) and (x, y+1) of a block column,
// shared by the lanes ky = 0, 1 (lane ^ 2).  Together they need the six rows y-2 .. y+3; each
// lane reduces three of them along x, rows[i] = y_lane + s (i - 2) with s = +1 for ky = 0 and
// -1 for ky = 1, i.e. the outer three rows of its own window listed from its far edge inwards.
// The periodic 1D factors m_y, a_y are symmetric, so in that order both lanes weight rows i by
// factor i for their own cell, and rows 1, 2 by factors 0, 1 for the partner's cell; the
// partner's share arrives by one DPP move.  15 LDS reads and 51 instructions per lane instead
// of 25 and 65.  Every lane of the quad must call this.
template <typename T>
__device__ __forceinline__ void gal_plane_pair(const T* __restrict__ P, int sy, const int* xs,
                                               const int (&rows)[3], const T* s1d, T& q0,
                                               T& q1) {
  T rm[3], ra[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const T* row = P + (size_t)rows[i] * sy;
    T sm = 0, sa = 0;
#pragma unroll
    for (int dx = 0; dx < 5; ++dx) {
      const T v = row[xs[dx]];
      sm = fma(s1d[dx], v, sm);
      sa = fma(s1d[5 + dx], v, sa);
    }
    rm[i] = sm;
    ra[i] = sa;
  }
  const T* my = s1d + 10;
  const T* ay = s1d + 15;
  T o0 = 0, o1 = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    o0 = fma(my[i], rm[i], o0);
    o1 = fma(ay[i], rm[i], o1);
    o1 = fma(my[i], ra[i], o1);
  }
  T p0 = my[0] * rm[1];
  p0 = fma(my[1], rm[2], p0);
  T p1 = ay[0] * rm[1];
  p1 = fma(ay[1], rm[2], p1);
  p1 = fma(my[0], ra[1], p1);
  p1 = fma(my[1], ra[2], p1);
  q0 = o0 + dpp_xor2(p0);
  q1 = o1 + dpp_xor2(p1);
}

// UNROLL_Z: all five planes in flight at once (global-memory operands, where load latency
// dominates); otherwise one plane at a time (LDS operands, fewer registers).
template <typename T, bool UNROLL_Z = false>
__device__ __forceinline__ T gal_apply(const T* __restrict__ X, int sy, int sz, const T* s1d,
                                       const T* __restrict__ zt, int nx, int ny, int nz, int cx,
                                       int cy, int cz) {
  const T* zr = zt + cz * 10;
  int xs[5], ys[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    xs[d] = wrapm(cx + d - 2, nx);
    ys[d] = wrapm(cy + d - 2, ny);
  }
  T acc0 = 0, acc1 = 0;
  auto plane = [&](int dz) {
    int zz = cz + dz - 2;
    zz = zz < 0 ? 0 : (zz >= nz ? nz - 1 : zz);
    T p1;
    const T p0 = gal_plane<T>(X + (size_t)zz * sz, sy, xs, ys, s1d, p1);
    acc0 = fma(zr[dz], p0, acc0);
    acc1 = fma(zr[5 + dz], p1, acc1);
  };
  if constexpr (UNROLL_Z) {
#pragma unroll
    for (int dz = 0; dz < 5; ++dz) plane(dz);
  } else {
#pragma unroll 1
    for (int dz = 0; dz < 5; ++dz) plane(dz);
  }
  return acc0 + acc1;
}

// The two z-layers of a 2x2x2 block see six Galerkin planes between them; lane kz of a block
// reduces planes 3kz .. 3kz+2 (q) and receives its partner's three (o).  The cell's own
// window of five planes (dz = 0 .. 4, i.e. planes kz .. kz+4) is then one select per entry
// between two registers, never an indexed access into a private array (which would be
// placed in scratch memory).
template <typename T>
__device__ __forceinline__ void plane_window(int kz, const T (&q)[3], const T (&o)[3],
                                             T (&w)[5]) {
  w[0] = kz ? o[1] : q[0];
  w[1] = kz ? o[2] : q[1];
  w[2] = kz ? q[0] : q[2];
  w[3] = kz ? q[1] : o[0];
  w[4] = kz ? q[2] : o[1];
}

// Block heat-bath lane: lane k (0..7) of 2x2x2 block (bx,by,bz) returns its new value
//   x_B[k] = sum_j A_BB^-1[k][j] rhs_j + sqrt(kT) sum_j L_BB^-T[k][j] n_j,
//   rhs_j  = b_j - (A x)_j + sum_i A_BB[j][i] x_B[i]   (= b_j - A_{j,rest} x_rest).
// The eight lanes of a block must be consecutive lanes of one wave (shuffle width 8) and all
// lanes of the wave must call this together; inactive lanes pass active = false.
// The lane's noise comes from a pregenerated field Z (natural layout of the level, one value
// per cell and sweep): the block's normals already multiplied by sqrt(kT) L_BB^-T.
template <typename T, bool NOISE>
__device__ __forceinline__ T block_lane(const T* __restrict__ X, int sy, int sz,
                                        const T* __restrict__ Bv, const T* s1d,
                                        const T* __restrict__ zt, const T* __restrict__ bfac,
                                        int nx, int ny, int nz, int bx, int by, int bz, int k,
                                        bool active, const T* __restrict__ Z,
                                        uint32_t& cell_out) {
  const int cx = 2 * bx + (k & 1);
  const int cy = 2 * by + ((k >> 1) & 1);
  const int cz = 2 * bz + (k >> 2);
  const uint32_t cell = (uint32_t)cz * sz + (uint32_t)cy * sy + cx;
  cell_out = cell;
  T ax = 0, xk = 0, bk = 0, nrm = 0;
  if (active) {
    if (NOISE) nrm = Z[((uint32_t)cz * ny + cy) * nx + cx];
    xk = X[cell];
    bk = Bv[cell];
  }
  {
    // The block's two z-layers reach the same six planes 2bz-2 .. 2bz+3 (clamped at the
    // walls, where their factors vanish): lane kz reduces planes 3kz .. 3kz+2 and trades them
    // with its partner lane ^ 4.  Every lane takes part (the shuffles need the partner).
    const int kz = k >> 2;
    int xs[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) xs[d] = wrapm(cx + d - 2, nx);
    const int ky = (k >> 1) & 1;
    int rows[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) rows[i] = wrapm(cy + (ky ? 2 - i : i - 2), ny);
    T q0[3], q1[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      int pz = 2 * bz - 2 + 3 * kz + j;
      pz = pz < 0 ? 0 : (pz >= nz ? nz - 1 : pz);
      gal_plane_pair<T>(X + (size_t)pz * sz, sy, xs, rows, s1d, q0[j], q1[j]);
    }
    T o0[3], o1[3], w0[5], w1[5];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      o0[j] = __shfl_xor(q0[j], 4, 8);
      o1[j] = __shfl_xor(q1[j], 4, 8);
    }
    plane_window(kz, q0, o0, w0);
    plane_window(kz, q1, o1, w1);
    if (active) {
      const T* zr = zt + cz * 10;
      T acc0 = 0, acc1 = 0;
#pragma unroll
      for (int dz = 0; dz < 5; ++dz) {
        acc0 = fma(zr[dz], w0[dz], acc0);
        acc1 = fma(zr[5 + dz], w1[dz], acc1);
      }
      ax = acc0 + acc1;
    }
  }
  // x_B + A_BB^-1 (b_B - (A x)_B) equals A_BB^-1 (b_B - A_B,rest x_rest): the block's own
  // coupling cancels, so only the residual needs to be shared across the block's lanes
  const T* F = bfac + (size_t)(active ? bz : 0) * 192;
  const T res = bk - ax;
  T v0 = xk, v1 = NOISE ? nrm : T(0);
#pragma unroll
  for (int j = 0; j < 8; j += 2) {
    v0 = fma(F[k * 8 + j], __shfl(res, j, 8), v0);
    v1 = fma(F[k * 8 + j + 1], __shfl(res, j + 1, 8), v1);
  }
  return v0 + v1;
}

// b_c = P^T r at coarse cell (X,Y,Z): 4x4x4 fine window 2J-1..2J+2 per axis, weights
// (1/4, 3/4, 3/4, 1/4); on the wall axis the fine cell next to a wall carries 1/2.
template <typename T>
__device__ __forceinline__ T restrict_at(const T* __restrict__ R, int sy, int sz, int nxf, int nyf,
                                         int nzf, int X, int Y, int Z) {
  const int nzc = nzf >> 1;
  T acc = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int zf = 2 * Z - 1 + c;
    if (zf < 0 || zf >= nzf) continue;
    T wz = pw<T>(c);
    if ((Z == 0 && zf == 0) || (Z == nzc - 1 && zf == nzf - 1)) wz = T(0.5);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int yf = wrapm(2 * Y - 1 + b, nyf);
      const T* Rr = R + (size_t)zf * sz + (size_t)yf * sy;
      T s = 0;
#pragma unroll
      for (int a = 0; a < 4; ++a) s = fma(pw<T>(a), Rr[wrapm(2 * X - 1 + a, nxf)], s);
      acc = fma(wz * pw<T>(b), s, acc);
    }
  }
  return acc;
}

// (P e) at fine cell (xf, yf, zf): trilinear, 3/4 to the own parent and 1/4 to the next one;
// beyond a wall the ghost parent carries -e, so the wall-layer cell gets 1/2 e.
template <typename T>
__device__ __forceinline__ T prolong_at(const T* __restrict__ E, int sy, int sz, int xf, int yf,
                                        int zf, int nxc, int nyc, int nzc) {
  const int X0 = xf >> 1, Y0 = yf >> 1, Z0 = zf >> 1;
  const int X1 = wrapm((xf & 1) ? X0 + 1 : X0 - 1, nxc);
  const int Y1 = wrapm((yf & 1) ? Y0 + 1 : Y0 - 1, nyc);
  int Z1 = (zf & 1) ? Z0 + 1 : Z0 - 1;
  T wz0 = T(0.75), wz1 = T(0.25);
  if (Z1 < 0 || Z1 >= nzc) {
    wz0 = T(0.5);
    wz1 = T(0);
    Z1 = Z0;
  }
  const T* r00 = E + (size_t)Z0 * sz + (size_t)Y0 * sy;
  const T* r01 = E + (size_t)Z0 * sz + (size_t)Y1 * sy;
  const T* r10 = E + (size_t)Z1 * sz + (size_t)Y0 * sy;
  const T* r11 = E + (size_t)Z1 * sz + (size_t)Y1 * sy;
  const T q = T(0.75), o = T(0.25);
  const T p0 = q * (q * r00[X0] + o * r00[X1]) + o * (q * r01[X0] + o * r01[X1]);
  const T p1 = q * (q * r10[X0] + o * r10[X1]) + o * (q * r11[X0] + o * r11[X1]);
  return wz0 * p0 + wz1 * p1;
}

}  // namespace smg
