// Kernels of the composite-grid FAC cycle: point heat-bath classes of the composite sweep, the
// composite residual, the transfers between the composite unknowns and the base grid, the
// 2x2x2 block heat bath and residual of the Galerkin base levels (sparse stencil dictionary)
// and the dense draw of the coarsest base level.  Operator, classes and noise streams as
// described in composite.hpp.  T is the storage and arithmetic type of a sweep: double in the
// FP64 form, float for the inner cycle of the FP32-refined form (whose residual, refinement and
// coarsest draw stay FP64).
#include "composite.hpp"
#include "device_common.hpp"

namespace smg {
namespace {

inline uint32_t grid_for(int64_t n) { return (uint32_t)((n + TPB - 1) / TPB); }

__device__ __forceinline__ bool covered(const CompGeom& g, int x, int y, int z) {
  return x >= g.x0 && x < g.x1 && y >= g.y0 && y < g.y1 && z >= g.z0 && z < g.z1;
}

// fine cells with a face on the box boundary towards coarse cells
__device__ __forceinline__ bool on_layer(const CompGeom& g, int i, int j, int k) {
  return i == 0 || i == g.fx - 1 || j == 0 || j == g.fy - 1 || (k == 0 && g.z0 > 0) ||
         (k == g.fz - 1 && g.z1 < g.nz);
}

__device__ __forceinline__ int fidx(const CompGeom& g, int i, int j, int k) {
  return i + g.fx * (j + g.fy * k);
}

// 1/sqrt(a) for a > 0: the hardware estimate refined by Newton steps y <- y (3/2 - (a/2) y^2),
// each of which roughly squares the relative error (two for FP64, one for FP32), within a few
// ulp.  The point passes take 1/a = r^2 and the noise scale sqrt(kT) r from it, instead of a
// division, a square root and a second division per cell.
template <typename T>
__device__ __forceinline__ T rsqrt_refined(T a);
template <>
__device__ __forceinline__ double rsqrt_refined<double>(double a) {
  double y = __builtin_amdgcn_rsq(a);
  const double h = 0.5 * a;
  y = y * fma(-h, y * y, 1.5);
  y = y * fma(-h, y * y, 1.5);
  return y;
}
template <>
__device__ __forceinline__ float rsqrt_refined<float>(float a) {
  float y = __builtin_amdgcn_rsqf(a);
  return y * fmaf(-0.5f * a, y * y, 1.5f);
}

// the normal of `site` in the stream of na: call site/2, first or second of the pair
template <typename T>
__device__ __forceinline__ T normal_at(const NoiseArgs& na, uint32_t site) {
  T z0, z1;
  normal_pair_t<T>(na, na.sid, 0u, site >> 1, z0, z1);
  return (site & 1) ? z1 : z0;
}

// Row of coarse cell (x,y,z) in units of 1/h^2: diag = A_ii, off = sum_j (-A_ij) x_j.  The six
// neighbour values are loaded back to back (a covered or wall neighbour loads the cell itself,
// an in-range address, and is discarded); the rare coarse-fine faces are added afterwards.
template <typename T>
__device__ __forceinline__ void coarse_row(const T* __restrict__ xc, const T* __restrict__ xf,
                                           const CompGeom& g, int x, int y, int z, T& diag,
                                           T& off) {
  const int self = x + g.nx * (y + g.ny * z);
  int q[6];
  bool wall[6], cov[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    const int axis = d >> 1;
    const int sgn = (d & 1) ? -1 : 1;
    const int qx = axis == 0 ? wrapm(x + sgn, g.nx) : x;
    const int qy = axis == 1 ? wrapm(y + sgn, g.ny) : y;
    const int qz = axis == 2 ? z + sgn : z;
    wall[d] = qz < 0 || qz >= g.nz;
    cov[d] = !wall[d] && covered(g, qx, qy, qz);
    q[d] = (wall[d] || cov[d]) ? self : qx + g.nx * (qy + g.ny * qz);
  }
  T v[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) v[d] = xc[q[d]];
  diag = T(0);
  off = T(0);
  bool any_cov = false;
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    any_cov |= cov[d];
    if (wall[d]) {
      diag += T(2);
    } else if (!cov[d]) {
      diag += T(1);
      off += v[d];
    }
  }
  if (any_cov) {
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      if (!cov[d]) continue;
      const int axis = d >> 1;
      const int sgn = (d & 1) ? -1 : 1;
      const int qx = axis == 0 ? wrapm(x + sgn, g.nx) : x;
      const int qy = axis == 1 ? wrapm(y + sgn, g.ny) : y;
      const int qz = axis == 2 ? z + sgn : z;
      // the four children of q on its face towards (x, y, z)
      const int i0 = 2 * (qx - g.x0), j0 = 2 * (qy - g.y0), k0 = 2 * (qz - g.z0);
      const int side = sgn > 0 ? 0 : 1;
      T s;
      if (axis == 0) {
        s = xf[fidx(g, i0 + side, j0, k0)] + xf[fidx(g, i0 + side, j0 + 1, k0)] +
            xf[fidx(g, i0 + side, j0, k0 + 1)] + xf[fidx(g, i0 + side, j0 + 1, k0 + 1)];
      } else if (axis == 1) {
        s = xf[fidx(g, i0, j0 + side, k0)] + xf[fidx(g, i0 + 1, j0 + side, k0)] +
            xf[fidx(g, i0, j0 + side, k0 + 1)] + xf[fidx(g, i0 + 1, j0 + side, k0 + 1)];
      } else {
        s = xf[fidx(g, i0, j0, k0 + side)] + xf[fidx(g, i0 + 1, j0, k0 + side)] +
            xf[fidx(g, i0, j0 + 1, k0 + side)] + xf[fidx(g, i0 + 1, j0 + 1, k0 + side)];
      }
      diag += T(4.0 / 3.0);
      off = fma(s, T(1.0 / 3.0), off);
    }
  }
}

// Rows (y, z) of the base grid more than one cell from the box in y (periodically) or in z: no
// cell of such a row and no face neighbour of one is covered.
__device__ __forceinline__ bool far_row(const CompGeom& g, int y, int z) {
  const bool zn = z >= g.z0 - 1 && z <= g.z1;
  const bool yn = (unsigned)wrapm(y - g.y0 + 1, g.ny) <= (unsigned)(g.y1 - g.y0 + 1);
  return !(yn && zn);
}

// coarse_row for cell x of a far row (index `row` = y + ny z, rows rp, rm of y + 1, y - 1, walls
// below / above when wlo / whi): the same loads, order and arithmetic without the cover tests.
template <typename T>
__device__ __forceinline__ void far_coarse_row(const T* __restrict__ xc, const CompGeom& g, int x,
                                               int row, int rp, int rm, bool wlo, bool whi,
                                               T& diag, T& off) {
  const int nx = g.nx;
  const int c = x + nx * row;
  const int xp = x + 1 == nx ? 0 : x + 1, xm = x == 0 ? nx - 1 : x - 1;
  const int plane = nx * g.ny;
  const T v0 = xc[xp + nx * row], v1 = xc[xm + nx * row];
  const T v2 = xc[x + nx * rp], v3 = xc[x + nx * rm];
  const T v4 = xc[whi ? c : c + plane], v5 = xc[wlo ? c : c - plane];
  diag = T(4) + (whi ? T(2) : T(1)) + (wlo ? T(2) : T(1));
  off = T(0);
  off += v0;
  off += v1;
  off += v2;
  off += v3;
  if (!whi) off += v4;
  if (!wlo) off += v5;
}

// Row of fine cell (i,j,k) (box coordinates) in units of 1/h^2, loads first as above: the six
// neighbours inside the box (an outside neighbour loads the cell itself), then the faces on the
// box boundary (walls, or coarse-fine faces, only on the interface layer).
template <typename T>
__device__ __forceinline__ void fine_row(const T* __restrict__ xf, const T* __restrict__ xc,
                                         const CompGeom& g, int i, int j, int k, T& diag,
                                         T& off) {
  const int me = fidx(g, i, j, k);
  int q[6];
  bool in[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    const int axis = d >> 1;
    const int sgn = (d & 1) ? -1 : 1;
    const int c = (axis == 0 ? i : (axis == 1 ? j : k)) + sgn;
    const int n = axis == 0 ? g.fx : (axis == 1 ? g.fy : g.fz);
    in[d] = c >= 0 && c < n;
    const int ni = axis == 0 ? c : i, nj = axis == 1 ? c : j, nk = axis == 2 ? c : k;
    q[d] = in[d] ? fidx(g, ni, nj, nk) : me;
  }
  T v[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) v[d] = xf[q[d]];
  const T self = xf[me];
  diag = T(0);
  off = T(0);
  bool edge = false;
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    edge |= !in[d];
    if (in[d]) {
      diag += T(0.5);
      off = fma(T(0.5), v[d], off);
    }
  }
  if (!edge) return;
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    if (in[d]) continue;
    const int axis = d >> 1;
    const int sgn = (d & 1) ? -1 : 1;
    int ax = g.x0 + (i >> 1), ay = g.y0 + (j >> 1), az = g.z0 + (k >> 1);
    if (axis == 0) {
      ax = sgn > 0 ? (g.x1 == g.nx ? 0 : g.x1) : (g.x0 == 0 ? g.nx - 1 : g.x0 - 1);
    } else if (axis == 1) {
      ay = sgn > 0 ? (g.y1 == g.ny ? 0 : g.y1) : (g.y0 == 0 ? g.ny - 1 : g.y0 - 1);
    } else {
      az = sgn > 0 ? g.z1 : g.z0 - 1;
      if (az < 0 || az >= g.nz) {  // wall face of a fine cell
        diag += T(1);
        continue;
      }
    }
    // coarse-fine face: the three other fine cells of the parent's face share its gradient
    const int ib = i & ~1, jb = j & ~1, kb = k & ~1;
    T s;
    if (axis == 0) {
      s = xf[fidx(g, i, jb, kb)] + xf[fidx(g, i, jb + 1, kb)] + xf[fidx(g, i, jb, kb + 1)] +
          xf[fidx(g, i, jb + 1, kb + 1)];
    } else if (axis == 1) {
      s = xf[fidx(g, ib, j, kb)] + xf[fidx(g, ib + 1, j, kb)] + xf[fidx(g, ib, j, kb + 1)] +
          xf[fidx(g, ib + 1, j, kb + 1)];
    } else {
      s = xf[fidx(g, ib, jb, k)] + xf[fidx(g, ib + 1, jb, k)] + xf[fidx(g, ib, jb + 1, k)] +
          xf[fidx(g, ib + 1, jb + 1, k)];
    }
    diag += T(1.0 / 12.0);
    off = fma(xc[ax + g.nx * (ay + g.ny * az)], T(1.0 / 3.0), off);
    off = fma(s - self, T(-1.0 / 12.0), off);
  }
}

// Coarse class `colour` (cells with (x+y+z) % 2 == colour).  Its noise site is the cell's base
// index halved, h = jx + (nx/2) row with x = 2 jx + ((y+z+colour) & 1); thread t takes the
// sites 2t and 2t + 1, the two normals of Philox call t.
template <typename T, bool NOISE>
__global__ __launch_bounds__(TPB) void k_comp_coarse_pass(T* __restrict__ xc,
                                                          const T* __restrict__ bc,
                                                          const T* __restrict__ xf, CompGeom g,
                                                          int colour, NoiseArgs na) {
  const int hx = g.nx >> 1;
  const uint32_t t = blockIdx.x * TPB + threadIdx.x;
  if (2 * t >= (uint32_t)hx * g.ny * g.nz) return;  // hx ny nz is even (ny is)
  T z[2] = {T(0), T(0)};
  if (NOISE) normal_pair_t<T>(na, na.sid, 0u, t, z[0], z[1]);
  if ((hx & 1) == 0) {
    // both sites in one row; a far row (the bulk of the grid) skips every cover test
    int row, jx, y, zz;
    divmod_uniform((int)(2 * t), hx, row, jx);
    divmod_uniform(row, g.ny, zz, y);
    if (far_row(g, y, zz)) {
      const int rp = y + 1 == g.ny ? row + 1 - g.ny : row + 1;
      const int rm = y == 0 ? row - 1 + g.ny : row - 1;
      const bool wlo = zz == 0, whi = zz == g.nz - 1;
      const int x0 = 2 * jx + ((y + zz + colour) & 1);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int x = x0 + 2 * q;
        T diag, off;
        far_coarse_row<T>(xc, g, x, row, rp, rm, wlo, whi, diag, off);
        const uint32_t cell = x + g.nx * row;
        const T ih2 = (T)g.ih2;
        const T ra = rsqrt_refined<T>(diag * ih2);
        T v = ((bc ? bc[cell] : T(0)) + off * ih2) * (ra * ra);
        if (NOISE) v = fma((T)na.sqkT * ra, z[q], v);
        xc[cell] = v;
      }
      return;
    }
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const uint32_t h = 2 * t + q;
    const int jx = h % hx;
    const int row = h / hx;
    const int y = row % g.ny, zz = row / g.ny;
    const int x = 2 * jx + ((y + zz + colour) & 1);
    if (covered(g, x, y, zz)) continue;
    T diag, off;
    coarse_row<T>(xc, xf, g, x, y, zz, diag, off);
    const uint32_t cell = x + g.nx * (y + g.ny * zz);
    const T ih2 = (T)g.ih2;
    const T ra = rsqrt_refined<T>(diag * ih2);
    T v = ((bc ? bc[cell] : T(0)) + off * ih2) * (ra * ra);
    if (NOISE) v = fma((T)na.sqkT * ra, z[q], v);
    xc[cell] = v;
  }
}

// Fine cell (i, j, k) with its normal n.
template <typename T, bool NOISE>
__device__ __forceinline__ void fine_update(T* __restrict__ xf, const T* __restrict__ bf,
                                            const T* __restrict__ xc, const CompGeom& g, int i,
                                            int j, int k, const NoiseArgs& na, T n) {
  T diag, off;
  fine_row<T>(xf, xc, g, i, j, k, diag, off);
  const uint32_t cell = fidx(g, i, j, k);
  const T ih2 = (T)g.ih2;
  const T ra = rsqrt_refined<T>(diag * ih2);
  T v = ((bf ? bf[cell] : T(0)) + off * ih2) * (ra * ra);
  if (NOISE) v = fma((T)na.sqkT * ra, n, v);
  xf[cell] = v;
}

// Fine class 2 + colour off the interface layer: noise sites as for the coarse classes (the
// box index halved), thread t the sites 2t and 2t + 1 of Philox call t.
template <typename T, bool NOISE>
__global__ __launch_bounds__(TPB) void k_comp_fine_pass(T* __restrict__ xf,
                                                        const T* __restrict__ bf, CompGeom g,
                                                        int colour, NoiseArgs na) {
  const int hx = g.fx >> 1;
  const uint32_t t = blockIdx.x * TPB + threadIdx.x;
  if (2 * t >= (uint32_t)hx * g.fy * g.fz) return;  // hx fy fz is even (fy is)
  T z[2] = {T(0), T(0)};
  if (NOISE) normal_pair_t<T>(na, na.sid, 0u, t, z[0], z[1]);
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const uint32_t h = 2 * t + q;
    const int jx = h % hx;
    const int row = h / hx;
    const int j = row % g.fy, k = row / g.fy;
    const int i = 2 * jx + ((j + k + colour) & 1);
    if (on_layer(g, i, j, k)) continue;
    // off the layer every neighbour is a fine cell or a wall: the coarse field is never read
    fine_update<T, NOISE>(xf, bf, nullptr, g, i, j, k, na, z[q]);
  }
}

template <typename T, bool NOISE>
__global__ __launch_bounds__(TPB) void k_comp_layer_pass(T* __restrict__ xf,
                                                         const T* __restrict__ bf,
                                                         const T* __restrict__ xc, CompGeom g,
                                                         const int32_t* __restrict__ cells,
                                                         int count, NoiseArgs na) {
  const int t = blockIdx.x * TPB + threadIdx.x;
  if (t >= count) return;
  const int site = cells[t];  // layer classes: the noise site is the box index itself
  const int i = site % g.fx;
  const int row = site / g.fx;
  fine_update<T, NOISE>(xf, bf, xc, g, i, row % g.fy, row / g.fy, na,
                        NOISE ? normal_at<T>(na, (uint32_t)site) : T(0));
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_comp_res_coarse(T* __restrict__ rc,
                                                         const T* __restrict__ xc,
                                                         const T* __restrict__ xf,
                                                         const T* __restrict__ bc, CompGeom g) {
  const uint32_t t = blockIdx.x * TPB + threadIdx.x;
  if (t >= (uint32_t)g.nx * g.ny * g.nz) return;
  int x, row, y, z;
  divmod_uniform((int)t, g.nx, row, x);
  divmod_uniform(row, g.ny, z, y);
  T diag, off;
  if (far_row(g, y, z)) {
    far_coarse_row<T>(xc, g, x, row, y + 1 == g.ny ? row + 1 - g.ny : row + 1,
                      y == 0 ? row - 1 + g.ny : row - 1, z == 0, z == g.nz - 1, diag, off);
  } else if (covered(g, x, y, z)) {
    rc[t] = T(0);
    return;
  } else {
    coarse_row<T>(xc, xf, g, x, y, z, diag, off);
  }
  rc[t] = (bc ? bc[t] : T(0)) - (diag * xc[t] - off) * (T)g.ih2;
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_comp_res_fine(T* __restrict__ rf,
                                                       const T* __restrict__ xf,
                                                       const T* __restrict__ xc,
                                                       const T* __restrict__ bf, CompGeom g) {
  const uint32_t t = blockIdx.x * TPB + threadIdx.x;
  if (t >= (uint32_t)g.fx * g.fy * g.fz) return;
  const int i = t % g.fx;
  const int row = t / g.fx;
  T diag, off;
  fine_row<T>(xf, xc, g, i, row % g.fy, row / g.fy, diag, off);
  rf[t] = (bf ? bf[t] : T(0)) - (diag * xf[t] - off) * (T)g.ih2;
}

// 1D weights P(p, J) of the fine cells p = 2J-1 .. 2J+2 (absolute fine coordinates) around base
// cell J; on the wall axis the child next to a wall takes 3/4 - 1/4 (antisymmetric ghost).
// Returns the count of fine cells inside [lo, lo + n) with their box coordinates.
template <typename T>
__device__ __forceinline__ int restrict_1d(int J, int nbase, bool periodic, int lo, int n,
                                           int* idx, T* w) {
  int cnt = 0;
#pragma unroll
  for (int d = -1; d <= 2; ++d) {
    int p = 2 * J + d;
    if (periodic) {
      p = p < 0 ? p + 2 * nbase : (p >= 2 * nbase ? p - 2 * nbase : p);
    } else if (p < 0 || p >= 2 * nbase) {
      continue;
    }
    const int q = p - lo;
    if (q < 0 || q >= n) continue;
    T wt = (d == 0 || d == 1) ? T(0.75) : T(0.25);
    if (!periodic && ((d == 0 && J == 0) || (d == 1 && J == nbase - 1))) wt -= T(0.25);
    idx[cnt] = q;
    w[cnt] = wt;
    ++cnt;
  }
  return cnt;
}

// b0 = P^T r over the base grid and x0 = 0.  The coarse residual either comes from rc or (rc
// null) is formed here from (xc, xf, bc), so the cycle never stores it.
template <typename T>
__global__ __launch_bounds__(TPB) void k_comp_restrict(T* __restrict__ b0, T* __restrict__ x0,
                                                       const T* __restrict__ rc,
                                                       const T* __restrict__ rf,
                                                       const T* __restrict__ xc,
                                                       const T* __restrict__ xf,
                                                       const T* __restrict__ bc, CompGeom g) {
  const uint32_t t = blockIdx.x * TPB + threadIdx.x;
  if (t >= (uint32_t)g.nx * g.ny * g.nz) return;
  int X, row, Y, Z;
  divmod_uniform((int)t, g.nx, row, X);
  divmod_uniform(row, g.ny, Z, Y);
  if (!rc && far_row(g, Y, Z)) {
    // no fine cell restricts onto a far row: the coarse residual alone
    T diag, off;
    far_coarse_row<T>(xc, g, X, row, Y + 1 == g.ny ? row + 1 - g.ny : row + 1,
                      Y == 0 ? row - 1 + g.ny : row - 1, Z == 0, Z == g.nz - 1, diag, off);
    b0[t] = (bc ? bc[t] : T(0)) - (diag * xc[t] - off) * (T)g.ih2;
    x0[t] = T(0);
    return;
  }
  T v;
  if (rc) {
    v = rc[t];
  } else if (covered(g, X, Y, Z)) {
    v = T(0);
  } else {
    T diag, off;
    coarse_row<T>(xc, xf, g, X, Y, Z, diag, off);
    v = (bc ? bc[t] : T(0)) - (diag * xc[t] - off) * (T)g.ih2;
  }
  int ix[4], iy[4], iz[4];
  T wx[4], wy[4], wz[4];
  const int cx = restrict_1d<T>(X, g.nx, true, 2 * g.x0, g.fx, ix, wx);
  if (cx > 0) {
    const int cy = restrict_1d<T>(Y, g.ny, true, 2 * g.y0, g.fy, iy, wy);
    const int cz = cy > 0 ? restrict_1d<T>(Z, g.nz, false, 2 * g.z0, g.fz, iz, wz) : 0;
    for (int c = 0; c < cz; ++c)
      for (int b = 0; b < cy; ++b) {
        T s = T(0);
        for (int a = 0; a < cx; ++a) s = fma(wx[a], rf[fidx(g, ix[a], iy[b], iz[c])], s);
        v = fma(wz[c] * wy[b], s, v);
      }
  }
  b0[t] = v;
  x0[t] = T(0);
}

// trilinear 1D entries of fine coordinate p: (J, 3/4) and (neighbour, 1/4); at a wall the
// neighbour is the ghost -c_J
template <typename T>
__device__ __forceinline__ void prolong_1d(int p, int nbase, bool periodic, int* J, T* w) {
  const int j = p >> 1;
  int o = (p & 1) ? j + 1 : j - 1;
  J[0] = j;
  w[0] = T(0.75);
  if (periodic) {
    J[1] = wrapm(o, nbase);
    w[1] = T(0.25);
  } else if (o >= 0 && o < nbase) {
    J[1] = o;
    w[1] = T(0.25);
  } else {
    J[1] = j;
    w[1] = T(-0.25);
  }
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_comp_prolong_coarse(T* __restrict__ xc,
                                                             const T* __restrict__ y,
                                                             CompGeom g) {
  const uint32_t t = blockIdx.x * TPB + threadIdx.x;
  if (t >= (uint32_t)g.nx * g.ny * g.nz) return;
  const int x = t % g.nx;
  const int row = t / g.nx;
  if (!covered(g, x, row % g.ny, row / g.ny)) xc[t] += y[t];
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_comp_prolong_fine(T* __restrict__ xf,
                                                           const T* __restrict__ y, CompGeom g) {
  const uint32_t t = blockIdx.x * TPB + threadIdx.x;
  if (t >= (uint32_t)g.fx * g.fy * g.fz) return;
  const int i = t % g.fx;
  const int row = t / g.fx;
  const int j = row % g.fy, k = row / g.fy;
  int JX[2], JY[2], JZ[2];
  T wx[2], wy[2], wz[2];
  prolong_1d<T>(2 * g.x0 + i, g.nx, true, JX, wx);
  prolong_1d<T>(2 * g.y0 + j, g.ny, true, JY, wy);
  prolong_1d<T>(2 * g.z0 + k, g.nz, false, JZ, wz);
  T v = T(0);
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const T* yr = y + (size_t)g.nx * (JY[b] + g.ny * JZ[c]);
      const T s = fma(wx[0], yr[JX[0]], wx[1] * yr[JX[1]]);
      v = fma(wz[c] * wy[b], s, v);
    }
  xf[t] += v;
}

// ---------------------------------------------------------------- Galerkin base levels
__device__ __forceinline__ void decode(int code, int& dx, int& dy, int& dz) {
  dz = code / 25 - 2;
  dy = (code / 5) % 5 - 2;
  dx = code % 5 - 2;
}

// Partial sum over the stencil entries e0 + sub, e0 + sub + S, ... of cell `cell` = (cx, cy, cz)
// with in-block index k: r -= a_e x[target_e], skipping targets inside the cell's 2x2x2 block
// when SKIP.  Eight (coefficient, offset) records are loaded at a time, then their eight
// gathers, with no branch between them (the record table is padded by kEntryPad records, and a
// slot past the row's end loads the cell itself with a zero coefficient), so the latencies
// overlap.  AWAY: the cell is at least two cells from the periodic seams in x and y and adds the
// record's linear offset to its index (walls never take a target out of the grid in z); else
// the decoded offsets are wrapped.
template <typename T, int S, bool SKIP, bool AWAY>
__device__ __forceinline__ T stencil_run(const GStencilT<T>& st, const T* __restrict__ x, int e,
                                         int e1, uint32_t kbit, uint32_t cell, int cx, int cy,
                                         int cz, T r) {
  for (; e < e1; e += 8 * S) {
    StEntryT<T> en[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) en[q] = st.ent[e + q * S];
    T xv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      uint32_t tgt;
      if (AWAY) {
        tgt = cell + en[q].lin;
      } else {
        int dx, dy, dz;
        decode(en[q].meta & 0xff, dx, dy, dz);
        tgt = wrapm(cx + dx, st.nx) + st.nx * (wrapm(cy + dy, st.ny) + st.ny * (cz + dz));
      }
      xv[q] = x[e + q * S < e1 ? tgt : cell];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const bool use = e + q * S < e1 && !(SKIP && (en[q].meta & kbit));
      r = fma(use ? -en[q].a : T(0), xv[q], r);
    }
  }
  return r;
}

// stencil_run for a wave whose cells all take row `sid` and lie away from the seams (no skip):
// the row's records are wave-uniform and come through scalar loads, each lane picking the one of
// its sub-lane, so a lane issues only its gathers; same entries, order and arithmetic.
// a value equal on every lane of the wave, marked as such (kept in scalar registers)
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float wave_uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double wave_uniform(double v) {
  const long long u = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)u);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <typename T, int S>
__device__ __forceinline__ T stencil_uniform(const GStencilT<T>& st, const T* __restrict__ x,
                                             int sid, int sub, uint32_t cell, T r) {
  const int e1 = wave_uniform(st.st_off[sid + 1]);
  for (int e = wave_uniform(st.st_off[sid]); e < e1; e += 8 * S) {
    T a[8], xv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      T aq = wave_uniform(st.ent[e + q * S].a);
      int lq = wave_uniform(st.ent[e + q * S].lin);
#pragma unroll
      for (int j = 1; j < S; ++j) {
        const T aj = wave_uniform(st.ent[e + q * S + j].a);
        const int lj = wave_uniform(st.ent[e + q * S + j].lin);
        aq = sub == j ? aj : aq;
        lq = sub == j ? lj : lq;
      }
      const bool in = e + q * S + sub < e1;
      a[q] = in ? -aq : T(0);
      xv[q] = x[in ? cell + lq : cell];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) r = fma(a[q], xv[q], r);
  }
  return r;
}

template <typename T, int S, bool SKIP>
__device__ __forceinline__ T stencil_partial(const GStencilT<T>& st, const T* __restrict__ x,
                                             int sid, int sub, int k, uint32_t cell, int cx,
                                             int cy, int cz, bool away, T r) {
  const int e = st.st_off[sid] + sub, e1 = st.st_off[sid + 1];
  const uint32_t kbit = 1u << (8 + k);
  return away ? stencil_run<T, S, SKIP, true>(st, x, e, e1, kbit, cell, cx, cy, cz, r)
              : stencil_run<T, S, SKIP, false>(st, x, e, e1, kbit, cell, cx, cy, cz, r);
}

// sum over the S consecutive lanes of a row
template <typename T, int S>
__device__ __forceinline__ T row_reduce(T r) {
#pragma unroll
  for (int m = 1; m < S; m <<= 1) r += __shfl_xor(r, m, S);
  return r;
}

// 8*S lanes per 2x2x2 block: S lanes share the row of each of its 8 cells (in-block index
// k = dx + 2dy + 4dz).  The cells' residuals against everything outside the block are
// exchanged within the group and the block is drawn from its conditional law
// x_B = A_BB^-1 r_B + sqrt(kT) L_BB^-T n_B; the first lane of each row writes it.
// MODE 0: every block of the colour; MODE 1: the plain 7-point blocks of the colour only (the
// others are left to MODE 2); MODE 2: the listed blocks of the colour.
template <typename T, bool NOISE, int S, int MODE>
__device__ __forceinline__ void gblock_body(T* __restrict__ x, const T* __restrict__ b,
                                            const GStencilT<T>& st, int colour,
                                            const NoiseArgs& na, uint32_t t) {
  const int nbx = st.nx >> 1, nby = st.ny >> 1, nbz = st.nz >> 1;
  const int hbx = nbx >> 1, hby = nby >> 1;
  const int pz = colour >> 2;
  const int nbzc = (nbz + 1 - pz) >> 1;
  // the total is a multiple of 8*S and so is TPB: a block's group of lanes is active as a whole
  const uint32_t nblocks = MODE == 2 ? (uint32_t)(st.list_off[colour + 1] - st.list_off[colour])
                                     : (uint32_t)hbx * hby * nbzc;
  if (t >= nblocks * 8 * S) return;
  const int sub = t % S;
  const int k = (t / S) & 7;
  const uint32_t q = t / (8 * S);
  int bx, by, bz;
  if (MODE == 2) {
    const int lb = st.list[st.list_off[colour] + q];
    bx = lb % nbx;
    by = (lb / nbx) % nby;
    bz = lb / (nbx * nby);
  } else {
    const int i = q % hbx;
    const uint32_t q2 = q / hbx;
    bx = 2 * i + (colour & 1);
    by = 2 * (int)(q2 % hby) + ((colour >> 1) & 1);
    bz = 2 * (int)(q2 / hby) + pz;
  }
  const int cx = 2 * bx + (k & 1), cy = 2 * by + ((k >> 1) & 1), cz = 2 * bz + (k >> 2);
  const uint32_t blk = bx + nbx * (by + nby * bz);
  const int typ = st.btype[blk];
  if (MODE == 1 && st.bt_c7[typ] == T(0)) return;  // the whole group shares the type
  const uint32_t cell = cx + st.nx * (cy + st.ny * cz);
  T r = (b && sub == 0) ? b[cell] : T(0);
  // the three face neighbours away from the block, loaded before the block type resolves (a
  // wall neighbour loads the cell itself and is dropped)
  T xn0 = T(0), xn1 = T(0), xn2 = T(0);
  bool zin = false;
  if (MODE == 1) {
    const int tx = wrapm(cx + ((k & 1) ? 1 : -1), st.nx);
    const int ty = wrapm(cy + ((k & 2) ? 1 : -1), st.ny);
    const int tz = cz + ((k & 4) ? 1 : -1);
    zin = tz >= 0 && tz < st.nz;
    xn0 = x[tx + st.nx * (cy + st.ny * cz)];
    xn1 = x[cx + st.nx * (ty + st.ny * cz)];
    xn2 = x[zin ? cx + st.nx * (cy + st.ny * tz) : cell];
  }
  const T c7 = MODE == 1 ? st.bt_c7[typ] : T(0);
  if (c7 != T(0)) {
    // plain 7-point rows: one coefficient for every off-block face neighbour
    r = fma(-c7, xn0 + xn1 + (zin ? xn2 : T(0)), r);
  } else {
    const int sid = st.bt_sid[typ * 8 + k];
    const bool away = bx >= 1 && bx + 2 <= nbx && by >= 1 && by + 2 <= nby;
    r = row_reduce<T, S>(
        stencil_partial<T, S, true>(st, x, sid, sub, k, cell, cx, cy, cz, away, r));
  }
  const T* F = st.bt_fac + (size_t)typ * 128;
  T v = T(0);
#pragma unroll
  for (int m = 0; m < 8; ++m) v = fma(F[k * 8 + m], __shfl(r, m * S, 8 * S), v);
  if (NOISE) {
    T z0, z1;
    normal_pair_t<T>(na, na.sid, 0u, (8u * blk + k) >> 1, z0, z1);
    const T nk = (k & 1) ? z1 : z0;
    T w = T(0);
#pragma unroll
    for (int m = 0; m < 8; ++m) w = fma(F[64 + k * 8 + m], __shfl(nk, m * S, 8 * S), w);
    v = fma((T)na.sqkT, w, v);
  }
  if (sub == 0) x[cell] = v;
}

template <typename T, bool NOISE, int S, int MODE>
__global__ __launch_bounds__(TPB) void k_gblock_pass(T* __restrict__ x, const T* __restrict__ b,
                                                     GStencilT<T> st, int colour, NoiseArgs na) {
  gblock_body<T, NOISE, S, MODE>(x, b, st, colour, na, blockIdx.x * TPB + threadIdx.x);
}

// MODE 2 and MODE 1 of one colour in one launch (the two touch disjoint blocks of the colour and
// read only the other colours): the first `listed_wg` work-groups take the listed blocks with S
// lanes per row, the rest every block of the colour with one lane per row.  The long-row groups
// come first so that their longer chains of gathers overlap the plain blocks.
template <typename T, bool NOISE, int S>
__global__ __launch_bounds__(TPB) void k_gblock_pass_mixed(T* __restrict__ x,
                                                           const T* __restrict__ b,
                                                           GStencilT<T> st, int colour,
                                                           NoiseArgs na, uint32_t listed_wg) {
  if (blockIdx.x < listed_wg)
    gblock_body<T, NOISE, S, 2>(x, b, st, colour, na, blockIdx.x * TPB + threadIdx.x);
  else
    gblock_body<T, NOISE, 1, 1>(x, b, st, colour, na,
                                (blockIdx.x - listed_wg) * TPB + threadIdx.x);
}

// MODE 0: every cell with S lanes per row; MODE 1: the cells of plain 7-point blocks only;
// MODE 2: the cells of the listed blocks (all colours), eight lanes per row.
template <typename T, int S, int MODE>
__device__ __forceinline__ void gresidual_body(T* __restrict__ r, const T* __restrict__ x,
                                               const T* __restrict__ b, const GStencilT<T>& st,
                                               uint32_t t) {
  const int sub = t % S;
  uint32_t c, blk;
  int cx, cy, cz, k;
  if (MODE == 2) {
    if (t >= (uint32_t)st.list_off[8] * 8 * S) return;
    k = (t / S) & 7;
    const int lb = st.list[t / (8 * S)];
    const int nbx = st.nx >> 1, nby = st.ny >> 1;
    cx = 2 * (lb % nbx) + (k & 1);
    cy = 2 * ((lb / nbx) % nby) + ((k >> 1) & 1);
    cz = 2 * (lb / (nbx * nby)) + (k >> 2);
    c = cx + st.nx * (cy + st.ny * cz);
    blk = lb;
  } else {
    if (t >= (uint32_t)st.nx * st.ny * st.nz * S) return;
    c = t / S;
    cx = c % st.nx;
    const int row = c / st.nx;
    cy = row % st.ny;
    cz = row / st.ny;
    blk = (cx >> 1) + (st.nx >> 1) * ((cy >> 1) + (st.ny >> 1) * (cz >> 1));
    k = (cx & 1) + 2 * (cy & 1) + 4 * (cz & 1);
  }
  const int typ = st.btype[blk];
  if (MODE == 1 && st.bt_c7[typ] == T(0)) return;
  T v = (b && sub == 0) ? b[c] : T(0);
  T sum = T(0), xs = T(0);
  if (MODE == 1) {
    // the six neighbours and the cell, loaded before the block type resolves
    const int xm = wrapm(cx - 1, st.nx), xp = wrapm(cx + 1, st.nx);
    const int ym = wrapm(cy - 1, st.ny), yp = wrapm(cy + 1, st.ny);
    const size_t rowo = (size_t)st.nx * (cy + st.ny * cz);
    const size_t pl = (size_t)st.nx * st.ny;
    const T zm = x[cz > 0 ? c - pl : c];
    const T zp = x[cz + 1 < st.nz ? c + pl : c];
    xs = x[c];
    sum = x[xm + rowo] + x[xp + rowo] + x[cx + st.nx * (ym + st.ny * cz)] +
          x[cx + st.nx * (yp + st.ny * cz)] + (cz > 0 ? zm : T(0)) +
          (cz + 1 < st.nz ? zp : T(0));
  }
  const T c7 = MODE == 1 ? st.bt_c7[typ] : T(0);
  if (c7 != T(0)) {
    v = fma(-st.bt_diag[typ * 8 + k], xs, fma(-c7, sum, v));
  } else {
    const int sid = st.bt_sid[typ * 8 + k];
    const bool away = cx >= 2 && cx + 3 <= st.nx && cy >= 2 && cy + 3 <= st.ny;
    const int sid0 = __builtin_amdgcn_readfirstlane(sid);
    if (MODE == 0 && S == 2 && __all(sid == sid0 && away))
      v = row_reduce<T, S>(stencil_uniform<T, S>(st, x, sid0, sub, c, v));
    else
      v = row_reduce<T, S>(
          stencil_partial<T, S, false>(st, x, sid, sub, k, c, cx, cy, cz, away, v));
  }
  if (sub == 0) r[c] = v;
}

template <typename T, int S, int MODE>
__global__ __launch_bounds__(TPB) void k_gresidual(T* __restrict__ r, const T* __restrict__ x,
                                                   const T* __restrict__ b, GStencilT<T> st) {
  gresidual_body<T, S, MODE>(r, x, b, st, blockIdx.x * TPB + threadIdx.x);
}

// MODE 2 and MODE 1 in one launch, as k_gblock_pass_mixed
template <typename T, int S>
__global__ __launch_bounds__(TPB) void k_gresidual_mixed(T* __restrict__ r,
                                                         const T* __restrict__ x,
                                                         const T* __restrict__ b, GStencilT<T> st,
                                                         uint32_t listed_wg) {
  if (blockIdx.x < listed_wg)
    gresidual_body<T, S, 2>(r, x, b, st, blockIdx.x * TPB + threadIdx.x);
  else
    gresidual_body<T, 1, 1>(r, x, b, st, (blockIdx.x - listed_wg) * TPB + threadIdx.x);
}

// Coarsest base level: z = the n normals of the level's stream (call j/2, first or second of the
// pair, FP64 in every form), then x = A_c^-1 b (+ sqrt(kT) L_c^-T z) in FP64 with one wave per
// row (A_c^-1 symmetric and L_c^-T stored row-major, so every lane reads along a row).
__global__ __launch_bounds__(TPB) void k_dense_noise(double* __restrict__ z, int n, NoiseArgs na) {
  const int q = blockIdx.x * TPB + threadIdx.x;
  if (2 * q >= n) return;
  double z0, z1;
  normal_pair(na, na.sid, 0u, (uint32_t)q, z0, z1);
  z[2 * q] = z0;
  if (2 * q + 1 < n) z[2 * q + 1] = z1;
}

template <typename T, bool NOISE>
__global__ __launch_bounds__(TPB) void k_dense_draw(T* __restrict__ x, const T* __restrict__ b,
                                                    const double* __restrict__ ainv,
                                                    const double* __restrict__ wt,
                                                    const double* __restrict__ z, int n,
                                                    double sqkT) {
  const int row = blockIdx.x * (TPB / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const double* a = ainv + (size_t)row * n;
  double acc = 0.0, an = 0.0;
  for (int j = lane; j < n; j += 64) acc = fma(a[j], (double)b[j], acc);
  if (NOISE) {
    const double* w = wt + (size_t)row * n;
    for (int j = row + lane; j < n; j += 64) an = fma(w[j], z[j], an);
    acc = fma(sqkT, an, acc);
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
  if (lane == 0) x[row] = (T)acc;
}


// Right-hand side of the field noise w = L^-1 Q eta with Q = diag(q) (Appendix A): since
// L = M^-1 S = -h^3 M^-1 A, the field solves A w = -(volume/h^3) q eta, with volume/h^3 = 1 on
// coarse cells and 1/8 on fine cells; covered base cells get 0.  One thread per Philox call (two
// sites): calls [0, nbase/2) fill the coarse part (stream nac, site = base cell), the rest the
// fine part (stream naf, site = fine index).  q null = 1.  nbase and nfine are even (nx and the
// fine extents are).
__global__ __launch_bounds__(TPB) void k_comp_forcing(double* __restrict__ bc,
                                                       double* __restrict__ bf,
                                                       const double* __restrict__ qc,
                                                       const double* __restrict__ qf, CompGeom g,
                                                       NoiseArgs nac, NoiseArgs naf) {
  const int64_t nbase = (int64_t)g.nx * g.ny * g.nz;
  const int64_t nf = (int64_t)g.fx * g.fy * g.fz;
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  double z[2];
  if (t < (nbase >> 1)) {
    normal_pair(nac, nac.sid, 0u, (uint32_t)t, z[0], z[1]);
    for (int k = 0; k < 2; ++k) {
      const int64_t i = 2 * t + k;
      const int x = (int)(i % g.nx);
      const int64_t row = i / g.nx;
      const int y = (int)(row % g.ny), zz = (int)(row / g.ny);
      bc[i] = covered(g, x, y, zz) ? 0.0 : -(qc ? qc[i] : 1.0) * z[k];
    }
  } else if (t - (nbase >> 1) < (nf >> 1)) {
    const int64_t c = t - (nbase >> 1);
    normal_pair(naf, naf.sid, 0u, (uint32_t)c, z[0], z[1]);
    for (int k = 0; k < 2; ++k) {
      const int64_t i = 2 * c + k;
      bf[i] = -0.125 * (qf ? qf[i] : 1.0) * z[k];
    }
  }
}
}  // namespace

template <typename T>
hipError_t launch_dense_draw(T* x, const T* b, const double* ainv, const double* wt, double* z,
                             int n, bool noise, const NoiseArgs& na, hipStream_t s) {
  if (noise) {
    k_dense_noise<<<grid_for((n + 1) / 2), TPB, 0, s>>>(z, n, na);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_dense_draw<T, true><<<(n + 3) / 4, TPB, 0, s>>>(x, b, ainv, wt, z, n, na.sqkT);
  } else {
    k_dense_draw<T, false><<<(n + 3) / 4, TPB, 0, s>>>(x, b, ainv, wt, z, n, na.sqkT);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_comp_coarse_pass(T* xc, const T* bc, const T* xf, const CompGeom& g, int colour,
                                   bool noise, const NoiseArgs& na, hipStream_t s) {
  const uint32_t grid = grid_for((int64_t)(g.nx / 2) * g.ny * g.nz / 2);  // two cells a thread
  if (noise) k_comp_coarse_pass<T, true><<<grid, TPB, 0, s>>>(xc, bc, xf, g, colour, na);
  else k_comp_coarse_pass<T, false><<<grid, TPB, 0, s>>>(xc, bc, xf, g, colour, na);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_comp_fine_pass(T* xf, const T* bf, const CompGeom& g, int colour, bool noise,
                                 const NoiseArgs& na, hipStream_t s) {
  const uint32_t grid = grid_for((int64_t)(g.fx / 2) * g.fy * g.fz / 2);  // two cells a thread
  if (noise) k_comp_fine_pass<T, true><<<grid, TPB, 0, s>>>(xf, bf, g, colour, na);
  else k_comp_fine_pass<T, false><<<grid, TPB, 0, s>>>(xf, bf, g, colour, na);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_comp_layer_pass(T* xf, const T* bf, const T* xc, const CompGeom& g,
                                  const int32_t* cells, int count, bool noise, const NoiseArgs& na,
                                  hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const uint32_t grid = grid_for(count);
  if (noise) k_comp_layer_pass<T, true><<<grid, TPB, 0, s>>>(xf, bf, xc, g, cells, count, na);
  else k_comp_layer_pass<T, false><<<grid, TPB, 0, s>>>(xf, bf, xc, g, cells, count, na);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_comp_residual(T* rc, T* rf, const T* xc, const T* xf, const T* bc, const T* bf,
                                const CompGeom& g, hipStream_t s) {
  k_comp_res_coarse<T><<<grid_for((int64_t)g.nx * g.ny * g.nz), TPB, 0, s>>>(rc, xc, xf, bc, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_comp_res_fine<T><<<grid_for((int64_t)g.fx * g.fy * g.fz), TPB, 0, s>>>(rf, xf, xc, bf, g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_comp_restrict(T* b0, T* x0, const T* rc, const T* rf, const CompGeom& g,
                                hipStream_t s) {
  k_comp_restrict<T><<<grid_for((int64_t)g.nx * g.ny * g.nz), TPB, 0, s>>>(
      b0, x0, rc, rf, nullptr, nullptr, nullptr, g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_comp_residual_restrict(T* b0, T* x0, T* rf, const T* xc, const T* xf,
                                         const T* bc, const T* bf, const CompGeom& g,
                                         hipStream_t s) {
  k_comp_res_fine<T><<<grid_for((int64_t)g.fx * g.fy * g.fz), TPB, 0, s>>>(rf, xf, xc, bf, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_comp_restrict<T><<<grid_for((int64_t)g.nx * g.ny * g.nz), TPB, 0, s>>>(b0, x0, nullptr, rf,
                                                                            xc, xf, bc, g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_comp_prolong(T* xc, T* xf, const T* y, const CompGeom& g, hipStream_t s) {
  k_comp_prolong_coarse<T><<<grid_for((int64_t)g.nx * g.ny * g.nz), TPB, 0, s>>>(xc, y, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_comp_prolong_fine<T><<<grid_for((int64_t)g.fx * g.fy * g.fz), TPB, 0, s>>>(xf, y, g);
  return hipGetLastError();
}

// Lanes per row of the long-row launches (every block of a long-row level, the listed blocks of
// a level of mostly plain 7-point blocks): two where the launch has enough rows to keep the chip
// busy with short per-lane loops, else eight, trading loop length for waves in flight (measured
// on 81- and 125-entry rows: a colour pass of 131 072 rows 20 us with two lanes against 28 us
// with eight, one of 16 384 rows 6.8 us with eight against 13 us with two).
constexpr int64_t kManyRowsPass = 1 << 16;
constexpr int64_t kManyRowsResidual = 1 << 19;

template <typename T>
bool two_lanes(const GStencilT<T>& st, int64_t rows, int64_t many) {
  return st.row_lanes == 2 || (st.row_lanes == 0 && rows >= many);
}

template <typename T, bool NOISE, int MODE>
void launch_long_pass(T* x, const T* b, const GStencilT<T>& st, int colour, const NoiseArgs& na,
                      int64_t rows, hipStream_t s) {
  if (two_lanes(st, rows, kManyRowsPass))
    k_gblock_pass<T, NOISE, 2, MODE><<<grid_for(rows * 2), TPB, 0, s>>>(x, b, st, colour, na);
  else
    k_gblock_pass<T, NOISE, 8, MODE><<<grid_for(rows * 8), TPB, 0, s>>>(x, b, st, colour, na);
}

template <typename T, int MODE>
void launch_long_residual(T* r, const T* x, const T* b, const GStencilT<T>& st, int64_t rows,
                          hipStream_t s) {
  if (two_lanes(st, rows, kManyRowsResidual))
    k_gresidual<T, 2, MODE><<<grid_for(rows * 2), TPB, 0, s>>>(r, x, b, st);
  else
    k_gresidual<T, 8, MODE><<<grid_for(rows * 8), TPB, 0, s>>>(r, x, b, st);
}

template <typename T>
hipError_t launch_gblock_pass(T* x, const T* b, const GStencilT<T>& st, int colour, bool noise,
                              const NoiseArgs& na, hipStream_t s) {
  const int nbz = st.nz / 2;
  // cells of the colour
  const int64_t rows = (int64_t)(st.nx / 4) * (st.ny / 4) * ((nbz + 1 - (colour >> 2)) / 2) * 8;
  if (rows <= 0) return hipSuccess;
  if (st.split == 8) {
    if (noise) launch_long_pass<T, true, 0>(x, b, st, colour, na, rows, s);
    else launch_long_pass<T, false, 0>(x, b, st, colour, na, rows, s);
    return hipGetLastError();
  }
  const int64_t listed = (int64_t)(st.list_off[colour + 1] - st.list_off[colour]) * 8;
  if (listed == 0) {
    if (noise) k_gblock_pass<T, true, 1, 1><<<grid_for(rows), TPB, 0, s>>>(x, b, st, colour, na);
    else k_gblock_pass<T, false, 1, 1><<<grid_for(rows), TPB, 0, s>>>(x, b, st, colour, na);
    return hipGetLastError();
  }
  // the listed (long-row) blocks and the plain blocks of the colour in one launch
  const bool two = two_lanes(st, listed, kManyRowsPass);
  const uint32_t lw = grid_for(listed * (two ? 2 : 8));
  const uint32_t grid = lw + grid_for(rows);
  if (two) {
    if (noise)
      k_gblock_pass_mixed<T, true, 2><<<grid, TPB, 0, s>>>(x, b, st, colour, na, lw);
    else
      k_gblock_pass_mixed<T, false, 2><<<grid, TPB, 0, s>>>(x, b, st, colour, na, lw);
  } else {
    if (noise)
      k_gblock_pass_mixed<T, true, 8><<<grid, TPB, 0, s>>>(x, b, st, colour, na, lw);
    else
      k_gblock_pass_mixed<T, false, 8><<<grid, TPB, 0, s>>>(x, b, st, colour, na, lw);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gresidual(T* r, const T* x, const T* b, const GStencilT<T>& st, hipStream_t s) {
  const int64_t n = (int64_t)st.nx * st.ny * st.nz;
  if (st.split == 8) {
    launch_long_residual<T, 0>(r, x, b, st, n, s);
    return hipGetLastError();
  }
  const int64_t listed = (int64_t)st.list_off[8] * 8;
  if (listed == 0) {
    k_gresidual<T, 1, 1><<<grid_for(n), TPB, 0, s>>>(r, x, b, st);
    return hipGetLastError();
  }
  if (two_lanes(st, listed, kManyRowsResidual)) {
    const uint32_t lw = grid_for(listed * 2);
    k_gresidual_mixed<T, 2><<<lw + grid_for(n), TPB, 0, s>>>(r, x, b, st, lw);
  } else {
    const uint32_t lw = grid_for(listed * 8);
    k_gresidual_mixed<T, 8><<<lw + grid_for(n), TPB, 0, s>>>(r, x, b, st, lw);
  }
  return hipGetLastError();
}

hipError_t launch_comp_forcing(double* bc, double* bf, const double* qc, const double* qf,
                               const CompGeom& g, const NoiseArgs& nac, const NoiseArgs& naf,
                               hipStream_t s) {
  const int64_t calls = ((int64_t)g.nx * g.ny * g.nz + (int64_t)g.fx * g.fy * g.fz) / 2;
  k_comp_forcing<<<grid_for(calls), TPB, 0, s>>>(bc, bf, qc, qf, g, nac, naf);
  return hipGetLastError();
}

#define SMG_COMP_INSTANTIATE(T)                                                                 \
  template hipError_t launch_dense_draw<T>(T*, const T*, const double*, const double*, double*,   \
                                           int, bool, const NoiseArgs&, hipStream_t);           \
  template hipError_t launch_comp_coarse_pass<T>(T*, const T*, const T*, const CompGeom&, int,  \
                                                 bool, const NoiseArgs&, hipStream_t);          \
  template hipError_t launch_comp_fine_pass<T>(T*, const T*, const CompGeom&, int, bool,        \
                                               const NoiseArgs&, hipStream_t);                  \
  template hipError_t launch_comp_layer_pass<T>(T*, const T*, const T*, const CompGeom&,        \
                                                const int32_t*, int, bool, const NoiseArgs&,    \
                                                hipStream_t);                                   \
  template hipError_t launch_comp_residual<T>(T*, T*, const T*, const T*, const T*, const T*,   \
                                              const CompGeom&, hipStream_t);                    \
  template hipError_t launch_comp_restrict<T>(T*, T*, const T*, const T*, const CompGeom&,      \
                                              hipStream_t);                                     \
  template hipError_t launch_comp_residual_restrict<T>(T*, T*, T*, const T*, const T*,          \
                                                       const T*, const T*, const CompGeom&,     \
                                                       hipStream_t);                            \
  template hipError_t launch_comp_prolong<T>(T*, T*, const T*, const CompGeom&, hipStream_t);   \
  template hipError_t launch_gblock_pass<T>(T*, const T*, const GStencilT<T>&, int, bool,       \
                                            const NoiseArgs&, hipStream_t);                     \
  template hipError_t launch_gresidual<T>(T*, const T*, const T*, const GStencilT<T>&,          \
                                          hipStream_t);

SMG_COMP_INSTANTIATE(double)
SMG_COMP_INSTANTIATE(float)

}  // namespace smg
