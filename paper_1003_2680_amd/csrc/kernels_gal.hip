// Galerkin-level kernels: 2x2x2 block heat bath, residual, restriction, prolongation, the
// coarsest exact draw, and the LDS-resident bottom of the V-cycle.
//
// Sec. "Stochastic Multigrid Methods": the coarse operators are Galerkin, A^(l+1) = P^T A^(l) P,
// which makes them 81-point (level 1) and 125-point (deeper) stencils.  Two cells of one
// red-black colour are coupled there, so each colour class is a set of 2x2x2 blocks
// (colour (bx%2) + 2(by%2) + 4(bz%2)); blocks of one colour are >= 3 cells apart and every
// block is redrawn from its exact 8-variable conditional law.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <type_traits>

#include "device_common.hpp"
#include "kernels.hpp"

namespace smg {
namespace {

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + TPB - 1) / TPB); }

// Block-level noise for whole sweeps, ready for the block passes: one thread per block draws
// the block's eight normals (Philox calls 4 bid .. 4 bid + 3, cells k = 2m, 2m+1 of call m) and
// writes sqrt(kT) L_BB^-T n, L_BB^-T being upper triangular.  When a wave's 64 blocks lie in
// one block row (the level's blocks per layer a multiple of 64) the factor rows are uniform
// and are read with scalar loads as FMA operands.  Grid: x over the blocks of one (sweep slot,
// component) of the largest level, y = level entry, z = slot * nact + component.
template <typename T, bool UNIFORM>
__device__ __forceinline__ void colour_block_noise(const T* __restrict__ W, const T (&n)[8],
                                                   T (&e)[8]) {
  typedef const __attribute__((address_space(4))) T* cptr;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    T acc = 0;
#pragma unroll
    for (int j = k; j < 8; ++j) acc = fma(UNIFORM ? ((cptr)W)[k * 8 + j] : W[k * 8 + j], n[j], acc);
    e[k] = acc;
  }
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_level_noise(NoiseGenArgs a, NoiseArgs na) {
  using V2 = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
  const NoiseLevel& L = a.lv[blockIdx.y];
  const uint32_t N = (uint32_t)L.nx * L.ny * L.nz;
  const uint32_t bid = blockIdx.x * TPB + threadIdx.x;  // block within (slot, comp)
  const uint32_t s = blockIdx.z / (uint32_t)a.nact;
  const uint32_t comp = blockIdx.z - s * (uint32_t)a.nact;
  if (bid >= (N >> 3) || (int)s >= L.nslot) return;
  const uint32_t nbx = (uint32_t)L.nx >> 1, nby = (uint32_t)L.ny >> 1;
  const uint32_t bz = udiv(bid, nbx * nby, L.lg_bxy);
  const uint32_t rem = bid - bz * nbx * nby;
  const uint32_t by = udiv(rem, nbx, L.lg_bx);
  const uint32_t bx = rem - by * nbx;
  const int colour = (bx & 1) + 2 * (by & 1) + 4 * (bz & 1);
  const uint32_t sid = (uint32_t)L.level | ((uint32_t)(L.slot0 + s) << 4) | ((uint32_t)colour << 12);
  T n[8], e[8];
#pragma unroll
  for (int m = 0; m < 4; ++m) normal_pair_t<T>(na, sid, comp, 4 * bid + m, n[2 * m], n[2 * m + 1]);
  if ((nbx * nby) % 64 == 0) {
    const uint32_t bzu = __builtin_amdgcn_readfirstlane(bz);
    colour_block_noise<T, true>((const T*)L.bfac + (size_t)bzu * 192 + 64, n, e);
  } else {
    colour_block_noise<T, false>((const T*)L.bfac + (size_t)bz * 192 + 64, n, e);
  }
  const T sq = (T)na.sqkT;
  T* out = (T*)L.out + ((size_t)s * a.ncomp + comp) * N;
#pragma unroll
  for (int m = 0; m < 4; ++m) {  // cells k = 2m, 2m+1: one row of the block (dy, dz) = (m&1, m>>1)
    const uint32_t c0 = ((2 * bz + (m >> 1)) * L.ny + (2 * by + (m & 1))) * L.nx + 2 * bx;
    V2 v;
    v.x = sq * e[2 * m];
    v.y = sq * e[2 * m + 1];
    *reinterpret_cast<V2*>(out + c0) = v;
  }
}

// One block-colour pass, LDS-staged.  A work-group owns a TI x TJ tile of the colour's blocks in
// one block layer (bz = 2l + colour/4) and stages the box of cells within 2 of them
// ((4TI+2) x (4TJ+2) x 6, periodic in x and y, wall planes clamped: their z-factors are zero)
// with coalesced row loads; the 125-point rows are then gathered from LDS.  The box never
// contains another work-group's blocks of this colour (blocks of one colour are >= 3 cells
// apart), so staging and the writes of other work-groups do not overlap.
// Tile shapes (blocks per work-group along x, y): 4x4 (128 threads), 4x2 (one wavefront) and
// 8x4 (256 threads); the shape changes only the work distribution, never a result.
constexpr int TILE_D = 6;

// The pass of one work-group: wg = (tile, block layer l, component).
template <typename T, bool NOISE, int TILE_I, int TILE_J>
__device__ __forceinline__ void block_tile_body(T* __restrict__ xg, const T* __restrict__ bg,
                                                const T* __restrict__ s1d,
                                                const T* __restrict__ zt,
                                                const T* __restrict__ bfac, int nx, int ny,
                                                int nz, uint32_t N, int colour, int nbx2,
                                                int nby2, int ntx, const T* __restrict__ zn,
                                                const Blk3 wg) {
  constexpr int TILE_W = 4 * TILE_I + 2, TILE_H = 4 * TILE_J + 2;
  constexpr int TILE_TPB = TILE_I * TILE_J * 8;
  // plane stride: the first count >= the plane that is 16 mod 32 elements.  The two z-layers
  // of a block read planes three apart, so their lanes then fall on opposite halves of the
  // 64 LDS banks and a wave's reads of one window offset are free of bank conflicts (FP64).
  constexpr int TP = TILE_H * TILE_W + ((48 - (TILE_H * TILE_W) % 32) % 32);
  __shared__ T Tl[TILE_D * TP];
  const uint32_t comp = wg.z;
  const int l = wg.y;
  const int ti = wg.x % ntx, tj = wg.x / ntx;
  const int cx = colour & 1, cy = (colour >> 1) & 1;
  const int bz = 2 * l + (colour >> 2);
  const int i0 = ti * TILE_I, j0 = tj * TILE_J;
  const int x0 = 4 * i0 + 2 * cx - 2, y0 = 4 * j0 + 2 * cy - 2, z0 = 2 * bz - 2;
  T* X = xg + (size_t)comp * N;
  const int tid = threadIdx.x;
  // this lane's cell: its b and noise loads go out before the tile is staged
  const int k = tid & 7;
  const int il = (tid >> 3) % TILE_I, jl = (tid >> 3) / TILE_I;
  const int i = i0 + il, j = j0 + jl;
  const bool active = i < nbx2 && j < nby2;
  const int bx = 2 * i + cx, by = 2 * j + cy;
  const int kx = k & 1, ky = (k >> 1) & 1, kz = k >> 2;
  const int tx = 4 * il + 2 + kx, ty = 4 * jl + 2 + ky, tz = 2 + kz;
  const int gcx = 2 * bx + kx, gcy = 2 * by + ky, gcz = 2 * bz + kz;
  const uint32_t cell = ((uint32_t)gcz * ny + gcy) * nx + gcx;
  T ax = 0, xk = 0, bk = 0, nrm = 0;
  if (active) {
    bk = bg[(size_t)comp * N + cell];
    if (NOISE) nrm = zn[(size_t)comp * N + cell];
  }
  // stage the box: each thread owns up to PPT (x, y) positions of a plane and loads them in all
  // TILE_D planes; every load is issued before the first LDS store, so the work-group waits for
  // global memory once, and the index arithmetic is done once per position, not per element
  constexpr int PLANE = TILE_W * TILE_H;
  constexpr int PPT = (PLANE + TILE_TPB - 1) / TILE_TPB;
  int goff[PPT], loff[PPT];
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    const int pos = tid + p * TILE_TPB;
    const int sx = pos % TILE_W, sy = pos / TILE_W;
    // positions past the plane store into its pad element (TP = PLANE + 1): no branch
    loff[p] = pos < PLANE ? pos : PLANE;
    goff[p] = pos < PLANE ? wrap_near(y0 + sy, ny) * nx + wrap_near(x0 + sx, nx) : 0;
  }
  T stage[TILE_D][PPT];
#pragma unroll
  for (int sz = 0; sz < TILE_D; ++sz) {
    int gz = z0 + sz;
    gz = gz < 0 ? 0 : (gz >= nz ? nz - 1 : gz);
    const T* P = X + (size_t)gz * nx * ny;
#pragma unroll
    for (int p = 0; p < PPT; ++p) stage[sz][p] = P[goff[p]];  // goff = 0 (in range) if unused
  }
#pragma unroll
  for (int sz = 0; sz < TILE_D; ++sz)
#pragma unroll
    for (int p = 0; p < PPT; ++p) Tl[sz * TP + loff[p]] = stage[sz][p];
  __syncthreads();
  {
    // The two z-layers of a block reach the same six staged planes (tile planes 0..5).  Lane
    // kz computes the in-plane sums of planes 3kz .. 3kz+2 and trades them with its partner
    // (lane ^ 4, same x and y), so each plane is reduced once per (x, y) pair, not twice.
    // and each plane's rows are shared with the y-partner (lane ^ 2) the same way
    const int xs[5] = {tx - 2, tx - 1, tx, tx + 1, tx + 2};
    const int rows[3] = {ky ? ty + 2 : ty - 2, ty + (ky ? 1 : -1), ty};
    T q0[3], q1[3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
      gal_plane_pair<T>(Tl + (3 * kz + j) * TP, TILE_W, xs, rows, s1d, q0[j], q1[j]);
    T o0[3], o1[3], w0[5], w1[5];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      o0[j] = __shfl_xor(q0[j], 4, 8);
      o1[j] = __shfl_xor(q1[j], 4, 8);
    }
    plane_window(kz, q0, o0, w0);
    plane_window(kz, q1, o1, w1);
    if (active) {
      // cell tz = 2 + kz sees planes kz .. kz + 4 as dz = 0 .. 4
      const T* zr = zt + gcz * 10;
      T ax0 = 0, ax1 = 0;
#pragma unroll
      for (int dz = 0; dz < 5; ++dz) {
        ax0 = fma(zr[dz], w0[dz], ax0);
        ax1 = fma(zr[5 + dz], w1[dz], ax1);
      }
      ax = ax0 + ax1;
      xk = Tl[tz * TP + ty * TILE_W + tx];
    }
  }
  // x_B + A_BB^-1 (b_B - (A x)_B) equals A_BB^-1 (b_B - A_B,rest x_rest): the block's own
  // coupling cancels, so only the residual needs to be shared across the block's lanes
  const T* F = bfac + (size_t)bz * 192;
  const T res = bk - ax;
  // the noise field already holds sqrt(kT) L_BB^-T n for the block
  T v0 = xk, v1 = NOISE ? nrm : T(0);
#pragma unroll
  for (int jj = 0; jj < 8; jj += 2) {
    v0 = fma(F[k * 8 + jj], __shfl(res, jj, 8), v0);
    v1 = fma(F[k * 8 + jj + 1], __shfl(res, jj + 1, 8), v1);
  }
  const T v = v0 + v1;
  if (active) X[cell] = v;
}

template <typename T, bool NOISE, int TILE_I, int TILE_J>
__global__ __launch_bounds__(TILE_I * TILE_J * 8) void k_block_tile(T* __restrict__ xg,
                                                          const T* __restrict__ bg,
                                                          const T* __restrict__ s1d,
                                                          const T* __restrict__ zt,
                                                          const T* __restrict__ bfac, int nx,
                                                          int ny, int nz, uint32_t N, int colour,
                                                          int nbx2, int nby2, int ntx,
                                                          const T* __restrict__ zn) {
  block_tile_body<T, NOISE, TILE_I, TILE_J>(xg, bg, s1d, zt, bfac, nx, ny, nz, N, colour, nbx2,
                                            nby2, ntx, zn, xcd_block());
}

// Two block colours c and c ^ 1 in one launch.  They differ only in the parity of bx, so a
// block of colour c ^ 1 depends on colour-c blocks only through its x-neighbours in the same
// block row and layer.  A work-group owns PJ (4, 2 or 1: see pair_rows) block rows
// by = 2 (j0 + jl) + cy of one block layer bz = 2 l + cz over the whole x-extent (periodic, so
// no x-halo), stages the cells within two
// of them (nx x (4 PJ + 2) x 6, wall planes clamped), draws colour c into the tile, then colour
// c ^ 1 from the updated tile, and writes both.  No other work-group stages a cell that this
// one writes (rows of parity cy are four cells apart, and rows and layers of the other parity
// are not written), and every value is computed by the arithmetic of the single-colour pass
// from the same inputs, so the result is that of the two single-colour passes in order.
// The work of one work-group wg = (row group, layer, component); threads past the level's
// (nx / 4) PJ 8 take part in the staging only.
template <typename T, bool NOISE, int PJ>
__device__ __forceinline__ void block_pair_body(T* __restrict__ xg, const T* __restrict__ bg,
                                                const T* __restrict__ s1d,
                                                const T* __restrict__ zt,
                                                const T* __restrict__ bfac, int nx, int ny,
                                                int nz, uint32_t N, int c_first, int nby2,
                                                int TP, const T* __restrict__ zn,
                                                const Blk3 wg) {
  extern __shared__ char smraw[];
  T* Tl = reinterpret_cast<T*>(smraw);
  const uint32_t comp = wg.z;
  const int cy = (c_first >> 1) & 1, cz = c_first >> 2;
  const int bz = 2 * (int)wg.y + cz;
  const int j0 = (int)wg.x * PJ;
  const int H = 4 * PJ + 2;  // staged rows
  const int RS = nx;         // row stride of the tile (padding it measured slower)
  const int y0 = 4 * j0 + 2 * cy - 2, z0 = 2 * bz - 2;
  const int nthr = (int)blockDim.x;  // >= (nx / 4) PJ 8
  T* X = xg + (size_t)comp * N;
  const int tid = threadIdx.x;
  const int k = tid & 7;
  const int nbx2 = nx >> 2;
  int il, jl;
  divmod_uniform(tid >> 3, nbx2, jl, il);
  const bool active = jl < PJ && j0 + jl < nby2;
  // rows of inactive lanes past the group's PJ rows are taken as row 0 for addressing only,
  // so that every tile read stays inside the staged rows
  const int jr = jl < PJ ? jl : 0;
  const int kx = k & 1, ky = (k >> 1) & 1, kz = k >> 2;
  const int by = 2 * (j0 + jr) + cy;
  const int ty = 4 * jr + 2 + ky, tz = 2 + kz;
  const int gcy = 2 * by + ky, gcz = 2 * bz + kz;
  // the lane's cell in each phase: bx = 2 il + (colour & 1)
  const int cx0 = c_first & 1, cx1 = cx0 ^ 1;
  const int gx0 = 2 * (2 * il + cx0) + kx, gx1 = 2 * (2 * il + cx1) + kx;
  const uint32_t row = ((uint32_t)gcz * ny + gcy) * nx;
  T bk0 = 0, bk1 = 0, n0 = 0, n1 = 0;
  if (active) {
    bk0 = bg[(size_t)comp * N + row + gx0];
    bk1 = bg[(size_t)comp * N + row + gx1];
    if (NOISE) {
      n0 = zn[(size_t)comp * N + row + gx0];
      n1 = zn[(size_t)comp * N + row + gx1];
    }
  }
  // stage: a plane has nx (4 PJ + 2) positions and the group (nx / 4) PJ 8 threads, so every
  // thread owns at most three positions (2 + 1/PJ per thread); all their loads in all six
  // planes are issued before the first store, so the group waits for memory once
  constexpr int PPT = 3;
  const int plane = nx * H;
  int goff[PPT], loff[PPT];
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    const int pos = tid + p * nthr;
    const bool in = pos < plane;
    int py, px;
    divmod_uniform(pos, nx, py, px);
    loff[p] = in ? py * RS + px : -1;
    goff[p] = in ? wrap_near(y0 + py, ny) * nx + px : 0;
  }
  T stage[TILE_D][PPT];
#pragma unroll
  for (int sz = 0; sz < TILE_D; ++sz) {
    int gz = z0 + sz;
    gz = gz < 0 ? 0 : (gz >= nz ? nz - 1 : gz);
    const T* P = X + (size_t)gz * ny * nx;
#pragma unroll
    for (int p = 0; p < PPT; ++p) stage[sz][p] = P[goff[p]];  // goff = 0 (in range) if unused
  }
#pragma unroll
  for (int sz = 0; sz < TILE_D; ++sz)
#pragma unroll
    for (int p = 0; p < PPT; ++p)
      if (loff[p] >= 0) Tl[sz * TP + loff[p]] = stage[sz][p];
  __syncthreads();
  const T* F = bfac + (size_t)bz * 192;
  const T* zr = zt + gcz * 10;
  // one phase: the lane's block of colour bit cxp (tile x = global x, periodic)
  auto lane_update = [&](int gx, T bk, T nrm) -> T {
    int xs[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) xs[d] = wrapm(gx + d - 2, nx);
    const int rows[3] = {ky ? ty + 2 : ty - 2, ty + (ky ? 1 : -1), ty};
    T q0[3], q1[3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
      gal_plane_pair<T>(Tl + (3 * kz + j) * TP, RS, xs, rows, s1d, q0[j], q1[j]);
    T o0[3], o1[3], w0[5], w1[5];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      o0[j] = __shfl_xor(q0[j], 4, 8);
      o1[j] = __shfl_xor(q1[j], 4, 8);
    }
    plane_window(kz, q0, o0, w0);
    plane_window(kz, q1, o1, w1);
    T ax = 0, xk = 0;
    if (active) {
      T ax0 = 0, ax1 = 0;
#pragma unroll
      for (int dz = 0; dz < 5; ++dz) {
        ax0 = fma(zr[dz], w0[dz], ax0);
        ax1 = fma(zr[5 + dz], w1[dz], ax1);
      }
      ax = ax0 + ax1;
      xk = Tl[tz * TP + ty * RS + gx];
    }
    const T res = bk - ax;
    T v0 = xk, v1 = NOISE ? nrm : T(0);
#pragma unroll
    for (int jj = 0; jj < 8; jj += 2) {
      v0 = fma(F[k * 8 + jj], __shfl(res, jj, 8), v0);
      v1 = fma(F[k * 8 + jj + 1], __shfl(res, jj + 1, 8), v1);
    }
    return v0 + v1;
  };
  // colour c is written into the tile in place: blocks of one colour never read each other's
  // cells, and the eight lanes of a block are one wave, whose reads precede its writes
  const T va = lane_update(gx0, bk0, n0);
  if (active) {
    Tl[tz * TP + ty * RS + gx0] = va;
    X[row + gx0] = va;
  }
  __syncthreads();
  const T vb = lane_update(gx1, bk1, n1);
  if (active) X[row + gx1] = vb;
}

template <typename T, bool NOISE, int PJ>
__global__ __launch_bounds__(512) void k_block_pair(T* __restrict__ xg, const T* __restrict__ bg,
                                                    const T* __restrict__ s1d,
                                                    const T* __restrict__ zt,
                                                    const T* __restrict__ bfac, int nx, int ny,
                                                    int nz, uint32_t N, int c_first, int nby2,
                                                    int TP, const T* __restrict__ zn) {
  block_pair_body<T, NOISE, PJ>(xg, bg, s1d, zt, bfac, nx, ny, nz, N, c_first, nby2, TP, zn,
                                xcd_block());
}

// Two-colour launches of several levels of different hierarchies (the same colour pair and
// rows per group) in one launch: the flat grid concatenates the items' (row group, layer,
// component) grids; the block size and the LDS are the largest the items need.
template <typename T, bool NOISE, int PJ>
__global__ __launch_bounds__(512) void k_block_pair_multi(PairMultiArgs<T> m) {
  const uint32_t lin = xcd_block().x;
  int i = 0;
  while (i + 1 < m.nitems && lin >= m.begin[i + 1]) ++i;
  const PairMultiItem<T>& it = m.it[i];
  const uint32_t local = lin - m.begin[i];
  Blk3 wg;
  wg.x = local % (uint32_t)it.ngx;
  const uint32_t rest = local / (uint32_t)it.ngx;
  wg.y = rest % (uint32_t)it.nbzc;
  wg.z = rest / (uint32_t)it.nbzc;
  block_pair_body<T, NOISE, PJ>(it.x, it.b, it.s1d, it.zt, it.bfac, it.nx, it.ny, it.nz, it.N,
                                m.c_first, it.nby2, it.TP, it.zn, wg);
}

// The same pass for several levels of different hierarchies (one colour) in one launch: the
// one-dimensional grid is the concatenation of every item's (tile, layer, component) grid, in
// XCD-aware order; a work-group finds its item from the offsets and runs the item's pass.
template <typename T, bool NOISE, int TILE_I, int TILE_J>
__global__ __launch_bounds__(TILE_I * TILE_J * 8) void k_block_tile_multi(BlockMultiArgs<T> m) {
  const uint32_t lin = xcd_block().x;
  int i = 0;
  while (i + 1 < m.nitems && lin >= m.begin[i + 1]) ++i;
  const BlockMultiItem<T>& it = m.it[i];
  const uint32_t local = lin - m.begin[i];
  const uint32_t tiles = (uint32_t)it.ntx * (uint32_t)it.nty;
  Blk3 wg;
  wg.x = local % tiles;
  const uint32_t rest = local / tiles;
  wg.y = rest % (uint32_t)it.nbzc;
  wg.z = rest / (uint32_t)it.nbzc;
  block_tile_body<T, NOISE, TILE_I, TILE_J>(it.x, it.b, it.s1d, it.zt, it.bfac, it.nx, it.ny,
                                            it.nz, it.N, m.colour, it.nbx2, it.nby2, it.ntx,
                                            it.zn, wg);
}

// r = b - A x on a Galerkin level, LDS-tiled: a work-group owns GR_X x GR_Y x GR_Z cells and
// stages the box within 2 of them; a thread takes a z-column of GR_Z cells and forms each of
// the GR_Z + 4 staged planes' two partial sums once, adding them into every cell of the
// column they reach (the per-cell order of the additions is that of gal_apply).
constexpr int GR_X = 16, GR_Y = 16, GR_Z = 4;
constexpr int GR_SX = GR_X + 4, GR_SY = GR_Y + 4, GR_SZ = GR_Z + 4;

template <typename T>
__global__ __launch_bounds__(TPB) void k_residual_gal_tile(T* __restrict__ r,
                                                            const T* __restrict__ xg,
                                                            const T* __restrict__ bg,
                                                            const T* __restrict__ s1d,
                                                            const T* __restrict__ zt, int nx,
                                                            int ny, int nz, int ntx) {
  __shared__ T Xs[GR_SZ * GR_SY * GR_SX];
  const Blk3 wg = xcd_block();
  const uint32_t comp = wg.z;
  const int X0 = (wg.x % ntx) * GR_X, Y0 = (wg.x / ntx) * GR_Y, Z0 = wg.y * GR_Z;
  const size_t N = (size_t)nx * ny * nz;
  const T* X = xg + comp * N;
  const int tid = threadIdx.x;
  {
    constexpr int PLANE = GR_SX * GR_SY;
    constexpr int PPT = (PLANE + TPB - 1) / TPB;
    int goff[PPT], loff[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      const int pos = tid + p * TPB;
      const int sx = pos % GR_SX, sy = pos / GR_SX;
      loff[p] = pos < PLANE ? sy * GR_SX + sx : -1;
      goff[p] = pos < PLANE ? wrap_near(Y0 - 2 + sy, ny) * nx + wrap_near(X0 - 2 + sx, nx) : 0;
    }
    T st[GR_SZ][PPT];
#pragma unroll
    for (int sz = 0; sz < GR_SZ; ++sz) {
      int gz = Z0 - 2 + sz;
      gz = gz < 0 ? 0 : (gz >= nz ? nz - 1 : gz);
#pragma unroll
      for (int p = 0; p < PPT; ++p) st[sz][p] = X[(size_t)gz * nx * ny + goff[p]];
    }
#pragma unroll
    for (int sz = 0; sz < GR_SZ; ++sz)
#pragma unroll
      for (int p = 0; p < PPT; ++p)
        if (loff[p] >= 0) Xs[sz * PLANE + loff[p]] = st[sz][p];
  }
  __syncthreads();
  const int lx = tid % GR_X, ly = tid / GR_X;
  const int cx = X0 + lx, cy = Y0 + ly;
  const int xs[5] = {lx, lx + 1, lx + 2, lx + 3, lx + 4};
  const int ys[5] = {ly, ly + 1, ly + 2, ly + 3, ly + 4};
  const int kmax = nz - Z0 < GR_Z ? nz - Z0 : GR_Z;
  T acc0[GR_Z], acc1[GR_Z];
#pragma unroll
  for (int k = 0; k < GR_Z; ++k) acc0[k] = acc1[k] = T(0);
#pragma unroll
  for (int p = 0; p < GR_SZ; ++p) {
    T p1;
    const T p0 = gal_plane<T>(Xs + p * (GR_SX * GR_SY), GR_SX, xs, ys, s1d, p1);
#pragma unroll
    for (int k = 0; k < GR_Z; ++k) {
      const int dz = p - k;  // plane offset + 2 seen from cell Z0 + k
      if (dz < 0 || dz > 4 || k >= kmax) continue;
      const T* zr = zt + (Z0 + k) * 10;
      acc0[k] = fma(zr[dz], p0, acc0[k]);
      acc1[k] = fma(zr[5 + dz], p1, acc1[k]);
    }
  }
  if (cx >= nx || cy >= ny) return;
#pragma unroll
  for (int k = 0; k < GR_Z; ++k) {
    if (k >= kmax) break;
    const size_t i = comp * N + ((size_t)(Z0 + k) * ny + cy) * nx + cx;
    r[i] = bg[i] - (acc0[k] + acc1[k]);
  }
}

// b_c = P^T r, and x_c = 0 (the coarse iterate of Alg. 3 starts from zero)
template <typename T>
__global__ __launch_bounds__(TPB) void k_restrict(T* __restrict__ bc, T* __restrict__ xc,
                                                   const T* __restrict__ r, int nxf, int nyf,
                                                   int nzf, uint32_t Nf, uint32_t Nc) {
  const uint32_t comp = blockIdx.y;
  const uint32_t I = blockIdx.x * TPB + threadIdx.x;
  if (I >= Nc) return;
  const int nxc = nxf >> 1, nyc = nyf >> 1;
  const int X = I % nxc;
  const uint32_t row = I / nxc;
  const int Y = row % nyc;
  const int Z = row / nyc;
  bc[(size_t)comp * Nc + I] =
      restrict_at<T>(r + (size_t)comp * Nf, nxf, nxf * nyf, nxf, nyf, nzf, X, Y, Z);
  if (xc) xc[(size_t)comp * Nc + I] = T(0);
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_prolong(T* __restrict__ x, const T* __restrict__ e,
                                                  int nxf, int nyf, int nzf, uint32_t Nf,
                                                  uint32_t Nc) {
  const uint32_t comp = blockIdx.y;
  const uint32_t i = blockIdx.x * TPB + threadIdx.x;
  if (i >= Nf) return;
  const int xf = i % nxf;
  const uint32_t row = i / nxf;
  const int yf = row % nyf;
  const int zf = row / nyf;
  const int nxc = nxf >> 1, nyc = nyf >> 1;
  x[(size_t)comp * Nf + i] +=
      prolong_at<T>(e + (size_t)comp * Nc, nxc, nxc * nyc, xf, yf, zf, nxc, nyc, nzf >> 1);
}

// x = A_c^-1 b (+ sqrt(kT) L_c^-T n) in FP64: rows split over work-groups; each work-group
// stages b and the whole noise vector in LDS.
template <typename T, bool NOISE>
__global__ __launch_bounds__(TPB) void k_coarsest(T* __restrict__ xg, const T* __restrict__ bg,
                                                   const double* __restrict__ ainv,
                                                   const double* __restrict__ w, int n,
                                                   NoiseArgs na) {
  extern __shared__ double sh[];
  const uint32_t comp = blockIdx.y;
  const T* B = bg + (size_t)comp * n;
  for (int i = threadIdx.x; i < n; i += TPB) sh[i] = (double)B[i];
  if (NOISE) {
    for (int q = threadIdx.x; 2 * q < n; q += TPB) {
      double z0, z1;
      normal_pair(na, na.sid, comp, (uint32_t)q, z0, z1);
      sh[n + 2 * q] = z0;
      if (2 * q + 1 < n) sh[n + 2 * q + 1] = z1;
    }
  }
  __syncthreads();
  const int row = blockIdx.x * TPB + threadIdx.x;
  if (row >= n) return;
  double acc = 0.0;
  for (int jj = 0; jj < n; ++jj) acc = fma(ainv[(size_t)jj * n + row], sh[jj], acc);
  if (NOISE) {
    double an = 0.0;
    for (int jj = row; jj < n; ++jj) an = fma(w[(size_t)jj * n + row], sh[n + jj], an);
    acc = fma(na.sqkT, an, acc);
  }
  xg[(size_t)comp * n + row] = (T)acc;
}

// ----------------------------------------------------------------------------- bottom of the V
// One work-group per component runs every level from the bottom level down to the coarsest
// and back up, with x, b and a scratch field of each level in LDS; only b of the bottom level
// comes from global memory and only its x goes back.  Colour passes are separated by
// work-group barriers instead of kernel launches.  The coarsest draw is FP64 in every mode.
constexpr int BOT_TPB = 512;

template <typename T, bool NOISE>
__device__ __forceinline__ void bot_block_pass(T* X, const T* Bv, const BotLevel& L, const T* tab,
                                               int colour, const T* Z) {
  // the 1D stencils are the same for every lane: scalar loads from the level descriptor
  T s1d[20];
#pragma unroll
  for (int q = 0; q < 20; ++q) s1d[q] = (T)L.s1d[q];
  const T* zt = tab;
  const T* bfac = tab + L.nz * 10;
  const int nbx2 = L.nx / 4, nby2 = L.ny / 4;
  const int nbzc = (L.nz / 2 + 1 - (colour >> 2)) / 2;
  const int total = nbx2 * nby2 * nbzc * 8;
#pragma unroll 1
  for (int base = 0; base < total; base += BOT_TPB) {
    const int t = base + (int)threadIdx.x;
    const bool active = t < total;
    const int k = t & 7;
    const int blk = active ? (t >> 3) : 0;
    const int i = blk % nbx2;
    const int rest = blk / nbx2;
    const int j = rest % nby2;
    const int l = rest / nby2;
    uint32_t cell;
    const T v = block_lane<T, NOISE>(X, L.sy, L.sz, Bv, s1d, zt, bfac, L.nx, L.ny, L.nz,
                                     2 * i + (colour & 1), 2 * j + ((colour >> 1) & 1),
                                     2 * l + (colour >> 2), k, active, Z, cell);
    if (active) X[cell] = v;
  }
  __syncthreads();
}

template <typename T, bool NOISE>
__device__ __forceinline__ void bot_sweep(T* X, const T* Bv, const BotLevel& L, const T* tab,
                                          int slot, bool post, int ncomp, uint32_t comp) {
  const int n = L.nx * L.ny * L.nz;
  const T* Z = NOISE ? (const T*)L.noise + ((size_t)slot * ncomp + comp) * n : nullptr;
#pragma unroll 1
  for (int t = 0; t < 8; ++t) {
    const int colour = post ? 7 - t : t;
    bot_block_pass<T, NOISE>(X, Bv, L, tab, colour, Z);
  }
}

__device__ __forceinline__ int bot_pos(const BotLevel& L, int q) {
  const int x = q % L.nx, r = q / L.nx;
  const int y = r % L.ny, z = r / L.ny;
  return z * L.sz + y * L.sy + x;
}

template <typename T, bool NOISE>
__device__ __forceinline__ void bottom_body(const BotArgs& a, const uint32_t comp,
                                            const NoiseArgs& na) {
  extern __shared__ char smraw[];
  T* sm = reinterpret_cast<T*>(smraw);
  const int tid = threadIdx.x;
  const BotLevel& L0 = a.lv[0];
  const int n0 = L0.nx * L0.ny * L0.nz;
  const int f0 = L0.nz * L0.sz;
  for (int q = tid; q < f0; q += BOT_TPB) sm[a.lds_off[0] + q] = T(0);
  __syncthreads();
  for (int q = tid; q < n0; q += BOT_TPB)
    sm[a.lds_off[0] + f0 + bot_pos(L0, q)] = ((const T*)a.b_in)[(size_t)comp * n0 + q];
  // operator tables of the block levels: [zt nz*10][bfac nz/2*192] at tab_off[i]
  for (int i = 0; i < a.nlev; ++i) {
    if (a.lv[i].kind != KIND_BLOCK) continue;
    const int nz = a.lv[i].nz;
    T* t = sm + a.tab_off[i];
    const T* zt = (const T*)a.lv[i].zt;
    const T* bf = (const T*)a.lv[i].bfac;
    for (int q = tid; q < nz * 10; q += BOT_TPB) t[q] = zt[q];
    for (int q = tid; q < (nz / 2) * 192; q += BOT_TPB) t[nz * 10 + q] = bf[q];
  }
  __syncthreads();
  int last = a.nlev - 1;
  for (int i = 0; i < a.nlev; ++i) {
    const BotLevel& L = a.lv[i];
    const int level = a.level0 + i;
    const int n = L.nx * L.ny * L.nz;
    const int f = L.nz * L.sz;
    T* xi = sm + a.lds_off[i];
    T* bi = xi + f;
    T* ri = bi + f;
    if (L.kind == KIND_CHOL) {
      // exact draw x = A_c^-1 b + sqrt(kT) L_c^-T n (natural layout on this level)
      if (NOISE) {
        const uint32_t sid = (uint32_t)level | (1u << 24);
        for (int q = tid; 2 * q < n; q += BOT_TPB) {
          double z0, z1;
          normal_pair(na, sid, comp, (uint32_t)q, z0, z1);
          ri[2 * q] = (T)z0;
          if (2 * q + 1 < n) ri[2 * q + 1] = (T)z1;
        }
        __syncthreads();
      }
      // G lanes per row (a power of two, G <= 32) split the columns, so that every lane has
      // only n/G loads of the dense factors in its chain; their sums meet by shuffles
      int G = 1;
      while (G < 32 && 2 * G * n <= BOT_TPB) G *= 2;
      const int part = tid % G;
      for (int row = tid / G; row < n; row += BOT_TPB / G) {
        double acc = 0.0, an = 0.0;
        for (int jj = part; jj < n; jj += G) {
          acc = fma(a.ainv[(size_t)jj * n + row], (double)bi[jj], acc);
          if (NOISE && jj >= row) an = fma(a.w[(size_t)jj * n + row], (double)ri[jj], an);
        }
        for (int off = G / 2; off >= 1; off >>= 1) {
          acc += __shfl_xor(acc, off, G);
          if (NOISE) an += __shfl_xor(an, off, G);
        }
        if (NOISE) acc = fma(na.sqkT, an, acc);
        if (part == 0) xi[row] = (T)acc;
      }
      __syncthreads();
      last = i;
      break;
    }
    const T* tab = sm + a.tab_off[i];
    for (int s = 0; s < a.nu1; ++s)
      bot_sweep<T, NOISE>(xi, bi, L, tab, s, false, a.ncomp, comp);
    if (i == a.nlev - 1) {
      // smoothing-only coarsest level: the post-sweeps follow at once
      for (int s = 0; s < a.nu2; ++s)
        bot_sweep<T, NOISE>(xi, bi, L, tab, a.nu1 + s, true, a.ncomp, comp);
      last = i;
      break;
    }
    // b_{i+1} = P^T (b_i - A_i x_i), x_{i+1} = 0
    {
      T s1d[20];
#pragma unroll
      for (int q = 0; q < 20; ++q) s1d[q] = (T)L.s1d[q];
      for (int q = tid; q < n; q += BOT_TPB) {
        const int x = q % L.nx, y = (q / L.nx) % L.ny, z = q / (L.nx * L.ny);
        const int p = z * L.sz + y * L.sy + x;
        ri[p] = bi[p] - gal_apply<T>(xi, L.sy, L.sz, s1d, tab, L.nx, L.ny, L.nz, x, y, z);
      }
    }
    __syncthreads();
    const BotLevel& C = a.lv[i + 1];
    const int nc = C.nx * C.ny * C.nz;
    const int fc = C.nz * C.sz;
    T* xc = sm + a.lds_off[i + 1];
    for (int q = tid; q < fc; q += BOT_TPB) xc[q] = T(0);
    for (int q = tid; q < nc; q += BOT_TPB) {
      const int X = q % C.nx, Y = (q / C.nx) % C.ny, Z = q / (C.nx * C.ny);
      xc[fc + Z * C.sz + Y * C.sy + X] = restrict_at<T>(ri, L.sy, L.sz, L.nx, L.ny, L.nz, X, Y, Z);
    }
    __syncthreads();
  }
  for (int i = last - 1; i >= 0; --i) {
    const BotLevel& L = a.lv[i];
    const BotLevel& C = a.lv[i + 1];
    const int n = L.nx * L.ny * L.nz;
    T* xi = sm + a.lds_off[i];
    const T* xc = sm + a.lds_off[i + 1];
    for (int q = tid; q < n; q += BOT_TPB) {
      const int x = q % L.nx, y = (q / L.nx) % L.ny, z = q / (L.nx * L.ny);
      xi[z * L.sz + y * L.sy + x] += prolong_at<T>(xc, C.sy, C.sz, x, y, z, C.nx, C.ny, C.nz);
    }
    __syncthreads();
    for (int s = 0; s < a.nu2; ++s)
      bot_sweep<T, NOISE>(xi, xi + L.nz * L.sz, L, sm + a.tab_off[i], a.nu1 + s, true, a.ncomp,
                          comp);
  }
  for (int q = tid; q < n0; q += BOT_TPB)
    ((T*)a.x_out)[(size_t)comp * n0 + q] = sm[a.lds_off[0] + bot_pos(L0, q)];
}

// One hierarchy, one work-group per component.
template <typename T, bool NOISE>
__global__ __launch_bounds__(BOT_TPB) void k_bottom(const BotArgs* __restrict__ ap, int c0,
                                                    NoiseArgs na) {
  bottom_body<T, NOISE>(*ap, c0 + (int)blockIdx.x, na);
}

// Several hierarchies (of any sizes) in one launch: work-group w runs component wg >> 16 of
// item wg & 0xffff, with that item's level descriptors and noise keys, so the latency-bound
// bottoms of uneven instances overlap instead of running one launch after another.
template <typename T, bool NOISE>
__global__ __launch_bounds__(BOT_TPB) void k_bottom_multi(BotMultiArgs m) {
  const uint32_t w = m.wg[blockIdx.x];
  const BotMultiItem& it = m.it[w & 0xffffu];
  NoiseArgs na;
  na.k0 = it.k0;
  na.k1 = it.k1;
  na.sid = 0;
  na.c2 = it.c2;
  na.c3 = it.c3;
  na.sqkT = it.sqkT;
  na.chains = it.chains;
  na.comps_per_chain = it.cpc;
  na.cpc_magic = it.cpc_magic;
  na.bm = m.bm;
  bottom_body<T, NOISE>(*it.args, w >> 16, na);
}

}  // namespace

template <typename T, int TI, int TJ>
void launch_block_tile(T* x, const T* b, const T* s1d, const T* zt, const T* bfac, int nx, int ny,
                       int nz, int ncomp, int colour, const T* zn, int nbx2,
                       int nby2, int nbzc, hipStream_t s) {
  const uint32_t N = (uint32_t)nx * ny * nz;
  const int ntx = (nbx2 + TI - 1) / TI, nty = (nby2 + TJ - 1) / TJ;
  dim3 grid(ntx * nty, nbzc, ncomp);
  if (zn)
    k_block_tile<T, true, TI, TJ><<<grid, TI * TJ * 8, 0, s>>>(
        x, b, s1d, zt, bfac, nx, ny, nz, N, colour, nbx2, nby2, ntx, zn);
  else
    k_block_tile<T, false, TI, TJ><<<grid, TI * TJ * 8, 0, s>>>(
        x, b, s1d, zt, bfac, nx, ny, nz, N, colour, nbx2, nby2, ntx, zn);
}

template <typename T>
hipError_t launch_block_pass(T* x, const T* b, const T* s1d, const T* zt, const T* bfac, int nx,
                             int ny, int nz, int ncomp, int colour, const T* zn,
                             int tile, hipStream_t s) {
  const int nbx2 = nx / 4, nby2 = ny / 4;
  const int nbz = nz / 2;
  const int nbzc = (nbz + 1 - (colour >> 2)) / 2;
  if (nbx2 * nby2 * nbzc == 0) return hipSuccess;
  if (tile == SMG_TILE_AUTO) {
    // the largest tile (least halo per block) that still gives every compute unit two
    // work-groups
    const int64_t layers = (int64_t)nbzc * ncomp;
    const int64_t wg84 = (int64_t)((nbx2 + 7) / 8) * ((nby2 + 3) / 4) * layers;
    const int64_t wg44 = (int64_t)((nbx2 + 3) / 4) * ((nby2 + 3) / 4) * layers;
    tile = wg84 >= 512 ? SMG_TILE_8X4 : (wg44 >= 512 ? SMG_TILE_4X4 : SMG_TILE_4X2);
  }
  if (tile == SMG_TILE_4X2)
    launch_block_tile<T, 4, 2>(x, b, s1d, zt, bfac, nx, ny, nz, ncomp, colour, zn, nbx2, nby2, nbzc, s);
  else if (tile == SMG_TILE_8X4)
    launch_block_tile<T, 8, 4>(x, b, s1d, zt, bfac, nx, ny, nz, ncomp, colour, zn, nbx2, nby2, nbzc, s);
  else
    launch_block_tile<T, 4, 4>(x, b, s1d, zt, bfac, nx, ny, nz, ncomp, colour, zn, nbx2, nby2, nbzc, s);
  return hipGetLastError();
}

// Block rows per work-group of a two-colour launch: the most (4, or 2 above 64 cells in x, for
// the least staging overlap) that still gives the launch about eight work-groups per compute
// unit, else one.
inline int pair_rows(int nx, int ny, int nz, int ncomp, int c_first) {
  const int nby2 = ny / 4, nbzc = (nz / 2 + 1 - (c_first >> 2)) / 2;
  int pj = nx <= 64 ? 4 : 2;
  while (pj > 1 && (int64_t)((nby2 + pj - 1) / pj) * nbzc * ncomp < 2048) pj /= 2;
  return pj;
}

template <typename T>
hipError_t launch_block_pair(T* x, const T* b, const T* s1d, const T* zt, const T* bfac, int nx,
                             int ny, int nz, int ncomp, int c_first, const T* zn,
                             hipStream_t s) {
  if (nx > 128 || nx % 4 || ny % 4) return hipErrorNotSupported;
  const int nby2 = ny / 4, nbzc = (nz / 2 + 1 - (c_first >> 2)) / 2;
  if (nby2 * nbzc == 0 || ncomp == 0) return hipSuccess;
  const int PJ = pair_rows(nx, ny, nz, ncomp, c_first);
  const int plane = nx * (4 * PJ + 2);
  const int TP = plane + ((48 - plane % 32) % 32);
  const size_t lds = (size_t)TILE_D * TP * sizeof(T);
  const int nthr = (nx / 4) * PJ * 8;
  dim3 grid((nby2 + PJ - 1) / PJ, nbzc, ncomp);
  const uint32_t N = (uint32_t)nx * ny * nz;
#define SMG_PAIR(NZ, P)                                                                   \
  k_block_pair<T, NZ, P><<<grid, nthr, lds, s>>>(x, b, s1d, zt, bfac, nx, ny, nz, N, c_first, \
                                                 nby2, TP, zn)
  if (PJ == 4) {
    if (zn) SMG_PAIR(true, 4); else SMG_PAIR(false, 4);
  } else if (PJ == 2) {
    if (zn) SMG_PAIR(true, 2); else SMG_PAIR(false, 2);
  } else {
    if (zn) SMG_PAIR(true, 1); else SMG_PAIR(false, 1);
  }
#undef SMG_PAIR
  return hipGetLastError();
}

template <typename T, int PJ>
hipError_t launch_pair_multi_pj(const BlockPassItem<T>* items, int n, int c_first, bool noise,
                                hipStream_t s) {
  PairMultiArgs<T> m{};
  m.c_first = c_first;
  uint32_t total = 0;
  int nthr = 0;
  size_t lds = 0;
  auto flush = [&]() -> hipError_t {
    if (m.nitems == 0) return hipSuccess;
    m.begin[m.nitems] = total;
    if (noise) k_block_pair_multi<T, true, PJ><<<total, nthr, lds, s>>>(m);
    else k_block_pair_multi<T, false, PJ><<<total, nthr, lds, s>>>(m);
    m.nitems = 0;
    total = 0;
    nthr = 0;
    lds = 0;
    return hipGetLastError();
  };
  for (int q = 0; q < n; ++q) {
    const BlockPassItem<T>& p = items[q];
    if (pair_rows(p.nx, p.ny, p.nz, p.ncomp, c_first) != PJ) continue;
    const int nby2 = p.ny / 4, nbzc = (p.nz / 2 + 1 - (c_first >> 2)) / 2;
    if (nby2 * nbzc == 0 || p.ncomp == 0) continue;
    if (m.nitems == kBlockMultiItems) {
      hipError_t e = flush();
      if (e != hipSuccess) return e;
    }
    PairMultiItem<T>& it = m.it[m.nitems];
    it.x = p.x;
    it.b = p.b;
    it.s1d = p.s1d;
    it.zt = p.zt;
    it.bfac = p.bfac;
    it.zn = p.zn;
    it.nx = p.nx;
    it.ny = p.ny;
    it.nz = p.nz;
    it.N = (uint32_t)p.nx * p.ny * p.nz;
    it.nby2 = nby2;
    it.nbzc = nbzc;
    it.ngx = (nby2 + PJ - 1) / PJ;
    const int plane = p.nx * (4 * PJ + 2);
    it.TP = plane + ((48 - plane % 32) % 32);
    m.begin[m.nitems] = total;
    total += (uint32_t)it.ngx * nbzc * p.ncomp;
    nthr = std::max(nthr, (p.nx / 4) * PJ * 8);
    lds = std::max(lds, (size_t)TILE_D * it.TP * sizeof(T));
    ++m.nitems;
  }
  return flush();
}

template <typename T>
hipError_t launch_block_pair_multi(const BlockPassItem<T>* items, int n, int c_first,
                                   bool noise, hipStream_t s) {
  for (int q = 0; q < n; ++q)
    if (!pair_level(items[q].nx, items[q].ny)) return hipErrorNotSupported;
  hipError_t e = launch_pair_multi_pj<T, 4>(items, n, c_first, noise, s);
  if (e == hipSuccess) e = launch_pair_multi_pj<T, 2>(items, n, c_first, noise, s);
  if (e == hipSuccess) e = launch_pair_multi_pj<T, 1>(items, n, c_first, noise, s);
  return e;
}

template <typename T, int TI, int TJ>
hipError_t launch_block_multi_tiled(const BlockPassItem<T>* items, int n, int colour, bool noise,
                                    hipStream_t s) {
  BlockMultiArgs<T> m{};
  m.colour = colour;
  uint32_t total = 0;
  auto flush = [&]() -> hipError_t {
    if (m.nitems == 0) return hipSuccess;
    m.begin[m.nitems] = total;
    if (noise) k_block_tile_multi<T, true, TI, TJ><<<total, TI * TJ * 8, 0, s>>>(m);
    else k_block_tile_multi<T, false, TI, TJ><<<total, TI * TJ * 8, 0, s>>>(m);
    m.nitems = 0;
    total = 0;
    return hipGetLastError();
  };
  for (int q = 0; q < n; ++q) {
    const BlockPassItem<T>& p = items[q];
    const int nbx2 = p.nx / 4, nby2 = p.ny / 4;
    const int nbzc = (p.nz / 2 + 1 - (colour >> 2)) / 2;
    if (nbx2 * nby2 * nbzc == 0 || p.ncomp == 0) continue;
    const int ntx = (nbx2 + TI - 1) / TI, nty = (nby2 + TJ - 1) / TJ;
    const uint32_t wgs = (uint32_t)ntx * nty * nbzc * p.ncomp;
    if (m.nitems == kBlockMultiItems) {
      hipError_t e = flush();
      if (e != hipSuccess) return e;
    }
    BlockMultiItem<T>& it = m.it[m.nitems];
    it.x = p.x;
    it.b = p.b;
    it.s1d = p.s1d;
    it.zt = p.zt;
    it.bfac = p.bfac;
    it.zn = p.zn;
    it.nx = p.nx;
    it.ny = p.ny;
    it.nz = p.nz;
    it.N = (uint32_t)p.nx * p.ny * p.nz;
    it.nbx2 = nbx2;
    it.nby2 = nby2;
    it.nbzc = nbzc;
    it.ntx = ntx;
    it.nty = nty;
    m.begin[m.nitems] = total;
    total += wgs;
    ++m.nitems;
  }
  return flush();
}

template <typename T>
hipError_t launch_block_pass_multi(const BlockPassItem<T>* items, int n, int colour, bool noise,
                                   int tile, hipStream_t s) {
  if (tile == SMG_TILE_AUTO) {
    // the rule of launch_block_pass over the work-groups of all items together
    int64_t wg84 = 0, wg44 = 0;
    for (int q = 0; q < n; ++q) {
      const int nbx2 = items[q].nx / 4, nby2 = items[q].ny / 4;
      const int64_t layers = (int64_t)((items[q].nz / 2 + 1 - (colour >> 2)) / 2) * items[q].ncomp;
      wg84 += (int64_t)((nbx2 + 7) / 8) * ((nby2 + 3) / 4) * layers;
      wg44 += (int64_t)((nbx2 + 3) / 4) * ((nby2 + 3) / 4) * layers;
    }
    tile = wg84 >= 512 ? SMG_TILE_8X4 : (wg44 >= 512 ? SMG_TILE_4X4 : SMG_TILE_4X2);
  }
  if (tile == SMG_TILE_4X2) return launch_block_multi_tiled<T, 4, 2>(items, n, colour, noise, s);
  if (tile == SMG_TILE_8X4) return launch_block_multi_tiled<T, 8, 4>(items, n, colour, noise, s);
  return launch_block_multi_tiled<T, 4, 4>(items, n, colour, noise, s);
}

template <typename T>
hipError_t launch_residual_gal(T* r, const T* x, const T* b, const T* s1d, const T* zt, int nx,
                               int ny, int nz, int ncomp, hipStream_t s) {
  const int ntx = (nx + GR_X - 1) / GR_X, nty = (ny + GR_Y - 1) / GR_Y;
  dim3 grid(ntx * nty, (nz + GR_Z - 1) / GR_Z, ncomp);
  k_residual_gal_tile<T><<<grid, TPB, 0, s>>>(r, x, b, s1d, zt, nx, ny, nz, ntx);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict(T* bc, T* xc, const T* r, int nxf, int nyf, int nzf, int ncomp,
                           hipStream_t s) {
  const uint32_t Nf = (uint32_t)nxf * nyf * nzf;
  const uint32_t Nc = Nf / 8;
  dim3 grid(blocks_for(Nc), ncomp);
  k_restrict<T><<<grid, TPB, 0, s>>>(bc, xc, r, nxf, nyf, nzf, Nf, Nc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong(T* x, const T* e, int nxf, int nyf, int nzf, int ncomp, hipStream_t s) {
  const uint32_t Nf = (uint32_t)nxf * nyf * nzf;
  dim3 grid(blocks_for(Nf), ncomp);
  k_prolong<T><<<grid, TPB, 0, s>>>(x, e, nxf, nyf, nzf, Nf, Nf / 8);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coarsest(T* x, const T* b, const double* ainv, const double* w, int n,
                           int ncomp, bool noise, const NoiseArgs& na, hipStream_t s) {
  dim3 grid(blocks_for(n), ncomp);
  size_t lds = (size_t)(noise ? 2 : 1) * n * sizeof(double);
  if (noise) k_coarsest<T, true><<<grid, TPB, lds, s>>>(x, b, ainv, w, n, na);
  else k_coarsest<T, false><<<grid, TPB, lds, s>>>(x, b, ainv, w, n, na);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_level_noise(const NoiseGenArgs& a, const NoiseArgs& na, hipStream_t s) {
  if (a.total == 0 || a.nlev == 0) return hipSuccess;
  uint32_t maxblk = 0;
  int maxslot = 0;
  for (int e = 0; e < a.nlev; ++e) {
    const uint32_t nb = (uint32_t)a.lv[e].nx * a.lv[e].ny * a.lv[e].nz / 8;
    maxblk = nb > maxblk ? nb : maxblk;
    maxslot = a.lv[e].nslot > maxslot ? a.lv[e].nslot : maxslot;
  }
  dim3 grid(blocks_for(maxblk), a.nlev, maxslot * a.nact);
  k_level_noise<T><<<grid, TPB, 0, s>>>(a, na);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bottom(const BotArgs* a, int ncomp, int c0, size_t lds, bool noise,
                         const NoiseArgs& na, hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_bottom<T, true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_bottom<T, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (noise) k_bottom<T, true><<<ncomp, BOT_TPB, lds, s>>>(a, c0, na);
  else k_bottom<T, false><<<ncomp, BOT_TPB, lds, s>>>(a, c0, na);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bottom_multi(const BotMultiArgs& m, int nwg, size_t lds, bool noise,
                               hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_bottom_multi<T, true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_bottom_multi<T, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (nwg <= 0) return hipSuccess;
  if (nwg > kBotMultiWG || m.nitems > kBotMultiItems) return hipErrorInvalidValue;
  if (noise) k_bottom_multi<T, true><<<nwg, BOT_TPB, lds, s>>>(m);
  else k_bottom_multi<T, false><<<nwg, BOT_TPB, lds, s>>>(m);
  return hipGetLastError();
}

#define SMG_INST(T)                                                                            \
  template hipError_t launch_block_pass<T>(T*, const T*, const T*, const T*, const T*, int, int, \
                                           int, int, int, const T*, int, hipStream_t);          \
  template hipError_t launch_block_pair<T>(T*, const T*, const T*, const T*, const T*, int, int,  \
                                           int, int, int, const T*, hipStream_t);               \
  template hipError_t launch_block_pair_multi<T>(const BlockPassItem<T>*, int, int, bool,          \
                                                 hipStream_t);                                   \
  template hipError_t launch_block_pass_multi<T>(const BlockPassItem<T>*, int, int, bool, int,    \
                                                 hipStream_t);                                   \
  template hipError_t launch_residual_gal<T>(T*, const T*, const T*, const T*, const T*, int,    \
                                             int, int, int, hipStream_t);                        \
  template hipError_t launch_restrict<T>(T*, T*, const T*, int, int, int, int, hipStream_t);    \
  template hipError_t launch_prolong<T>(T*, const T*, int, int, int, int, hipStream_t);         \
  template hipError_t launch_coarsest<T>(T*, const T*, const double*, const double*, int, int,  \
                                         bool, const NoiseArgs&, hipStream_t);                  \
  template hipError_t launch_level_noise<T>(const NoiseGenArgs&, const NoiseArgs&, hipStream_t); \
  template hipError_t launch_bottom<T>(const BotArgs*, int, int, size_t, bool,                 \
                                       const NoiseArgs&, hipStream_t);                           \
  template hipError_t launch_bottom_multi<T>(const BotMultiArgs&, int, size_t, bool, hipStream_t);
SMG_INST(double)
SMG_INST(float)
#undef SMG_INST

}  // namespace smg
