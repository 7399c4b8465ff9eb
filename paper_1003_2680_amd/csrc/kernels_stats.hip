// Statistics of an emitted sample, fused with its emission: per-cell FP64 moments, projections
// onto eigenvectors of A and the energy 1/2 x^T A x (the observables whose lag-k correlation
// measures how fast the chain decorrelates, Sec. "Stochastic Iterative Methods").
//
// A work-group takes STATS_CELLS consecutive cells of one component; a thread takes
// STATS_NB batches of STATS_CPT cells (256 apart, all loads of a batch issued before its
// arithmetic), so every wave keeps a batch in flight and the cross-lane sums at the end are
// paid once per 16 cells.  An eigenvector is a product e_a(x) e_b(y) w_m(z): when rows are a
// multiple of 64 cells a wavefront lies in one row and the (y, z) factor of each mode (a
// per-row table) is a uniform (scalar) load.  Sums run in a fixed order -- thread, butterfly
// over the lanes, the four waves of a work-group, then a tree over the work-groups -- so
// results do not depend on timing.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace smg {
namespace {

// One DPP step of a wave reduction on a double: v + (v moved by CTRL), lanes outside ROW_MASK
// adding zero.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double v) {
  const long long u = __double_as_longlong(v);
  int lo, hi;
  if (ROW_MASK == 0xf) {  // every lane is written: no old value to preset
    lo = __builtin_amdgcn_mov_dpp((int)u, CTRL, 0xf, 0xf, false);
    hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), CTRL, 0xf, 0xf, false);
  } else {
    lo = __builtin_amdgcn_update_dpp(0, (int)u, CTRL, ROW_MASK, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, ROW_MASK, 0xf, false);
  }
  return v + __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes in a fixed order (pairs, quads, eighths, rows, then rows 0+1 into
// row 1 and 2+3 into row 3, and the two halves into row 3); the total is in lane 63.
__device__ __forceinline__ double wave_sum63(double v) {
  v = dpp_add<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
  v = dpp_add<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xf>(v);  // row_half_mirror
  v = dpp_add<0x140, 0xf>(v);  // row_mirror
  v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

template <int KB, bool SPLIT, bool MOM, typename TO, bool UROW, bool XSAME>
__global__ __launch_bounds__(TPB) void k_stats(StatsArgs a) {
  // XCD-aware numbering: the +z neighbours of a work-group's cells belong to a work-group a
  // few ids on, which then runs on the same XCD and finds them in its L2
  const Blk3 wg = xcd_block();
  const uint32_t comp = wg.y;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const uint32_t N = (uint32_t)nx * ny * nz;
  const uint32_t plane = (uint32_t)nx * ny;
  // Split storage: the cell with natural index i sits at entry i >> 1 of its colour's array
  // (nx is even), and every face neighbour has the other colour.
  const double* __restrict__ Xr = a.xr + (size_t)comp * (SPLIT ? N >> 1 : N);
  const double* __restrict__ Xb = SPLIT ? a.xb + (size_t)comp * (N >> 1) : nullptr;
  auto load = [&](uint32_t cell, int par) -> double {
    if (SPLIT) return (par ? Xb : Xr)[cell >> 1];
    return Xr[cell];
  };
  TO* __restrict__ out = a.out ? (TO*)a.out + (size_t)comp * N : nullptr;
  double* __restrict__ m1 = MOM ? a.m1 + (size_t)comp * N : nullptr;
  double* __restrict__ m2 = MOM ? a.m2 + (size_t)comp * N : nullptr;
  const int K = a.nmodes;
  // the mode tables are read-only for the kernel's lifetime: through the constant address
  // space the row factor of a mode (a uniform address when a wave lies in one row) becomes a
  // scalar load used directly as an FMA operand
  typedef const __attribute__((address_space(4))) double* cptr;
  const double* __restrict__ tx = a.tx;
  const cptr trow = (cptr)a.trow;
  const uint32_t base = wg.x * STATS_CELLS;
  // A thread takes STATS_NB batches of STATS_CPT cells (TPB apart), all loads of a batch
  // before its arithmetic.  When a wavefront lies in one row (UROW) its row, y, z and the
  // wall and range tests are wave-uniform (scalar), the +x neighbour of a cell is the next
  // lane's value and only the wave's last lane loads it.  When a thread's cells are whole rows
  // apart (XSAME) they share their x: the x factor of a mode multiplies the thread's sum once
  // at the end.  Mode tables are zero beyond the K modes in use, so the first KB <= 8 sums
  // need no guard.
  double acc[KB > 0 ? KB : 1];
#pragma unroll
  for (int q = 0; q < (KB > 0 ? KB : 1); ++q) acc[q] = 0.0;
  double accE = 0.0;
  if constexpr (UROW) {
#pragma unroll 1
    for (int bt = 0; bt < STATS_NB; ++bt) {
      const uint32_t bbase = base + bt * (STATS_CPT * TPB);
      double v[STATS_CPT], ny1[STATS_CPT], nz1[STATS_CPT], nx1[STATS_CPT];
      int xs[STATS_CPT];
      uint32_t rows[STATS_CPT], zs[STATS_CPT];
#pragma unroll
      for (int c = 0; c < STATS_CPT; ++c) {
        const uint32_t cell = bbase + c * TPB + threadIdx.x;
        const uint32_t cell0 = __builtin_amdgcn_readfirstlane(cell - lane);  // the wave's row
        const bool in = cell0 < N;
        const uint32_t row = udiv(in ? cell0 : 0, nx, a.lgx);
        const uint32_t z = udiv(row, ny, a.lgy);
        const uint32_t y = row - z * ny;
        const int x = (int)(cell - row * nx);
        const int par = (x + (int)(y + z)) & 1;
        rows[c] = in ? row : 0xffffffffu;
        zs[c] = z;
        xs[c] = x;
        v[c] = 0.0;
        nx1[c] = ny1[c] = nz1[c] = 0.0;
        if (in) {
          v[c] = load(cell, par);
          if (KB > 0) {
            ny1[c] = load(y + 1 == (uint32_t)ny ? cell - (plane - nx) : cell + nx, par ^ 1);
            if (z + 1 < (uint32_t)nz) nz1[c] = load(cell + plane, par ^ 1);
            if (lane == 63) nx1[c] = load(x + 1 == nx ? cell + 1 - nx : cell + 1, par ^ 1);
          }
        }
      }
#pragma unroll
      for (int c = 0; c < STATS_CPT; ++c) {
        if (rows[c] == 0xffffffffu) continue;
        const uint32_t cell = bbase + c * TPB + threadIdx.x;
        const double x0 = v[c];
        if (out) out[cell] = (TO)x0;
        if (MOM) {
          m1[cell] += x0;
          m2[cell] = fma(x0, x0, m2[cell]);
        }
        if (KB > 0) {
          const uint32_t row = rows[c], z = zs[c];
          const cptr tr = trow + (size_t)row * KB;
#pragma unroll
          for (int q = 0; q < KB; ++q)
            if (KB <= 8 || q < K)
              acc[q] = XSAME ? fma(tr[q], x0, acc[q])
                             : fma(tx[q * nx + xs[c]] * tr[q], x0, acc[q]);
          // faces +x, +y (periodic) and +z (interior), plus the wall faces (ghost = -v)
          const double nxt = __shfl_down(x0, 1, 64);
          const double d1 = x0 - (lane == 63 ? nx1[c] : nxt);
          const double d2 = x0 - ny1[c];
          double e = fma(d1, d1, d2 * d2);
          if (z + 1 < (uint32_t)nz) {
            const double d3 = x0 - nz1[c];
            e = fma(d3, d3, e);
          }
          if (z == 0) e = fma(2.0 * x0, x0, e);
          if (z == (uint32_t)nz - 1) e = fma(2.0 * x0, x0, e);
          accE += e;
        }
      }
    }
    if (KB > 0 && XSAME) {
      const uint32_t c0 = base + threadIdx.x;
      const int x0 = (int)(c0 - udiv(c0, nx, a.lgx) * nx);
#pragma unroll
      for (int q = 0; q < KB; ++q)
        if (KB <= 8 || q < K) acc[q] *= tx[q * nx + x0];
    }
  } else {
#pragma unroll 1
    for (int bt = 0; bt < STATS_NB; ++bt) {
      const uint32_t bbase = base + bt * (STATS_CPT * TPB);
      double v[STATS_CPT], nb[STATS_CPT][3];
      int cx[STATS_CPT], cz[STATS_CPT];
      uint32_t rows[STATS_CPT];
#pragma unroll
      for (int c = 0; c < STATS_CPT; ++c) {
        const uint32_t cell = bbase + c * TPB + threadIdx.x;
        const bool in = cell < N;
        const uint32_t cc = in ? cell : 0;
        const uint32_t row = udiv(cc, nx, a.lgx);
        const int x = cc - row * nx;
        const uint32_t zz = udiv(row, ny, a.lgy);
        const int y = row - zz * ny, z = zz;
        const int par = (x + y + z) & 1;
        cx[c] = x;
        rows[c] = row;
        cz[c] = in ? z : -1;
        v[c] = in ? load(cc, par) : 0.0;
        if (KB > 0) {
          nb[c][0] = in ? load(x + 1 == nx ? cc + 1 - nx : cc + 1, par ^ 1) : 0.0;
          nb[c][1] = in ? load(y + 1 == ny ? cc - (plane - nx) : cc + nx, par ^ 1) : 0.0;
          nb[c][2] = (in && z + 1 < nz) ? load(cc + plane, par ^ 1) : 0.0;
        }
      }
#pragma unroll
      for (int c = 0; c < STATS_CPT; ++c) {
        if (cz[c] < 0) continue;
        const uint32_t cell = bbase + c * TPB + threadIdx.x;
        const double x0 = v[c];
        if (out) out[cell] = (TO)x0;
        if (MOM) {
          m1[cell] += x0;
          m2[cell] = fma(x0, x0, m2[cell]);
        }
        if (KB > 0) {
          const int z = cz[c];
#pragma unroll
          for (int q = 0; q < KB; ++q)
            if (KB <= 8 || q < K)
              acc[q] = fma(tx[q * nx + cx[c]] * a.trow[(size_t)rows[c] * KB + q], x0, acc[q]);
          const double d1 = x0 - nb[c][0];
          const double d2 = x0 - nb[c][1];
          double e = fma(d1, d1, d2 * d2);
          if (z + 1 < nz) {
            const double d3 = x0 - nb[c][2];
            e = fma(d3, d3, e);
          }
          if (z == 0) e = fma(2.0 * x0, x0, e);
          if (z == nz - 1) e = fma(2.0 * x0, x0, e);
          accE += e;
        }
      }
    }
  }
  if (KB == 0) return;
  __shared__ double red[4][KB + 1];
#pragma unroll
  for (int q = 0; q <= KB; ++q) {
    if (q < KB && !(KB <= 8 || q < K)) continue;
    const double s = wave_sum63(q < KB ? acc[q] : accE);
    if (lane == 63) red[w][q] = s;
  }
  __syncthreads();
  const int q = threadIdx.x;
  if (q <= K) {
    const int qi = q == K ? KB : q;
    a.part[((size_t)comp * a.nblk + wg.x) * (K + 1) + q] =
        ((red[0][qi] + red[1][qi]) + red[2][qi]) + red[3][qi];
  }
}

// obs[comp][q] = sum over work-groups of part[comp][blk][q]: one work-group per (comp, q),
// thread t adds partials t, t + 256, ... in order, then a fixed tree in LDS.  The energy
// (q = K) is scaled by 1/(2 h^2).
__global__ __launch_bounds__(TPB) void k_stats_final(double* __restrict__ obs,
                                                      const double* __restrict__ part, int nblk,
                                                      int K1, double escale) {
  __shared__ double sh[TPB];
  const int comp = blockIdx.y, q = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += TPB) s += part[((size_t)comp * nblk + b) * K1 + q];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int st = TPB / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) obs[comp * K1 + q] = q == K1 - 1 ? sh[0] * escale : sh[0];
}

template <int KB, bool SPLIT, bool MOM, bool UROW, bool XSAME>
void launch_stats_u(const StatsArgs& a, int ncomp, hipStream_t s) {
  dim3 grid(a.nblk, ncomp);
  if (a.out && a.out_f32) k_stats<KB, SPLIT, MOM, float, UROW, XSAME><<<grid, TPB, 0, s>>>(a);
  else k_stats<KB, SPLIT, MOM, double, UROW, XSAME><<<grid, TPB, 0, s>>>(a);
}

template <int KB, bool SPLIT, bool MOM>
void launch_stats_k(const StatsArgs& a, int ncomp, hipStream_t s) {
  // rows of 64, 128 or 256 cells: a wave lies in one row and a thread's cells are whole rows
  // apart
  if (a.nx % 64 == 0 && TPB % a.nx == 0) launch_stats_u<KB, SPLIT, MOM, true, true>(a, ncomp, s);
  else if (a.nx % 64 == 0) launch_stats_u<KB, SPLIT, MOM, true, false>(a, ncomp, s);
  else launch_stats_u<KB, SPLIT, MOM, false, false>(a, ncomp, s);
}

template <int KB>
void launch_stats_kb(const StatsArgs& a, int ncomp, hipStream_t s) {
  const bool split = a.xb != nullptr, mom = a.m1 != nullptr;
  if (split) {
    if (mom) launch_stats_k<KB, true, true>(a, ncomp, s);
    else launch_stats_k<KB, true, false>(a, ncomp, s);
  } else {
    if (mom) launch_stats_k<KB, false, true>(a, ncomp, s);
    else launch_stats_k<KB, false, false>(a, ncomp, s);
  }
}

}  // namespace

hipError_t launch_stats(const StatsArgs& a, int ncomp, double* obs, double escale,
                        hipStream_t s) {
  if (!obs) launch_stats_kb<0>(a, ncomp, s);
  else if (a.nmodes <= 8) launch_stats_kb<8>(a, ncomp, s);
  else launch_stats_kb<kMaxModes>(a, ncomp, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !obs) return e;
  const int K1 = a.nmodes + 1;
  k_stats_final<<<dim3(K1, ncomp), TPB, 0, s>>>(obs, a.part, a.nblk, K1, escale);
  return hipGetLastError();
}

}  // namespace smg
