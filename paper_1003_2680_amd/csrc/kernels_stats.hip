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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
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
  const uint32_t hN = N >> 1;
  const int nh = nx >> 1;
  const double* Xr = a.xr + (size_t)comp * (SPLIT ? hN : N);
  const double* Xb = SPLIT ? a.xb + (size_t)comp * hN : nullptr;
  auto load = [&](int x, int y, int z) -> double {
    if (SPLIT) {
      const uint32_t i = ((uint32_t)z * ny + y) * nh + (x >> 1);
      return ((x + y + z) & 1) ? Xb[i] : Xr[i];
    }
    return Xr[((uint32_t)z * ny + y) * nx + x];
  };
  TO* out = (TO*)a.out;
  const int K = a.nmodes;
  // the mode tables are read-only for the kernel's lifetime: through the constant address
  // space the row factor of a mode (a uniform address when a wave lies in one row) becomes a
  // scalar load used directly as an FMA operand
  typedef const __attribute__((address_space(4))) double* cptr;
  const double* __restrict__ tx = a.tx;
  const cptr trow = (cptr)a.trow;
  const uint32_t base = wg.x * STATS_CELLS;
  // A thread takes STATS_NB batches of STATS_CPT cells (TPB apart), all loads of a batch
  // before its arithmetic.  When a wavefront lies in one row (UROW) the +x neighbour of a cell
  // is the next lane's value and only the wave's last lane loads it, and a wave's cells are all
  // inside the grid or all outside; when a thread's cells are whole rows apart (XSAME) they
  // share their x, hence the x factors of the modes.  Mode tables are zero beyond the K modes
  // in use, so the first KB <= 8 sums need no guard.
  double acc[KB > 0 ? KB : 1];
#pragma unroll
  for (int q = 0; q < (KB > 0 ? KB : 1); ++q) acc[q] = 0.0;
  double accE = 0.0;
  double txs[KB > 0 ? KB : 1];
  if (KB > 0 && XSAME) {
    const uint32_t c0 = base + threadIdx.x;
    const int x0 = (int)(c0 - udiv(c0, nx, a.lgx) * nx);
#pragma unroll
    for (int q = 0; q < KB; ++q) txs[q] = (KB <= 8 || q < K) ? tx[q * nx + x0] : 0.0;
  }
#pragma unroll 1
  for (int bt = 0; bt < STATS_NB; ++bt) {
    const uint32_t bbase = base + bt * (STATS_CPT * TPB);
    double v[STATS_CPT], nb[STATS_CPT][3];
    int cx[STATS_CPT], cy[STATS_CPT], cz[STATS_CPT];
#pragma unroll
    for (int c = 0; c < STATS_CPT; ++c) {
      const uint32_t cell = bbase + c * TPB + threadIdx.x;
      const bool in = UROW ? __builtin_amdgcn_readfirstlane(cell) < N : cell < N;
      const uint32_t cc = in ? cell : 0;
      const uint32_t row = udiv(cc, nx, a.lgx);
      const int x = cc - row * nx;
      const uint32_t zz = udiv(row, ny, a.lgy);
      const int y = row - zz * ny, z = zz;
      cx[c] = x;
      cy[c] = y;
      cz[c] = in ? z : -1;
      v[c] = in ? load(x, y, z) : 0.0;
      if (KB > 0) {
        const int xp = x + 1 == nx ? 0 : x + 1;
        nb[c][0] = (in && (!UROW || lane == 63)) ? load(xp, y, z) : 0.0;
        nb[c][1] = in ? load(x, y + 1 == ny ? 0 : y + 1, z) : 0.0;
        nb[c][2] = (in && z + 1 < nz) ? load(x, y, z + 1) : 0.0;
      }
    }
    if (KB > 0 && UROW) {
#pragma unroll
      for (int c = 0; c < STATS_CPT; ++c) {
        const double nxt = __shfl_down(v[c], 1, 64);
        if (lane != 63) nb[c][0] = nxt;
      }
    }
#pragma unroll
    for (int c = 0; c < STATS_CPT; ++c) {
      if (cz[c] < 0) continue;
      const size_t gi = (size_t)comp * N + bbase + c * TPB + threadIdx.x;
      const double x0 = v[c];
      if (out) out[gi] = (TO)x0;
      if (MOM) {
        a.m1[gi] += x0;
        a.m2[gi] = fma(x0, x0, a.m2[gi]);
      }
      if (KB > 0) {
        const int z = cz[c];
        uint32_t row = (uint32_t)z * ny + cy[c];
        if (UROW) row = __builtin_amdgcn_readfirstlane(row);  // the wavefront lies in one row
#pragma unroll
        for (int q = 0; q < KB; ++q)
          if (KB <= 8 || q < K)
            acc[q] = fma((XSAME ? txs[q] : tx[q * nx + cx[c]]) * trow[(size_t)row * KB + q], x0,
                         acc[q]);
        // faces +x, +y (periodic) and +z (interior), plus the wall faces (ghost = -v)
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
  if (KB == 0) return;
  __shared__ double red[4][KB + 1];
#pragma unroll
  for (int q = 0; q <= KB; ++q) {
    const double s = wave_sum(q < KB ? acc[q] : accE);
    if (lane == 0) red[w][q] = s;
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
