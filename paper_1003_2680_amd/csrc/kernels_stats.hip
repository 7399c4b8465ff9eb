// Statistics of an emitted sample, fused with its emission: per-cell FP64 moments, projections
// onto eigenvectors of A and the energy 1/2 x^T A x (the observables whose lag-k correlation
// measures how fast the chain decorrelates, Sec. "Stochastic Iterative Methods").
//
// One wavefront walks whole grid rows (y, z uniform across the wave), its lanes along x.  An
// eigenvector is a product e_a(x) e_b(y) w_m(z), so the (y, z) factor of every mode is read
// once per row (uniform loads) and the x factor once per cell.  Sums run in a fixed order:
// lane partials over a wave's rows, a butterfly over the lanes, the four waves of a work-group,
// then a second kernel over the work-groups, so results do not depend on timing.
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

template <int KB, bool SPLIT, bool MOM, typename TO>
__global__ __launch_bounds__(TPB) void k_stats(StatsArgs a) {
  const uint32_t comp = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const size_t N = (size_t)nx * ny * nz;
  const size_t hN = N >> 1;
  const int nh = nx >> 1;
  const double* Xr = a.xr + comp * (SPLIT ? hN : N);
  const double* Xb = SPLIT ? a.xb + comp * hN : nullptr;
  auto load = [&](int x, int y, int z) -> double {
    if (SPLIT) {
      const size_t i = ((size_t)z * ny + y) * nh + (x >> 1);
      return ((x + y + z) & 1) ? Xb[i] : Xr[i];
    }
    return Xr[((size_t)z * ny + y) * nx + x];
  };
  TO* out = (TO*)a.out;
  const int K = a.nmodes;
  double acc[KB > 0 ? KB : 1];
#pragma unroll
  for (int q = 0; q < (KB > 0 ? KB : 1); ++q) acc[q] = 0.0;
  double accE = 0.0;
  const int rows = ny * nz;
  for (int r = blockIdx.x * 4 + w; r < rows; r += a.nblk * 4) {
    const int y = r % ny, z = r / ny;
    double u[KB > 0 ? KB : 1];
    if (KB > 0) {
#pragma unroll
      for (int q = 0; q < KB; ++q) u[q] = q < K ? a.ty[q * ny + y] * a.tz[q * nz + z] : 0.0;
    }
    for (int x = lane; x < nx; x += 64) {
      const double v = load(x, y, z);
      const size_t cell = comp * N + (size_t)r * nx + x;
      if (out) out[cell] = (TO)v;
      if (MOM) {
        a.m1[cell] += v;
        a.m2[cell] = fma(v, v, a.m2[cell]);
      }
      if (KB > 0) {
#pragma unroll
        for (int q = 0; q < KB; ++q)
          if (q < K) acc[q] = fma(a.tx[q * nx + x], v * u[q], acc[q]);
        // faces +x, +y (periodic) and +z (interior), plus the wall faces (ghost = -v)
        const double d1 = v - load(x + 1 == nx ? 0 : x + 1, y, z);
        const double d2 = v - load(x, y + 1 == ny ? 0 : y + 1, z);
        double e = fma(d1, d1, d2 * d2);
        if (z + 1 < nz) {
          const double d3 = v - load(x, y, z + 1);
          e = fma(d3, d3, e);
        }
        if (z == 0) e = fma(2.0 * v, v, e);
        if (z == nz - 1) e = fma(2.0 * v, v, e);
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
    a.part[((size_t)comp * a.nblk + blockIdx.x) * (K + 1) + q] =
        ((red[0][qi] + red[1][qi]) + red[2][qi]) + red[3][qi];
  }
}

// obs[comp][q] = sum over work-groups of part[comp][blk][q]; the energy (q = K) is scaled by
// 1/(2 h^2).
__global__ __launch_bounds__(TPB) void k_stats_final(double* __restrict__ obs,
                                                      const double* __restrict__ part, int nblk,
                                                      int K1, int ncomp, double escale) {
  const int t = blockIdx.x * TPB + threadIdx.x;
  if (t >= ncomp * K1) return;
  const int comp = t / K1, q = t % K1;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[((size_t)comp * nblk + b) * K1 + q];
  obs[t] = q == K1 - 1 ? s * escale : s;
}

template <int KB, bool SPLIT, bool MOM>
void launch_stats_k(const StatsArgs& a, int ncomp, hipStream_t s) {
  dim3 grid(a.nblk, ncomp);
  if (a.out && a.out_f32) k_stats<KB, SPLIT, MOM, float><<<grid, TPB, 0, s>>>(a);
  else k_stats<KB, SPLIT, MOM, double><<<grid, TPB, 0, s>>>(a);
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
  const int total = ncomp * K1;
  k_stats_final<<<(total + TPB - 1) / TPB, TPB, 0, s>>>(obs, a.part, a.nblk, K1, ncomp, escale);
  return hipGetLastError();
}

}  // namespace smg
