// Utility kernels: fills, copies, casts, the natural-layout 7-point residual and fixed-order
// FP64 sums of squares (residual norms of the solve).
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace smg {
namespace {

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

// ----------------------------------------------------------------------------- utilities
template <typename T>
__global__ __launch_bounds__(TPB) void k_zero(T* __restrict__ p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * TPB) p[i] = T(0);
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

__global__ void k_set_chains(ChainKey* __restrict__ dst, ChainKeyBatch b) {
  const int t = threadIdx.x;
  if (t < b.count) dst[b.first + t] = b.k[t];
}

__global__ __launch_bounds__(TPB) void k_advance_chains(ChainKey* __restrict__ dst, int n,
                                                         uint64_t cycles) {
  const int t = blockIdx.x * TPB + threadIdx.x;
  if (t >= n) return;
  ChainKey k = dst[t];
  const uint64_t c = ((((uint64_t)k.c1) << 32) | k.c0) + cycles;
  k.c0 = (uint32_t)c;
  k.c1 = (uint32_t)(c >> 32);
  dst[t] = k;
}

}  // namespace

hipError_t launch_residual7_nat(double* r, const double* x, const double* b, int nx, int ny,
                                int nz, int ncomp, double h, hipStream_t s) {
  const uint32_t N = (uint32_t)nx * ny * nz;
  dim3 grid(blocks_for(N), ncomp);
  k_residual7_nat<<<grid, TPB, 0, s>>>(r, x, b, nx, ny, nz, N, 1.0 / (h * h));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zero(T* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_zero<T><<<grid_stride_blocks(n), TPB, 0, s>>>(p, n);
  return hipGetLastError();
}
template hipError_t launch_zero<double>(double*, int64_t, hipStream_t);
template hipError_t launch_zero<float>(float*, int64_t, hipStream_t);

hipError_t launch_sumsq_final_parts(double* out, const double* part, uint32_t nparts, int ncomp,
                                    hipStream_t s) {
  k_sumsq_final<<<ncomp, TPB, 0, s>>>(out, part, nparts);
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

hipError_t launch_sumsq(double* out, double* part, const double* v, int64_t n, int ncomp,
                        hipStream_t s) {
  const uint32_t nblk = blocks_for(n);
  k_sumsq_part<<<dim3(nblk, ncomp), TPB, 0, s>>>(part, v, n, nblk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_sumsq_final<<<ncomp, TPB, 0, s>>>(out, part, nblk);
  return hipGetLastError();
}

hipError_t launch_set_chains(ChainKey* dst, const ChainKeyBatch& b, hipStream_t s) {
  if (b.count <= 0) return hipSuccess;
  k_set_chains<<<1, kChainsPerLaunch, 0, s>>>(dst, b);
  return hipGetLastError();
}

hipError_t launch_advance_chains(ChainKey* dst, int n, uint64_t cycles, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_advance_chains<<<(n + TPB - 1) / TPB, TPB, 0, s>>>(dst, n, cycles);
  return hipGetLastError();
}

}  // namespace smg
