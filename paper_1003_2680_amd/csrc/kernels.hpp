// Launchers of the HIP kernels (host-callable).  Fields are float64; level 0 of a
// point-smoothed hierarchy is stored split by colour: colour c (cells with (x+y+z)%2 == c)
// occupies [ncomp][nz][ny][nx/2], entry j of row (y,z) being x = 2j + ((y+z+c)&1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"

namespace smg {

// How a level is smoothed (Sec. "Stochastic Multigrid Methods": the smoother is stochastic
// Gauss-Seidel; on Galerkin levels a 2x2x2 block heat bath keeps every colour class
// uncoupled) or, for the coarsest level, drawn exactly.
enum LevelKind { KIND_POINT = 0, KIND_BLOCK = 1, KIND_CHOL = 2 };

// Levels of the LDS-resident bottom of the V-cycle (kernel argument).
constexpr int kMaxBotLevels = 6;
// Pregenerated block-level noise: for level `level` (dims nx, ny, nz) and sweep slots
// slot0 .. slot0+nslot-1, out[(s*ncomp + comp)*N + cell] is the standard normal of `cell`,
// drawn from the stream (level, slot, colour of the cell's 2x2x2 block, comp); the call of a
// cell is (8*block + in-block index) >> 1 and the even/odd in-block index takes z0/z1.
constexpr int kMaxNoiseLevels = 16;
struct NoiseLevel {
  int level, nx, ny, nz, nslot, slot0;
  double* out;
  uint32_t calls_before;  // prefix sum of nslot*ncomp*N/2 over the previous entries
};
struct NoiseGenArgs {
  int nlev, ncomp;
  uint32_t total;
  NoiseLevel lv[kMaxNoiseLevels];
};
hipError_t launch_level_noise(const NoiseGenArgs& a, const NoiseArgs& na, hipStream_t s);

struct BotLevel {
  int nx, ny, nz, kind;
  int sy, sz;          // LDS strides (doubles): padded for block levels, natural for the coarsest
  const double* noise; // pregenerated noise of this level: [slot][ncomp][N] (block levels)
  const double* g2d;   // KIND_BLOCK: [2][25]
  const double* zt;    // KIND_BLOCK: [nz][10]
  const double* bfac;  // KIND_BLOCK: [nz/2][3][64]
};
struct BotArgs {
  int nlev, level0, nu1, nu2, ncomp;
  BotLevel lv[kMaxBotLevels];
  int lds_off[kMaxBotLevels];  // LDS offset (doubles) of level i's x; b and scratch follow
  int tab_off[kMaxBotLevels];  // LDS offset (doubles) of level i's tables (g2d, zt, bfac)
  const double* b_in;  // [ncomp][n of the first bottom level]
  double* x_out;       // [ncomp][n of the first bottom level]
  const double* ainv;  // coarsest A_c^-1 (KIND_CHOL)
  const double* w;     // coarsest L_c^-1 (KIND_CHOL)
};

hipError_t launch_rb_pass(double* xc, const double* xo, const double* bc, int nx, int ny, int nz,
                          int ncomp, int colour, double h, double kT, bool noise,
                          const NoiseArgs& na, hipStream_t s);
hipError_t launch_residual0(double* r, const double* xr, const double* xb, const double* br,
                            const double* bb, int nx, int ny, int nz, int ncomp, double h,
                            hipStream_t s);
hipError_t launch_residual7_nat(double* r, const double* x, const double* b, int nx, int ny,
                                int nz, int ncomp, double h, hipStream_t s);
hipError_t launch_residual_gal(double* r, const double* x, const double* b, const double* g2d,
                               const double* zt, int nx, int ny, int nz, int ncomp,
                               hipStream_t s);
// b_c = P^T r; also x_c = 0 when xc is not null
hipError_t launch_restrict(double* bc, double* xc, const double* r, int nxf, int nyf, int nzf,
                           int ncomp, hipStream_t s);
hipError_t launch_prolong0(double* xr, double* xb, const double* e, int nxf, int nyf, int nzf,
                           int ncomp, hipStream_t s);
hipError_t launch_prolong(double* x, const double* e, int nxf, int nyf, int nzf, int ncomp,
                          hipStream_t s);
// z: pregenerated noise of this pass's sweep, [ncomp][N] (null without noise)
hipError_t launch_block_pass(double* x, const double* b, const double* g2d, const double* zt,
                             const double* bfac, int nx, int ny, int nz, int ncomp, int colour,
                             const double* z, double sqkT, hipStream_t s);
// LDS strides of a bottom level: rows padded to 2 mod 4 and planes to 1 mod 4 doubles on the
// block levels (bank spread of the 8 cells x 8 blocks of a wave); the coarsest stays natural.
inline void bot_strides(int kind, int nx, int ny, int& sy, int& sz) {
  if (kind == KIND_BLOCK) {
    sy = nx + 2;
    sz = ny * (nx + 2) + 1;
  } else {
    sy = nx;
    sz = nx * ny;
  }
}
inline size_t bot_field_doubles(int kind, int nx, int ny, int nz) {
  int sy, sz;
  bot_strides(kind, nx, ny, sy, sz);
  return (size_t)nz * sz;
}

// `a` points to a BotArgs in device memory
hipError_t launch_bottom(const BotArgs* a, int ncomp, size_t lds, bool noise, const NoiseArgs& na,
                         hipStream_t s);
hipError_t launch_coarsest(double* x, const double* b, const double* ainv, const double* w, int n,
                           int ncomp, bool noise, const NoiseArgs& na, hipStream_t s);
hipError_t launch_zero(double* p, int64_t n, hipStream_t s);
hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s);
hipError_t launch_to_split(double* xr, double* xb, const double* nat, int nx, int ny, int nz,
                           int ncomp, hipStream_t s);
hipError_t launch_from_split(void* nat, int out_f32, const double* xr, const double* xb, int nx,
                             int ny, int nz, int ncomp, hipStream_t s);
hipError_t launch_cast(void* dst, int out_f32, const double* src, int64_t n, hipStream_t s);
// sums of squares per component of v[ncomp][n] into out[ncomp] (fixed reduction order)
hipError_t launch_sumsq(double* out, double* part, const double* v, int64_t n, int ncomp,
                        hipStream_t s);

}  // namespace smg
