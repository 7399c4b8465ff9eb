// Launchers of the HIP kernels (host-callable).  T is the storage and arithmetic type of a
// sweep: double in SMG_FP64, float for the inner cycle of SMG_FP32_REFINED.  Level 0 of a
// point-smoothed hierarchy is stored split by colour: colour c (cells with (x+y+z)%2 == c)
// occupies [ncomp][nz][ny][nx/2], entry j of row (y,z) being x = 2j + ((y+z+c)&1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/smg.h"
#include "philox.hpp"

namespace smg {

// How a level is smoothed (Sec. "Stochastic Multigrid Methods": the smoother is stochastic
// Gauss-Seidel; on Galerkin levels a 2x2x2 block heat bath keeps every colour class
// uncoupled) or, for the coarsest level, drawn exactly.
enum LevelKind { KIND_POINT = 0, KIND_BLOCK = 1, KIND_CHOL = 2 };

// Pregenerated block-level noise: for level `level` (dims nx, ny, nz) and sweep slots
// slot0 .. slot0+nslot-1, out[(s*ncomp + comp)*N + cell] is the standard normal of `cell`,
// drawn from the stream (level, slot, colour of the cell's 2x2x2 block, comp); the call of a
// cell is (8*block + in-block index) >> 1 and the even/odd in-block index takes z0/z1.
constexpr int kMaxNoiseLevels = 16;
struct NoiseLevel {
  int level, nx, ny, nz, nslot, slot0;
  int lg_bx, lg_bxy;      // log2 of nx/2 and of (nx/2)(ny/2) when powers of two, else -1
  void* out;              // T[nslot][ncomp][N]
  const void* bfac;       // T[nz/2][192]: the level's block factors (L_BB^-T at offset 64)
  uint32_t calls_before;  // prefix sum of nslot*nact*N/2 over the previous entries
};
struct NoiseGenArgs {
  int nlev;
  int ncomp;   // component stride of the noise buffers
  int nact;    // components drawn (the first nact)
  uint32_t total;
  NoiseLevel lv[kMaxNoiseLevels];
};

// Levels of the LDS-resident bottom of the V-cycle (read by the kernel from device memory).
constexpr int kMaxBotLevels = 6;
struct BotLevel {
  int nx, ny, nz, kind;
  int sy, sz;          // LDS strides: padded for block levels, natural for the coarsest
  const void* noise;   // T: pregenerated noise of this level [slot][ncomp][N] (block levels)
  double s1d[20];      // 1D stencils (m_x, a_x, m_y, a_y), offsets -2..2
  const void* zt;      // T: [nz][10]
  const void* bfac;    // T: [nz/2][3][64]
};
struct BotArgs {
  int nlev, level0, nu1, nu2, ncomp;
  BotLevel lv[kMaxBotLevels];
  int lds_off[kMaxBotLevels];  // LDS offset (elements of T) of level i's x; b, scratch follow
  int tab_off[kMaxBotLevels];  // LDS offset (elements of T) of level i's tables
  const void* b_in;    // T [ncomp][n of the first bottom level]
  void* x_out;         // T [ncomp][n of the first bottom level]
  const double* ainv;  // coarsest A_c^-1 (FP64 in every mode)
  const double* w;     // coarsest L_c^-1
};

// LDS strides of a bottom level: on the block levels rows are padded by 2 elements and
// planes to the first count that is 16 mod 32 elements, which spreads a wave's reads of one
// window offset (8 cells x 8 blocks, the two z-layers of a block three planes apart) over the
// 64 banks; the coarsest stays natural.
inline void bot_strides(int kind, int nx, int ny, int& sy, int& sz) {
  if (kind == KIND_BLOCK) {
    sy = nx + 2;
    sz = ny * sy + (48 - (ny * sy) % 32) % 32;
  } else {
    sy = nx;
    sz = nx * ny;
  }
}
inline size_t bot_field_elems(int kind, int nx, int ny, int nz) {
  int sy, sz;
  bot_strides(kind, nx, ny, sy, sz);
  return (size_t)nz * sz;
}

template <typename T>
hipError_t launch_rb_pass(T* xc, const T* xo, const T* bc, int nx, int ny, int nz, int ncomp,
                          int colour, double h, double kT, bool noise, const NoiseArgs& na,
                          hipStream_t s);
template <typename T>
hipError_t launch_residual0(T* r, const T* xr, const T* xb, const T* br, const T* bb, int nx,
                            int ny, int nz, int ncomp, double h, hipStream_t s);
// b_c = P^T (b - A x) from split level-0 storage straight to the natural coarse level (r is
// never written); also x_c = 0 when xc is not null.  br/bb null = 0.
template <typename T>
hipError_t launch_restrict_residual0(T* bc, T* xc, const T* xr, const T* xb, const T* br,
                                     const T* bb, int nx, int ny, int nz, int ncomp, double h,
                                     hipStream_t s);
// colours: bit c set = add P e to the sites of colour c
template <typename T>
hipError_t launch_prolong0(T* xr, T* xb, const T* e, int nxf, int nyf, int nzf, int ncomp,
                           int colours, hipStream_t s);
template <typename T>
hipError_t launch_residual_gal(T* r, const T* x, const T* b, const T* s1d, const T* zt, int nx,
                               int ny, int nz, int ncomp, hipStream_t s);
// b_c = P^T r; also x_c = 0 when xc is not null
template <typename T>
hipError_t launch_restrict(T* bc, T* xc, const T* r, int nxf, int nyf, int nzf, int ncomp,
                           hipStream_t s);
template <typename T>
hipError_t launch_prolong(T* x, const T* e, int nxf, int nyf, int nzf, int ncomp, hipStream_t s);
// z: pregenerated noise of this pass's sweep, [ncomp][N], each block's normals already
// multiplied by sqrt(kT) L_BB^-T (null without noise); tile: one of the SMG_TILE_* shapes of
// smg.h (SMG_TILE_AUTO picks by work-group count)
template <typename T>
hipError_t launch_block_pass(T* x, const T* b, const T* s1d, const T* zt, const T* bfac, int nx,
                             int ny, int nz, int ncomp, int colour, const T* z, int tile,
                             hipStream_t s);
// Block colours c_first and then c_first ^ 1 of one sweep in one launch, with the result of
// the two single-colour passes in that order; levels with nx <= 128 and nx, ny multiples of 4
// (hipErrorNotSupported otherwise: the caller runs the two passes).
// true where a Galerkin level's sweeps can run as two-colour launches
inline bool pair_level(int nx, int ny) { return nx <= 128 && nx % 4 == 0 && ny % 4 == 0; }
template <typename T>
hipError_t launch_block_pair(T* x, const T* b, const T* s1d, const T* zt, const T* bfac, int nx,
                             int ny, int nz, int ncomp, int c_first, const T* z, hipStream_t s);

// One level-0 colour pass over several hierarchies in one launch (up to 8 per launch): each
// item as the arguments of launch_rb_pass (its colour arrays, right-hand side, shape, active
// components, h, kT and noise keys); every item has a right-hand side iff has_b.  The result
// of each item is that of launch_rb_pass on it alone.
template <typename T>
struct RbPassItem {
  T* xc;
  const T* xo;
  const T* bc;
  int nx, ny, nz, ncomp;
  double h, kT;
  NoiseArgs na;
};
template <typename T>
hipError_t launch_rb_pass_multi(const RbPassItem<T>* items, int n, int colour, bool has_b,
                               bool noise, hipStream_t s);

// One block-colour pass over the levels of several hierarchies in one launch (up to
// kBlockMultiItems per launch; more are split into several launches).  Each item is one level
// of one hierarchy: its fields and tables as for launch_block_pass, its active components and
// its own noise field (null when noise is off).  The items' passes are independent: the
// result of each is that of launch_block_pass on it alone.
template <typename T>
struct BlockPassItem {
  T* x;
  const T* b;
  const T* s1d;
  const T* zt;
  const T* bfac;
  const T* zn;
  int nx, ny, nz, ncomp;
};
constexpr int kBlockMultiItems = 16;
template <typename T>
struct BlockMultiItem {
  T* x;
  const T* b;
  const T* s1d;
  const T* zt;
  const T* bfac;
  const T* zn;
  int nx, ny, nz;
  uint32_t N;
  int nbx2, nby2, nbzc, ntx, nty;
};
template <typename T>
struct BlockMultiArgs {
  int nitems, colour;
  uint32_t begin[kBlockMultiItems + 1];  // first work-group of each item; begin[nitems] = total
  BlockMultiItem<T> it[kBlockMultiItems];
};
template <typename T>
hipError_t launch_block_pass_multi(const BlockPassItem<T>* items, int n, int colour, bool noise,
                                   int tile, hipStream_t s);
// Colours c_first, then c_first ^ 1, of several levels in as few launches as possible (items
// grouped by rows per work-group); every item must satisfy pair_level (hipErrorNotSupported
// otherwise, before any launch).
template <typename T>
struct PairMultiItem {
  T* x;
  const T* b;
  const T* s1d;
  const T* zt;
  const T* bfac;
  const T* zn;
  int nx, ny, nz;
  uint32_t N;
  int nby2, nbzc, ngx, TP;
};
template <typename T>
struct PairMultiArgs {
  int nitems, c_first;
  uint32_t begin[kBlockMultiItems + 1];
  PairMultiItem<T> it[kBlockMultiItems];
};
template <typename T>
hipError_t launch_block_pair_multi(const BlockPassItem<T>* items, int n, int c_first,
                                   bool noise, hipStream_t s);
template <typename T>
hipError_t launch_level_noise(const NoiseGenArgs& a, const NoiseArgs& na, hipStream_t s);
// `a` points to a BotArgs in device memory; the launch runs components c0 .. c0+ncomp-1 (one
// work-group each; the noise is keyed by those absolute component numbers)
template <typename T>
hipError_t launch_bottom(const BotArgs* a, int ncomp, int c0, size_t lds, bool noise,
                         const NoiseArgs& na, hipStream_t s);
// The bottoms of several hierarchies in one launch (kernel arguments only): item i brings its
// device BotArgs and its noise keys; work-group w runs component wg[w] >> 16 of item
// wg[w] & 0xffff.  lds: the largest bottom LDS size of the items.
constexpr int kBotMultiItems = 16;
constexpr int kBotMultiWG = 256;
struct BotMultiItem {
  const BotArgs* args;
  uint32_t k0, k1, c2, c3;   // as NoiseArgs
  const ChainKey* chains;
  uint32_t cpc, cpc_magic;
  double sqkT;
};
struct BotMultiArgs {
  BoxMullerCoef bm;
  int nitems;
  BotMultiItem it[kBotMultiItems];
  uint32_t wg[kBotMultiWG];
};
template <typename T>
hipError_t launch_bottom_multi(const BotMultiArgs& m, int nwg, size_t lds, bool noise,
                               hipStream_t s);
// x = A_c^-1 b (+ sqrt(kT) L_c^-T n), FP64 arithmetic, T storage
template <typename T>
hipError_t launch_coarsest(T* x, const T* b, const double* ainv, const double* w, int n,
                           int ncomp, bool noise, const NoiseArgs& na, hipStream_t s);
template <typename T>
hipError_t launch_zero(T* p, int64_t n, hipStream_t s);

hipError_t launch_residual7_nat(double* r, const double* x, const double* b, int nx, int ny,
                                int nz, int ncomp, double h, hipStream_t s);
hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s);
hipError_t launch_to_split(double* xr, double* xb, const double* nat, int nx, int ny, int nz,
                           int ncomp, hipStream_t s);
hipError_t launch_from_split(void* nat, int out_f32, const double* xr, const double* xb, int nx,
                             int ny, int nz, int ncomp, hipStream_t s);
hipError_t launch_cast(void* dst, int out_f32, const double* src, int64_t n, hipStream_t s);
// sums of squares per component of v[ncomp][n] into out[ncomp] (fixed reduction order)
hipError_t launch_sumsq(double* out, double* part, const double* v, int64_t n, int ncomp,
                        hipStream_t s);

// second stage of a fixed-order sum: out[comp] = sum of part[comp][0..nparts)
hipError_t launch_sumsq_final_parts(double* out, const double* part, uint32_t nparts, int ncomp,
                                    hipStream_t s);

// FP32-refined bridge on level 0 (split storage, colour 1 starting ncomp_stride*N/2 after
// colour 0), over the first ncomp components:
//   r32 = (float)(b64 - A x64)   (b64 null = 0); with `norm` non-null also
//   norm[comp] = ||b64 - A x64||_2^2 (fixed order, via `part`: ncomp * 2*ceil(N/512) doubles)
hipError_t launch_refine_residual(float* r32, const double* x64, const double* b64, int nx,
                                  int ny, int nz, int ncomp, int ncomp_stride, double h,
                                  double* part, double* norm, hipStream_t s);
//   x64 += (double)e32 over n elements (both colour arrays)
hipError_t launch_refine_update(double* x64, const float* e32, int64_t n, hipStream_t s);
//   x64 += (double)e32, then e32 = 0, over the spans [0, n) and [stride, stride + n) (the two
//   colour arrays of a component range), in one launch
hipError_t launch_refine_out(double* x64, float* e32, int64_t n, int64_t stride, hipStream_t s);

// Chain table of batched runs: dst[first .. first+count) = keys; advance adds `cycles` to the
// first cycle of chains 0..n-1 (so that a replayed launch sequence continues the chains).
constexpr int kChainsPerLaunch = 32;
struct ChainKeyBatch {
  int first, count;
  ChainKey k[kChainsPerLaunch];
};
hipError_t launch_set_chains(ChainKey* dst, const ChainKeyBatch& b, hipStream_t s);
hipError_t launch_advance_chains(ChainKey* dst, int n, uint64_t cycles, hipStream_t s);

// Statistics of one emitted sample of level 0 (FP64 state), fused with its emission.
constexpr int kMaxModes = 32;
constexpr int STATS_CPT = 2;                            // cells per thread and batch
constexpr int STATS_NB = 8;                             // batches per thread
constexpr int STATS_CELLS = STATS_NB * STATS_CPT * 256;  // cells per work-group
struct StatsArgs {
  const double* xr;   // split layout: colour-0 half [ncomp][N/2]; natural layout: [ncomp][N]
  const double* xb;   // split layout: colour-1 half; null for the natural layout
  int nx, ny, nz;
  int lgx, lgy;       // log2 of nx and ny when powers of two, else -1
  int nmodes;         // 0..kMaxModes projections (with obs)
  int nblk;           // work-groups per component: ceil(N / STATS_CELLS)
  const double* tx;   // [kMaxModes][nx]: x factor e_a(x) of each mode
  const double* trow; // [ny*nz][KB]: row factor e_b(y) w_m(z) of each mode, KB = 8 when
                      // nmodes <= 8 else kMaxModes
  void* out;          // [ncomp][N] natural emission (float or double) or null
  int out_f32;
  double* m1;         // [ncomp][N] running sum of x and of x^2, or null
  double* m2;
  double* part;       // [ncomp][nblk][nmodes + 1] partial sums
};
// obs (null: moments / emission only): [ncomp][nmodes + 1], the last entry escale * sum of
// squared face differences (wall faces against the antisymmetric ghost).
hipError_t launch_stats(const StatsArgs& a, int ncomp, double* obs, double escale, hipStream_t s);

}  // namespace smg
