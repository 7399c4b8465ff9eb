// Internal host-side structures of the stochastic multigrid library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/smg.h"
#include "kernels.hpp"

namespace smg {

constexpr int STENCIL = 125;  // 5x5x5 offsets of a Galerkin operator row
constexpr int kMaxChains = 255;  // batched chains per hierarchy (at most one per component)
constexpr int kMaxStreamGroups = 2;  // stream groups of a sampling call

struct Level {
  int nx = 0, ny = 0, nz = 0;
  int64_t n = 0;
  int kind = KIND_POINT;
  bool coarsest = false;
  // 1D factors of A^(l) = a_z (x) m_y (x) m_x + m_z (x) a_y (x) m_x + m_z (x) m_y (x) a_x
  double ax[5] = {0}, mx[5] = {0}, ay[5] = {0}, my[5] = {0};  // periodic stencils, offsets -2..2
  std::vector<double> az, mz;                                 // dense nz x nz (walls)
  std::vector<double> coef;  // KIND_BLOCK: [nz][125] row coefficients, index (dz+2)*25+(dy+2)*5+(dx+2)
  // The device kernels use the factored form of the same rows:
  //   coef[k][dz][dy][dx] = zt[k][dz] my[dy] mx[dx] + zt[k][5+dz] (ay[dy] mx[dx] + my[dy] ax[dx])
  // with zt[k] = (a_z[k][k+dz], m_z[k][k+dz]) and the uniform 1D stencils s1d = (mx, ax, my, ay).
  std::vector<double> s1d;   // KIND_BLOCK: [4][5]
  std::vector<double> zt;    // KIND_BLOCK: [nz][10]
  std::vector<double> bfac;  // KIND_BLOCK: [nz/2][3][64]: A_BB^-1, L_BB^-T, A_BB (row-major)
  // workspace offsets (bytes); level 0 of KIND_POINT stores x and b split by colour
  // Workspace offsets (bytes).  FP64 mode: x, b, r and the tables and noise in double.
  // FP32-refined mode: level 0 keeps x (the FP64 state) and b (the FP64 right-hand side), and
  // every level has FP32 fields xf, bf, rf (level 0: xf = correction e, bf = FP32 residual,
  // both split by colour), FP32 tables and FP32 noise.
  size_t off_x = 0, off_b = 0, off_r = 0, off_xf = 0, off_bf = 0, off_rf = 0;
  size_t off_s1d = 0, off_zt = 0, off_bfac = 0, off_noise = 0;
  double* x = nullptr;
  double* b = nullptr;
  double* r = nullptr;
  float* xf = nullptr;
  float* bf = nullptr;
  float* rf = nullptr;
  void* s1d_d = nullptr;    // T tables of the sweep precision
  void* zt_d = nullptr;
  void* bfac_d = nullptr;
  void* noise_d = nullptr;  // KIND_BLOCK: pregenerated noise [nu1+nu2][ncomp][n] of one cycle
};

struct Hierarchy {
  uint64_t uid = 0;              // unique per created hierarchy (never reused in a process)
  smg_grid_desc desc{};
  smg_cycle_params prm{};
  std::vector<Level> lv;
  int bottom = -1;               // first level handled by the LDS-resident bottom kernel
  size_t bottom_lds = 0;         // its LDS bytes
  bool use_bottom = true;        // false: run those levels with one launch per pass instead
  int block_tile = SMG_TILE_AUTO;  // tile shape of the block-pass launches
  bool block_pairs = true;         // two block colours per launch where the level allows
  // sampling calls: component groups on streams of their own (1: the caller's stream only)
  int stream_groups = 1;
  std::vector<hipStream_t> side;     // one side stream per group (made on first use)
  std::vector<hipEvent_t> ev_join;   // one per side stream
  std::vector<hipEvent_t> ev_mid;    // group i at the end of its down-leg
  hipEvent_t ev_fork = nullptr;
  int side_device = -1;
  size_t off_botargs = 0;
  BotArgs* botargs_d = nullptr;  // device copy of the bottom kernel's level descriptors
  int nc = 0;                    // unknowns of the coarsest level when it is drawn exactly
  std::vector<double> ainv, w;   // coarsest A_c^-1 and W = L_c^-1 (row-major, n_c x n_c)
  size_t off_ainv = 0, off_w = 0, off_part = 0, off_norm = 0;
  // statistics of emitted samples: mode tables [kMaxModes][nx + ny*nz] and partial
  // sums [ncomp][stats_nblk][kMaxModes + 1], stats_nblk = ceil(N / STATS_CELLS)
  size_t off_mtab = 0, off_spart = 0;
  int stats_nblk = 1;
  std::vector<int32_t> modes_loaded;  // modes whose tables are on the device
  bool modes_valid = false;
  // batched chains: device table of (seed, first cycle) per chain
  size_t off_chains = 0;
  ChainKey* chains_d = nullptr;
  int chains_set = 0, chains_cpc = 0;  // shape of the table last written
  size_t part_len = 0;
  size_t ws_bytes = 0;
  double* ainv_d = nullptr;
  double* w_d = nullptr;
  double* part_d = nullptr;      // partial sums of squares [ncomp][part_len]
  double* norm_d = nullptr;      // [2][ncomp]
  char* ws = nullptr;
  int device = -1;
  // kernel timing: events around every launch of one kernel class (SMG_TIMED_*)
  bool timing = false;
  int timed_kernel = 0;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_launches;  // launches bracketed by each event pair
  size_t ev_used = 0;
  int64_t tcount = 0;
  double tms = 0.0;
};

// plan.cpp
int build_plan(const smg_grid_desc& d, const smg_cycle_params& p, Hierarchy& h, std::string& err);
// 1D Galerkin pieces and dense factors (plan.cpp), shared by the other planners:
// the periodic-axis Galerkin step of a 5-entry stencil; the dense wall-axis prolongation
// (2nc x nc, the ghost beyond a wall is -c); P^T M P; in-place lower Cholesky (false if not
// positive definite); W = L^-1; A^-1 = W^T W.
void coarsen_stencil(const double s[5], double out[5]);
std::vector<double> prolong_wall(int nc);
std::vector<double> galerkin_dense(const std::vector<double>& M, const std::vector<double>& P,
                                   int nf, int nc);
bool cholesky(std::vector<double>& A, int n);
std::vector<double> lower_inverse(const std::vector<double>& L, int n);
std::vector<double> inverse_from_w(const std::vector<double>& W, int n);
// dense folded periodic matrix of a 5-entry stencil on an extent-n ring
std::vector<double> ring_matrix(const double s[5], int n);

// error helpers (capi.cpp)
void set_error(const std::string& msg);

// Destroys the hierarchy's side streams and their events.
inline void release_side_streams(Hierarchy& h) {
  for (hipStream_t st : h.side) (void)hipStreamDestroy(st);
  for (hipEvent_t e : h.ev_join) (void)hipEventDestroy(e);
  for (hipEvent_t e : h.ev_mid) (void)hipEventDestroy(e);
  if (h.ev_fork) (void)hipEventDestroy(h.ev_fork);
  h.side.clear();
  h.ev_join.clear();
  h.ev_mid.clear();
  h.ev_fork = nullptr;
  h.side_device = -1;
}

// capi.cpp: point (and with `upload` fill) the hierarchy's device fields and tables at ws;
// the sampling path of smg_sample_field (with at most `groups` stream groups)
int bind_impl(Hierarchy& h, char* ws, bool upload, hipStream_t s);
int sample_field_impl(smg_hierarchy* hh, int64_t n, uint64_t seed, uint64_t first_cycle,
                      void* state, void* out, int32_t out_dtype, void* stream, int groups);

}  // namespace smg

// The opaque handle of the C-ABI.
struct smg_hierarchy {
  smg::Hierarchy h;
};
