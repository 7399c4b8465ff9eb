// Hierarchy planning and the Galerkin coarse operators, built on the host.
//
// The fine operator A = -L (cell-centred 7-point Laplacian, periodic x/y, no-slip walls
// on the z faces through an antisymmetric ghost) is a Kronecker sum of 1D operators.
// The prolongation P = Pz (x) Py (x) Px is trilinear interpolation on cell centres and the
// restriction its transpose (Sec. "Stochastic Multigrid Methods", eq.
// restr_prolong_variation), so every Galerkin operator A^(l+1) = P^T A^(l) P keeps the form
//   A^(l) = a_z (x) m_y (x) m_x + m_z (x) a_y (x) m_x + m_z (x) m_y (x) a_x
// with the 1D recurrences a <- P^T a P and m <- P^T m P (m = I on the fine level).  On the
// periodic axes these are stencils on the infinite lattice (folded by modular indexing
// when the extent is small); on the wall axis they are dense nz x nz matrices.
#include <cmath>
#include <cstring>
#include <list>
#include <memory>
#include <mutex>

#include "smg_internal.hpp"

namespace smg {
namespace {

// 1D prolongation weights for the fine cells 2J-1, 2J, 2J+1, 2J+2 around coarse cell J.
const double kPW[4] = {0.25, 0.75, 0.75, 0.25};

bool can_smooth(int l, int nx, int ny, int nz) {
  if (l == 0) return nx % 2 == 0 && ny % 2 == 0;
  return nx % 4 == 0 && ny % 4 == 0 && nz % 2 == 0;
}

}  // namespace

// s'[D] = sum_{u,v in -1..2} p[u] p[v] s[2D + v - u]  (periodic-axis Galerkin step)
void coarsen_stencil(const double s[5], double out[5]) {
  for (int D = -2; D <= 2; ++D) {
    double acc = 0.0;
    for (int u = -1; u <= 2; ++u)
      for (int v = -1; v <= 2; ++v) {
        int k = 2 * D + v - u;
        if (k >= -2 && k <= 2) acc += kPW[u + 1] * kPW[v + 1] * s[k + 2];
      }
    out[D + 2] = acc;
  }
  // the coarse stencil is symmetric; make it so to the last bit (the block kernels rely on it)
  out[3] = out[1];
  out[4] = out[0];
}

// Dense wall-axis prolongation (2nc x nc, row-major); the ghost beyond a wall is -c_J.
std::vector<double> prolong_wall(int nc) {
  int nf = 2 * nc;
  std::vector<double> P((size_t)nf * nc, 0.0);
  for (int J = 0; J < nc; ++J) {
    for (int t = 0; t < 2; ++t) {
      int i = 2 * J + t;
      int other = t == 0 ? J - 1 : J + 1;
      P[(size_t)i * nc + J] += 0.75;
      if (other >= 0 && other < nc) P[(size_t)i * nc + other] += 0.25;
      else P[(size_t)i * nc + J] -= 0.25;
    }
  }
  return P;
}

// P^T M P for dense M (nf x nf) and P (nf x nc).
std::vector<double> galerkin_dense(const std::vector<double>& M, const std::vector<double>& P,
                                   int nf, int nc) {
  std::vector<double> MP((size_t)nf * nc, 0.0), out((size_t)nc * nc, 0.0);
  for (int i = 0; i < nf; ++i)
    for (int k = 0; k < nf; ++k) {
      double m = M[(size_t)i * nf + k];
      if (m == 0.0) continue;
      for (int j = 0; j < nc; ++j) MP[(size_t)i * nc + j] += m * P[(size_t)k * nc + j];
    }
  for (int i = 0; i < nf; ++i)
    for (int a = 0; a < nc; ++a) {
      double p = P[(size_t)i * nc + a];
      if (p == 0.0) continue;
      for (int j = 0; j < nc; ++j) out[(size_t)a * nc + j] += p * MP[(size_t)i * nc + j];
    }
  return out;
}

// In-place lower Cholesky of a dense SPD matrix (row-major); false if not positive definite.
bool cholesky(std::vector<double>& A, int n) {
  for (int j = 0; j < n; ++j) {
    double d = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    A[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = A[(size_t)i * n + j];
      const double* ri = &A[(size_t)i * n];
      const double* rj = &A[(size_t)j * n];
      for (int k = 0; k < j; ++k) s -= ri[k] * rj[k];
      A[(size_t)i * n + j] = s / d;
    }
    for (int k = j + 1; k < n; ++k) A[(size_t)j * n + k] = 0.0;
  }
  return true;
}

// W = L^-1 for lower-triangular L (row-major).
std::vector<double> lower_inverse(const std::vector<double>& L, int n) {
  std::vector<double> W((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c) {
    W[(size_t)c * n + c] = 1.0 / L[(size_t)c * n + c];
    for (int i = c + 1; i < n; ++i) {
      double s = 0.0;
      for (int k = c; k < i; ++k) s += L[(size_t)i * n + k] * W[(size_t)k * n + c];
      W[(size_t)i * n + c] = -s / L[(size_t)i * n + i];
    }
  }
  return W;
}

// A^-1 = W^T W (W lower triangular).
std::vector<double> inverse_from_w(const std::vector<double>& W, int n) {
  std::vector<double> Ai((size_t)n * n, 0.0);
  for (int k = 0; k < n; ++k) {
    const double* wk = &W[(size_t)k * n];
    for (int i = 0; i <= k; ++i) {
      double a = wk[i];
      if (a == 0.0) continue;
      double* row = &Ai[(size_t)i * n];
      for (int j = 0; j <= k; ++j) row[j] += a * wk[j];
    }
  }
  return Ai;
}

// Dense folded periodic matrix of a stencil on an extent-n ring.
std::vector<double> ring_matrix(const double s[5], int n) {
  std::vector<double> M((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int d = -2; d <= 2; ++d) M[(size_t)i * n + (((i + d) % n) + n) % n] += s[d + 2];
  return M;
}

namespace {

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

constexpr int64_t kBottomCells = 4096;
constexpr size_t kBottomLdsMax = 160 * 1024;
constexpr int kBottomLevelsMax = 6;

// The dense factors of the coarsest level depend only on the finest grid, h and the depth (the
// Galerkin recurrences are fixed by them), not on the component count, the sweeps or the
// precision.  A small process-wide cache keeps the last few, so that plans of one shape that
// differ only in those (an autotuner's candidates) factor the coarsest level once: at 1728
// unknowns the factorisation and the two inverses take seconds on the host.
struct CoarsestKey {
  int nx, ny, nz, levels;
  double h;
  bool operator==(const CoarsestKey& o) const {
    return nx == o.nx && ny == o.ny && nz == o.nz && levels == o.levels && h == o.h;
  }
};
struct CoarsestFactors {
  std::vector<double> w, ainv;
};
constexpr size_t kCoarsestCacheEntries = 4;
std::mutex g_coarsest_mu;
std::list<std::pair<CoarsestKey, std::shared_ptr<const CoarsestFactors>>> g_coarsest;

std::shared_ptr<const CoarsestFactors> cached_coarsest(const CoarsestKey& k) {
  std::lock_guard<std::mutex> lk(g_coarsest_mu);
  for (auto it = g_coarsest.begin(); it != g_coarsest.end(); ++it)
    if (it->first == k) {
      g_coarsest.splice(g_coarsest.begin(), g_coarsest, it);  // most recent first
      return g_coarsest.front().second;
    }
  return nullptr;
}

void store_coarsest(const CoarsestKey& k, const std::vector<double>& w,
                    const std::vector<double>& ainv) {
  auto f = std::make_shared<CoarsestFactors>();
  f->w = w;
  f->ainv = ainv;
  std::lock_guard<std::mutex> lk(g_coarsest_mu);
  g_coarsest.emplace_front(k, std::move(f));
  while (g_coarsest.size() > kCoarsestCacheEntries) g_coarsest.pop_back();
}

}  // namespace

int build_plan(const smg_grid_desc& d, const smg_cycle_params& p, Hierarchy& h, std::string& err) {
  if (d.nx <= 0 || d.ny <= 0 || d.nz <= 0 || d.nx % 2 || d.ny % 2) {
    err = "nx, ny must be positive and even, nz positive";
    return SMG_EINVAL;
  }
  if (d.ncomp < 1 || d.ncomp > 255 || !(d.h > 0.0) || !(d.kT >= 0.0)) {
    err = "ncomp must be in [1,255], h > 0, kT >= 0";
    return SMG_EINVAL;
  }
  {
    auto is = [](int32_t bc, int32_t want) { return bc == SMG_BC_DEFAULT || bc == want; };
    if (!is(d.bc_x, SMG_BC_PERIODIC) || !is(d.bc_y, SMG_BC_PERIODIC) ||
        !is(d.bc_z, SMG_BC_DIRICHLET_FACE)) {
      err = "boundary conditions: only periodic x and y with Dirichlet-face (no-slip) walls "
            "in z are implemented";
      return SMG_EINVAL;
    }
  }
  if (p.levels < 0 || p.levels > 15 || p.nu1 < 0 || p.nu2 < 0 || p.nu1 + p.nu2 > 255 ||
      p.stride < 1 || p.burn_in < 0 || p.coarsest_max < 1 || p.coarsest_max > 4096 ||
      (p.coarsest_mode != SMG_COARSEST_CHOLESKY && p.coarsest_mode != SMG_COARSEST_SMOOTH) ||
      (p.precision != SMG_FP64 && p.precision != SMG_FP32_REFINED)) {
    err = "invalid cycle parameters";
    return SMG_EINVAL;
  }

  // ---- level plan
  std::vector<int> dx{d.nx}, dy{d.ny}, dz{d.nz};
  for (;;) {
    int l = (int)dx.size() - 1;
    int64_t n = (int64_t)dx[l] * dy[l] * dz[l];
    bool want = p.levels > 0 ? (int)dx.size() < p.levels : n > p.coarsest_max;
    bool halvable = dx[l] % 2 == 0 && dy[l] % 2 == 0 && dz[l] % 2 == 0;
    if (want && halvable && can_smooth(l, dx[l], dy[l], dz[l]) && dx.size() < 15) {
      dx.push_back(dx[l] / 2);
      dy.push_back(dy[l] / 2);
      dz.push_back(dz[l] / 2);
    } else {
      break;
    }
  }
  int L = (int)dx.size();
  if (p.levels > 0 && L != p.levels) {
    err = "grid cannot be coarsened to the requested number of levels";
    return SMG_EINVAL;
  }
  h.desc = d;
  h.prm = p;
  h.lv.assign(L, Level());
  const double ih2 = 1.0 / (d.h * d.h);
  for (int l = 0; l < L; ++l) {
    Level& v = h.lv[l];
    v.nx = dx[l]; v.ny = dy[l]; v.nz = dz[l];
    v.n = (int64_t)v.nx * v.ny * v.nz;
    v.coarsest = (l == L - 1);
    if (v.coarsest && p.coarsest_mode == SMG_COARSEST_CHOLESKY) v.kind = KIND_CHOL;
    else v.kind = (l == 0) ? KIND_POINT : KIND_BLOCK;
    if (v.kind != KIND_CHOL && !can_smooth(l, v.nx, v.ny, v.nz)) {
      err = "coarsest level cannot be smoothed; use SMG_COARSEST_CHOLESKY";
      return SMG_EINVAL;
    }
    // 1D factors
    if (l == 0) {
      const double a0[5] = {0.0, -ih2, 2.0 * ih2, -ih2, 0.0};
      const double m0[5] = {0.0, 0.0, 1.0, 0.0, 0.0};
      std::memcpy(v.ax, a0, sizeof a0); std::memcpy(v.ay, a0, sizeof a0);
      std::memcpy(v.mx, m0, sizeof m0); std::memcpy(v.my, m0, sizeof m0);
      v.az.assign((size_t)v.nz * v.nz, 0.0);
      v.mz.assign((size_t)v.nz * v.nz, 0.0);
      for (int k = 0; k < v.nz; ++k) {
        v.mz[(size_t)k * v.nz + k] = 1.0;
        double diag = 2.0 * ih2;
        if (k == 0) diag += ih2;            // ghost -c below the bottom wall
        if (k == v.nz - 1) diag += ih2;     // ghost -c above the top wall
        v.az[(size_t)k * v.nz + k] = diag;
        if (k > 0) v.az[(size_t)k * v.nz + k - 1] = -ih2;
        if (k < v.nz - 1) v.az[(size_t)k * v.nz + k + 1] = -ih2;
      }
    } else {
      const Level& f = h.lv[l - 1];
      coarsen_stencil(f.ax, v.ax); coarsen_stencil(f.mx, v.mx);
      coarsen_stencil(f.ay, v.ay); coarsen_stencil(f.my, v.my);
      std::vector<double> Pz = prolong_wall(v.nz);
      v.az = galerkin_dense(f.az, Pz, f.nz, v.nz);
      v.mz = galerkin_dense(f.mz, Pz, f.nz, v.nz);
    }
    if (v.kind == KIND_BLOCK) {
      v.coef.assign((size_t)v.nz * STENCIL, 0.0);
      for (int k = 0; k < v.nz; ++k)
        for (int oz = -2; oz <= 2; ++oz) {
          int kk = k + oz;
          double az = 0.0, mz = 0.0;
          if (kk >= 0 && kk < v.nz) {
            az = v.az[(size_t)k * v.nz + kk];
            mz = v.mz[(size_t)k * v.nz + kk];
          }
          for (int oy = -2; oy <= 2; ++oy)
            for (int ox = -2; ox <= 2; ++ox) {
              double c = az * v.my[oy + 2] * v.mx[ox + 2] +
                         mz * (v.ay[oy + 2] * v.mx[ox + 2] + v.my[oy + 2] * v.ax[ox + 2]);
              v.coef[(size_t)k * STENCIL + (oz + 2) * 25 + (oy + 2) * 5 + (ox + 2)] = c;
            }
        }
      v.s1d.assign(20, 0.0);
      for (int o = 0; o < 5; ++o) {
        v.s1d[o] = v.mx[o];
        v.s1d[5 + o] = v.ax[o];
        v.s1d[10 + o] = v.my[o];
        v.s1d[15 + o] = v.ay[o];
      }
      v.zt.assign((size_t)v.nz * 10, 0.0);
      for (int k = 0; k < v.nz; ++k)
        for (int oz = -2; oz <= 2; ++oz) {
          int kk = k + oz;
          if (kk < 0 || kk >= v.nz) continue;
          v.zt[(size_t)k * 10 + oz + 2] = v.az[(size_t)k * v.nz + kk];
          v.zt[(size_t)k * 10 + 5 + oz + 2] = v.mz[(size_t)k * v.nz + kk];
        }
      // exact 8-variable conditionals of the 2x2x2 blocks, one factor per block row
      int nbz = v.nz / 2;
      v.bfac.assign((size_t)nbz * 192, 0.0);
      for (int bz = 0; bz < nbz; ++bz) {
        std::vector<double> ABB(64);
        for (int i = 0; i < 8; ++i)
          for (int j = 0; j < 8; ++j) {
            int ox = (j & 1) - (i & 1), oy = ((j >> 1) & 1) - ((i >> 1) & 1),
                oz = (j >> 2) - (i >> 2);
            int zi = 2 * bz + (i >> 2);
            ABB[i * 8 + j] = v.coef[(size_t)zi * STENCIL + (oz + 2) * 25 + (oy + 2) * 5 + (ox + 2)];
          }
        double* dst = &v.bfac[(size_t)bz * 192];
        for (int i = 0; i < 64; ++i) dst[128 + i] = ABB[i];
        if (!cholesky(ABB, 8)) {
          err = "block operator not positive definite";
          return SMG_EINVAL;
        }
        std::vector<double> W = lower_inverse(ABB, 8);
        std::vector<double> Ai = inverse_from_w(W, 8);
        for (int i = 0; i < 8; ++i)
          for (int j = 0; j < 8; ++j) {
            dst[i * 8 + j] = Ai[i * 8 + j];
            dst[64 + i * 8 + j] = W[j * 8 + i];  // L^-T
          }
      }
    }
    if (v.kind == KIND_CHOL) {
      if (v.n > 4096) {
        err = "coarsest level has more than 4096 unknowns (dense factor limit)";
        return SMG_EINVAL;
      }
      int n = (int)v.n;
      const CoarsestKey key{d.nx, d.ny, d.nz, L, d.h};
      if (std::shared_ptr<const CoarsestFactors> cf = cached_coarsest(key)) {
        h.w = cf->w;
        h.ainv = cf->ainv;
        h.nc = n;
        continue;
      }
      std::vector<double> MX = ring_matrix(v.mx, v.nx), AX = ring_matrix(v.ax, v.nx);
      std::vector<double> MY = ring_matrix(v.my, v.ny), AY = ring_matrix(v.ay, v.ny);
      std::vector<double> A((size_t)n * n, 0.0);
      for (int z = 0; z < v.nz; ++z)
        for (int y = 0; y < v.ny; ++y)
          for (int x = 0; x < v.nx; ++x) {
            size_t i = x + (size_t)v.nx * (y + (size_t)v.ny * z);
            for (int z2 = 0; z2 < v.nz; ++z2) {
              double az = v.az[(size_t)z * v.nz + z2], mz = v.mz[(size_t)z * v.nz + z2];
              if (az == 0.0 && mz == 0.0) continue;
              for (int y2 = 0; y2 < v.ny; ++y2) {
                double my = MY[(size_t)y * v.ny + y2], ay = AY[(size_t)y * v.ny + y2];
                for (int x2 = 0; x2 < v.nx; ++x2) {
                  double mx = MX[(size_t)x * v.nx + x2], ax = AX[(size_t)x * v.nx + x2];
                  size_t j = x2 + (size_t)v.nx * (y2 + (size_t)v.ny * z2);
                  A[i * n + j] += az * my * mx + mz * (ay * mx + my * ax);
                }
              }
            }
          }
      if (!cholesky(A, n)) {
        err = "coarsest operator not positive definite";
        return SMG_EINVAL;
      }
      h.w = lower_inverse(A, n);
      h.ainv = inverse_from_w(h.w, n);
      h.nc = n;
      store_coarsest(key, h.w, h.ainv);
    }
  }
  // ---- workspace layout
  const bool f32 = p.precision == SMG_FP32_REFINED;
  if (f32 && h.lv[0].kind != KIND_POINT) {
    err = "SMG_FP32_REFINED needs a smoothed finest level (use SMG_FP64 for one-level Cholesky)";
    return SMG_EINVAL;
  }
  const size_t ts = f32 ? sizeof(float) : sizeof(double);  // sweep element size
  const int nc = d.ncomp;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  for (int l = 0; l < L; ++l) {
    Level& v = h.lv[l];
    const size_t n = (size_t)nc * v.n;
    if (!f32) {
      v.off_x = take(n * sizeof(double));
      v.off_b = take(n * sizeof(double));
      // level 0 always has a residual buffer (the solve's norms); a drawn-exact level 0 (one
      // level) needs it for nothing else
      if (v.kind != KIND_CHOL || l == 0) v.off_r = take(n * sizeof(double));
    } else {
      if (l == 0) {
        v.off_x = take(n * sizeof(double));
        v.off_b = take(n * sizeof(double));
      }
      v.off_xf = take(n * sizeof(float));
      v.off_bf = take(n * sizeof(float));
      if (v.kind != KIND_CHOL) v.off_rf = take(n * sizeof(float));
    }
    if (v.kind == KIND_BLOCK) {
      v.off_s1d = take(v.s1d.size() * ts);
      v.off_zt = take(v.zt.size() * ts);
      v.off_bfac = take(v.bfac.size() * ts);
      v.off_noise = take((size_t)(p.nu1 + p.nu2) * n * ts);
    }
  }
  // Bottom of the V-cycle: the first Galerkin level with at most kBottomCells cells and every
  // level below it live in one work-group's LDS per component (x, b and one scratch field per
  // level; the coarsest draw stages b and the noise).
  for (int l = 1; l < L; ++l) {
    if (h.lv[l].n > kBottomCells) continue;
    size_t lds = 0;
    for (int m = l; m < L; ++m) {
      const Level& v = h.lv[m];
      lds += 3 * bot_field_elems(v.kind, v.nx, v.ny, v.nz) * ts;
      if (v.kind == KIND_BLOCK) lds += ((size_t)v.nz * 10 + (size_t)(v.nz / 2) * 192) * ts;
    }
    if (lds <= kBottomLdsMax && L - l <= kBottomLevelsMax) {
      h.bottom = l;
      h.bottom_lds = lds;
    }
    break;
  }
  if (h.nc > 0) {
    h.off_ainv = take((size_t)h.nc * h.nc * sizeof(double));
    h.off_w = take((size_t)h.nc * h.nc * sizeof(double));
  }
  if (h.bottom >= 0) h.off_botargs = take(sizeof(BotArgs));
  // partial sums for the residual norms: one per 256-cell block of level 0
  h.part_len = (size_t)((h.lv[0].n + 255) / 256) + 2;
  h.off_part = take((size_t)nc * h.part_len * sizeof(double));
  h.off_norm = take((size_t)2 * nc * sizeof(double));
  {
    const Level& v0 = h.lv[0];
    h.stats_nblk = (int)((v0.n + STATS_CELLS - 1) / STATS_CELLS);
    h.off_mtab = take((size_t)kMaxModes * (v0.nx + (size_t)v0.ny * v0.nz) * sizeof(double));
    h.off_spart = take((size_t)nc * h.stats_nblk * (kMaxModes + 1) * sizeof(double));
  }
  h.off_chains = take((size_t)kMaxChains * sizeof(ChainKey));
  h.ws_bytes = off;
  return SMG_OK;
}

}  // namespace smg
