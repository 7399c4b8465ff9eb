// C-ABI of the two-dimensional wall-bounded sampler and solver: cells (x, z) of width h on
// nx x nz, periodic in x, no-slip walls on the faces z = 0 and z = nz h (antisymmetric ghost);
// A = -L the 5-point operator.  The paper compares its multigrid sampler with stochastic
// Gauss-Seidel on two- and three-dimensional meshes (Sec. "Performance of the Stochastic
// Samplers in Practice"); this is the 2D form of the same method: red-black point heat bath on
// level 0, Galerkin levels A_{l+1} = P^T A_l P (bilinear P) with a 2 x 2 block heat bath (four
// block colours), an exact Cholesky draw (or nu1 + nu2 sweeps) on the coarsest level, V-cycles
// of Alg. 3.  Noise counters as on the 3D grid: (site pair, level | slot<<4 | colour<<12 |
// comp<<16 | kind<<24, cycle); level 0 site = (x + nx z) >> 1, block levels 4 block + in-block
// index, coarsest row.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "kernels2d.hpp"
#include "smg_internal.hpp"

namespace smg {
namespace {

struct Level2 {
  int nx = 0, nz = 0;
  int64_t n = 0;
  int kind = KIND_POINT;
  bool coarsest = false;
  double mx[5] = {0}, ax[5] = {0};
  std::vector<double> az, mz;     // dense nz x nz wall-axis pieces
  std::vector<double> s1d, zt;    // (m_x, a_x); per-row bands [nz][10]
  std::vector<double> bfac;       // [nz/2][32]
  size_t off_x = 0, off_b = 0, off_r = 0, off_s1d = 0, off_zt = 0, off_bfac = 0;
  double* x = nullptr;
  double* b = nullptr;
  double* r = nullptr;
  Lev2 dev{};
};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

bool smooths(int l, int nx, int nz) { return l == 0 ? nx % 2 == 0 : (nx % 4 == 0 && nz % 2 == 0); }

}  // namespace
}  // namespace smg

struct smg2d {
  smg2d_desc d{};
  std::vector<smg::Level2> lv;
  int nc = 0;
  std::vector<double> ainv, w;
  size_t off_ainv = 0, off_w = 0, off_part = 0, off_norm = 0, part_len = 0, ws_bytes = 0;
  double* ainv_d = nullptr;
  double* w_d = nullptr;
  double* part_d = nullptr;
  double* norm_d = nullptr;
  char* ws = nullptr;
};

namespace smg {
namespace {

#define S2_HIP(call)                                                               \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));                \
      return SMG_EHIP;                                                             \
    }                                                                              \
  } while (0)

#define S2_TRY(expr)               \
  do {                             \
    int rc_ = (expr);              \
    if (rc_ != SMG_OK) return rc_; \
  } while (0)

int plan2d(smg2d& h, std::string& err) {
  const smg2d_desc& d = h.d;
  if (d.nx < 2 || d.nx % 2 || d.nz < 1 || d.ncomp < 1 || d.ncomp > 255 || !(d.h > 0.0) ||
      !(d.kT >= 0.0)) {
    err = "nx must be even, nz >= 1, ncomp in [1, 255], h > 0, kT >= 0";
    return SMG_EINVAL;
  }
  if (d.levels < 0 || d.levels > 15 || d.nu1 < 0 || d.nu2 < 0 || d.nu1 + d.nu2 > 255 ||
      d.coarsest_max < 1 || d.coarsest_max > 4096 || d.stride < 1 ||
      (d.coarsest_mode != SMG_COARSEST_CHOLESKY && d.coarsest_mode != SMG_COARSEST_SMOOTH)) {
    err = "invalid cycle parameters";
    return SMG_EINVAL;
  }
  std::vector<int> dx{d.nx}, dz{d.nz};
  for (;;) {
    const int l = (int)dx.size() - 1;
    const bool want = d.levels > 0 ? (int)dx.size() < d.levels
                                   : (int64_t)dx[l] * dz[l] > d.coarsest_max;
    if (want && smooths(l, dx[l], dz[l]) && dx[l] % 2 == 0 && dz[l] % 2 == 0 && dx.size() < 15) {
      dx.push_back(dx[l] / 2);
      dz.push_back(dz[l] / 2);
    } else {
      break;
    }
  }
  const int L = (int)dx.size();
  if (d.levels > 0 && L != d.levels) {
    err = "grid cannot be coarsened to the requested number of levels";
    return SMG_EINVAL;
  }
  h.lv.assign(L, Level2());
  const double ih2 = 1.0 / (d.h * d.h);
  for (int l = 0; l < L; ++l) {
    Level2& v = h.lv[l];
    v.nx = dx[l];
    v.nz = dz[l];
    v.n = (int64_t)v.nx * v.nz;
    v.coarsest = l == L - 1;
    v.kind = (v.coarsest && d.coarsest_mode == SMG_COARSEST_CHOLESKY) ? KIND_CHOL
             : (l == 0 ? KIND_POINT : KIND_BLOCK);
    if (v.kind != KIND_CHOL && !smooths(l, v.nx, v.nz)) {
      err = "coarsest level cannot be smoothed; use SMG_COARSEST_CHOLESKY";
      return SMG_EINVAL;
    }
    if (l == 0) {
      const double a0[5] = {0.0, -ih2, 2.0 * ih2, -ih2, 0.0};
      const double m0[5] = {0.0, 0.0, 1.0, 0.0, 0.0};
      std::memcpy(v.ax, a0, sizeof a0);
      std::memcpy(v.mx, m0, sizeof m0);
      v.az.assign((size_t)v.nz * v.nz, 0.0);
      v.mz.assign((size_t)v.nz * v.nz, 0.0);
      for (int k = 0; k < v.nz; ++k) {
        v.mz[(size_t)k * v.nz + k] = 1.0;
        v.az[(size_t)k * v.nz + k] = 2.0 * ih2 + (k == 0 ? ih2 : 0.0) + (k == v.nz - 1 ? ih2 : 0.0);
        if (k > 0) v.az[(size_t)k * v.nz + k - 1] = -ih2;
        if (k < v.nz - 1) v.az[(size_t)k * v.nz + k + 1] = -ih2;
      }
    } else {
      const Level2& f = h.lv[l - 1];
      coarsen_stencil(f.ax, v.ax);
      coarsen_stencil(f.mx, v.mx);
      const std::vector<double> Pz = prolong_wall(v.nz);
      v.az = galerkin_dense(f.az, Pz, f.nz, v.nz);
      v.mz = galerkin_dense(f.mz, Pz, f.nz, v.nz);
    }
    v.s1d.assign(10, 0.0);
    for (int o = 0; o < 5; ++o) {
      v.s1d[o] = v.mx[o];
      v.s1d[5 + o] = v.ax[o];
    }
    v.zt.assign((size_t)v.nz * 10, 0.0);
    for (int k = 0; k < v.nz; ++k)
      for (int o = -2; o <= 2; ++o) {
        const int kk = k + o;
        if (kk < 0 || kk >= v.nz) continue;
        v.zt[(size_t)k * 10 + o + 2] = v.az[(size_t)k * v.nz + kk];
        v.zt[(size_t)k * 10 + 5 + o + 2] = v.mz[(size_t)k * v.nz + kk];
      }
    if (v.kind == KIND_BLOCK) {
      v.bfac.assign((size_t)(v.nz / 2) * 32, 0.0);
      for (int bz = 0; bz < v.nz / 2; ++bz) {
        std::vector<double> B(16);
        for (int i = 0; i < 4; ++i)
          for (int j = 0; j < 4; ++j) {
            const int zi = 2 * bz + (i >> 1), zj = 2 * bz + (j >> 1), ox = (j & 1) - (i & 1);
            B[i * 4 + j] = v.az[(size_t)zi * v.nz + zj] * v.mx[ox + 2] +
                           v.mz[(size_t)zi * v.nz + zj] * v.ax[ox + 2];
          }
        if (!cholesky(B, 4)) {
          err = "block operator not positive definite";
          return SMG_EINVAL;
        }
        const std::vector<double> W = lower_inverse(B, 4);
        const std::vector<double> Ai = inverse_from_w(W, 4);
        double* dst = &v.bfac[(size_t)bz * 32];
        for (int i = 0; i < 4; ++i)
          for (int j = 0; j < 4; ++j) {
            dst[i * 4 + j] = Ai[i * 4 + j];
            dst[16 + i * 4 + j] = W[j * 4 + i];  // L^-T
          }
      }
    }
    if (v.kind == KIND_CHOL) {
      if (v.n > 4096) {
        err = "coarsest level has more than 4096 unknowns (dense factor limit)";
        return SMG_EINVAL;
      }
      const int n = (int)v.n;
      const std::vector<double> MX = ring_matrix(v.mx, v.nx), AX = ring_matrix(v.ax, v.nx);
      std::vector<double> A((size_t)n * n, 0.0);
      for (int z = 0; z < v.nz; ++z)
        for (int x = 0; x < v.nx; ++x)
          for (int z2 = 0; z2 < v.nz; ++z2) {
            const double a = v.az[(size_t)z * v.nz + z2], m = v.mz[(size_t)z * v.nz + z2];
            if (a == 0.0 && m == 0.0) continue;
            for (int x2 = 0; x2 < v.nx; ++x2)
              A[(size_t)(x + v.nx * z) * n + x2 + v.nx * z2] +=
                  a * MX[(size_t)x * v.nx + x2] + m * AX[(size_t)x * v.nx + x2];
          }
      if (!cholesky(A, n)) {
        err = "coarsest operator not positive definite";
        return SMG_EINVAL;
      }
      h.w = lower_inverse(A, n);
      h.ainv = inverse_from_w(h.w, n);
      h.nc = n;
    }
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  for (Level2& v : h.lv) {
    const size_t n = (size_t)d.ncomp * v.n * sizeof(double);
    v.off_x = take(n);
    v.off_b = take(n);
    v.off_r = take(n);
    v.off_s1d = take(10 * sizeof(double));
    v.off_zt = take(v.zt.size() * sizeof(double));
    if (!v.bfac.empty()) v.off_bfac = take(v.bfac.size() * sizeof(double));
  }
  if (h.nc > 0) {
    h.off_ainv = take((size_t)h.nc * h.nc * sizeof(double));
    h.off_w = take((size_t)h.nc * h.nc * sizeof(double));
  }
  h.part_len = (size_t)((h.lv[0].n + 255) / 256) + 2;
  h.off_part = take((size_t)d.ncomp * h.part_len * sizeof(double));
  h.off_norm = take((size_t)2 * d.ncomp * sizeof(double));
  h.ws_bytes = off;
  return SMG_OK;
}

struct Run2 {
  smg2d* h;
  hipStream_t s;
  bool noise;
  bool has_b0;
  uint64_t seed, cycle;
};

NoiseArgs noise2(const Run2& r, int level, int slot, int colour, uint32_t kind) {
  NoiseArgs na{};
  na.k0 = (uint32_t)r.seed;
  na.k1 = (uint32_t)(r.seed >> 32);
  na.sid = (uint32_t)level | ((uint32_t)slot << 4) | ((uint32_t)colour << 12) | (kind << 24);
  na.c2 = (uint32_t)r.cycle;
  na.c3 = (uint32_t)(r.cycle >> 32);
  na.sqkT = std::sqrt(r.h->d.kT);
  na.chains = nullptr;
  na.comps_per_chain = 1;
  na.cpc_magic = 0;
  na.bm = box_muller_coef();
  return na;
}

int sweep2(Run2& r, int l, int slot, bool post) {
  smg2d& h = *r.h;
  Level2& v = h.lv[l];
  const int nc = h.d.ncomp;
  const int ncol = v.kind == KIND_POINT ? 2 : 4;
  for (int t = 0; t < ncol; ++t) {
    const int colour = post ? ncol - 1 - t : t;
    const NoiseArgs na = noise2(r, l, slot, colour, 0);
    if (v.kind == KIND_POINT)
      S2_HIP(launch2_point_pass(v.x, r.has_b0 ? v.b : nullptr, v.dev, nc, colour, h.d.kT,
                                r.noise, na, r.s));
    else
      S2_HIP(launch2_block_pass(v.x, v.b, v.dev, nc, colour, h.d.kT, r.noise, na, r.s));
  }
  return SMG_OK;
}

int vcycle2(Run2& r, int l) {
  smg2d& h = *r.h;
  Level2& v = h.lv[l];
  const int nc = h.d.ncomp;
  if (v.kind == KIND_CHOL) {
    const NoiseArgs na = noise2(r, l, 0, 0, 1);
    // level 0 drawn exactly: its b is the caller's (zero when sampling)
    S2_HIP(launch_coarsest<double>(v.x, v.b, h.ainv_d, h.w_d, h.nc, nc, r.noise, na, r.s));
    return SMG_OK;
  }
  for (int s = 0; s < h.d.nu1; ++s) S2_TRY(sweep2(r, l, s, false));
  if (!v.coarsest) {
    Level2& c = h.lv[l + 1];
    S2_HIP(launch2_residual(v.r, v.x, (l == 0 && !r.has_b0) ? nullptr : v.b, v.dev, nc, r.s));
    S2_HIP(launch2_restrict(c.b, c.x, v.r, v.nx, v.nz, nc, r.s));
    S2_TRY(vcycle2(r, l + 1));
    S2_HIP(launch2_prolong(v.x, c.x, v.nx, v.nz, nc, r.s));
  }
  for (int s = 0; s < h.d.nu2; ++s) S2_TRY(sweep2(r, l, h.d.nu1 + s, true));
  return SMG_OK;
}

int check2(const smg2d* h) {
  if (!h) {
    set_error("null 2D hierarchy");
    return SMG_EINVAL;
  }
  if (!h->ws) {
    set_error("2D hierarchy has no workspace bound (call smg2d_bind)");
    return SMG_ESTATE;
  }
  return SMG_OK;
}

bool al256(const void* p) { return p && ((uintptr_t)p & 255u) == 0; }

}  // namespace
}  // namespace smg

using namespace smg;

extern "C" {

int smg2d_create(const smg2d_desc* desc, smg2d** out) {
  if (!desc || !out) {
    set_error("null argument");
    return SMG_EINVAL;
  }
  *out = nullptr;
  smg2d* h = new (std::nothrow) smg2d();
  if (!h) {
    set_error("host allocation failed");
    return SMG_ENOMEM;
  }
  h->d = *desc;
  std::string err;
  const int rc = plan2d(*h, err);
  if (rc != SMG_OK) {
    set_error(err);
    delete h;
    return rc;
  }
  *out = h;
  return SMG_OK;
}

int smg2d_get_info(const smg2d* h, smg2d_info* info) {
  if (!h || !info) {
    set_error("null argument");
    return SMG_EINVAL;
  }
  std::memset(info, 0, sizeof(*info));
  info->workspace_bytes = h->ws_bytes;
  info->n_levels = (int32_t)h->lv.size();
  for (size_t l = 0; l < h->lv.size() && l < 16; ++l) {
    info->dims[l][0] = h->lv[l].nx;
    info->dims[l][1] = h->lv[l].nz;
  }
  return SMG_OK;
}

int smg2d_bind(smg2d* h, void* ws, size_t bytes, void* stream) {
  if (!h) {
    set_error("null 2D hierarchy");
    return SMG_EINVAL;
  }
  if (!al256(ws)) {
    set_error("workspace must be a non-null 256-byte aligned device pointer");
    return SMG_EINVAL;
  }
  if (bytes < h->ws_bytes) {
    set_error("workspace too small: need " + std::to_string(h->ws_bytes) + " bytes");
    return SMG_ENOMEM;
  }
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)ws;
  for (Level2& v : h->lv) {
    v.x = (double*)(base + v.off_x);
    v.b = (double*)(base + v.off_b);
    v.r = (double*)(base + v.off_r);
    v.dev.nx = v.nx;
    v.dev.nz = v.nz;
    v.dev.s1d = (const double*)(base + v.off_s1d);
    v.dev.zt = (const double*)(base + v.off_zt);
    v.dev.bfac = v.bfac.empty() ? nullptr : (const double*)(base + v.off_bfac);
    S2_HIP(hipMemcpyAsync(base + v.off_s1d, v.s1d.data(), 10 * sizeof(double),
                          hipMemcpyHostToDevice, s));
    S2_HIP(hipMemcpyAsync(base + v.off_zt, v.zt.data(), v.zt.size() * sizeof(double),
                          hipMemcpyHostToDevice, s));
    if (!v.bfac.empty())
      S2_HIP(hipMemcpyAsync(base + v.off_bfac, v.bfac.data(), v.bfac.size() * sizeof(double),
                            hipMemcpyHostToDevice, s));
  }
  if (h->nc > 0) {
    h->ainv_d = (double*)(base + h->off_ainv);
    h->w_d = (double*)(base + h->off_w);
    S2_HIP(hipMemcpyAsync(h->ainv_d, h->ainv.data(), h->ainv.size() * sizeof(double),
                          hipMemcpyHostToDevice, s));
    S2_HIP(hipMemcpyAsync(h->w_d, h->w.data(), h->w.size() * sizeof(double),
                          hipMemcpyHostToDevice, s));
  }
  h->part_d = (double*)(base + h->off_part);
  h->norm_d = (double*)(base + h->off_norm);
  S2_HIP(hipStreamSynchronize(s));
  h->ws = base;
  return SMG_OK;
}

int smg2d_sample(smg2d* h, int64_t n, uint64_t seed, uint64_t first_cycle, void* state,
                 void* out, void* stream) {
  S2_TRY(check2(h));
  if (n < 0 || !al256(state) || (n > 0 && !al256(out))) {
    set_error("n >= 0 with 256-byte aligned state (and out when n > 0) required");
    return SMG_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  Level2& v0 = h->lv[0];
  const int64_t field = (int64_t)h->d.ncomp * v0.n;
  S2_HIP(launch_copy(v0.x, (const double*)state, field, s));
  if (v0.kind == KIND_CHOL) S2_HIP(launch_zero<double>(v0.b, field, s));
  Run2 r{h, s, h->d.kT > 0.0, false, seed, first_cycle};
  int64_t k = 0;
  for (int64_t i = 0; i < n; ++i) {
    for (int t = 0; t < h->d.stride; ++t, ++k) {
      r.cycle = first_cycle + (uint64_t)k;
      S2_TRY(vcycle2(r, 0));
    }
    S2_HIP(launch_copy((double*)out + i * field, v0.x, field, s));
  }
  S2_HIP(launch_copy((double*)state, v0.x, field, s));
  return SMG_OK;
}

int smg2d_solve(smg2d* h, const void* f, void* u, double rtol, int32_t max_cycles, void* stream,
                smg_solve_info* info) {
  S2_TRY(check2(h));
  if (!al256(f) || !al256(u) || !(rtol >= 0.0) || max_cycles < 0) {
    set_error("aligned f, u, rtol >= 0 and max_cycles >= 0 required");
    return SMG_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  Level2& v0 = h->lv[0];
  const int nc = h->d.ncomp;
  const int64_t field = (int64_t)nc * v0.n;
  std::vector<double> fn(nc), rn(nc), rprev(nc, 0.0);
  S2_HIP(launch_sumsq(h->norm_d, h->part_d, (const double*)f, v0.n, nc, s));
  S2_HIP(hipMemcpyAsync(fn.data(), h->norm_d, nc * sizeof(double), hipMemcpyDeviceToHost, s));
  S2_HIP(hipStreamSynchronize(s));
  S2_HIP(launch_copy(v0.b, (const double*)f, field, s));
  S2_HIP(launch_zero<double>(v0.x, field, s));
  Run2 r{h, s, false, true, 0, 0};
  int cycles = 0;
  double relres = 0.0, ratio = 0.0;
  bool zero_f = true;
  for (double v : fn) zero_f = zero_f && v == 0.0;
  if (!zero_f) relres = 1.0;
  while (!zero_f && cycles < max_cycles) {
    S2_TRY(vcycle2(r, 0));
    ++cycles;
    S2_HIP(launch2_residual(v0.r, v0.x, v0.b, v0.dev, nc, s));
    S2_HIP(launch_sumsq(h->norm_d, h->part_d, v0.r, v0.n, nc, s));
    S2_HIP(hipMemcpyAsync(rn.data(), h->norm_d, nc * sizeof(double), hipMemcpyDeviceToHost, s));
    S2_HIP(hipStreamSynchronize(s));
    relres = 0.0;
    ratio = 0.0;
    for (int c = 0; c < nc; ++c) {
      if (!std::isfinite(rn[c])) {
        set_error("residual is not finite");
        return SMG_ENONFINITE;
      }
      const double q = fn[c] > 0.0 ? std::sqrt(rn[c] / fn[c]) : 0.0;
      relres = q > relres ? q : relres;
      if (cycles >= 2 && rprev[c] > 0.0) ratio = std::max(ratio, std::sqrt(rn[c] / rprev[c]));
    }
    rprev = rn;
    if (relres <= rtol) break;
  }
  S2_HIP(launch_copy((double*)u, v0.x, field, s));
  S2_HIP(hipStreamSynchronize(s));
  if (info) {
    info->cycles = cycles;
    info->relres = relres;
    info->last_ratio = ratio;
  }
  if (relres > rtol) {
    set_error("solve did not converge: relres " + std::to_string(relres));
    return SMG_ENOTCONV;
  }
  return SMG_OK;
}

void smg2d_destroy(smg2d* h) { delete h; }

}  // extern "C"
