// C-ABI of the SELM coupling: the mobility H F, the thermal driving field g and the
// Euler-Maruyama step of the structure points (Sec. "Discretization of SELM Hydrodynamic
// Coupling Tensor", Sec. "Generation of the Stochastic Driving Fields Accounting for Thermal
// Fluctuations", algorithm "Stochastic Dynamics of Elastic Structures with Hydrodynamic
// Coupling").
//
// Built on the uniform-grid library: a 3-component hierarchy at kT = 1/mu draws the driving
// field xi ~ N(0, A^-1 / mu) (the stochastic multigrid chain) and solves the three velocity
// components; a 1-component hierarchy solves A p = D u inside the projection
// P u = u - D^T A^-1 D u.  Host side: the square root S of the 1D wall operator, built from its
// closed-form eigenvectors (sin(pi m (z + 1/2) / nz), eigenvalues (4/h^2) sin^2(pi m / (2 nz))).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "selm.hpp"
#include "smg_internal.hpp"

struct smg_selm {
  smg_selm_desc d{};
  smg_hierarchy* h3 = nullptr;
  smg_hierarchy* h1 = nullptr;
  size_t ws3 = 0, ws1 = 0;
  size_t off_ws3 = 0, off_ws1 = 0, off_f = 0, off_u = 0, off_w = 0, off_div = 0, off_p = 0,
         off_S = 0, off_V = 0, off_g = 0;
  size_t total = 0;
  std::vector<double> S;
  char* ws = nullptr;
};

namespace smg {
namespace {

#define SELM_HIP(call)                                                             \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));                \
      return SMG_EHIP;                                                             \
    }                                                                              \
  } while (0)

#define SELM_TRY(expr)             \
  do {                             \
    int rc_ = (expr);              \
    if (rc_ != SMG_OK) return rc_; \
  } while (0)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// S = a_z^{1/2} = sum_m sqrt(lambda_m) v_m v_m^T over the orthonormal wall eigenvectors
std::vector<double> sqrt_wall(int nz, double h) {
  std::vector<double> S((size_t)nz * nz, 0.0);
  std::vector<double> v(nz);
  for (int m = 1; m <= nz; ++m) {
    double ss = 0.0;
    for (int z = 0; z < nz; ++z) {
      v[z] = std::sin(M_PI * m * (z + 0.5) / nz);
      ss += v[z] * v[z];
    }
    const double sn = std::sin(M_PI * m / (2.0 * nz));
    const double root = 2.0 * sn / h;  // sqrt(lambda_m)
    for (int a = 0; a < nz; ++a)
      for (int b = 0; b < nz; ++b) S[(size_t)a * nz + b] += root * v[a] * v[b] / ss;
  }
  return S;
}

int64_t cells(const smg_selm* s) { return (int64_t)s->d.nx * s->d.ny * s->d.nz; }

double* dev(const smg_selm* s, size_t off) { return (double*)(s->ws + off); }

int check_ready(const smg_selm* s) {
  if (!s) {
    set_error("null SELM object");
    return SMG_EINVAL;
  }
  if (!s->ws) {
    set_error("SELM object has no workspace bound (call smg_selm_bind)");
    return SMG_ESTATE;
  }
  return SMG_OK;
}

int check_points(const smg_selm* s, int32_t m, const void* X) {
  if (m < 0 || m > s->d.max_points || (m > 0 && !X)) {
    set_error("number of points must be in [0, max_points] with a position array");
    return SMG_EINVAL;
  }
  return SMG_OK;
}

// out = P in (in and out may be the same field)
int project(smg_selm* s, const double* in, double* out, double rtol, hipStream_t st) {
  const smg_selm_desc& d = s->d;
  SELM_HIP(launch_selm_div(dev(s, s->off_div), in, dev(s, s->off_S), d.nx, d.ny, d.nz, d.h, st));
  smg_solve_info info{};
  SELM_TRY(smg_solve(s->h1, dev(s, s->off_div), dev(s, s->off_p), rtol, 200, st, &info));
  SELM_HIP(launch_selm_grad_sub(out, in, dev(s, s->off_p), dev(s, s->off_S), d.nx, d.ny, d.nz,
                                d.h, st));
  return SMG_OK;
}

int mobility(smg_selm* s, int32_t m, const double* X, const double* F, double* V, double rtol,
             hipStream_t st) {
  const smg_selm_desc& d = s->d;
  const int64_t N = cells(s);
  double* f = dev(s, s->off_f);
  double* u = dev(s, s->off_u);
  const double alpha = 1.0 / (d.h * d.h * d.h);
  SELM_HIP(launch_zero<double>(f, 3 * N, st));
  SELM_HIP(launch_selm_spread(f, X, F, m, d.nx, d.ny, d.nz, d.h, alpha, st));
  SELM_TRY(project(s, f, f, rtol, st));
  smg_solve_info info[1];
  SELM_TRY(smg_solve(s->h3, f, u, rtol, 200, st, info));
  SELM_TRY(project(s, u, u, rtol, st));
  SELM_HIP(launch_selm_interp(V, X, u, m, d.nx, d.ny, d.nz, d.h, 1.0 / d.mu, st));
  return SMG_OK;
}

int drive(smg_selm* s, int32_t m, const double* X, uint64_t seed, uint64_t first_cycle,
          double* state, double* g, double rtol, hipStream_t st) {
  const smg_selm_desc& d = s->d;
  double* xi = dev(s, s->off_w);
  SELM_TRY(smg_sample_field(s->h3, 1, seed, first_cycle, state, xi, SMG_OUT_F64, st));
  SELM_TRY(project(s, xi, xi, rtol, st));
  const double alpha = 1.0 / (d.h * d.h * d.h);
  SELM_HIP(launch_selm_interp(g, X, xi, m, d.nx, d.ny, d.nz, d.h,
                              std::sqrt(2.0 * d.kT * alpha), st));
  return SMG_OK;
}

}  // namespace
}  // namespace smg

using namespace smg;

extern "C" {

int smg_selm_create(const smg_selm_desc* desc, smg_selm** out) {
  if (!desc || !out) {
    set_error("null argument");
    return SMG_EINVAL;
  }
  *out = nullptr;
  const smg_selm_desc& d = *desc;
  if (!(d.mu > 0.0) || !(d.kT >= 0.0) || d.stride < 1 || d.max_points < 0 ||
      d.max_points > (1 << 20)) {
    set_error("mu > 0, kT >= 0, stride >= 1 and 0 <= max_points <= 2^20 are required");
    return SMG_EINVAL;
  }
  smg_selm* s = new (std::nothrow) smg_selm();
  if (!s) {
    set_error("host allocation failed");
    return SMG_ENOMEM;
  }
  s->d = d;
  smg_grid_desc g{d.nx, d.ny, d.nz, 3, d.h, 1.0 / d.mu, SMG_BC_PERIODIC, SMG_BC_PERIODIC,
                  SMG_BC_DIRICHLET_FACE};
  smg_cycle_params p{d.levels, 2, 2, 512, SMG_COARSEST_CHOLESKY, SMG_FP64, d.stride, 0};
  int rc = smg_create_hierarchy(&g, &p, &s->h3);
  if (rc == SMG_OK) {
    g.ncomp = 1;
    g.kT = 1.0;
    p.stride = 1;
    rc = smg_create_hierarchy(&g, &p, &s->h1);
  }
  if (rc != SMG_OK) {
    smg_selm_destroy(s);
    return rc;
  }
  smg_info i3{}, i1{};
  smg_hierarchy_info(s->h3, &i3);
  smg_hierarchy_info(s->h1, &i1);
  s->ws3 = i3.workspace_bytes;
  s->ws1 = i1.workspace_bytes;
  const size_t N = (size_t)d.nx * d.ny * d.nz;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  s->off_ws3 = take(s->ws3);
  s->off_ws1 = take(s->ws1);
  s->off_f = take(3 * N * sizeof(double));
  s->off_u = take(3 * N * sizeof(double));
  s->off_w = take(3 * N * sizeof(double));
  s->off_div = take(N * sizeof(double));
  s->off_p = take(N * sizeof(double));
  s->off_S = take((size_t)d.nz * d.nz * sizeof(double));
  s->off_V = take(3 * (size_t)std::max(d.max_points, 1) * sizeof(double));
  s->off_g = take(3 * (size_t)std::max(d.max_points, 1) * sizeof(double));
  s->total = off;
  s->S = sqrt_wall(d.nz, d.h);
  *out = s;
  return SMG_OK;
}

int smg_selm_get_info(const smg_selm* s, smg_selm_info* info) {
  if (!s || !info) {
    set_error("null argument");
    return SMG_EINVAL;
  }
  std::memset(info, 0, sizeof(*info));
  info->workspace_bytes = s->total;
  info->state_bytes = 3 * (size_t)cells(s) * sizeof(double);
  smg_info i3{};
  smg_hierarchy_info(s->h3, &i3);
  info->n_levels = i3.n_levels;
  return SMG_OK;
}

int smg_selm_bind(smg_selm* s, void* ws, size_t bytes, void* stream) {
  if (!s) {
    set_error("null SELM object");
    return SMG_EINVAL;
  }
  if (!ws || ((uintptr_t)ws & 255u)) {
    set_error("workspace must be a non-null 256-byte aligned device pointer");
    return SMG_EINVAL;
  }
  if (bytes < s->total) {
    set_error("workspace too small: need " + std::to_string(s->total) + " bytes");
    return SMG_ENOMEM;
  }
  char* base = (char*)ws;
  hipStream_t st = (hipStream_t)stream;
  SELM_TRY(smg_bind_workspace(s->h3, base + s->off_ws3, s->ws3, stream));
  SELM_TRY(smg_bind_workspace(s->h1, base + s->off_ws1, s->ws1, stream));
  SELM_HIP(hipMemcpyAsync(base + s->off_S, s->S.data(), s->S.size() * sizeof(double),
                          hipMemcpyHostToDevice, st));
  SELM_HIP(hipStreamSynchronize(st));
  s->ws = base;
  return SMG_OK;
}

int smg_selm_project(smg_selm* s, const void* u, void* pu, double rtol, void* stream) {
  SELM_TRY(check_ready(s));
  if (!u || !pu || ((uintptr_t)u & 255u) || ((uintptr_t)pu & 255u)) {
    set_error("u and pu must be non-null 256-byte aligned device pointers");
    return SMG_EINVAL;
  }
  return project(s, (const double*)u, (double*)pu, rtol, (hipStream_t)stream);
}

int smg_selm_mobility(smg_selm* s, int32_t m, const void* X, const void* F, void* V, double rtol,
                      void* stream) {
  SELM_TRY(check_ready(s));
  SELM_TRY(check_points(s, m, X));
  if (m > 0 && (!F || !V)) {
    set_error("F and V must be device pointers");
    return SMG_EINVAL;
  }
  return mobility(s, m, (const double*)X, (const double*)F, (double*)V, rtol,
                  (hipStream_t)stream);
}

int smg_selm_drive(smg_selm* s, int32_t m, const void* X, uint64_t seed, uint64_t first_cycle,
                   void* state, void* g, double rtol, void* stream) {
  SELM_TRY(check_ready(s));
  SELM_TRY(check_points(s, m, X));
  if (!state || ((uintptr_t)state & 255u) || (m > 0 && !g)) {
    set_error("state must be a 256-byte aligned device pointer and g a device pointer");
    return SMG_EINVAL;
  }
  return drive(s, m, (const double*)X, seed, first_cycle, (double*)state, (double*)g, rtol,
               (hipStream_t)stream);
}

int smg_selm_step(smg_selm* s, int32_t m, void* X, const void* F, double dt, uint64_t seed,
                  uint64_t step, void* state, double rtol, void* stream) {
  SELM_TRY(check_ready(s));
  SELM_TRY(check_points(s, m, X));
  if (!(dt >= 0.0) || (m > 0 && !F) || !state || ((uintptr_t)state & 255u)) {
    set_error("dt >= 0, F and a 256-byte aligned state are required");
    return SMG_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  double* V = dev(s, s->off_V);
  double* g = dev(s, s->off_g);
  SELM_TRY(mobility(s, m, (const double*)X, (const double*)F, V, rtol, st));
  SELM_TRY(drive(s, m, (const double*)X, seed, step * (uint64_t)s->d.stride, (double*)state, g,
                 rtol, st));
  SELM_HIP(launch_selm_em((double*)X, V, g, 3 * m, dt, st));
  return SMG_OK;
}

void smg_selm_destroy(smg_selm* s) {
  if (!s) return;
  smg_destroy_hierarchy(s->h3);
  smg_destroy_hierarchy(s->h1);
  delete s;
}

}  // extern "C"
