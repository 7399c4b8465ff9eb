// C-ABI of the composite-grid FAC sampler/solver: host plan and the cycle driver.
//
// Plan (host, once): the rows of the composite operator (composite.hpp), the prolongation P
// from the base grid onto the composite unknowns, and the Galerkin base levels
// A_0 = P^T A P, A_{l+1} = P_l^T A_l P_l (trilinear P_l with wall ghosts; Sec. "Stochastic
// Multigrid Methods", variational property).  Only the rows near the refined box differ from
// the translation-invariant rows of a level; those are computed cell by cell inside a
// periodic box region R_l (the refined box dilated by two cells on level 0, then every cell
// whose prolongation support meets R_l), the others once per z-plane.  Equal rows share one
// stencil of the dictionary and equal 2x2x2 blocks share one block type (factors of A_BB).
// The coarsest level is factored densely.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/smg.h"
#include "composite.hpp"
#include "kernels.hpp"
#include "smg_internal.hpp"

namespace smg {
namespace {

constexpr uint32_t KIND_COMP = 2;
constexpr uint32_t KIND_FAC_BASE = 3;
constexpr uint32_t KIND_FAC_COARSEST = 4;
constexpr uint32_t KIND_FORCING = 5;
constexpr int kMaxCompLevels = 16;
constexpr int kMaxDense = 4096;

#define CMP_HIP(call)                                                \
  do {                                                               \
    hipError_t e_ = (call);                                          \
    if (e_ != hipSuccess) {                                          \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));  \
      return SMG_EHIP;                                               \
    }                                                                \
  } while (0)

inline int wrap(int v, int n) { return ((v % n) + n) % n; }

// representative of d modulo n in [-(n/2), n - n/2 - 1]
inline int canon(int d, int n) {
  const int m = wrap(d, n);
  return m > n - 1 - n / 2 ? m - n : m;
}

// periodic or clipped index range [lo, lo + len) on an axis of extent n
struct Range {
  int lo = 0, len = 0;
  bool full(int n) const { return len >= n; }
  bool has(int v, int n) const { return len >= n || wrap(v - lo, n) < len; }
};

struct GLevel {
  int nx = 0, ny = 0, nz = 0;
  int64_t n = 0;
  bool coarsest = false;
  Range rx, ry, rz;  // cells whose rows are computed one by one
  std::vector<int32_t> sid;
  std::vector<int32_t> st_off{0}, st_code;
  std::vector<double> st_val;
  std::unordered_map<std::string, int32_t> dedup;
  std::vector<int32_t> btype, bt_sid;
  std::vector<double> bt_fac;
  std::vector<double> bt_c7, bt_diag;
  int split = 1;
  std::vector<int32_t> list;  // split == 1: blocks of non-plain type, grouped by block colour
  int list_off[9] = {0};
  size_t off_list = 0;
  // device copies: fields x, b, r and the coefficient tables in the sweep precision (double, or
  // float in the FP32-refined form); the integer tables are shared
  size_t off_x = 0, off_b = 0, off_r = 0, off_btype = 0, off_btsid = 0, off_stoff = 0,
         off_btfac = 0, off_ent = 0, off_btc7 = 0, off_btdiag = 0;
  double* x = nullptr;
  double* b = nullptr;
  double* r = nullptr;
  float* x32 = nullptr;
  float* b32 = nullptr;
  float* r32 = nullptr;
  GStencilT<double> dev{};
  GStencilT<float> dev32{};
};

// Device record of stencil entry e of level L: the coefficient, the linear offset of its target
// (valid away from the periodic seams) and the offset code with the in-block mask (bit 8 + k set
// when the target of a cell with in-block index k lies in that cell's 2x2x2 block; on a periodic
// axis of even extent the target's block is the cell's exactly when k_a + d_a wraps to 0 or 1).
template <typename T>
smg::StEntryT<T> device_entry(const GLevel& L, size_t e) {
  const int code = L.st_code[e];
  const int dz = code / 25 - 2, dy = (code / 5) % 5 - 2, dx = code % 5 - 2;
  uint32_t mask = 0;
  for (int k = 0; k < 8; ++k) {
    const bool in = wrap((k & 1) + dx, L.nx) < 2 && wrap(((k >> 1) & 1) + dy, L.ny) < 2 &&
                    (unsigned)((k >> 2) + dz) < 2u;
    if (in) mask |= 1u << k;
  }
  return smg::StEntryT<T>{(T)L.st_val[e], dx + L.nx * (dy + L.ny * dz),
                          (int32_t)(code | (mask << 8))};
}

// A row as a dense 5x5x5 accumulator over canonical offsets (exact zeros dropped on encoding).
struct Acc {
  double v[125];
  void clear() { std::fill(v, v + 125, 0.0); }
};

}  // namespace

struct Composite {
  CompGeom g{};
  double h = 1.0, kT = 1.0;
  int nu = 2, mu1 = 2, mu2 = 2;
  bool gs_only = false;
  int row_lanes = 0;  // lanes per long row (0: by launch size)
  int prec = SMG_FP64;
  std::vector<GLevel> lv;
  int ncd = 0;
  std::vector<double> ainv, w;  // A_c^-1 and L_c^-T (row-major)
  std::vector<int32_t> layer;  // layer cells grouped by parity class
  int layer_off[9] = {0};
  size_t ws_bytes = 0, off_rc = 0, off_rf = 0, off_layer = 0, off_ainv = 0, off_w = 0,
         off_part = 0, off_norm = 0, off_znoise = 0, off_e32c = 0, off_e32f = 0, off_r32c = 0,
         off_r32f = 0, off_rf32 = 0, off_fc = 0, off_ff = 0;
  char* ws = nullptr;
  int device = -1;
  double* rc = nullptr;
  double* rf = nullptr;
  double* ainv_d = nullptr;
  double* w_d = nullptr;
  double* part = nullptr;
  double* norm = nullptr;
  double* znoise = nullptr;
  int32_t* layer_d = nullptr;
  // FP32-refined form: the correction e and the FP32 right-hand side of the inner cycle
  // (coarse part on the base grid, fine part on the box) and the inner fine residual
  float* e32c = nullptr;
  float* e32f = nullptr;
  float* r32c = nullptr;
  float* r32f = nullptr;
  float* rf32 = nullptr;
};

}  // namespace smg

struct smg_composite {
  smg::Composite c;
};

namespace smg {
namespace {

// ------------------------------------------------------------------ composite rows (host)
bool is_cov(const CompGeom& g, int x, int y, int z) {
  return x >= g.x0 && x < g.x1 && y >= g.y0 && y < g.y1 && z >= g.z0 && z < g.z1;
}

// composite unknown: base index for coarse cells, nbase + box index for fine cells
struct Ent {
  int64_t u;
  double a;
};

// Entries of row u of A in units of 1/h^2 (same rules as the kernels' rows).
void comp_row(const CompGeom& g, int64_t u, std::vector<Ent>& out) {
  out.clear();
  const int64_t nbase = (int64_t)g.nx * g.ny * g.nz;
  auto fid = [&](int i, int j, int k) { return nbase + i + (int64_t)g.fx * (j + (int64_t)g.fy * k); };
  if (u < nbase) {
    const int x = (int)(u % g.nx), y = (int)((u / g.nx) % g.ny), z = (int)(u / ((int64_t)g.nx * g.ny));
    double diag = 0.0;
    for (int d = 0; d < 6; ++d) {
      const int axis = d >> 1, sgn = (d & 1) ? -1 : 1;
      int q[3] = {x, y, z};
      q[axis] += sgn;
      if (axis == 2 && (q[2] < 0 || q[2] >= g.nz)) {
        diag += 2.0;
        continue;
      }
      q[0] = wrap(q[0], g.nx);
      q[1] = wrap(q[1], g.ny);
      if (is_cov(g, q[0], q[1], q[2])) {
        int c0[3] = {2 * (q[0] - g.x0), 2 * (q[1] - g.y0), 2 * (q[2] - g.z0)};
        c0[axis] += sgn > 0 ? 0 : 1;
        const int t0 = axis == 0 ? 1 : 0, t1 = axis == 2 ? 1 : 2;
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) {
            int c[3] = {c0[0], c0[1], c0[2]};
            c[t0] += a;
            c[t1] += b;
            out.push_back({fid(c[0], c[1], c[2]), -1.0 / 3.0});
          }
        diag += 4.0 / 3.0;
      } else {
        out.push_back({q[0] + (int64_t)g.nx * (q[1] + (int64_t)g.ny * q[2]), -1.0});
        diag += 1.0;
      }
    }
    out.push_back({u, diag});
    return;
  }
  const int64_t lf = u - nbase;
  const int i = (int)(lf % g.fx), j = (int)((lf / g.fx) % g.fy), k = (int)(lf / ((int64_t)g.fx * g.fy));
  const int p[3] = {i, j, k};
  const int ext[3] = {g.fx, g.fy, g.fz};
  double diag = 0.0;
  for (int d = 0; d < 6; ++d) {
    const int axis = d >> 1, sgn = (d & 1) ? -1 : 1;
    int c[3] = {i, j, k};
    c[axis] += sgn;
    if (c[axis] >= 0 && c[axis] < ext[axis]) {
      out.push_back({fid(c[0], c[1], c[2]), -0.5});
      diag += 0.5;
      continue;
    }
    int A[3] = {g.x0 + (i >> 1), g.y0 + (j >> 1), g.z0 + (k >> 1)};
    if (axis == 0) A[0] = wrap(sgn > 0 ? g.x1 : g.x0 - 1, g.nx);
    if (axis == 1) A[1] = wrap(sgn > 0 ? g.y1 : g.y0 - 1, g.ny);
    if (axis == 2) {
      A[2] = sgn > 0 ? g.z1 : g.z0 - 1;
      if (A[2] < 0 || A[2] >= g.nz) {
        diag += 1.0;
        continue;
      }
    }
    out.push_back({A[0] + (int64_t)g.nx * (A[1] + (int64_t)g.ny * A[2]), -1.0 / 3.0});
    diag += 1.0 / 12.0;
    const int t0 = axis == 0 ? 1 : 0, t1 = axis == 2 ? 1 : 2;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        int q[3] = {p[0], p[1], p[2]};
        q[t0] = (q[t0] & ~1) + a;
        q[t1] = (q[t1] & ~1) + b;
        if (q[0] == i && q[1] == j && q[2] == k) continue;
        out.push_back({fid(q[0], q[1], q[2]), 1.0 / 12.0});
      }
  }
  out.push_back({u, diag});
}

// 1D trilinear entries of fine coordinate p onto base cells (wall ghost on non-periodic axes)
int p1d(int p, int n, bool periodic, int* J, double* w) {
  const int j = p >> 1;
  const int o = (p & 1) ? j + 1 : j - 1;
  J[0] = j;
  w[0] = 0.75;
  if (periodic) {
    J[1] = wrap(o, n);
    w[1] = 0.25;
  } else if (o >= 0 && o < n) {
    J[1] = o;
    w[1] = 0.25;
  } else {
    J[1] = j;
    w[1] = -0.25;
  }
  return 2;
}

// 1D restriction weights: fine coordinates p in 2J-1..2J+2 (periodic wrap) with P(p, J) != 0
int r1d(int J, int n, bool periodic, int* p, double* w) {
  int c = 0;
  for (int d = -1; d <= 2; ++d) {
    int q = 2 * J + d;
    if (periodic) q = wrap(q, 2 * n);
    else if (q < 0 || q >= 2 * n) continue;
    double wt = (d == 0 || d == 1) ? 0.75 : 0.25;
    if (!periodic && ((d == 0 && J == 0) || (d == 1 && J == n - 1))) wt -= 0.25;
    p[c] = q;
    w[c] = wt;
    ++c;
  }
  return c;
}

std::string enc_key(const std::vector<int32_t>& codes, const std::vector<double>& vals) {
  std::string k;
  k.resize(codes.size() * 4 + vals.size() * 8);
  std::memcpy(&k[0], codes.data(), codes.size() * 4);
  std::memcpy(&k[codes.size() * 4], vals.data(), vals.size() * 8);
  return k;
}

// Adds the row held in `acc` (coefficients in absolute units) to the dictionary; returns its id.
int32_t intern(GLevel& L, const Acc& acc, std::mutex& mu) {
  std::vector<int32_t> codes;
  std::vector<double> vals;
  for (int c = 0; c < 125; ++c)
    if (acc.v[c] != 0.0) {
      codes.push_back(c);
      vals.push_back(acc.v[c]);
    }
  std::string key = enc_key(codes, vals);
  std::lock_guard<std::mutex> lk(mu);
  auto it = L.dedup.find(key);
  if (it != L.dedup.end()) return it->second;
  const int32_t id = (int32_t)L.st_off.size() - 1;
  L.st_code.insert(L.st_code.end(), codes.begin(), codes.end());
  L.st_val.insert(L.st_val.end(), vals.begin(), vals.end());
  L.st_off.push_back((int32_t)L.st_code.size());
  L.dedup.emplace(std::move(key), id);
  return id;
}

bool add_code(Acc& acc, int dx, int dy, int dz, const GLevel& L, double v) {
  dx = canon(dx, L.nx);
  dy = canon(dy, L.ny);
  if (dx < -2 || dx > 2 || dy < -2 || dy > 2 || dz < -2 || dz > 2) return v == 0.0;
  acc.v[(dz + 2) * 25 + (dy + 2) * 5 + (dx + 2)] += v;
  return true;
}

// Level-0 row of base cell (X, Y, Z): (P^T A P)_J, in absolute units.
bool row0(const CompGeom& g, const GLevel& L, int X, int Y, int Z, Acc& acc,
          std::vector<Ent>& tmp) {
  acc.clear();
  const int64_t nbase = (int64_t)g.nx * g.ny * g.nz;
  bool ok = true;
  auto add_u = [&](int64_t u, double pw) {
    comp_row(g, u, tmp);
    for (const Ent& e : tmp) {
      const double pa = pw * e.a * g.ih2;
      if (e.u < nbase) {
        const int x = (int)(e.u % g.nx), y = (int)((e.u / g.nx) % g.ny), z = (int)(e.u / ((int64_t)g.nx * g.ny));
        ok &= add_code(acc, x - X, y - Y, z - Z, L, pa);
      } else {
        const int64_t lf = e.u - nbase;
        const int i = (int)(lf % g.fx), j = (int)((lf / g.fx) % g.fy), k = (int)(lf / ((int64_t)g.fx * g.fy));
        int JX[2], JY[2], JZ[2];
        double wx[2], wy[2], wz[2];
        p1d(2 * g.x0 + i, g.nx, true, JX, wx);
        p1d(2 * g.y0 + j, g.ny, true, JY, wy);
        p1d(2 * g.z0 + k, g.nz, false, JZ, wz);
        for (int c = 0; c < 2; ++c)
          for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a)
              ok &= add_code(acc, JX[a] - X, JY[b] - Y, JZ[c] - Z, L, pa * wx[a] * wy[b] * wz[c]);
      }
    }
  };
  if (!is_cov(g, X, Y, Z)) add_u(X + (int64_t)g.nx * (Y + (int64_t)g.ny * Z), 1.0);
  int px[4], py[4], pz[4];
  double wx[4], wy[4], wz[4];
  const int cx = r1d(X, g.nx, true, px, wx);
  const int cy = r1d(Y, g.ny, true, py, wy);
  const int cz = r1d(Z, g.nz, false, pz, wz);
  for (int c = 0; c < cz; ++c) {
    const int k = pz[c] - 2 * g.z0;
    if (k < 0 || k >= g.fz) continue;
    for (int b = 0; b < cy; ++b) {
      const int j = py[b] - 2 * g.y0;
      if (j < 0 || j >= g.fy) continue;
      for (int a = 0; a < cx; ++a) {
        const int i = px[a] - 2 * g.x0;
        if (i < 0 || i >= g.fx) continue;
        add_u(nbase + i + (int64_t)g.fx * (j + (int64_t)g.fy * k), wx[a] * wy[b] * wz[c]);
      }
    }
  }
  return ok;
}

// Row (X, Y, Z) of level l+1 = P_l^T A_l P_l from the dictionary of level l (F).
bool row_next(const GLevel& F, const GLevel& L, int X, int Y, int Z, Acc& acc) {
  acc.clear();
  bool ok = true;
  int px[4], py[4], pz[4];
  double wx[4], wy[4], wz[4];
  const int cx = r1d(X, L.nx, true, px, wx);
  const int cy = r1d(Y, L.ny, true, py, wy);
  const int cz = r1d(Z, L.nz, false, pz, wz);
  for (int c = 0; c < cz; ++c)
    for (int b = 0; b < cy; ++b)
      for (int a = 0; a < cx; ++a) {
        const int fxp = px[a], fyp = py[b], fzp = pz[c];
        const double pf = wx[a] * wy[b] * wz[c];
        const int64_t f = fxp + (int64_t)F.nx * (fyp + (int64_t)F.ny * fzp);
        const int s = F.sid[f];
        for (int e = F.st_off[s]; e < F.st_off[s + 1]; ++e) {
          const int code = F.st_code[e];
          const int dz = code / 25 - 2, dy = (code / 5) % 5 - 2, dx = code % 5 - 2;
          const int gx = wrap(fxp + dx, F.nx), gy = wrap(fyp + dy, F.ny), gz = fzp + dz;
          const double pa = pf * F.st_val[e];
          int JX[2], JY[2], JZ[2];
          double qx[2], qy[2], qz[2];
          p1d(gx, L.nx, true, JX, qx);
          p1d(gy, L.ny, true, JY, qy);
          p1d(gz, L.nz, false, JZ, qz);
          for (int cc = 0; cc < 2; ++cc)
            for (int bb = 0; bb < 2; ++bb)
              for (int aa = 0; aa < 2; ++aa)
                ok &= add_code(acc, JX[aa] - X, JY[bb] - Y, JZ[cc] - Z, L,
                               pa * qx[aa] * qy[bb] * qz[cc]);
        }
      }
  return ok;
}

void parallel_planes(int nz, const std::function<void(int)>& fn) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  nt = std::min<unsigned>(nt, (unsigned)nz);
  std::vector<std::thread> th;
  std::atomic<int> next{0};
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      for (int z = next++; z < nz; z = next++) fn(z);
    });
  for (auto& t : th) t.join();
}

// Fills L.sid: cells of R one by one, the rest from one representative per z-plane.
bool fill_level(GLevel& L, const std::function<bool(int, int, int, Acc&)>& rowfn,
                std::string& err) {
  L.n = (int64_t)L.nx * L.ny * L.nz;
  L.sid.assign(L.n, -1);
  std::mutex mu;
  std::atomic<bool> bad{false};
  parallel_planes(L.nz, [&](int z) {
    Acc acc;
    int32_t uni = -1;
    const bool zin = L.rz.has(z, L.nz);
    for (int y = 0; y < L.ny; ++y)
      for (int x = 0; x < L.nx; ++x) {
        const bool in = zin && L.rx.has(x, L.nx) && L.ry.has(y, L.ny);
        int32_t id;
        if (in || uni < 0) {
          if (!rowfn(x, y, z, acc)) bad = true;
          id = intern(L, acc, mu);
          if (!in) uni = id;
        } else {
          id = uni;
        }
        L.sid[x + (int64_t)L.nx * (y + (int64_t)L.ny * z)] = id;
      }
  });
  if (bad) {
    err = "a Galerkin row reaches beyond two cells (unsupported geometry)";
    return false;
  }
  return true;
}

// 8x8 lower Cholesky in place; false if not positive definite
bool chol8(double* A) {
  for (int j = 0; j < 8; ++j) {
    double d = A[j * 8 + j];
    for (int k = 0; k < j; ++k) d -= A[j * 8 + k] * A[j * 8 + k];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    A[j * 8 + j] = d;
    for (int i = j + 1; i < 8; ++i) {
      double s = A[i * 8 + j];
      for (int k = 0; k < j; ++k) s -= A[i * 8 + k] * A[j * 8 + k];
      A[i * 8 + j] = s / d;
    }
    for (int k = j + 1; k < 8; ++k) A[j * 8 + k] = 0.0;
  }
  return true;
}

// W = L^-1 (lower, n x n row-major), row by row: W[i][c] = -(sum_{c<=k<i} L[i][k] W[k][c]) / L[i][i]
// accumulated over k with contiguous rows of W
std::vector<double> lower_inv(const std::vector<double>& Lm, int n) {
  std::vector<double> W((size_t)n * n, 0.0);
  std::vector<double> acc(n);
  for (int i = 0; i < n; ++i) {
    std::fill(acc.begin(), acc.begin() + i, 0.0);
    for (int k = 0; k < i; ++k) {
      const double a = Lm[(size_t)i * n + k];
      if (a == 0.0) continue;
      const double* wk = &W[(size_t)k * n];
      for (int c = 0; c <= k; ++c) acc[c] += a * wk[c];
    }
    const double d = Lm[(size_t)i * n + i];
    for (int c = 0; c < i; ++c) W[(size_t)i * n + c] = -acc[c] / d;
    W[(size_t)i * n + i] = 1.0 / d;
  }
  return W;
}

// rows [0, n) split over host threads
void parallel_rows(int n, const std::function<void(int)>& fn) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  std::atomic<int> next{0};
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      for (int i = next++; i < n; i = next++) fn(i);
    });
  for (auto& t : th) t.join();
}

bool chol_dense(std::vector<double>& A, int n) {
  for (int j = 0; j < n; ++j) {
    double d = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    A[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) s -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
      A[(size_t)i * n + j] = s / d;
    }
    for (int k = j + 1; k < n; ++k) A[(size_t)j * n + k] = 0.0;
  }
  return true;
}

bool build_blocks(GLevel& L, std::string& err) {
  const int nbx = L.nx / 2, nby = L.ny / 2, nbz = L.nz / 2;
  L.btype.assign((size_t)nbx * nby * nbz, -1);
  std::map<std::array<int32_t, 8>, int32_t> types;
  for (int bz = 0; bz < nbz; ++bz)
    for (int by = 0; by < nby; ++by)
      for (int bx = 0; bx < nbx; ++bx) {
        std::array<int32_t, 8> key;
        for (int k = 0; k < 8; ++k) {
          const int cx = 2 * bx + (k & 1), cy = 2 * by + ((k >> 1) & 1), cz = 2 * bz + (k >> 2);
          key[k] = L.sid[cx + (int64_t)L.nx * (cy + (int64_t)L.ny * cz)];
        }
        auto it = types.find(key);
        int32_t t;
        if (it == types.end()) {
          t = (int32_t)types.size();
          types.emplace(key, t);
          double A[64] = {0};
          for (int k = 0; k < 8; ++k) {
            const int lk[3] = {k & 1, (k >> 1) & 1, k >> 2};
            const int s = key[k];
            for (int e = L.st_off[s]; e < L.st_off[s + 1]; ++e) {
              const int code = L.st_code[e];
              const int d[3] = {code % 5 - 2, (code / 5) % 5 - 2, code / 25 - 2};
              int m = 0;
              bool in = true;
              for (int a = 0; a < 3; ++a) {
                const int q = lk[a] + d[a];
                if (q < 0 || q > 1) in = false;
                m |= (q & 1) << a;
              }
              if (in) A[k * 8 + m] += L.st_val[e];
            }
          }
          double Lc[64];
          std::memcpy(Lc, A, sizeof(A));
          if (!chol8(Lc)) {
            err = "a 2x2x2 diagonal block is not positive definite";
            return false;
          }
          std::vector<double> Lv(Lc, Lc + 64);
          std::vector<double> W = lower_inv(Lv, 8);
          double fac[128];
          for (int i = 0; i < 8; ++i)
            for (int j = 0; j < 8; ++j) {
              double s = 0.0;
              for (int k = 0; k < 8; ++k) s += W[k * 8 + i] * W[k * 8 + j];
              fac[i * 8 + j] = s;              // A_BB^-1 = W^T W
              fac[64 + i * 8 + j] = W[j * 8 + i];  // L^-T = W^T
            }
          L.bt_fac.insert(L.bt_fac.end(), fac, fac + 128);
          L.bt_sid.insert(L.bt_sid.end(), key.begin(), key.end());
        } else {
          t = it->second;
        }
        L.btype[bx + (size_t)nbx * (by + (size_t)nby * bz)] = t;
      }
  // plain 7-point block types: every row holds the centre plus face offsets only, all
  // off-diagonal coefficients equal; a row may lack a z face only where that face is a wall
  const size_t ntypes = L.bt_sid.size() / 8;
  L.bt_c7.assign(ntypes, 0.0);
  L.bt_diag.assign(ntypes * 8, 0.0);
  std::vector<int> zmask(ntypes * 8, 0);  // bit 0: row has -z, bit 1: row has +z
  for (size_t t = 0; t < ntypes; ++t) {
    double c7 = 0.0;
    bool plain = true;
    for (int k = 0; k < 8 && plain; ++k) {
      const int s = L.bt_sid[t * 8 + k];
      int faces = 0;
      for (int e = L.st_off[s]; e < L.st_off[s + 1]; ++e) {
        const int code = L.st_code[e];
        const int dx = code % 5 - 2, dy = (code / 5) % 5 - 2, dz = code / 25 - 2;
        const int ad = std::abs(dx) + std::abs(dy) + std::abs(dz);
        if (ad == 0) {
          L.bt_diag[t * 8 + k] = L.st_val[e];
          continue;
        }
        if (ad != 1) {
          plain = false;
          break;
        }
        if (c7 == 0.0) c7 = L.st_val[e];
        if (L.st_val[e] != c7) plain = false;
        if (dz == -1) faces |= 1;
        if (dz == 1) faces |= 2;
        if (dx != 0 || dy != 0) faces |= 4 << ((dx + 1) + 3 * (dy + 1));
      }
      // all four x/y faces present
      const int xy = (4 << (0 + 3)) | (4 << (2 + 3)) | (4 << (1 + 0)) | (4 << (1 + 6));
      if ((faces & xy) != xy) plain = false;
      zmask[t * 8 + k] = faces & 3;
    }
    if (plain && c7 != 0.0) L.bt_c7[t] = c7;
  }
  // a missing z face must be a wall for every block of the type
  for (int bz = 0; bz < nbz; ++bz)
    for (int by = 0; by < nby; ++by)
      for (int bx = 0; bx < nbx; ++bx) {
        const int t = L.btype[bx + (size_t)nbx * (by + (size_t)nby * bz)];
        if (L.bt_c7[t] == 0.0) continue;
        for (int k = 0; k < 8; ++k) {
          const int cz = 2 * bz + (k >> 2);
          const int want = (cz > 0 ? 1 : 0) | (cz + 1 < L.nz ? 2 : 0);
          if (zmask[t * 8 + k] != want) L.bt_c7[t] = 0.0;
        }
      }
  return true;
}

inline int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// R_{l+1}: the cells J whose prolongation support 2J-1 .. 2J+2 meets R_l = [lo, lo + len)
Range next_range(const Range& r, int nf, int nc, bool periodic) {
  Range o;
  if (r.len >= nf) {
    o.lo = 0;
    o.len = nc;
    return o;
  }
  const int lo = floordiv(r.lo - 1, 2);         // smallest J with 2J + 2 >= lo
  const int hi = floordiv(r.lo + r.len, 2);     // largest J with 2J - 1 <= lo + len - 1
  o.lo = lo;
  o.len = hi - lo + 1;
  if (!periodic) {
    o.lo = std::max(0, lo);
    o.len = std::min(nc - 1, hi) - o.lo + 1;
  }
  if (o.len >= nc) {
    o.lo = 0;
    o.len = nc;
  }
  return o;
}

int plan(Composite& C, const smg_composite_desc& d, const smg_fac_params& p, std::string& err) {
  CompGeom& g = C.g;
  g.nx = d.nx;
  g.ny = d.ny;
  g.nz = d.nz;
  g.x0 = d.box[0];
  g.x1 = d.box[1];
  g.y0 = d.box[2];
  g.y1 = d.box[3];
  g.z0 = d.box[4];
  g.z1 = d.box[5];
  if (g.nx < 4 || g.ny < 4 || g.nz < 1 || g.nx % 2 || g.ny % 2) {
    err = "base grid: nx, ny must be even and >= 4, nz >= 1";
    return SMG_EINVAL;
  }
  if (!(0 <= g.x0 && g.x0 < g.x1 && g.x1 <= g.nx && g.x1 - g.x0 < g.nx && 0 <= g.y0 &&
        g.y0 < g.y1 && g.y1 <= g.ny && g.y1 - g.y0 < g.ny && 0 <= g.z0 && g.z0 < g.z1 &&
        g.z1 <= g.nz)) {
    err = "refined box must lie inside the grid and not span a whole periodic extent";
    return SMG_EINVAL;
  }
  if (!(d.h > 0.0) || !(d.kT >= 0.0) || p.nu < 0 || p.mu1 < 0 || p.mu2 < 0 || p.nu > 64 ||
      p.mu1 + p.mu2 > 64 || p.levels < 0 || p.levels > kMaxCompLevels || p.coarsest_max < 1 ||
      p.coarsest_max > kMaxDense) {
    err = "invalid h, kT or cycle parameters";
    return SMG_EINVAL;
  }
  g.fx = 2 * (g.x1 - g.x0);
  g.fy = 2 * (g.y1 - g.y0);
  g.fz = 2 * (g.z1 - g.z0);
  g.ih2 = 1.0 / (d.h * d.h);
  C.h = d.h;
  C.kT = d.kT;
  C.nu = p.nu;
  C.mu1 = p.mu1;
  C.mu2 = p.mu2;
  C.gs_only = p.gs_only != 0;
  if (p.precision != SMG_FP64 && p.precision != SMG_FP32_REFINED) {
    err = "precision must be SMG_FP64 or SMG_FP32_REFINED";
    return SMG_EINVAL;
  }
  C.prec = p.precision;
  if (p.row_lanes != 0 && p.row_lanes != 2 && p.row_lanes != 8) {
    err = "row_lanes must be 0, 2 or 8";
    return SMG_EINVAL;
  }
  C.row_lanes = p.row_lanes;
  // base level plan (block smoothing needs nx, ny multiples of 4 and nz even)
  std::vector<std::array<int, 3>> dims{{g.nx, g.ny, g.nz}};
  for (;;) {
    const auto& q = dims.back();
    const bool sm = q[0] % 4 == 0 && q[1] % 4 == 0 && q[2] % 2 == 0;
    const bool want = p.levels > 0 ? (int)dims.size() < p.levels
                                   : (int64_t)q[0] * q[1] * q[2] > p.coarsest_max;
    if (!want || !sm || (int)dims.size() >= kMaxCompLevels) break;
    dims.push_back({q[0] / 2, q[1] / 2, q[2] / 2});
  }
  if (p.levels > 0 && (int)dims.size() != p.levels) {
    err = "base grid cannot be coarsened to the requested number of levels";
    return SMG_EINVAL;
  }
  const auto& cd = dims.back();
  if ((int64_t)cd[0] * cd[1] * cd[2] > kMaxDense) {
    err = "coarsest base level above 4096 unknowns";
    return SMG_EINVAL;
  }
  C.lv.resize(dims.size());
  for (size_t l = 0; l < dims.size(); ++l) {
    GLevel& L = C.lv[l];
    L.nx = dims[l][0];
    L.ny = dims[l][1];
    L.nz = dims[l][2];
    L.coarsest = l + 1 == dims.size();
  }
  // level 0: R_0 = the box dilated by two cells
  {
    GLevel& L = C.lv[0];
    L.rx = {g.x0 - 2, g.x1 - g.x0 + 4};
    L.ry = {g.y0 - 2, g.y1 - g.y0 + 4};
    L.rz.lo = std::max(0, g.z0 - 2);
    L.rz.len = std::min(g.nz, g.z1 + 2) - L.rz.lo;
    if (L.rx.len >= L.nx) L.rx = {0, L.nx};
    if (L.ry.len >= L.ny) L.ry = {0, L.ny};
    const CompGeom gg = g;
    if (!fill_level(L,
                    [&](int x, int y, int z, Acc& acc) {
                      thread_local std::vector<Ent> tmp;
                      return row0(gg, L, x, y, z, acc, tmp);
                    },
                    err))
      return SMG_EINVAL;
  }
  for (size_t l = 1; l < C.lv.size(); ++l) {
    GLevel& F = C.lv[l - 1];
    GLevel& L = C.lv[l];
    L.rx = next_range(F.rx, F.nx, L.nx, true);
    L.ry = next_range(F.ry, F.ny, L.ny, true);
    L.rz = next_range(F.rz, F.nz, L.nz, false);
    if (!fill_level(L, [&](int x, int y, int z, Acc& acc) { return row_next(F, L, x, y, z, acc); },
                    err))
      return SMG_EINVAL;
  }
  for (auto& L : C.lv) {
    if (L.coarsest) continue;
    if (!build_blocks(L, err)) return SMG_EINVAL;
  }
  // coarsest: dense factor
  {
    GLevel& L = C.lv.back();
    const int n = (int)L.n;
    std::vector<double> A((size_t)n * n, 0.0);
    for (int z = 0; z < L.nz; ++z)
      for (int y = 0; y < L.ny; ++y)
        for (int x = 0; x < L.nx; ++x) {
          const int i = x + L.nx * (y + L.ny * z);
          const int s = L.sid[i];
          for (int e = L.st_off[s]; e < L.st_off[s + 1]; ++e) {
            const int code = L.st_code[e];
            const int tx = wrap(x + code % 5 - 2, L.nx), ty = wrap(y + (code / 5) % 5 - 2, L.ny);
            const int tz = z + code / 25 - 2;
            if (tz < 0 || tz >= L.nz) {
              err = "coarsest row leaves the grid";
              return SMG_EINVAL;
            }
            A[(size_t)i * n + tx + L.nx * (ty + L.ny * tz)] += L.st_val[e];
          }
        }
    if (!chol_dense(A, n)) {
      err = "coarsest operator is not positive definite";
      return SMG_EINVAL;
    }
    const std::vector<double> W = lower_inv(A, n);  // L_c^-1
    // A_c^-1 = W^T W: row i = sum_{k >= i} W[k][i] W[k][:]
    C.ainv.assign((size_t)n * n, 0.0);
    parallel_rows(n, [&](int i) {
      double* row = &C.ainv[(size_t)i * n];
      for (int k = i; k < n; ++k) {
        const double a = W[(size_t)k * n + i];
        if (a == 0.0) continue;
        const double* wk = &W[(size_t)k * n];
        for (int j = 0; j <= k; ++j) row[j] += a * wk[j];
      }
    });
    C.w.assign((size_t)n * n, 0.0);  // L_c^-T = W^T
    for (int i = 0; i < n; ++i)
      for (int j = 0; j <= i; ++j) C.w[(size_t)j * n + i] = W[(size_t)i * n + j];
    C.ncd = n;
  }
  // layer cells by parity class
  {
    std::vector<int32_t> cls[8];
    for (int k = 0; k < g.fz; ++k)
      for (int j = 0; j < g.fy; ++j)
        for (int i = 0; i < g.fx; ++i) {
          const bool lay = i == 0 || i == g.fx - 1 || j == 0 || j == g.fy - 1 ||
                           (k == 0 && g.z0 > 0) || (k == g.fz - 1 && g.z1 < g.nz);
          if (lay) cls[(i & 1) + 2 * (j & 1) + 4 * (k & 1)].push_back(i + g.fx * (j + g.fy * k));
        }
    C.layer.clear();
    for (int c = 0; c < 8; ++c) {
      C.layer_off[c] = (int)C.layer.size();
      C.layer.insert(C.layer.end(), cls[c].begin(), cls[c].end());
    }
    C.layer_off[8] = (int)C.layer.size();
  }
  // workspace layout
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  const int64_t nbase = (int64_t)g.nx * g.ny * g.nz;
  const int64_t nf = (int64_t)g.fx * g.fy * g.fz;
  const bool f32 = C.prec == SMG_FP32_REFINED;
  const size_t es = f32 ? 4 : 8;  // bytes of a value of the sweep precision
  C.off_rc = take(nbase * 8);
  C.off_rf = take(nf * 8);
  C.off_fc = take(nbase * 8);  // right-hand side of the forced field
  C.off_ff = take(nf * 8);
  C.off_layer = take(std::max<size_t>(1, C.layer.size()) * 4);
  if (f32) {
    C.off_e32c = take(nbase * 4);
    C.off_e32f = take(nf * 4);
    C.off_r32c = take(nbase * 4);
    C.off_r32f = take(nf * 4);
    C.off_rf32 = take(nf * 4);
  }
  for (auto& L : C.lv) {
    L.off_x = take(L.n * es);
    L.off_b = take(L.n * es);
    L.off_r = take(L.n * es);
    if (L.coarsest) continue;
    L.off_btype = take(L.btype.size() * 4);
    L.off_btsid = take(L.bt_sid.size() * 4);
    L.off_btfac = take(L.bt_fac.size() * es);
    // rows longer than 16 entries on average over the cells: eight lanes per row
    double tot = 0.0;
    for (int64_t c = 0; c < L.n; ++c) tot += L.st_off[L.sid[c] + 1] - L.st_off[L.sid[c]];
    L.split = tot > 16.0 * (double)L.n ? 8 : 1;
    L.list.clear();
    if (L.split == 1) {
      const int nbx = L.nx / 2, nby = L.ny / 2, nbz = L.nz / 2;
      std::vector<int32_t> by_col[8];
      for (int bz = 0; bz < nbz; ++bz)
        for (int by = 0; by < nby; ++by)
          for (int bx = 0; bx < nbx; ++bx) {
            const int blk = bx + nbx * (by + nby * bz);
            if (L.bt_c7[L.btype[blk]] == 0.0)
              by_col[(bx & 1) + 2 * (by & 1) + 4 * (bz & 1)].push_back(blk);
          }
      for (int c = 0; c < 8; ++c) {
        L.list_off[c] = (int)L.list.size();
        L.list.insert(L.list.end(), by_col[c].begin(), by_col[c].end());
      }
      L.list_off[8] = (int)L.list.size();
    }
    L.off_list = take(std::max<size_t>(1, L.list.size()) * 4);
    L.off_btc7 = take(L.bt_c7.size() * es);
    L.off_btdiag = take(L.bt_diag.size() * es);
    L.off_stoff = take(L.st_off.size() * 4);
    L.off_ent = take((L.st_code.size() + kEntryPad) *
                     (f32 ? sizeof(StEntryT<float>) : sizeof(StEntryT<double>)));
  }
  C.off_ainv = take((size_t)C.ncd * C.ncd * 8);
  C.off_w = take((size_t)C.ncd * C.ncd * 8);
  C.off_part = take((size_t)((std::max(nbase, nf) + 255) / 256 + 1) * 8);
  C.off_norm = take(64);
  C.off_znoise = take((size_t)C.ncd * 8);
  C.ws_bytes = off;
  return SMG_OK;
}

NoiseArgs comp_noise(const Composite& C, uint64_t seed, uint64_t cycle, int level, int slot,
                     int colour, uint32_t kind) {
  NoiseArgs na;
  na.k0 = (uint32_t)seed;
  na.k1 = (uint32_t)(seed >> 32);
  na.sid = (uint32_t)level | ((uint32_t)slot << 4) | ((uint32_t)colour << 12) | (kind << 24);
  na.c2 = (uint32_t)cycle;
  na.c3 = (uint32_t)(cycle >> 32);
  na.sqkT = std::sqrt(C.kT);
  na.chains = nullptr;
  na.comps_per_chain = 1;
  na.cpc_magic = 0;
  na.bm = box_muller_coef();
  return na;
}

struct CRun {
  Composite* c;
  hipStream_t s;
  bool noise;
  uint64_t seed, cycle;
};

// fields and tables of a base level in the sweep precision
template <typename T>
struct LvF;
template <>
struct LvF<double> {
  static double* x(GLevel& L) { return L.x; }
  static double* b(GLevel& L) { return L.b; }
  static double* r(GLevel& L) { return L.r; }
  static const GStencilT<double>& st(GLevel& L) { return L.dev; }
};
template <>
struct LvF<float> {
  static float* x(GLevel& L) { return L.x32; }
  static float* b(GLevel& L) { return L.b32; }
  static float* r(GLevel& L) { return L.r32; }
  static const GStencilT<float>& st(GLevel& L) { return L.dev32; }
};

template <typename T>
int comp_class_pass(const CRun& r, int cls, int slot, T* xc, T* xf, const T* bc, const T* bf) {
  Composite& C = *r.c;
  const NoiseArgs na = comp_noise(C, r.seed, r.cycle, 0, slot, cls, KIND_COMP);
  if (cls < 2) {
    CMP_HIP(launch_comp_coarse_pass<T>(xc, bc, xf, C.g, cls, r.noise, na, r.s));
  } else if (cls < 4) {
    CMP_HIP(launch_comp_fine_pass<T>(xf, bf, C.g, cls - 2, r.noise, na, r.s));
  } else {
    const int p = cls - 4;
    CMP_HIP(launch_comp_layer_pass<T>(xf, bf, xc, C.g, C.layer_d + C.layer_off[p],
                                      C.layer_off[p + 1] - C.layer_off[p], r.noise, na, r.s));
  }
  return SMG_OK;
}

template <typename T>
int base_block_pass(const CRun& r, int l, int colour, int slot) {
  Composite& C = *r.c;
  GLevel& L = C.lv[l];
  const NoiseArgs na = comp_noise(C, r.seed, r.cycle, l, slot, colour, KIND_FAC_BASE);
  CMP_HIP(launch_gblock_pass<T>(LvF<T>::x(L), LvF<T>::b(L), LvF<T>::st(L), colour, r.noise, na,
                                r.s));
  return SMG_OK;
}

template <typename T>
int base_vcycle(const CRun& r, int l) {
  Composite& C = *r.c;
  GLevel& L = C.lv[l];
  if (L.coarsest) {
    const NoiseArgs na = comp_noise(C, r.seed, r.cycle, l, 0, 0, KIND_FAC_COARSEST);
    CMP_HIP(launch_dense_draw<T>(LvF<T>::x(L), LvF<T>::b(L), C.ainv_d, C.w_d, C.znoise, C.ncd,
                                 r.noise, na, r.s));
    return SMG_OK;
  }
  for (int s = 0; s < C.mu1; ++s)
    for (int c = 0; c < 8; ++c)
      if (int rc = base_block_pass<T>(r, l, c, s)) return rc;
  GLevel& K = C.lv[l + 1];
  CMP_HIP(launch_gresidual<T>(LvF<T>::r(L), LvF<T>::x(L), LvF<T>::b(L), LvF<T>::st(L), r.s));
  CMP_HIP(launch_restrict<T>(LvF<T>::b(K), LvF<T>::x(K), LvF<T>::r(L), L.nx, L.ny, L.nz, 1, r.s));
  if (int rc = base_vcycle<T>(r, l + 1)) return rc;
  CMP_HIP(launch_prolong<T>(LvF<T>::x(L), LvF<T>::x(K), L.nx, L.ny, L.nz, 1, r.s));
  for (int s = 0; s < C.mu2; ++s)
    for (int c = 7; c >= 0; --c)
      if (int rc = base_block_pass<T>(r, l, c, C.mu1 + s)) return rc;
  return SMG_OK;
}

// One FAC cycle in place in the sweep precision: b_0 = P^T (b - A x); y = V-cycle_0(0, b_0);
// x += P y; nu composite sweeps (gs_only: the sweeps alone).  rf: fine-residual scratch.
template <typename T>
int fac_cycle(const CRun& r, T* xc, T* xf, const T* bc, const T* bf, T* rf) {
  Composite& C = *r.c;
  GLevel& L0 = C.lv[0];
  if (!C.gs_only) {
    CMP_HIP(launch_comp_residual_restrict<T>(LvF<T>::b(L0), LvF<T>::x(L0), rf, xc, xf, bc, bf,
                                             C.g, r.s));
    if (int rc = base_vcycle<T>(r, 0)) return rc;
    CMP_HIP(launch_comp_prolong<T>(xc, xf, LvF<T>::x(L0), C.g, r.s));
  }
  for (int s = 0; s < C.nu; ++s)
    for (int cls = 0; cls < 12; ++cls)
      if (int rc = comp_class_pass<T>(r, cls, s, xc, xf, bc, bf)) return rc;
  return SMG_OK;
}

// The cycle on the caller's FP64 fields.  FP64 form: the cycle itself.  FP32-refined form (the
// correction form of the same affine cycle): r = b - A x in FP64, e = cycle_FP32(0, (float) r)
// with the same noise streams, x += e in FP64.
int run_cycle(const CRun& r, double* xc, double* xf, const double* bc, const double* bf) {
  Composite& C = *r.c;
  if (C.prec == SMG_FP64) return fac_cycle<double>(r, xc, xf, bc, bf, C.rf);
  const int64_t nbase = (int64_t)C.g.nx * C.g.ny * C.g.nz;
  const int64_t nf = (int64_t)C.g.fx * C.g.fy * C.g.fz;
  CMP_HIP(launch_comp_residual<double>(C.rc, C.rf, xc, xf, bc, bf, C.g, r.s));
  CMP_HIP(launch_cast(C.r32c, 1, C.rc, nbase, r.s));
  CMP_HIP(launch_cast(C.r32f, 1, C.rf, nf, r.s));
  CMP_HIP(launch_zero<float>(C.e32c, nbase, r.s));
  CMP_HIP(launch_zero<float>(C.e32f, nf, r.s));
  if (int rc = fac_cycle<float>(r, C.e32c, C.e32f, C.r32c, C.r32f, C.rf32)) return rc;
  CMP_HIP(launch_refine_update(xc, C.e32c, nbase, r.s));
  CMP_HIP(launch_refine_update(xf, C.e32f, nf, r.s));
  return SMG_OK;
}

bool aligned(const void* p) { return p && ((uintptr_t)p & 255) == 0; }

int check_bound(const smg_composite* h) {
  if (!h) {
    set_error("null composite");
    return SMG_EINVAL;
  }
  if (!h->c.ws) {
    set_error("composite has no workspace bound (call smg_composite_bind)");
    return SMG_ESTATE;
  }
  return SMG_OK;
}

// Solves A u = f from u = 0 with noise-free cycles until ||f - A u|| <= rtol ||f||; synchronises
// s after every cycle (the residual norm decides whether to continue).
int comp_solve(Composite& C, const double* fc, const double* ff, double* uc, double* uf,
               double rtol, int max_cycles, hipStream_t s, smg_solve_info* info) {
  const int64_t nbase = (int64_t)C.g.nx * C.g.ny * C.g.nz;
  const int64_t nf = (int64_t)C.g.fx * C.g.fy * C.g.fz;
  CMP_HIP(launch_zero<double>(uc, nbase, s));
  CMP_HIP(launch_zero<double>(uf, nf, s));
  auto resnorm = [&](double& out) -> int {
    CMP_HIP(launch_comp_residual(C.rc, C.rf, (const double*)uc, (const double*)uf, fc, ff,
                                 C.g, s));
    CMP_HIP(launch_sumsq(C.norm, C.part, C.rc, nbase, 1, s));
    CMP_HIP(launch_sumsq(C.norm + 1, C.part, C.rf, nf, 1, s));
    double hn[2];
    CMP_HIP(hipMemcpyAsync(hn, C.norm, 16, hipMemcpyDeviceToHost, s));
    CMP_HIP(hipStreamSynchronize(s));
    out = std::sqrt(hn[0] + hn[1]);
    return SMG_OK;
  };
  double f0, rn, prev;
  if (int e = resnorm(f0)) return e;
  smg_solve_info loc{0, 0.0, 0.0};
  if (!std::isfinite(f0)) {
    set_error("f is not finite");
    return SMG_ENONFINITE;
  }
  if (f0 == 0.0) {
    if (info) *info = loc;
    return SMG_OK;
  }
  prev = f0;
  int k = 0;
  double rel = 1.0;
  while (k < max_cycles) {
    CRun r{&C, s, false, 0, 0};
    if (int e = run_cycle(r, uc, uf, fc, ff)) return e;
    ++k;
    if (int e = resnorm(rn)) return e;
    if (!std::isfinite(rn)) {
      set_error("residual is not finite");
      return SMG_ENONFINITE;
    }
    rel = rn / f0;
    loc.last_ratio = k >= 2 ? rn / prev : 0.0;
    prev = rn;
    if (rel <= rtol) break;
  }
  loc.cycles = k;
  loc.relres = rel;
  if (info) *info = loc;
  if (rel > rtol) {
    set_error("solve did not converge: relres " + std::to_string(rel));
    return SMG_ENOTCONV;
  }
  return SMG_OK;
}

}  // namespace
}  // namespace smg

using smg::Composite;
using smg::set_error;

extern "C" {

int smg_composite_create(const smg_composite_desc* desc, const smg_fac_params* params,
                         smg_composite** out) {
  if (!desc || !params || !out) {
    set_error("null argument");
    return SMG_EINVAL;
  }
  *out = nullptr;
  smg_composite* h = new (std::nothrow) smg_composite();
  if (!h) {
    set_error("host allocation failed");
    return SMG_ENOMEM;
  }
  std::string err;
  int rc;
  try {
    rc = smg::plan(h->c, *desc, *params, err);
  } catch (const std::bad_alloc&) {
    rc = SMG_ENOMEM;
    err = "host allocation failed";
  }
  if (rc != SMG_OK) {
    set_error(err);
    delete h;
    return rc;
  }
  *out = h;
  set_error("");
  return SMG_OK;
}

int smg_composite_get_info(const smg_composite* h, smg_composite_info* info) {
  if (!h || !info) {
    set_error("null argument");
    return SMG_EINVAL;
  }
  const Composite& C = h->c;
  std::memset(info, 0, sizeof(*info));
  info->workspace_bytes = C.ws_bytes;
  info->base_cells = (int64_t)C.g.nx * C.g.ny * C.g.nz;
  info->fine_cells = (int64_t)C.g.fx * C.g.fy * C.g.fz;
  info->unknowns = info->base_cells -
                   (int64_t)(C.g.x1 - C.g.x0) * (C.g.y1 - C.g.y0) * (C.g.z1 - C.g.z0) +
                   info->fine_cells;
  info->fine_dims[0] = C.g.fx;
  info->fine_dims[1] = C.g.fy;
  info->fine_dims[2] = C.g.fz;
  info->n_levels = (int32_t)C.lv.size();
  for (size_t l = 0; l < C.lv.size(); ++l) {
    info->dims[l][0] = C.lv[l].nx;
    info->dims[l][1] = C.lv[l].ny;
    info->dims[l][2] = C.lv[l].nz;
    info->stencils[l] = (int32_t)C.lv[l].st_off.size() - 1;
    info->block_types[l] = (int32_t)(C.lv[l].bt_sid.size() / 8);
  }
  info->layer_cells = (int32_t)C.layer.size();
  info->coarsest_unknowns = C.ncd;
  return SMG_OK;
}

int smg_composite_bind(smg_composite* h, void* dev_ptr, size_t bytes, void* stream) {
  if (!h) {
    set_error("null composite");
    return SMG_EINVAL;
  }
  Composite& C = h->c;
  if (!smg::aligned(dev_ptr)) {
    set_error("workspace must be a non-null 256-byte aligned device pointer");
    return SMG_EINVAL;
  }
  if (bytes < C.ws_bytes) {
    set_error("workspace too small: need " + std::to_string(C.ws_bytes) + " bytes");
    return SMG_ENOMEM;
  }
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)dev_ptr;
  auto up = [&](size_t off, const void* src, size_t n) -> hipError_t {
    if (n == 0) return hipSuccess;
    return hipMemcpyAsync(ws + off, src, n, hipMemcpyHostToDevice, s);
  };
  CMP_HIP(up(C.off_layer, C.layer.data(), C.layer.size() * 4));
  const bool f32 = C.prec == SMG_FP32_REFINED;
  // host staging of converted tables, alive until the synchronisation below
  std::vector<std::vector<float>> keep32;
  std::vector<std::vector<smg::StEntryT<float>>> keepe32;
  std::vector<std::vector<smg::StEntryT<double>>> keepe64;
  keep32.reserve(4 * C.lv.size());
  keepe32.reserve(C.lv.size());
  keepe64.reserve(C.lv.size());
  auto as32 = [&](const std::vector<double>& v) -> const float* {
    keep32.emplace_back(v.begin(), v.end());
    return keep32.back().data();
  };
  for (auto& L : C.lv) {
    if (f32) {
      L.x32 = (float*)(ws + L.off_x);
      L.b32 = (float*)(ws + L.off_b);
      L.r32 = (float*)(ws + L.off_r);
    } else {
      L.x = (double*)(ws + L.off_x);
      L.b = (double*)(ws + L.off_b);
      L.r = (double*)(ws + L.off_r);
    }
    if (L.coarsest) continue;
    CMP_HIP(up(L.off_btype, L.btype.data(), L.btype.size() * 4));
    CMP_HIP(up(L.off_btsid, L.bt_sid.data(), L.bt_sid.size() * 4));
    CMP_HIP(up(L.off_list, L.list.data(), L.list.size() * 4));
    for (int c = 0; c < 9; ++c) {
      L.dev.list_off[c] = L.list_off[c];
      L.dev32.list_off[c] = L.list_off[c];
    }
    L.dev.list = (const int32_t*)(ws + L.off_list);
    L.dev32.list = (const int32_t*)(ws + L.off_list);
    if (f32) {
      CMP_HIP(up(L.off_stoff, L.st_off.data(), L.st_off.size() * 4));
      CMP_HIP(up(L.off_btfac, as32(L.bt_fac), L.bt_fac.size() * 4));
      CMP_HIP(up(L.off_btc7, as32(L.bt_c7), L.bt_c7.size() * 4));
      CMP_HIP(up(L.off_btdiag, as32(L.bt_diag), L.bt_diag.size() * 4));
      keepe32.emplace_back(L.st_code.size() + smg::kEntryPad, smg::StEntryT<float>{});
      for (size_t e = 0; e < L.st_code.size(); ++e)
        keepe32.back()[e] = device_entry<float>(L, e);
      CMP_HIP(up(L.off_ent, keepe32.back().data(),
                 keepe32.back().size() * sizeof(smg::StEntryT<float>)));
      smg::GStencilT<float>& d = L.dev32;
      d.btype = (const int32_t*)(ws + L.off_btype);
      d.bt_sid = (const int32_t*)(ws + L.off_btsid);
      d.st_off = (const int32_t*)(ws + L.off_stoff);
      d.bt_fac = (const float*)(ws + L.off_btfac);
      d.ent = (const smg::StEntryT<float>*)(ws + L.off_ent);
      d.bt_c7 = (const float*)(ws + L.off_btc7);
      d.bt_diag = (const float*)(ws + L.off_btdiag);
      d.nx = L.nx;
      d.ny = L.ny;
      d.nz = L.nz;
      d.split = L.split;
      d.row_lanes = C.row_lanes;
      continue;
    }
    CMP_HIP(up(L.off_btfac, L.bt_fac.data(), L.bt_fac.size() * 8));

    CMP_HIP(up(L.off_stoff, L.st_off.data(), L.st_off.size() * 4));
    keepe64.emplace_back(L.st_code.size() + smg::kEntryPad, smg::StEntryT<double>{});
    for (size_t e = 0; e < L.st_code.size(); ++e)
      keepe64.back()[e] = device_entry<double>(L, e);
    CMP_HIP(up(L.off_ent, keepe64.back().data(),
               keepe64.back().size() * sizeof(smg::StEntryT<double>)));
    CMP_HIP(up(L.off_btc7, L.bt_c7.data(), L.bt_c7.size() * 8));
    CMP_HIP(up(L.off_btdiag, L.bt_diag.data(), L.bt_diag.size() * 8));
    L.dev.btype = (const int32_t*)(ws + L.off_btype);
    L.dev.bt_sid = (const int32_t*)(ws + L.off_btsid);
    L.dev.bt_fac = (const double*)(ws + L.off_btfac);
    L.dev.st_off = (const int32_t*)(ws + L.off_stoff);
    L.dev.ent = (const smg::StEntryT<double>*)(ws + L.off_ent);
    L.dev.split = L.split;
    L.dev.row_lanes = C.row_lanes;
    L.dev.bt_c7 = (const double*)(ws + L.off_btc7);
    L.dev.bt_diag = (const double*)(ws + L.off_btdiag);
    L.dev.nx = L.nx;
    L.dev.ny = L.ny;
    L.dev.nz = L.nz;
  }
  CMP_HIP(up(C.off_ainv, C.ainv.data(), C.ainv.size() * 8));
  CMP_HIP(up(C.off_w, C.w.data(), C.w.size() * 8));
  CMP_HIP(hipStreamSynchronize(s));
  CMP_HIP(hipGetDevice(&C.device));
  C.ws = ws;
  C.rc = (double*)(ws + C.off_rc);
  C.rf = (double*)(ws + C.off_rf);
  C.layer_d = (int32_t*)(ws + C.off_layer);
  C.ainv_d = (double*)(ws + C.off_ainv);
  C.w_d = (double*)(ws + C.off_w);
  C.part = (double*)(ws + C.off_part);
  C.norm = (double*)(ws + C.off_norm);
  C.znoise = (double*)(ws + C.off_znoise);
  if (f32) {
    C.e32c = (float*)(ws + C.off_e32c);
    C.e32f = (float*)(ws + C.off_e32f);
    C.r32c = (float*)(ws + C.off_r32c);
    C.r32f = (float*)(ws + C.off_r32f);
    C.rf32 = (float*)(ws + C.off_rf32);
  }
  return SMG_OK;
}

int smg_composite_cycle(smg_composite* h, void* xc, void* xf, const void* bc, const void* bf,
                        uint64_t seed, uint64_t cycle, int32_t with_noise, void* stream) {
  if (int rc = smg::check_bound(h)) return rc;
  if (!smg::aligned(xc) || !smg::aligned(xf) || (bc && !smg::aligned(bc)) ||
      (bf && !smg::aligned(bf)) || (bc == nullptr) != (bf == nullptr)) {
    set_error("xc, xf (and bc, bf if given) must be 256-byte aligned device pointers");
    return SMG_EINVAL;
  }
  smg::CRun r{&h->c, (hipStream_t)stream, with_noise != 0, seed, cycle};
  return smg::run_cycle(r, (double*)xc, (double*)xf, (const double*)bc, (const double*)bf);
}

int smg_composite_sample(smg_composite* h, int64_t ncycles, uint64_t seed, uint64_t first_cycle,
                         void* xc, void* xf, void* stream) {
  if (int rc = smg::check_bound(h)) return rc;
  if (ncycles < 0 || !smg::aligned(xc) || !smg::aligned(xf)) {
    set_error("ncycles must be >= 0 and xc, xf 256-byte aligned device pointers");
    return SMG_EINVAL;
  }
  for (int64_t k = 0; k < ncycles; ++k) {
    smg::CRun r{&h->c, (hipStream_t)stream, true, seed, first_cycle + (uint64_t)k};
    if (int rc = smg::run_cycle(r, (double*)xc, (double*)xf, nullptr, nullptr)) return rc;
  }
  return SMG_OK;
}

int smg_composite_residual(smg_composite* h, const void* xc, const void* xf, const void* bc,
                           const void* bf, void* rc, void* rf, void* stream) {
  if (int e = smg::check_bound(h)) return e;
  if (!smg::aligned(xc) || !smg::aligned(xf) || !smg::aligned(rc) || !smg::aligned(rf) ||
      (bc == nullptr) != (bf == nullptr)) {
    set_error("invalid field pointers");
    return SMG_EINVAL;
  }
  CMP_HIP(smg::launch_comp_residual((double*)rc, (double*)rf, (const double*)xc,
                                    (const double*)xf, (const double*)bc, (const double*)bf,
                                    h->c.g, (hipStream_t)stream));
  return SMG_OK;
}

int smg_composite_solve(smg_composite* h, const void* fc, const void* ff, void* uc, void* uf,
                        double rtol, int32_t max_cycles, void* stream, smg_solve_info* info) {
  if (int e = smg::check_bound(h)) return e;
  if (!smg::aligned(fc) || !smg::aligned(ff) || !smg::aligned(uc) || !smg::aligned(uf) ||
      !(rtol >= 0.0) || max_cycles < 0) {
    set_error("invalid solve arguments");
    return SMG_EINVAL;
  }
  return smg::comp_solve(h->c, (const double*)fc, (const double*)ff, (double*)uc, (double*)uf,
                         rtol, max_cycles, (hipStream_t)stream, info);
}

int smg_composite_forced_field(smg_composite* h, int64_t n, uint64_t seed, uint64_t first_sample,
                               const void* qc, const void* qf, void* wc, void* wf, double rtol,
                               int32_t max_cycles, void* stream, smg_solve_info* infos) {
  if (int e = smg::check_bound(h)) return e;
  if (n < 0 || (n > 0 && (!smg::aligned(wc) || !smg::aligned(wf))) ||
      (qc && !smg::aligned(qc)) || (qf && !smg::aligned(qf)) || !(rtol >= 0.0) ||
      max_cycles < 0) {
    set_error("invalid forced-field arguments (n >= 0; wc, wf and given qc, qf 256-byte aligned "
              "device pointers; rtol >= 0; max_cycles >= 0)");
    return SMG_EINVAL;
  }
  Composite& C = h->c;
  hipStream_t s = (hipStream_t)stream;
  const int64_t nbase = (int64_t)C.g.nx * C.g.ny * C.g.nz;
  const int64_t nf = (int64_t)C.g.fx * C.g.fy * C.g.fz;
  double* fc = (double*)(C.ws + C.off_fc);
  double* ff = (double*)(C.ws + C.off_ff);
  for (int64_t i = 0; i < n; ++i) {
    const uint64_t sample = first_sample + (uint64_t)i;
    smg::NoiseArgs nac = smg::comp_noise(C, seed, sample, 0, 0, 0, smg::KIND_FORCING);
    smg::NoiseArgs naf = smg::comp_noise(C, seed, sample, 0, 0, 1, smg::KIND_FORCING);
    CMP_HIP(smg::launch_comp_forcing(fc, ff, (const double*)qc, (const double*)qf, C.g, nac, naf,
                                     s));
    if (int e = smg::comp_solve(C, fc, ff, (double*)wc + i * nbase, (double*)wf + i * nf, rtol,
                                max_cycles, s, infos ? infos + i : nullptr))
      return e;
  }
  return SMG_OK;
}

int smg_composite_debug_pass(smg_composite* h, int32_t cls, void* xc, void* xf, const void* bc,
                             const void* bf, uint64_t seed, uint64_t cycle, int32_t slot,
                             int32_t with_noise, void* stream) {
  if (int e = smg::check_bound(h)) return e;
  if (h->c.prec != SMG_FP64) {
    set_error("component entry points need a composite created with SMG_FP64");
    return SMG_EINVAL;
  }
  if (cls < 0 || cls >= 12 || slot < 0 || slot > 255 || !smg::aligned(xc) || !smg::aligned(xf)) {
    set_error("invalid class, slot or field pointers");
    return SMG_EINVAL;
  }
  smg::CRun r{&h->c, (hipStream_t)stream, with_noise != 0, seed, cycle};
  return smg::comp_class_pass<double>(r, cls, slot, (double*)xc, (double*)xf, (const double*)bc,
                              (const double*)bf);
}

int smg_composite_debug_base_pass(smg_composite* h, int32_t level, int32_t colour, void* x,
                                  const void* b, uint64_t seed, uint64_t cycle, int32_t slot,
                                  int32_t with_noise, void* stream) {
  if (int e = smg::check_bound(h)) return e;
  Composite& C = h->c;
  if (C.prec != SMG_FP64) {
    set_error("component entry points need a composite created with SMG_FP64");
    return SMG_EINVAL;
  }
  if (level < 0 || level >= (int)C.lv.size() || C.lv[level].coarsest || colour < 0 ||
      colour > 7 || slot < 0 || slot > 255 || !smg::aligned(x) || (b && !smg::aligned(b))) {
    set_error("invalid level, colour, slot or field pointers");
    return SMG_EINVAL;
  }
  smg::GLevel& L = C.lv[level];
  const smg::NoiseArgs na =
      smg::comp_noise(C, seed, cycle, level, slot, colour, smg::KIND_FAC_BASE);
  CMP_HIP(smg::launch_gblock_pass<double>((double*)x, (const double*)b, L.dev, colour, with_noise != 0,
                                  na, (hipStream_t)stream));
  return SMG_OK;
}

int smg_composite_debug_row(const smg_composite* h, int32_t level, int64_t cell,
                            int64_t* targets, double* vals, int32_t* count) {
  if (!h || !targets || !vals || !count) {
    set_error("null argument");
    return SMG_EINVAL;
  }
  const Composite& C = h->c;
  if (level < 0 || level >= (int)C.lv.size() || cell < 0 || cell >= C.lv[level].n) {
    set_error("invalid level or cell");
    return SMG_EINVAL;
  }
  const smg::GLevel& L = C.lv[level];
  const int x = (int)(cell % L.nx), y = (int)((cell / L.nx) % L.ny), z = (int)(cell / ((int64_t)L.nx * L.ny));
  const int s = L.sid[cell];
  int c = 0;
  for (int e = L.st_off[s]; e < L.st_off[s + 1]; ++e, ++c) {
    const int code = L.st_code[e];
    const int tx = smg::wrap(x + code % 5 - 2, L.nx), ty = smg::wrap(y + (code / 5) % 5 - 2, L.ny);
    const int tz = z + code / 25 - 2;
    targets[c] = tx + (int64_t)L.nx * (ty + (int64_t)L.ny * tz);
    vals[c] = L.st_val[e];
  }
  *count = c;
  return SMG_OK;
}

void smg_composite_destroy(smg_composite* h) { delete h; }

}  // extern "C"
