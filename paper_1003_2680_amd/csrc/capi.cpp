// C-ABI entry points and the host-side cycle driver.
//
// The V-cycle follows Alg. 3 of the paper: nu1 pre-sweeps; b^(l+1) = P^T (b^(l) - A^(l) v^(l));
// v^(l+1) = 0; recurse; v^(l) += P v^(l+1); nu2 post-sweeps.  The coarsest level is either an
// exact draw (dense Cholesky) or nu1 + nu2 sweeps.  Sampling runs the cycle with b = 0 and the
// noise on (target N(0, kT A^-1)); the solve runs it with the noise off from u = 0 (its fixed
// point is A^-1 f).  Noise counters: level | slot<<4 | colour<<12 | comp<<16 | kind<<24, where
// slot is the sweep number within the level's visit (pre-sweeps first) and kind is 0 for
// smoother noise, 1 for the coarsest draw.
//
// SMG_FP32_REFINED runs the same cycle in correction form (Alg. 1, with the residual
// r = b - A x): per cycle r = b - A x in FP64, e = V-cycle(e = 0, rhs r) with FP32 sweeps and
// transfers (FP64 coarsest arithmetic), x += e in FP64.  In exact arithmetic this is the same
// chain: every step of the cycle is affine in (x, b), so running it on (x, b) equals x plus
// running it on (0, b - A x).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "smg_internal.hpp"

struct smg_hierarchy {
  smg::Hierarchy h;
};

namespace smg {
namespace {

thread_local std::string g_err;

#define SMG_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));                \
      return SMG_EHIP;                                                             \
    }                                                                              \
  } while (0)

#define SMG_TRY(expr)              \
  do {                             \
    int rc_ = (expr);              \
    if (rc_ != SMG_OK) return rc_; \
  } while (0)

constexpr uint32_t KIND_SMOOTH_NOISE = 0;
constexpr uint32_t KIND_COARSEST_NOISE = 1;

struct Run {
  Hierarchy* h;
  hipStream_t s;
  bool noise;
  bool has_b0;  // level-0 right-hand side present (solve, and the refined inner cycle)
  uint64_t seed;
  uint64_t cycle;
};

NoiseArgs make_noise(const Run& r, int level, int slot, int colour, uint32_t kind) {
  NoiseArgs na;
  na.k0 = (uint32_t)r.seed;
  na.k1 = (uint32_t)(r.seed >> 32);
  na.sid = (uint32_t)level | ((uint32_t)slot << 4) | ((uint32_t)colour << 12) | (kind << 24);
  na.c2 = (uint32_t)r.cycle;
  na.c3 = (uint32_t)(r.cycle >> 32);
  na.sqkT = std::sqrt(r.h->desc.kT);
  return na;
}

bool refined(const Hierarchy& h) { return h.prm.precision == SMG_FP32_REFINED; }

size_t half_field(const Hierarchy& h) { return (size_t)h.desc.ncomp * (h.lv[0].n / 2); }

// The fields a sweep of precision T works on: FP64 mode x, b, r; refined mode xf, bf, rf.
template <typename T>
struct Fld;
template <>
struct Fld<double> {
  static double* x(Level& v) { return v.x; }
  static double* b(Level& v) { return v.b; }
  static double* r(Level& v) { return v.r; }
};
template <>
struct Fld<float> {
  static float* x(Level& v) { return v.xf; }
  static float* b(Level& v) { return v.bf; }
  static float* r(Level& v) { return v.rf; }
};

// Events around one launch of the timed kernel class (measurement support).
struct TimedScope {
  Hierarchy& h;
  hipStream_t s;
  hipEvent_t e1 = nullptr;
  int rc = SMG_OK;
  TimedScope(Hierarchy& hh, hipStream_t ss, int kind) : h(hh), s(ss) {
    if (!h.timing || h.timed_kernel != kind) return;
    if (h.ev_used + 2 > h.ev_pool.size()) {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) {
          set_error("hipEventCreate failed");
          rc = SMG_EHIP;
          return;
        }
        h.ev_pool.push_back(e);
      }
    }
    hipEvent_t e0 = h.ev_pool[h.ev_used++];
    e1 = h.ev_pool[h.ev_used++];
    if (hipEventRecord(e0, s) != hipSuccess) {
      set_error("hipEventRecord failed");
      rc = SMG_EHIP;
    }
  }
  int close() {
    if (rc == SMG_OK && e1 && hipEventRecord(e1, s) != hipSuccess) {
      set_error("hipEventRecord failed");
      rc = SMG_EHIP;
    }
    return rc;
  }
};

template <typename T>
int timed_rb_pass(Run& r, T* xc, const T* xo, const T* bc, int colour, const NoiseArgs& na) {
  Hierarchy& h = *r.h;
  const Level& v = h.lv[0];
  TimedScope ts(h, r.s, SMG_TIMED_FINE_PASS);
  SMG_TRY(ts.rc);
  SMG_HIP(launch_rb_pass<T>(xc, xo, bc, v.nx, v.ny, v.nz, h.desc.ncomp, colour, h.desc.h,
                            h.desc.kT, r.noise, na, r.s));
  return ts.close();
}

template <typename T>
int sweep(Run& r, int l, int slot, bool post) {
  Hierarchy& h = *r.h;
  Level& v = h.lv[l];
  const int nc = h.desc.ncomp;
  if (v.kind == KIND_POINT) {
    T* xr = Fld<T>::x(v);
    T* xb = xr + half_field(h);
    const T* br = Fld<T>::b(v);
    const T* bb = br + half_field(h);
    for (int t = 0; t < 2; ++t) {
      const int colour = post ? 1 - t : t;
      NoiseArgs na = make_noise(r, l, slot, colour, KIND_SMOOTH_NOISE);
      const T* bc = r.has_b0 ? (colour ? bb : br) : nullptr;
      SMG_TRY(timed_rb_pass<T>(r, colour ? xb : xr, colour ? xr : xb, bc, colour, na));
    }
  } else {
    const T* noise = (const T*)v.noise_d;
    for (int t = 0; t < 8; ++t) {
      const int colour = post ? 7 - t : t;
      const T* zn = r.noise ? noise + (size_t)slot * nc * v.n : nullptr;
      TimedScope ts(h, r.s, l == 1 ? SMG_TIMED_LEVEL1_BLOCK_PASS : -1);
      SMG_TRY(ts.rc);
      SMG_HIP(launch_block_pass<T>(Fld<T>::x(v), Fld<T>::b(v), (const T*)v.g2d_d,
                                   (const T*)v.zt_d, (const T*)v.bfac_d, v.nx, v.ny, v.nz, nc,
                                   colour, zn, std::sqrt(h.desc.kT), r.s));
      SMG_TRY(ts.close());
    }
  }
  return SMG_OK;
}

// b^(l+1) = P^T (b^(l) - A^(l) x^(l)); the coarse iterate starts from zero
template <typename T>
int restrict_residual(Run& r, int l) {
  Hierarchy& h = *r.h;
  Level& v = h.lv[l];
  const int nc = h.desc.ncomp;
  T* rr = Fld<T>::r(v);
  if (v.kind == KIND_POINT) {
    T* xr = Fld<T>::x(v);
    T* br = Fld<T>::b(v);
    SMG_HIP(launch_residual0<T>(rr, xr, xr + half_field(h), r.has_b0 ? br : nullptr,
                                r.has_b0 ? br + half_field(h) : nullptr, v.nx, v.ny, v.nz, nc,
                                h.desc.h, r.s));
  } else {
    SMG_HIP(launch_residual_gal<T>(rr, Fld<T>::x(v), Fld<T>::b(v), (const T*)v.g2d_d,
                                   (const T*)v.zt_d, v.nx, v.ny, v.nz, nc, r.s));
  }
  Level& c = h.lv[l + 1];
  const bool bottom_next = (l + 1 == h.bottom) && h.use_bottom;
  SMG_HIP(launch_restrict<T>(Fld<T>::b(c), bottom_next ? nullptr : Fld<T>::x(c), rr, v.nx, v.ny,
                             v.nz, nc, r.s));
  return SMG_OK;
}

template <typename T>
int prolong_add(Run& r, int l) {
  Hierarchy& h = *r.h;
  Level& v = h.lv[l];
  const int nc = h.desc.ncomp;
  const T* e = Fld<T>::x(h.lv[l + 1]);
  if (v.kind == KIND_POINT) {
    T* xr = Fld<T>::x(v);
    SMG_HIP(launch_prolong0<T>(xr, xr + half_field(h), e, v.nx, v.ny, v.nz, nc, r.s));
  } else {
    SMG_HIP(launch_prolong<T>(Fld<T>::x(v), e, v.nx, v.ny, v.nz, nc, r.s));
  }
  return SMG_OK;
}

template <typename T>
int coarsest_step(Run& r, int l) {
  Hierarchy& h = *r.h;
  Level& v = h.lv[l];
  NoiseArgs na = make_noise(r, l, 0, 0, KIND_COARSEST_NOISE);
  SMG_HIP(launch_coarsest<T>(Fld<T>::x(v), Fld<T>::b(v), h.ainv_d, h.w_d, h.nc, h.desc.ncomp,
                             r.noise, na, r.s));
  return SMG_OK;
}

// Noise of every sweep of every block level for the cycle r.cycle, in one launch (or of one
// level and slot when only_level >= 0).
template <typename T>
int gen_level_noise(Run& r, int only_level = -1, int only_slot = 0) {
  Hierarchy& h = *r.h;
  NoiseGenArgs a{};
  a.ncomp = h.desc.ncomp;
  uint32_t calls = 0;
  for (int l = 0; l < (int)h.lv.size(); ++l) {
    const Level& v = h.lv[l];
    if (v.kind != KIND_BLOCK || (only_level >= 0 && l != only_level)) continue;
    if (a.nlev == kMaxNoiseLevels) {
      set_error("too many block levels");
      return SMG_EINVAL;
    }
    NoiseLevel& e = a.lv[a.nlev++];
    e.level = l;
    e.nx = v.nx;
    e.ny = v.ny;
    e.nz = v.nz;
    e.nslot = only_level >= 0 ? 1 : h.prm.nu1 + h.prm.nu2;
    e.slot0 = only_level >= 0 ? only_slot : 0;
    e.out = v.noise_d;
    e.calls_before = calls;
    calls += (uint32_t)(e.nslot * a.ncomp * (v.n / 2));
  }
  if (a.nlev == 0) return SMG_OK;
  a.total = calls;
  NoiseArgs na = make_noise(r, 0, 0, 0, KIND_SMOOTH_NOISE);
  SMG_HIP(launch_level_noise<T>(a, na, r.s));
  return SMG_OK;
}

// Level descriptors of the bottom kernel (device pointers are known once bound).
BotArgs make_botargs(Hierarchy& h) {
  BotArgs a{};
  const bool f32 = refined(h);
  a.nlev = (int)h.lv.size() - h.bottom;
  a.level0 = h.bottom;
  a.nu1 = h.prm.nu1;
  a.nu2 = h.prm.nu2;
  a.ncomp = h.desc.ncomp;
  int off = 0;
  for (int i = 0; i < a.nlev; ++i) {
    const Level& v = h.lv[h.bottom + i];
    int sy, sz;
    bot_strides(v.kind, v.nx, v.ny, sy, sz);
    a.lv[i] = BotLevel{v.nx, v.ny, v.nz, v.kind, sy, sz, v.noise_d, v.g2d_d, v.zt_d, v.bfac_d};
    a.lds_off[i] = off;
    off += 3 * (int)bot_field_elems(v.kind, v.nx, v.ny, v.nz);
  }
  for (int i = 0; i < a.nlev; ++i) {
    const Level& v = h.lv[h.bottom + i];
    a.tab_off[i] = off;
    if (v.kind == KIND_BLOCK) off += 50 + v.nz * 10 + (v.nz / 2) * 192;
  }
  Level& b0 = h.lv[h.bottom];
  a.b_in = f32 ? (const void*)b0.bf : (const void*)b0.b;
  a.x_out = f32 ? (void*)b0.xf : (void*)b0.x;
  a.ainv = h.ainv_d;
  a.w = h.w_d;
  return a;
}

// Every level from h.bottom down, in one launch (LDS-resident, one work-group per component).
template <typename T>
int bottom_cycle(Run& r) {
  Hierarchy& h = *r.h;
  NoiseArgs na = make_noise(r, 0, 0, 0, KIND_SMOOTH_NOISE);
  TimedScope ts(h, r.s, SMG_TIMED_BOTTOM);
  SMG_TRY(ts.rc);
  SMG_HIP(launch_bottom<T>(h.botargs_d, h.desc.ncomp, h.bottom_lds, r.noise, na, r.s));
  return ts.close();
}

template <typename T>
int vcycle(Run& r, int l) {
  Hierarchy& h = *r.h;
  Level& v = h.lv[l];
  const int nu1 = h.prm.nu1, nu2 = h.prm.nu2;
  if (l == h.bottom && h.use_bottom) return bottom_cycle<T>(r);
  if (v.kind == KIND_CHOL) return coarsest_step<T>(r, l);
  for (int s = 0; s < nu1; ++s) SMG_TRY(sweep<T>(r, l, s, false));
  if (!v.coarsest) {
    SMG_TRY(restrict_residual<T>(r, l));
    Level& c = h.lv[l + 1];
    if (l + 1 == h.bottom && !h.use_bottom)
      SMG_HIP(launch_zero<T>(Fld<T>::x(c), (int64_t)h.desc.ncomp * c.n, r.s));
    SMG_TRY(vcycle<T>(r, l + 1));
    SMG_TRY(prolong_add<T>(r, l));
  }
  for (int s = 0; s < nu2; ++s) SMG_TRY(sweep<T>(r, l, nu1 + s, true));
  return SMG_OK;
}

// One cycle on the FP64 level-0 state x.  Refined mode: residual_ready says that lv[0].bf
// already holds the FP32 residual of the current x (the solve computes it with the norms).
int full_cycle(Run& r, bool residual_ready = false) {
  Hierarchy& h = *r.h;
  Level& v0 = h.lv[0];
  if (!refined(h)) {
    if (r.noise) SMG_TRY(gen_level_noise<double>(r));
    return vcycle<double>(r, 0);
  }
  if (r.noise) SMG_TRY(gen_level_noise<float>(r));
  if (!residual_ready)
    SMG_HIP(launch_refine_residual(v0.bf, v0.x, r.has_b0 ? v0.b : nullptr, v0.nx, v0.ny, v0.nz,
                                   h.desc.ncomp, h.desc.h, nullptr, nullptr, r.s));
  SMG_HIP(launch_zero<float>(v0.xf, (int64_t)2 * half_field(h), r.s));
  Run ri = r;
  ri.has_b0 = true;
  SMG_TRY(vcycle<float>(ri, 0));
  SMG_HIP(launch_refine_update(v0.x, v0.xf, (int64_t)2 * half_field(h), r.s));
  return SMG_OK;
}

// natural [ncomp][N] field -> level-0 storage (x or b)
int import_level0(Hierarchy& h, double* dst, const double* nat, hipStream_t s) {
  Level& v = h.lv[0];
  if (v.kind == KIND_POINT)
    SMG_HIP(launch_to_split(dst, dst + half_field(h), nat, v.nx, v.ny, v.nz, h.desc.ncomp, s));
  else
    SMG_HIP(launch_copy(dst, nat, (int64_t)h.desc.ncomp * v.n, s));
  return SMG_OK;
}

int export_level0(Hierarchy& h, void* nat, int out_f32, const double* src, hipStream_t s) {
  Level& v = h.lv[0];
  if (v.kind == KIND_POINT)
    SMG_HIP(launch_from_split(nat, out_f32, src, src + half_field(h), v.nx, v.ny, v.nz,
                              h.desc.ncomp, s));
  else
    SMG_HIP(launch_cast(nat, out_f32, src, (int64_t)h.desc.ncomp * v.n, s));
  return SMG_OK;
}

bool aligned(const void* p) { return ((uintptr_t)p & 255u) == 0; }

int check_bound(const smg_hierarchy* hh) {
  if (!hh) {
    set_error("null hierarchy");
    return SMG_EINVAL;
  }
  if (!hh->h.ws) {
    set_error("hierarchy has no workspace bound (call smg_bind_workspace)");
    return SMG_ESTATE;
  }
  return SMG_OK;
}

int check_ptr(const void* p, const char* what) {
  if (!p || !aligned(p)) {
    set_error(std::string(what) + " must be a non-null 256-byte aligned device pointer");
    return SMG_EINVAL;
  }
  return SMG_OK;
}

// The per-component entry points drive the FP64 kernels on FP64 level storage.
int check_fp64(const Hierarchy& h) {
  if (refined(h)) {
    set_error("component entry points need a hierarchy created with SMG_FP64");
    return SMG_EINVAL;
  }
  return SMG_OK;
}

// Block-level tables in the sweep precision T (rounded from the FP64 tables in refined mode).
template <typename T>
int upload_tables(Level& v, char* ws, hipStream_t s) {
  std::vector<T> g(v.g2d.begin(), v.g2d.end());
  std::vector<T> z(v.zt.begin(), v.zt.end());
  std::vector<T> b(v.bfac.begin(), v.bfac.end());
  v.g2d_d = ws + v.off_g2d;
  v.zt_d = ws + v.off_zt;
  v.bfac_d = ws + v.off_bfac;
  v.noise_d = ws + v.off_noise;
  SMG_HIP(hipMemcpyAsync(v.g2d_d, g.data(), g.size() * sizeof(T), hipMemcpyHostToDevice, s));
  SMG_HIP(hipMemcpyAsync(v.zt_d, z.data(), z.size() * sizeof(T), hipMemcpyHostToDevice, s));
  SMG_HIP(hipMemcpyAsync(v.bfac_d, b.data(), b.size() * sizeof(T), hipMemcpyHostToDevice, s));
  // the staging vectors die on return
  SMG_HIP(hipStreamSynchronize(s));
  return SMG_OK;
}

}  // namespace

void set_error(const std::string& msg) { g_err = msg; }

}  // namespace smg

using namespace smg;

extern "C" {

int smg_create_hierarchy(const smg_grid_desc* desc, const smg_cycle_params* params,
                         smg_hierarchy** out) {
  if (!desc || !params || !out) {
    set_error("null argument");
    return SMG_EINVAL;
  }
  *out = nullptr;
  smg_hierarchy* hh = new (std::nothrow) smg_hierarchy();
  if (!hh) {
    set_error("host allocation failed");
    return SMG_ENOMEM;
  }
  std::string err;
  int rc = build_plan(*desc, *params, hh->h, err);
  if (rc != SMG_OK) {
    set_error(err);
    delete hh;
    return rc;
  }
  *out = hh;
  return SMG_OK;
}

int smg_hierarchy_info(const smg_hierarchy* hh, smg_info* info) {
  if (!hh || !info) {
    set_error("null argument");
    return SMG_EINVAL;
  }
  const Hierarchy& h = hh->h;
  std::memset(info, 0, sizeof(*info));
  info->workspace_bytes = h.ws_bytes;
  info->state_bytes = (size_t)h.desc.ncomp * h.lv[0].n * sizeof(double);
  info->n_levels = (int32_t)h.lv.size();
  for (size_t l = 0; l < h.lv.size() && l < 16; ++l) {
    info->dims[l][0] = h.lv[l].nx;
    info->dims[l][1] = h.lv[l].ny;
    info->dims[l][2] = h.lv[l].nz;
  }
  info->coarsest_unknowns = (int32_t)h.lv.back().n;
  return SMG_OK;
}

int smg_bind_workspace(smg_hierarchy* hh, void* dev_ptr, size_t bytes, void* stream) {
  if (!hh) {
    set_error("null hierarchy");
    return SMG_EINVAL;
  }
  SMG_TRY(check_ptr(dev_ptr, "workspace"));
  Hierarchy& h = hh->h;
  if (bytes < h.ws_bytes) {
    set_error("workspace too small: need " + std::to_string(h.ws_bytes) + " bytes");
    return SMG_ENOMEM;
  }
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)dev_ptr;
  const bool f32 = refined(h);
  SMG_HIP(hipGetDevice(&h.device));
  for (size_t l = 0; l < h.lv.size(); ++l) {
    Level& v = h.lv[l];
    if (!f32 || l == 0) {
      v.x = (double*)(ws + v.off_x);
      v.b = (double*)(ws + v.off_b);
    }
    if (!f32) {
      v.r = v.kind == KIND_CHOL ? nullptr : (double*)(ws + v.off_r);
    } else {
      v.xf = (float*)(ws + v.off_xf);
      v.bf = (float*)(ws + v.off_bf);
      v.rf = v.kind == KIND_CHOL ? nullptr : (float*)(ws + v.off_rf);
    }
    if (v.kind == KIND_BLOCK) {
      if (f32) SMG_TRY(upload_tables<float>(v, ws, s));
      else SMG_TRY(upload_tables<double>(v, ws, s));
    }
  }
  if (h.nc > 0) {
    h.ainv_d = (double*)(ws + h.off_ainv);
    h.w_d = (double*)(ws + h.off_w);
    SMG_HIP(hipMemcpyAsync(h.ainv_d, h.ainv.data(), h.ainv.size() * sizeof(double),
                           hipMemcpyHostToDevice, s));
    SMG_HIP(hipMemcpyAsync(h.w_d, h.w.data(), h.w.size() * sizeof(double),
                           hipMemcpyHostToDevice, s));
  }
  h.part_d = (double*)(ws + h.off_part);
  h.norm_d = (double*)(ws + h.off_norm);
  BotArgs ba{};
  if (h.bottom >= 0) {
    h.botargs_d = (BotArgs*)(ws + h.off_botargs);
    ba = make_botargs(h);
    SMG_HIP(hipMemcpyAsync(h.botargs_d, &ba, sizeof(BotArgs), hipMemcpyHostToDevice, s));
  }
  SMG_HIP(hipStreamSynchronize(s));
  h.ws = ws;
  return SMG_OK;
}

int smg_sample_field(smg_hierarchy* hh, int64_t n, uint64_t seed, uint64_t first_cycle,
                     void* state, void* out, int32_t out_dtype, void* stream) {
  SMG_TRY(check_bound(hh));
  SMG_TRY(check_ptr(state, "state"));
  if (n < 0 || (n > 0 && !out) || (out_dtype != SMG_OUT_F64 && out_dtype != SMG_OUT_F32)) {
    set_error("invalid n / out / out_dtype");
    return SMG_EINVAL;
  }
  if (n > 0) SMG_TRY(check_ptr(out, "out"));
  Hierarchy& h = hh->h;
  hipStream_t s = (hipStream_t)stream;
  Level& v0 = h.lv[0];
  const int64_t field = (int64_t)h.desc.ncomp * v0.n;
  SMG_TRY(import_level0(h, v0.x, (const double*)state, s));
  if (v0.kind == KIND_CHOL) SMG_HIP(launch_zero<double>(v0.b, field, s));
  Run r{&h, s, h.desc.kT > 0.0, false, seed, first_cycle};
  const int64_t total = (int64_t)h.prm.burn_in + n * (int64_t)h.prm.stride;
  const size_t out_elem = out_dtype == SMG_OUT_F32 ? sizeof(float) : sizeof(double);
  for (int64_t k = 0; k < total; ++k) {
    r.cycle = first_cycle + (uint64_t)k;
    SMG_TRY(full_cycle(r));
    const int64_t after = k + 1 - h.prm.burn_in;
    if (after > 0 && after % h.prm.stride == 0) {
      const int64_t idx = after / h.prm.stride - 1;
      SMG_TRY(export_level0(h, (char*)out + (size_t)idx * field * out_elem,
                            out_dtype == SMG_OUT_F32, v0.x, s));
    }
  }
  SMG_TRY(export_level0(h, state, 0, v0.x, s));
  return SMG_OK;
}

int smg_solve(smg_hierarchy* hh, const void* f, void* u, double rtol, int32_t max_cycles,
              void* stream, smg_solve_info* info) {
  SMG_TRY(check_bound(hh));
  SMG_TRY(check_ptr(f, "f"));
  SMG_TRY(check_ptr(u, "u"));
  if (!(rtol >= 0.0) || max_cycles < 0) {
    set_error("rtol must be >= 0 and max_cycles >= 0");
    return SMG_EINVAL;
  }
  Hierarchy& h = hh->h;
  hipStream_t s = (hipStream_t)stream;
  Level& v0 = h.lv[0];
  const int nc = h.desc.ncomp;
  const int64_t field = (int64_t)nc * v0.n;
  const bool f32 = refined(h);
  std::vector<double> fn(nc), rn(nc), rprev(nc, 0.0);
  double last_ratio = 0.0;
  SMG_HIP(launch_sumsq(h.norm_d, h.part_d, (const double*)f, v0.n, nc, s));
  SMG_HIP(hipMemcpyAsync(fn.data(), h.norm_d, nc * sizeof(double), hipMemcpyDeviceToHost, s));
  SMG_HIP(hipStreamSynchronize(s));
  for (int c = 0; c < nc; ++c)
    if (!std::isfinite(fn[c])) {
      set_error("f is not finite");
      return SMG_ENONFINITE;
    }
  SMG_TRY(import_level0(h, v0.b, (const double*)f, s));
  SMG_HIP(launch_zero<double>(v0.x, field, s));
  Run r{&h, s, false, true, 0, 0};
  double relres = 0.0;
  bool all_zero = true;
  for (int c = 0; c < nc; ++c) all_zero = all_zero && fn[c] == 0.0;
  int cycles = 0;
  // squared residual norms of the current iterate -> relres (max over components) and the
  // contraction of the last cycle; refined mode leaves the FP32 residual in lv[0].bf
  auto residual_norms = [&]() -> int {
    if (f32) {
      SMG_HIP(launch_refine_residual(v0.bf, v0.x, v0.b, v0.nx, v0.ny, v0.nz, nc, h.desc.h,
                                     h.part_d, h.norm_d, s));
    } else if (v0.kind == KIND_POINT) {
      SMG_HIP(launch_residual0<double>(v0.r, v0.x, v0.x + half_field(h), v0.b,
                                       v0.b + half_field(h), v0.nx, v0.ny, v0.nz, nc, h.desc.h,
                                       s));
      SMG_HIP(launch_sumsq(h.norm_d, h.part_d, v0.r, v0.n, nc, s));
    } else {
      // a level 0 that is drawn exactly has no residual buffer: u serves as scratch
      SMG_HIP(launch_residual7_nat((double*)u, v0.x, v0.b, v0.nx, v0.ny, v0.nz, nc, h.desc.h, s));
      SMG_HIP(launch_sumsq(h.norm_d, h.part_d, (const double*)u, v0.n, nc, s));
    }
    SMG_HIP(hipMemcpyAsync(rn.data(), h.norm_d, nc * sizeof(double), hipMemcpyDeviceToHost, s));
    SMG_HIP(hipStreamSynchronize(s));
    relres = 0.0;
    last_ratio = 0.0;
    for (int c = 0; c < nc; ++c) {
      if (!std::isfinite(rn[c])) {
        set_error("residual is not finite");
        return SMG_ENONFINITE;
      }
      double rr = fn[c] > 0.0 ? std::sqrt(rn[c] / fn[c]) : (rn[c] > 0.0 ? INFINITY : 0.0);
      relres = rr > relres ? rr : relres;
      if (cycles >= 2 && rprev[c] > 0.0) {
        double q = std::sqrt(rn[c] / rprev[c]);
        last_ratio = q > last_ratio ? q : last_ratio;
      }
      rprev[c] = rn[c];
    }
    return SMG_OK;
  };
  if (!all_zero) {
    relres = 1.0;
    bool ready = false;
    if (f32 && max_cycles > 0) {
      SMG_TRY(residual_norms());  // residual of u = 0, i.e. f, rounded to FP32
      ready = true;
    }
    while (cycles < max_cycles) {
      SMG_TRY(full_cycle(r, ready));
      ++cycles;
      SMG_TRY(residual_norms());
      if (relres <= rtol) break;
    }
  }
  SMG_TRY(export_level0(h, u, 0, v0.x, s));
  SMG_HIP(hipStreamSynchronize(s));
  if (info) {
    info->cycles = cycles;
    info->relres = relres;
    info->last_ratio = last_ratio;
  }
  if (!all_zero && relres > rtol) {
    set_error("solve did not converge: relres " + std::to_string(relres));
    return SMG_ENOTCONV;
  }
  return SMG_OK;
}

void smg_destroy_hierarchy(smg_hierarchy* hh) {
  if (!hh) return;
  for (hipEvent_t e : hh->h.ev_pool) (void)hipEventDestroy(e);
  delete hh;
}

const char* smg_last_error(void) { return g_err.c_str(); }

int smg_debug_smooth(smg_hierarchy* hh, int32_t level, int32_t colour, void* x, const void* b,
                     uint64_t seed, uint64_t cycle, int32_t slot, int32_t with_noise,
                     void* stream) {
  SMG_TRY(check_bound(hh));
  SMG_TRY(check_ptr(x, "x"));
  Hierarchy& h = hh->h;
  SMG_TRY(check_fp64(h));
  if (level < 0 || level >= (int)h.lv.size() || h.lv[level].kind == KIND_CHOL || slot < 0 ||
      slot > 255) {
    set_error("level has no smoother / invalid slot");
    return SMG_EINVAL;
  }
  Level& v = h.lv[level];
  if (colour < 0 || colour >= (v.kind == KIND_POINT ? 2 : 8) || (level > 0 && !b)) {
    set_error("invalid colour or missing b");
    return SMG_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  Run r{&h, s, with_noise != 0, b != nullptr, seed, cycle};
  if (v.kind == KIND_POINT) {
    NoiseArgs na = make_noise(r, level, slot, colour, KIND_SMOOTH_NOISE);
    SMG_TRY(import_level0(h, v.x, (const double*)x, s));
    if (b) SMG_TRY(import_level0(h, v.b, (const double*)b, s));
    double* xr = v.x;
    double* xb = v.x + half_field(h);
    const double* bc = b ? (colour ? v.b + half_field(h) : v.b) : nullptr;
    SMG_TRY(timed_rb_pass<double>(r, colour ? xb : xr, colour ? xr : xb, bc, colour, na));
    SMG_TRY(export_level0(h, x, 0, v.x, s));
  } else {
    if (r.noise) SMG_TRY(gen_level_noise<double>(r, level, slot));
    SMG_HIP(launch_block_pass<double>((double*)x, (const double*)b, (const double*)v.g2d_d,
                                      (const double*)v.zt_d, (const double*)v.bfac_d, v.nx, v.ny,
                                      v.nz, h.desc.ncomp, colour,
                                      r.noise ? (const double*)v.noise_d : nullptr,
                                      std::sqrt(h.desc.kT), s));
  }
  return SMG_OK;
}

int smg_debug_restrict_residual(smg_hierarchy* hh, int32_t level, const void* x, const void* b,
                                void* b_coarse, void* stream) {
  SMG_TRY(check_bound(hh));
  SMG_TRY(check_ptr(x, "x"));
  SMG_TRY(check_ptr(b_coarse, "b_coarse"));
  Hierarchy& h = hh->h;
  SMG_TRY(check_fp64(h));
  if (level < 0 || level + 1 >= (int)h.lv.size()) {
    set_error("level has no coarser level");
    return SMG_EINVAL;
  }
  Level& v = h.lv[level];
  if (level > 0 && !b) {
    set_error("missing b");
    return SMG_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  const int nc = h.desc.ncomp;
  if (v.kind == KIND_POINT) {
    SMG_TRY(import_level0(h, v.x, (const double*)x, s));
    if (b) SMG_TRY(import_level0(h, v.b, (const double*)b, s));
    SMG_HIP(launch_residual0<double>(v.r, v.x, v.x + half_field(h), b ? v.b : nullptr,
                                     b ? v.b + half_field(h) : nullptr, v.nx, v.ny, v.nz, nc,
                                     h.desc.h, s));
  } else {
    SMG_HIP(launch_residual_gal<double>(v.r, (const double*)x, (const double*)b,
                                        (const double*)v.g2d_d, (const double*)v.zt_d, v.nx,
                                        v.ny, v.nz, nc, s));
  }
  SMG_HIP(launch_restrict<double>((double*)b_coarse, nullptr, v.r, v.nx, v.ny, v.nz, nc, s));
  return SMG_OK;
}

int smg_debug_prolong_add(smg_hierarchy* hh, int32_t level, void* x, const void* e_coarse,
                          void* stream) {
  SMG_TRY(check_bound(hh));
  SMG_TRY(check_ptr(x, "x"));
  SMG_TRY(check_ptr(e_coarse, "e_coarse"));
  Hierarchy& h = hh->h;
  SMG_TRY(check_fp64(h));
  if (level < 0 || level + 1 >= (int)h.lv.size()) {
    set_error("level has no coarser level");
    return SMG_EINVAL;
  }
  Level& v = h.lv[level];
  hipStream_t s = (hipStream_t)stream;
  const int nc = h.desc.ncomp;
  if (v.kind == KIND_POINT) {
    SMG_TRY(import_level0(h, v.x, (const double*)x, s));
    SMG_HIP(launch_prolong0<double>(v.x, v.x + half_field(h), (const double*)e_coarse, v.nx, v.ny,
                                    v.nz, nc, s));
    SMG_TRY(export_level0(h, x, 0, v.x, s));
  } else {
    SMG_HIP(launch_prolong<double>((double*)x, (const double*)e_coarse, v.nx, v.ny, v.nz, nc, s));
  }
  return SMG_OK;
}

int smg_debug_coarsest(smg_hierarchy* hh, void* x, const void* b, uint64_t seed, uint64_t cycle,
                       int32_t with_noise, void* stream) {
  SMG_TRY(check_bound(hh));
  SMG_TRY(check_ptr(x, "x"));
  SMG_TRY(check_ptr(b, "b"));
  Hierarchy& h = hh->h;
  SMG_TRY(check_fp64(h));
  if (h.lv.back().kind != KIND_CHOL) {
    set_error("coarsest level is not drawn exactly (SMG_COARSEST_SMOOTH)");
    return SMG_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  Run r{&h, s, with_noise != 0, false, seed, cycle};
  const int l = (int)h.lv.size() - 1;
  NoiseArgs na = make_noise(r, l, 0, 0, KIND_COARSEST_NOISE);
  SMG_HIP(launch_coarsest<double>((double*)x, (const double*)b, h.ainv_d, h.w_d, h.nc,
                                  h.desc.ncomp, r.noise, na, s));
  return SMG_OK;
}

int smg_debug_host_table(const smg_hierarchy* hh, int32_t level, int32_t which, double* out,
                         size_t count) {
  if (!hh || !out) {
    set_error("null argument");
    return SMG_EINVAL;
  }
  const Hierarchy& h = hh->h;
  if (level < 0 || level >= (int)h.lv.size()) {
    set_error("invalid level");
    return SMG_EINVAL;
  }
  const Level& v = h.lv[level];
  const std::vector<double>* src = nullptr;
  if (which == 0) src = &v.coef;
  else if (which == 1) src = &v.bfac;
  else if (which == 2 && v.kind == KIND_CHOL) src = &h.ainv;
  else if (which == 3 && v.kind == KIND_CHOL) src = &h.w;
  if (!src || src->empty() || src->size() != count) {
    set_error("table not present on this level or wrong count");
    return SMG_EINVAL;
  }
  std::memcpy(out, src->data(), count * sizeof(double));
  return SMG_OK;
}

int smg_set_option(smg_hierarchy* hh, int32_t option, int64_t value) {
  if (!hh) {
    set_error("null hierarchy");
    return SMG_EINVAL;
  }
  if (option == SMG_OPT_BOTTOM_KERNEL && (value == 0 || value == 1)) {
    hh->h.use_bottom = value != 0;
    return SMG_OK;
  }
  if (option == SMG_OPT_TIMED_KERNEL && value >= SMG_TIMED_FINE_PASS && value <= SMG_TIMED_BOTTOM) {
    hh->h.timed_kernel = (int)value;
    return SMG_OK;
  }
  set_error("unknown option or value");
  return SMG_EINVAL;
}

int smg_kernel_timing(smg_hierarchy* hh, int32_t enable) {
  if (!hh) {
    set_error("null hierarchy");
    return SMG_EINVAL;
  }
  Hierarchy& h = hh->h;
  h.timing = enable != 0;
  h.ev_used = 0;
  h.tcount = 0;
  h.tms = 0.0;
  return SMG_OK;
}

int smg_kernel_timing_read(smg_hierarchy* hh, int64_t* count, double* total_ms) {
  if (!hh || !count || !total_ms) {
    set_error("null argument");
    return SMG_EINVAL;
  }
  Hierarchy& h = hh->h;
  for (size_t i = 0; i + 1 < h.ev_used; i += 2) {
    float ms = 0.0f;
    SMG_HIP(hipEventElapsedTime(&ms, h.ev_pool[i], h.ev_pool[i + 1]));
    h.tms += ms;
    h.tcount += 1;
  }
  h.ev_used = 0;
  *count = h.tcount;
  *total_ms = h.tms;
  return SMG_OK;
}

}  // extern "C"
