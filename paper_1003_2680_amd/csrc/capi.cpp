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

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "smg_internal.hpp"

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
  uint64_t cycle;  // with `chains`: cycles since each chain's first cycle
  int nc;          // components processed: c0 .. c0+nc-1 of the hierarchy's ncomp
  const ChainKey* chains;  // batched chains (device table) or null
  uint32_t cpc;            // components per chain
  int c0;                  // first component
  // FP32-refined form: the correction e is known to be zero (the previous cycle of this run
  // folded it into x and cleared it), so the next cycle need not clear it
  bool e_zero;
};

Run make_run(Hierarchy& h, hipStream_t s, bool noise, bool has_b0, uint64_t seed,
             uint64_t cycle) {
  return Run{&h, s, noise, has_b0, seed, cycle, h.desc.ncomp, nullptr, 1, 0, false};
}

// The run's share of a component-major buffer with `per` elements per component (null stays
// null).  Kernels index components from 0 on shifted pointers, so a run over components
// c0 .. c0+nc-1 touches exactly the memory that a run over all of them gives to those.
template <typename P>
P* comp_at(P* base, int64_t per, const Run& r) {
  return base ? base + (int64_t)r.c0 * per : nullptr;
}

NoiseArgs make_noise(const Run& r, int level, int slot, int colour, uint32_t kind) {
  NoiseArgs na;
  na.k0 = (uint32_t)r.seed;
  na.k1 = (uint32_t)(r.seed >> 32);
  na.sid = (uint32_t)level | ((uint32_t)slot << 4) | ((uint32_t)colour << 12) | (kind << 24);
  na.c2 = (uint32_t)r.cycle;
  na.c3 = (uint32_t)(r.cycle >> 32);
  na.sqkT = std::sqrt(r.h->desc.kT);
  na.chains = r.chains;
  na.comps_per_chain = r.cpc;
  // the kernels number the run's components from 0: component c of the run draws as
  // component c0 + c of the hierarchy
  na.comp0 = (uint32_t)r.c0;
  na.cpc_magic = chain_divisor_magic((uint32_t)r.cpc);
  na.bm = box_muller_coef();
  return na;
}

bool refined(const Hierarchy& h) { return h.prm.precision == SMG_FP32_REFINED; }

// log2(v) if v is a power of two, else -1
int log2_exact(int v) {
  if (v <= 0 || (v & (v - 1))) return -1;
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

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

// Events around a run of back-to-back launches of the timed kernel class (measurement
// support): the colour passes of one sweep, or one bottom launch.  Bracketing the run rather
// than each launch keeps the event overhead out of the per-launch average.
struct TimedScope {
  Hierarchy& h;
  hipStream_t s;
  hipEvent_t e1 = nullptr;
  int launches;
  int rc = SMG_OK;
  TimedScope(Hierarchy& hh, hipStream_t ss, int kind, int nlaunch)
      : h(hh), s(ss), launches(nlaunch) {
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
    if (rc == SMG_OK && e1) {
      if (hipEventRecord(e1, s) != hipSuccess) {
        set_error("hipEventRecord failed");
        rc = SMG_EHIP;
      }
      h.ev_launches.push_back(launches);
    }
    return rc;
  }
};

template <typename T>
int rb_pass(Run& r, T* xc, const T* xo, const T* bc, int colour, const NoiseArgs& na) {
  Hierarchy& h = *r.h;
  const Level& v = h.lv[0];
  SMG_HIP(launch_rb_pass<T>(xc, xo, bc, v.nx, v.ny, v.nz, r.nc, colour, h.desc.h,
                            h.desc.kT, r.noise, na, r.s));
  return SMG_OK;
}

template <typename T>
int sweep(Run& r, int l, int slot, bool post) {
  Hierarchy& h = *r.h;
  Level& v = h.lv[l];
  const int nc = h.desc.ncomp;
  if (v.kind == KIND_POINT) {
    const int64_t hn = v.n / 2;
    T* xr = comp_at(Fld<T>::x(v), hn, r);
    T* xb = comp_at(Fld<T>::x(v) + half_field(h), hn, r);
    const T* br = comp_at(Fld<T>::b(v), hn, r);
    const T* bb = comp_at(Fld<T>::b(v) + half_field(h), hn, r);
    TimedScope ts(h, r.s, SMG_TIMED_FINE_PASS, 2);
    SMG_TRY(ts.rc);
    for (int t = 0; t < 2; ++t) {
      const int colour = post ? 1 - t : t;
      NoiseArgs na = make_noise(r, l, slot, colour, KIND_SMOOTH_NOISE);
      const T* bc = r.has_b0 ? (colour ? bb : br) : nullptr;
      SMG_TRY(rb_pass<T>(r, colour ? xb : xr, colour ? xr : xb, bc, colour, na));
    }
    SMG_TRY(ts.close());
  } else {
    const T* noise = (const T*)v.noise_d;
    const T* zn = r.noise ? noise + ((size_t)slot * nc + r.c0) * v.n : nullptr;
    T* x = comp_at(Fld<T>::x(v), v.n, r);
    const T* b = comp_at(Fld<T>::b(v), v.n, r);
    const bool pairs = h.block_pairs && pair_level(v.nx, v.ny);
    TimedScope ts(h, r.s, l == 1 ? SMG_TIMED_LEVEL1_BLOCK_PASS : -1, pairs ? 4 : 8);
    SMG_TRY(ts.rc);
    for (int t = 0; t < 8; t += pairs ? 2 : 1) {
      const int colour = post ? 7 - t : t;  // with pairs: colour, then colour ^ 1
      if (pairs) {
        SMG_HIP(launch_block_pair<T>(x, b, (const T*)v.s1d_d, (const T*)v.zt_d,
                                     (const T*)v.bfac_d, v.nx, v.ny, v.nz, r.nc, colour, zn,
                                     r.s));
      } else {
        SMG_HIP(launch_block_pass<T>(x, b, (const T*)v.s1d_d, (const T*)v.zt_d,
                                     (const T*)v.bfac_d, v.nx, v.ny, v.nz, r.nc, colour, zn,
                                     h.block_tile, r.s));
      }
    }
    SMG_TRY(ts.close());
  }
  return SMG_OK;
}

// b^(l+1) = P^T (b^(l) - A^(l) x^(l)); the coarse iterate starts from zero
template <typename T>
int restrict_residual(Run& r, int l) {
  Hierarchy& h = *r.h;
  Level& v = h.lv[l];
  const int nc = r.nc;
  T* rr = comp_at(Fld<T>::r(v), v.n, r);
  Level& c = h.lv[l + 1];
  const bool bottom_next = (l + 1 == h.bottom) && h.use_bottom;
  T* bc = comp_at(Fld<T>::b(c), c.n, r);
  T* xc = bottom_next ? nullptr : comp_at(Fld<T>::x(c), c.n, r);
  if (v.kind == KIND_POINT) {
    // level 0: fused, the fine residual never goes to memory
    const int64_t hn = v.n / 2;
    T* xr = Fld<T>::x(v);
    T* br = Fld<T>::b(v);
    SMG_HIP(launch_restrict_residual0<T>(
        bc, xc, comp_at(xr, hn, r), comp_at(xr + half_field(h), hn, r),
        r.has_b0 ? comp_at(br, hn, r) : nullptr,
        r.has_b0 ? comp_at(br + half_field(h), hn, r) : nullptr, v.nx, v.ny, v.nz, nc, h.desc.h,
        r.s));
    return SMG_OK;
  }
  SMG_HIP(launch_residual_gal<T>(rr, comp_at(Fld<T>::x(v), v.n, r), comp_at(Fld<T>::b(v), v.n, r),
                                 (const T*)v.s1d_d, (const T*)v.zt_d, v.nx, v.ny, v.nz, nc, r.s));
  SMG_HIP(launch_restrict<T>(bc, xc, rr, v.nx, v.ny, v.nz, nc, r.s));
  return SMG_OK;
}

template <typename T>
int prolong_add(Run& r, int l) {
  Hierarchy& h = *r.h;
  Level& v = h.lv[l];
  const int nc = r.nc;
  const T* e = comp_at(Fld<T>::x(h.lv[l + 1]), h.lv[l + 1].n, r);
  if (v.kind == KIND_POINT) {
    T* xr = Fld<T>::x(v);
    const int64_t hn = v.n / 2;
    // The first post-sweep pass draws every colour-1 site afresh from its colour-0 neighbours
    // (a heat-bath update never reads the value it replaces), so with post-sweeps only the
    // colour-0 sites need the correction.
    const int colours = h.prm.nu2 > 0 ? 1 : 3;
    SMG_HIP(launch_prolong0<T>(comp_at(xr, hn, r), comp_at(xr + half_field(h), hn, r), e, v.nx,
                               v.ny, v.nz, nc, colours, r.s));
  } else {
    SMG_HIP(launch_prolong<T>(comp_at(Fld<T>::x(v), v.n, r), e, v.nx, v.ny, v.nz, nc, r.s));
  }
  return SMG_OK;
}

template <typename T>
int coarsest_step(Run& r, int l) {
  Hierarchy& h = *r.h;
  Level& v = h.lv[l];
  NoiseArgs na = make_noise(r, l, 0, 0, KIND_COARSEST_NOISE);
  SMG_HIP(launch_coarsest<T>(comp_at(Fld<T>::x(v), v.n, r), comp_at(Fld<T>::b(v), v.n, r),
                             h.ainv_d, h.w_d, h.nc, r.nc, r.noise, na, r.s));
  return SMG_OK;
}

// Noise of every sweep of every block level for the cycle r.cycle, in one launch (or of one
// level and slot when only_level >= 0).
template <typename T>
int gen_level_noise(Run& r, int only_level = -1, int only_slot = 0) {
  Hierarchy& h = *r.h;
  NoiseGenArgs a{};
  a.ncomp = h.desc.ncomp;
  a.nact = r.nc;
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
    e.out = comp_at((T*)v.noise_d, v.n, r);
    e.bfac = v.bfac_d;
    e.lg_bx = log2_exact(v.nx / 2);
    e.lg_bxy = log2_exact((v.nx / 2) * (v.ny / 2));
    e.calls_before = calls;
    calls += (uint32_t)(e.nslot * a.nact * (v.n / 2));
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
    BotLevel& bl = a.lv[i];
    bl.nx = v.nx;
    bl.ny = v.ny;
    bl.nz = v.nz;
    bl.kind = v.kind;
    bl.sy = sy;
    bl.sz = sz;
    bl.noise = v.noise_d;
    for (int q = 0; q < 20; ++q) bl.s1d[q] = v.s1d.empty() ? 0.0 : v.s1d[q];
    bl.zt = v.zt_d;
    bl.bfac = v.bfac_d;
    a.lds_off[i] = off;
    off += 3 * (int)bot_field_elems(v.kind, v.nx, v.ny, v.nz);
  }
  for (int i = 0; i < a.nlev; ++i) {
    const Level& v = h.lv[h.bottom + i];
    a.tab_off[i] = off;
    if (v.kind == KIND_BLOCK) off += v.nz * 10 + (v.nz / 2) * 192;
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
  na.comp0 = 0;  // this kernel numbers components absolutely (from c0)
  TimedScope ts(h, r.s, SMG_TIMED_BOTTOM, 1);
  SMG_TRY(ts.rc);
  SMG_HIP(launch_bottom<T>(h.botargs_d, r.nc, r.c0, h.bottom_lds, r.noise, na, r.s));
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
      SMG_HIP(launch_zero<T>(comp_at(Fld<T>::x(c), c.n, r), (int64_t)r.nc * c.n, r.s));
    SMG_TRY(vcycle<T>(r, l + 1));
    SMG_TRY(prolong_add<T>(r, l));
  }
  for (int s = 0; s < nu2; ++s) SMG_TRY(sweep<T>(r, l, nu1 + s, true));
  return SMG_OK;
}

// The cycle split around the LDS-resident bottom: the down-leg (levels above the bottom: pre-
// sweeps and restrictions) and the up-leg (prolongations and post-sweeps), in the order of
// vcycle, so that down-leg + bottom + up-leg is vcycle(0) exactly.
bool split_bottom(const Hierarchy& h) { return h.use_bottom && h.bottom > 0; }

template <typename T>
int vdown(Run& r) {
  Hierarchy& h = *r.h;
  for (int l = 0; l < h.bottom; ++l) {
    for (int s = 0; s < h.prm.nu1; ++s) SMG_TRY(sweep<T>(r, l, s, false));
    SMG_TRY(restrict_residual<T>(r, l));
  }
  return SMG_OK;
}

template <typename T>
int vup(Run& r) {
  Hierarchy& h = *r.h;
  for (int l = h.bottom - 1; l >= 0; --l) {
    SMG_TRY(prolong_add<T>(r, l));
    for (int s = 0; s < h.prm.nu2; ++s) SMG_TRY(sweep<T>(r, l, h.prm.nu1 + s, true));
  }
  return SMG_OK;
}

// Phases of one cycle on the FP64 level-0 state x: PH_IN (the block-level noise, the refined
// bridge in), PH_DOWN (the down-leg), PH_BOTTOM (the bottom launch), PH_UP (the up-leg) and
// PH_OUT (the refined bridge out); PH_PRE = PH_IN | PH_DOWN, PH_POST = PH_UP | PH_OUT.  A
// hierarchy without a split bottom runs its whole V-cycle in PH_DOWN.  Refined mode:
// residual_ready says that lv[0].bf already holds the FP32 residual of the current x (the solve
// computes it with the norms).  The legs run on `leg_run(r)`, the run the cycle's levels see.
enum {
  PH_IN = 1,
  PH_BOTTOM = 2,
  PH_OUT = 4,
  PH_DOWN = 8,
  PH_UP = 16,
  PH_PRE = PH_IN | PH_DOWN,
  PH_POST = PH_UP | PH_OUT,
  PH_ALL = 31
};

// The run the levels of a cycle see: in the refined form the inner cycle always has a
// right-hand side (the FP64 residual).
Run leg_run(const Run& r) {
  Run ri = r;
  if (refined(*r.h)) ri.has_b0 = true;
  return ri;
}

int cycle_phases(Run& r, int phases, bool residual_ready = false) {
  Hierarchy& h = *r.h;
  Level& v0 = h.lv[0];
  const bool split = split_bottom(h);
  Run ri = leg_run(r);
  if (!refined(h)) {
    if ((phases & PH_IN) && r.noise) SMG_TRY(gen_level_noise<double>(r));
    if (phases & PH_DOWN) SMG_TRY(split ? vdown<double>(ri) : vcycle<double>(ri, 0));
    if (split && (phases & PH_BOTTOM)) SMG_TRY(bottom_cycle<double>(ri));
    if (split && (phases & PH_UP)) SMG_TRY(vup<double>(ri));
    return SMG_OK;
  }
  // the processed components of both colour arrays
  const int64_t hn = v0.n / 2;
  const int64_t act = (int64_t)r.nc * hn;
  const size_t half = half_field(h);
  float* xf = comp_at(v0.xf, hn, r);
  double* x = comp_at(v0.x, hn, r);
  if (phases & PH_IN) {
    if (r.noise) SMG_TRY(gen_level_noise<float>(r));
    if (!residual_ready)
      SMG_HIP(launch_refine_residual(comp_at(v0.bf, hn, r), x,
                                     r.has_b0 ? comp_at(v0.b, hn, r) : nullptr, v0.nx, v0.ny,
                                     v0.nz, r.nc, h.desc.ncomp, h.desc.h, nullptr, nullptr, r.s));
    if (!r.e_zero) {
      SMG_HIP(launch_zero<float>(xf, act, r.s));
      SMG_HIP(launch_zero<float>(xf + half, act, r.s));
    }
    r.e_zero = false;
  }
  if (phases & PH_DOWN) SMG_TRY(split ? vdown<float>(ri) : vcycle<float>(ri, 0));
  if (split && (phases & PH_BOTTOM)) SMG_TRY(bottom_cycle<float>(ri));
  if (split && (phases & PH_UP)) SMG_TRY(vup<float>(ri));
  if (phases & PH_OUT) {
    // x += e on both colour arrays, clearing e for the next cycle
    SMG_HIP(launch_refine_out(x, xf, act, (int64_t)half, r.s));
    r.e_zero = true;
  }
  return SMG_OK;
}

// The block-colour pass of colour `colour` in sweep `t` (0-based; pre-sweeps first) of level l
// for every listed run that has it (level l above its bottom, t < its nu1 + nu2 and on the
// given leg), in one launch.
// The block-colour passes of colours `colour` and then colour ^ 1 (pairs), or of `colour`
// alone, for the listed runs as in block_pass_lockstep: levels that take two-colour launches in
// one pair launch per group, the others in single-colour launches.
template <typename T>
int block_pass_lockstep(const std::vector<Run>& legs, int l, int t, bool post, int colour,
                        bool noise, hipStream_t s, bool pairs) {
  std::vector<BlockPassItem<T>> items, paired;
  int tile = -1;
  for (const Run& r : legs) {
    Hierarchy& h = *r.h;
    if (r.noise != noise || l >= h.bottom) continue;
    Level& v = h.lv[l];
    if (v.kind != KIND_BLOCK) continue;
    const int nsw = post ? h.prm.nu2 : h.prm.nu1;
    if (t >= nsw) continue;
    const int slot = post ? h.prm.nu1 + t : t;
    BlockPassItem<T> it;
    it.x = comp_at(Fld<T>::x(v), v.n, r);
    it.b = comp_at(Fld<T>::b(v), v.n, r);
    it.s1d = (const T*)v.s1d_d;
    it.zt = (const T*)v.zt_d;
    it.bfac = (const T*)v.bfac_d;
    it.zn = noise ? (const T*)v.noise_d + ((size_t)slot * h.desc.ncomp + r.c0) * v.n : nullptr;
    it.nx = v.nx;
    it.ny = v.ny;
    it.nz = v.nz;
    it.ncomp = r.nc;
    if (pairs && h.block_pairs && pair_level(v.nx, v.ny)) {
      paired.push_back(it);
      continue;
    }
    items.push_back(it);
    // one tile shape per launch: the common choice of the items, else by work-group count
    tile = tile == -1 ? h.block_tile : (tile == h.block_tile ? tile : SMG_TILE_AUTO);
  }
  if (!paired.empty())
    SMG_HIP(launch_block_pair_multi<T>(paired.data(), (int)paired.size(), colour, noise, s));
  if (!items.empty()) {
    SMG_HIP(launch_block_pass_multi<T>(items.data(), (int)items.size(), colour, noise, tile, s));
    if (pairs)
      SMG_HIP(launch_block_pass_multi<T>(items.data(), (int)items.size(), colour ^ 1, noise,
                                         tile, s));
  }
  return SMG_OK;
}

// The down-leg (or up-leg) of several runs with a split bottom, of one sweep precision, in
// lockstep: level by level and sweep by sweep, the colour passes of all runs at the same point
// of their legs share one launch (level-0 point passes and Galerkin block passes alike); the
// transfers stay per run.  The runs
// touch disjoint memory and each keeps the order of its own vdown / vup, so each computes
// exactly what vdown / vup computes.
template <typename T>
int legs_lockstep(const std::vector<Run>& legs, bool down) {
  if (legs.empty()) return SMG_OK;
  hipStream_t s = legs[0].s;
  int maxb = 0, maxnu = 0;
  for (const Run& r : legs) {
    maxb = std::max(maxb, r.h->bottom);
    maxnu = std::max(maxnu, down ? r.h->prm.nu1 : r.h->prm.nu2);
  }
  auto sweeps = [&](int l) -> int {
    for (int t = 0; t < maxnu; ++t) {
      // point-smoothed levels (level 0): each colour of all runs in one launch per (right-hand
      // side present, noise) setting
      for (int k = 0; k < 2; ++k) {
        const int colour = down ? k : 1 - k;
        for (int hb = 0; hb < 2; ++hb)
          for (int nz = 0; nz < 2; ++nz) {
            std::vector<RbPassItem<T>> items;
            for (const Run& r : legs) {
              Hierarchy& h = *r.h;
              if (l >= h.bottom || h.lv[l].kind != KIND_POINT) continue;
              if (t >= (down ? h.prm.nu1 : h.prm.nu2)) continue;
              if ((int)r.has_b0 != hb || (int)r.noise != nz) continue;
              Level& v = h.lv[l];
              const int64_t hn = v.n / 2;
              T* xr = comp_at(Fld<T>::x(v), hn, r);
              T* xb = comp_at(Fld<T>::x(v) + half_field(h), hn, r);
              const T* br = comp_at(Fld<T>::b(v), hn, r);
              const T* bb = comp_at(Fld<T>::b(v) + half_field(h), hn, r);
              RbPassItem<T> it;
              it.xc = colour ? xb : xr;
              it.xo = colour ? xr : xb;
              it.bc = r.has_b0 ? (colour ? bb : br) : nullptr;
              it.nx = v.nx;
              it.ny = v.ny;
              it.nz = v.nz;
              it.ncomp = r.nc;
              it.h = h.desc.h;
              it.kT = h.desc.kT;
              it.na = make_noise(r, l, down ? t : h.prm.nu1 + t, colour, KIND_SMOOTH_NOISE);
              items.push_back(it);
            }
            if (!items.empty())
              SMG_HIP(launch_rb_pass_multi<T>(items.data(), (int)items.size(), colour, hb != 0,
                                              nz != 0, s));
          }
      }
      for (int k = 0; k < 8; k += 2) {  // colour pairs (c, c ^ 1) in sweep order
        const int colour = down ? k : 7 - k;
        for (int nz = 0; nz < 2; ++nz)
          SMG_TRY(block_pass_lockstep<T>(legs, l, t, !down, colour, nz != 0, s, true));
      }
    }
    return SMG_OK;
  };
  if (down) {
    for (int l = 0; l < maxb; ++l) {
      SMG_TRY(sweeps(l));
      for (const Run& r0 : legs) {
        Run r = r0;
        if (l < r.h->bottom) SMG_TRY(restrict_residual<T>(r, l));
      }
    }
  } else {
    for (int l = maxb - 1; l >= 0; --l) {
      for (const Run& r0 : legs) {
        Run r = r0;
        if (l < r.h->bottom) SMG_TRY(prolong_add<T>(r, l));
      }
      SMG_TRY(sweeps(l));
    }
  }
  return SMG_OK;
}

int full_cycle(Run& r, bool residual_ready = false) {
  return cycle_phases(r, PH_ALL, residual_ready);
}

// The LDS-resident bottoms of every run that has one, in as few launches as possible (one per
// sweep precision and noise setting, up to kBotMultiItems hierarchies and kBotMultiWG
// components each; a run with more components takes a launch of its own).
int batch_bottoms(const std::vector<Run*>& runs) {
  for (int f32 = 0; f32 < 2; ++f32)
    for (int nz = 0; nz < 2; ++nz) {
      BotMultiArgs m{};
      m.bm = box_muller_coef();
      int nwg = 0;
      size_t lds = 0;
      hipStream_t s = nullptr;
      auto flush = [&]() -> int {
        if (m.nitems == 0) return SMG_OK;
        hipError_t e = f32 ? launch_bottom_multi<float>(m, nwg, lds, nz != 0, s)
                           : launch_bottom_multi<double>(m, nwg, lds, nz != 0, s);
        if (e != hipSuccess) {
          set_error(std::string("launch_bottom_multi: ") + hipGetErrorString(e));
          return SMG_EHIP;
        }
        m.nitems = 0;
        nwg = 0;
        lds = 0;
        return SMG_OK;
      };
      for (Run* r : runs) {
        Hierarchy& h = *r->h;
        if (!split_bottom(h) || (int)refined(h) != f32 || (int)r->noise != nz) continue;
        if (r->nc > kBotMultiWG) {  // more components than one launch holds: its own launch
          Run ri = *r;
          ri.has_b0 = ri.has_b0 || refined(h);
          SMG_TRY(f32 ? bottom_cycle<float>(ri) : bottom_cycle<double>(ri));
          continue;
        }
        if (m.nitems == kBotMultiItems || nwg + r->nc > kBotMultiWG) SMG_TRY(flush());
        const NoiseArgs na = make_noise(*r, 0, 0, 0, KIND_SMOOTH_NOISE);
        BotMultiItem& it = m.it[m.nitems];
        it.args = h.botargs_d;
        it.k0 = na.k0;
        it.k1 = na.k1;
        it.c2 = na.c2;
        it.c3 = na.c3;
        it.chains = na.chains;
        it.cpc = na.comps_per_chain;
        it.cpc_magic = na.cpc_magic;
        it.sqkT = na.sqkT;
        // the bottom numbers components absolutely (its noise keys take the chain table as is)
        for (int c = r->c0; c < r->c0 + r->nc; ++c)
          m.wg[nwg++] = (uint32_t)m.nitems | ((uint32_t)c << 16);
        ++m.nitems;
        lds = std::max(lds, h.bottom_lds);
        s = r->s;
      }
      SMG_TRY(flush());
    }
  return SMG_OK;
}

// One cycle of several runs on one stream (distinct hierarchies): every run's down-leg, then
// the LDS-resident bottoms of all runs that have one in as few launches as possible (one per
// sweep precision and noise setting, up to kBotMultiItems hierarchies and kBotMultiWG
// components each), then every run's up-leg.  Each run's own kernels keep their order and the
// runs touch disjoint memory, so every run computes exactly what full_cycle computes.
// `phases`: PH_PRE (noise, bridge in, down-legs), PH_BOTTOM, PH_POST (up-legs, bridge out), or
// any union; a cycle is PH_PRE, then PH_BOTTOM, then PH_POST.
int batch_cycle(const std::vector<Run*>& runs, const std::vector<char>& ready,
                int phases = PH_ALL) {
  // the legs of the runs with a split bottom go in lockstep (one launch per block-colour pass
  // for all of them, per sweep precision); the others run their whole V-cycle in PH_DOWN
  std::vector<Run> legs64, legs32;
  for (size_t i = 0; i < runs.size(); ++i) {
    Run& r = *runs[i];
    if (phases & PH_IN) SMG_TRY(cycle_phases(r, PH_IN, ready[i]));
    if (!split_bottom(*r.h)) {
      if (phases & PH_DOWN) SMG_TRY(cycle_phases(r, PH_DOWN, ready[i]));
    } else {
      (refined(*r.h) ? legs32 : legs64).push_back(leg_run(r));
    }
  }
  if (phases & PH_DOWN) {
    SMG_TRY(legs_lockstep<double>(legs64, true));
    SMG_TRY(legs_lockstep<float>(legs32, true));
  }
  if (phases & PH_BOTTOM) SMG_TRY(batch_bottoms(runs));
  if (phases & PH_UP) {
    SMG_TRY(legs_lockstep<double>(legs64, false));
    SMG_TRY(legs_lockstep<float>(legs32, false));
  }
  if (phases & PH_OUT)
    for (size_t i = 0; i < runs.size(); ++i) SMG_TRY(cycle_phases(*runs[i], PH_OUT, ready[i]));
  return SMG_OK;
}

// natural [nc][N] field -> components c0 .. c0+nc-1 of the level-0 storage (x or b)
int import_level0(Hierarchy& h, double* dst, const double* nat, hipStream_t s, int nc = -1,
                  int c0 = 0) {
  Level& v = h.lv[0];
  if (nc < 0) nc = h.desc.ncomp;
  if (v.kind == KIND_POINT) {
    const size_t off = (size_t)c0 * (v.n / 2);
    SMG_HIP(launch_to_split(dst + off, dst + half_field(h) + off, nat, v.nx, v.ny, v.nz, nc, s));
  } else {
    SMG_HIP(launch_copy(dst + (size_t)c0 * v.n, nat, (int64_t)nc * v.n, s));
  }
  return SMG_OK;
}

// components c0 .. c0+nc-1 of the level-0 storage -> natural [nc][N] (float64 or float32)
int export_level0(Hierarchy& h, void* nat, int out_f32, const double* src, hipStream_t s,
                  int nc = -1, int c0 = 0) {
  Level& v = h.lv[0];
  if (nc < 0) nc = h.desc.ncomp;
  if (v.kind == KIND_POINT) {
    const size_t off = (size_t)c0 * (v.n / 2);
    SMG_HIP(launch_from_split(nat, out_f32, src + off, src + half_field(h) + off, v.nx, v.ny,
                              v.nz, nc, s));
  } else {
    SMG_HIP(launch_cast(nat, out_f32, src + (size_t)c0 * v.n, (int64_t)nc * v.n, s));
  }
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
  std::vector<T> g(v.s1d.begin(), v.s1d.end());
  std::vector<T> z(v.zt.begin(), v.zt.end());
  std::vector<T> b(v.bfac.begin(), v.bfac.end());
  v.s1d_d = ws + v.off_s1d;
  v.zt_d = ws + v.off_zt;
  v.bfac_d = ws + v.off_bfac;
  v.noise_d = ws + v.off_noise;
  SMG_HIP(hipMemcpyAsync(v.s1d_d, g.data(), g.size() * sizeof(T), hipMemcpyHostToDevice, s));
  SMG_HIP(hipMemcpyAsync(v.zt_d, z.data(), z.size() * sizeof(T), hipMemcpyHostToDevice, s));
  SMG_HIP(hipMemcpyAsync(v.bfac_d, b.data(), b.size() * sizeof(T), hipMemcpyHostToDevice, s));
  // the staging vectors die on return
  SMG_HIP(hipStreamSynchronize(s));
  return SMG_OK;
}

// Real 1D eigenvectors (see smg.h, observables): periodic axis on n points, index a.
double periodic_factor(int n, int a, int i) {
  if (a == 0) return 1.0 / std::sqrt((double)n);
  if (a == n - 1) return ((i & 1) ? -1.0 : 1.0) / std::sqrt((double)n);
  const int j = (a + 1) / 2;
  const double t = 2.0 * M_PI * j * i / n;
  return std::sqrt(2.0 / n) * ((a & 1) ? std::cos(t) : std::sin(t));
}

// wall axis, m = 1..nz: sin(pi m (z + 1/2) / nz), normalised
void wall_vector(int nz, int m, double* out) {
  double ss = 0.0;
  for (int z = 0; z < nz; ++z) {
    out[z] = std::sin(M_PI * m * (z + 0.5) / nz);
    ss += out[z] * out[z];
  }
  const double inv = 1.0 / std::sqrt(ss);
  for (int z = 0; z < nz; ++z) out[z] *= inv;
}

int periodic_wavenumber(int n, int a) {
  if (a == 0) return 0;
  if (a == n - 1) return n / 2;
  return (a + 1) / 2;
}

int check_modes(const Hierarchy& h, const int32_t* modes, int k) {
  const Level& v = h.lv[0];
  if (k < 0 || k > kMaxModes || (k > 0 && !modes)) {
    set_error("n_modes must be in [0, " + std::to_string(kMaxModes) + "] with a mode list");
    return SMG_EINVAL;
  }
  for (int q = 0; q < k; ++q) {
    const int a = modes[3 * q], b = modes[3 * q + 1], m = modes[3 * q + 2];
    if (a < 0 || a >= v.nx || b < 0 || b >= v.ny || m < 1 || m > v.nz) {
      set_error("mode " + std::to_string(q) + " out of range for the grid");
      return SMG_EINVAL;
    }
  }
  return SMG_OK;
}

// Device tables of the modes (uploaded when the mode list changes): the x factor e_a(x) and
// the row factor e_b(y) w_m(z) of each mode.
int load_modes(Hierarchy& h, const int32_t* modes, int k, hipStream_t s) {
  std::vector<int32_t> want(modes, modes + 3 * k);
  if (h.modes_valid && want == h.modes_loaded) return SMG_OK;
  const Level& v = h.lv[0];
  const size_t rows = (size_t)v.ny * v.nz;
  std::vector<double> tab((size_t)kMaxModes * (v.nx + rows), 0.0);
  double* tx = tab.data();
  double* tr = tx + (size_t)kMaxModes * v.nx;
  std::vector<double> wz(v.nz);
  // row factors row-major with the stride the kernel sums over (8 or kMaxModes): the factors
  // of one row share a scalar cache line
  const size_t ks = k <= 8 ? 8 : kMaxModes;
  for (int q = 0; q < k; ++q) {
    for (int i = 0; i < v.nx; ++i) tx[q * v.nx + i] = periodic_factor(v.nx, modes[3 * q], i);
    wall_vector(v.nz, modes[3 * q + 2], wz.data());
    for (int z = 0; z < v.nz; ++z)
      for (int y = 0; y < v.ny; ++y)
        tr[((size_t)z * v.ny + y) * ks + q] = periodic_factor(v.ny, modes[3 * q + 1], y) * wz[z];
  }
  SMG_HIP(hipMemcpyAsync(h.ws + h.off_mtab, tab.data(), tab.size() * sizeof(double),
                         hipMemcpyHostToDevice, s));
  SMG_HIP(hipStreamSynchronize(s));  // the staging vector dies on return
  h.modes_loaded = want;
  h.modes_valid = true;
  return SMG_OK;
}

// Emission of components c0 .. c0+nc-1 of the level-0 state with optional statistics (one
// fused pass; obs, m1, m2 and out are laid out over those nc components).
int emit(Hierarchy& h, void* out, int out_f32, double* obs, double* m1, double* m2, int k,
         int nc, int c0, hipStream_t s) {
  Level& v0 = h.lv[0];
  if (!obs && !m1) {
    if (out) SMG_TRY(export_level0(h, out, out_f32, v0.x, s, nc, c0));
    return SMG_OK;
  }
  StatsArgs a{};
  const bool split = v0.kind == KIND_POINT;
  const int64_t per = split ? v0.n / 2 : v0.n;
  a.xr = v0.x + (int64_t)c0 * per;
  a.xb = split ? v0.x + half_field(h) + (int64_t)c0 * per : nullptr;
  a.nx = v0.nx;
  a.ny = v0.ny;
  a.nz = v0.nz;
  a.lgx = log2_exact(v0.nx);
  a.lgy = log2_exact(v0.ny);
  a.nmodes = obs ? k : 0;
  a.nblk = h.stats_nblk;
  a.tx = (const double*)(h.ws + h.off_mtab);
  a.trow = a.tx + (size_t)kMaxModes * v0.nx;
  a.out = out;
  a.out_f32 = out_f32;
  a.m1 = m1;
  a.m2 = m2;
  // partial sums: [ncomp][stats_nblk][kMaxModes + 1] are allotted, so each component range has
  // a region of its own
  a.part = (double*)(h.ws + h.off_spart) + (size_t)c0 * h.stats_nblk * (kMaxModes + 1);
  SMG_HIP(launch_stats(a, nc, obs, 0.5 / (h.desc.h * h.desc.h), s));
  return SMG_OK;
}

// Batch description of a call: nchains chains of cpc components each (the first
// nchains*cpc components of the hierarchy); nchains == 0 means one chain over all components.
struct Batch {
  int nchains = 0;
  int cpc = 0;
  int nc(const Hierarchy& h) const { return nchains > 0 ? nchains * cpc : h.desc.ncomp; }
};

int check_batch(const Hierarchy& h, const Batch& bt) {
  if (bt.nchains == 0) return SMG_OK;
  if (bt.nchains < 0 || bt.cpc < 1 || (int64_t)bt.nchains * bt.cpc > h.desc.ncomp ||
      bt.nchains > kMaxChains) {
    set_error("chains * comps_per_chain must be within the hierarchy's ncomp (and chains <= " +
              std::to_string(kMaxChains) + ")");
    return SMG_EINVAL;
  }
  return SMG_OK;
}

// Writes the chain table (seeds and first cycles) into the workspace, stream-ordered.
int set_chains(Hierarchy& h, const Batch& bt, const uint64_t* seeds, const uint64_t* first,
               hipStream_t s) {
  for (int c0 = 0; c0 < bt.nchains; c0 += kChainsPerLaunch) {
    ChainKeyBatch kb{};
    kb.first = c0;
    kb.count = std::min(kChainsPerLaunch, bt.nchains - c0);
    for (int i = 0; i < kb.count; ++i) {
      const uint64_t sd = seeds[c0 + i], fc = first ? first[c0 + i] : 0;
      kb.k[i] = ChainKey{(uint32_t)sd, (uint32_t)(sd >> 32), (uint32_t)fc, (uint32_t)(fc >> 32)};
    }
    SMG_HIP(launch_set_chains(h.chains_d, kb, s));
  }
  h.chains_set = bt.nchains;
  h.chains_cpc = bt.cpc;
  return SMG_OK;
}

// A sampling call as a job: begin() checks the arguments, writes the chain table and the mode
// tables and imports the chain state; cycle(k) runs cycle k (k = 0 .. total-1) and emits when
// due; finish() exports the state.  smg_sample_* run one job; smg_batch_run interleaves
// several, cycle by cycle, with their bottoms merged.
struct SampleJob {
  smg_hierarchy* hh = nullptr;
  Batch bt;
  int64_t n = 0, total = 0;
  uint64_t first_cycle = 0;
  void* state = nullptr;
  void* out = nullptr;
  int32_t out_dtype = SMG_OUT_F64;
  double* obs = nullptr;
  double* m1 = nullptr;
  double* m2 = nullptr;
  int n_modes = 0;
  int nc = 0;
  int64_t field = 0;
  Run r{};

  int begin(smg_hierarchy* h_, const Batch& bt_, const uint64_t* seeds,
            const uint64_t* first_cycles, int64_t n_, uint64_t seed, uint64_t first_cycle_,
            void* state_, void* out_, int32_t out_dtype_, const int32_t* modes,
            int32_t n_modes_, void* obs_, void* moments, hipStream_t s) {
    hh = h_;
    bt = bt_;
    SMG_TRY(check_bound(hh));
    SMG_TRY(check_ptr(state_, "state"));
    if (n_ < 0 || (out_dtype_ != SMG_OUT_F64 && out_dtype_ != SMG_OUT_F32)) {
      set_error("invalid n / out_dtype");
      return SMG_EINVAL;
    }
    if (n_ > 0 && out_) SMG_TRY(check_ptr(out_, "out"));
    if (moments) SMG_TRY(check_ptr(moments, "moments"));
    if (obs_ && ((uintptr_t)obs_ & 7u)) {
      set_error("obs must be 8-byte aligned");
      return SMG_EINVAL;
    }
    Hierarchy& h = hh->h;
    SMG_TRY(check_batch(h, bt));
    if (bt.nchains > 0) {
      if (seeds) {
        SMG_TRY(set_chains(h, bt, seeds, first_cycles, s));
      } else if (h.chains_set != bt.nchains || h.chains_cpc != bt.cpc) {
        set_error("no chain table of this shape was set (pass seeds)");
        return SMG_ESTATE;
      }
    }
    if (obs_) {
      SMG_TRY(check_modes(h, modes, n_modes_));
      SMG_TRY(load_modes(h, modes, n_modes_, s));
    }
    n = n_;
    first_cycle = first_cycle_;
    state = state_;
    out = out_;
    out_dtype = out_dtype_;
    obs = (double*)obs_;
    n_modes = n_modes_;
    Level& v0 = h.lv[0];
    nc = bt.nc(h);
    field = (int64_t)nc * v0.n;
    SMG_TRY(import_level0(h, v0.x, (const double*)state, s, nc));
    if (v0.kind == KIND_CHOL) SMG_HIP(launch_zero<double>(v0.b, field, s));
    r = make_run(h, s, h.desc.kT > 0.0, false, seed, first_cycle);
    r.nc = nc;
    if (bt.nchains > 0) {
      r.chains = h.chains_d;
      r.cpc = (uint32_t)bt.cpc;
    }
    total = (int64_t)h.prm.burn_in + n * (int64_t)h.prm.stride;
    m1 = (double*)moments;
    m2 = m1 ? m1 + field : nullptr;
    return SMG_OK;
  }

  // the noise cycle of cycle k of the call (with chains: counted from each chain's first)
  uint64_t cycle_of(int64_t k) const {
    return bt.nchains > 0 ? (uint64_t)k : first_cycle + (uint64_t)k;
  }
  void set_cycle(int64_t k) { r.cycle = cycle_of(k); }

  // emission after cycle k, when it is due, of the components of run g (the whole job, or one
  // of its stream groups)
  int emit_after(int64_t k, const Run& g) {
    Hierarchy& h = hh->h;
    const int64_t after = k + 1 - h.prm.burn_in;
    if (after <= 0 || after % h.prm.stride != 0) return SMG_OK;
    const int64_t idx = after / h.prm.stride - 1;
    const size_t out_elem = out_dtype == SMG_OUT_F32 ? sizeof(float) : sizeof(double);
    const size_t obs_stride = (size_t)nc * (n_modes + 1);
    const size_t n0 = (size_t)h.lv[0].n;
    const size_t c0 = (size_t)g.c0;
    return emit(h, out ? (char*)out + ((size_t)idx * field + c0 * n0) * out_elem : nullptr,
                out_dtype == SMG_OUT_F32,
                obs ? obs + (size_t)idx * obs_stride + c0 * (n_modes + 1) : nullptr,
                m1 ? m1 + c0 * n0 : nullptr, m2 ? m2 + c0 * n0 : nullptr, n_modes, g.nc, g.c0,
                g.s);
  }
  int emit_after(int64_t k) { return emit_after(k, r); }

  int finish() {
    Hierarchy& h = hh->h;
    SMG_TRY(export_level0(h, state, 0, h.lv[0].x, r.s, nc));
    // the chains continue from here: a repeated (or replayed) call draws the next cycles
    if (bt.nchains > 0)
      SMG_HIP(launch_advance_chains(h.chains_d, bt.nchains, (uint64_t)total, r.s));
    return SMG_OK;
  }
};

// Streams and events of ng stream groups: ng side streams (default priority), made together so
// that the runtime spreads them over its hardware queues, with their join and stagger events
// and a fork event; made on the current device (again when the device changed).  Every group
// runs on a side stream and the caller's stream only forks and joins: a group left on the
// caller's stream could share a hardware queue with a side stream, which serialises the two
// groups behind the stagger's waits (measured 40 % slower than one stream).
int ensure_side_streams(Hierarchy& h, int ng) {
  int dev = -1;
  SMG_HIP(hipGetDevice(&dev));
  if (dev != h.side_device) release_side_streams(h);
  if (!h.ev_fork) {
    SMG_HIP(hipEventCreateWithFlags(&h.ev_fork, hipEventDisableTiming));
    h.side_device = dev;
  }
  while ((int)h.side.size() < ng) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    SMG_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    h.side.push_back(st);
    SMG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    h.ev_join.push_back(ev);
    SMG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    h.ev_mid.push_back(ev);
  }
  return SMG_OK;
}

// `groups`: the most stream groups the call may use (1: the caller's stream only).
int sample_impl(smg_hierarchy* hh, const Batch& bt, const uint64_t* seeds,
                const uint64_t* first_cycles, int64_t n, uint64_t seed, uint64_t first_cycle,
                void* state, void* out, int32_t out_dtype, const int32_t* modes,
                int32_t n_modes, void* obs, void* moments, void* stream, int groups) {
  SampleJob j;
  SMG_TRY(j.begin(hh, bt, seeds, first_cycles, n, seed, first_cycle, state, out, out_dtype,
                  modes, n_modes, obs, moments, (hipStream_t)stream));
  Hierarchy& h = hh->h;
  const int ng = h.timing ? 1 : std::min(groups, j.nc);
  if (ng < 2) {
    for (int64_t k = 0; k < j.total; ++k) {
      j.set_cycle(k);
      SMG_TRY(full_cycle(j.r));
      SMG_TRY(j.emit_after(k));
    }
    return j.finish();
  }
  // Component groups on streams of their own: group i takes components [i nc / ng, (i+1) nc /
  // ng) on the hierarchy's side stream i; the side streams wait for the caller's stream first
  // and it waits for them at the end.  The groups
  // touch disjoint components (and regions of every shared buffer), and a component's work and
  // noise are the same whatever the group, so the results are those of one stream.
  SMG_TRY(ensure_side_streams(h, ng));
  std::vector<Run> g(ng, j.r);
  for (int i = 0; i < ng; ++i) {
    g[i].c0 = i * j.nc / ng;
    g[i].nc = (i + 1) * j.nc / ng - g[i].c0;
    g[i].s = h.side[i];
  }
  SMG_HIP(hipEventRecord(h.ev_fork, j.r.s));
  for (int i = 0; i < ng; ++i) SMG_HIP(hipStreamWaitEvent(g[i].s, h.ev_fork, 0));
  // Staggered: group i starts cycle k once group i-1 has finished the down-leg of cycle k, so
  // that its down-leg runs beside the other group's bottom instead of all groups reaching their
  // bottoms at once (identical groups issued together otherwise stay in phase).
  int rc = SMG_OK;
  for (int64_t k = 0; k < j.total && rc == SMG_OK; ++k)
    for (int i = 0; i < ng && rc == SMG_OK; ++i) {
      g[i].cycle = j.cycle_of(k);
      if (i > 0 && hipStreamWaitEvent(g[i].s, h.ev_mid[i - 1], 0) != hipSuccess) {
        set_error("hipStreamWaitEvent failed");
        rc = SMG_EHIP;
        break;
      }
      rc = cycle_phases(g[i], PH_PRE);
      if (rc == SMG_OK && i + 1 < ng && hipEventRecord(h.ev_mid[i], g[i].s) != hipSuccess) {
        set_error("hipEventRecord failed");
        rc = SMG_EHIP;
      }
      if (rc == SMG_OK) rc = cycle_phases(g[i], PH_BOTTOM | PH_POST);
      if (rc == SMG_OK) rc = j.emit_after(k, g[i]);
    }
  // join even after an error, so that nothing the side streams hold outlives the call's stream
  for (int i = 0; i < ng; ++i) {
    const hipError_t e1 = hipEventRecord(h.ev_join[i], g[i].s);
    const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(j.r.s, h.ev_join[i], 0) : e1;
    if (e2 != hipSuccess && rc == SMG_OK) {
      set_error(std::string("joining a chain-group stream: ") + hipGetErrorString(e2));
      rc = SMG_EHIP;
    }
  }
  SMG_TRY(rc);
  return j.finish();
}

// A solve as a job (one chain = cpc components, or all components when nchains == 0).  A chain
// stops counting once all its components reach rtol: its u is written at that cycle, so each
// result equals that of a solve of the chain alone.  The host reads norms after each stream
// synchronisation; the steps between synchronisations are split so that smg_batch_run can
// run several jobs with one synchronisation per cycle for all of them:
//   enqueue_fnorm / [sync] / after_fnorm (+ enqueue_norms when initial_norms) / [sync] /
//   after_initial_norms, then per cycle: full_cycle / enqueue_norms / [sync] / after_norms;
//   finish.
struct SolveJob {
  struct ChainState {
    bool done = false, all_zero = true;
    int cycles = 0;
    double relres = 0.0, last_ratio = 0.0;
  };
  smg_hierarchy* hh = nullptr;
  Batch bt;
  const void* f = nullptr;
  void* u = nullptr;
  double rtol = 0.0;
  int max_cycles = 0;
  smg_solve_info* infos = nullptr;
  int nc = 0, nch = 1, cpc = 1;
  bool f32 = false;
  std::vector<double> fn, rn, rprev;
  std::vector<ChainState> cs;
  int pending = 0, cycles = 0;
  bool ready = false;          // refined mode: lv[0].bf holds the FP32 residual of x
  bool initial_norms = false;  // refined mode: the residual of u = 0 is taken before cycle 1
  Run r{};

  int begin(smg_hierarchy* h_, const Batch& bt_, const void* f_, void* u_, double rtol_,
            int32_t max_cycles_, smg_solve_info* infos_, hipStream_t s) {
    hh = h_;
    bt = bt_;
    SMG_TRY(check_bound(hh));
    SMG_TRY(check_ptr(f_, "f"));
    SMG_TRY(check_ptr(u_, "u"));
    if (!(rtol_ >= 0.0) || max_cycles_ < 0) {
      set_error("rtol must be >= 0 and max_cycles >= 0");
      return SMG_EINVAL;
    }
    Hierarchy& h = hh->h;
    SMG_TRY(check_batch(h, bt));
    f = f_;
    u = u_;
    rtol = rtol_;
    max_cycles = max_cycles_;
    infos = infos_;
    nc = bt.nc(h);
    nch = bt.nchains > 0 ? bt.nchains : 1;
    cpc = bt.nchains > 0 ? bt.cpc : nc;
    f32 = refined(h);
    fn.assign(nc, 0.0);
    rn.assign(nc, 0.0);
    rprev.assign(nc, 0.0);
    cs.assign(nch, ChainState());
    r = make_run(h, s, false, true, 0, 0);
    r.nc = nc;
    return SMG_OK;
  }

  int enqueue_fnorm() {
    Hierarchy& h = hh->h;
    SMG_HIP(launch_sumsq(h.norm_d, h.part_d, (const double*)f, h.lv[0].n, nc, r.s));
    SMG_HIP(hipMemcpyAsync(fn.data(), h.norm_d, nc * sizeof(double), hipMemcpyDeviceToHost,
                           r.s));
    return SMG_OK;
  }

  int after_fnorm() {
    Hierarchy& h = hh->h;
    Level& v0 = h.lv[0];
    hipStream_t s = r.s;
    for (int c = 0; c < nc; ++c)
      if (!std::isfinite(fn[c])) {
        set_error("f is not finite");
        return SMG_ENONFINITE;
      }
    SMG_TRY(import_level0(h, v0.b, (const double*)f, s, nc));
    if (v0.kind == KIND_POINT) {
      // split storage: the processed components of both colour arrays (colour 1 starts after
      // all components of colour 0, not after the processed ones)
      const int64_t act = (int64_t)nc * (v0.n / 2);
      SMG_HIP(launch_zero<double>(v0.x, act, s));
      SMG_HIP(launch_zero<double>(v0.x + half_field(h), act, s));
    } else {
      SMG_HIP(launch_zero<double>(v0.x, (int64_t)nc * v0.n, s));
    }
    for (int ch = 0; ch < nch; ++ch) {
      for (int c = ch * cpc; c < (ch + 1) * cpc; ++c)
        cs[ch].all_zero = cs[ch].all_zero && fn[c] == 0.0;
      if (cs[ch].all_zero) {
        cs[ch].done = true;  // u = 0 after zero cycles
        SMG_TRY(export_level0(h, (double*)u + (size_t)ch * cpc * v0.n, 0, v0.x, s, cpc,
                              ch * cpc));
      } else {
        cs[ch].relres = 1.0;
        ++pending;
      }
    }
    initial_norms = pending > 0 && f32 && max_cycles > 0;
    if (initial_norms) SMG_TRY(enqueue_norms());  // residual of u = 0, i.e. f, in FP32
    return SMG_OK;
  }

  // residual norms of the current iterate into rn (refined mode leaves the FP32 residual in
  // lv[0].bf)
  int enqueue_norms() {
    Hierarchy& h = hh->h;
    Level& v0 = h.lv[0];
    hipStream_t s = r.s;
    if (f32) {
      SMG_HIP(launch_refine_residual(v0.bf, v0.x, v0.b, v0.nx, v0.ny, v0.nz, nc, h.desc.ncomp,
                                     h.desc.h, h.part_d, h.norm_d, s));
    } else if (v0.kind == KIND_POINT) {
      SMG_HIP(launch_residual0<double>(v0.r, v0.x, v0.x + half_field(h), v0.b,
                                       v0.b + half_field(h), v0.nx, v0.ny, v0.nz, nc, h.desc.h,
                                       s));
      SMG_HIP(launch_sumsq(h.norm_d, h.part_d, v0.r, v0.n, nc, s));
    } else {
      // a level 0 drawn exactly (one level) is stored in natural layout; its residual goes to
      // its own buffer, never to u (which holds the exported solutions of finished chains)
      SMG_HIP(launch_residual7_nat(v0.r, v0.x, v0.b, v0.nx, v0.ny, v0.nz, nc, h.desc.h, s));
      SMG_HIP(launch_sumsq(h.norm_d, h.part_d, v0.r, v0.n, nc, s));
    }
    SMG_HIP(hipMemcpyAsync(rn.data(), h.norm_d, nc * sizeof(double), hipMemcpyDeviceToHost, s));
    return SMG_OK;
  }

  int check_norms() {
    for (int c = 0; c < nc; ++c)
      if (!std::isfinite(rn[c])) {
        set_error("residual is not finite");
        return SMG_ENONFINITE;
      }
    return SMG_OK;
  }

  int after_initial_norms() {
    SMG_TRY(check_norms());
    rprev = rn;
    ready = true;
    return SMG_OK;
  }

  bool wants_cycle() const { return pending > 0 && cycles < max_cycles; }

  // after the norms of cycle `cycles` (already counted) are on the host
  int after_norms() {
    Hierarchy& h = hh->h;
    SMG_TRY(check_norms());
    for (int ch = 0; ch < nch; ++ch) {
      if (cs[ch].done) continue;
      double relres = 0.0, ratio = 0.0;
      for (int c = ch * cpc; c < (ch + 1) * cpc; ++c) {
        const double rr =
            fn[c] > 0.0 ? std::sqrt(rn[c] / fn[c]) : (rn[c] > 0.0 ? INFINITY : 0.0);
        relres = rr > relres ? rr : relres;
        if (cycles >= 2 && rprev[c] > 0.0) {
          const double q = std::sqrt(rn[c] / rprev[c]);
          ratio = q > ratio ? q : ratio;
        }
      }
      cs[ch].relres = relres;
      cs[ch].last_ratio = ratio;
      cs[ch].cycles = cycles;
      if (relres <= rtol) {
        cs[ch].done = true;
        --pending;
        SMG_TRY(export_level0(h, (double*)u + (size_t)ch * cpc * h.lv[0].n, 0, h.lv[0].x, r.s,
                              cpc, ch * cpc));
      }
    }
    rprev = rn;
    return SMG_OK;
  }

  // exports the chains that did not converge; the caller synchronises before reading infos
  int finish_enqueue() {
    Hierarchy& h = hh->h;
    for (int ch = 0; ch < nch; ++ch)
      if (!cs[ch].done)
        SMG_TRY(export_level0(h, (double*)u + (size_t)ch * cpc * h.lv[0].n, 0, h.lv[0].x, r.s,
                              cpc, ch * cpc));
    return SMG_OK;
  }

  int finish_report() {
    if (infos)
      for (int ch = 0; ch < nch; ++ch) {
        infos[ch].cycles = cs[ch].cycles;
        infos[ch].relres = cs[ch].relres;
        infos[ch].last_ratio = cs[ch].last_ratio;
      }
    if (pending > 0) {
      double worst = 0.0;
      for (const auto& c : cs) worst = c.relres > worst ? c.relres : worst;
      set_error("solve did not converge: relres " + std::to_string(worst));
      return SMG_ENOTCONV;
    }
    return SMG_OK;
  }
};

int solve_impl(smg_hierarchy* hh, const Batch& bt, const void* f, void* u, double rtol,
               int32_t max_cycles, void* stream, smg_solve_info* infos) {
  SolveJob j;
  hipStream_t s = (hipStream_t)stream;
  SMG_TRY(j.begin(hh, bt, f, u, rtol, max_cycles, infos, s));
  SMG_TRY(j.enqueue_fnorm());
  SMG_HIP(hipStreamSynchronize(s));
  SMG_TRY(j.after_fnorm());
  if (j.initial_norms) {
    SMG_HIP(hipStreamSynchronize(s));
    SMG_TRY(j.after_initial_norms());
  }
  while (j.wants_cycle()) {
    SMG_TRY(full_cycle(j.r, j.ready));
    ++j.cycles;
    SMG_TRY(j.enqueue_norms());
    SMG_HIP(hipStreamSynchronize(s));
    SMG_TRY(j.after_norms());
  }
  SMG_TRY(j.finish_enqueue());
  SMG_HIP(hipStreamSynchronize(s));
  return j.finish_report();
}

}  // namespace

void set_error(const std::string& msg) { g_err = msg; }

// Points every device field and table of the hierarchy into ws (at least ws_bytes, 256-byte
// aligned, on the current device); with `upload` also copies the operator tables, factors and
// bottom-kernel descriptors there on stream s and synchronises it.  Without `upload` only the
// host-side pointers change: ws must already hold this hierarchy's tables.
int bind_impl(Hierarchy& h, char* ws, bool upload, hipStream_t s) {
  const bool f32 = refined(h);
  SMG_HIP(hipGetDevice(&h.device));
  for (size_t l = 0; l < h.lv.size(); ++l) {
    Level& v = h.lv[l];
    if (!f32 || l == 0) {
      v.x = (double*)(ws + v.off_x);
      v.b = (double*)(ws + v.off_b);
    }
    if (!f32) {
      v.r = (v.kind == KIND_CHOL && l > 0) ? nullptr : (double*)(ws + v.off_r);
    } else {
      v.xf = (float*)(ws + v.off_xf);
      v.bf = (float*)(ws + v.off_bf);
      v.rf = v.kind == KIND_CHOL ? nullptr : (float*)(ws + v.off_rf);
    }
    if (v.kind == KIND_BLOCK) {
      v.s1d_d = ws + v.off_s1d;
      v.zt_d = ws + v.off_zt;
      v.bfac_d = ws + v.off_bfac;
      v.noise_d = ws + v.off_noise;
      if (upload) {
        if (f32) SMG_TRY(upload_tables<float>(v, ws, s));
        else SMG_TRY(upload_tables<double>(v, ws, s));
      }
    }
  }
  if (h.nc > 0) {
    h.ainv_d = (double*)(ws + h.off_ainv);
    h.w_d = (double*)(ws + h.off_w);
    if (upload) {
      SMG_HIP(hipMemcpyAsync(h.ainv_d, h.ainv.data(), h.ainv.size() * sizeof(double),
                             hipMemcpyHostToDevice, s));
      SMG_HIP(hipMemcpyAsync(h.w_d, h.w.data(), h.w.size() * sizeof(double),
                             hipMemcpyHostToDevice, s));
    }
  }
  h.part_d = (double*)(ws + h.off_part);
  h.norm_d = (double*)(ws + h.off_norm);
  h.chains_d = (ChainKey*)(ws + h.off_chains);
  // the chain table and mode tables are workspace contents: taken as absent after a re-bind
  h.chains_set = 0;
  h.modes_valid = false;
  if (h.bottom >= 0) {
    h.botargs_d = (BotArgs*)(ws + h.off_botargs);
    if (upload) {
      BotArgs ba = make_botargs(h);
      SMG_HIP(hipMemcpyAsync(h.botargs_d, &ba, sizeof(BotArgs), hipMemcpyHostToDevice, s));
      SMG_HIP(hipStreamSynchronize(s));  // ba dies on return
    }
  }
  if (upload) SMG_HIP(hipStreamSynchronize(s));
  h.ws = ws;
  return SMG_OK;
}

int sample_field_impl(smg_hierarchy* hh, int64_t n, uint64_t seed, uint64_t first_cycle,
                      void* state, void* out, int32_t out_dtype, void* stream, int groups) {
  if (n > 0 && !out) {
    set_error("out is null");
    return SMG_EINVAL;
  }
  return sample_impl(hh, Batch{}, nullptr, nullptr, n, seed, first_cycle, state, out, out_dtype,
                     nullptr, 0, nullptr, nullptr, stream, groups);
}

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
  static std::atomic<uint64_t> next_uid{1};
  hh->h.uid = next_uid.fetch_add(1);
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
  return bind_impl(h, (char*)dev_ptr, true, (hipStream_t)stream);
}

int smg_sample_field(smg_hierarchy* hh, int64_t n, uint64_t seed, uint64_t first_cycle,
                     void* state, void* out, int32_t out_dtype, void* stream) {
  if (!hh) {
    set_error("null hierarchy");
    return SMG_EINVAL;
  }
  return sample_field_impl(hh, n, seed, first_cycle, state, out, out_dtype, stream,
                           hh->h.stream_groups);
}

int smg_sample_stats(smg_hierarchy* hh, int64_t n, uint64_t seed, uint64_t first_cycle,
                     void* state, void* out, int32_t out_dtype, const int32_t* modes,
                     int32_t n_modes, void* obs, void* moments, void* stream) {
  if (!hh) {
    set_error("null hierarchy");
    return SMG_EINVAL;
  }
  return sample_impl(hh, Batch{}, nullptr, nullptr, n, seed, first_cycle, state, out, out_dtype,
                     modes, n_modes, obs, moments, stream, hh->h.stream_groups);
}

int smg_sample_batch(smg_hierarchy* hh, int32_t nchains, int32_t comps_per_chain,
                     const uint64_t* seeds, const uint64_t* first_cycles, int64_t n, void* state,
                     void* out, int32_t out_dtype, const int32_t* modes, int32_t n_modes,
                     void* obs, void* moments, void* stream) {
  if (nchains < 1) {
    set_error("nchains must be >= 1");
    return SMG_EINVAL;
  }
  if (!hh) {
    set_error("null hierarchy");
    return SMG_EINVAL;
  }
  Batch bt;
  bt.nchains = nchains;
  bt.cpc = comps_per_chain;
  return sample_impl(hh, bt, seeds, first_cycles, n, 0, 0, state, out, out_dtype, modes, n_modes,
                     obs, moments, stream, hh->h.stream_groups);
}

int smg_solve_batch(smg_hierarchy* hh, int32_t nchains, int32_t comps_per_chain, const void* f,
                    void* u, double rtol, int32_t max_cycles, void* stream,
                    smg_solve_info* infos) {
  if (nchains < 1) {
    set_error("nchains must be >= 1");
    return SMG_EINVAL;
  }
  Batch bt;
  bt.nchains = nchains;
  bt.cpc = comps_per_chain;
  return solve_impl(hh, bt, f, u, rtol, max_cycles, stream, infos);
}

int smg_batch_run(smg_batch_item* items, int32_t n_items, void* stream) {
  if (n_items < 0 || (n_items > 0 && !items)) {
    set_error("invalid item list");
    return SMG_EINVAL;
  }
  for (int i = 0; i < n_items; ++i) {
    items[i].status = SMG_OK;
    for (int j = 0; j < i; ++j)
      if (items[i].h == items[j].h) {
        set_error("a hierarchy may appear only once in a batch");
        return SMG_EINVAL;
      }
  }
  hipStream_t s = (hipStream_t)stream;
  int first_err = SMG_OK;
  std::vector<char> alive(n_items, 0);
  auto fail = [&](int i, int rc) {
    items[i].status = rc;
    alive[i] = 0;
    if (first_err == SMG_OK) first_err = rc;
  };
  auto batch_of = [](const smg_batch_item& it) {
    Batch bt;
    if (it.nchains > 0) {
      bt.nchains = it.nchains;
      bt.cpc = it.comps_per_chain;
    }
    return bt;
  };
  for (int i = 0; i < n_items; ++i)
    if (items[i].op != SMG_OP_SAMPLE && items[i].op != SMG_OP_SOLVE) {
      set_error("unknown batch op");
      fail(i, SMG_EINVAL);
    } else if (items[i].nchains < 0) {
      set_error("nchains must be >= 0");
      fail(i, SMG_EINVAL);
    }
  // ---- sampling items: every cycle of every item, the bottoms of one cycle merged
  std::vector<SampleJob> sj(n_items);
  int64_t kmax = 0;
  for (int i = 0; i < n_items; ++i) {
    smg_batch_item& it = items[i];
    if (it.op != SMG_OP_SAMPLE || items[i].status != SMG_OK) continue;
    const int rc = sj[i].begin(it.h, batch_of(it), it.seeds, it.first_cycles, it.n, it.seed,
                               it.first_cycle, it.state, it.out, it.out_dtype, nullptr, 0,
                               nullptr, nullptr, s);
    if (rc != SMG_OK) {
      fail(i, rc);
      continue;
    }
    alive[i] = 1;
    kmax = std::max(kmax, sj[i].total);
  }
  // Stream groups (the largest setting among the sampling items' hierarchies; one stream while
  // any of them times kernels): group g takes components [g nc / ng, (g+1) nc / ng) of every
  // item, on its own stream, and starts each cycle once group g - 1 has finished that cycle's
  // down-legs, as in a single sampling call.
  int ng = 1;
  bool timing = false;
  Hierarchy* hs = nullptr;
  for (int i = 0; i < n_items; ++i)
    if (alive[i] && items[i].op == SMG_OP_SAMPLE) {
      Hierarchy& h = items[i].h->h;
      if (!hs) hs = &h;
      ng = std::max(ng, h.stream_groups);
      timing = timing || h.timing;
    }
  if (timing) ng = 1;
  if (ng > 1) {
    bool forked = ensure_side_streams(*hs, ng) == SMG_OK &&
                  hipEventRecord(hs->ev_fork, s) == hipSuccess;
    for (int g = 0; g < ng && forked; ++g)
      forked = hipStreamWaitEvent(hs->side[g], hs->ev_fork, 0) == hipSuccess;
    if (!forked) {
      set_error("could not set up the stream groups");
      for (int i = 0; i < n_items; ++i)
        if (alive[i] && items[i].op == SMG_OP_SAMPLE) fail(i, SMG_EHIP);
      ng = 1;
    }
  }
  std::vector<std::vector<Run>> gr(ng, std::vector<Run>(n_items));
  for (int g = 0; g < ng; ++g)
    for (int i = 0; i < n_items; ++i)
      if (alive[i] && items[i].op == SMG_OP_SAMPLE) {
        Run& r = gr[g][i];
        r = sj[i].r;
        r.c0 = g * sj[i].nc / ng;
        r.nc = (g + 1) * sj[i].nc / ng - r.c0;
        if (ng > 1) r.s = hs->side[g];
      }
  for (int64_t k = 0; k < kmax; ++k) {
    bool any_run = false;
    for (int g = 0; g < ng; ++g) {
      std::vector<Run*> runs;
      std::vector<int> who;
      for (int i = 0; i < n_items; ++i)
        if (alive[i] && items[i].op == SMG_OP_SAMPLE && k < sj[i].total && gr[g][i].nc > 0) {
          gr[g][i].cycle = sj[i].cycle_of(k);
          runs.push_back(&gr[g][i]);
          who.push_back(i);
        }
      if (runs.empty()) continue;
      any_run = true;
      const hipStream_t gs = runs[0]->s;
      const std::vector<char> ready(runs.size(), 0);
      int rc = SMG_OK;
      if (g > 0 && hipStreamWaitEvent(gs, hs->ev_mid[g - 1], 0) != hipSuccess) {
        set_error("hipStreamWaitEvent failed");
        rc = SMG_EHIP;
      }
      if (rc == SMG_OK) rc = batch_cycle(runs, ready, PH_IN | PH_DOWN);
      if (rc == SMG_OK && g + 1 < ng && hipEventRecord(hs->ev_mid[g], gs) != hipSuccess) {
        set_error("hipEventRecord failed");
        rc = SMG_EHIP;
      }
      if (rc == SMG_OK) rc = batch_cycle(runs, ready, PH_BOTTOM | PH_UP | PH_OUT);
      for (size_t q = 0; q < who.size(); ++q) {
        const int i = who[q];
        if (rc != SMG_OK) {
          fail(i, rc);
          continue;
        }
        const int re = sj[i].emit_after(k, *runs[q]);
        if (re != SMG_OK) fail(i, re);
      }
    }
    if (!any_run) break;
  }
  // the call's stream waits for the side streams before the state exports
  for (int g = 0; g < ng && ng > 1; ++g) {
    SMG_HIP(hipEventRecord(hs->ev_join[g], hs->side[g]));
    SMG_HIP(hipStreamWaitEvent(s, hs->ev_join[g], 0));
  }
  for (int i = 0; i < n_items; ++i)
    if (alive[i] && items[i].op == SMG_OP_SAMPLE) {
      const int rc = sj[i].finish();
      if (rc != SMG_OK) fail(i, rc);
      alive[i] = 0;
    }
  // ---- solve items: every cycle of every unfinished item, one synchronisation per cycle
  std::vector<SolveJob> vj(n_items);
  bool any = false;
  for (int i = 0; i < n_items; ++i) {
    smg_batch_item& it = items[i];
    if (it.op != SMG_OP_SOLVE || items[i].status != SMG_OK) continue;
    int rc = vj[i].begin(it.h, batch_of(it), it.f, it.u, it.rtol, it.max_cycles, it.infos, s);
    if (rc == SMG_OK) rc = vj[i].enqueue_fnorm();
    if (rc != SMG_OK) {
      fail(i, rc);
      continue;
    }
    alive[i] = 1;
    any = true;
  }
  if (any) {
    SMG_HIP(hipStreamSynchronize(s));
    bool init = false;
    for (int i = 0; i < n_items; ++i)
      if (alive[i]) {
        const int rc = vj[i].after_fnorm();
        if (rc != SMG_OK) fail(i, rc);
        init = init || (alive[i] && vj[i].initial_norms);
      }
    if (init) {
      SMG_HIP(hipStreamSynchronize(s));
      for (int i = 0; i < n_items; ++i)
        if (alive[i] && vj[i].initial_norms) {
          const int rc = vj[i].after_initial_norms();
          if (rc != SMG_OK) fail(i, rc);
        }
    }
    for (;;) {
      std::vector<Run*> runs;
      std::vector<char> ready;
      std::vector<int> who;
      for (int i = 0; i < n_items; ++i)
        if (alive[i] && vj[i].wants_cycle()) {
          runs.push_back(&vj[i].r);
          ready.push_back(vj[i].ready);
          who.push_back(i);
        }
      if (runs.empty()) break;
      const int rc = batch_cycle(runs, ready);
      for (int i : who) {
        if (rc != SMG_OK) {
          fail(i, rc);
          continue;
        }
        ++vj[i].cycles;
        const int re = vj[i].enqueue_norms();
        if (re != SMG_OK) fail(i, re);
      }
      SMG_HIP(hipStreamSynchronize(s));
      for (int i : who)
        if (alive[i]) {
          const int re = vj[i].after_norms();
          if (re != SMG_OK) fail(i, re);
        }
    }
    for (int i = 0; i < n_items; ++i)
      if (alive[i]) {
        const int rc = vj[i].finish_enqueue();
        if (rc != SMG_OK) fail(i, rc);
      }
    SMG_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < n_items; ++i)
      if (alive[i]) {
        const int rc = vj[i].finish_report();
        if (rc != SMG_OK) fail(i, rc);
        alive[i] = 0;
      }
  }
  return first_err;
}

int smg_lowest_modes(int32_t nx, int32_t ny, int32_t nz, int32_t k, int32_t* modes) {
  if (nx < 2 || ny < 2 || nz < 1 || (nx & 1) || (ny & 1) || k < 0 || k > kMaxModes ||
      (int64_t)k > (int64_t)nx * ny * nz || (k > 0 && !modes)) {
    set_error("invalid grid or k");
    return SMG_EINVAL;
  }
  struct Cand {
    int64_t key;
    int m, b, a;
  };
  std::vector<Cand> c;
  const int am = std::min(nx, 2 * k + 2), bm = std::min(ny, 2 * k + 2), mm = std::min(nz, k + 1);
  for (int m = 1; m <= mm; ++m)
    for (int b = 0; b < bm; ++b)
      for (int a = 0; a < am; ++a) {
        const double jx = periodic_wavenumber(nx, a), jy = periodic_wavenumber(ny, b);
        const double sx = std::sin(M_PI * jx / nx), sy = std::sin(M_PI * jy / ny);
        const double sz = std::sin(M_PI * m / (2.0 * nz));
        const double lam = 4.0 * sx * sx + 4.0 * sy * sy + 4.0 * sz * sz;
        c.push_back({(int64_t)std::llround(lam * 1073741824.0), m, b, a});
      }
  std::sort(c.begin(), c.end(), [](const Cand& p, const Cand& q) {
    if (p.key != q.key) return p.key < q.key;
    if (p.m != q.m) return p.m < q.m;
    if (p.b != q.b) return p.b < q.b;
    return p.a < q.a;
  });
  for (int q = 0; q < k; ++q) {
    modes[3 * q] = c[q].a;
    modes[3 * q + 1] = c[q].b;
    modes[3 * q + 2] = c[q].m;
  }
  return SMG_OK;
}

int smg_solve(smg_hierarchy* hh, const void* f, void* u, double rtol, int32_t max_cycles,
              void* stream, smg_solve_info* info) {
  return solve_impl(hh, Batch{}, f, u, rtol, max_cycles, stream, info);
}

void smg_destroy_hierarchy(smg_hierarchy* hh) {
  if (!hh) return;
  for (hipEvent_t e : hh->h.ev_pool) (void)hipEventDestroy(e);
  release_side_streams(hh->h);
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
  Run r = make_run(h, s, with_noise != 0, b != nullptr, seed, cycle);
  if (v.kind == KIND_POINT) {
    NoiseArgs na = make_noise(r, level, slot, colour, KIND_SMOOTH_NOISE);
    SMG_TRY(import_level0(h, v.x, (const double*)x, s));
    if (b) SMG_TRY(import_level0(h, v.b, (const double*)b, s));
    double* xr = v.x;
    double* xb = v.x + half_field(h);
    const double* bc = b ? (colour ? v.b + half_field(h) : v.b) : nullptr;
    SMG_TRY(rb_pass<double>(r, colour ? xb : xr, colour ? xr : xb, bc, colour, na));
    SMG_TRY(export_level0(h, x, 0, v.x, s));
  } else {
    if (r.noise) SMG_TRY(gen_level_noise<double>(r, level, slot));
    SMG_HIP(launch_block_pass<double>((double*)x, (const double*)b, (const double*)v.s1d_d,
                                      (const double*)v.zt_d, (const double*)v.bfac_d, v.nx, v.ny,
                                      v.nz, h.desc.ncomp, colour,
                                      r.noise ? (const double*)v.noise_d : nullptr,
                                      h.block_tile, s));
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
    // level 0: the cycle's own fused residual + restriction (the fine residual is never stored)
    SMG_TRY(import_level0(h, v.x, (const double*)x, s));
    if (b) SMG_TRY(import_level0(h, v.b, (const double*)b, s));
    SMG_HIP(launch_restrict_residual0<double>((double*)b_coarse, nullptr, v.x,
                                              v.x + half_field(h), b ? v.b : nullptr,
                                              b ? v.b + half_field(h) : nullptr, v.nx, v.ny,
                                              v.nz, nc, h.desc.h, s));
    return SMG_OK;
  } else {
    SMG_HIP(launch_residual_gal<double>(v.r, (const double*)x, (const double*)b,
                                        (const double*)v.s1d_d, (const double*)v.zt_d, v.nx,
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
                                    v.nz, nc, 3, s));
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
  Run r = make_run(h, s, with_noise != 0, false, seed, cycle);
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
  if (option == SMG_OPT_BLOCK_PAIRS && (value == 0 || value == 1)) {
    hh->h.block_pairs = value != 0;
    return SMG_OK;
  }
  if (option == SMG_OPT_STREAM_GROUPS && value >= 1 && value <= kMaxStreamGroups) {
    hh->h.stream_groups = (int)value;
    return SMG_OK;
  }
  if (option == SMG_OPT_BLOCK_TILE && value >= SMG_TILE_AUTO && value <= SMG_TILE_8X4) {
    hh->h.block_tile = (int)value;
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
  h.ev_launches.clear();
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
    h.tcount += i / 2 < h.ev_launches.size() ? h.ev_launches[i / 2] : 1;
  }
  h.ev_used = 0;
  h.ev_launches.clear();
  *count = h.tcount;
  *total_ms = h.tms;
  return SMG_OK;
}

}  // extern "C"
