// Fine-level kernels (red-black point heat bath on the 7-point operator).
//
// The fine field is stored split by colour: colour c (cells with (x+y+z)%2 == c) occupies
// [ncomp][nz][ny][nx/2], entry j of row (y,z) being x = 2j + ((y+z+c)&1).  Its y- and
// z-neighbours sit at the same entry j of the adjacent rows of the other colour, its
// x-neighbours at entries (j-1, j) or (j, j+1) of the same row.  A heat-bath update never
// reads the old value of the site it replaces, so one colour pass streams
// read(other colour) + write(own colour): the minimum traffic of a sweep.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.hpp"
#include "kernels.hpp"

namespace smg {
namespace {

template <typename T>
struct Vec2;
template <>
struct Vec2<double> {
  using type = double2;
};
template <>
struct Vec2<float> {
  using type = float2;
};

template <typename T>
struct Diag3 {
  T inv_d[3];  // h^2 / (6 + walls)
  T sig[3];    // sqrt(kT h^2 / (6 + walls))
  T inv_n[3];  // 1 / (6 + walls): the neighbour sum's weight when b = 0
};

template <typename T, int S>
struct Arr {
  T v[S];
};

// Normals of the level-0 colour passes: FP64 without the table load (the field loads issued
// before them stay in flight), FP32 as everywhere.
template <typename T>
__device__ __forceinline__ void level0_normals(const NoiseArgs& na, uint32_t comp, uint32_t call,
                                               T& z0, T& z1) {
  if constexpr (sizeof(T) == 8) {
    normal_pair_notable(na, na.sid, comp, call, z0, z1);
  } else {
    normal_pair_t<T>(na, comp, call, z0, z1);
  }
}

// 16 bytes of consecutive colour entries: the unit of a thread's loads and stores
template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
  using type = double2;
};
template <>
struct Vec16<float> {
  using type = float4;
};

// Colour pass, nh = nx/2 a multiple of S = 16/sizeof(T): thread (row, jt) owns the S sites
// j = S jt .. S jt + S-1 of a row (FP64: one pair, FP32: two pairs; pair p of the row is
// Philox call row*nh/2 + p, whatever the launch) and moves them with one 16-byte load per
// neighbour row and one 16-byte store.  The first site's entry is S t; every access is a
// 32-bit byte offset from the component's base (the launch checks that a component's colour
// array is below 4 GiB), so the loads take a scalar base and a 32-bit lane offset.  ZU: the
// launch guarantees that every wave stays in one z-plane (nh/S * ny a multiple of 64), so the
// wall tests and the diagonal of the plane are taken once per wave on the scalar unit.  A wall
// side enters the z-sum with weight 0.
// The pass of work-group `blk` of component `comp`.
template <typename T, bool HAS_B, bool NOISE, bool ZU>
__device__ __forceinline__ void rb_pass_vec_body(T* __restrict__ xc, const T* __restrict__ xo,
                                                 const T* __restrict__ bc, int nh, int ny, int nz,
                                                 uint32_t nthreads, int lg_nht, int lg_ny,
                                                 int colour, T inv_h2, const Diag3<T>& dg,
                                                 const NoiseArgs& na, uint32_t blk,
                                                 uint32_t comp) {
  using V = typename Vec16<T>::type;
  constexpr uint32_t W = sizeof(T), S = 16 / W;
  // FP64 with noise: a new wave issues its addressing and loads at raised priority, ahead of the
  // resident waves' noise arithmetic, so its memory latency starts as early as possible (each
  // wave waits on its loads for much of its life); it drops to the normal priority for its own
  // noise.  The FP32 pass, bound by memory, gains nothing.
  constexpr bool PRIO = NOISE && sizeof(T) == 8;
  if (PRIO) __builtin_amdgcn_s_setprio(3);
  const uint32_t t = blk * TPB + threadIdx.x;
  if (t >= nthreads) return;
  const uint32_t nht = (uint32_t)nh / S;
  uint32_t row, jt, z, y;
  if (lg_nht >= 0) {
    row = t >> lg_nht;
    jt = t & (nht - 1);
  } else {
    row = t / nht;
    jt = t - row * nht;
  }
  if (lg_ny >= 0) {
    z = row >> lg_ny;
    y = row & ((uint32_t)ny - 1);
  } else {
    z = row / (uint32_t)ny;
    y = row - z * (uint32_t)ny;
  }
  const uint32_t nsite = (uint32_t)nh * ny * nz;
  const size_t base = (size_t)comp * nsite;
  const char* __restrict__ ob = reinterpret_cast<const char*>(xo + base);
  const uint32_t plane = (uint32_t)nh * ny;
  const uint32_t ic = S * t;          // row * nh + S jt
  const uint32_t rb = ic - S * jt;    // row * nh
  const uint32_t xs = (y + z + (uint32_t)colour) & 1u;
  // 16-byte vector <-> S scalars by value copies (no type punning of registers)
  auto ld = [&](uint32_t e) {
    const V t = *reinterpret_cast<const V*>(ob + e * W);
    Arr<T, S> a;
    __builtin_memcpy(a.v, &t, sizeof(V));
    return a;
  };

  // own row: the S entries and the one beyond on the side the x-neighbours lie
  const Arr<T, S> c = ld(ic);
  const uint32_t ie = xs ? (jt + 1 == nht ? rb : ic + S) : (jt == 0 ? rb + (uint32_t)nh - 1 : ic - 1);
  const T ex = *reinterpret_cast<const T*>(ob + ie * W);
  const uint32_t in = ic + (y + 1 == (uint32_t)ny ? (uint32_t)nh - plane : (uint32_t)nh);
  const uint32_t is = ic + (y == 0 ? plane - (uint32_t)nh : 0u - (uint32_t)nh);
  const Arr<T, S> n = ld(in), so = ld(is);
  // the planes above and below, clamped at the walls (all loads unconditional and in flight
  // at once)
  const uint32_t zw = ZU ? __builtin_amdgcn_readfirstlane(z) : z;
  const bool top = zw + 1 >= (uint32_t)nz, bottom = zw == 0;
  const Arr<T, S> u = ld(ic + (top ? 0u : plane)), d = ld(ic - (bottom ? 0u : plane));
  Arr<T, S> b;
  if (HAS_B) {
    const V t = *reinterpret_cast<const V*>(reinterpret_cast<const char*>(bc + base) + ic * W);
    __builtin_memcpy(b.v, &t, sizeof(V));
  }
  const int nw = (int)top + (int)bottom;
  const T wu = top ? T(0) : T(1), wd = bottom ? T(0) : T(1);
  const T idg = dg.inv_d[nw], sgm = dg.sig[nw], inn = dg.inv_n[nw];
  // The normals depend on no load: with every load issued above, the Philox and Box-Muller
  // arithmetic runs while they are in flight (the scheduling barriers keep the compiler from
  // hoisting the sums, which wait for the loads, in front of it).
  T zn[S];
#pragma unroll
  for (uint32_t k = 0; k < S; ++k) zn[k] = T(0);
  if (NOISE) {
    __builtin_amdgcn_sched_barrier(0);
    if (PRIO) __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (uint32_t p = 0; p < S / 2; ++p)
      level0_normals<T>(na, comp, (S / 2) * t + p, zn[2 * p], zn[2 * p + 1]);
    __builtin_amdgcn_sched_barrier(0);
  }
  // x-neighbour sums: xs == 1 -> (j, j+1), xs == 0 -> (j-1, j); the entry beyond the owned
  // ones closes the last pair on the side it lies
  T a[S];
#pragma unroll
  for (uint32_t k = 0; k + 1 < S; ++k) a[k] = c.v[k] + c.v[k + 1];
  const T ed = ex + (xs ? c.v[S - 1] : c.v[0]);
  T out[S];
#pragma unroll
  for (uint32_t k = 0; k < S; ++k) {
    const T sx = xs ? (k + 1 < S ? a[k] : ed) : (k > 0 ? a[k - 1] : ed);
    const T sum = (sx + (n.v[k] + so.v[k])) + fma(u.v[k], wu, d.v[k] * wd);
    T v;
    if (HAS_B)
      v = fma(sum, inv_h2, b.v[k]) * idg;
    else
      v = sum * inn;
    if (NOISE) v = fma(sgm, zn[k], v);
    out[k] = v;
  }
  V ov;
  __builtin_memcpy(&ov, out, sizeof(V));
  *reinterpret_cast<V*>(reinterpret_cast<char*>(xc + base) + ic * W) = ov;
}

template <typename T, bool HAS_B, bool NOISE, bool ZU = false>
__global__ __launch_bounds__(TPB) void k_rb_pass_vec(T* __restrict__ xc, const T* __restrict__ xo,
                                                      const T* __restrict__ bc, int nh, int ny,
                                                      int nz, uint32_t nthreads, int lg_nht,
                                                      int lg_ny, int colour, T inv_h2,
                                                      Diag3<T> dg, NoiseArgs na) {
  rb_pass_vec_body<T, HAS_B, NOISE, ZU>(xc, xo, bc, nh, ny, nz, nthreads, lg_nht, lg_ny, colour,
                                        inv_h2, dg, na, blockIdx.x, blockIdx.y);
}

// The same colour pass on the level 0 of several hierarchies in one launch: the grid is the
// concatenation of every item's (block, component) grid; a work-group finds its item from the
// offsets.  Each item brings its own noise keys; the Box-Muller coefficients are shared.
struct RbNoiseKey {
  uint32_t k0, k1, sid, c2, c3, cpc, cpc_magic, comp0;
  double sqkT;
  const ChainKey* chains;
};
constexpr int kRbMultiItems = 8;
template <typename T>
struct RbMultiItem {
  T* xc;
  const T* xo;
  const T* bc;
  int nh, ny, nz, lg_nht, lg_ny;
  uint32_t nthreads, nblk;
  T inv_h2;
  Diag3<T> dg;
  RbNoiseKey nk;
};
template <typename T>
struct RbMultiArgs {
  int nitems, colour;
  uint32_t begin[kRbMultiItems + 1];
  BoxMullerCoef bm;
  RbMultiItem<T> it[kRbMultiItems];
};

template <typename T, bool HAS_B, bool NOISE>
__global__ __launch_bounds__(TPB) void k_rb_pass_vec_multi(RbMultiArgs<T> m) {
  const uint32_t lin = blockIdx.x;
  int i = 0;
  while (i + 1 < m.nitems && lin >= m.begin[i + 1]) ++i;
  const RbMultiItem<T>& it = m.it[i];
  const uint32_t local = lin - m.begin[i];
  NoiseArgs na;
  na.k0 = it.nk.k0;
  na.k1 = it.nk.k1;
  na.sid = it.nk.sid;
  na.c2 = it.nk.c2;
  na.c3 = it.nk.c3;
  na.sqkT = it.nk.sqkT;
  na.chains = it.nk.chains;
  na.comps_per_chain = it.nk.cpc;
  na.cpc_magic = it.nk.cpc_magic;
  na.comp0 = it.nk.comp0;
  na.bm = m.bm;
  rb_pass_vec_body<T, HAS_B, NOISE, false>(it.xc, it.xo, it.bc, it.nh, it.ny, it.nz,
                                           it.nthreads, it.lg_nht, it.lg_ny, m.colour, it.inv_h2,
                                           it.dg, na, local % it.nblk, local / it.nblk);
}

// Generic colour pass (any even nx): thread q owns colour sites 2q and 2q+1 (one Philox call).
template <typename T, bool HAS_B, bool NOISE>
__global__ __launch_bounds__(TPB) void k_rb_pass(T* __restrict__ xc, const T* __restrict__ xo,
                                                  const T* __restrict__ bc, int nh, int ny, int nz,
                                                  uint32_t nsite, int colour, T inv_h2,
                                                  Diag3<T> dg, NoiseArgs na) {
  const uint32_t comp = blockIdx.y;
  const uint32_t q = blockIdx.x * TPB + threadIdx.x;
  const uint32_t p0 = 2u * q;
  if (p0 >= nsite) return;
  const size_t base = (size_t)comp * nsite;
  const T* __restrict__ o = xo + base;
  T z0 = 0, z1 = 0;
  if (NOISE) level0_normals<T>(na, comp, q, z0, z1);
  const uint32_t plane = (uint32_t)nh * ny;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const uint32_t p = p0 + t;
    if (p >= nsite) break;
    const uint32_t row = p / nh;
    const int j = p - row * nh;
    const int y = row % ny;
    const int z = row / ny;
    const int xs = (y + z + colour) & 1;
    const uint32_t rb = row * nh;
    const int jl = xs ? j : (j == 0 ? nh - 1 : j - 1);
    const int jr = xs ? (j == nh - 1 ? 0 : j + 1) : j;
    T s = o[rb + jl] + o[rb + jr];
    const int yn = (y + 1 == ny) ? 0 : y + 1;
    const int ys = (y == 0) ? ny - 1 : y - 1;
    s += o[((uint32_t)z * ny + yn) * nh + j] + o[((uint32_t)z * ny + ys) * nh + j];
    int nw = 0;
    if (z + 1 < nz) s += o[rb + j + plane]; else ++nw;
    if (z > 0) s += o[rb + j - plane]; else ++nw;
    T v = s * inv_h2;
    if (HAS_B) v += bc[base + p];
    v *= dg.inv_d[nw];
    if (NOISE) v += dg.sig[nw] * (t == 0 ? z0 : z1);
    xc[base + p] = v;
  }
}

template <typename T>
__device__ __forceinline__ T split_at(const T* __restrict__ xr, const T* __restrict__ xb,
                                      size_t cbase, int x, int y, int z, int nh, int ny) {
  const T* a = ((x + y + z) & 1) ? xb : xr;
  return a[cbase + ((size_t)z * ny + y) * nh + (x >> 1)];
}

// r = b - A x on level 0 (split input, natural output).
template <typename T, bool HAS_B>
__global__ __launch_bounds__(TPB) void k_residual0(T* __restrict__ r, const T* __restrict__ xr,
                                                    const T* __restrict__ xb,
                                                    const T* __restrict__ br,
                                                    const T* __restrict__ bb, int nx, int ny,
                                                    int nz, uint32_t N, T inv_h2) {
  const uint32_t comp = blockIdx.y;
  const uint32_t i = blockIdx.x * TPB + threadIdx.x;
  if (i >= N) return;
  const int x = i % nx;
  const uint32_t row = i / nx;
  const int y = row % ny;
  const int z = row / ny;
  const int nh = nx >> 1;
  const size_t cb = (size_t)comp * (N >> 1);
  T c = split_at(xr, xb, cb, x, y, z, nh, ny);
  T s = split_at(xr, xb, cb, wrapm(x - 1, nx), y, z, nh, ny) +
        split_at(xr, xb, cb, wrapm(x + 1, nx), y, z, nh, ny) +
        split_at(xr, xb, cb, x, wrapm(y - 1, ny), z, nh, ny) +
        split_at(xr, xb, cb, x, wrapm(y + 1, ny), z, nh, ny);
  int nw = 0;
  if (z + 1 < nz) s += split_at(xr, xb, cb, x, y, z + 1, nh, ny); else ++nw;
  if (z > 0) s += split_at(xr, xb, cb, x, y, z - 1, nh, ny); else ++nw;
  T ax = (T(6 + nw) * c - s) * inv_h2;
  T bv = HAS_B ? split_at(br, bb, cb, x, y, z, nh, ny) : T(0);
  r[(size_t)comp * N + i] = bv - ax;
}

// Fused residual and restriction from level 0: b_c = P^T (b - A x) without writing r.
// A work-group owns an RX x RY column of coarse cells over up to RR_Z coarse layers and
// marches up through the fine planes of their restriction windows, [2Z0-1, 2Z0+2RZ].  For
// each fine plane f it stages x plane f+1 into a ring of four LDS planes (the global loads
// of the planes up to four steps ahead are in flight meanwhile), forms the residual of
// plane f over the (2RX+2) x (2RY+2) window of the column, and every coarse cell of the column
// takes that plane's 4x4 window sum (weights 1/4, 3/4, 3/4, 1/4 per axis; 1/2 for a fine cell
// next to a wall) into the running sums of the two coarse layers the plane belongs to: 4, 2 or
// 1 lanes per coarse cell (TPB / (RX RY)), each summing 1, 2 or 4 window columns, joined by
// shuffles in the same order for every shape.  Each x plane is loaded once per column and each
// residual plane formed once, instead of once per coarse layer pair.  Also zeroes the coarse
// iterate when xc is not null.
constexpr int RR_Z = 8;
constexpr int RR_PF = 4;  // x planes loaded ahead
template <int RX, int RY>
struct RRShape {
  static constexpr int FX = 2 * RX + 2, FY = 2 * RY + 2;  // residual window of a plane
  static constexpr int SX = FX + 2, SY = FY + 2;          // x box of a plane
  static constexpr int XP = SX * SY;                      // x plane in LDS
  // The residual window is formed and stored with the x box's row stride SX (two idle lanes
  // per row), so consecutive lanes touch consecutive LDS words: no bank conflicts.
  static constexpr int RP = SX * FY;                      // residual plane in LDS
  static constexpr int PPT = (XP + TPB - 1) / TPB;        // x positions per thread
  static constexpr int RPT = (RP + TPB - 1) / TPB;        // residual positions per thread
  static constexpr int LPC = TPB / (RX * RY);             // lanes per coarse cell
  static constexpr int CPL = 4 / LPC;                     // window columns per lane
  static_assert(RX * RY * LPC == TPB && (LPC == 1 || LPC == 2 || LPC == 4),
                "1, 2 or 4 lanes per coarse cell of the column");
};

template <typename T, bool HAS_B, int RX, int RY>
__global__ __launch_bounds__(TPB) void k_restrict_residual0(
    T* __restrict__ bc, T* __restrict__ xc, const T* __restrict__ xr, const T* __restrict__ xb,
    const T* __restrict__ br, const T* __restrict__ bb, int nx, int ny, int nz, int ntx,
    T inv_h2) {
  using Sh = RRShape<RX, RY>;
  constexpr int RR_SX = Sh::SX, RR_XP = Sh::XP, RR_RP = Sh::RP, RR_FX = Sh::FX;
  constexpr int RR_PPT = Sh::PPT, RR_RPT = Sh::RPT;
  __shared__ T Xs[4 * RR_XP + 1];  // + a pad element for positions past the plane
  __shared__ T Rs[2 * RR_RP];
  const Blk3 wg = xcd_block();
  const uint32_t comp = wg.z;
  const int nxc = nx >> 1, nyc = ny >> 1, nzc = nz >> 1;
  const int X0 = (wg.x % ntx) * RX, Y0 = (wg.x / ntx) * RY;
  const int Z0 = wg.y * RR_Z;
  const int zc = min(RR_Z, nzc - Z0);
  const int nh = nx >> 1;
  const size_t cb = (size_t)comp * ((size_t)(nx >> 1) * ny * nz);
  const int tid = threadIdx.x;
  // x positions this thread stages (box origin 2X0-2, 2Y0-2) and residual positions it forms
  // (window origin 2X0-1, 2Y0-1)
  // per staged position: its entry within a plane of the split arrays and its colour in
  // plane 0 (the colour alternates with the plane)
  uint32_t xent[RR_PPT];
  int xpar[RR_PPT], xoff[RR_PPT];
#pragma unroll
  for (int p = 0; p < RR_PPT; ++p) {
    const int pos = tid + p * TPB;
    const int sx = pos % RR_SX, sy = pos / RR_SX;
    xoff[p] = pos < RR_XP ? pos : -1;
    const int gx = wrap_near(2 * X0 - 2 + sx, nx);
    const int gy = pos < RR_XP ? wrap_near(2 * Y0 - 2 + sy, ny) : 0;
    xent[p] = (uint32_t)gy * nh + (gx >> 1);
    xpar[p] = (gx + gy) & 1;
  }
  const uint32_t hplane = (uint32_t)nh * ny;
  int roff[RR_RPT], rxo[RR_RPT];
#pragma unroll
  for (int p = 0; p < RR_RPT; ++p) {
    const int q = tid + p * TPB;
    const int rx = q % RR_SX, ry = q / RR_SX;
    roff[p] = (q < RR_RP && rx < RR_FX) ? q : -1;
    rxo[p] = (ry + 1) * RR_SX + rx + 1;  // centre of the 7-point star in an x plane
  }
  const int f0 = 2 * Z0 - 1, f1 = 2 * (Z0 + zc);  // residual planes of the column
  auto load_plane = [&](T (&reg)[RR_PPT], int g) {
    g = g < 0 ? 0 : (g >= nz ? nz - 1 : g);  // planes beyond the walls are never read
    const T* pr = xr + cb + (size_t)g * hplane;
    const T* pb = xb + cb + (size_t)g * hplane;
#pragma unroll
    for (int p = 0; p < RR_PPT; ++p) reg[p] = ((xpar[p] ^ g) & 1 ? pb : pr)[xent[p]];
  };
  auto store_plane = [&](const T (&reg)[RR_PPT], int g) {
    const int slot = (g & 3) * RR_XP;
#pragma unroll
    for (int p = 0; p < RR_PPT; ++p)  // positions past the plane store into the pad element
      Xs[xoff[p] >= 0 ? slot + xoff[p] : 4 * RR_XP] = reg[p];
  };
  auto load_b = [&](T (&reg)[RR_RPT], int f) {
    const int g = f < 0 ? 0 : (f >= nz ? nz - 1 : f);
#pragma unroll
    for (int p = 0; p < RR_RPT; ++p) {
      const int q = roff[p] < 0 ? 0 : roff[p];
      const int fx = wrap_near(2 * X0 - 1 + q % RR_SX, nx);
      const int fy = wrap_near(2 * Y0 - 1 + q / RR_SX, ny);
      reg[p] = HAS_B ? split_at(br, bb, cb, fx, fy, g, nh, ny) : T(0);
    }
  };
  // this lane's coarse cell and window columns
  const int wb = tid % Sh::LPC, cell = tid / Sh::LPC;
  const int lx = cell % RX, ly = cell / RX;
  const int X = X0 + lx, Y = Y0 + ly;
  const bool owner = wb == 0 && X < nxc && Y < nyc;
  T acc0 = 0, acc1 = 0;  // running sums of the even and the odd coarse layer
  // one fine plane f: stage x plane f+1 (held in `cur`), start loading plane f+1+RR_PF into
  // `cur` once stored, form the residual of plane f, and take its window sums
  auto step = [&](int f, T (&cur)[RR_PPT], T (&bcur)[RR_RPT]) {
    store_plane(cur, f + 1);
    if (f + 1 + RR_PF <= f1 + 1) load_plane(cur, f + 1 + RR_PF);
    __syncthreads();
    T* R = Rs + (f & 1) * RR_RP;
    if (f >= 0 && f < nz) {
      const T* Pm = Xs + ((f - 1) & 3) * RR_XP;
      const T* P0 = Xs + (f & 3) * RR_XP;
      const T* Pp = Xs + ((f + 1) & 3) * RR_XP;
#pragma unroll
      for (int p = 0; p < RR_RPT; ++p) {
        if (roff[p] < 0) continue;
        const T* c = P0 + rxo[p];
        T sn = (c[-1] + c[1]) + (c[-RR_SX] + c[RR_SX]);
        int nw = 0;
        if (f + 1 < nz) sn += Pp[rxo[p]]; else ++nw;
        if (f > 0) sn += Pm[rxo[p]]; else ++nw;
        T rv = -(T(6 + nw) * c[0] - sn) * inv_h2;
        if (HAS_B) rv += bcur[p];
        R[roff[p]] = rv;
      }
    }
    if (HAS_B && f + 2 <= f1) load_b(bcur, f + 2);
    __syncthreads();
    if (f < 0 || f >= nz) return;
    // lane wb takes window columns wb CPL .. wb CPL + CPL - 1 (x offsets) down the four rows
    // (with four lanes per cell the lanes of a wave read one contiguous run of the row at a
    // time); the column sums join as ((c0 + c1) + (c2 + c3)) whatever the lanes per cell
    T cs[Sh::CPL];
#pragma unroll
    for (int q = 0; q < Sh::CPL; ++q) {
      const int col = wb * Sh::CPL + q;
      const T* Rr = R + 2 * ly * RR_SX + 2 * lx + col;
      T c = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) c = fma(pw<T>(b), Rr[b * RR_SX], c);
      cs[q] = c * pw<T>(col);
    }
    T s;
    if constexpr (Sh::LPC == 4) {
      s = cs[0];
      s += __shfl_xor(s, 1, 4);
      s += __shfl_xor(s, 2, 4);
    } else if constexpr (Sh::LPC == 2) {
      s = cs[0] + cs[1];
      s += __shfl_xor(s, 1, 2);
    } else {
      s = (cs[0] + cs[1]) + (cs[2] + cs[3]);
    }
    // plane f is window plane c1 of coarse layer Z1 and plane c1 + 2 of layer Z1 - 1
    const int Z1 = (f + 1) >> 1, c1 = f - (2 * Z1 - 1);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int Z = Z1 - k, c = c1 + 2 * k;
      if (Z < Z0 || Z >= Z0 + zc) continue;
      T wz = pw<T>(c);
      if ((Z == 0 && f == 0) || (Z == nzc - 1 && f == nz - 1)) wz = T(0.5);
      if (Z & 1) acc1 = fma(wz, s, acc1);
      else acc0 = fma(wz, s, acc0);
    }
  };
  // the layer Z1 - 1 is complete after its window plane 3, i.e. after an even plane f
  auto finish = [&](int f) {
    if (f & 1) return;
    const int Z = (f >> 1) - 1;
    if (Z < Z0 || Z >= Z0 + zc) return;
    if (owner) {
      const size_t I = (size_t)comp * nxc * nyc * nzc + ((size_t)Z * nyc + Y) * nxc + X;
      bc[I] = (Z & 1) ? acc1 : acc0;
      if (xc) xc[I] = T(0);
    }
    if (Z & 1) acc1 = T(0);
    else acc0 = T(0);
  };
  // prologue: planes f0-1 and f0 in the ring, f0+1 .. f0+RR_PF in the register sets
  T r0[RR_PPT], r1[RR_PPT], r2[RR_PPT], r3[RR_PPT], ba[RR_RPT], bbn[RR_RPT];
  load_plane(r0, f0 - 1);
  load_plane(r1, f0);
  if (HAS_B) {
    load_b(ba, f0);
    load_b(bbn, f0 + 1);
  }
  store_plane(r0, f0 - 1);
  store_plane(r1, f0);
  load_plane(r0, f0 + 1);
  load_plane(r1, f0 + 2);
  if (f0 + 3 <= f1 + 1) load_plane(r2, f0 + 3);
  if (f0 + 4 <= f1 + 1) load_plane(r3, f0 + 4);
  // RR_PF planes at a time, so that the register sets keep their roles (x planes RR_PF ahead,
  // b two ahead)
  for (int f = f0; f <= f1; f += RR_PF) {
    step(f, r0, ba);
    finish(f);
    if (f + 1 > f1) break;
    step(f + 1, r1, bbn);
    finish(f + 1);
    if (f + 2 > f1) break;
    step(f + 2, r2, ba);
    finish(f + 2);
    if (f + 3 > f1) break;
    step(f + 3, r3, bbn);
    finish(f + 3);
  }
}

// FP32-refined bridge: r32 = (float)(b - A x) from FP64 split storage, written split; the
// optional fixed-order partial sums of (b - A x)^2 go to part[comp][colour*nblk + block].
template <bool HAS_B, bool NORM>
__global__ __launch_bounds__(TPB) void k_refine_residual(float* __restrict__ r32,
                                                          const double* __restrict__ x64,
                                                          const double* __restrict__ b64, int nx,
                                                          int ny, int nz, uint32_t nsite,
                                                          double inv_h2, double* __restrict__ part,
                                                          uint32_t nblk, size_t half) {
  __shared__ double sh[TPB];
  const uint32_t comp = blockIdx.y;
  const int colour = blockIdx.z;
  const uint32_t p = blockIdx.x * TPB + threadIdx.x;
  const int nh = nx >> 1;
  const double* xr = x64;
  const double* xb = x64 + half;
  double rr = 0.0;
  if (p < nsite) {
    const uint32_t row = p / nh;
    const int j = p - row * nh;
    const int y = row % ny;
    const int z = row / ny;
    const int x = 2 * j + ((y + z + colour) & 1);
    const size_t cb = (size_t)comp * nsite;
    const double c = split_at(xr, xb, cb, x, y, z, nh, ny);
    double s = split_at(xr, xb, cb, wrapm(x - 1, nx), y, z, nh, ny) +
               split_at(xr, xb, cb, wrapm(x + 1, nx), y, z, nh, ny) +
               split_at(xr, xb, cb, x, wrapm(y - 1, ny), z, nh, ny) +
               split_at(xr, xb, cb, x, wrapm(y + 1, ny), z, nh, ny);
    int nw = 0;
    if (z + 1 < nz) s += split_at(xr, xb, cb, x, y, z + 1, nh, ny); else ++nw;
    if (z > 0) s += split_at(xr, xb, cb, x, y, z - 1, nh, ny); else ++nw;
    const double bv = HAS_B ? b64[colour * half + cb + p] : 0.0;
    rr = bv - ((6 + nw) * c - s) * inv_h2;
    r32[colour * half + cb + p] = (float)rr;
  }
  if (NORM) {
    sh[threadIdx.x] = rr * rr;
    __syncthreads();
    for (int st = TPB / 2; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)comp * 2 * nblk + colour * nblk + blockIdx.x] = sh[0];
  }
}

// The same residual (without norms) two sites per thread, as the colour passes move the field:
// thread (row, jt) of colour c owns sites 2 jt, 2 jt + 1 of its row, reads them and b with one
// 16-byte load each and its neighbours in the other colour's array with one 16-byte load per
// neighbour row (plus the entry beyond on the side its x-neighbours lie), and writes both
// residuals with one 8-byte store.  The neighbour sums run in the order of k_refine_residual,
// so both kernels give the same bits.
template <bool HAS_B, bool ZU>
__global__ __launch_bounds__(TPB) void k_refine_residual_vec(float* __restrict__ r32,
                                                              const double* __restrict__ x64,
                                                              const double* __restrict__ b64,
                                                              int nh, int ny, int nz,
                                                              uint32_t nthreads, int lg_nht,
                                                              int lg_ny, double inv_h2,
                                                              size_t half) {
  constexpr uint32_t S = 2;
  // Work-group order: the two colours of a tile run one after the other and, by the XCD-aware
  // numbering, on one XCD, so the rows that one colour reads as neighbours and the other as
  // its own sites come from HBM once and from that XCD's L2 the second time
  const uint32_t nb = gridDim.x, ncw = gridDim.y;
  uint32_t lin = blockIdx.x + nb * (blockIdx.y + ncw * blockIdx.z);
  const uint32_t per = (2 * nb * ncw) / kXcds;
  if (lin < per * kXcds) lin = (lin % kXcds) * per + lin / kXcds;
  const int colour = (int)(lin & 1u);
  const uint32_t comp = (lin >> 1) / nb;
  const uint32_t t = ((lin >> 1) - comp * nb) * TPB + threadIdx.x;
  if (t >= nthreads) return;
  const uint32_t nht = (uint32_t)nh / S;
  uint32_t row, jt, z, y;
  if (lg_nht >= 0) {
    row = t >> lg_nht;
    jt = t & (nht - 1);
  } else {
    row = t / nht;
    jt = t - row * nht;
  }
  if (lg_ny >= 0) {
    z = row >> lg_ny;
    y = row & ((uint32_t)ny - 1);
  } else {
    z = row / (uint32_t)ny;
    y = row - z * (uint32_t)ny;
  }
  const uint32_t nsite = (uint32_t)nh * ny * nz;
  const size_t base = (size_t)comp * nsite;
  const double* __restrict__ own = x64 + (size_t)colour * half + base;
  const char* __restrict__ ob = reinterpret_cast<const char*>(x64 + (size_t)(colour ^ 1) * half + base);
  const uint32_t plane = (uint32_t)nh * ny;
  const uint32_t ic = S * t;
  const uint32_t rb = ic - S * jt;
  const uint32_t xs = (y + z + (uint32_t)colour) & 1u;
  auto ld = [&](uint32_t e) {
    const double2 v = *reinterpret_cast<const double2*>(ob + e * 8u);
    return v;
  };
  const double2 c = ld(ic);
  const uint32_t ie = xs ? (jt + 1 == nht ? rb : ic + S) : (jt == 0 ? rb + (uint32_t)nh - 1 : ic - 1);
  const double ex = *reinterpret_cast<const double*>(ob + ie * 8u);
  const uint32_t in = ic + (y + 1 == (uint32_t)ny ? (uint32_t)nh - plane : (uint32_t)nh);
  const uint32_t is = ic + (y == 0 ? plane - (uint32_t)nh : 0u - (uint32_t)nh);
  const double2 n = ld(in), so = ld(is);
  const uint32_t zw = ZU ? __builtin_amdgcn_readfirstlane(z) : z;
  const bool top = zw + 1 >= (uint32_t)nz, bottom = zw == 0;
  const double2 u = ld(ic + (top ? 0u : plane)), d = ld(ic - (bottom ? 0u : plane));
  const double2 xo = *reinterpret_cast<const double2*>(own + ic);
  double2 bv = make_double2(0.0, 0.0);
  if (HAS_B) bv = *reinterpret_cast<const double2*>(b64 + (size_t)colour * half + base + ic);
  const int nw = (int)top + (int)bottom;
  // x-neighbour sums (x - 1) + (x + 1): xs == 1 -> (j, j+1), xs == 0 -> (j-1, j); the entry
  // beyond the owned ones closes the last pair on the side it lies
  const double sx0 = xs ? c.x + c.y : ex + c.x;
  const double sx1 = xs ? c.y + ex : c.x + c.y;
  auto res = [&](double sx, double nv, double sv, double uv, double dv, double xv, double b) {
    double s = (sx + sv) + nv;
    if (!top) s += uv;
    if (!bottom) s += dv;
    return b - ((6 + nw) * xv - s) * inv_h2;
  };
  float2 out;
  out.x = (float)res(sx0, n.x, so.x, u.x, d.x, xo.x, bv.x);
  out.y = (float)res(sx1, n.y, so.y, u.y, d.y, xo.y, bv.y);
  *reinterpret_cast<float2*>(r32 + (size_t)colour * half + base + ic) = out;
}

__global__ __launch_bounds__(TPB) void k_refine_update(double* __restrict__ x64,
                                                        const float* __restrict__ e32, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * TPB) x64[i] += (double)e32[i];
}

// x += e and then e = 0 on the two colour arrays of a component range in one launch (span s of
// n elements at offset s * stride), two elements per thread when n is even (16- and 8-byte
// accesses).
template <bool PAIR>
__global__ __launch_bounds__(TPB) void k_refine_out(double* __restrict__ x64,
                                                     float* __restrict__ e32, int64_t n,
                                                     int64_t stride) {
  const int64_t off = (int64_t)blockIdx.y * stride;
  double* __restrict__ X = x64 + off;
  float* __restrict__ E = e32 + off;
  const int64_t m = PAIR ? n / 2 : n;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < m; i += (int64_t)gridDim.x * TPB) {
    if (PAIR) {
      double2 x = reinterpret_cast<double2*>(X)[i];
      const float2 e = reinterpret_cast<float2*>(E)[i];
      x.x += (double)e.x;
      x.y += (double)e.y;
      reinterpret_cast<double2*>(X)[i] = x;
      reinterpret_cast<float2*>(E)[i] = make_float2(0.0f, 0.0f);
    } else {
      X[i] += (double)E[i];
      E[i] = 0.0f;
    }
  }
}

// x += P e into the split level-0 storage (grid.z = colour).
template <typename T>
__global__ __launch_bounds__(TPB) void k_prolong0(T* __restrict__ xr, T* __restrict__ xb,
                                                   const T* __restrict__ e, int nxf, int nyf,
                                                   int nzf, uint32_t nsite, uint32_t Nc,
                                                   int cfirst) {
  const uint32_t comp = blockIdx.y;
  const int colour = cfirst + blockIdx.z;
  const uint32_t p = blockIdx.x * TPB + threadIdx.x;
  if (p >= nsite) return;
  const int nh = nxf >> 1;
  const uint32_t row = p / nh;
  const int j = p - row * nh;
  const int yf = row % nyf;
  const int zf = row / nyf;
  const int xf = 2 * j + ((yf + zf + colour) & 1);
  T* X = (colour ? xb : xr) + (size_t)comp * nsite;
  const int nxc = nxf >> 1, nyc = nyf >> 1;
  X[p] += prolong_at<T>(e + (size_t)comp * Nc, nxc, nxc * nyc, xf, yf, zf, nxc, nyc, nzf >> 1);
}

// The same for nx/2 even, two sites per thread: sites j0 = 2jp and j0 + 1 of a colour row sit
// two cells apart, so their trilinear windows share the coarse row pairs and two of three
// coarse columns: per coarse row one 16-byte load of columns (j0, j0+1) and one load of the
// column beyond on the side of the sites' x offset (8 loads of e for both sites), and x moves
// with one 16-byte load and store.  Row and plane come by shifts when the row counts are powers
// of two.
template <typename T>
__global__ __launch_bounds__(TPB) void k_prolong0_pair(T* __restrict__ xr, T* __restrict__ xb,
                                                        const T* __restrict__ e, int nxf, int nyf,
                                                        int nzf, uint32_t npairs, uint32_t Nc,
                                                        int cfirst, int lg_nhp, int lg_ny) {
  using V2 = typename Vec2<T>::type;
  const uint32_t comp = blockIdx.y;
  const int colour = cfirst + blockIdx.z;
  const uint32_t t = blockIdx.x * TPB + threadIdx.x;
  if (t >= npairs) return;
  const int nh = nxf >> 1;
  const uint32_t nhp = (uint32_t)nh >> 1;
  uint32_t row, jp, zf, yf;
  if (lg_nhp >= 0) {
    row = t >> lg_nhp;
    jp = t & (nhp - 1);
  } else {
    row = t / nhp;
    jp = t - row * nhp;
  }
  if (lg_ny >= 0) {
    zf = row >> lg_ny;
    yf = row & ((uint32_t)nyf - 1);
  } else {
    zf = row / (uint32_t)nyf;
    yf = row - zf * (uint32_t)nyf;
  }
  const int sx = (int)((yf + zf + (uint32_t)colour) & 1u);  // x = 2j + sx
  const int j0 = 2 * (int)jp;
  const int nxc = nh, nyc = nyf >> 1, nzc = nzf >> 1;
  // the coarse column beyond the pair on the side of sx
  const int Xo = sx ? (j0 + 2 == nxc ? 0 : j0 + 2) : (j0 == 0 ? nxc - 1 : j0 - 1);
  const int Y0 = (int)(yf >> 1);
  const int Y1 = (yf & 1) ? (Y0 + 1 == nyc ? 0 : Y0 + 1) : (Y0 == 0 ? nyc - 1 : Y0 - 1);
  const int Z0 = (int)(zf >> 1);
  int Z1 = (zf & 1) ? Z0 + 1 : Z0 - 1;
  T wz0 = T(0.75), wz1 = T(0.25);
  if (Z1 < 0 || Z1 >= nzc) {
    wz0 = T(0.5);
    wz1 = T(0);
    Z1 = Z0;
  }
  const T* E = e + (size_t)comp * Nc;
  const T* r00 = E + ((size_t)Z0 * nyc + Y0) * nxc;
  const T* r01 = E + ((size_t)Z0 * nyc + Y1) * nxc;
  const T* r10 = E + ((size_t)Z1 * nyc + Y0) * nxc;
  const T* r11 = E + ((size_t)Z1 * nyc + Y1) * nxc;
  T* X = (colour ? xb : xr) + (size_t)comp * (npairs * 2);
  V2 xv = *reinterpret_cast<const V2*>(X + 2 * t);
  const V2 v00 = *reinterpret_cast<const V2*>(r00 + j0), v01 = *reinterpret_cast<const V2*>(r01 + j0);
  const V2 v10 = *reinterpret_cast<const V2*>(r10 + j0), v11 = *reinterpret_cast<const V2*>(r11 + j0);
  const T u00 = r00[Xo], u01 = r01[Xo], u10 = r10[Xo], u11 = r11[Xo];
  // site a: own column j0, other (sx ? j0+1 : the outer one); site b: own j0+1, other
  // (sx ? the outer one : j0)
  const T q = T(0.75), o = T(0.25);
  auto w = [&](const V2& v, T u, T& a, T& b) {
    a = q * v.x + o * (sx ? v.y : u);
    b = q * v.y + o * (sx ? u : v.x);
  };
  T a00, b00, a01, b01, a10, b10, a11, b11;
  w(v00, u00, a00, b00);
  w(v01, u01, a01, b01);
  w(v10, u10, a10, b10);
  w(v11, u11, a11, b11);
  const T pa0 = q * a00 + o * a01, pa1 = q * a10 + o * a11;
  const T pb0 = q * b00 + o * b01, pb1 = q * b10 + o * b11;
  xv.x += wz0 * pa0 + wz1 * pa1;
  xv.y += wz0 * pb0 + wz1 * pb1;
  *reinterpret_cast<V2*>(X + 2 * t) = xv;
}

__global__ __launch_bounds__(TPB) void k_to_split(double* __restrict__ xr,
                                                   double* __restrict__ xb,
                                                   const double* __restrict__ nat, int nx,
                                                   int ny, uint32_t N) {
  const uint32_t comp = blockIdx.y;
  const uint32_t i = blockIdx.x * TPB + threadIdx.x;
  if (i >= N) return;
  const int x = i % nx;
  const uint32_t row = i / nx;
  const int y = row % ny;
  const int z = row / ny;
  double* a = ((x + y + z) & 1) ? xb : xr;
  a[(size_t)comp * (N >> 1) + row * (nx >> 1) + (x >> 1)] = nat[(size_t)comp * N + i];
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_from_split(T* __restrict__ nat,
                                                     const double* __restrict__ xr,
                                                     const double* __restrict__ xb, int nx,
                                                     int ny, uint32_t N) {
  const uint32_t comp = blockIdx.y;
  const uint32_t i = blockIdx.x * TPB + threadIdx.x;
  if (i >= N) return;
  const int x = i % nx;
  const uint32_t row = i / nx;
  const int y = row % ny;
  const int z = row / ny;
  const double* a = ((x + y + z) & 1) ? xb : xr;
  nat[(size_t)comp * N + i] = (T)a[(size_t)comp * (N >> 1) + row * (nx >> 1) + (x >> 1)];
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + TPB - 1) / TPB); }

int ilog2_exact(uint32_t v) {
  if (v == 0 || (v & (v - 1))) return -1;
  int s = 0;
  while ((1u << s) != v) ++s;
  return s;
}

}  // namespace

template <typename T>
hipError_t launch_rb_pass(T* xc, const T* xo, const T* bc, int nx, int ny, int nz, int ncomp,
                          int colour, double h, double kT, bool noise, const NoiseArgs& na,
                          hipStream_t s) {
  const int nh = nx / 2;
  const uint32_t nsite = (uint32_t)nh * ny * nz;
  Diag3<T> dg;
  for (int w = 0; w < 3; ++w) {
    dg.inv_d[w] = (T)(h * h / (6.0 + w));
    dg.sig[w] = (T)sqrt(kT * h * h / (6.0 + w));
    dg.inv_n[w] = (T)(1.0 / (6.0 + w));
  }
  const T ih2 = (T)(1.0 / (h * h));
  constexpr int S = 16 / (int)sizeof(T);
  if (nh % S == 0 && (uint64_t)nsite * sizeof(T) < (1ull << 32)) {
    const uint32_t nthreads = nsite / S;
    const int lg_nht = ilog2_exact((uint32_t)(nh / S)), lg_ny = ilog2_exact((uint32_t)ny);
    dim3 grid(blocks_for(nthreads), ncomp);
    const bool zu = ((uint64_t)(nh / S) * ny) % 64 == 0;
#define SMG_RBV(HB, NZ, ZU)                                                                  \
  k_rb_pass_vec<T, HB, NZ, ZU><<<grid, TPB, 0, s>>>(xc, xo, bc, nh, ny, nz, nthreads, lg_nht, \
                                                    lg_ny, colour, ih2, dg, na)
    if (zu) {
      if (bc) { if (noise) SMG_RBV(true, true, true); else SMG_RBV(true, false, true); }
      else { if (noise) SMG_RBV(false, true, true); else SMG_RBV(false, false, true); }
    } else {
      if (bc) { if (noise) SMG_RBV(true, true, false); else SMG_RBV(true, false, false); }
      else { if (noise) SMG_RBV(false, true, false); else SMG_RBV(false, false, false); }
    }
#undef SMG_RBV
  } else {
    dim3 grid(blocks_for((nsite + 1) / 2), ncomp);
#define SMG_RB(HB, NZ) \
  k_rb_pass<T, HB, NZ><<<grid, TPB, 0, s>>>(xc, xo, bc, nh, ny, nz, nsite, colour, ih2, dg, na)
    if (bc) { if (noise) SMG_RB(true, true); else SMG_RB(true, false); }
    else { if (noise) SMG_RB(false, true); else SMG_RB(false, false); }
#undef SMG_RB
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rb_pass_multi(const RbPassItem<T>* items, int n, int colour, bool has_b,
                               bool noise, hipStream_t s) {
  constexpr int S = 16 / (int)sizeof(T);
  RbMultiArgs<T> m{};
  m.colour = colour;
  m.bm = box_muller_coef();
  uint32_t total = 0;
  auto flush = [&]() -> hipError_t {
    if (m.nitems == 0) return hipSuccess;
    m.begin[m.nitems] = total;
#define SMG_RBM(HB, NZ) k_rb_pass_vec_multi<T, HB, NZ><<<total, TPB, 0, s>>>(m)
    if (has_b) { if (noise) SMG_RBM(true, true); else SMG_RBM(true, false); }
    else { if (noise) SMG_RBM(false, true); else SMG_RBM(false, false); }
#undef SMG_RBM
    m.nitems = 0;
    total = 0;
    return hipGetLastError();
  };
  for (int q = 0; q < n; ++q) {
    const RbPassItem<T>& p = items[q];
    const int nh = p.nx / 2;
    const uint32_t nsite = (uint32_t)nh * p.ny * p.nz;
    if ((p.bc != nullptr) != has_b) return hipErrorInvalidValue;
    if (nh % S != 0 || (uint64_t)nsite * sizeof(T) >= (1ull << 32)) {
      // shapes the vector pass does not take: a launch of their own
      hipError_t e = launch_rb_pass<T>(p.xc, p.xo, p.bc, p.nx, p.ny, p.nz, p.ncomp, colour, p.h,
                                       p.kT, noise, p.na, s);
      if (e != hipSuccess) return e;
      continue;
    }
    if (p.ncomp == 0) continue;
    if (m.nitems == kRbMultiItems) {
      hipError_t e = flush();
      if (e != hipSuccess) return e;
    }
    RbMultiItem<T>& it = m.it[m.nitems];
    it.xc = p.xc;
    it.xo = p.xo;
    it.bc = p.bc;
    it.nh = nh;
    it.ny = p.ny;
    it.nz = p.nz;
    it.nthreads = nsite / S;
    it.lg_nht = ilog2_exact((uint32_t)(nh / S));
    it.lg_ny = ilog2_exact((uint32_t)p.ny);
    it.nblk = blocks_for(it.nthreads);
    it.inv_h2 = (T)(1.0 / (p.h * p.h));
    for (int w = 0; w < 3; ++w) {
      it.dg.inv_d[w] = (T)(p.h * p.h / (6.0 + w));
      it.dg.sig[w] = (T)sqrt(p.kT * p.h * p.h / (6.0 + w));
      it.dg.inv_n[w] = (T)(1.0 / (6.0 + w));
    }
    it.nk.k0 = p.na.k0;
    it.nk.k1 = p.na.k1;
    it.nk.sid = p.na.sid;
    it.nk.c2 = p.na.c2;
    it.nk.c3 = p.na.c3;
    it.nk.cpc = p.na.comps_per_chain;
    it.nk.cpc_magic = p.na.cpc_magic;
    it.nk.sqkT = p.na.sqkT;
    it.nk.chains = p.na.chains;
    it.nk.comp0 = p.na.comp0;
    m.begin[m.nitems] = total;
    total += it.nblk * (uint32_t)p.ncomp;
    ++m.nitems;
  }
  return flush();
}

template <typename T>
hipError_t launch_residual0(T* r, const T* xr, const T* xb, const T* br, const T* bb, int nx,
                            int ny, int nz, int ncomp, double h, hipStream_t s) {
  const uint32_t N = (uint32_t)nx * ny * nz;
  dim3 grid(blocks_for(N), ncomp);
  const T ih2 = (T)(1.0 / (h * h));
  if (br) k_residual0<T, true><<<grid, TPB, 0, s>>>(r, xr, xb, br, bb, nx, ny, nz, N, ih2);
  else k_residual0<T, false><<<grid, TPB, 0, s>>>(r, xr, xb, br, bb, nx, ny, nz, N, ih2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict_residual0(T* bc, T* xc, const T* xr, const T* xb, const T* br,
                                     const T* bb, int nx, int ny, int nz, int ncomp, double h,
                                     hipStream_t s) {
  const int nxc = nx >> 1, nyc = ny >> 1, nzc = nz >> 1;
  if (nxc * nyc * nzc == 0) return hipSuccess;
  const T ih2 = (T)(1.0 / (h * h));
  auto go = [&](auto rx, auto ry) {
    constexpr int RX = decltype(rx)::value, RY = decltype(ry)::value;
    const int ntx = (nxc + RX - 1) / RX, nty = (nyc + RY - 1) / RY;
    dim3 grid(ntx * nty, (nzc + RR_Z - 1) / RR_Z, ncomp);
    if (br)
      k_restrict_residual0<T, true, RX, RY>
          <<<grid, TPB, 0, s>>>(bc, xc, xr, xb, br, bb, nx, ny, nz, ntx, ih2);
    else
      k_restrict_residual0<T, false, RX, RY>
          <<<grid, TPB, 0, s>>>(bc, xc, xr, xb, br, bb, nx, ny, nz, ntx, ih2);
  };
  // 16 x 8 coarse cells per work-group where the grid is that wide (less halo and scalar work
  // per cell: 190 us against 229 us for 8 x 8 at 128^3 x 24; 16 x 16 took 219 us at half the
  // occupancy), else 8 x 8
  if (nxc >= 16)
    go(std::integral_constant<int, 16>(), std::integral_constant<int, 8>());
  else
    go(std::integral_constant<int, 8>(), std::integral_constant<int, 8>());
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong0(T* xr, T* xb, const T* e, int nxf, int nyf, int nzf, int ncomp,
                           int colours, hipStream_t s) {
  const uint32_t nsite = (uint32_t)(nxf / 2) * nyf * nzf;
  const uint32_t Nc = (uint32_t)(nxf / 2) * (nyf / 2) * (nzf / 2);
  colours &= 3;
  if (colours == 0) return hipSuccess;
  if ((nxf / 2) % 2 == 0 && ((uintptr_t)e & 15) == 0) {
    dim3 grid(blocks_for(nsite / 2), ncomp, colours == 3 ? 2 : 1);
    k_prolong0_pair<T><<<grid, TPB, 0, s>>>(xr, xb, e, nxf, nyf, nzf, nsite / 2, Nc,
                                            colours == 2 ? 1 : 0, ilog2_exact((uint32_t)nxf / 4),
                                            ilog2_exact((uint32_t)nyf));
    return hipGetLastError();
  }
  dim3 grid(blocks_for(nsite), ncomp, colours == 3 ? 2 : 1);
  k_prolong0<T><<<grid, TPB, 0, s>>>(xr, xb, e, nxf, nyf, nzf, nsite, Nc, colours == 2 ? 1 : 0);
  return hipGetLastError();
}

template hipError_t launch_rb_pass<double>(double*, const double*, const double*, int, int, int,
                                           int, int, double, double, bool, const NoiseArgs&,
                                           hipStream_t);
template hipError_t launch_rb_pass<float>(float*, const float*, const float*, int, int, int, int,
                                          int, double, double, bool, const NoiseArgs&,
                                          hipStream_t);
template hipError_t launch_rb_pass_multi<double>(const RbPassItem<double>*, int, int, bool, bool,
                                                 hipStream_t);
template hipError_t launch_rb_pass_multi<float>(const RbPassItem<float>*, int, int, bool, bool,
                                                hipStream_t);
template hipError_t launch_residual0<double>(double*, const double*, const double*, const double*,
                                             const double*, int, int, int, int, double,
                                             hipStream_t);
template hipError_t launch_residual0<float>(float*, const float*, const float*, const float*,
                                            const float*, int, int, int, int, double, hipStream_t);
template hipError_t launch_prolong0<double>(double*, double*, const double*, int, int, int, int,
                                            int, hipStream_t);
template hipError_t launch_restrict_residual0<double>(double*, double*, const double*,
                                                      const double*, const double*,
                                                      const double*, int, int, int, int, double,
                                                      hipStream_t);
template hipError_t launch_restrict_residual0<float>(float*, float*, const float*, const float*,
                                                     const float*, const float*, int, int, int,
                                                     int, double, hipStream_t);
template hipError_t launch_prolong0<float>(float*, float*, const float*, int, int, int, int,
                                            int, hipStream_t);

hipError_t launch_refine_residual(float* r32, const double* x64, const double* b64, int nx,
                                  int ny, int nz, int ncomp, int ncomp_stride, double h,
                                  double* part, double* norm, hipStream_t s) {
  const uint32_t nsite = (uint32_t)(nx / 2) * ny * nz;
  const uint32_t nblk = blocks_for(nsite);
  dim3 grid(nblk, ncomp, 2);
  const double ih2 = 1.0 / (h * h);
  const int nh = nx / 2;
  const size_t half = (size_t)ncomp_stride * nsite;
  if (!norm && nh % 2 == 0 && (uint64_t)nsite * sizeof(double) < (1ull << 32)) {
    // no norms: two sites per thread
    const uint32_t nthreads = nsite / 2;
    const int lg_nht = ilog2_exact((uint32_t)(nh / 2)), lg_ny = ilog2_exact((uint32_t)ny);
    const bool zu = ((uint64_t)(nh / 2) * ny) % 64 == 0;
    dim3 gv(blocks_for(nthreads), ncomp, 2);
#define SMG_RRV(HB, ZU)                                                                     \
  k_refine_residual_vec<HB, ZU><<<gv, TPB, 0, s>>>(r32, x64, b64, nh, ny, nz, nthreads, lg_nht, \
                                                   lg_ny, ih2, half)
    if (zu) { if (b64) SMG_RRV(true, true); else SMG_RRV(false, true); }
    else { if (b64) SMG_RRV(true, false); else SMG_RRV(false, false); }
#undef SMG_RRV
    return hipGetLastError();
  }
#define SMG_RR(HB, NM) \
  k_refine_residual<HB, NM><<<grid, TPB, 0, s>>>(r32, x64, b64, nx, ny, nz, nsite, ih2, part, nblk, \
                                                 (size_t)ncomp_stride * nsite)
  if (b64) { if (norm) SMG_RR(true, true); else SMG_RR(true, false); }
  else { if (norm) SMG_RR(false, true); else SMG_RR(false, false); }
#undef SMG_RR
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !norm) return e;
  // second stage of the fixed-order sum over the 2*nblk partials of each component
  return launch_sumsq_final_parts(norm, part, 2 * nblk, ncomp, s);
}

hipError_t launch_refine_out(double* x64, float* e32, int64_t n, int64_t stride,
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const bool pair = n % 2 == 0 && stride % 2 == 0 && ((uintptr_t)x64 & 15) == 0 &&
                    ((uintptr_t)e32 & 7) == 0;
  const int64_t m = pair ? n / 2 : n;
  const int64_t b = (m + TPB - 1) / TPB;
  dim3 grid((unsigned)(b < 32768 ? b : 32768), 2);
  if (pair) k_refine_out<true><<<grid, TPB, 0, s>>>(x64, e32, n, stride);
  else k_refine_out<false><<<grid, TPB, 0, s>>>(x64, e32, n, stride);
  return hipGetLastError();
}

hipError_t launch_refine_update(double* x64, const float* e32, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t b = (n + TPB - 1) / TPB;
  k_refine_update<<<(unsigned)(b < 65536 ? b : 65536), TPB, 0, s>>>(x64, e32, n);
  return hipGetLastError();
}

hipError_t launch_to_split(double* xr, double* xb, const double* nat, int nx, int ny, int nz,
                           int ncomp, hipStream_t s) {
  const uint32_t N = (uint32_t)nx * ny * nz;
  dim3 grid(blocks_for(N), ncomp);
  k_to_split<<<grid, TPB, 0, s>>>(xr, xb, nat, nx, ny, N);
  return hipGetLastError();
}

hipError_t launch_from_split(void* nat, int out_f32, const double* xr, const double* xb, int nx,
                             int ny, int nz, int ncomp, hipStream_t s) {
  const uint32_t N = (uint32_t)nx * ny * nz;
  dim3 grid(blocks_for(N), ncomp);
  if (out_f32) k_from_split<float><<<grid, TPB, 0, s>>>((float*)nat, xr, xb, nx, ny, N);
  else k_from_split<double><<<grid, TPB, 0, s>>>((double*)nat, xr, xb, nx, ny, N);
  return hipGetLastError();
}

}  // namespace smg
