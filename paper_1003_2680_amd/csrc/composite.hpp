// Spatially adaptive composite grid (one box refined by two) and its FAC cycle: device-side
// descriptors and kernel launchers.
//
// Mesh and operator (Sec. "Spatially Adaptive Discretizations"): base cells of width h outside
// the box, fine cells of width h/2 inside it; L = D G with the same-level face gradient
// (eq. def_discr_grad0), the coarse-fine face gradient (eq. def_discr_grad, read in 3D as the
// mean of the four fine cells on the coarse face minus the coarse value over 3/4 h) and the
// conservative coarse face value (eq. def_discr_grad_last); walls by the antisymmetric ghost.
// The sampling precision is A = -S/h^3 with S = diag(volume) L symmetric, so in units of 1/h^2:
//   coarse row: +1 per coarse neighbour face (-1 off-diagonal), +2 per wall face, +4/3 per
//               coarse-fine face (-1/3 to each of its four fine cells);
//   fine row:   +1/2 per fine neighbour face (-1/2), +1 per wall face, and per coarse-fine
//               face +1/12 on the diagonal, +1/12 to each of the three other fine cells of that
//               face, -1/3 to the coarse cell.
// Storage: the coarse field uses the whole base grid [nz][ny][nx] (entries of covered cells are
// never read and are written as zero by the residual); the fine field is the box [fz][fy][fx].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"

namespace smg {

struct CompGeom {
  int nx, ny, nz;              // base grid
  int x0, x1, y0, y1, z0, z1;  // refined box in base cells (0 <= x0 < x1 <= nx, x1-x0 < nx, ...)
  int fx, fy, fz;              // fine extents 2(x1-x0), 2(y1-y0), 2(z1-z0)
  double ih2;                  // 1/h^2
};

// Operator of a Galerkin base level as a dictionary of sparse stencils: every 2x2x2 block has a
// block type, a block type names the stencil of each of its 8 cells (in-block index
// dx + 2dy + 4dz) and carries the factors of its 8x8 diagonal block; a stencil is a list of
// (coefficient, offset) records, offset code = (dz+2)*25 + (dy+2)*5 + (dx+2), offsets periodic in
// x, y.  T: double (FP64 sweeps) or float (the inner cycle of the FP32-refined form).
template <typename T>
struct alignas(sizeof(T) == 8 ? 16 : 4) StEntryT {
  T a;           // coefficient
  int32_t lin;   // dx + nx (dy + ny dz): the target's index minus the cell's, away from the seams
  int32_t meta;  // offset code in bits 0-7; bit 8 + k: the target lies in the 2x2x2 block of a
                 // cell with in-block index k (periodic wrap included)
};
using StEntry = StEntryT<double>;
// records past the end of a level's table, so that the launches may load whole groups of eight
// (times the lanes per row) without a bounds test
constexpr int kEntryPad = 64;
template <typename T>
struct GStencilT {
  const int32_t* btype;   // [n/8]
  const int32_t* bt_sid;  // [types][8]
  const T* bt_fac;        // [types][128]: A_BB^-1 then L_BB^-T, row-major
  const int32_t* st_off;  // [stencils + 1]
  const StEntryT<T>* ent; // entries of every stencil
  // block types whose 8 rows are plain 7-point (the centre and every in-grid face neighbour,
  // one common off-diagonal coefficient): that coefficient, else 0; and the 8 diagonals
  const T* bt_c7;         // [types]
  const T* bt_diag;       // [types][8]
  int nx, ny, nz;
  int split;              // 8: long rows (every block by the long-row launch), else 1
  int row_lanes;          // lanes per long row: 2 or 8, 0 = by the launch's row count
  // split == 1 levels: the blocks whose type is not plain 7-point, by block colour
  // (list[list_off[c] .. list_off[c+1])), run by a second, long-row launch
  const int32_t* list;
  int list_off[9];
};

// Point heat bath of one class of the composite sweep (x_i = (b_i - sum_j A_ij x_j)/A_ii +
// sqrt(kT/A_ii) n_i), b null = 0.  Classes: coarse cells of parity `colour`; fine cells off the
// interface layer of parity `colour`; the listed layer cells (one parity class per list).
template <typename T>
hipError_t launch_comp_coarse_pass(T* xc, const T* bc, const T* xf, const CompGeom& g, int colour,
                                   bool noise, const NoiseArgs& na, hipStream_t s);
template <typename T>
hipError_t launch_comp_fine_pass(T* xf, const T* bf, const CompGeom& g, int colour, bool noise,
                                 const NoiseArgs& na, hipStream_t s);
template <typename T>
hipError_t launch_comp_layer_pass(T* xf, const T* bf, const T* xc, const CompGeom& g,
                                  const int32_t* cells, int count, bool noise, const NoiseArgs& na,
                                  hipStream_t s);
// rc = bc - (A x)_coarse on every base cell (covered cells: 0), rf = bf - (A x)_fine
template <typename T>
hipError_t launch_comp_residual(T* rc, T* rf, const T* xc, const T* xf, const T* bc, const T* bf,
                                const CompGeom& g, hipStream_t s);
// b0 = P^T (rc, rf) over the base grid and x0 = 0 (P: identity on coarse cells, trilinear
// onto fine cells)
template <typename T>
hipError_t launch_comp_restrict(T* b0, T* x0, const T* rc, const T* rf, const CompGeom& g,
                                hipStream_t s);
// the two above fused for the cycle: rf = bf - (A x)_fine, then b0 = P^T (b - A x) with the
// coarse residual formed inside the restriction (never stored), x0 = 0
template <typename T>
hipError_t launch_comp_residual_restrict(T* b0, T* x0, T* rf, const T* xc, const T* xf,
                                         const T* bc, const T* bf, const CompGeom& g,
                                         hipStream_t s);
// (xc, xf) += P y
template <typename T>
hipError_t launch_comp_prolong(T* xc, T* xf, const T* y, const CompGeom& g, hipStream_t s);
// 2x2x2 block heat bath of one block colour on a Galerkin base level (b null = 0)
template <typename T>
hipError_t launch_gblock_pass(T* x, const T* b, const GStencilT<T>& st, int colour, bool noise,
                              const NoiseArgs& na, hipStream_t s);
// coarsest base level (FP64 arithmetic, T storage): x = A_c^-1 b (+ sqrt(kT) L_c^-T z), z (n
// doubles of scratch) filled with the level's FP64 normals; wt = L_c^-T row-major
template <typename T>
hipError_t launch_dense_draw(T* x, const T* b, const double* ainv, const double* wt, double* z,
                             int n, bool noise, const NoiseArgs& na, hipStream_t s);
// r = b - A x on a Galerkin base level
template <typename T>
hipError_t launch_gresidual(T* r, const T* x, const T* b, const GStencilT<T>& st, hipStream_t s);
// right-hand side of the forced field (Appendix A): (bc, bf) = -(volume/h^3) q eta, covered
// base cells 0, eta from the streams nac (coarse part) and naf (fine part), q null = 1
hipError_t launch_comp_forcing(double* bc, double* bf, const double* qc, const double* qf,
                               const CompGeom& g, const NoiseArgs& nac, const NoiseArgs& naf,
                               hipStream_t s);

}  // namespace smg
