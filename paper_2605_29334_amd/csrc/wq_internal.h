// Internal definitions shared by the libwq translation units (gfx950, HIP).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/wq.h"

namespace wq {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);

#define WQ_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      ::wq::set_error(std::string(#call) + ": " + hipGetErrorString(e_));         \
      return WQ_EDEVICE;                                                          \
    }                                                                             \
  } while (0)

#define WQ_CHECK(cond, code, msg)                                                 \
  do {                                                                            \
    if (!(cond)) {                                                                \
      ::wq::set_error(msg);                                                       \
      return code;                                                                \
    }                                                                             \
  } while (0)

#define WQ_TRY(expr)                                                              \
  do {                                                                            \
    wq_status s_ = (expr);                                                        \
    if (s_ != WQ_OK) return s_;                                                   \
  } while (0)

// ------------------------------------------------------------------ device buffers
// A device allocation owned by a handle; freed by release().
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;  // requested size
  size_t cap = 0;    // size of the block (its size class)
  int dev = 0;       // device the block lives on
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Device buffers come from a per-device cache of freed blocks (size classes of 512 bytes
// below 1 MiB, one eighth of a power of two above). Freeing keeps hipFree's guarantee: the
// device is synchronised before the block can be handed out again, so no queued work on
// any stream still uses it; dfree_many does so once for a whole set of buffers. What the
// cache holds beyond 8 GiB per device goes back to the runtime, and a failed allocation
// returns the cache's blocks to the runtime before it tries again.
wq_status dalloc(DBuf& b, size_t bytes);
void dfree(DBuf& b);
void dfree_many(DBuf* const* bufs, size_t n);

template <class T> inline wq_status dalloc_n(DBuf& b, size_t n) { return dalloc(b, n * sizeof(T)); }

// element type codes (WQ_ARR_ETYPE)
enum : uint8_t { ET_PASSIVE = 0, ET_REGULAR = 1, ET_BOUNDARY = 2, ET_IRREGULAR = 3, ET_TRANSITION = 4 };

constexpr int TILE_ROWS = 8;
constexpr int T2_ROWS = 16;    // rows per cell-major assembly tile (MFMA 16 x 16 x 4 columns)
constexpr int T2_NZCAP = 416;  // CSR entries per cell-major tile (8 rows of 52; 16 short rows)
constexpr int T2_STEPCAP = 128;  // default: summed row steps (support cells' blocks of 4 points) per tile

}  // namespace wq

struct wq_mesh {
  int device = 0;
  int32_t nv = 0, nf = 0, n_fn = 0;
  int32_t dim = 2;  // coordinates per control point: 2 (planar) or 3 (surface)
  int64_t n_ext = 0, n_coef = 0;
  wq::DBuf face_vtx, split, ext_ptr, ext_fn, coef_ptr, coef, ctrl;
  // host copies needed by the (rare) min-max fallback of Eq. (18)
  std::vector<int64_t> h_ext_ptr;
};

struct wq_points {
  wq_mesh* mesh = nullptr;
  int32_t ncell = 0;
  int64_t n_rows = 0, nnz = 0, n_points = 0, n_pairs = 0, n_slots = 0, n_cfn = 0, n_basis = 0;
  int32_t max_row = 0;     // max n_i
  int32_t max_r = 0;       // max r_i
  int32_t max_cell_m = 0;  // max functions on a cell
  int32_t max_cell_np = 0; // max points on a cell
  int has_lap = 0;
  // per face
  wq::DBuf etype, s;
  // per cell
  wq::DBuf cell_face, cell_sub, cell_pt_off /*int64 [ncell+1]*/, cfn_ptr /*int64 [ncell+1]*/,
      cfn /*int32*/, cfn_loc /*uint8*/, dptr /*int64 [ncell+1]*/;
  // per function (row)
  wq::DBuf supp_ptr /*int64 [n+1]*/, supp_cell /*int32*/, row_ptr /*int64*/, col /*int32*/,
      qptr /*int64*/, qidx /*int32*/;
  // per (row, cell) pair = supp entry
  wq::DBuf soff /*int64 [pairs+1]*/, slot /*uint8*/, kself /*uint8*/;
  // assembly tiles: TILE_ROWS consecutive rows; one entry per (tile, cell), cells ascending
  int64_t n_tiles = 0, n_entries = 0;
  int32_t max_tile_nnz = 0, max_tile_ent = 0, max_tile_mem = 0;
  int32_t max_tile_nd = 0 /*max np*m of an entry*/, max_tile_nw = 0 /*max members*np*/;
  int32_t asm_chunk = 64;  // consecutive tiles per XCD turn in the assembly launch (tunable)
  int32_t t2_stepcap = wq::T2_STEPCAP;  // summed row steps per cell-major tile (tunable)
  int64_t t2_gen = 0;  // counts (re)builds of the cell-major tiles and schedule changes
  wq::DBuf tile_eptr /*int64 [tiles+1]*/, tile_ent /*int4 [entries]: dptr, pt0, mask|np<<16|m<<24, mbase*/,
      tile_mem /*int2 [pairs]: qoff | rowloc<<28, soff*/;
  // cell-major assembly tiles: runs of up to T2_ROWS consecutive rows with at most T2_NZCAP CSR
  // entries; one entry per (tile, cell in the support of some row of the tile), cells
  // ascending: int4 (basis block offset, first point, member mask | np << 16 | m << 24, byte
  // offset of the entry's slot maps in t2_slot: one per member row, rows ascending, each the
  // (row, cell) pair's map padded to a multiple of 4 bytes)
  int64_t n_t2 = 0, n_e2 = 0;
  int32_t t2_maxnz = 0, t2_maxent = 0;  // largest CSR entries, largest cell entries of a tile
  wq::DBuf t2_row0 /*int32 [n_t2+1]*/, t2_eptr /*int64 [n_t2+1]*/, t2_ent /*int4*/, t2_slot /*uint8*/;
  // per point
  wq::DBuf x /*double [2 np]*/, detJ /*double [np]*/;
  // per (cell, point, cell function); DZ only on a surface (third gradient component),
  // where DL holds the Laplace-Beltrami operator
  wq::DBuf DN, DX, DY, DZ, DL;
  // scratch owned by the handle, allocated on first use: tangent point fields
  // (4 x n_points doubles) and the Newton / PCG vectors of wq_heat_step
  wq::DBuf tangent_ws, newton_ws;
  // scratch for the third gradient term of a surface stiffness (nnz doubles, first use)
  wq::DBuf zterm_ws;
  // basis data split for the low-precision contraction (built on first use):
  // FP16 x 2: uint32 per value (hi | lo << 16) of D * 2^-ds_exp[f];
  // BF16 x 3: uint2 per value (hi | mid << 16, lo)
  wq::DBuf DS[4];
  int ds_prec = 0;
  int ds_exp[4] = {0, 0, 0, 0};
};

struct wq_weights {
  wq_points* pts = nullptr;
  unsigned fam_mask = 0;
  wq::DBuf W[5];    // weights per family (mass, dx, dy, lap, dz), aligned with qidx
  wq::DBuf rhs[5];  // Gauss right-hand sides per family, aligned with col
};

// ------------------------------------------------------------------ device helpers
namespace wq {

__host__ __device__ inline int fam_index(unsigned fam) {
  return fam == WQ_FAM_MASS ? 0 : fam == WQ_FAM_DX ? 1 : fam == WQ_FAM_DY ? 2 : fam == WQ_FAM_LAP ? 3 : 4;
}

// cubic Bernstein values and derivatives
__device__ inline void bern3(double t, double b[4], double d[4], double s[4]) {
  const double u = 1.0 - t;
  b[0] = u * u * u;
  b[1] = 3.0 * t * u * u;
  b[2] = 3.0 * t * t * u;
  b[3] = t * t * t;
  d[0] = -3.0 * u * u;
  d[1] = 3.0 * u * u - 6.0 * t * u;
  d[2] = 6.0 * t * u - 3.0 * t * t;
  d[3] = 3.0 * t * t;
  s[0] = 6.0 * u;
  s[1] = -12.0 * u + 6.0 * t;
  s[2] = 6.0 * u - 12.0 * t;
  s[3] = 6.0 * t;
}

// exclusive scan of n int64 values in place on the device. *total receives the result at
// index n-1, i.e. the sum of the first n-1 inputs (callers scan count+1 entries).
wq_status exclusive_scan_i64(int64_t* d, int64_t n, int64_t* total, hipStream_t st);

// whether kernel timing records are being taken (wq_timing_enable)
bool timing_enabled();
// side streams for independent launches of one call (wq_set_side_streams; 1: none)
int side_streams();

// kernel timing (wq_timing_enable): records events around a launch when enabled
struct KTimer {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t st = nullptr;
  const char* name = nullptr;
  int64_t work = 0;
  KTimer(const char* n, int64_t w, hipStream_t s);
  void stop();
};


// 64-bit index launch helper
inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Geometry of a 2-manifold in 3-D at one point (Section 4.1, Eqs. (13)-(17) on a surface):
// from the tangent vectors a_1, a_2 (columns of A) and the second derivatives x_11, x_12,
// x_22 (columns of X2), the area element sqrt(det g), the inverse metric and the
// Christoffel coefficients Gamma^c_ab = g^{cd} a_d . x_ab.
struct SurfGeom {
  double A[3][2];
  double gi00, gi01, gi11;
  double sg;
  double gam[2][3];  // [c][ab], ab = 11, 12, 22
};
__device__ inline SurfGeom surf_geom(const double A[3][2], const double X2[3][3]) {
  SurfGeom G;
  for (int a = 0; a < 3; ++a) {
    G.A[a][0] = A[a][0];
    G.A[a][1] = A[a][1];
  }
  const double g00 = A[0][0] * A[0][0] + A[1][0] * A[1][0] + A[2][0] * A[2][0];
  const double g01 = A[0][0] * A[0][1] + A[1][0] * A[1][1] + A[2][0] * A[2][1];
  const double g11 = A[0][1] * A[0][1] + A[1][1] * A[1][1] + A[2][1] * A[2][1];
  const double det = g00 * g11 - g01 * g01;
  G.sg = sqrt(det);
  const double id = 1.0 / det;
  G.gi00 = g11 * id;
  G.gi01 = -g01 * id;
  G.gi11 = g00 * id;
  for (int ab = 0; ab < 3; ++ab) {
    const double t0 = A[0][0] * X2[0][ab] + A[1][0] * X2[1][ab] + A[2][0] * X2[2][ab];
    const double t1 = A[0][1] * X2[0][ab] + A[1][1] * X2[1][ab] + A[2][1] * X2[2][ab];
    G.gam[0][ab] = G.gi00 * t0 + G.gi01 * t1;
    G.gam[1][ab] = G.gi01 * t0 + G.gi11 * t1;
  }
  return G;
}
// Surface gradient g^{ab} N_b a_a (three components) and Laplace-Beltrami operator
// g^{ab} (N_ab - Gamma^c_ab N_c) of a function with parametric derivatives v = (N, N_1,
// N_2, N_11, N_12, N_22).
__device__ inline void surf_basis(const SurfGeom& G, const double v[6], double* gr, double* lb) {
  const double c0 = G.gi00 * v[1] + G.gi01 * v[2];
  const double c1 = G.gi01 * v[1] + G.gi11 * v[2];
  for (int a = 0; a < 3; ++a) gr[a] = G.A[a][0] * c0 + G.A[a][1] * c1;
  const double h00 = v[3] - G.gam[0][0] * v[1] - G.gam[1][0] * v[2];
  const double h01 = v[4] - G.gam[0][1] * v[1] - G.gam[1][1] * v[2];
  const double h11 = v[5] - G.gam[0][2] * v[1] - G.gam[1][2] * v[2];
  *lb = G.gi00 * h00 + 2.0 * G.gi01 * h01 + G.gi11 * h11;
}

// Basis data at the 4 x 4 Gauss points of every cell (values, physical gradients, Laplacians
// when GL is given; point-major per cell like the WQ data), gw = Gauss weight * |det J|, and
// the physical points when gx is given (dim coordinates per point). On a surface also GZ
// (the third surface-gradient component) and GL holds the Laplace-Beltrami operator.
// Asynchronous on st.
wq_status gauss_basis(wq_mesh* M, wq_points* P, double* GN, double* GX, double* GY, double* GZ, double* GL,
                      double* gw, double* gx, hipStream_t st);

// Rebuilds the cell-major assembly tiles of P with its current t2_stepcap (and counts the
// rebuild in t2_gen). Synchronises st.
wq_status rebuild_tiles2(wq_points* P, hipStream_t st);
// One heat time step (as wq_heat_step) on rows split into nseg consecutive segments
// [seg_row0[k], seg_row0[k + 1]) (host array) whose rows couple only within the segment
// (the meshes of a union): every segment is solved as if alone (its own reductions in its
// own block order, scalars, Newton and Krylov stops), in shared launches. reps[k] and
// stats[k] receive segment k's report and status; the return value is the call's own
// (arguments, device).
wq_status heat_step_segments(const wq_points* P, const wq_weights* w, const wq_heat_params* hp,
                             const uint8_t* dirichlet, const double* g_next, const double* f_at_pts, double* T,
                             double* Tdot, double* S_vals, int32_t nseg, const int64_t* seg_row0,
                             wq_heat_report* reps, wq_status* stats, hipStream_t st);

}  // namespace wq
