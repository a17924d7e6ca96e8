// solve_weights: exact right-hand sides by Gauss quadrature (Section 2, Section 4.2)
// and truncated-SVD weights (Section 4.3, Eqs. (19)-(22)) for every (row, family).
#include "wq_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>

using namespace wq;

namespace {

constexpr int BS = 256;
constexpr int GQ_GROUP = 16;   // lanes per row in the Gauss row kernel
constexpr int NFAM = 5;        // weight families: mass, d/dx, d/dy, Laplacian, d/dz (bit f of a mask)
constexpr int MAX_SWEEPS = 40;

// 4-point Gauss-Legendre on [0, 1]
__constant__ double c_gp[4] = {0.0694318442029737124, 0.3300094782075718676, 0.6699905217924281324,
                               0.9305681557970262876};
__constant__ double c_gw[4] = {0.1739274225687269287, 0.3260725774312730713, 0.3260725774312730713,
                               0.1739274225687269287};

__device__ inline void eval_fn(const double* C, const double b1[4], const double d1[4], const double s1[4],
                               const double b2[4], const double d2[4], const double s2[4], double out[6]) {
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int l = 0; l < 4; ++l) {
    double r0 = 0, r1 = 0, r2 = 0;
    for (int k = 0; k < 4; ++k) {
      const double c = C[k + 4 * l];
      r0 += c * b1[k];
      r1 += c * d1[k];
      r2 += c * s1[k];
    }
    v[0] += r0 * b2[l];
    v[1] += r1 * b2[l];
    v[2] += r0 * d2[l];
    v[3] += r2 * b2[l];
    v[4] += r1 * d2[l];
    v[5] += r0 * s2[l];
  }
  for (int q = 0; q < 6; ++q) out[q] = v[q];
}

// Basis data at the 16 Gauss points of every cell: G?[c*16*? ...] laid out like the WQ
// data (point-major, cell functions contiguous), plus gw = weight * |det J| and, when gx is
// given, the physical points at gx[dim (16 c + g) ..]. On a surface (dim 3) GX, GY, GZ hold
// the surface gradient and GL the Laplace-Beltrami operator.
__global__ void k_gauss_basis(int32_t ncell, const int32_t* cell_face, const uint8_t* cell_sub,
                              const int64_t* ext_ptr, const int64_t* coef_ptr, const double* coef,
                              const double* ctrl, const int64_t* cfn_ptr, const int32_t* cfn, const uint8_t* cfn_loc,
                              double* GN, double* GX, double* GY, double* GZ, double* GL, double* gw, double* gx,
                              int dim) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= 16LL * ncell) return;
  const int64_t c = t / 16;
  const int g = (int)(t % 16);
  const int32_t f = cell_face[c];
  const int sub = cell_sub[c];
  double b1[4], d1[4], s1[4], b2[4], d2[4], s2[4];
  bern3(c_gp[g % 4], b1, d1, s1);
  bern3(c_gp[g / 4], b2, d2, s2);
  const int mf = (int)(ext_ptr[f + 1] - ext_ptr[f]);
  const double* Cf = coef + coef_ptr[f] + (int64_t)sub * mf * 16;
  const int64_t f0 = cfn_ptr[c];
  const int m = (int)(cfn_ptr[c + 1] - f0);
  if (dim == 3) {  // a surface
    double x3[3] = {0, 0, 0}, A[3][2] = {{0, 0}, {0, 0}, {0, 0}}, X2[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int k = 0; k < m; ++k) {
      double v[6];
      eval_fn(Cf + 16 * (int)cfn_loc[f0 + k], b1, d1, s1, b2, d2, s2, v);
      const int32_t j = cfn[f0 + k];
      for (int a = 0; a < 3; ++a) {
        const double P = ctrl[3 * (int64_t)j + a];
        x3[a] += P * v[0];
        A[a][0] += P * v[1];
        A[a][1] += P * v[2];
        X2[a][0] += P * v[3];
        X2[a][1] += P * v[4];
        X2[a][2] += P * v[5];
      }
    }
    const SurfGeom SG = surf_geom(A, X2);
    gw[16 * c + g] = c_gw[g % 4] * c_gw[g / 4] * SG.sg;
    if (gx)
      for (int a = 0; a < 3; ++a) gx[3 * (16 * c + g) + a] = x3[a];
    const int64_t o = 16 * f0 + (int64_t)g * m;
    for (int k = 0; k < m; ++k) {
      double v[6], gr[3], lb;
      eval_fn(Cf + 16 * (int)cfn_loc[f0 + k], b1, d1, s1, b2, d2, s2, v);
      surf_basis(SG, v, gr, &lb);
      GN[o + k] = v[0];
      GX[o + k] = gr[0];
      GY[o + k] = gr[1];
      GZ[o + k] = gr[2];
      if (GL) GL[o + k] = lb;
    }
    return;
  }
  double J[2][2] = {{0, 0}, {0, 0}}, H[2][3] = {{0, 0, 0}, {0, 0, 0}}, X[2] = {0, 0};
  for (int k = 0; k < m; ++k) {
    double v[6];
    eval_fn(Cf + 16 * (int)cfn_loc[f0 + k], b1, d1, s1, b2, d2, s2, v);
    const int32_t j = cfn[f0 + k];
    for (int a = 0; a < 2; ++a) {
      const double P = ctrl[2 * (int64_t)j + a];
      X[a] += P * v[0];
      J[a][0] += P * v[1];
      J[a][1] += P * v[2];
      H[a][0] += P * v[3];
      H[a][1] += P * v[4];
      H[a][2] += P * v[5];
    }
  }
  const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const double id = 1.0 / det;
  const double Ji[2][2] = {{J[1][1] * id, -J[0][1] * id}, {-J[1][0] * id, J[0][0] * id}};
  const double G00 = Ji[0][0] * Ji[0][0] + Ji[0][1] * Ji[0][1];
  const double G01 = Ji[0][0] * Ji[1][0] + Ji[0][1] * Ji[1][1];
  const double G11 = Ji[1][0] * Ji[1][0] + Ji[1][1] * Ji[1][1];
  gw[16 * c + g] = c_gw[g % 4] * c_gw[g / 4] * fabs(det);
  if (gx) {
    gx[2 * (16 * c + g)] = X[0];
    gx[2 * (16 * c + g) + 1] = X[1];
  }
  const int64_t o = 16 * f0 + (int64_t)g * m;
  for (int k = 0; k < m; ++k) {
    double v[6];
    eval_fn(Cf + 16 * (int)cfn_loc[f0 + k], b1, d1, s1, b2, d2, s2, v);
    const double nx = Ji[0][0] * v[1] + Ji[1][0] * v[2];
    const double ny = Ji[0][1] * v[1] + Ji[1][1] * v[2];
    GN[o + k] = v[0];
    GX[o + k] = nx;
    GY[o + k] = ny;
    if (GL) {
      const double h00 = v[3] - nx * H[0][0] - ny * H[1][0];
      const double h01 = v[4] - nx * H[0][1] - ny * H[1][1];
      const double h11 = v[5] - nx * H[0][2] - ny * H[1][2];
      GL[o + k] = h00 * G00 + 2.0 * h01 * G01 + h11 * G11;
    }
  }
}

// Row i of the Gauss matrices on the CSR pattern, one 16-lane group per row:
// b^f_i[slot(j)] = sum_{cells c in supp i} sum_g gw_g D^f N_i(g) D^f N_j(g).
// Cells are visited in ascending order and each lane owns distinct slots at every
// step, so the summation order is fixed (deterministic, no atomics). Per cell, lane g of
// the group forms u_g = gw_g D^f N_i(g) once into LDS for the whole group (a group is
// part of one wave: its LDS accesses are ordered, the wave barriers only keep the
// compiler from moving them). LDS: the families in the mask, compacted.
__global__ void k_gauss_rows(int64_t n, const int64_t* sptr, const int32_t* scell, const int64_t* cfn_ptr,
                             const int64_t* soff, const uint8_t* slot, const uint8_t* kself, const int64_t* row_ptr,
                             const double* G0, const double* G1, const double* G2, const double* G3,
                             const double* G4, const double* gw, unsigned mask, int max_row, double* R0, double* R1,
                             double* R2, double* R3, double* R4) {
  extern __shared__ double sh_acc[];
  const int grp = threadIdx.x / GQ_GROUP;
  const int lane = threadIdx.x % GQ_GROUP;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / GQ_GROUP) + grp;
  const int nfam = __popc(mask);
  double* acc = sh_acc + (size_t)grp * nfam * max_row;
  double* su = sh_acc + (size_t)(blockDim.x / GQ_GROUP) * nfam * max_row + grp * NFAM * GQ_GROUP;
  const double* Gs[NFAM] = {G0, G1, G2, G3, G4};
  double* Rs[NFAM] = {R0, R1, R2, R3, R4};
  const bool active = i < n;
  for (int t = lane; t < nfam * max_row; t += GQ_GROUP) acc[t] = 0.0;
  __syncthreads();
  if (active) {
    for (int64_t p = sptr[i]; p < sptr[i + 1]; ++p) {
      const int32_t c = scell[p];
      const int64_t f0 = cfn_ptr[c];
      const int m = (int)(cfn_ptr[c + 1] - f0);
      const int ks = kself[p];
      const uint8_t* sl = slot + soff[p];
      for (int fam = 0, a = 0; fam < NFAM; ++fam) {
        if (!(mask & (1u << fam))) continue;
        su[a * GQ_GROUP + lane] = gw[16 * (int64_t)c + lane] * Gs[fam][16 * f0 + lane * m + ks];
        ++a;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int k = lane; k < m; k += GQ_GROUP) {
        const int sk = sl[k];
        for (int fam = 0, a = 0; fam < NFAM; ++fam) {
          if (!(mask & (1u << fam))) continue;
          const double* G = Gs[fam] + 16 * f0;
          const double* u = su + a * GQ_GROUP;
          double v = 0.0;
          for (int g = 0; g < 16; ++g) v += u[g] * G[g * m + k];
          acc[a * max_row + sk] += v;
          ++a;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  __syncthreads();
  if (active) {
    const int ni = (int)(row_ptr[i + 1] - row_ptr[i]);
    for (int fam = 0, a = 0; fam < NFAM; ++fam) {
      if (!(mask & (1u << fam))) continue;
      for (int t = lane; t < ni; t += GQ_GROUP) Rs[fam][row_ptr[i] + t] = acc[a * max_row + t];
      ++a;
    }
  }
}

// ------------------------------------------------------------------ TSVD
struct SysClass {
  int max_n, max_r;
};

// Size buckets of the weight systems: LDS is sized per bucket, so typical systems are
// not charged for the largest one. n bounds x r bounds.
// (The split at n = 56 keeps the instances with 7 and with 8 rows of M per lane in buckets
// of their own: a bucket's instance follows from its bounds alone.)
__constant__ int c_nb[6] = {32, 48, 56, 64, 96, 128};
__constant__ int c_rb[7] = {64, 80, 96, 128, 160, 192, 256};
constexpr int NB_N = 6, NB_R = 7, NBKT = NB_N * NB_R;

// Also sums, per bucket, the algorithmic FLOPs of its systems, 9 r n^2 - n^3: the work of a
// thin SVD of the n x r system by Golub-Kahan bidiagonalisation (4 r n^2 - 4 n^3 / 3), the
// formation of its left and right singular vectors (4 n^3 / 3 and 4 r n^2 - 4 n^3 / 3), the
// r x t Gram matrix of Z V_t (r t^2) and its Cholesky factor (t^3 / 3), at full rank
// t = n: the method's lower bound, the measure of useful work for the roofline (about
// 1.27 MFLOP for the 49 x 64 systems of regular rows).
__global__ void k_sys_bucket(int64_t n, const int64_t* row_ptr, const int64_t* qptr, uint8_t* bkt, int* hist,
                             int* bad, unsigned long long* flops) {
  // per-workgroup tallies in LDS, then one global update per touched bucket
  __shared__ int cnt[NBKT], mxn[NBKT], mxr[NBKT];
  __shared__ unsigned long long fl[NBKT];
  for (int b = threadIdx.x; b < NBKT; b += blockDim.x) {
    cnt[b] = 0;
    mxn[b] = 0;
    mxr[b] = 0;
    fl[b] = 0ULL;
  }
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) {
    const int ni = (int)(row_ptr[i + 1] - row_ptr[i]);
    const int ri = (int)(qptr[i + 1] - qptr[i]);
    int bn = 0, br = 0;
    while (bn < NB_N && ni > c_nb[bn]) ++bn;
    while (br < NB_R && ri > c_rb[br]) ++br;
    if (bn == NB_N || br == NB_R) {
      atomicOr(bad, 1);
      bn = NB_N - 1;
      br = NB_R - 1;
    }
    const int b = bn * NB_R + br;
    bkt[i] = (uint8_t)b;
    atomicAdd(&cnt[b], 1);
    atomicMax(&mxn[b], ni);  // per-bucket maxima (LDS sizing)
    atomicMax(&mxr[b], ri);
    const long long nn = ni, rr = ri;
    atomicAdd(&fl[b], (unsigned long long)(9 * rr * nn * nn - nn * nn * nn));
  }
  __syncthreads();
  for (int b = threadIdx.x; b < NBKT; b += blockDim.x)
    if (cnt[b]) {
      atomicAdd(&hist[b], cnt[b]);
      atomicMax(&hist[2 * (NBKT + 1) + 2 * b], mxn[b]);
      atomicMax(&hist[2 * (NBKT + 1) + 2 * b + 1], mxr[b]);
      atomicAdd(&flops[b], fl[b]);
    }
}

// Bucket lists: each workgroup reserves one range per touched bucket; the order of the
// systems inside a bucket is irrelevant (they are independent).
__global__ void k_sys_scatter(int64_t n, const uint8_t* bkt, const int64_t* start, int* cur, int32_t* lists) {
  __shared__ int cnt[NBKT], base[NBKT];
  for (int b = threadIdx.x; b < NBKT; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int b = -1, k = 0;
  if (i < n) {
    b = bkt[i];
    k = atomicAdd(&cnt[b], 1);
  }
  __syncthreads();
  for (int bb = threadIdx.x; bb < NBKT; bb += blockDim.x)
    if (cnt[bb]) base[bb] = atomicAdd(&cur[bb], cnt[bb]);
  __syncthreads();
  if (b >= 0) lists[start[b] + base[b] + k] = (int32_t)i;
}

// Cross-lane moves inside a row of 16 lanes by DPP (VALU, no LDS round trip).
// Every lane reads an existing lane of its row (no bound_ctrl case), so no old value.
template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over aligned groups of G = 4, 8 or 16 lanes; every lane of a group gets the same
// bits (quad_perm [1,0,3,2], then [2,3,0,1], then the mirrored quad, then the mirrored 8).
template <int G>
__device__ inline double group_sum(double v) {
  static_assert(G == 4 || G == 8 || G == 16, "group of 4, 8 or 16 lanes");
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  if (G >= 8) v += dpp_f64<0x141>(v);  // row_half_mirror: the other quad of the 8
  if (G >= 16) v += dpp_f64<0x140>(v); // row_mirror: the other 8 of the row
  return v;
}

// 1/x and 1/sqrt(x) for positive normal x: the hardware estimates refined by two Newton
// steps (each doubles the number of correct bits).
__device__ inline double rcp_f64(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  return fma(y, fma(-x, y, 1.0), y);
}

__device__ inline double rsq_f64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// order-preserving bit pattern of a non-negative double for atomicMin/atomicMax
__device__ inline unsigned long long dbits(double v) { return (unsigned long long)__double_as_longlong(v); }

struct TsvdArgs {
  const int32_t* rows;
  int64_t nsys;
  int ld;   // leading dimension (doubles) of a column of A^T in LDS, >= r_max + 1
  int ldm;  // leading dimension of a column of R^T in LDS, >= n_max rounded up to 8, <= ld
  int nfam;  // families in this launch: workgroup b solves system b % nsys of family b / nsys
  double tau;
  const int64_t* sptr;
  const int32_t* scell;
  const int64_t* cfn_ptr;
  const int64_t* cell_pt_off;
  const int64_t* dptr;
  const int64_t* soff;
  const uint8_t* slot;
  const uint8_t* kself;
  const int64_t* row_ptr;
  const int64_t* qptr;
  const double* D[NFAM];    // basis data of each family of the launch
  const double* DN;         // values (for Z)
  const double* rhs[NFAM];  // Gauss right-hand side of each family, aligned with col
  double* W[NFAM];          // output weights of each family, aligned with qidx
  int* max_sweeps;
  unsigned long long* min_kept;     // bits of a double
  unsigned long long* max_dropped;  // bits of a double
  unsigned long long* truncated;
  unsigned long long* certified;  // systems solved on the certified-rank path
  int* fail;
  const int32_t* sel;  // nullable: workgroup b solves system sel[b] (family-major index) instead of b
  int32_t* fb_list;    // one-wave solver: systems left to the SVD kernel (family-major index)
  int rp_n;            // one-wave solver: the largest n its dynamic LDS holds R11 for
  int* fb_count;
  unsigned direct_mask;  // SVD kernel: family slots whose systems first try the direct proof
  int fam_base;          // one-wave solver: family slot of the launch's first workgroups
};

__device__ inline double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
  return s;
}

__device__ inline double block_max(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s = fmax(s, red[k]);
  return s;
}

// Householder reflector for a column whose trailing part (rows j..) has first entry x0
// and squared norm s2: H = I - tau v v^T maps it to R_jj e_j, with v_j = 1 and
// v_m = x_m * rv0 below (rv0 = 1 / (x0 - R_jj)). s2 = 0: identity (tau = 0, R_jj = x0).
__device__ inline void householder(double x0, double s2, double* rjj, double* rv0, double* tau) {
  if (s2 == 0.0) {
    *rjj = x0;
    *rv0 = 0.0;
    *tau = 0.0;
    return;
  }
  const double b = -copysign(sqrt(s2), x0);
  *rjj = b;
  *rv0 = 1.0 / (x0 - b);
  *tau = (b - x0) / b;
}

// double <-> lane moves for the pivot search
__device__ inline double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Largest (value, index) of a wave, ties to the smaller index; every LPP-lane group holds
// one candidate (the same bits in all its lanes). Lane 0 stores it at cv[w], ci[w].
template <int LPP>
__device__ inline void wave_argmax(double v, int i, double* cv, double* ci) {
  if (LPP == 8) {  // the two groups of a 16-lane row: rotate the row by 8
    const double ov = dpp_f64<0x128>(v);
    const int oi = __builtin_amdgcn_mov_dpp(i, 0x128, 0xF, 0xF, false);
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
  double bv = readlane_f64(v, 0);
  int bi = __builtin_amdgcn_readlane(i, 0);
#pragma unroll
  for (int row = 1; row < 4; ++row) {
    const double rv = readlane_f64(v, 16 * row);
    const int ri = __builtin_amdgcn_readlane(i, 16 * row);
    if (rv > bv || (rv == bv && ri < bi)) {
      bv = rv;
      bi = ri;
    }
  }
  if ((threadIdx.x & 63) == 0) {
    cv[threadIdx.x >> 6] = bv;
    ci[threadIdx.x >> 6] = (double)bi;
  }
}

// Largest (value, index) over aligned groups of G = 8 or 16 lanes, ties to the smaller
// index; every lane of a group gets the result. The choice is a maximum in a total order,
// so it is the same as that of a scan in any order.
template <int G>
__device__ inline void group_argmax(double& v, int& i) {
  static_assert(G == 8 || G == 16, "group of 8 or 16 lanes");
  auto step = [&](double ov, int oi) {
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  };
  step(dpp_f64<0xB1>(v), __builtin_amdgcn_mov_dpp(i, 0xB1, 0xF, 0xF, false));
  step(dpp_f64<0x4E>(v), __builtin_amdgcn_mov_dpp(i, 0x4E, 0xF, 0xF, false));
  step(dpp_f64<0x141>(v), __builtin_amdgcn_mov_dpp(i, 0x141, 0xF, 0xF, false));
  if (G >= 16) step(dpp_f64<0x140>(v), __builtin_amdgcn_mov_dpp(i, 0x140, 0xF, 0xF, false));
}

// Apply reflector j (stored unscaled in physical column pc: v_j = 1, v_m = x_m rv0 below)
// to the logical columns l > j (physical phys(l): cur[l], except cj for l = bi, the pivot's
// old position), LPP lanes per column, and recompute their trailing squared norms (rows
// > j) exactly; returns this group's largest (norm, l), ties to the smaller l.
// Largest (value, lane) of the wave, ties to the smaller lane: the same in every lane.
__device__ inline void wave_argmax64(double v, int i, double& bv, int& bi) {
  group_argmax<16>(v, i);
  bv = readlane_f64(v, 0);
  bi = __builtin_amdgcn_readlane(i, 0);
#pragma unroll
  for (int row = 1; row < 4; ++row) {
    const double rv = readlane_f64(v, 16 * row);
    const int ri = __builtin_amdgcn_readlane(i, 16 * row);
    if (rv > bv || (rv == bv && ri < bi)) {
      bv = rv;
      bi = ri;
    }
  }
}

// Sum over the wave in a fixed order, the same bits in every lane.
__device__ inline double wave_sum64(double v) {
  v = group_sum<16>(v);
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

template <int LPP, int EPR, int NG>
__device__ inline double qr_update(double* G, int ld, int r, int ncol, int j, int pc, const int* cur, int bi, int cj,
                                   double tau, double rv0, int g, int sub, int* best_l) {
  const double* cp = G + (size_t)pc * ld;
  double best = -1.0;
  int bl = 0x7fffffff;
  for (int l = j + 1 + g; l < ncol; l += NG) {
    double* cl = G + (size_t)(l == bi ? cj : cur[l]) * ld;
    double x[EPR], v[EPR];
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < EPR; ++e) {
      const int m = j + sub + LPP * e;
      x[e] = (m < r) ? cl[m] : 0.0;
      v[e] = (m == j) ? 1.0 : ((m < r) ? cp[m] * rv0 : 0.0);
      s += v[e] * x[e];
    }
    s = tau * group_sum<LPP>(s);
    double ns = 0.0;
#pragma unroll
    for (int e = 0; e < EPR; ++e) {
      const int m = j + sub + LPP * e;
      if (m < r) {
        const double y = x[e] - s * v[e];
        if (tau != 0.0) cl[m] = y;
        if (m > j) ns += y * y;
      }
    }
    ns = group_sum<LPP>(ns);
    if (ns > best) {  // l ascends: ties keep the smaller l
      best = ns;
      bl = l;
    }
  }
  *best_l = bl;
  return best;
}

// One Jacobi rotation of the columns p, q (LPP lanes, rows sub + e LPP at gp[e LPP],
// gq[e LPP]): the 2x2 Gram block is diagonalised when the columns are not yet orthogonal
// to working precision and neither is negligible. Rows past the column's length are
// zero. GUARD: only the first ne rows of a lane exist; otherwise all EPJ do.
// The squared column norms are tracked in *np, *nq (the exact update of a rotation that
// zeroes the off-diagonal: |p'|^2 = |p|^2 - t g, |q'|^2 = |q|^2 + t g), so only the inner
// product is reduced per rotation; where the update cancels (a norm drops below 1e-3 of
// its old value) both are recomputed from the rotated columns. Returns whether the columns
// met at |cos| above 3e-8 (cos^2 = g^2 / (|p|^2 |q|^2) > 1e-15, tested without a division).
template <int LPP, int EPJ, bool GUARD>
__device__ inline bool jacobi_pair(double* gp, double* gq, double* np, double* nq, int sub, int ne, double negl) {
  double u[EPJ], v[EPJ];
#pragma unroll
  for (int e = 0; e < EPJ; ++e) {
    u[e] = (!GUARD || e < ne) ? gp[e * LPP] : 0.0;
    v[e] = (!GUARD || e < ne) ? gq[e * LPP] : 0.0;
  }
  const double al = *np, be = *nq;
  double ga = 0;
#pragma unroll
  for (int e = 0; e < EPJ; ++e) ga += u[e] * v[e];
  ga = group_sum<LPP>(ga);
  if (!(ga * ga > 1e-30 * al * be && fmin(al, be) > negl)) return false;
  // t = tan of the rotation angle (the smaller root), c = 1 / sqrt(1 + t^2), s = c t. t
  // only has to be close to the exact angle; c is accurate to rounding for the t used, so
  // the rotation is orthogonal to working precision.
  const double dba = be - al;
  const double h = dba * dba + 4.0 * ga * ga;
  const double t = (dba >= 0 ? 2.0 * ga : -2.0 * ga) * rcp_f64(fabs(dba) + h * rsq_f64(h));
  const double cs = rsq_f64(1.0 + t * t);
  const double sn = cs * t;
#pragma unroll
  for (int e = 0; e < EPJ; ++e) {
    const double pu = cs * u[e] - sn * v[e];
    const double qv = sn * u[e] + cs * v[e];
    u[e] = pu;
    v[e] = qv;
    if (!GUARD || e < ne) {
      gp[e * LPP] = pu;
      gq[e * LPP] = qv;
    }
  }
  double an = al - t * ga, bn = be + t * ga;
  if (an < 1e-3 * al || bn < 1e-3 * be) {  // uniform over the LPP lanes of the pair
    an = 0.0;
    bn = 0.0;
#pragma unroll
    for (int e = 0; e < EPJ; ++e) {
      an += u[e] * u[e];
      bn += v[e] * v[e];
    }
    an = group_sum<LPP>(an);
    bn = group_sum<LPP>(bn);
  }
  if (sub == 0) {
    *np = an;
    *nq = bn;
  }
  return ga * ga > 1e-15 * (al * be);
}

// One rotation of the pair (s, t) where the lanes of the group hold column s in registers
// (u, squared norm al, the same in every lane of the group) and column t sits in LDS at gq
// (squared norm *nq). Only column t is read and written back. Returns whether the columns
// met at |cos| above 3e-8, as jacobi_pair does.
template <int LPP, int EPJ, bool GUARD>
__device__ inline bool jacobi_held(double (&u)[EPJ], double& al, double* gq, double* nq, int sub, int ne,
                                     double negl) {
  double v[EPJ];
#pragma unroll
  for (int e = 0; e < EPJ; ++e) v[e] = (!GUARD || e < ne) ? gq[e * LPP] : 0.0;
  const double be = *nq;
  double ga = 0;
#pragma unroll
  for (int e = 0; e < EPJ; ++e) ga += u[e] * v[e];
  ga = group_sum<LPP>(ga);
  if (!(ga * ga > 1e-30 * al * be && fmin(al, be) > negl)) return false;
  // t = tan of the rotation angle (the smaller root), c = 1 / sqrt(1 + t^2), s = c t
  const double dba = be - al;
  const double h = dba * dba + 4.0 * ga * ga;
  const double t = (dba >= 0 ? 2.0 * ga : -2.0 * ga) * rcp_f64(fabs(dba) + h * rsq_f64(h));
  const double cs = rsq_f64(1.0 + t * t);
  const double sn = cs * t;
#pragma unroll
  for (int e = 0; e < EPJ; ++e) {
    const double pu = cs * u[e] - sn * v[e];
    const double qv = sn * u[e] + cs * v[e];
    u[e] = pu;
    v[e] = qv;
    if (!GUARD || e < ne) gq[e * LPP] = qv;
  }
  double an = al - t * ga, bn = be + t * ga;
  if (an < 1e-3 * al || bn < 1e-3 * be) {  // uniform over the LPP lanes of the pair
    an = 0.0;
    bn = 0.0;
#pragma unroll
    for (int e = 0; e < EPJ; ++e) {
      an += u[e] * u[e];
      bn += v[e] * v[e];
    }
    an = group_sum<LPP>(an);
    bn = group_sum<LPP>(bn);
  }
  const bool big = ga * ga > 1e-15 * (al * be);
  al = an;
  if (sub == 0) *nq = bn;
  return big;
}

// Recursive-halving pair ordering for the Jacobi sweeps. A block of m columns [lo, hi)
// splits into S = its first ceil(m/2) columns and T = the rest; the S x T pairs take
// ceil(m/2) rounds, in which the group of S column j meets T column (j + round) mod
// ceil(m/2) (when that exists), holding its S column in registers throughout; then both
// halves recurse, side by side. Level L holds the blocks L splits down. Every pair of
// the n columns meets once per sweep, and in each round a column is touched by one group.
__device__ inline int halving_groups(int m) { return m >= 2 ? (m + 1) / 2 : 0; }
// groups used k levels below a block of m columns (its parts there have floor or ceil of
// m / 2^k columns; m mod 2^k of them the larger)
__device__ inline int halving_groups_at(int m, int k) {
  const int q0 = m >> k, c = m - (q0 << k);
  return c * halving_groups(q0 + 1) + ((1 << k) - c) * halving_groups(q0);
}
struct HalvingSlot {
  int s, tlo, tcnt, h, j;  // S column, first T column, T count, S count of the block, rank in S
};
// the block and S column of group g at level L (j >= h: the group has no S column there)
__device__ inline HalvingSlot halving_slot(int n, int L, int g) {
  int lo = 0, hi = n, g0 = 0;
  for (int l2 = 0; l2 < L; ++l2) {
    const int a = (hi - lo + 1) / 2;
    const int gA = halving_groups_at(a, L - l2 - 1);
    if (g < g0 + gA) {
      hi = lo + a;
    } else {
      g0 += gA;
      lo += a;
    }
  }
  const int m = hi - lo, h = halving_groups(m);
  return HalvingSlot{lo + (g - g0), lo + h, m - h, h, g - g0};
}

// Weight system of one (row i, family): A (n x r, A[l][m] = D N_{S_i[l]}(x_{Q_i[m]})),
// z (r, z_m = N_i(x_{Q_i[m]})), b (n). Truncated SVD of Eqs. (20)-(22) with the weighted
// solution of Eqs. (5)-(6):
//  1. A^T (r x n) is reduced by Householder QR with column pivoting, A^T P = Q1 R1
//     (P permutes the constraints);
//  2. one-sided Jacobi on the columns of M = R1^T (n x n): M J = W has orthogonal columns,
//     sigma_k = |w_k|, and the left singular vectors of A are U = P W Sigma^-1 (Q1 is never
//     needed). Jacobi on the triangular factor of a pivoted QR converges in fewer sweeps
//     than on A^T itself, and its columns have length n instead of r;
//  3. keep sigma_k > tau sigma_1; c_k = u_k^T b / sigma_k; V_t = A^T U_t Sigma_t^-1 (A
//     re-read from the basis blocks), X = Z V_t;
//  4. X = Q R (Householder), y = R^-T c, w = Z Q [y; 0].
// Where the pivoted QR already proves which singular values the cutoff keeps (a gap at
// tau around its k-th step, certified by bounds on ||R22|| and ||R11^-1||), the QR stops
// at step k and steps 2-3 are skipped: X = Z A_k^T over the k pivot rows of A and c =
// their entries of b give the same solution (the kept span is that of those rows). The
// derivative families always have such a gap (their rows sum to zero, and the geometry's
// other coordinate is a second null direction), as do the mass rows of regular cells.
// One workgroup per system; everything lives in LDS.
template <int LPP, int EPR, int EPJ, int NT>
__global__ void __launch_bounds__(NT) k_tsvd2(TsvdArgs a) {
  extern __shared__ double sh[];
  constexpr int NG = NT / LPP;  // lane groups
  const int64_t wg = a.sel ? (int64_t)a.sel[blockIdx.x] : (int64_t)blockIdx.x;
  const int fs = (int)(wg / a.nsys);
  const int64_t sys = wg - (int64_t)fs * a.nsys;
  const double* AD = a.D[fs];
  const int tid = threadIdx.x;
  const int g = tid / LPP, sub = tid % LPP;
  const int64_t i = a.rows[sys];
  const int n = (int)(a.row_ptr[i + 1] - a.row_ptr[i]);
  const int r = (int)(a.qptr[i + 1] - a.qptr[i]);
  const int ld = a.ld, ldm = a.ldm;
  // host sizing violated (QR row slots, X formation rows, Jacobi rows, strides): report,
  // touch nothing
  if (r > EPR * LPP || r > NT || n > EPJ * LPP || n > 2 * NG || (n + LPP - 1) / LPP * LPP > ldm || ldm > ld ||
      ld < r + 1) {
    if (tid == 0) atomicOr(a.fail, 2);
    return;
  }
  double* G = sh;                   // n * ld: columns of A^T, later of X
  double* z = G + (size_t)n * ld;   // r
  double* sig = z + r;              // n
  double* Rk = sig + n;             // n: b
  double* yv = Rk + n;              // n: c
  double* nrm = yv + n;             // n: squared column norms of M in the Jacobi sweeps
  double* beta = nrm + n;           // n: R_jj of a QR
  double* red = beta + n;           // 96: block reductions [0, 32), pivot candidates [32, 96)
  int* keep = (int*)(red + 96);     // n + 1
  int* piv = keep + n + 1;          // n: the column permutation (two buffers in the QR)
  int* pinv = piv + n;              // n
  int* cmap = pinv + n;             // n
  int* ptc = cmap + n;              // r: support entry of the point's cell
  int* ptq = ptc + r;               // r: point index inside its cell
  // ---- 1. gather A^T, z, b
  for (int t = tid; t < n * ld; t += NT) G[t] = 0.0;
  __syncthreads();
  {
    int moff = 0;
    for (int64_t p = a.sptr[i]; p < a.sptr[i + 1]; ++p) {
      const int32_t c = a.scell[p];
      const int m = (int)(a.cfn_ptr[c + 1] - a.cfn_ptr[c]);
      const int np = (int)(a.cell_pt_off[c + 1] - a.cell_pt_off[c]);
      const double* Dc = AD + a.dptr[c];
      const double* Nc = a.DN + a.dptr[c];
      const uint8_t* sl = a.slot + a.soff[p];
      const int ks = a.kself[p];
      for (int t = tid; t < np * m; t += NT) {
        const int q = t / m, k = t - q * m;
        G[(size_t)sl[k] * ld + moff + q] = Dc[t];
      }
      for (int q = tid; q < np; q += NT) {
        z[moff + q] = Nc[q * m + ks];
        ptc[moff + q] = (int)(p - a.sptr[i]);
        ptq[moff + q] = q;
      }
      moff += np;
    }
    for (int l = tid; l < n; l += NT) {
      Rk[l] = a.rhs[fs][a.row_ptr[i] + l];
      piv[l] = l;
    }
  }
  __syncthreads();
  // ||A||_F^2: columns of M below 1e-15 ||A||_F are numerical null space (dropped with a
  // 1000x margin by the 1e-12 cutoff); pairs involving them need no rotation
  double fro2 = 0.0;
  for (int e = tid; e < n * r; e += NT) {
    const int l = e / r, m = e - l * r;
    const double v = G[(size_t)l * ld + m];
    fro2 += v * v;
  }
  const double fa2 = block_sum(fro2, red);
  const double negl = 1e-30 * fa2;
  // Direct path (the families whose systems are full rank but for rare exceptions, the mass
  // family): the rank is proved from the R of X = Z A^T itself, sigma_n(A) >= sigma_n(Z A^T)
  // / max z = 1 / (||R^-1||_2 max z), so the pivoted QR, which only serves the proof, is
  // skipped. X is A^T scaled in place, c = b, all n constraints kept; the proof follows the
  // second factorisation (step 4). A system it does not cover is listed and solved by the
  // full path in a second launch.
  const bool direct = ((a.direct_mask >> fs) & 1u) && a.sel == nullptr && n <= r;
  int t;  // the kept count
  if (direct) {
    for (int e = tid; e < n * r; e += NT) {
      const int l = e / r, m = e - l * r;
      G[(size_t)l * ld + m] *= z[m];
    }
    for (int l = tid; l < n; l += NT) yv[l] = Rk[l];
    __syncthreads();
    t = n;
  } else {
    // ---- 2. Householder QR of A^T with column pivoting (largest trailing norm first).
    // Columns are addressed through a permutation (no data swaps); reflector j is kept
    // unscaled in its column (v_j = 1, v_m = x_m / (x_j - R_jj) below), R_jj in beta[j].
    // One barrier per column: every thread picks the pivot from the per-wave candidates of
    // the previous update and forms the reflector itself; the permutation and the
    // candidates are double-buffered (read one buffer, write the other).
    constexpr int NW = NT / 64;
    {
      double best = -1.0;
      int bl = 0x7fffffff;
      for (int l = g; l < n; l += NG) {
        double s2 = 0.0;
        for (int m = sub; m < r; m += LPP) s2 += G[(size_t)l * ld + m] * G[(size_t)l * ld + m];
        s2 = group_sum<LPP>(s2);
        if (s2 > best) {
          best = s2;
          bl = l;
        }
      }
      wave_argmax<LPP>(best, bl, red + 32, red + 48);
    }
    __syncthreads();
    const int kmax = min(n, r);
    // With early set, the factorisation stops before step j once the trailing block is
    // negligible: ||R22||_F^2 <= (n - j) * (largest trailing column norm^2) below
    // (tau / 10)^2 R_00^2 (R_00^2 = s20, the largest column norm^2 of A^T), a hundred times
    // the rounding level of the factorisation for tau = 1e-12. Returns the
    // step it stopped before (kmax when it ran to the end); s2stop is that step's pivot norm^2.
    double s20 = 0.0, s2stop = 0.0;
    auto qr_steps = [&](int j0, bool early) -> int {
      for (int j = j0; j < kmax; ++j) {
        const double* cv = red + 32 + 32 * (j & 1);
        const int* cur = (j & 1) ? cmap : piv;
        int* nxt = (j & 1) ? piv : cmap;
        double s2;
        int bi;
        if constexpr (NW >= 8) {  // one candidate per lane of each group of NW lanes
          s2 = cv[tid & (NW - 1)];
          bi = (int)cv[16 + (tid & (NW - 1))];
          group_argmax<NW>(s2, bi);
        } else {
          s2 = cv[0];
          bi = (int)cv[16];
          for (int w = 1; w < NW; ++w) {
            const double v = cv[w];
            const int i2 = (int)cv[16 + w];
            if (v > s2 || (v == s2 && i2 < bi)) {
              s2 = v;
              bi = i2;
            }
          }
        }
        if (j == 0) s20 = s2;
        if (early && (double)(n - j) * s2 < 1e-2 * a.tau * a.tau * s20) {
          s2stop = s2;
          return j;
        }
        const int cj = cur[j], pc = cur[bi];
        double rjj, rv0, tj;
        householder(G[(size_t)pc * ld + j], s2, &rjj, &rv0, &tj);
        if (tid == 0) beta[j] = rjj;
        for (int l = tid; l < n; l += NT) nxt[l] = l == j ? pc : (l == bi ? cj : cur[l]);
        int bl;
        const double best = qr_update<LPP, EPR, NG>(G, ld, r, n, j, pc, cur, bi, cj, tj, rv0, g, sub, &bl);
        double* nv = red + 32 + 32 * ((j + 1) & 1);
        wave_argmax<LPP>(best, bl, nv, nv + 16);
        __syncthreads();
      }
      return kmax;
    };
    const int kq = qr_steps(0, true);
    // ---- certified rank. The truncated-SVD solution only depends on the kept count t, the
    // span of the kept right singular vectors and the kept part of b. sigma_{k+1} <= ||R22||
    // and sigma_k >= sigma_min(R11) - ||R22|| >= 1 / ||R11^-1||_F - ||R22|| (R11: the
    // leading k x k block, R22: the trailing block, k = kq), and tau sigma_1 lies between
    // tau R_00 and tau ||A||_F. So when ||R22|| is below tau R_00 / 10 and the kept bound
    // is above 100 tau ||A||_F, the cutoff keeps exactly k singular values, and their span is
    // that of the k pivot rows of A up to O(eps / gap): the solution is then the weighted
    // minimum-norm solution of those k equations, w = Z Q R^-T b_k for Z A_k^T = Q R (step 4
    // below), the same as the SVD's to rounding times the conditioning. Otherwise the
    // factorisation runs to the end and the Jacobi SVD decides.
    // Column c of S = R11^-T (lower triangular), eight lanes per column: S[ii][c] = (delta -
    // sum_{jj = c}^{ii - 1} R[jj][ii] S[jj][c]) / R[ii][ii], with R[.][ii] read down the
    // physical column of logical column ii (rows < ii) and S[.][c] kept in rows c+1 .. kq of
    // the physical column of logical column c (its reflector rows, no longer needed: no
    // thread reads R there). Lane s of a column's group takes jj = c + s (mod 8), the group
    // sums by DPP, and its first lane stores S[ii][c] (read by the group's lanes, in the same
    // wave, at the next steps: one LDS latency per step instead of one per four terms).
    const int* pk = (kq & 1) ? cmap : piv;  // logical column l of R is constraint pk[l]
    const double r22 = kq < kmax ? sqrt((double)(n - kq) * s2stop) : 0.0;
    double lo = 0.0;
    bool fast = false;
    if (s20 > 0.0 && kq > 0) {
      double tn = 0.0;
      const int cs = tid & 7;
      for (int c = tid >> 3; c < kq; c += NT / 8) {  // (whole groups of eight lanes)
        double* Sc = G + (size_t)pk[c] * ld + 1;  // S[jj][c] at Sc[jj]
        for (int ii = c; ii < kq; ++ii) {
          const double* Rc = G + (size_t)pk[ii] * ld;  // R[jj][ii] at Rc[jj], jj < ii
          double s0 = 0.0, s1 = 0.0;
          int jj = c + cs;
          for (; jj + 8 < ii; jj += 16) {
            s0 = fma(Rc[jj], Sc[jj], s0);
            s1 = fma(Rc[jj + 8], Sc[jj + 8], s1);
          }
          if (jj < ii) s0 = fma(Rc[jj], Sc[jj], s0);
          const double sum = group_sum<8>(s0 + s1);
          const double v = ((ii == c ? 1.0 : 0.0) - sum) / beta[ii];
          if (cs == 0) {
            Sc[ii] = v;
            tn = fma(v, v, tn);
          }
          __builtin_amdgcn_wave_barrier();
        }
      }
      tn = block_sum(tn, red);  // the same bits in every thread: the branch is uniform
      lo = 1.0 / sqrt(tn) - r22;
      fast = lo > 100.0 * a.tau * sqrt(fa2);
    }
    if (fast) {
      // X = Z A_k^T: the k pivot rows of A, re-read from the basis blocks, as the columns
      for (int l = tid; l < n; l += NT) pinv[pk[l]] = l;
      for (int c = tid; c < kq; c += NT) yv[c] = Rk[pk[c]];
      if (tid == 0) {
        atomicMin(a.min_kept, dbits(lo / sqrt(fa2)));       // a lower bound of sigma_k / sigma_1
        atomicMax(a.max_dropped, dbits(r22 / sqrt(s20)));  // an upper bound of sigma_{k+1} / sigma_1
        if (kq < n) atomicAdd(a.truncated, 1ULL);
        atomicAdd(a.certified, 1ULL);
      }
      __syncthreads();
      for (int e = tid; e < kq * ld; e += NT) G[e] = 0.0;
      __syncthreads();
      int moff = 0;
      for (int64_t p = a.sptr[i]; p < a.sptr[i + 1]; ++p) {
        const int32_t c = a.scell[p];
        const int m = (int)(a.cfn_ptr[c + 1] - a.cfn_ptr[c]);
        const int np = (int)(a.cell_pt_off[c + 1] - a.cell_pt_off[c]);
        const double* Dc = AD + a.dptr[c];
        const uint8_t* sl = a.slot + a.soff[p];
        for (int e = tid; e < np * m; e += NT) {
          const int q = e / m, k = e - q * m;
          const int col = pinv[sl[k]];
          if (col < kq) G[(size_t)col * ld + moff + q] = z[moff + q] * Dc[e];
        }
        moff += np;
      }
      __syncthreads();
      t = kq;
    } else {
      if (kq < kmax) qr_steps(kq, false);
      // the final permutation: logical column l of R is constraint perm[l]
      const int* perm = (kmax & 1) ? cmap : piv;
      // ---- M = R1^T: column k of M is row k of R1, M[k][i] = R1[k][i] = G[i][k] for i >= k.
      // M sits at the end of the G area (X is later written from the start; see step 3).
      double* M = G + (size_t)n * ld - (size_t)n * ldm;
      {
        constexpr int MS = (EPJ * LPP * EPJ * LPP + NT - 1) / NT;  // n^2 <= (EPJ LPP)^2
        double val[MS];
    #pragma unroll
        for (int s2 = 0; s2 < MS; ++s2) {
          const int e = tid + NT * s2;
          const int k = e / n, ii = e - k * n;
          val[s2] = (e < n * n && ii >= k && k < kmax) ? (ii == k ? beta[k] : G[(size_t)perm[ii] * ld + k]) : 0.0;
        }
        __syncthreads();
    #pragma unroll
        for (int s2 = 0; s2 < MS; ++s2) {
          const int e = tid + NT * s2;
          const int k = e / n, ii = e - k * n;
          if (e < n * n) M[(size_t)k * ldm + ii] = val[s2];
        }
        for (int e = tid; e < n * (ldm - n); e += NT) M[(size_t)(e / (ldm - n)) * ldm + n + e % (ldm - n)] = 0.0;
        for (int l = tid; l < n; l += NT) pinv[perm[l]] = l;
      }
      __syncthreads();
      // ---- one-sided Jacobi on the columns of M. Rows [n, ldm) of every column are zero, and
      // ne LPP <= ldm. Two pair orderings (each visits every pair once per sweep):
      //  - recursive halving: each group holds the S column of its pairs in registers for a
      //    whole level, so a rotation reads and writes only its T column in LDS (half the LDS
      //    traffic) and sweeps are fewer; it costs registers and a few more rounds and barriers;
      //  - the circle method: both columns of a pair through LDS in every round.
      // Instances take the ordering that measured faster for their buckets: halving for
      // 48 < n <= 56 (r <= 128), for 48 < n <= 64 with 80 < r <= 128 and for n <= 64 with
      // r > 128; circle for the rest, where the held column cost occupancy or the extra rounds
      // cost more than the LDS traffic saved.
      constexpr bool HALVING = (NT == 256 && (EPJ == 7 || EPR == 32)) || (NT == 512 && LPP == 16);
      const int ne = (n + LPP - 1) / LPP;
      const bool full = ldm >= EPJ * LPP;  // all EPJ rows of a lane inside the column: no checks
      int sweeps = 0;
      bool converged = false;
      double* cn = nrm;  // squared column norms of M (nrm is free after the QR)
      if constexpr (HALVING) {
        int nlev = 0;
        while (((n + (1 << nlev) - 1) >> nlev) >= 2) ++nlev;
        for (sweeps = 0; sweeps < MAX_SWEEPS && !converged; ++sweeps) {
          bool big = false;  // a pair of this sweep met at |cos| above 3e-8
          // fresh norms at each sweep bound the drift of the tracked updates
          for (int l = g; l < n; l += NG) {
            double s2 = 0.0;
            for (int m = sub; m < n; m += LPP) s2 += M[(size_t)l * ldm + m] * M[(size_t)l * ldm + m];
            s2 = group_sum<LPP>(s2);
            if (sub == 0) cn[l] = s2;
          }
          __syncthreads();
          double u[EPJ];
          double al = 0.0;
          int held = -1;  // the column in u, or -1
          for (int L = 0; L < nlev; ++L) {
            const HalvingSlot sl = halving_slot(n, L, g);
            const bool act = sl.j < sl.h;
            const int want = act ? sl.s : -1;
            if (L > 0) {
              // a column no longer held goes back to LDS before anyone reads it
              if (held >= 0 && held != want) {
                double* gp = M + (size_t)held * ldm + sub;
    #pragma unroll
                for (int e = 0; e < EPJ; ++e)
                  if (full || e < ne) gp[e * LPP] = u[e];
                if (sub == 0) cn[held] = al;
                held = -1;
              }
              __syncthreads();
            }
            if (act && held != want) {
              const double* gp = M + (size_t)want * ldm + sub;
    #pragma unroll
              for (int e = 0; e < EPJ; ++e) u[e] = (full || e < ne) ? gp[e * LPP] : 0.0;
              al = cn[want];
              held = want;
            }
            const int rounds = halving_groups((n + (1 << L) - 1) >> L);
            for (int rd = 0; rd < rounds; ++rd) {
              if (act && rd < sl.h) {
                int k = sl.j + rd;
                if (k >= sl.h) k -= sl.h;
                if (k < sl.tcnt) {
                  const int cQ = sl.tlo + k;
                  double* gq = M + (size_t)cQ * ldm + sub;
                  big |= full ? jacobi_held<LPP, EPJ, false>(u, al, gq, cn + cQ, sub, ne, negl)
                              : jacobi_held<LPP, EPJ, true>(u, al, gq, cn + cQ, sub, ne, negl);
                }
              }
              __syncthreads();
            }
          }
          if (held >= 0) {
            double* gp = M + (size_t)held * ldm + sub;
    #pragma unroll
            for (int e = 0; e < EPJ; ++e)
              if (full || e < ne) gp[e * LPP] = u[e];
            if (sub == 0) cn[held] = al;
          }
          __syncthreads();
          // Cyclic Jacobi converges quadratically: after a sweep whose rotations all had |cos|
          // below 3e-8, the columns are orthogonal to about |cos| ~ 1e-15, the level at which a
          // pair is rotated at all, so the sweep that would only confirm it is skipped.
          converged = !__syncthreads_or(big);
        }
      } else {
        const int nn = n + (n & 1);
        const int npair = nn / 2;
        for (sweeps = 0; sweeps < MAX_SWEEPS && !converged; ++sweeps) {
          bool big = false;  // a pair of this sweep met at |cos| above 3e-8
          // fresh norms at each sweep bound the drift of the tracked updates
          for (int l = g; l < n; l += NG) {
            double s2 = 0.0;
            for (int m = sub; m < n; m += LPP) s2 += M[(size_t)l * ldm + m] * M[(size_t)l * ldm + m];
            s2 = group_sum<LPP>(s2);
            if (sub == 0) cn[l] = s2;
          }
          __syncthreads();
          // Circle method on positions 0..nn-1: pair p starts at positions (p, nn - 1 - p);
          // position 0 stays, positions 1..nn-1 advance by one per round (cyclically), so every
          // two positions meet once per sweep. Position 0 holds column nn - 1 (the padding
          // column when n is odd), position c > 0 column c - 1; pair 0 (which holds the padding
          // column in every round for odd n) runs on the last group, so for odd n the last pair
          // group does no work and a wave whose groups are all past the real pairs skips the
          // round entirely.
          const int pp = (g + 1 == npair) ? 0 : g + 1;
          int P = pp, Q = nn - 1 - pp;
          for (int rd = 0; rd < nn - 1; ++rd) {
            const int cP = P == 0 ? nn - 1 : P - 1, cQ = Q - 1;
            if (g < npair && cP < n && cQ < n) {
              double* gp = M + (size_t)cP * ldm + sub;
              double* gq = M + (size_t)cQ * ldm + sub;
              big |= full ? jacobi_pair<LPP, EPJ, false>(gp, gq, cn + cP, cn + cQ, sub, ne, negl)
                          : jacobi_pair<LPP, EPJ, true>(gp, gq, cn + cP, cn + cQ, sub, ne, negl);
            }
            P = (P == 0) ? 0 : (P == nn - 1 ? 1 : P + 1);
            Q = (Q == nn - 1) ? 1 : Q + 1;
            __syncthreads();
          }
          // Cyclic Jacobi converges quadratically: after a sweep whose rotations all had |cos|
          // below 3e-8, the columns are orthogonal to about |cos| ~ 1e-15, the level at which a
          // pair is rotated at all, so the sweep that would only confirm it is skipped.
          converged = !__syncthreads_or(big);
        }
      }
      if (!converged && tid == 0) atomicOr(a.fail, 1);
      if (tid == 0) atomicMax(a.max_sweeps, sweeps);
      // ---- 3. singular values, truncation, c
      double smax = 0.0;
      for (int l = g; l < n; l += NG) {
        double s2 = 0.0;
        for (int m = sub; m < n; m += LPP) s2 += M[(size_t)l * ldm + m] * M[(size_t)l * ldm + m];
        s2 = group_sum<LPP>(s2);
        if (sub == 0) sig[l] = sqrt(s2);
        smax = fmax(smax, sqrt(s2));
      }
      smax = block_max(smax, red);
      if (tid == 0) {
        int t = 0;
        double kmin = INFINITY, dmax = 0.0;
        for (int l = 0; l < n; ++l) {
          if (sig[l] > a.tau * smax) {
            keep[t++] = l;
            kmin = fmin(kmin, sig[l] / smax);
          } else {
            dmax = fmax(dmax, sig[l] / smax);
          }
        }
        keep[n] = t;
        atomicMin(a.min_kept, dbits(kmin));
        atomicMax(a.max_dropped, dbits(dmax));
        if (t < n) atomicAdd(a.truncated, 1ULL);
      }
      __syncthreads();
      t = keep[n];
      // c_k = u_k^T b / sigma_k = (w_k . P^T b) / sigma_k^2
      for (int k = g; k < t; k += NG) {
        const double* wk = M + (size_t)keep[k] * ldm;
        double s2 = 0.0;
        for (int m = sub; m < n; m += LPP) s2 += wk[m] * Rk[perm[m]];
        s2 = group_sum<LPP>(s2);
        if (sub == 0) yv[k] = s2 / (sig[keep[k]] * sig[keep[k]]);
      }
      // X[m][k] = z_m sum_l A[l][m] U[l][k] / sigma_k with U[l][k] = M[pinv[l]][keep[k]] /
      // sigma_k. The threads form NP parts of RW (r rounded up to whole waves) rows each; part
      // g2 forms columns k0 + g2 KC + (0 .. KC-1) of a chunk of NP KC columns. Columns are
      // written from the start of G, M's columns sit at the end: the writes of a chunk never
      // reach a column of M still to be read (n ld >= k ld + n ldm - (n - k) ldm for k <= n,
      // as ldm <= ld), and a chunk's own columns are read before the barrier.
      constexpr int KC = 8;
      {
        const int RW = (r + 63) / 64 * 64;
        const int NP = NT / RW;  // >= 1: r <= NT
        const int g2 = tid / RW, m = tid - g2 * RW;
        const bool row = g2 < NP && m < r;
        const double* Dc = nullptr;
        const uint8_t* sl = nullptr;
        int mc = 0;
        if (row) {
          const int64_t p = a.sptr[i] + ptc[m];
          const int32_t c = a.scell[p];
          mc = (int)(a.cfn_ptr[c + 1] - a.cfn_ptr[c]);
          Dc = AD + a.dptr[c] + (int64_t)ptq[m] * mc;
          sl = a.slot + a.soff[p];
        }
        for (int k0 = 0; k0 < t; k0 += NP * KC) {
          const int kb = k0 + g2 * KC;
          double acc[KC];
    #pragma unroll
          for (int kq = 0; kq < KC; ++kq) acc[kq] = 0.0;
          if (row)
            for (int kk = 0; kk < mc; ++kk) {
              const double av = Dc[kk];
              const int ii = pinv[sl[kk]];
    #pragma unroll
              for (int kq = 0; kq < KC; ++kq)
                if (kb + kq < t) acc[kq] += av * M[(size_t)keep[kb + kq] * ldm + ii];
            }
          __syncthreads();
          if (row) {
    #pragma unroll
            for (int kq = 0; kq < KC; ++kq)
              if (kb + kq < t) {
                const double sk = sig[keep[kb + kq]];
                G[(size_t)(kb + kq) * ld + m] = z[m] * acc[kq] / (sk * sk);
              }
          }
          __syncthreads();
        }
      }
    }
  }
  // ---- 4. Householder QR of X (no pivoting; reflector j kept unscaled in its column as in
  // step 2, R_jj in beta, tau in tq, 1 / (x_j - R_jj) in rvq, the trailing squared norms
  // in nq), one barrier per column; then, in the first wave, y = R^-T c over c (lanes over
  // columns, y_j handed on by read-lane) and u = Q [y; 0] = H_0 ... H_{t-1} [y; 0] (the
  // reflectors in reverse, u in registers, four points per lane); w = Z u.
  double* tq = sig;   // free: the singular values only formed X and c
  double* rvq = Rk;   // free: b is in c (yv) by now
  double* nq = nrm;   // free after the Jacobi sweeps
  if (g == 0 && t > 0) {  // the first column's norm (each step forms the next one's)
    double s2 = 0.0;
    for (int m = sub; m < r; m += LPP) s2 += G[m] * G[m];
    s2 = group_sum<LPP>(s2);
    if (sub == 0) nq[0] = s2;
  }
  __syncthreads();
  for (int j = 0; j < t; ++j) {
    double rjj, rv0, tj;
    householder(G[(size_t)j * ld + j], nq[j], &rjj, &rv0, &tj);
    if (tid == 0) {
      beta[j] = rjj;
      tq[j] = tj;
      rvq[j] = rv0;
    }
    const double* cp = G + (size_t)j * ld;
    for (int l = j + 1 + g; l < t; l += NG) {
      double* cl = G + (size_t)l * ld;
      double x[EPR], v[EPR];
      double sv = 0.0;
#pragma unroll
      for (int e = 0; e < EPR; ++e) {
        const int m = j + sub + LPP * e;
        x[e] = (m < r) ? cl[m] : 0.0;
        v[e] = (m == j) ? 1.0 : ((m < r) ? cp[m] * rv0 : 0.0);
        sv += v[e] * x[e];
      }
      sv = tj * group_sum<LPP>(sv);
      // (no pivoting: only the next column's trailing norm is needed)
      const bool next = l == j + 1;
      double ns = 0.0;
#pragma unroll
      for (int e = 0; e < EPR; ++e) {
        const int m = j + sub + LPP * e;
        if (m < r) {
          const double y = x[e] - sv * v[e];
          if (tj != 0.0) cl[m] = y;
          if (next && m > j) ns += y * y;
        }
      }
      if (next) {  // (one whole group)
        ns = group_sum<LPP>(ns);
        if (sub == 0) nq[l] = ns;
      }
    }
    __syncthreads();
  }
  if (direct) {
    // column c of S = R^-T, eight lanes per column, lane s holding rows c + s + 8q in
    // registers (the reflectors below the diagonal of X stay for the solve): S[c+d][c] =
    // (delta_{d0} - sum_{d' < d} R[c+d'][c+d] S[c+d'][c]) / R[c+d][c+d]
    constexpr int SR = (EPJ * LPP + 7) / 8;
    const int cs = tid & 7;
    double tn = 0.0;
    for (int c = tid >> 3; c < t; c += NT / 8) {  // (whole groups of eight lanes)
      double sv[SR];
#pragma unroll
      for (int q = 0; q < SR; ++q) sv[q] = 0.0;
#pragma unroll
      for (int d = 0; d < 8 * SR; ++d) {
        if (c + d < t) {
          const double* Rc = G + (size_t)(c + d) * ld + c;  // R[c+d'][c+d] at Rc[d']
          double sacc = 0.0;
#pragma unroll
          for (int q = 0; q < SR; ++q)
            if (cs + 8 * q < d) sacc = fma(Rc[cs + 8 * q], sv[q], sacc);
          const double v = ((d == 0 ? 1.0 : 0.0) - group_sum<8>(sacc)) / beta[c + d];
          if ((d & 7) == cs) sv[d >> 3] = v;
          if (cs == 0) tn = fma(v, v, tn);
        }
      }
    }
    tn = block_sum(tn, red);
    double zm = 0.0;
    for (int m = tid; m < r; m += NT) zm = fmax(zm, z[m]);
    zm = block_max(zm, red);
    const double lo = 1.0 / (sqrt(tn) * zm);
    if (!(tn > 0.0 && lo > 100.0 * a.tau * sqrt(fa2))) {  // (uniform)
      if (tid == 0) a.fb_list[atomicAdd(a.fb_count, 1)] = (int32_t)wg;
      return;
    }
    if (tid == 0) {
      atomicMin(a.min_kept, dbits(lo / sqrt(fa2)));  // a lower bound of sigma_n / sigma_1
      atomicAdd(a.certified, 1ULL);
    }
  }
  if (tid >= 64) return;
  {
    const int lane = tid;
    // y_jj = (c_jj - sum_{jj' < jj} R[jj'][jj] y_jj') / R_jj; lane l accumulates the sums of
    // columns l and 64 + l (R[jj][k] at G[k ld + jj])
    double a0 = 0.0, a1 = 0.0;
    for (int jj = 0; jj < t; ++jj) {
      const double aj = readlane_f64(jj < 64 ? a0 : a1, jj & 63);
      const double yj = (yv[jj] - aj) / beta[jj];
      if (lane == 0) yv[jj] = yj;
      if (lane > jj && lane < t) a0 = fma(G[(size_t)lane * ld + jj], yj, a0);
      if (64 + lane > jj && 64 + lane < t) a1 = fma(G[(size_t)(64 + lane) * ld + jj], yj, a1);
    }
    __builtin_amdgcn_wave_barrier();
    double u[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = lane + 64 * q;
      u[q] = m < t ? yv[m] : 0.0;
    }
    for (int j = t - 1; j >= 0; --j) {
      const double* cp = G + (size_t)j * ld;
      const double rv = rvq[j], tj = tq[j];
      double vm[4];
      double d = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = lane + 64 * q;
        vm[q] = m == j ? 1.0 : (m > j && m < r ? cp[m] * rv : 0.0);
        d = fma(vm[q], u[q], d);
      }
      d = wave_sum64(d);
#pragma unroll
      for (int q = 0; q < 4; ++q) u[q] = fma(-tj * d, vm[q], u[q]);
    }
    double* W = a.W[fs] + a.qptr[i];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = lane + 64 * q;
      if (m < r) W[m] = z[m] * u[q];
    }
  }
}


// ---------------------------------------------------------------------------------
// One wave per weight system, for systems of at most 64 constraints and 64 points (the
// rows of regular cells and most of their neighbours). Lane l holds a column of the
// factorised matrix in registers, one double per point, so the Householder steps need no
// cross-lane reductions: the reflector's column is broadcast through LDS and every lane
// forms its own dot product and update. The steps are those of the certified path of
// k_tsvd2 (the kept count proved from the pivoted QR of A^T), with the second
// factorisation and the solve held in registers:
//  1. pivoted Householder QR of A^T, stopped once the trailing block is negligible;
//  2. the rank proof (||R11^-1||_F from R11^-T, one column per lane);
//  3. Householder QR of X = Z A_k^T (the k pivot rows of A, re-read from the basis blocks);
//  4. y = R^-T b_k, u = Q [y; 0] (the reflectors applied in reverse), w = Z u, and one
//     step of iterative refinement on the residual of the k kept equations where that
//     residual is above rounding level.
// Rows above the current step are zero in the broadcast column, so the passes skip the
// blocks of 16 rows that lie wholly above it (a uniform branch; the sums are unchanged,
// the skipped terms being exact zeros).
// A system the proof does not cover is appended to a list for k_tsvd2 (the Jacobi SVD).
constexpr int WR = 64;     // points (rows) held per lane
constexpr int WB = 16;     // rows per skipped block
constexpr int WMAXC = 40;  // support cells of a row in the gather tables

// DIRECT (the mass family, full rank but for rare exceptions): no pivoted QR. X = Z A^T over
// all n constraints is factorised and solved and the weights written; the rank is then proved
// from that QR's R, sigma_n(A) >= sigma_n(Z A^T) / max z >= 1 / (||R^-1||_F max z), once the
// reflectors' registers are free. A system the proof does not cover is listed for k_tsvd2,
// whose full path overwrites its weights. (A separate instance, so that the pivoted path's
// register allocation stays as it is.)
template <bool DIRECT>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) k_wsolve(TsvdArgs a) {
  __shared__ double vb[WR + 4];  // the current reflector's column (4 zero pads past the rows)
  __shared__ double zv[WR], bv[WR], beta[WR], ib[WR], tau2[WR], rv2[WR], uv2[WR];
  extern __shared__ double rp[];  // R11 above the diagonal by columns: n_max (n_max - 1) / 2
  __shared__ int64_t cbase[WMAXC];
  __shared__ int cmc[WMAXC];
  __shared__ uint8_t invk[WMAXC * WR];  // local index of row function l in support cell p, 255: none
  __shared__ uint8_t ptp[WR + 4], ptq[WR + 4];  // support cell and local index of every point
  __shared__ int pk[WR];                        // position -> constraint of the pivoted QR
  const int lane = threadIdx.x;
  const int fl = (int)(blockIdx.x / a.nsys);
  const int64_t sys = blockIdx.x - (int64_t)fl * a.nsys;
  const int fs = a.fam_base + fl;  // family slot
  const double* AD = a.D[fs];
  const int64_t i = a.rows[sys];
  const int n = (int)(a.row_ptr[i + 1] - a.row_ptr[i]);
  const int r = (int)(a.qptr[i + 1] - a.qptr[i]);
  const int64_t s0 = a.sptr[i];
  const int nc = (int)(a.sptr[i + 1] - s0);
  auto to_svd = [&]() {  // (the family-major index over all the bucket's families)
    if (lane == 0) a.fb_list[atomicAdd(a.fb_count, 1)] = (int32_t)((int64_t)a.fam_base * a.nsys + blockIdx.x);
  };
  if (n > WR || n > a.rp_n || r > WR || nc < 1 || nc >= WMAXC || (DIRECT && n > r)) {
    to_svd();
    return;
  }
  // ---- gather tables (every point belongs to one support cell; np, m <= r, n <= 64).
  // Rows past r point at a sentinel cell nc whose functions are all absent.
  {
    int moff = 0;
    for (int p = 0; p < nc; ++p) {
      const int32_t c = a.scell[s0 + p];
      const int mc = (int)(a.cfn_ptr[c + 1] - a.cfn_ptr[c]);
      const int np = (int)(a.cell_pt_off[c + 1] - a.cell_pt_off[c]);
      const int64_t d0 = a.dptr[c];
      invk[p * WR + lane] = 255;
      __builtin_amdgcn_wave_barrier();
      if (lane < mc) invk[p * WR + a.slot[a.soff[s0 + p] + lane]] = (uint8_t)lane;
      if (lane < np) {
        ptp[moff + lane] = (uint8_t)p;
        ptq[moff + lane] = (uint8_t)lane;
        zv[moff + lane] = a.DN[d0 + (int64_t)lane * mc + a.kself[s0 + p]];
      }
      if (lane == 0) {
        cbase[p] = d0;
        cmc[p] = mc;
      }
      moff += np;
    }
    invk[nc * WR + lane] = 255;
    if (lane == 0) {
      cbase[nc] = cbase[0];
      cmc[nc] = 0;
    }
    if (lane >= r) {
      ptp[lane] = (uint8_t)nc;
      ptq[lane] = 0;
      zv[lane] = 0.0;
    }
    if (lane < 4) {  // pads read by the residual loop (rows in fours)
      ptp[WR + lane] = (uint8_t)nc;
      ptq[WR + lane] = 0;
      vb[WR + lane] = 0.0;
    }
    if (lane < n) bv[lane] = a.rhs[fs][a.row_ptr[i] + lane];
  }
  __syncthreads();
  // Column of A^T for row function fl (every point), times z when zs; zero where !valid.
  // Branch-free: every lane loads from a valid address and selects away what it does not
  // have; the loads go out in batches of 16.
  auto gather = [&](int fl, bool valid, bool zs, double(&x)[WR]) {
    const int fq = valid ? fl : 0;
#pragma unroll
    for (int m = 0; m < WR; ++m) {
      const int p = ptp[m];
      const int kk = invk[p * WR + fq];
      const bool has = valid && kk != 255;
      const double v = AD[cbase[p] + (int64_t)ptq[m] * cmc[p] + (has ? kk : 0)];
      x[m] = has ? (zs ? v * zv[m] : v) : 0.0;
      if ((m & 15) == 15) asm volatile("" ::: "memory");
    }
  };
  // The pivot column (lane p) of step j into vb, rows above j zero, and its reflector: vb[j]
  // = x0 - R_jj = 1 / rv0 (so v_j = 1 up to rounding). Blocks wholly above row j are neither
  // written nor read. Returns x0.
  auto load_pivot = [&](const double(&x)[WR], int j, int p, double s2, double& rjj, double& rv0,
                        double& tj) -> double {
    if (lane == p) {
#pragma unroll
      for (int b = 0; b < WR / WB; ++b)
        if (j < WB * b + WB) {
#pragma unroll
          for (int m = WB * b; m < WB * b + WB; ++m) vb[m] = x[m];
        }
    }
    if (lane < j) vb[lane] = 0.0;
    __syncthreads();
    const double x0 = vb[j];
    householder(x0, s2, &rjj, &rv0, &tj);
    if (lane == 0) vb[j] = x0 - rjj;
    __syncthreads();
    return x0;
  };
  // v^T x (v = vb, zero above row j).
  auto dot = [&](const double(&x)[WR], int j) -> double {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int b = 0; b < WR / WB; ++b)
      if (j < WB * b + WB) {
#pragma unroll
        for (int m = WB * b; m < WB * b + WB; ++m) acc[m & 3] = fma(vb[m], x[m], acc[m & 3]);
      }
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
  };
  // x -= sv v; returns the squared norm of the rows below j. Every lane runs it (sv = 0
  // leaves a column as it is).
  auto update = [&](double(&x)[WR], int j, double sv) -> double {
    asm volatile("" ::: "memory");  // re-read vb rather than hold 64 more doubles
#pragma unroll
    for (int b = 0; b < WR / WB; ++b)
      if (j < WB * b + WB) {
#pragma unroll
        for (int m = WB * b; m < WB * b + WB; ++m) x[m] = fma(-sv, vb[m], x[m]);
      }
    double ns[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int b = 0; b < WR / WB; ++b) {
      if (j < WB * b) {
#pragma unroll
        for (int m = WB * b; m < WB * b + WB; ++m) ns[m & 3] = fma(x[m], x[m], ns[m & 3]);
      } else if (j < WB * b + WB) {
#pragma unroll
        for (int m = WB * b; m < WB * b + WB; ++m) ns[m & 3] = fma(x[m], m > j ? x[m] : 0.0, ns[m & 3]);
      }
    }
    return (ns[0] + ns[1]) + (ns[2] + ns[3]);
  };
  double x[WR];
  // ---- 1. pivoted Householder QR of A^T (lane l: column l), with the early stop of k_tsvd2
  gather(lane, lane < n, false, x);
  double nrm = 0.0;  // squared norm of the rows from the current step on
#pragma unroll
  for (int m = 0; m < WR; ++m) nrm = fma(x[m], x[m], nrm);
  const double fa2 = wave_sum64(nrm);
  const int kmax = min(n, r);
  int pos = lane < n ? -1 : WR;  // position once pivoted (lanes past n never are)
  double s20 = 0.0, s2stop = 0.0;
  int kq = kmax;
  for (int j = 0; j < (DIRECT ? 0 : kmax); ++j) {  // (DIRECT: no pivoted QR)
    double s2;
    int p;
    wave_argmax64(pos < 0 ? nrm : -1.0, lane, s2, p);
    if (j == 0) s20 = s2;
    if ((double)(n - j) * s2 < 1e-2 * a.tau * a.tau * s20) {
      kq = j;
      s2stop = s2;
      break;
    }
    double rjj, rv0, tj;
    load_pivot(x, j, p, s2, rjj, rv0, tj);
    if (lane == p) {
      pk[j] = p;
      beta[j] = rjj;
      pos = j;
    }
    const double d = dot(x, j);
    nrm = update(x, j, pos < 0 ? tj * rv0 * rv0 * d : 0.0);
  }
  // ---- 2. rank proof: sigma_{k+1} <= ||R22||_F <= sqrt((n - k) s2stop) and sigma_k >=
  // 1 / ||R11^-1||_F - ||R22||_F (as in k_tsvd2)
  const double r22 = kq < kmax ? sqrt((double)(n - kq) * s2stop) : 0.0;
  if (!DIRECT && pos >= 1 && pos < kq) {
    const int base = pos * (pos - 1) / 2;
#pragma unroll
    for (int m = 0; m < WR - 1; ++m)
      if (m < pos) rp[base + m] = x[m];
  }
  if (!DIRECT && lane < kq) ib[lane] = 1.0 / beta[lane];
  if (DIRECT && lane < n) pk[lane] = lane;  // (kq = n: all constraints, in order)
  __syncthreads();
  double lo = 0.0;
  bool fast = DIRECT;
  if (!DIRECT && s20 > 0.0 && kq > 0) {
    // column `lane` of S = R11^-T (lower triangular): S[ii][c] = (delta - sum_{jj < ii}
    // R[jj][ii] S[jj][c]) / R[ii][ii]; the entries above the diagonal come out zero
    double t[WR];
    double tn = 0.0;
#pragma unroll
    for (int ii = 0; ii < WR; ++ii) {
      if (ii < kq) {  // a uniform branch, not an exit: the loop unrolls fully
        double sa[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int jj = 0; jj < ii; ++jj) {
          sa[jj & 3] = fma(rp[ii * (ii - 1) / 2 + jj], t[jj], sa[jj & 3]);
          if ((jj & 15) == 15) asm volatile("" ::: "memory");  // at most 16 loads in flight
        }
        const double v = ((lane == ii ? 1.0 : 0.0) - ((sa[0] + sa[1]) + (sa[2] + sa[3]))) * ib[ii];
        t[ii] = v;
        tn = fma(v, v, tn);
      }
    }
    lo = 1.0 / sqrt(wave_sum64(tn)) - r22;
    fast = lo > 100.0 * a.tau * sqrt(fa2);
  }
  if (!fast) {
    to_svd();
    return;
  }
  // ---- 3. Householder QR of X = Z A_k^T (lane c: position c)
  if constexpr (DIRECT) {  // the columns of A^T in order, already held: scaled by z
#pragma unroll
    for (int m = 0; m < WR; ++m) x[m] *= zv[m];
  } else {
    gather(lane < kq ? pk[lane] : 0, lane < kq, true, x);
  }
  nrm = 0.0;
#pragma unroll
  for (int m = 0; m < WR; ++m) nrm = fma(x[m], x[m], nrm);
  for (int j = 0; j < kq; ++j) {
    double rjj, rv0, tj;
    const double x0 = load_pivot(x, j, j, readlane_f64(nrm, j), rjj, rv0, tj);
    if (lane == 0) {
      beta[j] = rjj;
      tau2[j] = tj;
      rv2[j] = rv0;
      uv2[j] = x0 - rjj;
    }
    const double d = dot(x, j);
    nrm = update(x, j, lane > j && lane < kq ? tj * rv0 * rv0 * d : 0.0);
  }
  // X has full column rank (sigma_k(A) > 0 and z > 0 on the points); R_jj != 0 is checked
  // anyway before dividing by it
  if (__any(lane < kq && !(fabs(beta[lane]) > 0.0 && fabs(beta[lane]) < INFINITY))) {
    to_svd();
    return;
  }
  if (!DIRECT && lane == 0) {
    atomicMin(a.min_kept, dbits(lo / sqrt(fa2)));       // a lower bound of sigma_k / sigma_1
    atomicMax(a.max_dropped, dbits(r22 / sqrt(s20)));  // an upper bound of sigma_{k+1} / sigma_1
    if (kq < n) atomicAdd(a.truncated, 1ULL);
    atomicAdd(a.certified, 1ULL);
  }
  // ---- 4. u = Q [R^-T c; 0] for the right-hand side c (lane c: c_c; result: lane m, row
  // m). R^-T by columns of R (lane c holds R[0..c-1][c]); Q = H_0 ... H_{k-1} applied to
  // [y; 0] in reverse, with the reflectors of step 3.
  auto solve = [&](double cv) -> double {
    const double id = lane < kq ? 1.0 / beta[lane] : 0.0;
    double u = 0.0, acc = 0.0;
#pragma unroll
    for (int ii = 0; ii < WR; ++ii) {
      if (ii < kq) {
        const double yi = readlane_f64((cv - acc) * id, ii);
        if (lane == ii) u = yi;
        acc = fma(x[ii], yi, acc);
      }
    }
    for (int j = kq - 1; j >= 0; --j) {
      if (lane == j) {
#pragma unroll
        for (int b = 0; b < WR / WB; ++b)
          if (j < WB * b + WB) {
#pragma unroll
            for (int m = WB * b; m < WB * b + WB; ++m) vb[m] = x[m];
          }
      }
      if (lane < j) vb[lane] = 0.0;
      if (lane == 0) vb[j] = uv2[j];
      __syncthreads();
      const double vm = lane < r ? vb[lane] * rv2[j] : 0.0;
      const double d = wave_sum64(vm * u);
      u = fma(-tau2[j] * d, vm, u);
      __syncthreads();
    }
    return u;
  };
  // w = Z u, then one step of iterative refinement on the k kept equations: rho = b_k -
  // A_k w (A_k re-read from the basis blocks, w broadcast through vb), w += Z solve(rho).
  // It takes the residual of the kept equations from about eps kappa(X) to rounding level.
  // (solve runs in every lane: it holds barriers and cross-lane sums)
  const double u0 = solve(lane < kq ? bv[pk[lane]] : 0.0);
  const double w = lane < r ? zv[lane] * u0 : 0.0;
  vb[lane] = w;
  __syncthreads();
  double rho = 0.0;
  {
    const int fq = lane < kq ? pk[lane] : 0;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int m0 = 0; m0 < r; m0 += 4) {  // a runtime loop (no register index depends on m); rows
      // past r read the pads (sentinel cell, vb = 0)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + e;
        const int p = ptp[m];
        const int kk = invk[p * WR + fq];
        const bool has = lane < kq && kk != 255;
        const double v = AD[cbase[p] + (int64_t)ptq[m] * cmc[p] + (has ? kk : 0)];
        acc[e] = fma(has ? v : 0.0, vb[m], acc[e]);
      }
    }
    if (lane < kq) rho = bv[fq] - ((acc[0] + acc[1]) + (acc[2] + acc[3]));
  }
  __syncthreads();
  // The step only moves w when the residual is above rounding level: where every kept
  // equation already holds to 1e-14 of the largest |b_k| (most systems), w stands.
  double bmax;
  int bl;
  wave_argmax64(lane < kq ? fabs(bv[pk[lane]]) : 0.0, 0, bmax, bl);
  const bool settled = !__any(fabs(rho) > 1e-14 * bmax);
  if (settled) {
    if (lane < r) a.W[fs][a.qptr[i] + lane] = w;
    if constexpr (!DIRECT) return;
  }
  if (!DIRECT || !settled) {
    const double dw = solve(rho);
    if (lane < r) a.W[fs][a.qptr[i] + lane] = fma(zv[lane], dw, w);
  }
  if constexpr (DIRECT) {
    // the rank proof from the R of X (column c above the diagonal in lane c's points below
    // c): all n kept where 1 / (||R^-1||_F max z) > 100 tau ||A||_F
    if (lane >= 1 && lane < n) {
      const int base = lane * (lane - 1) / 2;
#pragma unroll
      for (int m = 0; m < WR - 1; ++m)
        if (m < lane) rp[base + m] = x[m];
    }
    if (lane < n) ib[lane] = 1.0 / beta[lane];
    __syncthreads();
    double zm;
    wave_argmax64(lane < r ? zv[lane] : 0.0, 0, zm, bl);
    double t[WR];
    double tn = 0.0;
#pragma unroll
    for (int ii = 0; ii < WR; ++ii) {
      if (ii < n) {  // a uniform branch, not an exit: the loop unrolls fully
        double sa[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int jj = 0; jj < ii; ++jj) {
          sa[jj & 3] = fma(rp[ii * (ii - 1) / 2 + jj], t[jj], sa[jj & 3]);
          if ((jj & 15) == 15) asm volatile("" ::: "memory");  // at most 16 loads in flight
        }
        const double v = ((lane == ii ? 1.0 : 0.0) - ((sa[0] + sa[1]) + (sa[2] + sa[3]))) * ib[ii];
        t[ii] = v;
        tn = fma(v, v, tn);
      }
    }
    tn = wave_sum64(tn);
    lo = 1.0 / (sqrt(tn) * zm);
    if (!(tn > 0.0 && lo > 100.0 * a.tau * sqrt(fa2))) {
      to_svd();
      return;
    }
    if (lane == 0) {
      atomicMin(a.min_kept, dbits(lo / sqrt(fa2)));  // a lower bound of sigma_n / sigma_1
      atomicAdd(a.certified, 1ULL);
    }
  }
}


// Side streams for the independent launches of one call (the size buckets): created per
// call (wq_set_side_streams of them, 4 by default), non-blocking and of default priority,
// forked from the caller's stream and joined back into it by events. Launch k goes to side
// stream k mod N, so that the small launches (a bucket's last partial round of workgroups,
// the second launches of the few systems a first pass leaves) fill the CUs the large ones
// leave idle. With one (or if creation fails) every launch stays on the caller's stream.
struct Fork {
  static constexpr int NMAX = 8;
  hipStream_t home;
  hipStream_t s[NMAX] = {};
  hipEvent_t e[NMAX + 1] = {};
  int n = 0;
  bool ok = false;
  int next = 0;
  explicit Fork(hipStream_t st) : home(st) {
    const int want = std::min(std::max(side_streams(), 1), NMAX);
    if (want < 2) return;
    ok = true;
    for (; n < want && ok; ++n) ok = hipStreamCreateWithFlags(&s[n], hipStreamNonBlocking) == hipSuccess;
    for (int k = 0; k <= n && ok; ++k) ok = hipEventCreateWithFlags(&e[k], hipEventDisableTiming) == hipSuccess;
  }
  ~Fork() {
    for (int k = 0; k < NMAX; ++k)
      if (s[k]) (void)hipStreamDestroy(s[k]);
    for (int k = 0; k <= NMAX; ++k)
      if (e[k]) (void)hipEventDestroy(e[k]);
  }
  // the side streams wait for the caller's work so far
  bool fork() {
    next = 0;
    if (!ok) return true;
    if (hipEventRecord(e[n], home) != hipSuccess) return false;
    for (int k = 0; k < n; ++k)
      if (hipStreamWaitEvent(s[k], e[n], 0) != hipSuccess) return false;
    return true;
  }
  hipStream_t lane() { return ok ? s[next++ % n] : home; }
  // the caller's stream waits for the side streams' work
  bool join() {
    if (!ok) return true;
    for (int k = 0; k < n; ++k)
      if (hipEventRecord(e[k], s[k]) != hipSuccess || hipStreamWaitEvent(home, e[k], 0) != hipSuccess) return false;
    return true;
  }
};

void release_weights(wq_weights* w) {
  DBuf* all[2 * NFAM];
  for (int f = 0; f < NFAM; ++f) {
    all[2 * f] = &w->W[f];
    all[2 * f + 1] = &w->rhs[f];
  }
  dfree_many(all, 2 * NFAM);
}

}  // namespace

wq_status wq::gauss_basis(wq_mesh* M, wq_points* P, double* GN, double* GX, double* GY, double* GZ, double* GL,
                          double* gw, double* gx, hipStream_t st) {
  KTimer tm("k_gauss_basis", 16LL * P->ncell, st);
  k_gauss_basis<<<nblocks(16LL * P->ncell, BS), BS, 0, st>>>(
      P->ncell, P->cell_face.as<int32_t>(), P->cell_sub.as<uint8_t>(), M->ext_ptr.as<int64_t>(),
      M->coef_ptr.as<int64_t>(), M->coef.as<double>(), M->ctrl.as<double>(), P->cfn_ptr.as<int64_t>(),
      P->cfn.as<int32_t>(), P->cfn_loc.as<uint8_t>(), GN, GX, GY, GZ, GL, gw, gx, M->dim);
  tm.stop();
  return hipGetLastError() == hipSuccess ? WQ_OK : WQ_EDEVICE;
}

extern "C" wq_status solve_weights(wq_mesh* M, wq_points* P, unsigned fam_mask, double tau, wq_stream stream,
                                   wq_weights** out, wq_solve_report* rep) {
  WQ_CHECK(M && P && out && P->mesh == M, WQ_EINVAL, "solve_weights: bad arguments");
  WQ_CHECK(fam_mask && !(fam_mask & ~31u), WQ_EINVAL, "solve_weights: bad family mask");
  WQ_CHECK(!(fam_mask & WQ_FAM_DZ) || M->dim == 3, WQ_EINVAL,
           "solve_weights: the d/dz family exists on surfaces (dim 3) only");
  WQ_CHECK(!(fam_mask & WQ_FAM_LAP) || P->has_lap, WQ_EINVAL,
           "solve_weights: Laplacian weights need build_points(want_laplacian=1)");
  WQ_CHECK(tau > 0.0 && tau < 1.0, WQ_EINVAL, "solve_weights: cutoff must be in (0,1)");
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = P->n_rows;
  wq_weights* w = new wq_weights();
  w->pts = P;
  w->fam_mask = fam_mask;
  wq_status s = WQ_OK;
  // Gauss data
  DBuf G[NFAM], gw;
  const int64_t ng = 16 * P->n_cfn;
  for (int f = 0; f < NFAM && s == WQ_OK; ++f)
    if (f < 3 || (fam_mask & (1u << f)) || (f == 4 && M->dim == 3)) s = dalloc_n<double>(G[f], ng);
  if (s == WQ_OK) s = dalloc_n<double>(gw, 16 * (size_t)P->ncell);
  if (s == WQ_OK)
    s = gauss_basis(M, P, G[0].as<double>(), G[1].as<double>(), G[2].as<double>(), G[4].as<double>(),
                    (fam_mask & WQ_FAM_LAP) ? G[3].as<double>() : nullptr, gw.as<double>(), nullptr, st);
  for (int f = 0; f < NFAM && s == WQ_OK; ++f)
    if (fam_mask & (1u << f)) s = dalloc_n<double>(w->rhs[f], P->nnz);
  if (s == WQ_OK) {
    const int rows_per_block = BS / GQ_GROUP;
    int nfam = 0;
    for (int f = 0; f < NFAM; ++f) nfam += (fam_mask >> f) & 1;
    const size_t lds = (size_t)rows_per_block * (nfam * P->max_row + NFAM * GQ_GROUP) * sizeof(double);
    if (lds > 64 * 1024 &&
        hipFuncSetAttribute((const void*)k_gauss_rows, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
            hipSuccess)
      s = WQ_EDEVICE;
    KTimer tm("k_gauss_rows", n, st);
    if (s == WQ_OK) k_gauss_rows<<<nblocks(n, rows_per_block), BS, lds, st>>>(
        n, P->supp_ptr.as<int64_t>(), P->supp_cell.as<int32_t>(), P->cfn_ptr.as<int64_t>(), P->soff.as<int64_t>(),
        P->slot.as<uint8_t>(), P->kself.as<uint8_t>(), P->row_ptr.as<int64_t>(), G[0].as<double>(),
        G[1].as<double>(), G[2].as<double>(), G[3].as<double>(), G[4].as<double>(), gw.as<double>(), fam_mask,
        P->max_row, w->rhs[0].as<double>(), w->rhs[1].as<double>(), w->rhs[2].as<double>(), w->rhs[3].as<double>(),
        w->rhs[4].as<double>());
    tm.stop();
    if (hipGetLastError() != hipSuccess) s = WQ_EDEVICE;
  }
  // systems by size bucket (order inside a bucket is irrelevant: systems are independent)
  DBuf bkt, lists, stats, dstart, dflops;
  int hist[4 * (NBKT + 1)];
  unsigned long long bflops[NBKT];
  int64_t start[NBKT + 1];
  if (s == WQ_OK) s = dalloc_n<uint8_t>(bkt, n);
  if (s == WQ_OK) s = dalloc(stats, 4 * (NBKT + 1) * sizeof(int));
  if (s == WQ_OK) s = dalloc_n<int64_t>(dstart, NBKT + 1);
  if (s == WQ_OK) s = dalloc(dflops, NBKT * sizeof(unsigned long long));
  if (s == WQ_OK && hipMemsetAsync(stats.p, 0, 4 * (NBKT + 1) * sizeof(int), st) != hipSuccess) s = WQ_EDEVICE;
  if (s == WQ_OK && hipMemsetAsync(dflops.p, 0, NBKT * sizeof(unsigned long long), st) != hipSuccess)
    s = WQ_EDEVICE;
  if (s == WQ_OK) {
    k_sys_bucket<<<nblocks(n, BS), BS, 0, st>>>(n, P->row_ptr.as<int64_t>(), P->qptr.as<int64_t>(),
                                                 bkt.as<uint8_t>(), stats.as<int>(), stats.as<int>() + NBKT,
                                                 dflops.as<unsigned long long>());
    if (hipMemcpyAsync(hist, stats.p, 4 * (NBKT + 1) * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(bflops, dflops.p, NBKT * sizeof(unsigned long long), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      s = WQ_EDEVICE;
  }
  if (s == WQ_OK && hist[NBKT]) {
    set_error("solve_weights: a weight system exceeds n = 128 constraints or r = 256 points");
    s = WQ_EINVAL;
  }
  if (s == WQ_OK) {
    start[0] = 0;
    for (int b = 0; b < NBKT; ++b) start[b + 1] = start[b] + hist[b];
    s = dalloc_n<int32_t>(lists, n);
  }
  if (s == WQ_OK && hipMemcpyAsync(dstart.p, start, (NBKT + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st) !=
                        hipSuccess)
    s = WQ_EDEVICE;
  if (s == WQ_OK) {
    k_sys_scatter<<<nblocks(n, BS), BS, 0, st>>>(n, bkt.as<uint8_t>(), dstart.as<int64_t>(),
                                                  stats.as<int>() + NBKT + 1, lists.as<int32_t>());
    if (hipGetLastError() != hipSuccess) s = WQ_EDEVICE;
  }
  // report accumulators
  struct Rep {
    int fail, max_sweeps;
    unsigned long long min_kept, max_dropped, truncated, certified;
  };
  DBuf drep;
  if (s == WQ_OK) s = dalloc(drep, sizeof(Rep));
  if (s == WQ_OK) {
    Rep init{0, 0, 0x7ff0000000000000ULL /* +inf */, 0ULL, 0ULL, 0ULL};
    if (hipMemcpyAsync(drep.p, &init, sizeof(Rep), hipMemcpyHostToDevice, st) != hipSuccess) s = WQ_EDEVICE;
  }
  // one launch per size bucket covers every family asked for (more workgroups per launch,
  // fewer partly idle tails)
  int nfam = 0;
  unsigned direct_mask = 0;  // family slots whose systems try the SVD kernel's direct proof
  const double* famD[NFAM] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  const double* famR[NFAM] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  double* famW[NFAM] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  for (int f = 0; f < NFAM && s == WQ_OK; ++f) {
    if (!(fam_mask & (1u << f))) continue;
    s = dalloc_n<double>(w->W[f], (size_t)(P->qidx.bytes / sizeof(int32_t)));
    famD[nfam] = f == 0 ? P->DN.as<double>() : f == 1 ? P->DX.as<double>() : f == 2 ? P->DY.as<double>()
                 : f == 3 ? P->DL.as<double>() : P->DZ.as<double>();
    famR[nfam] = w->rhs[f].as<double>();
    famW[nfam] = w->W[f].as<double>();
    if (f == 0) direct_mask |= 1u << nfam;  // the mass family: full rank but for exceptions
    ++nfam;
  }
  // common kernel arguments
  TsvdArgs base{};
  base.nfam = nfam;
  base.tau = tau;
  base.sptr = P->supp_ptr.as<int64_t>();
  base.scell = P->supp_cell.as<int32_t>();
  base.cfn_ptr = P->cfn_ptr.as<int64_t>();
  base.cell_pt_off = P->cell_pt_off.as<int64_t>();
  base.dptr = P->dptr.as<int64_t>();
  base.soff = P->soff.as<int64_t>();
  base.slot = P->slot.as<uint8_t>();
  base.kself = P->kself.as<uint8_t>();
  base.row_ptr = P->row_ptr.as<int64_t>();
  base.qptr = P->qptr.as<int64_t>();
  for (int q = 0; q < NFAM; ++q) {
    base.D[q] = famD[q];
    base.rhs[q] = famR[q];
    base.W[q] = famW[q];
  }
  base.DN = P->DN.as<double>();
  base.direct_mask = direct_mask;
  // systems the SVD kernel's direct proof or the one-wave solver's proof does not cover,
  // per bucket (solved in a second launch)
  int32_t* fb_lists = nullptr;
  int* fb_counts = nullptr;
  if (s == WQ_OK) {
    Rep* R = drep.as<Rep>();
    base.max_sweeps = &R->max_sweeps;
    base.min_kept = &R->min_kept;
    base.max_dropped = &R->max_dropped;
    base.truncated = &R->truncated;
    base.certified = &R->certified;
    base.fail = &R->fail;
  }
  // The SVD kernel for the systems of bucket b (all of them, or the `grid` listed in sel).
  auto svd_launch = [&](int b, const int32_t* sel, int64_t grid, int64_t flops, hipStream_t ls) -> wq_status {
    const int64_t ns = hist[b];
    const int mn = hist[2 * (NBKT + 1) + 2 * b];      // largest n in the bucket
    const int mr = hist[2 * (NBKT + 1) + 2 * b + 1];  // largest r in the bucket
    // column stride: 8 (mod 32) doubles (consecutive columns start 16 banks apart) unless
    // a shorter stride fits more workgroups of the bucket on a CU (160 KiB of LDS,
    // allocated in 512-byte granules); then the longest stride with the most workgroups
    int ld = ((mr + 1 + 23) / 32) * 32 + 8;
    if (ld < mr + 1) ld += 32;
    auto lds_of = [&](int l) {
      return ((size_t)mn * l + (size_t)mr + 5 * (size_t)mn + 96) * sizeof(double) +
             (4 * (size_t)mn + 1 + 2 * (size_t)mr) * sizeof(int);
    };
    // (the kernels also hold 256 bytes of static LDS; the launch checks the exact figure)
    auto per_cu = [&](int l) { return (int)((160 * 1024) / ((lds_of(l) + 256 + 511) / 512 * 512)); };
    for (int l = ld - 1, best = per_cu(ld); l >= mr + 1; --l)
      if (per_cu(l) > best) {
        best = per_cu(l);
        ld = l;
      }
    // M = R1^T columns: stride = 8 (mod 16) doubles, at most ld, at least mn rounded up
    // to the 8 lanes of a Jacobi pair (those rows are zero-padded). For 48 < n <= 64 this
    // covers all EPJ rows of a lane of the instance chosen below (no per-row checks).
    // n > 64: a 512-thread instance (8 lanes per pair) where two workgroups fit on a CU
    // (n <= 96, r <= 128), else the 1024-thread one (16 lanes per pair)
    // The thread count and the lanes per pair or column set the summation orders, so they
    // follow from the bucket's bounds alone: a system gets the same bits whatever else is
    // in the bucket (a mesh alone or in a batch). Only strides and per-lane slot counts,
    // which do not change the arithmetic, follow the bucket's actual maxima.
    //  - 64 < n <= 96, r <= 128: 512 threads, 8 lanes per pair (two workgroups per CU fit
    //    where the 1024-thread instance's registers allow one);
    //  - 48 < n <= 64, 80 < r <= 128: 512 threads, 16 lanes per pair and per column (these
    //    buckets hold two or three workgroups per CU by LDS: twice the resident waves);
    //  - other n > 64: 1024 threads, 16 lanes (6 rows of M per lane up to n = 96, so that
    //    no lane runs zero rows through the rotations, 8 above); other n <= 64: 256
    //    threads, 8 lanes.
    const int bn = b / NB_R, br = b % NB_R;
    const bool w512 = bn == 4 && br <= 3;                          // 64 < n <= 96, r <= 128
    const bool m512 = (bn == 2 || bn == 3) && br >= 2 && br <= 3;  // 48 < n <= 64, 80 < r <= 128
    const bool wide = bn >= 4;                                     // n > 64
    const int lpp = ((wide && !w512) || m512) ? 16 : 8;  // lanes per column pair of the instance
    int ldm = ((mn + 8) / 16) * 16 + 8;
    if (ldm < (mn + lpp - 1) / lpp * lpp) ldm += 16;
    if (ldm > ld) ldm = (mn + lpp - 1) / lpp * lpp;
    if (ldm > ld) ld = ldm;
    const size_t lds = lds_of(ld);
    if (lds + 256 > 160 * 1024) {
      set_error("solve_weights: a weight system (n=" + std::to_string(mn) + ", r=" + std::to_string(mr) +
                ") does not fit in LDS");
      return WQ_EINVAL;
    }
    TsvdArgs ta = base;
    ta.rows = lists.as<int32_t>() + start[b];
    ta.nsys = ns;
    ta.ld = ld;
    ta.ldm = ldm;
    ta.sel = sel;
    if (!sel && direct_mask) {
      ta.fb_list = fb_lists + start[b] * nfam;
      ta.fb_count = fb_counts + b;
    }
    // 8 lanes per column pair; systems with more than 64 constraints (more than 32
    // pairs) take 1024 threads with 16 lanes per column pair (more waves per CU to hide
    // latency: such systems fill most of a CU's LDS on their own).
    const void* fn = nullptr;
    const char* kname = nullptr;  // timing record: the kernel instance
    int nt = 0;
    {
      // EPR: register elements per lane of a column of A^T (r), EPJ: of M (n)
      const int epr = (mr + 7) / 8;
      nt = !wide ? (m512 ? 512 : 256) : w512 ? 512 : 1024;
      const bool j7 = bn == 2;  // 48 < n <= 56: 7 rows of M per lane
      if (m512) fn = (const void*)k_tsvd2<16, 8, 4, 512>, kname = "k_tsvd2<16,8,4,512>";
      else if (!wide && epr <= 8 && j7) fn = (const void*)k_tsvd2<8, 8, 7, 256>, kname = "k_tsvd2<8,8,7,256>";
      else if (!wide && epr <= 16 && j7) fn = (const void*)k_tsvd2<8, 16, 7, 256>, kname = "k_tsvd2<8,16,7,256>";
      else if (!wide && epr <= 8) fn = (const void*)k_tsvd2<8, 8, 8, 256>, kname = "k_tsvd2<8,8,8,256>";
      else if (!wide && epr <= 16) fn = (const void*)k_tsvd2<8, 16, 8, 256>, kname = "k_tsvd2<8,16,8,256>";
      else if (!wide) fn = (const void*)k_tsvd2<8, 32, 8, 256>, kname = "k_tsvd2<8,32,8,256>";
      else if (w512) fn = (const void*)k_tsvd2<8, 16, 12, 512>, kname = "k_tsvd2<8,16,12,512>";
      else if (bn == 4) fn = (const void*)k_tsvd2<16, 16, 6, 1024>, kname = "k_tsvd2<16,16,6,1024>";
      else fn = (const void*)k_tsvd2<16, 16, 8, 1024>, kname = "k_tsvd2<16,16,8,1024>";
    }
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, fn) != hipSuccess || fa.sharedSizeBytes + lds > 160 * 1024) {
      set_error("solve_weights: a weight system (n=" + std::to_string(mn) + ", r=" + std::to_string(mr) +
                ") does not fit in LDS");
      return WQ_EINVAL;
    }
    if (lds > 64 * 1024 &&
        hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) {
      set_error("solve_weights: cannot raise the LDS limit of the TSVD kernel");
      return WQ_EDEVICE;
    }
    KTimer tm(kname, flops, ls);
    void* args[] = {&ta};
    wq_status res = WQ_OK;
    if (hipLaunchKernel(fn, dim3((unsigned)grid), dim3(nt), args, lds, ls) != hipSuccess) {
      set_error("solve_weights: TSVD launch failed");
      res = WQ_EDEVICE;
    }
    tm.stop();
    return res;
  };
  // Systems of at most 64 constraints and 64 points go to the one-wave solver first; the
  // ones its rank proof does not cover are listed and solved by the SVD kernel of their
  // bucket afterwards (one synchronisation to read the list lengths). (Several waves per
  // system, for more points or constraints, lost to the SVD kernel's certified path once
  // its second factorisation was Householder: their barriers cost more than they save.)
  DBuf fbl, fbc;
  int fbn[NBKT];
  bool any_w = false;
  if (s == WQ_OK) s = dalloc_n<int32_t>(fbl, (size_t)n * nfam);
  if (s == WQ_OK) s = dalloc_n<int>(fbc, NBKT);
  if (s == WQ_OK && hipMemsetAsync(fbc.p, 0, NBKT * sizeof(int), st) != hipSuccess) s = WQ_EDEVICE;
  fb_lists = fbl.as<int32_t>();
  fb_counts = fbc.as<int>();
  // the buckets' launches are independent (each system's weights are written by one
  // workgroup; the reports and the second-launch lists are updated atomically)
  Fork fk(st);
  if (s == WQ_OK && !fk.fork()) s = WQ_EDEVICE;
  for (int b = 0; b < NBKT && s == WQ_OK; ++b) {
    const int64_t ns = hist[b];
    if (ns == 0) continue;
    const int bn = b / NB_R, br = b % NB_R;
    if (bn <= 3 && br == 0) {  // n <= 64, r <= 64
      TsvdArgs ta = base;
      ta.rows = lists.as<int32_t>() + start[b];
      ta.nsys = ns;
      ta.fb_list = fbl.as<int32_t>() + start[b] * nfam;
      ta.fb_count = fbc.as<int>() + b;
      // dynamic LDS: R11 of the bucket's largest system (more workgroups per CU for the
      // smaller buckets; the layout, and so the arithmetic, does not depend on it)
      const int mn = hist[2 * (NBKT + 1) + 2 * b];
      ta.rp_n = mn;
      const size_t lds = (size_t)mn * (mn - 1) / 2 * sizeof(double);
      // the mass family's slot (slot 0) through the direct instance, the others pivoted
      const int nd = (direct_mask & 1u) ? 1 : 0;
      if (nd) {
        ta.fam_base = 0;
        const hipStream_t ls = fk.lane();
        KTimer tm("k_wsolve_direct", (int64_t)bflops[b], ls);
        k_wsolve<true><<<dim3((unsigned)ns), dim3(64), lds, ls>>>(ta);
        tm.stop();
      }
      if (nfam > nd) {
        ta.fam_base = nd;
        const hipStream_t ls = fk.lane();
        KTimer tm("k_wsolve", (int64_t)bflops[b] * (nfam - nd), ls);
        k_wsolve<false><<<dim3((unsigned)(ns * (nfam - nd))), dim3(64), lds, ls>>>(ta);
        tm.stop();
      }
      if (hipGetLastError() != hipSuccess) {
        set_error("solve_weights: one-wave solver launch failed");
        s = WQ_EDEVICE;
      }
      any_w = true;
    } else {
      s = svd_launch(b, nullptr, ns * nfam, (int64_t)bflops[b] * nfam, fk.lane());
      any_w = any_w || direct_mask != 0;
    }
  }
  if (!fk.join() && s == WQ_OK) s = WQ_EDEVICE;
  if (s == WQ_OK && any_w) {
    if (hipMemcpyAsync(fbn, fbc.p, NBKT * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      s = WQ_EDEVICE;
    if (s == WQ_OK && !fk.fork()) s = WQ_EDEVICE;
    for (int b = 0; b < NBKT && s == WQ_OK; ++b)
      if (hist[b] && fbn[b] > 0) s = svd_launch(b, fbl.as<int32_t>() + start[b] * nfam, fbn[b], 0, fk.lane());
    if (!fk.join() && s == WQ_OK) s = WQ_EDEVICE;
  }
  dfree(fbl);
  dfree(fbc);
  Rep hrep{};
  if (s == WQ_OK && hipMemcpyAsync(&hrep, drep.p, sizeof(Rep), hipMemcpyDeviceToHost, st) != hipSuccess)
    s = WQ_EDEVICE;
  if (s == WQ_OK && hipStreamSynchronize(st) != hipSuccess) s = WQ_EDEVICE;
  {
    DBuf* tmp[] = {&G[0], &G[1], &G[2], &G[3], &G[4], &gw, &bkt, &lists, &stats, &dstart, &dflops, &drep};
    static_assert(NFAM == 5, "temporaries of solve_weights");
    dfree_many(tmp, sizeof(tmp) / sizeof(tmp[0]));
  }
  if (s == WQ_OK && (hrep.fail & 2)) {
    set_error("solve_weights: internal LDS sizing error (column stride)");
    s = WQ_EDEVICE;
  } else if (s == WQ_OK && hrep.fail) {
    set_error("solve_weights: a Jacobi SVD did not converge in 40 sweeps");
    s = WQ_ESVD;
  }
  if (s != WQ_OK) {
    release_weights(w);
    delete w;
    return s;
  }
  if (rep) {
    int nf = 0;
    for (int f = 0; f < NFAM; ++f) nf += (fam_mask >> f) & 1;
    rep->systems = n * nf;
    rep->truncated = (int64_t)hrep.truncated;
    rep->certified = (int64_t)hrep.certified;
    rep->max_sweeps = hrep.max_sweeps;
    double v;
    std::memcpy(&v, &hrep.min_kept, 8);
    rep->min_kept_ratio = v;
    std::memcpy(&v, &hrep.max_dropped, 8);
    rep->max_dropped_ratio = v;
  }
  *out = w;
  return WQ_OK;
}

extern "C" void wq_weights_destroy(wq_weights* w) {
  if (!w) return;
  release_weights(w);
  delete w;
}

extern "C" wq_status wq_weights_get(const wq_weights* w, wq_family fam, double* dst, wq_stream stream) {
  WQ_CHECK(w && dst, WQ_EINVAL, "wq_weights_get: null argument");
  const int f = fam_index(fam);
  WQ_CHECK(w->fam_mask & fam, WQ_EINVAL, "wq_weights_get: family not solved");
  WQ_HIP(hipMemcpyAsync(dst, w->W[f].p, w->W[f].bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return WQ_OK;
}

extern "C" wq_status wq_rhs_get(const wq_weights* w, wq_family fam, double* dst, wq_stream stream) {
  WQ_CHECK(w && dst, WQ_EINVAL, "wq_rhs_get: null argument");
  const int f = fam_index(fam);
  WQ_CHECK(w->fam_mask & fam, WQ_EINVAL, "wq_rhs_get: family not solved");
  WQ_HIP(hipMemcpyAsync(dst, w->rhs[f].p, (size_t)w->pts->nnz * sizeof(double), hipMemcpyDeviceToDevice,
                        (hipStream_t)stream));
  return WQ_OK;
}
