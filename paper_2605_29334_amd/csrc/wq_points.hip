// build_points: element classification (Section 3, Table 2, Eq. (18)), Bezier cells,
// supports, the CSR pattern of Eq. (10), point sets Q_i, scatter slots, and basis /
// geometry at the WQ points (Section 4.1; planar Eqs. (13)-(17)).
#include "wq_internal.h"

#include <algorithm>
#include <climits>
#include <cmath>

using namespace wq;

namespace {

constexpr int BS = 256;
constexpr int MAX_VF = 16;      // faces around a vertex
constexpr int MAX_SUPP = 64;    // cells in the support of one function
constexpr int MAX_ROW = 255;    // entries of one CSR row (slots are bytes)

// ------------------------------------------------------------------ topology
__global__ void k_vf_count(const int32_t* fv, int32_t nf, int64_t* cnt) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= 4LL * nf) return;
  atomicAdd((unsigned long long*)&cnt[fv[t]], 1ULL);
}

__global__ void k_vf_fill(const int32_t* fv, int32_t nf, const int64_t* ptr, int64_t* cur, int32_t* idx) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= 4LL * nf) return;
  int32_t v = fv[t];
  int64_t k = (int64_t)atomicAdd((unsigned long long*)&cur[v], 1ULL);
  idx[ptr[v] + k] = (int32_t)(t / 4);
}

// sorts a short int32 list in place (insertion sort)
__device__ inline void small_sort(int32_t* a, int n) {
  for (int i = 1; i < n; ++i) {
    int32_t x = a[i];
    int j = i - 1;
    while (j >= 0 && a[j] > x) {
      a[j + 1] = a[j];
      --j;
    }
    a[j + 1] = x;
  }
}

__global__ void k_sort_lists(const int64_t* ptr, int64_t n, int32_t* idx) {
  int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  small_sort(idx + ptr[v], (int)(ptr[v + 1] - ptr[v]));
}

// a directed edge a->b of some face has a twin b->a iff some face around b contains it
__global__ void k_boundary(const int32_t* fv, int32_t nf, const int64_t* vptr, const int32_t* vidx,
                           uint8_t* bnd) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= 4LL * nf) return;
  const int64_t f = t / 4;
  const int k = (int)(t % 4);
  const int32_t a = fv[4 * f + k], b = fv[4 * f + (k + 1) % 4];
  bool twin = false;
  for (int64_t p = vptr[b]; p < vptr[b + 1]; ++p) {
    const int32_t g = vidx[p];
    for (int j = 0; j < 4; ++j)
      if (fv[4 * g + j] == b && fv[4 * g + (j + 1) % 4] == a) twin = true;
  }
  if (!twin) {
    bnd[a] = 1;
    bnd[b] = 1;
  }
}

// valence = edges at v = faces around v (+1 on the boundary); EP per Section 3
__global__ void k_vertex_flags(int32_t nv, const int64_t* vptr, const uint8_t* bnd, int32_t* val, uint8_t* ep) {
  int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const int nfa = (int)(vptr[v + 1] - vptr[v]);
  const int va = nfa + (bnd[v] ? 1 : 0);
  val[v] = va;
  ep[v] = (nfa > 0) && ((!bnd[v] && va != 4) || (bnd[v] && va > 3));
}

__global__ void k_face_flags1(const int32_t* fv, int32_t nf, const uint8_t* bnd, const uint8_t* ep,
                              uint8_t* passive, uint8_t* enriched) {
  int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= nf) return;
  bool pb = false, ir = false;
  for (int k = 0; k < 4; ++k) {
    pb |= bnd[fv[4 * f + k]] != 0;
    ir |= ep[fv[4 * f + k]] != 0;
  }
  passive[f] = pb;            // 1-ring neighbourhood of the boundary
  enriched[f] = (!pb) && ir;  // initial mesh: enriched = irregular
}

__global__ void k_vertex_flags2(int32_t nv, const int64_t* vptr, const int32_t* vidx, const uint8_t* passive,
                                const uint8_t* enriched, uint8_t* pvtx, uint8_t* tpoint) {
  int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= nv) return;
  bool anyp = false, anye = false, anyn = false;
  for (int64_t p = vptr[v]; p < vptr[v + 1]; ++p) {
    const int32_t g = vidx[p];
    anyp |= passive[g] != 0;
    if (enriched[g]) anye = true; else anyn = true;
  }
  pvtx[v] = anyp;
  tpoint[v] = anye && anyn;  // shared by an enriched and a non-enriched element
}

__global__ void k_classify(const int32_t* fv, int32_t nf, const int64_t* vptr, const int32_t* vidx,
                           const int32_t* val, const uint8_t* ep, const uint8_t* passive, const uint8_t* enriched,
                           const uint8_t* pvtx, const uint8_t* tpoint, uint8_t* etype, uint8_t* s) {
  int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= nf) return;
  if (passive[f]) {
    etype[f] = ET_PASSIVE;
    s[f] = 0;
    return;
  }
  bool b2 = false, tr = false;
  for (int k = 0; k < 4; ++k) {
    b2 |= pvtx[fv[4 * f + k]] != 0;  // 2nd ring of the boundary
    tr |= tpoint[fv[4 * f + k]] != 0;
  }
  const bool ir = enriched[f] != 0;
  int sv = 2;  // regular: 2x2
  uint8_t et = ET_REGULAR;
  if (ir) {
    et = ET_IRREGULAR;
  } else if (tr) {
    et = ET_TRANSITION;
  } else if (b2) {
    et = ET_BOUNDARY;
  }
  if (ir) sv = max(sv, 4);               // irregular: 4x4
  if (b2) sv = max(sv, 4);               // boundary: 4x4
  if (tr && ir) sv = max(sv, 4);         // enriched transition: 4x4
  if (tr && !ir) {                       // non-enriched transition: 3x3 or 4x4
    int32_t eps[MAX_VF * 4];
    int ne = 0;
    bool high = false;
    for (int k = 0; k < 4; ++k) {
      const int32_t v = fv[4 * f + k];
      if (!tpoint[v]) continue;
      for (int64_t p = vptr[v]; p < vptr[v + 1]; ++p) {
        const int32_t g = vidx[p];
        if (!enriched[g]) continue;
        for (int j = 0; j < 4; ++j) {
          const int32_t w = fv[4 * g + j];
          if (!ep[w]) continue;
          bool seen = false;
          for (int q = 0; q < ne; ++q) seen |= eps[q] == w;
          if (!seen && ne < MAX_VF * 4) eps[ne++] = w;
          high |= val[w] >= 7;
        }
      }
    }
    sv = max(sv, (ne >= 2 || high) ? 4 : 3);
  }
  etype[f] = et;
  s[f] = (uint8_t)sv;
}

// ------------------------------------------------------------------ cells
__global__ void k_cell_count(int32_t nf, const uint8_t* s, const uint8_t* split, int64_t* cnt, int* bad) {
  int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= nf) return;
  cnt[f] = (s[f] == 0) ? 0 : (split[f] ? 4 : 1);
  if (s[f] && split[f] && (s[f] & 1)) atomicOr(bad, 1);  // split elements need even s
}

__global__ void k_cell_fill(int32_t nf, const uint8_t* s, const uint8_t* split, const int64_t* cptr,
                            int32_t* cell_face, uint8_t* cell_sub, int64_t* npts) {
  int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const int64_t c0 = cptr[f], c1 = cptr[f + 1];
  for (int64_t c = c0; c < c1; ++c) {
    cell_face[c] = (int32_t)f;
    cell_sub[c] = (uint8_t)(c - c0);
    const int sv = s[f];
    npts[c] = split[f] ? (int64_t)(sv / 2) * (sv / 2) : (int64_t)sv * sv;
  }
}

// functions with a nonzero Bernstein coefficient on the cell
__global__ void k_cfn_count(int32_t ncell, const int32_t* cell_face, const uint8_t* cell_sub, const int64_t* ext_ptr,
                            const int64_t* coef_ptr, const double* coef, int64_t* cnt) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int32_t f = cell_face[c];
  const int m = (int)(ext_ptr[f + 1] - ext_ptr[f]);
  const double* C = coef + coef_ptr[f] + (int64_t)cell_sub[c] * m * 16;
  int n = 0;
  for (int k = 0; k < m; ++k) {
    bool nz = false;
    for (int q = 0; q < 16; ++q) nz |= C[k * 16 + q] != 0.0;
    n += nz;
  }
  cnt[c] = n;
}

__global__ void k_cfn_fill(int32_t ncell, const int32_t* cell_face, const uint8_t* cell_sub, const int64_t* ext_ptr,
                           const int32_t* ext_fn, const int64_t* coef_ptr, const double* coef, const int64_t* cfn_ptr,
                           int32_t* cfn, uint8_t* cfn_loc) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int32_t f = cell_face[c];
  const int m = (int)(ext_ptr[f + 1] - ext_ptr[f]);
  const double* C = coef + coef_ptr[f] + (int64_t)cell_sub[c] * m * 16;
  int64_t o = cfn_ptr[c];
  for (int k = 0; k < m; ++k) {
    bool nz = false;
    for (int q = 0; q < 16; ++q) nz |= C[k * 16 + q] != 0.0;
    if (nz) {
      cfn[o] = ext_fn[ext_ptr[f] + k];
      cfn_loc[o] = (uint8_t)k;
      ++o;
    }
  }
}

__global__ void k_supp_count(int64_t n_cfn, const int32_t* cfn, int64_t* cnt) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n_cfn) return;
  atomicAdd((unsigned long long*)&cnt[cfn[t]], 1ULL);
}

__global__ void k_supp_fill(int32_t ncell, const int64_t* cfn_ptr, const int32_t* cfn, const int64_t* sptr,
                            int64_t* cur, int32_t* scell) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  for (int64_t t = cfn_ptr[c]; t < cfn_ptr[c + 1]; ++t) {
    const int32_t j = cfn[t];
    const int64_t k = (int64_t)atomicAdd((unsigned long long*)&cur[j], 1ULL);
    scell[sptr[j] + k] = (int32_t)c;
  }
}

// ------------------------------------------------------------------ pattern
// Wave-wide helpers: 64 lanes, the same result in every lane.
__device__ inline int32_t wave_min_i32(int32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ inline int wave_sum_i32(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// k-way merge of the ascending function lists of the cells in supp(N_i): S_i. One wave
// per row: lane k holds the head of the list of support cell k (np <= 64 cells); each
// round takes the smallest head (a wave minimum), lane 0 writes it, and the lanes holding
// it advance. Returns |S_i| in every lane.
__device__ int wave_merge_row(int64_t p0, int np, const int32_t* scell, const int64_t* cfn_ptr, const int32_t* cfn,
                              int32_t* out, int lane) {
  int64_t pos = 0, end = 0;
  if (lane < np) {
    const int32_t c = scell[p0 + lane];
    pos = cfn_ptr[c];
    end = cfn_ptr[c + 1];
  }
  int count = 0;
  while (true) {
    const int32_t head = pos < end ? cfn[pos] : INT_MAX;
    const int32_t best = wave_min_i32(head);
    if (best == INT_MAX) break;
    if (out && lane == 0) out[count] = best;
    ++count;
    if (head == best) ++pos;
  }
  return count;
}

// Row sizes: |S_i| and the point count of the row. One wave per row, the waves striding
// over the rows; each wave keeps its maxima and updates the global ones once at the end
// (one atomic per row on the same address would serialise).
__global__ void k_row_count(int64_t n, const int64_t* sptr, const int32_t* scell, const int64_t* cfn_ptr,
                            const int32_t* cfn, const int64_t* cell_pt_off, int64_t* ncnt, int64_t* rcnt,
                            int* err, int* wp_bad, int* maxrow, int* maxr) {
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  int mrow = 0, mr = 0;
  for (int64_t i = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); i < n; i += nwaves) {
    const int64_t p0 = sptr[i];
    const int np = (int)(sptr[i + 1] - p0);
    if (np > MAX_SUPP || np == 0) {
      if (lane == 0) {
        atomicOr(err, np == 0 ? 2 : 1);
        ncnt[i] = 0;
        rcnt[i] = 0;
      }
      continue;
    }
    const int ni = wave_merge_row(p0, np, scell, cfn_ptr, cfn, nullptr, lane);
    int rl = 0;
    if (lane < np) {
      const int32_t c = scell[p0 + lane];
      rl = (int)(cell_pt_off[c + 1] - cell_pt_off[c]);
    }
    const int r = wave_sum_i32(rl);
    if (lane == 0) {
      ncnt[i] = ni;
      rcnt[i] = r;
      if (ni > MAX_ROW) atomicOr(err, 4);
      if (r < ni) atomicAdd(wp_bad, 1);
    }
    mrow = max(mrow, ni);
    mr = max(mr, r);
  }
  if (lane == 0) {
    atomicMax(maxrow, mrow);
    atomicMax(maxr, mr);
  }
}

// S_i into col and the row's points (support cells in order) into qidx; one wave per row.
__global__ void k_row_fill(int64_t n, const int64_t* sptr, const int32_t* scell, const int64_t* cfn_ptr,
                           const int32_t* cfn, const int64_t* cell_pt_off, const int64_t* row_ptr, const int64_t* qptr,
                           int32_t* col, int32_t* qidx) {
  const int lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= n) return;
  const int64_t p0 = sptr[i];
  const int np = (int)(sptr[i + 1] - p0);
  wave_merge_row(p0, np, scell, cfn_ptr, cfn, col + row_ptr[i], lane);
  int64_t o = qptr[i];
  for (int k = 0; k < np; ++k) {
    const int32_t c = scell[p0 + k];
    const int64_t q0 = cell_pt_off[c], nq = cell_pt_off[c + 1] - q0;
    for (int64_t q = lane; q < nq; q += 64) qidx[o + q] = (int32_t)(q0 + q);
    o += nq;
  }
}

__global__ void k_pair_m(int64_t npairs, const int32_t* scell, const int64_t* cfn_ptr, int64_t* m) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const int32_t c = scell[p];
  m[p] = (cfn_ptr[c + 1] - cfn_ptr[c] + 3) & ~int64_t(3);  // padded: slot maps start 4-byte aligned
}

// slot of every cell function in row i (position in S_i) and of N_i itself in the cell;
// one wave per row, a lane per cell function (binary search in S_i)
__global__ void k_slots(int64_t n, const int64_t* sptr, const int32_t* scell, const int64_t* cfn_ptr,
                        const int32_t* cfn, const int64_t* row_ptr, const int32_t* col, const int64_t* soff,
                        uint8_t* slot, uint8_t* kself) {
  const int lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= n) return;
  const int32_t* row = col + row_ptr[i];
  const int ni = (int)(row_ptr[i + 1] - row_ptr[i]);
  for (int64_t p = sptr[i]; p < sptr[i + 1]; ++p) {
    const int32_t c = scell[p];
    const int64_t f0 = cfn_ptr[c];
    const int m = (int)(cfn_ptr[c + 1] - f0);
    for (int k = lane; k < m; k += 64) {
      const int32_t j = cfn[f0 + k];
      int lo = 0, hi = ni - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (row[mid] < j) lo = mid + 1; else hi = mid;
      }
      slot[soff[p] + k] = (uint8_t)lo;
      if (j == (int32_t)i) kself[p] = (uint8_t)k;
    }
  }
}

// ------------------------------------------------------------------ basis at points
__global__ void k_cell_np_m(int32_t ncell, const int64_t* cell_pt_off, const int64_t* cfn_ptr, int64_t* out,
                            int* maxm, int* maxnp) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int64_t np = cell_pt_off[c + 1] - cell_pt_off[c];
  const int64_t m = cfn_ptr[c + 1] - cfn_ptr[c];
  out[c] = np * m;
  atomicMax(maxm, (int)m);
  atomicMax(maxnp, (int)np);
}

// cell-local coordinate of local point lp of cell c (see build_points in wq.h)
__device__ inline void point_eta(int sv, bool split, int sub, int lp, double* e1, double* e2) {
  if (!split) {
    const int a = lp % sv, b = lp / sv;
    *e1 = (2.0 * a + 1.0) / (2.0 * sv);
    *e2 = (2.0 * b + 1.0) / (2.0 * sv);
  } else {
    const int sd = sv / 2, sx = sub & 1, sy = sub >> 1;
    const int a = sx * sd + lp % sd, b = sy * sd + lp / sd;
    *e1 = 2.0 * ((2.0 * a + 1.0) / (2.0 * sv)) - sx;
    *e2 = 2.0 * ((2.0 * b + 1.0) / (2.0 * sv)) - sy;
  }
}

// N, dN/deta1, dN/deta2, d2N/deta1^2, d2N/deta1deta2, d2N/deta2^2 of one function
__device__ inline void eval_fn(const double* C, const double b1[4], const double d1[4], const double s1[4],
                               const double b2[4], const double d2[4], const double s2[4], double out[6]) {
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int l = 0; l < 4; ++l) {
    double r0 = 0, r1 = 0, r2 = 0;  // sum_k C b_k, C d_k, C s_k
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

// One thread per point: geometry (x, J, Hessian of x) then the cell functions' values,
// physical gradients (J^{-T} grad_eta) and Laplacians (chain rule).
__global__ void k_basis(int64_t npts_total, int32_t ncell, const int64_t* cell_pt_off, const int32_t* cell_face,
                        const uint8_t* cell_sub, const uint8_t* s, const uint8_t* split, const int64_t* ext_ptr,
                        const int64_t* coef_ptr, const double* coef, const double* ctrl, const int64_t* cfn_ptr,
                        const int32_t* cfn, const uint8_t* cfn_loc, const int64_t* dptr, double* X, double* DJ,
                        double* DN, double* DX, double* DY, double* DZ, double* DL, int dim, int* bad_jac) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= npts_total) return;
  int lo = 0, hi = ncell - 1;  // cell holding point p
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cell_pt_off[mid] <= p) lo = mid; else hi = mid - 1;
  }
  const int c = lo;
  const int32_t f = cell_face[c];
  const int sub = cell_sub[c];
  const bool sp = split[f] != 0;
  const int lp = (int)(p - cell_pt_off[c]);
  double e1, e2;
  point_eta(s[f], sp, sub, lp, &e1, &e2);
  double b1[4], d1[4], s1[4], b2[4], d2[4], s2[4];
  bern3(e1, b1, d1, s1);
  bern3(e2, b2, d2, s2);
  const int mf = (int)(ext_ptr[f + 1] - ext_ptr[f]);
  const double* Cf = coef + coef_ptr[f] + (int64_t)sub * mf * 16;
  const int64_t f0 = cfn_ptr[c];
  const int m = (int)(cfn_ptr[c + 1] - f0);
  if (dim == 3) {  // a surface: tangent vectors, metric, surface gradient, Laplace-Beltrami
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
    const SurfGeom G = surf_geom(A, X2);
    for (int a = 0; a < 3; ++a) X[3 * p + a] = x3[a];
    DJ[p] = G.sg;
    if (!(G.sg > 0.0)) atomicOr(bad_jac, 1);
    const int64_t o = dptr[c] + (int64_t)lp * m;
    for (int k = 0; k < m; ++k) {
      double v[6], gr[3], lb;
      eval_fn(Cf + 16 * (int)cfn_loc[f0 + k], b1, d1, s1, b2, d2, s2, v);
      surf_basis(G, v, gr, &lb);
      DN[o + k] = v[0];
      DX[o + k] = gr[0];
      DY[o + k] = gr[1];
      DZ[o + k] = gr[2];
      if (DL) DL[o + k] = lb;
    }
    return;
  }
  // geometry: x = sum P_j N_j, J = dx/deta, H_eta x
  double x[2] = {0, 0}, J[2][2] = {{0, 0}, {0, 0}}, H[2][3] = {{0, 0, 0}, {0, 0, 0}};
  for (int k = 0; k < m; ++k) {
    double v[6];
    eval_fn(Cf + 16 * (int)cfn_loc[f0 + k], b1, d1, s1, b2, d2, s2, v);
    const int32_t j = cfn[f0 + k];
    for (int a = 0; a < 2; ++a) {
      const double P = ctrl[2 * (int64_t)j + a];
      x[a] += P * v[0];
      J[a][0] += P * v[1];
      J[a][1] += P * v[2];
      H[a][0] += P * v[3];
      H[a][1] += P * v[4];
      H[a][2] += P * v[5];
    }
  }
  const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  X[2 * p] = x[0];
  X[2 * p + 1] = x[1];
  DJ[p] = det;
  if (!(det > 0.0)) atomicOr(bad_jac, 1);
  // J^{-1}
  const double id = 1.0 / det;
  const double Ji[2][2] = {{J[1][1] * id, -J[0][1] * id}, {-J[1][0] * id, J[0][0] * id}};
  // G = J^{-1} J^{-T}
  const double G00 = Ji[0][0] * Ji[0][0] + Ji[0][1] * Ji[0][1];
  const double G01 = Ji[0][0] * Ji[1][0] + Ji[0][1] * Ji[1][1];
  const double G11 = Ji[1][0] * Ji[1][0] + Ji[1][1] * Ji[1][1];
  const int64_t o = dptr[c] + (int64_t)lp * m;
  for (int k = 0; k < m; ++k) {
    double v[6];
    eval_fn(Cf + 16 * (int)cfn_loc[f0 + k], b1, d1, s1, b2, d2, s2, v);
    // grad_x N = J^{-T} grad_eta N
    const double nx = Ji[0][0] * v[1] + Ji[1][0] * v[2];
    const double ny = Ji[0][1] * v[1] + Ji[1][1] * v[2];
    DN[o + k] = v[0];
    DX[o + k] = nx;
    DY[o + k] = ny;
    if (DL) {
      const double h00 = v[3] - nx * H[0][0] - ny * H[1][0];
      const double h01 = v[4] - nx * H[0][1] - ny * H[1][1];
      const double h11 = v[5] - nx * H[0][2] - ny * H[1][2];
      DL[o + k] = h00 * G00 + 2.0 * h01 * G01 + h11 * G11;
    }
  }
}

// ------------------------------------------------------------------ assembly tiles
// Weight offset of every (row, cell) pair: qptr[i] + points of the earlier cells of row i.
__global__ void k_pair_qoff(int64_t n, const int64_t* sptr, const int32_t* scell, const int64_t* cell_pt_off,
                            const int64_t* qptr, int64_t* qoff) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t o = qptr[i];
  for (int64_t p = sptr[i]; p < sptr[i + 1]; ++p) {
    qoff[p] = o;
    const int32_t c = scell[p];
    o += cell_pt_off[c + 1] - cell_pt_off[c];
  }
}

// Merge of the (ascending) cell lists of the rows of one tile; one wave per tile, lane r
// holding the head of row r's list. fill == false: count the distinct cells; fill ==
// true: write one entry per cell and its member records (in row order).
template <bool FILL>
__global__ void k_tile_entries(int64_t n, const int64_t* sptr, const int32_t* scell, const int64_t* cfn_ptr,
                               const int64_t* cell_pt_off, const int64_t* dptr, const int64_t* qoff,
                               const int64_t* soff, const int64_t* row_ptr, int64_t* eptr, int4* ent, int2* mem,
                               int* maxnnz, int* overflow) {
  const int lane = threadIdx.x & 63;
  const int64_t n_tiles = (n + TILE_ROWS - 1) / TILE_ROWS;
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  // maxima of this wave's tiles (counting pass): nnz, -, members, entries, basis block,
  // member weights; the global ones are updated once at the end
  int mx[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t tile = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); tile < n_tiles;
       tile += nwaves) {
    const int64_t i0 = tile * TILE_ROWS;
    const int nr = (int)min((int64_t)TILE_ROWS, n - i0);
    int64_t pos = 0, end = 0;
    if (lane < nr) {
      pos = sptr[i0 + lane];
      end = sptr[i0 + lane + 1];
    }
    if (!FILL) {
      mx[0] = max(mx[0], (int)(row_ptr[i0 + nr] - row_ptr[i0]));
      mx[2] = max(mx[2], (int)(sptr[i0 + nr] - sptr[i0]));  // members of the tile
    }
    int64_t e = FILL ? eptr[tile] : 0;
    int64_t mb = FILL ? sptr[i0] : 0;  // members are stored in (entry, row) order
    int count = 0;
    while (true) {
      const int32_t head = pos < end ? scell[pos] : INT_MAX;
      const int32_t best = wave_min_i32(head);
      if (best == INT_MAX) break;
      const bool member = head == best;
      const unsigned long long bal = __ballot(member);
      const unsigned mask = (unsigned)bal;  // rows of the tile (nr <= 8 lanes)
      const int nm = __popcll(bal);
      const int rank = __popcll(bal & ((1ULL << lane) - 1ULL));
      const int np = (int)(cell_pt_off[best + 1] - cell_pt_off[best]);
      const int m = (int)(cfn_ptr[best + 1] - cfn_ptr[best]);
      if (FILL) {
        if (member) {
          const int64_t q = qoff[pos], so = soff[pos];
          if (q >= (1LL << 28) || so >= (1LL << 31)) atomicOr(overflow, 1);
          mem[mb + rank] = make_int2((int)(q | ((int64_t)lane << 28)), (int)so);
        }
        if (lane == 0) {
          const int64_t d0 = dptr[best];
          if (d0 >= (1LL << 31) || cell_pt_off[best] >= (1LL << 31) || np > 255 || m > 255) atomicOr(overflow, 1);
          ent[e] = make_int4((int)d0, (int)cell_pt_off[best], (int)(mask | (np << 16) | (m << 24)), (int)mb);
        }
        ++e;
        mb += nm;
      } else {
        // per-entry staging sizes of the assembly: the cell's basis block and the member weights
        mx[4] = max(mx[4], np * m);
        mx[5] = max(mx[5], nm * np);
      }
      if (member) ++pos;
      ++count;
    }
    if (!FILL) {
      if (lane == 0) eptr[tile] = count;
      mx[3] = max(mx[3], count);
    }
  }
  if (!FILL && lane == 0) {
    atomicMax(maxnnz, mx[0]);
    atomicMax(maxnnz + 2, mx[2]);
    atomicMax(maxnnz + 3, mx[3]);
    atomicMax(maxnnz + 4, mx[4]);
    atomicMax(maxnnz + 5, mx[5]);
  }
}

// Cell-major tiles: merge of the (ascending) cell lists of the rows [row0[t], row0[t+1]);
// one wave per tile, lane r holding the head of row r's list.
// FILL == false: count the distinct cells and the slot-map bytes of their members;
// FILL == true: write one entry per cell and copy its member rows' slot maps behind the
// tile's earlier ones (row order; each map padded to whole blocks of 16 functions and
// stored in the order the assembly's lanes read it: byte 16 cb + 4 g + v of a map holds the
// slot of function 16 cb + g + 4 v, and for positions past the cell's m functions some
// slot of the row, where only zero products land).
template <bool FILL>
__global__ void k_tile2_entries(int64_t n_tiles, const int32_t* row0, const int64_t* sptr, const int32_t* scell,
                                const int64_t* cfn_ptr, const int64_t* cell_pt_off, const int64_t* dptr,
                                const int64_t* soff, const uint8_t* slot, int64_t* eptr, int64_t* bptr, int4* ent,
                                uint8_t* tslot, int* overflow) {
  __shared__ int64_t msoff[BS / 64][T2_ROWS];  // per wave: slot-map offsets of an entry's members
  const int lane = threadIdx.x & 63;
  const int64_t tile = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  if (tile >= n_tiles) return;
  const int i0 = row0[tile];
  const int nr = row0[tile + 1] - i0;
  int64_t pos = 0, end = 0;
  if (lane < nr) {
    pos = sptr[i0 + lane];
    end = sptr[i0 + lane + 1];
  }
  int64_t e = FILL ? eptr[tile] : 0;
  int64_t sb = FILL ? bptr[tile] : 0;  // slot-map bytes
  int count = 0;
  while (true) {
    const int32_t head = pos < end ? scell[pos] : INT_MAX;
    const int32_t best = wave_min_i32(head);
    if (best == INT_MAX) break;
    const bool member = head == best;
    const unsigned long long bal = __ballot(member);
    const unsigned mask = (unsigned)bal;  // rows of the tile (nr <= 16 lanes)
    const int nm = __popcll(bal);
    const int rank = __popcll(bal & ((1ULL << lane) - 1ULL));
    const int np = (int)(cell_pt_off[best + 1] - cell_pt_off[best]);
    const int m = (int)(cfn_ptr[best + 1] - cfn_ptr[best]);
    const int mpad = (m + 15) & ~15;
    if (FILL) {
      // the members' slot maps, nm * mpad bytes behind sb, copied by all lanes (the
      // members' map offsets handed over through LDS)
      if (member) msoff[threadIdx.x >> 6][rank] = soff[pos];
      __builtin_amdgcn_wave_barrier();
      for (int t = lane; t < nm * mpad; t += 64) {
        const int u = t / mpad, tt = t - u * mpad;
        const int k = (tt & ~15) + ((tt >> 2) & 3) + 4 * (tt & 3);
        // a position past the cell's functions gets some slot of the row: the kernel adds
        // zero products there (no per-function predicate)
        tslot[sb + t] = slot[msoff[threadIdx.x >> 6][u] + (k < m ? k : k % m)];
      }
      __builtin_amdgcn_wave_barrier();
      if (lane == 0) {
        const int64_t d0 = dptr[best];
        const int64_t sbe = sb + (int64_t)nm * mpad;
        if (d0 > (int64_t)INT32_MAX || cell_pt_off[best] > (int64_t)INT32_MAX || sbe > (int64_t)INT32_MAX || np > 255 ||
            m > 255)
          atomicOr(overflow, 1);
        ent[e] = make_int4((int)d0, (int)cell_pt_off[best], (int)(mask | (np << 16) | (m << 24)), (int)sb);
      }
      ++e;
    }
    sb += (int64_t)nm * mpad;
    if (member) ++pos;
    ++count;
  }
  if (!FILL && lane == 0) {
    eptr[tile] = count;
    bptr[tile] = sb;
  }
}

struct Tmp {
  DBuf vptr, vcur, vidx, bnd, val, ep, passive, enriched, pvtx, tpoint, flags;
  void release() {
    DBuf* all[] = {&vptr, &vcur, &vidx, &bnd, &val, &ep, &passive, &enriched, &pvtx, &tpoint, &flags};
    dfree_many(all, sizeof(all) / sizeof(all[0]));
  }
};

void release_points(wq_points* P) {
  DBuf* all[] = {&P->etype, &P->s, &P->cell_face, &P->cell_sub, &P->cell_pt_off, &P->cfn_ptr, &P->cfn,
                 &P->cfn_loc, &P->dptr, &P->supp_ptr, &P->supp_cell, &P->row_ptr, &P->col, &P->qptr,
                 &P->qidx, &P->soff, &P->slot, &P->kself, &P->x, &P->detJ, &P->DN, &P->DX, &P->DY,
                 &P->DZ, &P->DL, &P->zterm_ws, &P->tile_eptr, &P->tile_ent, &P->tile_mem, &P->t2_row0,
                 &P->t2_eptr, &P->t2_ent, &P->t2_slot, &P->tangent_ws, &P->newton_ws, &P->DS[0],
                 &P->DS[1], &P->DS[2], &P->DS[3]};
  dfree_many(all, sizeof(all) / sizeof(all[0]));
  P->ds_prec = 0;
}

wq_status sync_flags(DBuf& flags, int* h, int n, hipStream_t st) {
  WQ_HIP(hipMemcpyAsync(h, flags.p, n * sizeof(int), hipMemcpyDeviceToHost, st));
  WQ_HIP(hipStreamSynchronize(st));
  return WQ_OK;
}

// Table 2 + classification on the device. etype/s are written to P.
wq_status classify(wq_mesh* M, wq_points* P, Tmp& T, hipStream_t st) {
  const int32_t nv = M->nv, nf = M->nf;
  WQ_TRY(dalloc_n<int64_t>(T.vptr, nv + 1));
  WQ_TRY(dalloc_n<int64_t>(T.vcur, nv));
  WQ_HIP(hipMemsetAsync(T.vptr.p, 0, (nv + 1) * sizeof(int64_t), st));
  WQ_HIP(hipMemsetAsync(T.vcur.p, 0, nv * sizeof(int64_t), st));
  const int32_t* fv = M->face_vtx.as<int32_t>();
  k_vf_count<<<nblocks(4LL * nf, BS), BS, 0, st>>>(fv, nf, T.vptr.as<int64_t>());
  int64_t tot = 0;
  WQ_TRY(exclusive_scan_i64(T.vptr.as<int64_t>(), nv + 1, &tot, st));
  WQ_TRY(dalloc_n<int32_t>(T.vidx, (size_t)tot));
  k_vf_fill<<<nblocks(4LL * nf, BS), BS, 0, st>>>(fv, nf, T.vptr.as<int64_t>(), T.vcur.as<int64_t>(),
                                                   T.vidx.as<int32_t>());
  k_sort_lists<<<nblocks(nv, BS), BS, 0, st>>>(T.vptr.as<int64_t>(), nv, T.vidx.as<int32_t>());
  WQ_TRY(dalloc_n<uint8_t>(T.bnd, nv));
  WQ_HIP(hipMemsetAsync(T.bnd.p, 0, nv, st));
  k_boundary<<<nblocks(4LL * nf, BS), BS, 0, st>>>(fv, nf, T.vptr.as<int64_t>(), T.vidx.as<int32_t>(),
                                                    T.bnd.as<uint8_t>());
  WQ_TRY(dalloc_n<int32_t>(T.val, nv));
  WQ_TRY(dalloc_n<uint8_t>(T.ep, nv));
  k_vertex_flags<<<nblocks(nv, BS), BS, 0, st>>>(nv, T.vptr.as<int64_t>(), T.bnd.as<uint8_t>(),
                                                  T.val.as<int32_t>(), T.ep.as<uint8_t>());
  WQ_TRY(dalloc_n<uint8_t>(T.passive, nf));
  WQ_TRY(dalloc_n<uint8_t>(T.enriched, nf));
  k_face_flags1<<<nblocks(nf, BS), BS, 0, st>>>(fv, nf, T.bnd.as<uint8_t>(), T.ep.as<uint8_t>(),
                                                 T.passive.as<uint8_t>(), T.enriched.as<uint8_t>());
  WQ_TRY(dalloc_n<uint8_t>(T.pvtx, nv));
  WQ_TRY(dalloc_n<uint8_t>(T.tpoint, nv));
  k_vertex_flags2<<<nblocks(nv, BS), BS, 0, st>>>(nv, T.vptr.as<int64_t>(), T.vidx.as<int32_t>(),
                                                   T.passive.as<uint8_t>(), T.enriched.as<uint8_t>(),
                                                   T.pvtx.as<uint8_t>(), T.tpoint.as<uint8_t>());
  WQ_TRY(dalloc_n<uint8_t>(P->etype, nf));
  WQ_TRY(dalloc_n<uint8_t>(P->s, nf));
  k_classify<<<nblocks(nf, BS), BS, 0, st>>>(fv, nf, T.vptr.as<int64_t>(), T.vidx.as<int32_t>(), T.val.as<int32_t>(),
                                              T.ep.as<uint8_t>(), T.passive.as<uint8_t>(), T.enriched.as<uint8_t>(),
                                              T.pvtx.as<uint8_t>(), T.tpoint.as<uint8_t>(), P->etype.as<uint8_t>(),
                                              P->s.as<uint8_t>());
  WQ_HIP(hipGetLastError());
  return WQ_OK;
}

// Everything that depends on s: cells, supports, pattern, point sets, slots.
// Sets *wp_bad to the number of rows with r_i < n_i.
wq_status build_structure(wq_mesh* M, wq_points* P, DBuf& flags, int* wp_bad, hipStream_t st) {
  const int32_t nf = M->nf;
  const int64_t n = M->n_fn;
  int hf[8];
  WQ_HIP(hipMemsetAsync(flags.p, 0, 8 * sizeof(int), st));
  int* df = flags.as<int>();
  // cells
  DBuf cptr;
  WQ_TRY(dalloc_n<int64_t>(cptr, nf + 1));
  k_cell_count<<<nblocks(nf, BS), BS, 0, st>>>(nf, P->s.as<uint8_t>(), M->split.as<uint8_t>(), cptr.as<int64_t>(), df);
  int64_t ncell = 0;
  WQ_TRY(exclusive_scan_i64(cptr.as<int64_t>(), nf + 1, &ncell, st));
  WQ_TRY(sync_flags(flags, hf, 1, st));
  if (hf[0]) {
    dfree(cptr);
    set_error("build_points: a split element has an odd number of points per direction");
    return WQ_EINVAL;
  }
  WQ_CHECK(ncell > 0 && ncell < INT32_MAX, WQ_EINVAL, "build_points: no cells (all faces passive?)");
  P->ncell = (int32_t)ncell;
  WQ_TRY(dalloc_n<int32_t>(P->cell_face, ncell));
  WQ_TRY(dalloc_n<uint8_t>(P->cell_sub, ncell));
  WQ_TRY(dalloc_n<int64_t>(P->cell_pt_off, ncell + 1));
  k_cell_fill<<<nblocks(nf, BS), BS, 0, st>>>(nf, P->s.as<uint8_t>(), M->split.as<uint8_t>(), cptr.as<int64_t>(),
                                               P->cell_face.as<int32_t>(), P->cell_sub.as<uint8_t>(),
                                               P->cell_pt_off.as<int64_t>());
  dfree(cptr);
  WQ_TRY(exclusive_scan_i64(P->cell_pt_off.as<int64_t>(), ncell + 1, &P->n_points, st));
  // cell functions
  WQ_TRY(dalloc_n<int64_t>(P->cfn_ptr, ncell + 1));
  WQ_HIP(hipMemsetAsync(P->cfn_ptr.p, 0, (ncell + 1) * sizeof(int64_t), st));
  k_cfn_count<<<nblocks(ncell, BS), BS, 0, st>>>((int32_t)ncell, P->cell_face.as<int32_t>(), P->cell_sub.as<uint8_t>(),
                                                  M->ext_ptr.as<int64_t>(), M->coef_ptr.as<int64_t>(),
                                                  M->coef.as<double>(), P->cfn_ptr.as<int64_t>());
  WQ_TRY(exclusive_scan_i64(P->cfn_ptr.as<int64_t>(), ncell + 1, &P->n_cfn, st));
  WQ_TRY(dalloc_n<int32_t>(P->cfn, P->n_cfn));
  WQ_TRY(dalloc_n<uint8_t>(P->cfn_loc, P->n_cfn));
  k_cfn_fill<<<nblocks(ncell, BS), BS, 0, st>>>((int32_t)ncell, P->cell_face.as<int32_t>(), P->cell_sub.as<uint8_t>(),
                                                 M->ext_ptr.as<int64_t>(), M->ext_fn.as<int32_t>(),
                                                 M->coef_ptr.as<int64_t>(), M->coef.as<double>(),
                                                 P->cfn_ptr.as<int64_t>(), P->cfn.as<int32_t>(),
                                                 P->cfn_loc.as<uint8_t>());
  // supports (function -> cells, ascending)
  WQ_TRY(dalloc_n<int64_t>(P->supp_ptr, n + 1));
  WQ_HIP(hipMemsetAsync(P->supp_ptr.p, 0, (n + 1) * sizeof(int64_t), st));
  k_supp_count<<<nblocks(P->n_cfn, BS), BS, 0, st>>>(P->n_cfn, P->cfn.as<int32_t>(), P->supp_ptr.as<int64_t>());
  WQ_TRY(exclusive_scan_i64(P->supp_ptr.as<int64_t>(), n + 1, &P->n_pairs, st));
  {
    DBuf cur;
    WQ_TRY(dalloc_n<int64_t>(cur, n));
    WQ_HIP(hipMemsetAsync(cur.p, 0, n * sizeof(int64_t), st));
    WQ_TRY(dalloc_n<int32_t>(P->supp_cell, P->n_pairs));
    k_supp_fill<<<nblocks(ncell, BS), BS, 0, st>>>((int32_t)ncell, P->cfn_ptr.as<int64_t>(), P->cfn.as<int32_t>(),
                                                    P->supp_ptr.as<int64_t>(), cur.as<int64_t>(),
                                                    P->supp_cell.as<int32_t>());
    k_sort_lists<<<nblocks(n, BS), BS, 0, st>>>(P->supp_ptr.as<int64_t>(), n, P->supp_cell.as<int32_t>());
    WQ_HIP(hipStreamSynchronize(st));
    dfree(cur);
  }
  // pattern sizes
  WQ_TRY(dalloc_n<int64_t>(P->row_ptr, n + 1));
  WQ_TRY(dalloc_n<int64_t>(P->qptr, n + 1));
  WQ_HIP(hipMemsetAsync(P->row_ptr.p, 0, (n + 1) * sizeof(int64_t), st));
  WQ_HIP(hipMemsetAsync(P->qptr.p, 0, (n + 1) * sizeof(int64_t), st));
  k_row_count<<<std::min(nblocks(n, BS / 64), 1024u), BS, 0, st>>>(n, P->supp_ptr.as<int64_t>(), P->supp_cell.as<int32_t>(),
                                              P->cfn_ptr.as<int64_t>(), P->cfn.as<int32_t>(),
                                              P->cell_pt_off.as<int64_t>(), P->row_ptr.as<int64_t>(),
                                              P->qptr.as<int64_t>(), df + 1, df + 2, df + 3, df + 4);
  WQ_TRY(sync_flags(flags, hf, 5, st));
  if (hf[1]) {
    set_error(hf[1] & 2 ? "build_points: a function has an empty support"
              : hf[1] & 1 ? "build_points: a support exceeds 64 Bezier cells"
                          : "build_points: a row exceeds 255 entries");
    return WQ_EINVAL;
  }
  *wp_bad = hf[2];
  P->max_row = hf[3];
  P->max_r = hf[4];
  WQ_TRY(exclusive_scan_i64(P->row_ptr.as<int64_t>(), n + 1, &P->nnz, st));
  int64_t sum_r = 0;
  WQ_TRY(exclusive_scan_i64(P->qptr.as<int64_t>(), n + 1, &sum_r, st));
  WQ_TRY(dalloc_n<int32_t>(P->col, P->nnz));
  WQ_TRY(dalloc_n<int32_t>(P->qidx, sum_r));
  k_row_fill<<<nblocks(n, BS / 64), BS, 0, st>>>(n, P->supp_ptr.as<int64_t>(), P->supp_cell.as<int32_t>(),
                                             P->cfn_ptr.as<int64_t>(), P->cfn.as<int32_t>(),
                                             P->cell_pt_off.as<int64_t>(), P->row_ptr.as<int64_t>(),
                                             P->qptr.as<int64_t>(), P->col.as<int32_t>(), P->qidx.as<int32_t>());
  // scatter slots per (row, cell) pair
  WQ_TRY(dalloc_n<int64_t>(P->soff, P->n_pairs + 1));
  WQ_HIP(hipMemsetAsync(P->soff.p, 0, (P->n_pairs + 1) * sizeof(int64_t), st));
  k_pair_m<<<nblocks(P->n_pairs, BS), BS, 0, st>>>(P->n_pairs, P->supp_cell.as<int32_t>(), P->cfn_ptr.as<int64_t>(),
                                                    P->soff.as<int64_t>());
  WQ_TRY(exclusive_scan_i64(P->soff.as<int64_t>(), P->n_pairs + 1, &P->n_slots, st));
  WQ_TRY(dalloc_n<uint8_t>(P->slot, P->n_slots));
  WQ_TRY(dalloc_n<uint8_t>(P->kself, P->n_pairs));
  k_slots<<<nblocks(n, BS / 64), BS, 0, st>>>(n, P->supp_ptr.as<int64_t>(), P->supp_cell.as<int32_t>(),
                                          P->cfn_ptr.as<int64_t>(), P->cfn.as<int32_t>(), P->row_ptr.as<int64_t>(),
                                          P->col.as<int32_t>(), P->soff.as<int64_t>(), P->slot.as<uint8_t>(),
                                          P->kself.as<uint8_t>());
  WQ_HIP(hipGetLastError());
  return WQ_OK;
}

// Eq. (18) "min-max" fallback on the host (rare: only when Table 2 leaves a row with
// r_i < n_i). r_{i,k} = m_k / sum_{l in supp i \ R} m_l (n_i - 4 e^r_i - 16 e^b_i) for the
// elements k of supp N_i that are neither regular nor boundary; r_k = max_i ceil(r_{i,k});
// s_k = smallest s >= 2 with s^2 >= r_k (even for split elements).
wq_status minmax_update(wq_mesh* M, wq_points* P, std::vector<uint8_t>& hs, bool* changed, hipStream_t st) {
  const int64_t n = M->n_fn;
  std::vector<uint8_t> het(M->nf), hsplit(M->nf);
  std::vector<int64_t> sptr(n + 1), rptr(n + 1);
  std::vector<int32_t> scell(P->n_pairs), cface(P->ncell);
  WQ_HIP(hipMemcpyAsync(het.data(), P->etype.p, M->nf, hipMemcpyDeviceToHost, st));
  WQ_HIP(hipMemcpyAsync(hsplit.data(), M->split.p, M->nf, hipMemcpyDeviceToHost, st));
  WQ_HIP(hipMemcpyAsync(sptr.data(), P->supp_ptr.p, (n + 1) * 8, hipMemcpyDeviceToHost, st));
  WQ_HIP(hipMemcpyAsync(rptr.data(), P->row_ptr.p, (n + 1) * 8, hipMemcpyDeviceToHost, st));
  WQ_HIP(hipMemcpyAsync(scell.data(), P->supp_cell.p, P->n_pairs * 4, hipMemcpyDeviceToHost, st));
  WQ_HIP(hipMemcpyAsync(cface.data(), P->cell_face.p, P->ncell * 4, hipMemcpyDeviceToHost, st));
  WQ_HIP(hipStreamSynchronize(st));
  std::vector<int64_t> need(M->nf, 0);
  std::vector<int32_t> els;
  for (int64_t i = 0; i < n; ++i) {
    els.clear();
    for (int64_t p = sptr[i]; p < sptr[i + 1]; ++p) els.push_back(cface[scell[p]]);
    std::sort(els.begin(), els.end());
    els.erase(std::unique(els.begin(), els.end()), els.end());
    int64_t er = 0, eb = 0, msum = 0;
    for (int32_t f : els) {
      if (het[f] == ET_REGULAR) ++er;
      else if (het[f] == ET_BOUNDARY) ++eb;
      else msum += M->h_ext_ptr[f + 1] - M->h_ext_ptr[f];
    }
    if (msum == 0) continue;
    const double ni = (double)(rptr[i + 1] - rptr[i]);
    for (int32_t f : els) {
      if (het[f] == ET_REGULAR || het[f] == ET_BOUNDARY) continue;
      const double mk = (double)(M->h_ext_ptr[f + 1] - M->h_ext_ptr[f]);
      const double rik = mk / (double)msum * (ni - 4.0 * er - 16.0 * eb);
      need[f] = std::max<int64_t>(need[f], (int64_t)std::ceil(rik - 1e-12));
    }
  }
  *changed = false;
  for (int32_t f = 0; f < M->nf; ++f) {
    if (!need[f]) continue;
    int sk = 2;
    while ((int64_t)sk * sk < need[f] || (hsplit[f] && (sk & 1))) ++sk;
    if (sk > hs[f]) {
      WQ_CHECK(sk <= 254, WQ_EILLPOSED, "min-max allocation needs more than 254 points per direction");
      hs[f] = (uint8_t)sk;
      *changed = true;
    }
  }
  return WQ_OK;
}

wq_status build_tiles(wq_mesh* M, wq_points* P, DBuf& flags, hipStream_t st) {
  const int64_t n = P->n_rows;
  P->n_tiles = (n + TILE_ROWS - 1) / TILE_ROWS;
  DBuf qoff;
  int hf[6];
  WQ_TRY(dalloc_n<int64_t>(qoff, P->n_pairs));
  WQ_TRY(dalloc_n<int64_t>(P->tile_eptr, P->n_tiles + 1));
  WQ_HIP(hipMemsetAsync(P->tile_eptr.p, 0, (P->n_tiles + 1) * sizeof(int64_t), st));
  WQ_HIP(hipMemsetAsync(flags.p, 0, 8 * sizeof(int), st));
  k_pair_qoff<<<nblocks(n, BS), BS, 0, st>>>(n, P->supp_ptr.as<int64_t>(), P->supp_cell.as<int32_t>(),
                                              P->cell_pt_off.as<int64_t>(), P->qptr.as<int64_t>(), qoff.as<int64_t>());
  k_tile_entries<false><<<std::min(nblocks(P->n_tiles, BS / 64), 1024u), BS, 0, st>>>(
      n, P->supp_ptr.as<int64_t>(), P->supp_cell.as<int32_t>(), P->cfn_ptr.as<int64_t>(), P->cell_pt_off.as<int64_t>(),
      P->dptr.as<int64_t>(), qoff.as<int64_t>(), P->soff.as<int64_t>(), P->row_ptr.as<int64_t>(),
      P->tile_eptr.as<int64_t>(), nullptr, nullptr, flags.as<int>(), flags.as<int>() + 1);
  WQ_TRY(exclusive_scan_i64(P->tile_eptr.as<int64_t>(), P->n_tiles + 1, &P->n_entries, st));
  WQ_TRY(dalloc(P->tile_ent, (size_t)P->n_entries * sizeof(int4)));
  WQ_TRY(dalloc(P->tile_mem, (size_t)P->n_pairs * sizeof(int2)));
  k_tile_entries<true><<<std::min(nblocks(P->n_tiles, BS / 64), 1024u), BS, 0, st>>>(
      n, P->supp_ptr.as<int64_t>(), P->supp_cell.as<int32_t>(), P->cfn_ptr.as<int64_t>(), P->cell_pt_off.as<int64_t>(),
      P->dptr.as<int64_t>(), qoff.as<int64_t>(), P->soff.as<int64_t>(), P->row_ptr.as<int64_t>(),
      P->tile_eptr.as<int64_t>(), P->tile_ent.as<int4>(), P->tile_mem.as<int2>(), flags.as<int>(),
      flags.as<int>() + 1);
  WQ_TRY(sync_flags(flags, hf, 6, st));
  dfree(qoff);
  P->max_tile_nd = hf[4];
  P->max_tile_nw = hf[5];
  P->max_tile_nnz = hf[0];
  P->max_tile_mem = hf[2];
  P->max_tile_ent = hf[3];
  WQ_CHECK(!hf[1], WQ_EINVAL, "build_points: mesh too large for 32-bit tile offsets; split it");
  WQ_HIP(hipGetLastError());
  return WQ_OK;
}

// Work of each row in the cell-major assembly: one step per block of four points of each of
// its support cells.
__global__ void k_row_steps(int64_t n, const int64_t* sptr, const int32_t* scell, const int64_t* cell_pt_off,
                            int32_t* steps) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int w = 0;
  for (int64_t p = sptr[i]; p < sptr[i + 1]; ++p) {
    const int32_t c = scell[p];
    w += (int)((cell_pt_off[c + 1] - cell_pt_off[c] + 3) / 4);
  }
  steps[i] = w;
}

// Cell-major tiles: runs of consecutive rows, at most T2_ROWS rows, T2_NZCAP CSR entries
// (the tile's accumulators live in LDS) and P->t2_stepcap summed row steps each, cut greedily in
// row order on the host. The step cap keeps the tiles next to extraordinary points (rows of
// many cells with many points) from taking several times the average tile's time: one wave
// runs a tile, so the heaviest tile sets the launch's end. (A row's sums do not depend on
// the tile it is in.)
wq_status build_tiles2(wq_points* P, DBuf& flags, hipStream_t st) {
  const int64_t n = P->n_rows;
  WQ_CHECK(n < INT32_MAX, WQ_EINVAL, "build_points: too many rows for 32-bit tile row ids");
  std::vector<int64_t> rp(n + 1);
  std::vector<int32_t> rw(n);
  {
    DBuf steps;
    WQ_TRY(dalloc_n<int32_t>(steps, (size_t)n));
    if (n > 0)
      k_row_steps<<<nblocks(n, BS), BS, 0, st>>>(n, P->supp_ptr.as<int64_t>(), P->supp_cell.as<int32_t>(),
                                                  P->cell_pt_off.as<int64_t>(), steps.as<int32_t>());
    WQ_HIP(hipMemcpyAsync(rp.data(), P->row_ptr.p, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    WQ_HIP(hipMemcpyAsync(rw.data(), steps.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    WQ_HIP(hipStreamSynchronize(st));
    dfree(steps);
  }
  std::vector<int32_t> row0;
  row0.reserve(n / 8 + 2);
  int32_t maxnz = 0;
  for (int64_t i = 0; i < n;) {
    const int64_t s = i;
    int64_t nz = 0, w = 0;
    while (i < n && i - s < T2_ROWS && nz + (rp[i + 1] - rp[i]) <= T2_NZCAP && (i == s || w + rw[i] <= P->t2_stepcap))
      nz += rp[i + 1] - rp[i], w += rw[i], ++i;
    WQ_CHECK(i > s, WQ_EINVAL, "build_points: a row exceeds the cell-major tile capacity");
    row0.push_back((int32_t)s);
    maxnz = std::max(maxnz, (int32_t)nz);
  }
  row0.push_back((int32_t)n);
  P->n_t2 = (int64_t)row0.size() - 1;
  P->t2_maxnz = maxnz;
  DBuf bptr;
  WQ_TRY(dalloc_n<int32_t>(P->t2_row0, row0.size()));
  WQ_HIP(hipMemcpyAsync(P->t2_row0.p, row0.data(), row0.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
  WQ_TRY(dalloc_n<int64_t>(P->t2_eptr, P->n_t2 + 1));
  WQ_TRY(dalloc_n<int64_t>(bptr, P->n_t2 + 1));
  WQ_HIP(hipMemsetAsync(P->t2_eptr.p, 0, (P->n_t2 + 1) * sizeof(int64_t), st));
  WQ_HIP(hipMemsetAsync(bptr.p, 0, (P->n_t2 + 1) * sizeof(int64_t), st));
  WQ_HIP(hipMemsetAsync(flags.p, 0, 8 * sizeof(int), st));
  k_tile2_entries<false><<<nblocks(P->n_t2, BS / 64), BS, 0, st>>>(
      P->n_t2, P->t2_row0.as<int32_t>(), P->supp_ptr.as<int64_t>(), P->supp_cell.as<int32_t>(),
      P->cfn_ptr.as<int64_t>(), P->cell_pt_off.as<int64_t>(), P->dptr.as<int64_t>(), P->soff.as<int64_t>(),
      P->slot.as<uint8_t>(), P->t2_eptr.as<int64_t>(), bptr.as<int64_t>(), nullptr, nullptr, flags.as<int>());
  int64_t nbytes = 0;
  {
    std::vector<int64_t> cnt(P->n_t2);
    WQ_HIP(hipMemcpyAsync(cnt.data(), P->t2_eptr.p, P->n_t2 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    WQ_HIP(hipStreamSynchronize(st));
    int64_t mx = 0;
    for (int64_t c : cnt) mx = std::max(mx, c);
    P->t2_maxent = (int32_t)mx;
  }
  WQ_TRY(exclusive_scan_i64(P->t2_eptr.as<int64_t>(), P->n_t2 + 1, &P->n_e2, st));
  WQ_TRY(exclusive_scan_i64(bptr.as<int64_t>(), P->n_t2 + 1, &nbytes, st));
  WQ_TRY(dalloc(P->t2_ent, (size_t)P->n_e2 * sizeof(int4)));
  WQ_TRY(dalloc(P->t2_slot, (size_t)nbytes + 4));
  k_tile2_entries<true><<<nblocks(P->n_t2, BS / 64), BS, 0, st>>>(
      P->n_t2, P->t2_row0.as<int32_t>(), P->supp_ptr.as<int64_t>(), P->supp_cell.as<int32_t>(),
      P->cfn_ptr.as<int64_t>(), P->cell_pt_off.as<int64_t>(), P->dptr.as<int64_t>(), P->soff.as<int64_t>(),
      P->slot.as<uint8_t>(), P->t2_eptr.as<int64_t>(), bptr.as<int64_t>(), P->t2_ent.as<int4>(),
      P->t2_slot.as<uint8_t>(), flags.as<int>());
  int hf[1];
  WQ_TRY(sync_flags(flags, hf, 1, st));
  dfree(bptr);
  WQ_CHECK(!hf[0], WQ_EINVAL, "build_points: mesh too large for 32-bit cell-major tile offsets; split it");
  WQ_HIP(hipGetLastError());
  ++P->t2_gen;
  return WQ_OK;
}

wq_status build_points_impl(wq_mesh* M, int want_lap, const uint8_t* s_host, hipStream_t st, wq_points** out,
                            int64_t* n_rows, int64_t* nnz, int64_t* n_points) {
  WQ_CHECK(M && out, WQ_EINVAL, "build_points: null argument");
  int dev = 0;
  WQ_HIP(hipGetDevice(&dev));
  WQ_CHECK(dev == M->device, WQ_EINVAL, "build_points: mesh was created on another device");
  wq_points* P = new wq_points();
  P->mesh = M;
  P->n_rows = M->n_fn;
  P->has_lap = want_lap ? 1 : 0;
  Tmp T;
  DBuf flags;
  wq_status s = dalloc_n<int>(flags, 8);
  if (s == WQ_OK) s = classify(M, P, T, st);
  if (s == WQ_OK && s_host) {
    s = (hipMemcpyAsync(P->s.p, s_host, M->nf, hipMemcpyHostToDevice, st) == hipSuccess) ? WQ_OK : WQ_EDEVICE;
  }
  T.release();
  int wp_bad = 0;
  for (int iter = 0; s == WQ_OK && iter < 16; ++iter) {
    s = build_structure(M, P, flags, &wp_bad, st);
    if (s != WQ_OK || wp_bad == 0) break;
    std::vector<uint8_t> hs(M->nf);
    if (hipMemcpy(hs.data(), P->s.p, M->nf, hipMemcpyDeviceToHost) != hipSuccess) { s = WQ_EDEVICE; break; }
    bool changed = false;
    s = minmax_update(M, P, hs, &changed, st);
    if (s != WQ_OK) break;
    if (!changed) {
      set_error("build_points: " + std::to_string(wp_bad) +
                " rows have fewer points than constraints and the min-max allocation cannot fix them");
      s = WQ_EILLPOSED;
      break;
    }
    if (hipMemcpy(P->s.p, hs.data(), M->nf, hipMemcpyHostToDevice) != hipSuccess) { s = WQ_EDEVICE; break; }
    wq_points tmp;  // keep etype/s, drop the rest
    std::swap(tmp.etype, P->etype);
    std::swap(tmp.s, P->s);
    release_points(P);
    std::swap(tmp.etype, P->etype);
    std::swap(tmp.s, P->s);
  }
  if (s == WQ_OK && wp_bad) {
    set_error("build_points: min-max allocation did not converge");
    s = WQ_EILLPOSED;
  }
  // basis and geometry at the points
  if (s == WQ_OK) {
    int hf[4];
    DBuf npm;
    s = dalloc_n<int64_t>(P->dptr, P->ncell + 1);
    if (s == WQ_OK && hipMemsetAsync(flags.p, 0, 8 * sizeof(int), st) != hipSuccess) s = WQ_EDEVICE;
    if (s == WQ_OK && hipMemsetAsync(P->dptr.p, 0, (P->ncell + 1) * sizeof(int64_t), st) != hipSuccess) s = WQ_EDEVICE;
    if (s == WQ_OK) {
      k_cell_np_m<<<nblocks(P->ncell, BS), BS, 0, st>>>(P->ncell, P->cell_pt_off.as<int64_t>(),
                                                          P->cfn_ptr.as<int64_t>(), P->dptr.as<int64_t>(),
                                                          flags.as<int>() + 1, flags.as<int>() + 2);
      s = exclusive_scan_i64(P->dptr.as<int64_t>(), P->ncell + 1, &P->n_basis, st);
    }
    if (s == WQ_OK) s = sync_flags(flags, hf, 3, st);
    if (s == WQ_OK) {
      P->max_cell_m = hf[1];
      P->max_cell_np = hf[2];
    }
    if (s == WQ_OK) s = dalloc_n<double>(P->x, (size_t)M->dim * P->n_points);
    if (s == WQ_OK) s = dalloc_n<double>(P->detJ, P->n_points);
    if (s == WQ_OK) s = dalloc_n<double>(P->DN, P->n_basis);
    if (s == WQ_OK) s = dalloc_n<double>(P->DX, P->n_basis);
    if (s == WQ_OK) s = dalloc_n<double>(P->DY, P->n_basis);
    if (s == WQ_OK && M->dim == 3) s = dalloc_n<double>(P->DZ, P->n_basis);
    if (s == WQ_OK && want_lap) s = dalloc_n<double>(P->DL, P->n_basis);
    if (s == WQ_OK && hipMemsetAsync(flags.p, 0, 8 * sizeof(int), st) != hipSuccess) s = WQ_EDEVICE;
    if (s == WQ_OK) {
      KTimer tm("k_basis", P->n_points, st);
      k_basis<<<nblocks(P->n_points, BS), BS, 0, st>>>(
          P->n_points, P->ncell, P->cell_pt_off.as<int64_t>(), P->cell_face.as<int32_t>(), P->cell_sub.as<uint8_t>(),
          P->s.as<uint8_t>(), M->split.as<uint8_t>(), M->ext_ptr.as<int64_t>(), M->coef_ptr.as<int64_t>(),
          M->coef.as<double>(), M->ctrl.as<double>(), P->cfn_ptr.as<int64_t>(), P->cfn.as<int32_t>(),
          P->cfn_loc.as<uint8_t>(), P->dptr.as<int64_t>(), P->x.as<double>(), P->detJ.as<double>(),
          P->DN.as<double>(), P->DX.as<double>(), P->DY.as<double>(), P->DZ.as<double>(),
          want_lap ? P->DL.as<double>() : nullptr, M->dim, flags.as<int>());
      tm.stop();
      if (hipGetLastError() != hipSuccess) s = WQ_EDEVICE;
    }
    if (s == WQ_OK) s = sync_flags(flags, hf, 1, st);
    if (s == WQ_OK && hf[0]) {
      set_error(M->dim == 3 ? "build_points: a degenerate surface point (det g <= 0)"
                            : "build_points: det J <= 0 at some point (geometry map not orientation-preserving)");
      s = WQ_EINVAL;
    }
    dfree(npm);
  }
  // assembly tiles (need dptr)
  if (s == WQ_OK) s = build_tiles(M, P, flags, st);
  if (s == WQ_OK) s = build_tiles2(P, flags, st);
  dfree(flags);
  if (s != WQ_OK) {
    release_points(P);
    delete P;
    return s;
  }
  *out = P;
  if (n_rows) *n_rows = P->n_rows;
  if (nnz) *nnz = P->nnz;
  if (n_points) *n_points = P->n_points;
  return WQ_OK;
}

}  // namespace

wq_status wq::rebuild_tiles2(wq_points* P, hipStream_t st) {
  DBuf flags;
  WQ_TRY(dalloc_n<int>(flags, 8));
  const wq_status s = build_tiles2(P, flags, st);
  dfree(flags);
  return s;
}

void wq_release_points(wq_points* P) { release_points(P); }

extern "C" wq_status build_points(wq_mesh* M, int want_lap, wq_stream stream, wq_points** out, int64_t* n_rows,
                                  int64_t* nnz, int64_t* n_points) {
  return build_points_impl(M, want_lap, nullptr, (hipStream_t)stream, out, n_rows, nnz, n_points);
}

extern "C" wq_status build_points_with_s(wq_mesh* M, const uint8_t* s_host, int want_lap, wq_stream stream,
                                         wq_points** out, int64_t* n_rows, int64_t* nnz, int64_t* n_points) {
  WQ_CHECK(s_host && M, WQ_EINVAL, "build_points_with_s: null argument");
  for (int32_t f = 0; f < M->nf; ++f) {
    const bool has_fn = M->h_ext_ptr[f + 1] > M->h_ext_ptr[f];
    WQ_CHECK(s_host[f] <= 254 && (s_host[f] == 0 || has_fn), WQ_EINVAL,
             "build_points_with_s: s > 0 on a face without functions");
  }
  return build_points_impl(M, want_lap, s_host, (hipStream_t)stream, out, n_rows, nnz, n_points);
}

extern "C" void wq_points_destroy(wq_points* P) {
  if (!P) return;
  release_points(P);
  delete P;
}

extern "C" int64_t wq_points_size(const wq_points* P, wq_array what) {
  if (!P) return -1;
  switch (what) {
    case WQ_ARR_ROW_PTR: case WQ_ARR_QPTR: return P->n_rows + 1;
    case WQ_ARR_COL: return P->nnz;
    case WQ_ARR_QIDX: return (int64_t)(P->qidx.bytes / sizeof(int32_t));
    case WQ_ARR_ETYPE: case WQ_ARR_S: return P->mesh->nf;
    case WQ_ARR_X: return (int64_t)P->mesh->dim * P->n_points;
    case WQ_ARR_DETJ: return P->n_points;
  }
  return -1;
}

extern "C" int64_t wq_points_info(const wq_points* P, int what) {
  if (!P) return -1;
  switch (what) {
    case 0: return P->max_row;
    case 1: return P->max_r;
    case 2: return P->ncell;
    case 3: return P->n_t2;
    case 4: return P->n_e2;
    case 5: return P->t2_maxnz;
    case 6: return P->max_tile_ent;
    case 7: return P->max_tile_mem;
    case 8: return P->n_pairs;
    case 9: return P->max_tile_nd;
    case 10: return P->max_tile_nw;
  }
  return -1;
}

extern "C" wq_status wq_points_get(const wq_points* P, wq_array what, void* dst, wq_stream stream) {
  WQ_CHECK(P && dst, WQ_EINVAL, "wq_points_get: null argument");
  const DBuf* b = nullptr;
  size_t es = 0;
  switch (what) {
    case WQ_ARR_ROW_PTR: b = &P->row_ptr; es = 8; break;
    case WQ_ARR_COL: b = &P->col; es = 4; break;
    case WQ_ARR_QPTR: b = &P->qptr; es = 8; break;
    case WQ_ARR_QIDX: b = &P->qidx; es = 4; break;
    case WQ_ARR_ETYPE: b = &P->etype; es = 1; break;
    case WQ_ARR_S: b = &P->s; es = 1; break;
    case WQ_ARR_X: b = &P->x; es = 8; break;
    case WQ_ARR_DETJ: b = &P->detJ; es = 8; break;
    default: WQ_CHECK(false, WQ_EINVAL, "wq_points_get: unknown array");
  }
  const int64_t n = wq_points_size(P, what);
  WQ_HIP(hipMemcpyAsync(dst, b->p, (size_t)n * es, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return WQ_OK;
}
