// Nonlinear heat transfer time step (Section 5.2): predictor, corrector Newton iterations
// with the WQ tangent of Eq. (36), and the linear solves of Eq. (33) by Jacobi-
// preconditioned BiCGStab on the device.
#include "wq_internal.h"

#include <cmath>
#include <vector>

using namespace wq;

namespace {

constexpr int RB = 256;        // threads per block of the vector kernels
constexpr int ROW_LANES = 8;   // lanes per CSR row in the matrix-vector product
constexpr int CHECK_EVERY = 4; // Krylov iterations between host convergence checks

// scalar slots in the workspace (NSC per segment)
enum { S_RHO = 0, S_ALPHA, S_OMEGA, S_BETA, S_RR, S_NORM, S_SS, S_COUNT };
constexpr int NSC = 8;

struct Ws {
  double *Tn, *Tdn, *R, *x, *r, *rh, *p, *v, *y, *s, *z, *t, *d;
  double* part;      // per-block partial sums (two lanes per block)
  double* sc;        // scalars, NSC per segment
  unsigned* ticket;  // last-block counters, one per segment (each returns to 0 after its reduction)
};
constexpr int NVEC = 13;

// Segments: the rows are split into consecutive segments (the meshes of a union), each
// solved as if alone: its own blocks start at its first row, its reductions add its own
// blocks' partial sums in block order, and its scalars and convergence are its own.
// Two block layouts: vector kernels take RB rows a block, row products RB / ROW_LANES.
struct Seg {
  const int64_t* row0;     // [nseg + 1] first row of each segment
  const int32_t* bseg;     // segment of each block (vector layout)
  const int32_t* bfirst;   // [nseg + 1] first block of each segment (vector layout)
  const int32_t* bseg8;    // the same for the row-product layout
  const int32_t* bfirst8;
  const uint8_t* act;      // [nseg] 1: the segment takes part in the launch (nullptr: all do)
};

struct SegRow {
  int k;         // segment
  int64_t i;     // row
  bool in;       // the row exists (i < the segment's end)
  int32_t b0;    // the segment's first block
  int32_t nbk;   // its block count
};

// row of this thread: one per thread (vector layout) or one per ROW_LANES lanes
template <int LANES>
__device__ inline SegRow seg_row(const Seg& g) {
  const int32_t* bs = LANES == 1 ? g.bseg : g.bseg8;
  const int32_t* bf = LANES == 1 ? g.bfirst : g.bfirst8;
  SegRow q;
  q.k = bs[blockIdx.x];
  q.b0 = bf[q.k];
  q.nbk = bf[q.k + 1] - q.b0;
  q.i = g.row0[q.k] + ((int64_t)(blockIdx.x - q.b0) * blockDim.x + threadIdx.x) / LANES;
  q.in = q.i < g.row0[q.k + 1];
  return q;
}

__device__ inline bool seg_active(const Seg& g, int k) { return g.act == nullptr || g.act[k] != 0; }

__device__ inline double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < (int)blockDim.x / 64; ++k) s += sh[k];
  return s;
}

// Deterministic reduction over a segment's blocks: each block stores its partial sums
// (a, b); the segment's last block to finish adds the segment's partials in block order
// and calls fin(total_a, total_b, its scalars).
template <class Fin>
__device__ inline void seg_reduce(double a, double b, Ws ws, double* sh, const SegRow& q, Fin fin) {
  __shared__ bool last;
  a = block_sum(a, sh);
  b = block_sum(b, sh + 8);
  if (threadIdx.x == 0) {
    ws.part[2 * blockIdx.x] = a;
    ws.part[2 * blockIdx.x + 1] = b;
    __threadfence();
    last = atomicAdd(ws.ticket + q.k, 1u) == (unsigned)q.nbk - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double ta = 0.0, tb = 0.0;
  for (int j = threadIdx.x; j < q.nbk; j += blockDim.x) {
    ta += ws.part[2 * (q.b0 + j)];
    tb += ws.part[2 * (q.b0 + j) + 1];
  }
  ta = block_sum(ta, sh);
  tb = block_sum(tb, sh + 8);
  if (threadIdx.x == 0) {
    fin(ta, tb, ws.sc + NSC * q.k);
    ws.ticket[q.k] = 0u;
  }
}

__device__ inline double safe_div(double a, double b) { return b != 0.0 ? a / b : 0.0; }

// y = S u on free rows (0 on prescribed rows; u is 0 on prescribed DOFs), 8 lanes per row;
// returns the row value on lane 0 of the row group
__device__ inline double row_product(int64_t i, bool in, int sub, const int64_t* row_ptr, const int32_t* col,
                                     const double* S, const uint8_t* dir, const double* u) {
  double v = 0.0;
  if (in) {
    for (int64_t e = row_ptr[i] + sub; e < row_ptr[i + 1]; e += ROW_LANES) v += S[e] * u[col[e]];
  }
  for (int off = ROW_LANES / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return (in && !dir[i]) ? v : 0.0;
}

__global__ void k_predict(int64_t n, double* T, double* Td, Ws ws, double c1, const uint8_t* dir, const double* g) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  ws.Tn[i] = T[i];
  ws.Tdn[i] = Td[i];
  T[i] = dir[i] ? (g ? g[i] : 0.0) : T[i] + c1 * Td[i];
}

// Tdot = (T - T_n - (1 - theta) dt Tdot_n) / (theta dt)
__global__ void k_rate(int64_t n, const double* T, double* Td, Ws ws, double c1, double inv_tdt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  Td[i] = (T[i] - ws.Tn[i] - c1 * ws.Tdn[i]) * inv_tdt;
}

__global__ void k_norm_free(const double* R, const uint8_t* dir, Ws ws, Seg g) {
  __shared__ double sh[16];
  const SegRow q = seg_row<1>(g);
  const double v = (q.in && !dir[q.i]) ? R[q.i] : 0.0;
  seg_reduce(v * v, 0.0, ws, sh, q, [&](double a, double, double* sc) { sc[S_NORM] = a; });
}

// Jacobi-preconditioned BiCGStab for S_ff x = -R_f (the WQ tangent with a variable
// conductivity is not symmetric: rows are integrated by their own weights).
// Start: x = 0, r = r^ = -R (0 on prescribed DOFs), p = v = 0, d = diag(S) (1 on
// prescribed DOFs); rho = r^.r, rr = r.r, alpha = omega = 1.
__global__ void k_bi_init(const int64_t* row_ptr, const int32_t* col, const double* S, const uint8_t* dir, Ws ws,
                          Seg g) {
  __shared__ double sh[16];
  const SegRow q = seg_row<1>(g);
  if (!seg_active(g, q.k)) return;  // (uniform: a block lies in one segment)
  const int64_t i = q.i;
  double rr = 0.0;
  if (q.in) {
    double di = 1.0, ri = 0.0;
    if (!dir[i]) {
      int64_t lo = row_ptr[i], hi = row_ptr[i + 1] - 1;
      while (lo < hi) {  // the diagonal: column i in the ascending row
        const int64_t mid = (lo + hi) / 2;
        if (col[mid] < i) lo = mid + 1;
        else hi = mid;
      }
      di = S[lo];
      ri = -ws.R[i];
    }
    ws.d[i] = di;
    ws.x[i] = 0.0;
    ws.r[i] = ri;
    ws.rh[i] = ri;
    ws.p[i] = 0.0;
    ws.v[i] = 0.0;
    rr = ri * ri;
  }
  seg_reduce(rr, rr, ws, sh, q, [&](double a, double b, double* sc) {
    sc[S_RHO] = a;
    sc[S_RR] = b;
    sc[S_ALPHA] = 1.0;
    sc[S_OMEGA] = 1.0;
    sc[S_BETA] = 0.0;
  });
}

// p = r + beta (p - omega v); y = p / d
__global__ void k_bi_dir(Ws ws, Seg g) {
  const SegRow q = seg_row<1>(g);
  if (!q.in || !seg_active(g, q.k)) return;
  const double* sc = ws.sc + NSC * q.k;
  const int64_t i = q.i;
  const double pi = ws.r[i] + sc[S_BETA] * (ws.p[i] - sc[S_OMEGA] * ws.v[i]);
  ws.p[i] = pi;
  ws.y[i] = pi / ws.d[i];
}

// v = S y; alpha = rho / (r^.v)
__global__ void k_bi_sv(const int64_t* row_ptr, const int32_t* col, const double* S, const uint8_t* dir, Ws ws,
                        Seg g) {
  __shared__ double sh[16];
  const SegRow q = seg_row<ROW_LANES>(g);
  if (!seg_active(g, q.k)) return;
  const int sub = threadIdx.x % ROW_LANES;
  const double vi = row_product(q.i, q.in, sub, row_ptr, col, S, dir, ws.y);
  double a = 0.0;
  if (q.in && sub == 0) {
    ws.v[q.i] = vi;
    a = ws.rh[q.i] * vi;
  }
  seg_reduce(a, 0.0, ws, sh, q, [&](double t, double, double* sc) { sc[S_ALPHA] = safe_div(sc[S_RHO], t); });
}

// x += alpha y; s = r - alpha v; z = s / d
__global__ void k_bi_s(Ws ws, Seg g) {
  const SegRow q = seg_row<1>(g);
  if (!q.in || !seg_active(g, q.k)) return;
  const int64_t i = q.i;
  const double al = ws.sc[NSC * q.k + S_ALPHA];
  ws.x[i] += al * ws.y[i];
  const double si = ws.r[i] - al * ws.v[i];
  ws.s[i] = si;
  ws.z[i] = si / ws.d[i];
}

// t = S z; omega = (t.s) / (t.t)
__global__ void k_bi_tz(const int64_t* row_ptr, const int32_t* col, const double* S, const uint8_t* dir, Ws ws,
                        Seg g) {
  __shared__ double sh[16];
  const SegRow q = seg_row<ROW_LANES>(g);
  if (!seg_active(g, q.k)) return;
  const int sub = threadIdx.x % ROW_LANES;
  const double ti = row_product(q.i, q.in, sub, row_ptr, col, S, dir, ws.z);
  double ts = 0.0, tt = 0.0;
  if (q.in && sub == 0) {
    ws.t[q.i] = ti;
    ts = ti * ws.s[q.i];
    tt = ti * ti;
  }
  seg_reduce(ts, tt, ws, sh, q, [&](double a, double b, double* sc) { sc[S_OMEGA] = safe_div(a, b); });
}

// x += omega z; r = s - omega t; rho' = r^.r, rr = r.r; beta = (rho' / rho) (alpha / omega)
__global__ void k_bi_r(Ws ws, Seg g) {
  __shared__ double sh[16];
  const SegRow q = seg_row<1>(g);
  if (!seg_active(g, q.k)) return;
  const double om = ws.sc[NSC * q.k + S_OMEGA];
  double a = 0.0, b = 0.0;
  if (q.in) {
    const int64_t i = q.i;
    ws.x[i] += om * ws.z[i];
    const double ri = ws.s[i] - om * ws.t[i];
    ws.r[i] = ri;
    a = ws.rh[i] * ri;
    b = ri * ri;
  }
  seg_reduce(a, b, ws, sh, q, [&](double rho1, double rr, double* sc) {
    sc[S_BETA] = safe_div(rho1, sc[S_RHO]) * safe_div(sc[S_ALPHA], om);
    sc[S_RHO] = rho1;
    sc[S_RR] = rr;
  });
}

__global__ void k_add(double* T, const double* dT, Seg g) {
  const SegRow q = seg_row<1>(g);
  if (q.in && seg_active(g, q.k)) T[q.i] += dT[q.i];
}

}  // namespace

wq_status wq::heat_step_segments(const wq_points* P, const wq_weights* w, const wq_heat_params* hp,
                                 const uint8_t* dirichlet, const double* g_next, const double* f_at_pts, double* T,
                                 double* Tdot, double* S_vals, int32_t nseg, const int64_t* seg_row0,
                                 wq_heat_report* reps, wq_status* stats, hipStream_t st) {
  WQ_CHECK(P && w && hp && dirichlet && T && Tdot && S_vals && seg_row0 && reps && stats && nseg >= 1, WQ_EINVAL,
           "wq_heat_step: null argument");
  WQ_CHECK(P->mesh->dim == 2, WQ_EINVAL, "wq_heat_step: the heat solve is planar (dim 2)");
  WQ_CHECK(hp->dt > 0 && hp->theta > 0 && hp->theta <= 1 && hp->tol > 0 && hp->max_newton >= 0 && hp->max_cg > 0 &&
               (hp->tangent == WQ_TANGENT_SYMMETRIC || hp->tangent == WQ_TANGENT_EXACT),
           WQ_EINVAL, "wq_heat_step: bad parameters");
  const int64_t n = P->n_rows;
  WQ_CHECK(seg_row0[0] == 0 && seg_row0[nseg] == n, WQ_EINVAL, "wq_heat_step: segments must cover the rows");
  // block tables of the two layouts
  std::vector<int64_t> hrow0(seg_row0, seg_row0 + nseg + 1);
  std::vector<int32_t> bfirst(nseg + 1), bfirst8(nseg + 1), bseg, bseg8;
  for (int32_t k = 0; k < nseg; ++k) {
    const int64_t nk = hrow0[k + 1] - hrow0[k];
    WQ_CHECK(nk >= 0, WQ_EINVAL, "wq_heat_step: segments must not decrease");
    bfirst[k] = (int32_t)bseg.size();
    bfirst8[k] = (int32_t)bseg8.size();
    bseg.insert(bseg.end(), (size_t)((nk + RB - 1) / RB), k);
    bseg8.insert(bseg8.end(), (size_t)((nk * ROW_LANES + RB - 1) / RB), k);
  }
  bfirst[nseg] = (int32_t)bseg.size();
  bfirst8[nseg] = (int32_t)bseg8.size();
  const unsigned nb = (unsigned)bseg.size(), nbs = (unsigned)bseg8.size();
  const unsigned nbf = nblocks(n, RB);  // the flat vector kernels
  // workspace: vectors, partial sums, scalars | row0 | block tables, tickets | flags
  const size_t nd = NVEC * (size_t)n + 2 * (size_t)std::max(nb, nbs) + NSC * (size_t)nseg;
  const size_t ni = 2 * (size_t)nseg + 2 + nb + nbs + 2 * ((size_t)nseg + 1) + nseg;  // int32 slots
  const size_t need = nd * sizeof(double) + (nseg + 1) * sizeof(int64_t) + ni * sizeof(int32_t) + 2 * (size_t)nseg + 64;
  wq_points* Pm = const_cast<wq_points*>(P);
  if (Pm->newton_ws.bytes < need) WQ_TRY(dalloc(Pm->newton_ws, need));
  Ws ws;
  double* base = Pm->newton_ws.as<double>();
  double** vec[NVEC] = {&ws.Tn, &ws.Tdn, &ws.R, &ws.x, &ws.r, &ws.rh, &ws.p, &ws.v, &ws.y, &ws.s, &ws.z, &ws.t, &ws.d};
  for (int k = 0; k < NVEC; ++k) *vec[k] = base + k * n;
  ws.part = base + NVEC * n;
  ws.sc = ws.part + 2 * std::max(nb, nbs);
  int64_t* drow0 = (int64_t*)(ws.sc + NSC * nseg);
  int32_t* dbfirst = (int32_t*)(drow0 + nseg + 1);
  int32_t* dbfirst8 = dbfirst + nseg + 1;
  int32_t* dbseg = dbfirst8 + nseg + 1;
  int32_t* dbseg8 = dbseg + nb;
  ws.ticket = (unsigned*)(dbseg8 + nbs);
  uint8_t* dact = (uint8_t*)(ws.ticket + nseg);  // [newton-active | krylov-active]
  {
    // one upload of the tables (row0, bfirst, bfirst8, bseg, bseg8 are contiguous), the
    // tickets cleared (the layout moves with n and nseg)
    std::vector<int32_t> tab(2 * ((size_t)nseg + 1) + nb + nbs);
    std::copy(bfirst.begin(), bfirst.end(), tab.begin());
    std::copy(bfirst8.begin(), bfirst8.end(), tab.begin() + nseg + 1);
    std::copy(bseg.begin(), bseg.end(), tab.begin() + 2 * (nseg + 1));
    std::copy(bseg8.begin(), bseg8.end(), tab.begin() + 2 * (nseg + 1) + nb);
    WQ_HIP(hipMemcpyAsync(drow0, hrow0.data(), (nseg + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
    WQ_HIP(hipMemcpyAsync(dbfirst, tab.data(), tab.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    WQ_HIP(hipMemsetAsync(ws.ticket, 0, nseg * sizeof(unsigned), st));
    WQ_HIP(hipStreamSynchronize(st));  // (the host tables go out of scope)
  }
  Seg gall{drow0, dbseg, dbfirst, dbseg8, dbfirst8, nullptr};
  Seg gnewton = gall, gkrylov = gall;
  gnewton.act = dact;
  gkrylov.act = dact + nseg;
  std::vector<uint8_t> act(2 * (size_t)nseg, 0);
  std::vector<double> sc((size_t)NSC * nseg);
  auto upload_act = [&]() -> wq_status {
    WQ_HIP(hipMemcpyAsync(dact, act.data(), act.size(), hipMemcpyHostToDevice, st));
    return WQ_OK;
  };
  auto read_sc = [&]() -> wq_status {  // all segments' scalars; synchronises the stream
    WQ_HIP(hipMemcpyAsync(sc.data(), ws.sc, sc.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    WQ_HIP(hipStreamSynchronize(st));
    return WQ_OK;
  };
  for (int32_t k = 0; k < nseg; ++k) {
    reps[k] = wq_heat_report{0, 0, 0.0, 0.0};
    stats[k] = WQ_OK;
    act[k] = hrow0[k + 1] > hrow0[k];  // (an empty segment has nothing to solve)
  }
  const double c1 = (1.0 - hp->theta) * hp->dt;
  const double inv_tdt = 1.0 / (hp->theta * hp->dt);
  k_predict<<<nbf, RB, 0, st>>>(n, T, Tdot, ws, c1, dirichlet, g_next);
  WQ_HIP(hipGetLastError());
  const int64_t* row_ptr = P->row_ptr.as<int64_t>();
  const int32_t* col = P->col.as<int32_t>();
  std::vector<double> target(nseg), rr(nseg);
  for (int it = 0;; ++it) {
    // the tangent of the whole union (segments that have stopped keep their T, so their
    // rows come out as before)
    k_rate<<<nbf, RB, 0, st>>>(n, T, Tdot, ws, c1, inv_tdt);
    if (hp->tangent == WQ_TANGENT_EXACT)
      WQ_TRY(assemble_tangent_exact(P, w, T, Tdot, inv_tdt, hp->k, f_at_pts, S_vals, ws.R, WQ_FP64, (wq_stream)st));
    else
      WQ_TRY(assemble_tangent(P, w, T, Tdot, inv_tdt, hp->k, f_at_pts, S_vals, ws.R, WQ_FP64, (wq_stream)st));
    if (nb > 0) k_norm_free<<<nb, RB, 0, st>>>(ws.R, dirichlet, ws, gall);
    WQ_HIP(hipGetLastError());
    WQ_TRY(read_sc());
    bool any = false;
    for (int32_t k = 0; k < nseg; ++k) {
      if (!act[k]) continue;
      const double nr = std::sqrt(sc[NSC * k + S_NORM]);
      if (it == 0) reps[k].residual0 = nr;
      reps[k].residual = nr;
      act[k] = 0;
      if (!std::isfinite(nr)) {
        set_error("wq_heat_step: residual is not finite");
        stats[k] = WQ_ENOCONV;
      } else if (nr <= hp->tol) {
      } else if (it >= hp->max_newton) {
        set_error("wq_heat_step: Newton iteration cap reached, ||R|| = " + std::to_string(nr));
        stats[k] = WQ_ENOCONV;
      } else {
        act[k] = 1;
        target[k] = std::max(hp->cg_rtol * nr, 0.1 * hp->tol);
        any = true;
      }
    }
    if (!any) break;
    // BiCGStab on S_ff dT_f = -R_f, segment by segment: a segment's iterations stop at the
    // first check (every CHECK_EVERY iterations) where its ||r|| <= its target
    WQ_TRY(upload_act());
    k_bi_init<<<nb, RB, 0, st>>>(row_ptr, col, (const double*)S_vals, dirichlet, ws, gnewton);
    WQ_HIP(hipGetLastError());
    WQ_TRY(read_sc());
    for (int32_t k = 0; k < nseg; ++k) {
      act[nseg + k] = act[k];
      rr[k] = sc[NSC * k + S_RR];
    }
    int kk = 0;
    for (;;) {
      bool running = false, changed = false;
      for (int32_t k = 0; k < nseg; ++k) {
        if (!act[nseg + k]) continue;
        if (std::sqrt(rr[k]) > target[k]) {
          running = true;
          continue;
        }
        act[nseg + k] = 0;  // converged: Newton adds its update
        reps[k].cg_iters += kk;
        changed = true;
      }
      if (!running) break;
      if (kk >= hp->max_cg) {
        for (int32_t k = 0; k < nseg; ++k) {
          if (!act[nseg + k]) continue;
          set_error("wq_heat_step: BiCGStab iteration cap reached, ||r|| = " + std::to_string(std::sqrt(rr[k])));
          stats[k] = WQ_ENOCONV;
          act[nseg + k] = act[k] = 0;
          reps[k].cg_iters += kk;
        }
        break;
      }
      if (changed || kk == 0) WQ_TRY(upload_act());
      for (int s = 0; s < CHECK_EVERY; ++s, ++kk) {
        k_bi_dir<<<nb, RB, 0, st>>>(ws, gkrylov);
        k_bi_sv<<<nbs, RB, 0, st>>>(row_ptr, col, (const double*)S_vals, dirichlet, ws, gkrylov);
        k_bi_s<<<nb, RB, 0, st>>>(ws, gkrylov);
        k_bi_tz<<<nbs, RB, 0, st>>>(row_ptr, col, (const double*)S_vals, dirichlet, ws, gkrylov);
        k_bi_r<<<nb, RB, 0, st>>>(ws, gkrylov);
      }
      WQ_HIP(hipGetLastError());
      WQ_TRY(read_sc());
      for (int32_t k = 0; k < nseg; ++k) {
        if (!act[nseg + k]) continue;
        rr[k] = sc[NSC * k + S_RR];
        if (!std::isfinite(rr[k])) {
          set_error("wq_heat_step: BiCGStab residual is not finite");
          stats[k] = WQ_ENOCONV;
          act[nseg + k] = act[k] = 0;
          reps[k].cg_iters += kk;
        }
      }
    }
    // T += dT on the segments whose solve converged
    bool add = false;
    for (int32_t k = 0; k < nseg; ++k) add = add || act[k];
    if (add) {
      WQ_TRY(upload_act());
      k_add<<<nb, RB, 0, st>>>(T, ws.x, gnewton);
      WQ_HIP(hipGetLastError());
    }
    for (int32_t k = 0; k < nseg; ++k)
      if (act[k]) reps[k].newton_iters = it + 1;
  }
  return WQ_OK;
}

extern "C" wq_status wq_heat_step(const wq_points* P, const wq_weights* w, const wq_heat_params* hp,
                                  const uint8_t* dirichlet, const double* g_next, const double* f_at_pts, double* T,
                                  double* Tdot, double* S_vals, wq_heat_report* rep, wq_stream stream) {
  WQ_CHECK(P, WQ_EINVAL, "wq_heat_step: null argument");
  const int64_t row0[2] = {0, P->n_rows};
  wq_heat_report rp{};
  wq_status st1 = WQ_OK;
  WQ_TRY(heat_step_segments(P, w, hp, dirichlet, g_next, f_at_pts, T, Tdot, S_vals, 1, row0, &rp, &st1,
                            (hipStream_t)stream));
  if (rep) *rep = rp;
  return st1;
}
