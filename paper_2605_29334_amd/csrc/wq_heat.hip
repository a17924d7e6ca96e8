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

// scalar slots in the workspace
enum { S_RHO = 0, S_ALPHA, S_OMEGA, S_BETA, S_RR, S_NORM, S_SS, S_COUNT };

struct Ws {
  double *Tn, *Tdn, *R, *x, *r, *rh, *p, *v, *y, *s, *z, *t, *d;
  double* part;      // per-block partial sums (two lanes per block)
  double* sc;        // scalars
  unsigned* ticket;  // last-block counter (returns to 0 after each reduction)
};
constexpr int NVEC = 13;

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

// Deterministic grid reduction: each block stores its partial sums (a, b); the last
// block to finish adds all partials in block order and calls fin(total_a, total_b).
template <class Fin>
__device__ inline void grid_reduce(double a, double b, Ws ws, double* sh, Fin fin) {
  __shared__ bool last;
  a = block_sum(a, sh);
  b = block_sum(b, sh + 8);
  if (threadIdx.x == 0) {
    ws.part[2 * blockIdx.x] = a;
    ws.part[2 * blockIdx.x + 1] = b;
    __threadfence();
    last = atomicAdd(ws.ticket, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double ta = 0.0, tb = 0.0;
  for (unsigned k = threadIdx.x; k < gridDim.x; k += blockDim.x) {
    ta += ws.part[2 * k];
    tb += ws.part[2 * k + 1];
  }
  ta = block_sum(ta, sh);
  tb = block_sum(tb, sh + 8);
  if (threadIdx.x == 0) {
    fin(ta, tb);
    *ws.ticket = 0u;
  }
}

__device__ inline double safe_div(double a, double b) { return b != 0.0 ? a / b : 0.0; }

// y = S u on free rows (0 on prescribed rows; u is 0 on prescribed DOFs), 8 lanes per row;
// returns the row value on lane 0 of the row group
__device__ inline double row_product(int64_t i, int sub, int64_t n, const int64_t* row_ptr, const int32_t* col,
                                     const double* S, const uint8_t* dir, const double* u) {
  double v = 0.0;
  if (i < n) {
    for (int64_t e = row_ptr[i] + sub; e < row_ptr[i + 1]; e += ROW_LANES) v += S[e] * u[col[e]];
  }
  for (int off = ROW_LANES / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return (i < n && !dir[i]) ? v : 0.0;
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

__global__ void k_norm_free(int64_t n, const double* R, const uint8_t* dir, Ws ws) {
  __shared__ double sh[16];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const double v = (i < n && !dir[i]) ? R[i] : 0.0;
  grid_reduce(v * v, 0.0, ws, sh, [&](double a, double) { ws.sc[S_NORM] = a; });
}

// Jacobi-preconditioned BiCGStab for S_ff x = -R_f (the WQ tangent with a variable
// conductivity is not symmetric: rows are integrated by their own weights).
// Start: x = 0, r = r^ = -R (0 on prescribed DOFs), p = v = 0, d = diag(S) (1 on
// prescribed DOFs); rho = r^.r, rr = r.r, alpha = omega = 1.
__global__ void k_bi_init(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* S,
                          const uint8_t* dir, Ws ws) {
  __shared__ double sh[16];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double rr = 0.0;
  if (i < n) {
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
  grid_reduce(rr, rr, ws, sh, [&](double a, double b) {
    ws.sc[S_RHO] = a;
    ws.sc[S_RR] = b;
    ws.sc[S_ALPHA] = 1.0;
    ws.sc[S_OMEGA] = 1.0;
    ws.sc[S_BETA] = 0.0;
  });
}

// p = r + beta (p - omega v); y = p / d
__global__ void k_bi_dir(int64_t n, Ws ws) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double pi = ws.r[i] + ws.sc[S_BETA] * (ws.p[i] - ws.sc[S_OMEGA] * ws.v[i]);
  ws.p[i] = pi;
  ws.y[i] = pi / ws.d[i];
}

// v = S y; alpha = rho / (r^.v)
__global__ void k_bi_sv(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* S, const uint8_t* dir,
                        Ws ws) {
  __shared__ double sh[16];
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / ROW_LANES;
  const int sub = threadIdx.x % ROW_LANES;
  const double vi = row_product(i, sub, n, row_ptr, col, S, dir, ws.y);
  double a = 0.0;
  if (i < n && sub == 0) {
    ws.v[i] = vi;
    a = ws.rh[i] * vi;
  }
  grid_reduce(a, 0.0, ws, sh, [&](double t, double) { ws.sc[S_ALPHA] = safe_div(ws.sc[S_RHO], t); });
}

// x += alpha y; s = r - alpha v; z = s / d
__global__ void k_bi_s(int64_t n, Ws ws) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double al = ws.sc[S_ALPHA];
  ws.x[i] += al * ws.y[i];
  const double si = ws.r[i] - al * ws.v[i];
  ws.s[i] = si;
  ws.z[i] = si / ws.d[i];
}

// t = S z; omega = (t.s) / (t.t)
__global__ void k_bi_tz(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* S, const uint8_t* dir,
                        Ws ws) {
  __shared__ double sh[16];
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / ROW_LANES;
  const int sub = threadIdx.x % ROW_LANES;
  const double ti = row_product(i, sub, n, row_ptr, col, S, dir, ws.z);
  double ts = 0.0, tt = 0.0;
  if (i < n && sub == 0) {
    ws.t[i] = ti;
    ts = ti * ws.s[i];
    tt = ti * ti;
  }
  grid_reduce(ts, tt, ws, sh, [&](double a, double b) { ws.sc[S_OMEGA] = safe_div(a, b); });
}

// x += omega z; r = s - omega t; rho' = r^.r, rr = r.r; beta = (rho' / rho) (alpha / omega)
__global__ void k_bi_r(int64_t n, Ws ws) {
  __shared__ double sh[16];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const double om = ws.sc[S_OMEGA];
  double a = 0.0, b = 0.0;
  if (i < n) {
    ws.x[i] += om * ws.z[i];
    const double ri = ws.s[i] - om * ws.t[i];
    ws.r[i] = ri;
    a = ws.rh[i] * ri;
    b = ri * ri;
  }
  grid_reduce(a, b, ws, sh, [&](double rho1, double rr) {
    ws.sc[S_BETA] = safe_div(rho1, ws.sc[S_RHO]) * safe_div(ws.sc[S_ALPHA], om);
    ws.sc[S_RHO] = rho1;
    ws.sc[S_RR] = rr;
  });
}

__global__ void k_add(int64_t n, double* T, const double* dT) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) T[i] += dT[i];
}

wq_status read_scalar(const Ws& ws, int k, double* out, hipStream_t st) {
  WQ_HIP(hipMemcpyAsync(out, ws.sc + k, sizeof(double), hipMemcpyDeviceToHost, st));
  WQ_HIP(hipStreamSynchronize(st));
  return WQ_OK;
}

}  // namespace

extern "C" wq_status wq_heat_step(const wq_points* P, const wq_weights* w, const wq_heat_params* hp,
                                  const uint8_t* dirichlet, const double* g_next, const double* f_at_pts, double* T,
                                  double* Tdot, double* S_vals, wq_heat_report* rep, wq_stream stream) {
  WQ_CHECK(P && w && hp && dirichlet && T && Tdot && S_vals, WQ_EINVAL, "wq_heat_step: null argument");
  WQ_CHECK(P->mesh->dim == 2, WQ_EINVAL, "wq_heat_step: the heat solve is planar (dim 2)");
  WQ_CHECK(hp->dt > 0 && hp->theta > 0 && hp->theta <= 1 && hp->tol > 0 && hp->max_newton >= 0 && hp->max_cg > 0 &&
               (hp->tangent == WQ_TANGENT_SYMMETRIC || hp->tangent == WQ_TANGENT_EXACT),
           WQ_EINVAL, "wq_heat_step: bad parameters");
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = P->n_rows;
  const unsigned nb = nblocks(n, RB);
  const unsigned nbs = nblocks(n * ROW_LANES, RB);
  const size_t need = (NVEC * (size_t)n + 2 * (size_t)std::max(nb, nbs) + 8) * sizeof(double) + 64;
  wq_points* Pm = const_cast<wq_points*>(P);
  if (Pm->newton_ws.bytes < need) {
    WQ_TRY(dalloc(Pm->newton_ws, need));
    WQ_HIP(hipMemsetAsync(Pm->newton_ws.p, 0, need, st));  // the reduction ticket starts at 0
  }
  Ws ws;
  double* base = Pm->newton_ws.as<double>();
  double** vec[NVEC] = {&ws.Tn, &ws.Tdn, &ws.R, &ws.x, &ws.r, &ws.rh, &ws.p, &ws.v, &ws.y, &ws.s, &ws.z, &ws.t, &ws.d};
  for (int k = 0; k < NVEC; ++k) *vec[k] = base + k * n;
  ws.part = base + NVEC * n;
  ws.sc = ws.part + 2 * std::max(nb, nbs);
  ws.ticket = (unsigned*)(ws.sc + 8);
  const double c1 = (1.0 - hp->theta) * hp->dt;
  const double inv_tdt = 1.0 / (hp->theta * hp->dt);
  wq_heat_report rp{0, 0, 0.0, 0.0};
  k_predict<<<nb, RB, 0, st>>>(n, T, Tdot, ws, c1, dirichlet, g_next);
  WQ_HIP(hipGetLastError());
  const int64_t* row_ptr = P->row_ptr.as<int64_t>();
  const int32_t* col = P->col.as<int32_t>();
  wq_status status = WQ_OK;
  for (int it = 0;; ++it) {
    k_rate<<<nb, RB, 0, st>>>(n, T, Tdot, ws, c1, inv_tdt);
    if (hp->tangent == WQ_TANGENT_EXACT)
      WQ_TRY(assemble_tangent_exact(P, w, T, Tdot, inv_tdt, hp->k, f_at_pts, S_vals, ws.R, WQ_FP64, stream));
    else
      WQ_TRY(assemble_tangent(P, w, T, Tdot, inv_tdt, hp->k, f_at_pts, S_vals, ws.R, WQ_FP64, stream));
    k_norm_free<<<nb, RB, 0, st>>>(n, ws.R, dirichlet, ws);
    WQ_HIP(hipGetLastError());
    double nr2 = 0.0;
    WQ_TRY(read_scalar(ws, S_NORM, &nr2, st));
    const double nr = std::sqrt(nr2);
    if (it == 0) rp.residual0 = nr;
    rp.residual = nr;
    WQ_CHECK(std::isfinite(nr), WQ_ENOCONV, "wq_heat_step: residual is not finite");
    if (nr <= hp->tol) break;
    if (it >= hp->max_newton) {
      set_error("wq_heat_step: Newton iteration cap reached, ||R|| = " + std::to_string(nr));
      status = WQ_ENOCONV;
      break;
    }
    // BiCGStab on S_ff dT_f = -R_f
    const double target = std::max(hp->cg_rtol * nr, 0.1 * hp->tol);
    k_bi_init<<<nb, RB, 0, st>>>(n, row_ptr, col, (const double*)S_vals, dirichlet, ws);
    WQ_HIP(hipGetLastError());
    double rr = 0.0;
    WQ_TRY(read_scalar(ws, S_RR, &rr, st));
    int k = 0;
    while (std::sqrt(rr) > target) {
      if (k >= hp->max_cg) {
        set_error("wq_heat_step: BiCGStab iteration cap reached, ||r|| = " + std::to_string(std::sqrt(rr)));
        status = WQ_ENOCONV;
        break;
      }
      for (int s = 0; s < CHECK_EVERY; ++s, ++k) {
        k_bi_dir<<<nb, RB, 0, st>>>(n, ws);
        k_bi_sv<<<nbs, RB, 0, st>>>(n, row_ptr, col, (const double*)S_vals, dirichlet, ws);
        k_bi_s<<<nb, RB, 0, st>>>(n, ws);
        k_bi_tz<<<nbs, RB, 0, st>>>(n, row_ptr, col, (const double*)S_vals, dirichlet, ws);
        k_bi_r<<<nb, RB, 0, st>>>(n, ws);
      }
      WQ_HIP(hipGetLastError());
      WQ_TRY(read_scalar(ws, S_RR, &rr, st));
      WQ_CHECK(std::isfinite(rr), WQ_ENOCONV, "wq_heat_step: BiCGStab residual is not finite");
    }
    rp.cg_iters += k;
    if (status != WQ_OK) break;
    k_add<<<nb, RB, 0, st>>>(n, T, ws.x);
    WQ_HIP(hipGetLastError());
    rp.newton_iters = it + 1;
  }
  if (rep) *rep = rp;
  return status;
}
