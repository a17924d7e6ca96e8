// Row-wise WQ assembly (Eqs. (9), (11), (12)); Section 6.1 forms the matrix row by row.
// The tangent of the nonlinear heat problem (Eq. (36)) and its residual use the same
// kernel with the conductivity evaluated at the points.
#include "wq_internal.h"

#include <cmath>

using namespace wq;

namespace {

constexpr int WAVE = 64;
constexpr int NXCD = 8;    // MI355X: workgroups are dispatched round-robin over 8 XCDs
constexpr int CHUNK = 64;  // consecutive tiles per XCD turn

// Families per kernel: K = 0 mass, 1 stiffness, 2 biharmonic, 3 mass + stiffness,
// 4 tangent (Eq. (36)) + residual.
// N basis arrays (N or Delta N; dN/dx, dN/dy) and as many weight families; weight family
// a is scaled by the coefficient array cof(a) (or, for the tangent's mass term, by the
// constant 1/(theta dt)).
template <int K> struct Fam {
  static constexpr int N = (K >= 3) ? 3 : (K == 1 ? 2 : 1);
  static constexpr int NACC = (K == 3) ? 2 : 1;
  static constexpr int NC = (K == 3) ? 2 : 1;
  static constexpr bool RES = (K == 4);
  __device__ static constexpr int cof(int a) { return (K == 3 && a > 0) ? 1 : 0; }
  // tangent: mass term scaled by a constant, conductivity terms by C[0]
  __device__ static constexpr bool constant(int a) { return K == 4 && a == 0; }
};

struct Src {
  const double* D[3];   // basis blocks, point-major per cell: D[d0 + q * m + k]
  const double* W[3];   // weights aligned with Q_i
  const double* C[2];   // coefficients at the points (nullptr: 1)
  double scale;         // tangent: 1 / (theta dt) on the mass term
  const double* Pf[3];  // tangent residual point fields: Tdot - f, k dT/dx, k dT/dy
};

constexpr int PFD = 4;  // register slots (x 64 lanes) prefetched for a cell's basis block
constexpr int PFW = 1;  // ... for the member rows' weights on the cell
constexpr int PFS = 4;  // ... for the members' column slots

// Entry e of a tile: cell block at d0, points pt0.., np points, m functions; member rows
// are the set bits of the 16-bit mask, their records at smem[mb ..] in row order.
struct Ent {
  int64_t d0, pt0;
  int np, m, R, mb;
  float rnp, rm;  // 1/np, 1/m for exact small-integer division (see qdiv)
};

__device__ inline Ent decode(const int4 E, int64_t m0) {
  Ent e;
  e.d0 = (uint32_t)E.x;
  e.pt0 = (uint32_t)E.y;
  e.np = (E.z >> 16) & 0xff;
  e.m = (int)((unsigned)E.z >> 24);
  e.R = __popc((unsigned)E.z & 0xffffu);
  e.mb = (int)((int64_t)(uint32_t)E.w - m0);
  e.rnp = 1.0f / (float)e.np;
  e.rm = 1.0f / (float)e.m;
  return e;
}

// floor(t / d) for 0 <= t < 4096, 1 <= d <= 255, with r = 1/d rounded to fp32: the
// quotient (t + 1/2) / d is at least 1/(2d) >= 1/510 away from an integer and the fp32
// product errs by < 4096 * 2^-23 < 5e-4, so truncation is exact.
__device__ inline int qdiv(int t, float r) { return (int)(((float)t + 0.5f) * r); }

template <int K> struct Pre {
  double d[Fam<K>::N][PFD];
  double w[Fam<K>::N][PFW];
  double c[Fam<K>::NC][PFW];
  double pf[Fam<K>::RES ? 3 : 1][PFW];
  int s[PFS];
  int rl[PFS];
};

// Issue the global loads of one entry into registers (consumed by stage()).
template <int K>
__device__ inline void prefetch(const Ent& e, int lane, const Src& S, const int2* smem,
                                const uint8_t* __restrict__ slot, Pre<K>& p) {
  constexpr int N = Fam<K>::N;
  const int nd = e.np * e.m, nw = e.R * e.np, ns = e.R * e.m;
#pragma unroll
  for (int u = 0; u < PFD; ++u) {
    const int t = lane + WAVE * u;
    if (t < nd) {
#pragma unroll
      for (int a = 0; a < N; ++a) p.d[a][u] = S.D[a][e.d0 + t];
    }
  }
#pragma unroll
  for (int u = 0; u < PFW; ++u) {
    const int t = lane + WAVE * u;
    if (t < nw) {
      const int j = qdiv(t, e.rnp), q = t - j * e.np;
      const int64_t qo = smem[e.mb + j].x & ((1 << 28) - 1);
#pragma unroll
      for (int a = 0; a < N; ++a) p.w[a][u] = S.W[a][qo + q];
#pragma unroll
      for (int a = 0; a < Fam<K>::NC; ++a) p.c[a][u] = S.C[a] ? S.C[a][e.pt0 + q] : 1.0;
      if (Fam<K>::RES) {
#pragma unroll
        for (int a = 0; a < 3; ++a) p.pf[a][u] = S.Pf[a][e.pt0 + q];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < PFS; ++u) {
    const int t = lane + WAVE * u;
    if (t < ns) {
      const int j = qdiv(t, e.rm), k = t - j * e.m;
      const int2 mm = smem[e.mb + j];
      p.s[u] = slot[(uint32_t)mm.y + k];
      p.rl[u] = (int)((unsigned)mm.x >> 28);
    }
  }
}

template <int K>
__device__ inline double scaled(const Src& S, int a, double w, double c) {
  return Fam<K>::constant(a) ? w * S.scale : w * c;
}

// Write one prefetched entry into the LDS stage: basis blocks sd[a][q * m + k] and
// coefficient-scaled weights sw[a][j * np + q]; parts beyond the register slots are
// loaded here directly. Tangent: also the residual terms of (member j, point q),
// rho[j * np + q] = w0 (Tdot - f) + wx k dT/dx + wy k dT/dy.
template <int K>
__device__ inline void stage(const Ent& e, int lane, const Src& S, const int2* smem, const Pre<K>& p,
                             double* sd, int nd_cap, double* sw, int nw_cap, double* rho) {
  constexpr int N = Fam<K>::N;
  const int nd = e.np * e.m, nw = e.R * e.np;
#pragma unroll
  for (int u = 0; u < PFD; ++u) {
    const int t = lane + WAVE * u;
    if (t < nd) {
#pragma unroll
      for (int a = 0; a < N; ++a) sd[a * nd_cap + t] = p.d[a][u];
    }
  }
  for (int t = lane + WAVE * PFD; t < nd; t += WAVE)
    for (int a = 0; a < N; ++a) sd[a * nd_cap + t] = S.D[a][e.d0 + t];
#pragma unroll
  for (int u = 0; u < PFW; ++u) {
    const int t = lane + WAVE * u;
    if (t < nw) {
#pragma unroll
      for (int a = 0; a < N; ++a) sw[a * nw_cap + t] = scaled<K>(S, a, p.w[a][u], p.c[Fam<K>::cof(a)][u]);
      if (Fam<K>::RES)
        rho[t] = p.w[0][u] * p.pf[0][u] + (p.w[N - 2][u] * p.pf[1][u] + p.w[N - 1][u] * p.pf[2][u]);
    }
  }
  for (int t = lane + WAVE * PFW; t < nw; t += WAVE) {
    const int j = qdiv(t, e.rnp), q = t - j * e.np;
    const int64_t qo = smem[e.mb + j].x & ((1 << 28) - 1);
    double wv[N];
    for (int a = 0; a < N; ++a) {
      const double* C = S.C[Fam<K>::cof(a)];
      wv[a] = S.W[a][qo + q];
      sw[a * nw_cap + t] = scaled<K>(S, a, wv[a], C ? C[e.pt0 + q] : 1.0);
    }
    if (Fam<K>::RES)
      rho[t] = wv[0] * S.Pf[0][e.pt0 + q] + (wv[N - 2] * S.Pf[1][e.pt0 + q] + wv[N - 1] * S.Pf[2][e.pt0 + q]);
  }
}

// lane (j, k): v = sum_q sw[j][q] sd[q][k] (per family), added to acc[row j][slot k].
template <int K>
__device__ inline void accumulate(const Ent& e, int t, int sk, int rl, const double* sd, int nd_cap,
                                  const double* sw, int nw_cap, const int* ro, double* acc, int acc_stride) {
  const int j = qdiv(t, e.rm), k = t - j * e.m;
  const double* w = sw + j * e.np;
  double va = 0.0, vb = 0.0;
  for (int q = 0; q < e.np; ++q) {
    const int dq = q * e.m + k;
    if (K == 0 || K == 2) {
      va += w[q] * sd[dq];
    } else if (K == 1) {
      va += w[q] * sd[dq] + w[nw_cap + q] * sd[nd_cap + dq];
    } else if (K == 3) {
      va += w[q] * sd[dq];
      vb += w[nw_cap + q] * sd[nd_cap + dq] + w[2 * nw_cap + q] * sd[2 * nd_cap + dq];
    } else {
      va += w[q] * sd[dq] + (w[nw_cap + q] * sd[nd_cap + dq] + w[2 * nw_cap + q] * sd[2 * nd_cap + dq]);
    }
  }
  const int at = ro[rl] + sk;
  acc[at] += va;
  if (K == 3) acc[acc_stride + at] += vb;
}

// One wavefront owns a tile of TILE_ROWS consecutive rows and their accumulators in LDS.
// It visits the tile's cells once each, in ascending order (one precomputed entry per
// cell: basis block, points, member rows). Per entry, the whole wave loads the cell's
// basis block and the members' weights with coalesced loads into an LDS stage, then
// lane (j, k) forms v = sum_{points q of the cell} w_{i_j q} coef_q D_k(x_q) for member
// row i_j and cell function k and adds it to acc[i_j][slot]. The next entry's loads are
// issued into registers before the current one is computed. Within an entry the (j, k)
// are distinct and entries are applied in order: no atomics, fixed summation order.
// Tangent: lane j < R also adds its member's residual terms (sum over the cell's points,
// in point order) to racc[i_j]; R is written once per row.
// Workgroups of one XCD take chunks of consecutive tiles (L2 reuse between neighbours).
template <int K>
__global__ void __launch_bounds__(WAVE) k_assemble(int64_t n, int64_t n_tiles, int64_t per_xcd, int acc_stride,
                                                   int mem_cap, int nd_cap, int nw_cap,
                                                   const int64_t* __restrict__ eptr, const int4* __restrict__ ent,
                                                   const int2* __restrict__ mem, const int64_t* __restrict__ sptr,
                                                   const uint8_t* __restrict__ slot,
                                                   const int64_t* __restrict__ row_ptr, Src S,
                                                   double* __restrict__ out0, double* __restrict__ out1) {
  constexpr int N = Fam<K>::N;
  constexpr int NACC = Fam<K>::NACC;
  constexpr bool RES = Fam<K>::RES;
  extern __shared__ double acc[];
  __shared__ int ro[TILE_ROWS + 1];
  __shared__ double racc[TILE_ROWS];
  double* sd = acc + NACC * acc_stride;
  double* sw = sd + N * nd_cap;
  double* rho = sw + N * nw_cap;  // tangent only (nw_cap doubles)
  int2* smem = (int2*)(rho + (RES ? nw_cap : 0));
  const int64_t b = blockIdx.x;
  const int64_t turn = b / NXCD;
  const int64_t tile = (turn / CHUNK) * (NXCD * CHUNK) + (b % NXCD) * CHUNK + turn % CHUNK;
  if (tile >= n_tiles) return;
  const int lane = threadIdx.x;
  const int64_t i0 = tile * TILE_ROWS;
  const int nr = (int)min((int64_t)TILE_ROWS, n - i0);
  const int64_t a0 = row_ptr[i0];
  const int nz = (int)(row_ptr[i0 + nr] - a0);
  const int64_t e0 = eptr[tile];
  const int ne = (int)(eptr[tile + 1] - e0);
  const int64_t m0 = sptr[i0];
  const int nm = (int)(sptr[i0 + nr] - m0);
  if (lane <= nr) ro[lane] = (int)(row_ptr[i0 + lane] - a0);
  if (RES && lane < TILE_ROWS) racc[lane] = 0.0;
  for (int t = lane; t < NACC * acc_stride; t += WAVE) acc[t] = 0.0;
  for (int t = lane; t < nm; t += WAVE) smem[t] = mem[m0 + t];
  __syncthreads();
  if (ne > 0) {
    Pre<K> p;
    Ent cur = decode(ent[e0], m0);
    prefetch<K>(cur, lane, S, smem, slot, p);
    stage<K>(cur, lane, S, smem, p, sd, nd_cap, sw, nw_cap, rho);
    int cs[PFS], cr[PFS];
#pragma unroll
    for (int u = 0; u < PFS; ++u) {
      cs[u] = p.s[u];
      cr[u] = p.rl[u];
    }
    __syncthreads();
    for (int e = 0; e < ne; ++e) {
      Ent nxt;
      const bool more = e + 1 < ne;
      if (more) {
        nxt = decode(ent[e0 + e + 1], m0);
        prefetch<K>(nxt, lane, S, smem, slot, p);
      }
      const int ns = cur.R * cur.m;
#pragma unroll
      for (int u = 0; u < PFS; ++u) {
        const int t = lane + WAVE * u;
        if (t < ns) accumulate<K>(cur, t, cs[u], cr[u], sd, nd_cap, sw, nw_cap, ro, acc, acc_stride);
      }
      for (int t = lane + WAVE * PFS; t < ns; t += WAVE) {
        const int j = qdiv(t, cur.rm), k = t - j * cur.m;
        const int2 mm = smem[cur.mb + j];
        accumulate<K>(cur, t, slot[(uint32_t)mm.y + k], (int)((unsigned)mm.x >> 28), sd, nd_cap, sw, nw_cap, ro,
                      acc, acc_stride);
      }
      if (RES && lane < cur.R) {
        double v = 0.0;
        for (int q = 0; q < cur.np; ++q) v += rho[lane * cur.np + q];
        racc[(unsigned)smem[cur.mb + lane].x >> 28] += v;
      }
      __syncthreads();
      if (more) {
        stage<K>(nxt, lane, S, smem, p, sd, nd_cap, sw, nw_cap, rho);
#pragma unroll
        for (int u = 0; u < PFS; ++u) {
          cs[u] = p.s[u];
          cr[u] = p.rl[u];
        }
        cur = nxt;
      }
      __syncthreads();
    }
  }
  for (int t = lane; t < nz; t += WAVE) {
    out0[a0 + t] = acc[t];
    if (K == 3) out1[a0 + t] = acc[acc_stride + t];
  }
  if (RES && lane < nr) out1[i0 + lane] = racc[lane];
}

template <int K>
wq_status launch(const wq_points* P, const wq_weights* w, Src S, double* o0, double* o1, hipStream_t st) {
  constexpr int N = Fam<K>::N;
  constexpr int NACC = Fam<K>::NACC;
  const int nd_cap = P->max_tile_nd, nw_cap = P->max_tile_nw;
  const size_t lds = (size_t)NACC * P->max_tile_nnz * sizeof(double) +
                     (size_t)(N * (nd_cap + nw_cap) + (Fam<K>::RES ? nw_cap : 0)) * sizeof(double) +
                     (size_t)P->max_tile_mem * sizeof(int2);
  WQ_CHECK(lds <= 150 * 1024, WQ_EINVAL, "assemble: tile accumulators and stage exceed LDS");
  WQ_CHECK(nw_cap < 4096 && (int64_t)TILE_ROWS * 255 < 4096, WQ_EINVAL, "assemble: entry too large");
  if (K == 0) {
    S.D[0] = P->DN.as<double>();
    S.W[0] = w->W[0].as<double>();
  } else if (K == 1) {
    S.D[0] = P->DX.as<double>();
    S.D[1] = P->DY.as<double>();
    S.W[0] = w->W[1].as<double>();
    S.W[1] = w->W[2].as<double>();
  } else if (K == 2) {
    S.D[0] = P->DL.as<double>();
    S.W[0] = w->W[3].as<double>();
  } else {
    S.D[0] = P->DN.as<double>();
    S.D[1] = P->DX.as<double>();
    S.D[2] = P->DY.as<double>();
    S.W[0] = w->W[0].as<double>();
    S.W[1] = w->W[1].as<double>();
    S.W[2] = w->W[2].as<double>();
  }
  // grid covers whole rounds of NXCD * CHUNK tiles; blocks past the end exit
  const int64_t per_xcd = ((P->n_tiles + NXCD * CHUNK - 1) / (NXCD * CHUNK)) * CHUNK;
  static const char* names[5] = {"k_assemble_mass", "k_assemble_stiffness", "k_assemble_biharmonic",
                                  "k_assemble_mass_stiffness", "k_assemble_tangent"};
  if (lds > 64 * 1024)
    WQ_HIP(hipFuncSetAttribute((const void*)k_assemble<K>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  // algorithmic bytes: every basis value and weight once, the coefficients, the output
  const int64_t sum_r = (int64_t)(P->qidx.bytes / sizeof(int32_t));
  int64_t nc = 0;
  for (int a = 0; a < 2; ++a) nc += S.C[a] ? 1 : 0;
  if (K == 4) nc = 4;  // k, Tdot - f, k dT/dx, k dT/dy
  const int64_t outb = K == 4 ? P->nnz + P->n_rows : NACC * P->nnz;
  KTimer tm(names[K], 8 * (2 * N * sum_r + nc * P->n_points + outb), st);
  k_assemble<K><<<(unsigned)(per_xcd * NXCD), WAVE, lds, st>>>(
      P->n_rows, P->n_tiles, per_xcd, P->max_tile_nnz, P->max_tile_mem, nd_cap, nw_cap, P->tile_eptr.as<int64_t>(),
      P->tile_ent.as<int4>(), P->tile_mem.as<int2>(), P->supp_ptr.as<int64_t>(), P->slot.as<uint8_t>(),
      P->row_ptr.as<int64_t>(), S, o0, o1);
  tm.stop();
  WQ_HIP(hipGetLastError());
  return WQ_OK;
}

wq_status check(const wq_points* P, const wq_weights* w, unsigned need, const void* out, wq_precision prec) {
  WQ_CHECK(P && w && out && w->pts == P, WQ_EINVAL, "assemble: bad arguments");
  WQ_CHECK((w->fam_mask & need) == need, WQ_EINVAL, "assemble: weights for a needed family were not solved");
  WQ_CHECK(prec == WQ_FP64, WQ_EINVAL, "assemble: precision not available in this entry point");
  return WQ_OK;
}

Src src_coef(const double* c0, const double* c1) {
  Src S{};
  S.C[0] = c0;
  S.C[1] = c1;
  return S;
}

// ------------------------------------------------------------------ tangent point fields
// Thermal conductivity k(u) (Section 6.3 uses 1, e^{-T}, sin(pi T), 200 - 0.05 T).
__device__ inline double kval(const wq_conductivity& k, double u) {
  switch (k.kind) {
    case WQ_K_LINEAR: return k.a + k.b * u;
    case WQ_K_QUADRATIC: return k.a + k.b * u * u;
    case WQ_K_EXP: return k.a * exp(k.b * u);
    default: return k.a * sin(k.b * u);
  }
}

// One thread per (cell, point): T, Tdot, dT/dx, dT/dy at the point from the cell's
// functions (T(x_q) = sum_j T_j N_j(x_q)); k_q = k(T_q) and the residual point fields.
__global__ void k_point_fields(int32_t ncell, int max_np, const int64_t* __restrict__ cell_pt_off,
                               const int64_t* __restrict__ cfn_ptr, const int32_t* __restrict__ cfn,
                               const int64_t* __restrict__ dptr, const double* __restrict__ DN,
                               const double* __restrict__ DX, const double* __restrict__ DY,
                               const double* __restrict__ T, const double* __restrict__ Td,
                               const double* __restrict__ f, wq_conductivity kc, double* __restrict__ kq,
                               double* __restrict__ p0, double* __restrict__ p1, double* __restrict__ p2) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t c = g / max_np;
  const int q = (int)(g - c * max_np);
  if (c >= ncell) return;
  const int64_t pt0 = cell_pt_off[c];
  const int np = (int)(cell_pt_off[c + 1] - pt0);
  if (q >= np) return;
  const int64_t f0 = cfn_ptr[c];
  const int m = (int)(cfn_ptr[c + 1] - f0);
  const int64_t d = dptr[c] + (int64_t)q * m;
  double u = 0.0, ud = 0.0, ux = 0.0, uy = 0.0;
  for (int k = 0; k < m; ++k) {
    const int32_t j = cfn[f0 + k];
    const double tj = T[j];
    u += tj * DN[d + k];
    ud += Td[j] * DN[d + k];
    ux += tj * DX[d + k];
    uy += tj * DY[d + k];
  }
  const int64_t pt = pt0 + q;
  const double kk = kval(kc, u);
  kq[pt] = kk;
  p0[pt] = ud - (f ? f[pt] : 0.0);
  p1[pt] = kk * ux;
  p2[pt] = kk * uy;
}

}  // namespace

extern "C" wq_status assemble_mass(const wq_points* P, const wq_weights* w, const double* c, void* vals,
                                   wq_precision prec, wq_stream stream) {
  WQ_TRY(check(P, w, WQ_FAM_MASS, vals, prec));
  return launch<0>(P, w, src_coef(c, nullptr), (double*)vals, nullptr, (hipStream_t)stream);
}

extern "C" wq_status assemble_stiffness(const wq_points* P, const wq_weights* w, const double* k, void* vals,
                                        wq_precision prec, wq_stream stream) {
  WQ_TRY(check(P, w, WQ_FAM_DX | WQ_FAM_DY, vals, prec));
  return launch<1>(P, w, src_coef(k, nullptr), (double*)vals, nullptr, (hipStream_t)stream);
}

extern "C" wq_status assemble_biharmonic(const wq_points* P, const wq_weights* w, const double* d, void* vals,
                                         wq_precision prec, wq_stream stream) {
  WQ_TRY(check(P, w, WQ_FAM_LAP, vals, prec));
  WQ_CHECK(P->has_lap, WQ_EINVAL, "assemble_biharmonic: build_points without Laplacians");
  return launch<2>(P, w, src_coef(d, nullptr), (double*)vals, nullptr, (hipStream_t)stream);
}

extern "C" wq_status assemble_mass_stiffness(const wq_points* P, const wq_weights* w, const double* c,
                                             const double* k, void* mv, void* kv, wq_precision prec,
                                             wq_stream stream) {
  WQ_TRY(check(P, w, WQ_FAM_MASS | WQ_FAM_DX | WQ_FAM_DY, mv, prec));
  WQ_CHECK(kv, WQ_EINVAL, "assemble_mass_stiffness: null stiffness output");
  return launch<3>(P, w, src_coef(c, k), (double*)mv, (double*)kv, (hipStream_t)stream);
}

extern "C" wq_status assemble_tangent(const wq_points* P, const wq_weights* w, const double* T, const double* Tdot,
                                      double inv_theta_dt, wq_conductivity k, const double* f_at_pts, void* S_vals,
                                      double* R, wq_precision prec, wq_stream stream) {
  WQ_TRY(check(P, w, WQ_FAM_MASS | WQ_FAM_DX | WQ_FAM_DY, S_vals, prec));
  WQ_CHECK(T && Tdot && R, WQ_EINVAL, "assemble_tangent: null T, Tdot or R");
  WQ_CHECK(k.kind >= WQ_K_LINEAR && k.kind <= WQ_K_SIN, WQ_EINVAL, "assemble_tangent: unknown conductivity kind");
  WQ_CHECK(std::isfinite(inv_theta_dt), WQ_EINVAL, "assemble_tangent: 1/(theta dt) not finite");
  hipStream_t st = (hipStream_t)stream;
  wq_points* Pm = const_cast<wq_points*>(P);
  if (Pm->tangent_ws.bytes < 4 * (size_t)P->n_points * sizeof(double))
    WQ_TRY(dalloc_n<double>(Pm->tangent_ws, 4 * (size_t)P->n_points));
  double* kq = Pm->tangent_ws.as<double>();
  double* p0 = kq + P->n_points;
  double* p1 = p0 + P->n_points;
  double* p2 = p1 + P->n_points;
  const int mnp = P->max_cell_np;
  {
    KTimer tm("k_point_fields", P->n_points, st);
    k_point_fields<<<nblocks((int64_t)P->ncell * mnp, 256), 256, 0, st>>>(
        P->ncell, mnp, P->cell_pt_off.as<int64_t>(), P->cfn_ptr.as<int64_t>(), P->cfn.as<int32_t>(),
        P->dptr.as<int64_t>(), P->DN.as<double>(), P->DX.as<double>(), P->DY.as<double>(), T, Tdot, f_at_pts, k, kq,
        p0, p1, p2);
    tm.stop();
    WQ_HIP(hipGetLastError());
  }
  Src S = src_coef(kq, nullptr);
  S.scale = inv_theta_dt;
  S.Pf[0] = p0;
  S.Pf[1] = p1;
  S.Pf[2] = p2;
  return launch<4>(P, w, S, (double*)S_vals, R, st);
}
