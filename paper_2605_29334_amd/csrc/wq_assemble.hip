// Row-wise WQ assembly (Eqs. (9), (11), (12)); Section 6.1 forms the matrix row by row.
// The tangent of the nonlinear heat problem (Eq. (36)) and its residual use the same
// kernel with the conductivity evaluated at the points.
#include "wq_internal.h"

#include <cmath>
#include <cstring>

using namespace wq;

namespace {

constexpr int WAVE = 64;
constexpr int NXCD = 8;    // MI355X: workgroups are dispatched round-robin over 8 XCDs

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
constexpr int DEPTH = 2;  // cell entries in flight per wavefront

// Entry e of a tile: cell block at d0, points pt0.., np points, m functions; member rows
// are the set bits of the row mask (bits 0..15), their records at smem[mb ..] in row order.
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
__global__ void __launch_bounds__(WAVE) k_assemble(int64_t n, int64_t n_tiles, int64_t chunk, int acc_stride,
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
  // the tile's entry records (16-byte aligned after the member records): decoding an entry
  // then waits on LDS, not on a global load ahead of the entry's own loads
  int4* sent = (int4*)(((uintptr_t)(smem + mem_cap) + 15) & ~(uintptr_t)15);
  const int64_t b = blockIdx.x;
  const int64_t turn = b / NXCD;
  const int64_t tile = (turn / chunk) * (NXCD * chunk) + (b % NXCD) * chunk + turn % chunk;
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
  for (int t = lane; t < ne; t += WAVE) sent[t] = ent[e0 + t];
  __syncthreads();
  // Entries are pipelined DEPTH deep: while entry e is computed from the LDS stage, the
  // loads of entries e+1 .. e+DEPTH-1 are in flight in registers (ring slot e % DEPTH).
  if (ne > 0) {
    Pre<K> p[DEPTH];
    Ent en[DEPTH];
#pragma unroll
    for (int u = 0; u < DEPTH; ++u)
      if (u < ne) {
        en[u] = decode(sent[u], m0);
        prefetch<K>(en[u], lane, S, smem, slot, p[u]);
      }
    stage<K>(en[0], lane, S, smem, p[0], sd, nd_cap, sw, nw_cap, rho);
    __syncthreads();
    for (int eb = 0; eb < ne; eb += DEPTH) {
#pragma unroll
      for (int u = 0; u < DEPTH; ++u) {
        const int e = eb + u;
        if (e < ne) {
          const Ent& cur = en[u];
          const int ns = cur.R * cur.m;
#pragma unroll
          for (int v = 0; v < PFS; ++v) {
            const int t = lane + WAVE * v;
            if (t < ns) accumulate<K>(cur, t, p[u].s[v], p[u].rl[v], sd, nd_cap, sw, nw_cap, ro, acc, acc_stride);
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
          const int un = (u + 1) % DEPTH;
          if (e + 1 < ne) stage<K>(en[un], lane, S, smem, p[un], sd, nd_cap, sw, nw_cap, rho);
          if (e + DEPTH < ne) {  // slot u is free: start entry e + DEPTH
            en[u] = decode(sent[e + DEPTH], m0);
            prefetch<K>(en[u], lane, S, smem, slot, p[u]);
          }
          __syncthreads();
        }
      }
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
                     (size_t)P->max_tile_mem * sizeof(int2) + 16 + (size_t)P->max_tile_ent * sizeof(int4);
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
  // workgroup b runs on XCD b % 8 and takes, in turn, chunks of `chunk` consecutive tiles
  // (L2 reuse between neighbouring rows on one XCD); the grid covers whole rounds of
  // 8 * chunk tiles and blocks past the end exit
  const int64_t chunk = P->asm_chunk;
  const int64_t per_xcd = ((P->n_tiles + NXCD * chunk - 1) / (NXCD * chunk)) * chunk;
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
      P->n_rows, P->n_tiles, chunk, P->max_tile_nnz, P->max_tile_mem, nd_cap, nw_cap, P->tile_eptr.as<int64_t>(),
      P->tile_ent.as<int4>(), P->tile_mem.as<int2>(), P->supp_ptr.as<int64_t>(), P->slot.as<uint8_t>(),
      P->row_ptr.as<int64_t>(), S, o0, o1);
  tm.stop();
  WQ_HIP(hipGetLastError());
  return WQ_OK;
}

wq_status check(const wq_points* P, const wq_weights* w, unsigned need, const void* out, wq_precision prec) {
  WQ_CHECK(P && w && out && w->pts == P, WQ_EINVAL, "assemble: bad arguments");
  WQ_CHECK((w->fam_mask & need) == need, WQ_EINVAL, "assemble: weights for a needed family were not solved");
  WQ_CHECK(prec == WQ_FP64 || prec == WQ_SPLIT_FP16 || prec == WQ_SPLIT_BF16 || prec == WQ_SLICED_FP16, WQ_EINVAL,
           "assemble: unknown precision");
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

// ------------------------------------------------------------------ split precision
// The row contraction V[j][k] = sum_q (w c)_{jq} D_k(x_q) of a cell entry is a small
// GEMM (members x points) x (points x functions); here it runs on MFMA with operands
// split into low-precision terms and FP32 accumulation:
//   FP16 x 2: a = 2^ea (a_hi + a_lo), b = 2^eb (b_hi + b_lo), ab ~ a_hi b_hi + a_hi b_lo
//             + a_lo b_hi (dropped a_lo b_lo ~ 2^-22 relative); ea per member row and
//             entry (the row's largest |w c| is scaled into [1/2, 1)), eb per family;
//   BF16 x 3: a = a_hi + a_mid + a_lo (24 bits, FP32 range, no scaling), six products
//             (all with combined weight above 2^-24).
// Each entry's FP32 result is scaled back and added into FP64 LDS accumulators (fixed
// order as in the FP64 kernel); the CSR values are stored as FP32.
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// fp32 -> bf16 bits, round to nearest even (inputs are finite)
__host__ __device__ inline uint16_t bf16_bits(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_val(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

struct Split3 {
  uint16_t h, m, l;
};
__device__ inline Split3 split_bf16(double x) {
  Split3 s;
  s.h = bf16_bits((float)x);
  const double r1 = x - (double)bf16_val(s.h);
  s.m = bf16_bits((float)r1);
  const double r2 = r1 - (double)bf16_val(s.m);
  s.l = bf16_bits((float)r2);
  return s;
}

// packed basis values; FP16: value scaled by 2^-e (e per family)
__global__ void k_split_basis(int64_t n, const double* __restrict__ D, int e, int prec, uint32_t* __restrict__ out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double x = D[t];
  if (prec == WQ_SPLIT_FP16) {
    const double y = ldexp(x, -e);
    const _Float16 hi = (_Float16)(float)y;
    const _Float16 lo = (_Float16)(float)(y - (double)(float)hi);
    out[t] = (uint32_t)__builtin_bit_cast(uint16_t, hi) | ((uint32_t)__builtin_bit_cast(uint16_t, lo) << 16);
  } else {
    const Split3 s = split_bf16(x);
    out[2 * t] = (uint32_t)s.h | ((uint32_t)s.m << 16);
    out[2 * t + 1] = (uint32_t)s.l;
  }
}

__global__ void k_absmax(int64_t n, const double* __restrict__ D, unsigned long long* out) {
  double m = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, fabs(D[t]));
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

wq_status prepare_split(wq_points* P, wq_precision prec, hipStream_t st) {
  if (P->ds_prec == (int)prec) return WQ_OK;
  const DBuf* src[4] = {&P->DN, &P->DX, &P->DY, P->has_lap ? &P->DL : nullptr};
  const int64_t n = P->n_basis;
  DBuf mx;
  WQ_TRY(dalloc_n<unsigned long long>(mx, 4));
  WQ_HIP(hipMemsetAsync(mx.p, 0, 4 * sizeof(unsigned long long), st));
  for (int f = 0; f < 4; ++f)
    if (src[f]) k_absmax<<<1024, 256, 0, st>>>(n, src[f]->as<double>(), mx.as<unsigned long long>() + f);
  unsigned long long hm[4];
  WQ_HIP(hipMemcpyAsync(hm, mx.p, sizeof(hm), hipMemcpyDeviceToHost, st));
  WQ_HIP(hipStreamSynchronize(st));
  dfree(mx);
  for (int f = 0; f < 4; ++f) {
    dfree(P->DS[f]);
    if (!src[f]) continue;
    double m;
    std::memcpy(&m, &hm[f], sizeof(m));
    int e = 0;
    if (m > 0) (void)std::frexp(m, &e);  // m = f 2^e, f in [1/2, 1)
    P->ds_exp[f] = prec == WQ_SPLIT_FP16 ? e : 0;
    WQ_TRY(dalloc_n<uint32_t>(P->DS[f], (prec == WQ_SPLIT_FP16 ? 1 : 2) * (size_t)n));
    k_split_basis<<<nblocks(n, 256), 256, 0, st>>>(n, src[f]->as<double>(), P->ds_exp[f], (int)prec,
                                                    P->DS[f].as<uint32_t>());
    WQ_HIP(hipGetLastError());
  }
  P->ds_prec = (int)prec;
  return WQ_OK;
}

struct SrcS {
  const uint32_t* D[3];
  const double* W[3];
  const double* C[2];
  int eb[3];
};

// Sliced operand: x in (-1, 1) as sum_i k_i 2^{-10 (i + 1)}, integers |k_i| <= 1024 held
// exactly in FP16 (the steps are exact in FP64: scaling by 2^10 and removing the rounded
// integer part).
__device__ inline void slice4(double x, _Float16 k[4]) {
  for (int i = 0; i < 4; ++i) {
    const double y = x * 1024.0;
    const double r = rint(y);
    k[i] = (_Float16)(float)r;
    x = y - r;
  }
}

// Error-free sliced product: the k_i k'_j of a 16x16x16 MFMA are integers below 2^20
// and at most 16 are summed per output, so each FP32 sum is exact; pairs with
// i + j = s share accumulator s (s <= 3). Exponents: ea per member row (shared along the
// points), eb per function column (shared along the points). Returns the FP64 result
// for the lane's four outputs, scaled back.
__device__ inline void contract_sliced(const double* sw, const double* sd, int R, int np, int m, int cb, int lane,
                                       double out[4]) {
  const int j = lane & 15, g = lane >> 4;
  const int k = (lane & 15) + 16 * cb;
  double mxa = 0.0, mxb = 0.0;
  for (int q = 4 * g; q < np; q += 16)
    for (int i = 0; i < 4 && q + i < np; ++i) {
      if (j < R) mxa = fmax(mxa, fabs(sw[j * np + q + i]));
      if (k < m) mxb = fmax(mxb, fabs(sd[(q + i) * m + k]));
    }
  mxa = fmax(mxa, __shfl_xor(mxa, 16, 64));
  mxa = fmax(mxa, __shfl_xor(mxa, 32, 64));
  mxb = fmax(mxb, __shfl_xor(mxb, 16, 64));
  mxb = fmax(mxb, __shfl_xor(mxb, 32, 64));
  int ea = 0, eb = 0;
  if (mxa > 0) (void)frexp(mxa, &ea);
  if (mxb > 0) (void)frexp(mxb, &eb);
  f4 c[4];
  for (int s = 0; s < 4; ++s) c[s] = f4{0.f, 0.f, 0.f, 0.f};
  for (int kc = 0; kc < np; kc += 16) {
    h4 a[4], b[4];
    for (int i = 0; i < 4; ++i) {
      const int q = kc + 4 * g + i;
      _Float16 ka[4], kb[4];
      slice4((j < R && q < np) ? ldexp(sw[j * np + q], -ea) : 0.0, ka);
      slice4((k < m && q < np) ? ldexp(sd[q * m + k], -eb) : 0.0, kb);
      for (int t = 0; t < 4; ++t) {
        a[t][i] = ka[t];
        b[t][i] = kb[t];
      }
    }
    c[0] = __builtin_amdgcn_mfma_f32_16x16x16f16(a[0], b[0], c[0], 0, 0, 0);
    c[1] = __builtin_amdgcn_mfma_f32_16x16x16f16(a[0], b[1], c[1], 0, 0, 0);
    c[1] = __builtin_amdgcn_mfma_f32_16x16x16f16(a[1], b[0], c[1], 0, 0, 0);
    c[2] = __builtin_amdgcn_mfma_f32_16x16x16f16(a[0], b[2], c[2], 0, 0, 0);
    c[2] = __builtin_amdgcn_mfma_f32_16x16x16f16(a[1], b[1], c[2], 0, 0, 0);
    c[2] = __builtin_amdgcn_mfma_f32_16x16x16f16(a[2], b[0], c[2], 0, 0, 0);
    c[3] = __builtin_amdgcn_mfma_f32_16x16x16f16(a[0], b[3], c[3], 0, 0, 0);
    c[3] = __builtin_amdgcn_mfma_f32_16x16x16f16(a[1], b[2], c[3], 0, 0, 0);
    c[3] = __builtin_amdgcn_mfma_f32_16x16x16f16(a[2], b[1], c[3], 0, 0, 0);
    c[3] = __builtin_amdgcn_mfma_f32_16x16x16f16(a[3], b[0], c[3], 0, 0, 0);
  }
  for (int i = 0; i < 4; ++i) {
    const int eaj = __shfl(ea, 4 * g + i, 64);
    const double v = (double)c[0][i] + ldexp((double)c[1][i], -10) + ldexp((double)c[2][i], -20) +
                     ldexp((double)c[3][i], -30);
    out[i] = ldexp(v, eaj + eb - 20);
  }
}

// MFMA 16x16x16 lane layout (A: M x K, B: K x N, C: M x N, 64 lanes, g = lane / 16):
// lane holds A[lane % 16][4g + i], B[4g + i][lane % 16], C[4g + i][lane % 16], i < 4.
template <int PREC>
__device__ inline f4 contract_split(const double* sw, int nw_cap, const uint32_t* sd, int nd_cap, int R, int np, int m,
                                    int cb, int lane, int* ea_out) {
  const int j = lane & 15, g = lane >> 4;
  const int k = (lane & 15) + 16 * cb;
  f4 c = {0.f, 0.f, 0.f, 0.f};
  // row scale (FP16): the largest |w c| of member row j over all points of the cell
  int ea = 0;
  if (PREC == WQ_SPLIT_FP16) {
    double mx = 0.0;
    if (j < R)
      for (int q = 4 * g; q < np; q += 16)
        for (int i = 0; i < 4 && q + i < np; ++i) mx = fmax(mx, fabs(sw[j * np + q + i]));
    mx = fmax(mx, __shfl_xor(mx, 16, 64));
    mx = fmax(mx, __shfl_xor(mx, 32, 64));
    if (mx > 0) (void)frexp(mx, &ea);
  }
  *ea_out = ea;
  for (int kc = 0; kc < np; kc += 16) {
    if (PREC == WQ_SPLIT_FP16) {
      h4 ah, al, bh, bl;
      for (int i = 0; i < 4; ++i) {
        const int q = kc + 4 * g + i;
        const double x = (j < R && q < np) ? ldexp(sw[j * np + q], -ea) : 0.0;
        const _Float16 hi = (_Float16)(float)x;
        ah[i] = hi;
        al[i] = (_Float16)(float)(x - (double)(float)hi);
        const uint32_t v = (k < m && q < np) ? sd[q * m + k] : 0u;
        bh[i] = __builtin_bit_cast(_Float16, (uint16_t)(v & 0xffffu));
        bl[i] = __builtin_bit_cast(_Float16, (uint16_t)(v >> 16));
      }
      c = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, bh, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, bl, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x16f16(al, bh, c, 0, 0, 0);
    } else {
      s4 ah, am, al, bh, bm, bl;
      for (int i = 0; i < 4; ++i) {
        const int q = kc + 4 * g + i;
        const Split3 a = (j < R && q < np) ? split_bf16(sw[j * np + q]) : Split3{0, 0, 0};
        ah[i] = (short)a.h;
        am[i] = (short)a.m;
        al[i] = (short)a.l;
        uint32_t v0 = 0u, v1 = 0u;
        if (k < m && q < np) {
          v0 = sd[2 * (q * m + k)];
          v1 = sd[2 * (q * m + k) + 1];
        }
        bh[i] = (short)(v0 & 0xffffu);
        bm[i] = (short)(v0 >> 16);
        bl[i] = (short)(v1 & 0xffffu);
      }
      // smallest terms first
      c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(am, bm, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bm, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(am, bh, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, c, 0, 0, 0);
    }
  }
  return c;
}

// The FP64 tile kernel's structure (row tiles, cell entries in order, LDS stage),
// with the per-entry contraction on MFMA. K = 0 mass, 1 stiffness, 2 biharmonic,
// 3 mass + stiffness. Output FP32.
template <int K, int PREC>
__global__ void __launch_bounds__(WAVE) k_assemble_split(int64_t n, int64_t n_tiles, int64_t chunk, int acc_stride,
                                                         int nd_cap, int nw_cap, const int64_t* __restrict__ eptr,
                                                         const int4* __restrict__ ent, const int2* __restrict__ mem,
                                                         const int64_t* __restrict__ sptr,
                                                         const uint8_t* __restrict__ slot,
                                                         const int64_t* __restrict__ row_ptr, SrcS S,
                                                         float* __restrict__ out0, float* __restrict__ out1) {
  constexpr int N = Fam<K>::N;
  constexpr int NACC = Fam<K>::NACC;
  constexpr int VW = PREC == WQ_SPLIT_FP16 ? 1 : 2;  // uint32 words per basis value (sliced: FP64)
  extern __shared__ double acc[];
  __shared__ int ro[TILE_ROWS + 1];
  double* sw = acc + NACC * acc_stride;
  uint32_t* sd = (uint32_t*)(sw + N * nw_cap);
  int2* smem = (int2*)(sd + ((N * nd_cap * VW + 1) & ~1));
  const int64_t b = blockIdx.x;
  const int64_t turn = b / NXCD;
  const int64_t tile = (turn / chunk) * (NXCD * chunk) + (b % NXCD) * chunk + turn % chunk;
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
  for (int t = lane; t < NACC * acc_stride; t += WAVE) acc[t] = 0.0;
  for (int t = lane; t < nm; t += WAVE) smem[t] = mem[m0 + t];
  __syncthreads();
  for (int e = 0; e < ne; ++e) {
    const Ent E = decode(ent[e0 + e], m0);
    const int nd = E.np * E.m, nw = E.R * E.np;
    // stage: packed basis block per family, (w c) per family (FP64)
    for (int t = lane; t < nd * VW; t += WAVE)
      for (int a = 0; a < N; ++a) sd[a * nd_cap * VW + t] = S.D[a][E.d0 * VW + t];
    for (int t = lane; t < nw; t += WAVE) {
      const int j = qdiv(t, E.rnp), q = t - j * E.np;
      const int64_t qo = smem[E.mb + j].x & ((1 << 28) - 1);
      for (int a = 0; a < N; ++a) {
        const double* C = S.C[Fam<K>::cof(a)];
        sw[a * nw_cap + t] = S.W[a][qo + q] * (C ? C[E.pt0 + q] : 1.0);
      }
    }
    __syncthreads();
    for (int cb = 0; cb * 16 < E.m; ++cb) {
      double v0[4] = {0, 0, 0, 0}, v1[4] = {0, 0, 0, 0};
      for (int a = 0; a < N; ++a) {
        double v[4];
        if (PREC == WQ_SLICED_FP16) {
          contract_sliced(sw + a * nw_cap, (const double*)(sd + a * nd_cap * VW), E.R, E.np, E.m, cb, lane, v);
        } else {
          int ea;
          const f4 c = contract_split<PREC>(sw + a * nw_cap, nw_cap, sd + a * nd_cap * VW, nd_cap, E.R, E.np, E.m, cb,
                                            lane, &ea);
          const int g = lane >> 4;
          for (int i = 0; i < 4; ++i) v[i] = ldexp((double)c[i], __shfl(ea, 4 * g + i, 64) + S.eb[a]);
        }
        for (int i = 0; i < 4; ++i) {
          if (K == 3 && a > 0) v1[i] += v[i];
          else v0[i] += v[i];
        }
      }
      const int k = (lane & 15) + 16 * cb;
      for (int i = 0; i < 4; ++i) {
        const int j = 4 * (lane >> 4) + i;
        if (j < E.R && k < E.m) {
          const int2 mm = smem[E.mb + j];
          const int at = ro[(unsigned)mm.x >> 28] + slot[(uint32_t)mm.y + k];
          acc[at] += v0[i];
          if (K == 3) acc[acc_stride + at] += v1[i];
        }
      }
    }
    __syncthreads();
  }
  for (int t = lane; t < nz; t += WAVE) {
    out0[a0 + t] = (float)acc[t];
    if (K == 3) out1[a0 + t] = (float)acc[acc_stride + t];
  }
}

template <int K, int PREC>
wq_status launch_split(const wq_points* P, const wq_weights* w, const double* c0, const double* c1, float* o0,
                       float* o1, hipStream_t st) {
  constexpr int N = Fam<K>::N;
  constexpr int NACC = Fam<K>::NACC;
  constexpr int VW = PREC == WQ_SPLIT_FP16 ? 1 : 2;
  if (PREC != WQ_SLICED_FP16) WQ_TRY(prepare_split(const_cast<wq_points*>(P), (wq_precision)PREC, st));
  const int nd_cap = P->max_tile_nd, nw_cap = P->max_tile_nw;
  const size_t lds = (size_t)NACC * P->max_tile_nnz * sizeof(double) + (size_t)N * nw_cap * sizeof(double) +
                     (size_t)((N * nd_cap * VW + 1) & ~1) * sizeof(uint32_t) + (size_t)P->max_tile_mem * sizeof(int2);
  WQ_CHECK(lds <= 150 * 1024, WQ_EINVAL, "assemble: tile accumulators and stage exceed LDS");
  WQ_CHECK(nw_cap < 4096 && (int64_t)TILE_ROWS * 255 < 4096, WQ_EINVAL, "assemble: entry too large");
  SrcS S{};
  S.C[0] = c0;
  S.C[1] = c1;
  const int fam[4][3] = {{0, -1, -1}, {1, 2, -1}, {3, -1, -1}, {0, 1, 2}};
  const DBuf* D64[4] = {&P->DN, &P->DX, &P->DY, &P->DL};
  for (int a = 0; a < N; ++a) {
    const int f = fam[K][a];
    S.D[a] = PREC == WQ_SLICED_FP16 ? D64[f]->as<uint32_t>() : P->DS[f].as<uint32_t>();
    S.W[a] = w->W[f].as<double>();
    S.eb[a] = PREC == WQ_SLICED_FP16 ? 0 : P->ds_exp[f];
  }
  const int64_t chunk = P->asm_chunk;
  const int64_t per_xcd = ((P->n_tiles + NXCD * chunk - 1) / (NXCD * chunk)) * chunk;
  static const char* names[3][4] = {{"k_assemble_mass_fp16x2", "k_assemble_stiffness_fp16x2",
                                     "k_assemble_biharmonic_fp16x2", "k_assemble_mass_stiffness_fp16x2"},
                                    {"k_assemble_mass_bf16x3", "k_assemble_stiffness_bf16x3",
                                     "k_assemble_biharmonic_bf16x3", "k_assemble_mass_stiffness_bf16x3"},
                                    {"k_assemble_mass_sliced", "k_assemble_stiffness_sliced",
                                     "k_assemble_biharmonic_sliced", "k_assemble_mass_stiffness_sliced"}};
  if (lds > 64 * 1024)
    WQ_HIP(hipFuncSetAttribute((const void*)k_assemble_split<K, PREC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
  const int64_t sum_r = (int64_t)(P->qidx.bytes / sizeof(int32_t));
  const int64_t nc = (c0 ? 1 : 0) + (K == 3 && c1 ? 1 : 0);
  KTimer tm(names[PREC - 1][K], N * sum_r * (4 * VW + 8) + 8 * nc * P->n_points + 4 * NACC * P->nnz, st);
  k_assemble_split<K, PREC><<<(unsigned)(per_xcd * NXCD), WAVE, lds, st>>>(
      P->n_rows, P->n_tiles, chunk, P->max_tile_nnz, nd_cap, nw_cap, P->tile_eptr.as<int64_t>(),
      P->tile_ent.as<int4>(), P->tile_mem.as<int2>(), P->supp_ptr.as<int64_t>(), P->slot.as<uint8_t>(),
      P->row_ptr.as<int64_t>(), S, o0, o1);
  tm.stop();
  WQ_HIP(hipGetLastError());
  return WQ_OK;
}

template <int K>
wq_status dispatch(const wq_points* P, const wq_weights* w, const double* c0, const double* c1, void* o0, void* o1,
                   wq_precision prec, hipStream_t st) {
  if (prec == WQ_FP64) return launch<K>(P, w, src_coef(c0, c1), (double*)o0, (double*)o1, st);
  if (prec == WQ_SPLIT_FP16) return launch_split<K, WQ_SPLIT_FP16>(P, w, c0, c1, (float*)o0, (float*)o1, st);
  if (prec == WQ_SPLIT_BF16) return launch_split<K, WQ_SPLIT_BF16>(P, w, c0, c1, (float*)o0, (float*)o1, st);
  return launch_split<K, WQ_SLICED_FP16>(P, w, c0, c1, (float*)o0, (float*)o1, st);
}

}  // namespace

extern "C" wq_status assemble_mass(const wq_points* P, const wq_weights* w, const double* c, void* vals,
                                   wq_precision prec, wq_stream stream) {
  WQ_TRY(check(P, w, WQ_FAM_MASS, vals, prec));
  return dispatch<0>(P, w, c, nullptr, vals, nullptr, prec, (hipStream_t)stream);
}

extern "C" wq_status assemble_stiffness(const wq_points* P, const wq_weights* w, const double* k, void* vals,
                                        wq_precision prec, wq_stream stream) {
  WQ_TRY(check(P, w, WQ_FAM_DX | WQ_FAM_DY, vals, prec));
  return dispatch<1>(P, w, k, nullptr, vals, nullptr, prec, (hipStream_t)stream);
}

extern "C" wq_status assemble_biharmonic(const wq_points* P, const wq_weights* w, const double* d, void* vals,
                                         wq_precision prec, wq_stream stream) {
  WQ_TRY(check(P, w, WQ_FAM_LAP, vals, prec));
  WQ_CHECK(P->has_lap, WQ_EINVAL, "assemble_biharmonic: build_points without Laplacians");
  return dispatch<2>(P, w, d, nullptr, vals, nullptr, prec, (hipStream_t)stream);
}

extern "C" wq_status assemble_mass_stiffness(const wq_points* P, const wq_weights* w, const double* c,
                                             const double* k, void* mv, void* kv, wq_precision prec,
                                             wq_stream stream) {
  WQ_TRY(check(P, w, WQ_FAM_MASS | WQ_FAM_DX | WQ_FAM_DY, mv, prec));
  WQ_CHECK(kv, WQ_EINVAL, "assemble_mass_stiffness: null stiffness output");
  return dispatch<3>(P, w, c, k, mv, kv, prec, (hipStream_t)stream);
}

extern "C" wq_status assemble_tangent(const wq_points* P, const wq_weights* w, const double* T, const double* Tdot,
                                      double inv_theta_dt, wq_conductivity k, const double* f_at_pts, void* S_vals,
                                      double* R, wq_precision prec, wq_stream stream) {
  WQ_TRY(check(P, w, WQ_FAM_MASS | WQ_FAM_DX | WQ_FAM_DY, S_vals, prec));
  WQ_CHECK(prec == WQ_FP64, WQ_EINVAL, "assemble_tangent: the Newton tangent and residual are FP64 only");
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
