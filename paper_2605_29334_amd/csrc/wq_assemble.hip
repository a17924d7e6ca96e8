// Row-wise WQ assembly (Eqs. (9), (11), (12)); Section 6.1 forms the matrix row by row.
// The tangent of the nonlinear heat problem (Eq. (36)) and its residual use the same
// kernel with the conductivity evaluated at the points.
#include "wq_internal.h"

#include <cmath>
#include <cstring>
#include <mutex>

using namespace wq;

namespace {

constexpr int WAVE = 64;
constexpr int NXCD = 8;    // MI355X: workgroups are dispatched round-robin over 8 XCDs

// Families per kernel: K = 0 mass, 1 stiffness, 2 biharmonic, 3 mass + stiffness,
// 4 tangent (Eq. (36)) + residual, 5 exact tangent (Eq. (34): Eq. (36) plus the
// non-symmetric term k'(T) N_j grad T . grad N_i) + residual.
// N basis arrays (N or Delta N; dN/dx, dN/dy) and as many weight families; weight family
// a is scaled by the coefficient array cof(a) (or, for the tangent's mass term, by the
// constant 1/(theta dt)).
template <int K> struct Fam {
  static constexpr int N = (K >= 3) ? 3 : (K == 1 ? 2 : 1);
  static constexpr int NACC = (K == 3) ? 2 : 1;
  static constexpr int NC = (K == 3) ? 2 : 1;
  static constexpr bool RES = (K >= 4);
  static constexpr bool EXACT = (K == 5);
  static constexpr int NPF = RES ? (EXACT ? 5 : 3) : 1;  // point fields read by the kernel
  __device__ static constexpr int cof(int a) { return (K == 3 && a > 0) ? 1 : 0; }
  // tangent: mass term scaled by a constant, conductivity terms by C[0]
  __device__ static constexpr bool constant(int a) { return K >= 4 && a == 0; }
};

struct Src {
  const double* D[3];   // basis blocks, point-major per cell: D[d0 + q * m + k]
  const double* W[3];   // weights aligned with Q_i
  const double* C[2];   // coefficients at the points (nullptr: 1)
  double scale;         // tangent: 1 / (theta dt) on the mass term
  const double* Pf[5];  // tangent point fields: Tdot - f, k dT/dx, k dT/dy (residual);
                        // k' dT/dx, k' dT/dy (non-symmetric term of the exact tangent)
};

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

// ------------------------------------------------------------------ cell-major MFMA kernel
// One wavefront owns a tile of up to 16 consecutive rows; its CSR values are accumulated in
// LDS. It visits the cells of the tile rows' supports once each, in ascending order. For a
// cell with np points and m functions, the contribution to member row i and cell function
// k is P[k][i] = sum_q D_k(x_q) (w_iq coef_q): the cell's basis block (transposed, m x np)
// times the member rows' weights (np x 16), on the FP64 MFMA 16 x 16 x 4, one step per 4
// points and 16 functions. The A operand of a step is one row of the point-major basis
// block (a coalesced load), the B operand the rows' weights (each row's weights on a cell
// are consecutive). Lane (row r = lane % 16, g = lane / 16) then holds P for its own row and
// functions g, g + 4, g + 8, g + 12 of the block (register v holds output row 4 v + g of the
// MFMA) and adds them to the row's CSR slots in LDS (the (row, cell) pair's slot map, stored
// so that those four slots are one dword). Every row receives its cells' contributions in ascending
// cell order, and a row's contribution depends on that row's weights only: the values do
// not depend on which rows share a tile (a mesh gives the same bits alone and in a batch).
// No global atomics; LDS adds are to distinct slots within an instruction.
// The steps of a tile run as a pipeline: the loads of the next STEPS - 1 steps are in
// flight while one is multiplied and scattered. Every load is a buffer load; lanes with
// nothing to load use an offset past the buffer's end, which returns 0 without a memory
// access, so each step issues the same loads and the waits stay static.
// Tangent (K = 4): each lane also sums its row's residual terms over its points; the four
// lanes of a row are added in a fixed order at the end.
typedef double d4 __attribute__((ext_vector_type(4)));
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr uint32_t OOB = 0x80000000u;  // byte offset past the end of every buffer (all < 2 GiB)
constexpr int STEPS = 3;                // pipeline depth (steps in flight per wavefront)

__device__ inline Rsrc make_rsrc(const void* p, int64_t bytes) {
  // raw buffer (stride 0); the range check returns 0 for offsets at or past `bytes`
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, p ? (int)bytes : 0, 0x00020000);
}
__device__ inline double bload64(Rsrc r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ inline uint32_t bload32(Rsrc r, uint32_t off) {
  return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
}

template <int K> struct Bufs {
  Rsrc D[Fam<K>::N], W[Fam<K>::N], C[Fam<K>::NC], Pf[Fam<K>::NPF], slot;
  bool cnull[Fam<K>::NC];
};

// Per-lane constants: MFMA B column / output row r, point group g.
struct Lane {
  int r, g;
  uint32_t lane8, g8;  // lane * 8, g * 8 (byte offsets inside a basis row block / point group)
  uint32_t lowmask;    // rows of the tile below r
  int ro;              // CSR offset of the lane's row inside the tile
};

// A step: entry e (record E), point block ks, function block cb. Uniform. Entries of
// regular cells (4 points, 16 functions: one step) take a short path ("fast").
struct Step {
  int e, ks, cb;
  int4 E;
  bool valid, fast;
};
__device__ inline int st_np(const Step& s) { return (s.E.z >> 16) & 0xff; }
__device__ inline int st_m(const Step& s) { return (int)((unsigned)s.E.z >> 24); }
__device__ inline bool fast_record(const int4& E) { return ((E.z >> 16) & 0xff) == 4 && ((unsigned)E.z >> 24) == 16u; }

__device__ inline int4 uniform_record(const int4* sent, int e) {
  const int4 v = sent[e];
  return make_int4(__builtin_amdgcn_readfirstlane(v.x), __builtin_amdgcn_readfirstlane(v.y),
                   __builtin_amdgcn_readfirstlane(v.z), __builtin_amdgcn_readfirstlane(v.w));
}

// The step after s; entering a new entry moves the lane's weight offset past the points of
// the old cell if its row is a member there.
__device__ inline Step advance(const Step& s, uint32_t& qoff, int r, int ne, const int4* sent) {
  Step n = s;
  if (!s.valid) return n;
  const int np = st_np(s), m = st_m(s);
  if (++n.ks * 4 < np) return n;
  n.ks = 0;
  if (++n.cb * 16 < m) return n;
  n.cb = 0;
  if ((((unsigned)s.E.z >> r) & 1u)) qoff += np;
  if (++n.e < ne) {
    n.E = uniform_record(sent, n.e);
    n.fast = fast_record(n.E);
  } else {
    n.valid = false;
    n.fast = false;
    n.E = make_int4(0, 0, 0, 0);
  }
  return n;
}

template <int K> struct Ops {
  double d[Fam<K>::N], w[Fam<K>::N], c[Fam<K>::NC], pf[Fam<K>::NPF];
  uint32_t sl;
};

__device__ inline double bload64s(Rsrc r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
__device__ inline uint32_t bload32s(Rsrc r, uint32_t voff, uint32_t soff) {
  return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
}

// Issue the loads of one step. Every step issues the same loads in the same order (the
// waits on them stay static); regular cells (4 points x 16 functions: the basis row block
// is one contiguous run, lane = function + 16 point) take their basis offset from the
// record and a lane constant instead of the general index arithmetic.
template <int K>
__device__ inline void fetch(const Step& s, uint32_t qoff, const Lane& L, const Bufs<K>& B, Ops<K>& o) {
  constexpr int N = Fam<K>::N;
  const unsigned mask = (unsigned)s.E.z & 0xffffu;
  const bool mem = (mask >> L.r) & 1u;
  const int np = st_np(s), m = st_m(s);
  const int q = 4 * s.ks + L.g;
  const uint32_t d0 = (uint32_t)s.E.x, pt0 = (uint32_t)s.E.y;
  uint32_t offD, sD;
  if (s.fast) {
    offD = L.lane8;
    sD = d0 * 8u;
  } else {
    const int k = 16 * s.cb + L.r;
    offD = (q < np && k < m) ? (d0 + (uint32_t)(q * m + k)) * 8u : OOB;
    sD = 0u;
  }
  const bool wv = mem && q < np;
  const uint32_t offW = wv ? (qoff + (uint32_t)q) * 8u : OOB;
  const uint32_t offC = wv ? (pt0 + (uint32_t)q) * 8u : OOB;
  const int mpad = (m + 15) & ~15;
  const uint32_t offS = mem ? (uint32_t)(__popc(mask & L.lowmask) * mpad + 16 * s.cb + 4 * L.g) : OOB;
#pragma unroll
  for (int a = 0; a < N; ++a) o.d[a] = bload64s(B.D[a], offD, sD);
#pragma unroll
  for (int a = 0; a < N; ++a) o.w[a] = bload64s(B.W[a], offW, 0u);
#pragma unroll
  for (int a = 0; a < Fam<K>::NC; ++a) o.c[a] = bload64s(B.C[a], offC, 0u);
  if (Fam<K>::RES) {
#pragma unroll
    for (int a = 0; a < Fam<K>::NPF; ++a) o.pf[a] = bload64s(B.Pf[a], offC, 0u);
  }
  o.sl = bload32s(B.slot, offS, (uint32_t)s.E.w);
}

// The products of one step (4 points x 16 functions x the 16 rows of the tile).
template <int K>
__device__ inline void mfma_step(const double (&da)[Fam<K>::N], const double (&wb)[Fam<K>::N], d4& c0, d4& c1) {
  const d4 z = {0.0, 0.0, 0.0, 0.0};
  if (K == 0 || K == 2) {
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(da[0], wb[0], z, 0, 0, 0);
  } else if (K == 1) {
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(da[0], wb[0], z, 0, 0, 0);
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(da[1], wb[1], c0, 0, 0, 0);
  } else if (K == 3) {
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(da[0], wb[0], z, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(da[1], wb[1], z, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(da[2], wb[2], c1, 0, 0, 0);
  } else {
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(da[0], wb[0], z, 0, 0, 0);
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(da[1], wb[1], c0, 0, 0, 0);
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(da[2], wb[2], c0, 0, 0, 0);
  }
}

// Add the lane's four products (functions kb, kb + 4, kb + 8, kb + 12 of its row) to the
// row's CSR slots (four slot bytes in sl). Products of positions past the cell's functions
// are exact zeros (their basis operand is zero) and their slot bytes name some slot of the
// row, so member lanes add all four without a per-function test.
template <int NACC>
__device__ inline void scatter(const d4& c0, const d4& c1, uint32_t sl, bool mem, int ro, double* acc, int nzcap) {
  // The products are moved to ordinary registers before the LDS adds read them: an LDS
  // instruction that read the MFMA's accumulation registers directly was scheduled too
  // soon after the FP64 MFMA on gfx950 and read unfinished sums (the register copies get
  // the full wait).
  double p0[4], p1[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    p0[v] = c0[v];
    asm volatile("" : "+v"(p0[v]));
    if (NACC == 2) {
      p1[v] = c1[v];
      asm volatile("" : "+v"(p1[v]));
    }
  }
  if (mem) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int at = ro + (int)((sl >> (8 * v)) & 0xffu);
      __hip_atomic_fetch_add(acc + at, p0[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
      if (NACC == 2) __hip_atomic_fetch_add(acc + nzcap + at, p1[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
  }
}

// Multiply one step and add its products to the member rows' CSR slots. A cell with more
// than 4 points adds one partial sum per block of 4 points (in block order).
template <int K>
__device__ inline void compute(const Step& s, const Ops<K>& o, const Lane& L, int nzcap, const Src& S,
                               const Bufs<K>& B, double* acc, double& rsum) {
  constexpr int N = Fam<K>::N;
  double wb[N];
#pragma unroll
  for (int a = 0; a < N; ++a) {
    const double cf = B.cnull[Fam<K>::cof(a)] ? 1.0 : o.c[Fam<K>::cof(a)];
    wb[a] = Fam<K>::constant(a) ? o.w[a] * S.scale : o.w[a] * cf;
  }
  // exact tangent: the mass-basis operand also carries k'(T_q) (w^x dT/dx + w^y dT/dy)
  if (Fam<K>::EXACT) wb[0] += o.w[1] * o.pf[3] + o.w[2] * o.pf[4];
  if (Fam<K>::RES && s.cb == 0) rsum += o.w[0] * o.pf[0] + (o.w[N - 2] * o.pf[1] + o.w[N - 1] * o.pf[2]);
  d4 c0, c1;
  mfma_step<K>(o.d, wb, c0, c1);
  const unsigned mask = (unsigned)s.E.z & 0xffffu;
  const bool mem = (mask >> L.r) & 1u;
  scatter<Fam<K>::NACC>(c0, c1, o.sl, mem, L.ro, acc, nzcap);
}

template <int K>
__global__ void __launch_bounds__(WAVE)
    k_asm_mfma(int64_t n_tiles, int64_t chunk, int nzcap, int entcap, const int32_t* __restrict__ trow0,
               const int64_t* __restrict__ teptr, const int4* __restrict__ tent, const uint8_t* __restrict__ tslot,
               int64_t slot_bytes, const int64_t* __restrict__ row_ptr, const int64_t* __restrict__ qptr,
               int64_t basis_bytes, int64_t weight_bytes, int64_t point_bytes, Src S, double* __restrict__ out0,
               double* __restrict__ out1) {
  constexpr int N = Fam<K>::N;
  constexpr int NACC = Fam<K>::NACC;
  constexpr bool RES = Fam<K>::RES;
  extern __shared__ double acc[];
  const int lane = threadIdx.x;
  // workgroup b runs on XCD b % 8; the XCD's workgroups take runs of `chunk` consecutive
  // tiles (L2 reuse of the cells that neighbouring rows share)
  const int64_t b = blockIdx.x;
  const int64_t turn = b / NXCD;
  const int64_t tile = (turn / chunk) * (NXCD * chunk) + (b % NXCD) * chunk + turn % chunk;
  if (tile >= n_tiles) return;
  Bufs<K> B;
#pragma unroll
  for (int a = 0; a < N; ++a) {
    B.D[a] = make_rsrc(S.D[a], basis_bytes);
    B.W[a] = make_rsrc(S.W[a], weight_bytes);
  }
#pragma unroll
  for (int a = 0; a < Fam<K>::NC; ++a) {
    B.C[a] = make_rsrc(S.C[a], point_bytes);
    B.cnull[a] = S.C[a] == nullptr;
  }
  if (RES) {
#pragma unroll
    for (int a = 0; a < Fam<K>::NPF; ++a) B.Pf[a] = make_rsrc(S.Pf[a], point_bytes);
  }
  B.slot = make_rsrc(tslot, slot_bytes);
  const int r = lane & 15, g = lane >> 4;
  const int i0 = trow0[tile];
  const int nr = trow0[tile + 1] - i0;
  const int64_t a0 = row_ptr[i0];
  const int nz = (int)(row_ptr[i0 + nr] - a0);
  const bool live = r < nr;
  Lane L;
  L.r = r;
  L.g = g;
  L.lane8 = (uint32_t)lane * 8u;
  L.g8 = (uint32_t)g * 8u;
  L.lowmask = (1u << r) - 1u;
  L.ro = live ? (int)(row_ptr[i0 + r] - a0) : 0;
  for (int t = lane; t < NACC * nzcap; t += WAVE) acc[t] = 0.0;
  const int64_t e0 = teptr[tile];
  const int ne = (int)(teptr[tile + 1] - e0);
  // the tile's entry records, staged in LDS behind the accumulators (one coalesced read;
  // the steps then decode them from LDS instead of waiting on memory for each cell)
  int4* sent = (int4*)(acc + NACC * nzcap);
  for (int t = lane; t < ne && t < entcap; t += WAVE) sent[t] = tent[e0 + t];
  double rsum = 0.0;
  if (ne > 0) {
    Step st[STEPS];
    uint32_t qo[STEPS];
    Ops<K> op[STEPS];
    uint32_t qnext = live ? (uint32_t)qptr[i0 + r] : 0u;
    st[0].e = 0;
    st[0].ks = 0;
    st[0].cb = 0;
    st[0].E = uniform_record(sent, 0);
    st[0].valid = true;
    st[0].fast = fast_record(st[0].E);
    qo[0] = qnext;
    fetch<K>(st[0], qo[0], L, B, op[0]);
#pragma unroll
    for (int u = 1; u < STEPS; ++u) {
      st[u] = advance(st[u - 1], qnext, r, ne, sent);
      qo[u] = qnext;
      fetch<K>(st[u], qo[u], L, B, op[u]);
    }
    // Steps are valid up to some point and invalid after it; an invalid step computes
    // nothing and fetches nothing but out-of-range offsets, so every pass of the loop body
    // issues the same loads.
    while (st[0].valid) {
#pragma unroll
      for (int u = 0; u < STEPS; ++u) {
        if (st[u].valid) compute<K>(st[u], op[u], L, nzcap, S, B, acc, rsum);
        st[u] = advance(st[(u + STEPS - 1) % STEPS], qnext, r, ne, sent);
        qo[u] = qnext;
        fetch<K>(st[u], qo[u], L, B, op[u]);
      }
    }
  }
  if (RES) {
    const double t0 = __shfl(rsum, r, WAVE), t1 = __shfl(rsum, r + 16, WAVE), t2 = __shfl(rsum, r + 32, WAVE),
                 t3 = __shfl(rsum, r + 48, WAVE);
    if (g == 0 && live) out1[i0 + r] = (t0 + t1) + (t2 + t3);
  }
  for (int t = lane; t < nz; t += WAVE) {
    out0[a0 + t] = acc[t];
    if (K == 3) out1[a0 + t] = acc[nzcap + t];
  }
}

template <int K>
wq_status launch(const wq_points* P, const wq_weights* w, Src S, double* o0, double* o1, hipStream_t st,
                 bool timed = true, bool zterm = false) {
  constexpr int N = Fam<K>::N;
  constexpr int NACC = Fam<K>::NACC;
  const int nzcap = (P->t2_maxnz + 1) & ~1;
  const int entcap = P->t2_maxent;
  const size_t lds = (size_t)NACC * nzcap * sizeof(double) + (size_t)entcap * sizeof(int4);
  WQ_CHECK(lds <= 64 * 1024, WQ_EINVAL, "assemble: tile accumulators exceed LDS");
  // buffer loads take 32-bit byte offsets
  const int64_t sum_r = (int64_t)(P->qidx.bytes / sizeof(int32_t));
  const int64_t lim = (int64_t)OOB;
  WQ_CHECK(P->n_basis * 8 < lim && sum_r * 8 < lim && P->n_points * 8 < lim && (int64_t)P->t2_slot.bytes < lim,
           WQ_EINVAL, "assemble: mesh too large for one launch (2 GiB per array); split it");
  if (K == 0 && zterm) {  // the third surface-gradient term of a surface stiffness
    S.D[0] = P->DZ.as<double>();
    S.W[0] = w->W[4].as<double>();
  } else if (K == 0) {
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
  const int64_t chunk = P->asm_chunk;
  const int64_t per_xcd = ((P->n_t2 + NXCD * chunk - 1) / (NXCD * chunk)) * chunk;
  static const char* names[6] = {"k_assemble_mass", "k_assemble_stiffness", "k_assemble_biharmonic",
                                  "k_assemble_mass_stiffness", "k_assemble_tangent", "k_assemble_tangent_exact"};
  // algorithmic bytes: every basis value and weight once, the coefficients, the output
  int64_t nc = 0;
  for (int a = 0; a < 2; ++a) nc += S.C[a] ? 1 : 0;
  if (K >= 4) nc = 1 + Fam<K>::NPF;  // k and the point fields
  const int64_t outb = K >= 4 ? P->nnz + P->n_rows : NACC * P->nnz;
  KTimer tm(timed ? (zterm ? "k_assemble_stiffness_z" : names[K]) : nullptr,
            8 * (2 * N * sum_r + nc * P->n_points + outb), timed ? st : nullptr);
  if (P->n_t2 > 0)
    k_asm_mfma<K><<<(unsigned)(per_xcd * NXCD), WAVE, lds, st>>>(
        P->n_t2, chunk, nzcap, entcap, P->t2_row0.as<int32_t>(), P->t2_eptr.as<int64_t>(), P->t2_ent.as<int4>(),
        P->t2_slot.as<uint8_t>(), (int64_t)P->t2_slot.bytes, P->row_ptr.as<int64_t>(), P->qptr.as<int64_t>(),
        P->n_basis * 8, sum_r * 8, P->n_points * 8, S, o0, o1);
  if (timed) tm.stop();
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

// k'(u)
__device__ inline double kder(const wq_conductivity& k, double u) {
  switch (k.kind) {
    case WQ_K_LINEAR: return k.b;
    case WQ_K_QUADRATIC: return 2.0 * k.b * u;
    case WQ_K_EXP: return k.a * k.b * exp(k.b * u);
    default: return k.a * k.b * cos(k.b * u);
  }
}

// One thread per (cell, point): T, Tdot, dT/dx, dT/dy at the point from the cell's
// functions (T(x_q) = sum_j T_j N_j(x_q)); k_q = k(T_q) and the residual point fields;
// with p3 (exact tangent) also k'(T_q) dT/dx and k'(T_q) dT/dy.
__global__ void k_point_fields(int32_t ncell, int max_np, const int64_t* __restrict__ cell_pt_off,
                               const int64_t* __restrict__ cfn_ptr, const int32_t* __restrict__ cfn,
                               const int64_t* __restrict__ dptr, const double* __restrict__ DN,
                               const double* __restrict__ DX, const double* __restrict__ DY,
                               const double* __restrict__ T, const double* __restrict__ Td,
                               const double* __restrict__ f, wq_conductivity kc, double* __restrict__ kq,
                               double* __restrict__ p0, double* __restrict__ p1, double* __restrict__ p2,
                               double* __restrict__ p3, double* __restrict__ p4) {
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
  if (p3) {
    const double dk = kder(kc, u);
    p3[pt] = dk * ux;
    p4[pt] = dk * uy;
  }
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

__global__ void k_add(double* v, const double* z, int64_t n) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) v[t] += z[t];
}

// On a surface the stiffness has a third gradient family: its weights are needed, and the
// low-precision contractions, which carry two derivative families, do not apply.
wq_status surface_check(const wq_points* P, const wq_weights* w, wq_precision prec) {
  if (P->mesh->dim != 3) return WQ_OK;
  WQ_CHECK(w->fam_mask & WQ_FAM_DZ, WQ_EINVAL, "assemble: a surface stiffness needs the d/dz weights (WQ_FAM_DZ)");
  WQ_CHECK(prec == WQ_FP64, WQ_EINVAL, "assemble: surface stiffness is FP64 only");
  return WQ_OK;
}

// Surface stiffness: K += sum_q k_q w^z_iq dN_j/dz (the same kernel as the mass matrix,
// on the third gradient family), into scratch held by the points handle, then added.
wq_status add_zterm(const wq_points* P, const wq_weights* w, const double* k, double* kv, hipStream_t st) {
  if (P->mesh->dim != 3) return WQ_OK;
  wq_points* Pm = const_cast<wq_points*>(P);
  if (Pm->zterm_ws.bytes < (size_t)P->nnz * sizeof(double)) {
    dfree(Pm->zterm_ws);
    WQ_TRY(dalloc_n<double>(Pm->zterm_ws, (size_t)P->nnz));
  }
  WQ_TRY(launch<0>(P, w, src_coef(k, nullptr), Pm->zterm_ws.as<double>(), nullptr, st, true, true));
  if (P->nnz > 0) k_add<<<nblocks(P->nnz, 256), 256, 0, st>>>(kv, Pm->zterm_ws.as<double>(), P->nnz);
  WQ_HIP(hipGetLastError());
  return WQ_OK;
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
  WQ_TRY(surface_check(P, w, prec));
  WQ_TRY(dispatch<1>(P, w, k, nullptr, vals, nullptr, prec, (hipStream_t)stream));
  return add_zterm(P, w, k, (double*)vals, (hipStream_t)stream);
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
  WQ_TRY(surface_check(P, w, prec));
  WQ_TRY(dispatch<3>(P, w, c, k, mv, kv, prec, (hipStream_t)stream));
  return add_zterm(P, w, k, (double*)kv, (hipStream_t)stream);
}

// ------------------------------------------------------------------ no-allocation scratch
// Point fields of assemble_tangent_noalloc (4 x n_points doubles): a fixed array, one copy
// per GPU, held until the process ends and shared by every call on that GPU.
constexpr int64_t NOALLOC_MAX_POINTS = int64_t(1) << 19;
static __device__ __align__(256) double scratch[4 * NOALLOC_MAX_POINTS];

namespace {

// Eq. (36) tangent and residual with the point fields (k_q and the three residual terms,
// 4 x n_points doubles) in `ws`. `timed`: record kernel timings when enabled.
wq_status tangent_impl(const wq_points* P, const wq_weights* w, const double* T, const double* Tdot,
                       double inv_theta_dt, wq_conductivity k, const double* f_at_pts, void* S_vals, double* R,
                       double* ws, hipStream_t st, bool timed, bool exact = false) {
  double* kq = ws;
  double* p0 = kq + P->n_points;
  double* p1 = p0 + P->n_points;
  double* p2 = p1 + P->n_points;
  double* p3 = exact ? p2 + P->n_points : nullptr;  // exact tangent: 6 x n_points in ws
  double* p4 = exact ? p3 + P->n_points : nullptr;
  const int mnp = P->max_cell_np;
  {
    KTimer tm(timed ? "k_point_fields" : nullptr, P->n_points, timed ? st : nullptr);
    k_point_fields<<<nblocks((int64_t)P->ncell * mnp, 256), 256, 0, st>>>(
        P->ncell, mnp, P->cell_pt_off.as<int64_t>(), P->cfn_ptr.as<int64_t>(), P->cfn.as<int32_t>(),
        P->dptr.as<int64_t>(), P->DN.as<double>(), P->DX.as<double>(), P->DY.as<double>(), T, Tdot, f_at_pts, k, kq,
        p0, p1, p2, p3, p4);
    if (timed) tm.stop();
    WQ_HIP(hipGetLastError());
  }
  Src S = src_coef(kq, nullptr);
  S.scale = inv_theta_dt;
  S.Pf[0] = p0;
  S.Pf[1] = p1;
  S.Pf[2] = p2;
  if (exact) {
    S.Pf[3] = p3;
    S.Pf[4] = p4;
    return launch<5>(P, w, S, (double*)S_vals, R, st, timed);
  }
  return launch<4>(P, w, S, (double*)S_vals, R, st, timed);
}

wq_status tangent_check(const wq_points* P, const wq_weights* w, const double* T, const double* Tdot,
                        double inv_theta_dt, wq_conductivity k, void* S_vals, double* R, wq_precision prec) {
  WQ_TRY(check(P, w, WQ_FAM_MASS | WQ_FAM_DX | WQ_FAM_DY, S_vals, prec));
  WQ_CHECK(P->mesh->dim == 2, WQ_EINVAL, "assemble_tangent: the heat tangent is planar (dim 2)");
  WQ_CHECK(prec == WQ_FP64, WQ_EINVAL, "assemble_tangent: the Newton tangent and residual are FP64 only");
  WQ_CHECK(T && Tdot && R, WQ_EINVAL, "assemble_tangent: null T, Tdot or R");
  WQ_CHECK(k.kind >= WQ_K_LINEAR && k.kind <= WQ_K_SIN, WQ_EINVAL, "assemble_tangent: unknown conductivity kind");
  WQ_CHECK(std::isfinite(inv_theta_dt), WQ_EINVAL, "assemble_tangent: 1/(theta dt) not finite");
  return WQ_OK;
}

// ------------------------------------------------------------------ no-allocation tangent
// Host code never passes `scratch` itself to a kernel (on the host the name stands for a
// host-side stand-in, not device memory): its device address is looked up once per device
// with hipGetSymbolAddress and kept.
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up on the first call there).
wq_status scratch_on_current_device(int want_device, double** out) {
  int dev = -1;
  WQ_HIP(hipGetDevice(&dev));
  WQ_CHECK(dev == want_device, WQ_EINVAL,
           "assemble_tangent_noalloc: the handle's device must be the current device");
  WQ_CHECK(dev >= 0 && dev < MAX_DEVICES, WQ_EINVAL, "assemble_tangent_noalloc: device index out of range");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    WQ_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    WQ_CHECK(p != nullptr, WQ_EDEVICE, "assemble_tangent_noalloc: no device address for the scratch array");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return WQ_OK;
}

}  // namespace

extern "C" wq_status assemble_tangent(const wq_points* P, const wq_weights* w, const double* T, const double* Tdot,
                                      double inv_theta_dt, wq_conductivity k, const double* f_at_pts, void* S_vals,
                                      double* R, wq_precision prec, wq_stream stream) {
  WQ_TRY(tangent_check(P, w, T, Tdot, inv_theta_dt, k, S_vals, R, prec));
  wq_points* Pm = const_cast<wq_points*>(P);
  if (Pm->tangent_ws.bytes < 4 * (size_t)P->n_points * sizeof(double))
    WQ_TRY(dalloc_n<double>(Pm->tangent_ws, 4 * (size_t)P->n_points));
  return tangent_impl(P, w, T, Tdot, inv_theta_dt, k, f_at_pts, S_vals, R, Pm->tangent_ws.as<double>(),
                      (hipStream_t)stream, true);
}

extern "C" wq_status assemble_tangent_exact(const wq_points* P, const wq_weights* w, const double* T,
                                            const double* Tdot, double inv_theta_dt, wq_conductivity k,
                                            const double* f_at_pts, void* S_vals, double* R, wq_precision prec,
                                            wq_stream stream) {
  WQ_TRY(tangent_check(P, w, T, Tdot, inv_theta_dt, k, S_vals, R, prec));
  wq_points* Pm = const_cast<wq_points*>(P);
  if (Pm->tangent_ws.bytes < 6 * (size_t)P->n_points * sizeof(double))
    WQ_TRY(dalloc_n<double>(Pm->tangent_ws, 6 * (size_t)P->n_points));
  return tangent_impl(P, w, T, Tdot, inv_theta_dt, k, f_at_pts, S_vals, R, Pm->tangent_ws.as<double>(),
                      (hipStream_t)stream, true, true);
}

extern "C" wq_status assemble_tangent_noalloc(const wq_points* P, const wq_weights* w, const double* T,
                                              const double* Tdot, double inv_theta_dt, wq_conductivity k,
                                              const double* f_at_pts, void* S_vals, double* R, wq_precision prec,
                                              wq_stream stream) {
  WQ_TRY(tangent_check(P, w, T, Tdot, inv_theta_dt, k, S_vals, R, prec));
  WQ_CHECK(P->n_points <= NOALLOC_MAX_POINTS, WQ_EINVAL,
           "assemble_tangent_noalloc: more points than the fixed scratch holds (524288)");
  double* ws = nullptr;
  WQ_TRY(scratch_on_current_device(P->mesh->device, &ws));
  return tangent_impl(P, w, T, Tdot, inv_theta_dt, k, f_at_pts, S_vals, R, ws, (hipStream_t)stream, false);
}
