// Element-wise Gauss quadrature assembly: the comparison system of the method. The paper
// replaces the standard loop over elements with p+1 Gauss points per direction (Section 1)
// by row-wise weighted quadrature and times the two against each other for the Poisson and
// biharmonic problems (Section 6.1, with the basis at the quadrature points computed ahead
// and excluded from the timing). Here both run on the GPU over the same CSR pattern.
#include "wq_internal.h"

using namespace wq;

struct wq_gauss {
  wq_points* pts = nullptr;
  int has_lap = 0;
  // basis at the 16 Gauss points of every cell, point-major per cell like the WQ data
  DBuf GN, GX, GY, GZ /*surfaces*/, GL, gw /*[16 ncell]*/, gx /*[dim x 16 ncell]*/;
  int dim = 2;
  // per (cell, cell function a): the CSR offset of the row of function a and the offset of
  // the slot map of the (row, cell) pair, so that entry (a, b) of the cell's local matrix
  // goes to vals[pbase + slot[pslot + b]]
  DBuf pbase, pslot;
};

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// Where the local matrix of every cell goes in the CSR values: one workgroup per cell, one
// thread per cell function; the (row, cell) pair is found in the row's support list.
__global__ void k_gq_pairs(int32_t ncell, const int64_t* cfn_ptr, const int32_t* cfn, const int64_t* supp_ptr,
                           const int32_t* supp_cell, const int64_t* soff, const int64_t* row_ptr, int64_t* pbase,
                           int64_t* pslot, int* bad) {
  const int32_t c = blockIdx.x;
  const int64_t f0 = cfn_ptr[c];
  const int m = (int)(cfn_ptr[c + 1] - f0);
  for (int a = threadIdx.x; a < m; a += blockDim.x) {
    const int32_t i = cfn[f0 + a];
    int64_t p = -1;
    for (int64_t q = supp_ptr[i]; q < supp_ptr[i + 1]; ++q)
      if (supp_cell[q] == c) {
        p = q;
        break;
      }
    if (p < 0) {
      atomicOr(bad, 1);
      continue;
    }
    pbase[f0 + a] = row_ptr[i];
    pslot[f0 + a] = soff[p];
  }
}

__global__ void k_zero(double* v, int64_t n) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) v[t] = 0.0;
}

// Local matrices E_ab = sum_g gw_g coef_g sum_t G_t[g][a] G_t[g][b] (t: one term for the
// mass and biharmonic kinds, the x and y gradients for the stiffness) of one cell per
// workgroup, in 16 x 16 tiles on FP64 MFMA: A[a][k] = G[g_k][a] and B[k][b] = W[g_k]
// G[g_k][b] over the 16 points in four steps of four (lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]: the same basis entry, once weighted), D[4 v + l / 16][l % 16] in
// result register v. Every entry is added into the CSR values with an FP64 atomic, so
// the order of the additions, and with it the last bits, varies between runs.
template <int NT>  // terms of the integrand: 1, 2 or 3 (the gradient components)
__global__ void __launch_bounds__(64) k_gq_assemble(const int64_t* cfn_ptr, const double* G0, const double* G1,
                                                    const double* G2, const double* gw, const double* coef, const int64_t* pbase,
                                                    const int64_t* pslot, const uint8_t* slot, double* vals) {
  const int32_t c = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t f0 = cfn_ptr[c];
  const int m = (int)(cfn_ptr[c + 1] - f0);
  const int gq = lane >> 4, col = lane & 15;
  double W[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int g = 4 * s + gq;
    W[s] = gw[16 * (int64_t)c + g] * (coef ? coef[16 * (int64_t)c + g] : 1.0);
  }
  const double* Gt[3] = {G0 + 16 * f0, G1 ? G1 + 16 * f0 : nullptr, G2 ? G2 + 16 * f0 : nullptr};
  const int nt = (m + 15) / 16;
  for (int ta = 0; ta < nt; ++ta) {
    const int a = 16 * ta + col;
    for (int tb = 0; tb < nt; ++tb) {
      const int b = 16 * tb + col;
      d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int g = 4 * s + gq;
          const double av = a < m ? Gt[t][g * m + a] : 0.0;
          const double bv = b < m ? W[s] * Gt[t][g * m + b] : 0.0;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
      // the products to ordinary registers before any memory instruction reads them
      double e[4] = {acc[0], acc[1], acc[2], acc[3]};
#pragma unroll
      for (int v = 0; v < 4; ++v) asm volatile("" : "+v"(e[v]));
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ar = 16 * ta + 4 * v + gq;
        if (ar < m && b < m) unsafeAtomicAdd(&vals[pbase[f0 + ar] + slot[pslot[f0 + ar] + b]], e[v]);
      }
    }
  }
}

}  // namespace

extern "C" wq_status gauss_setup(wq_mesh* M, wq_points* P, int want_laplacian, wq_stream stream, wq_gauss** out) {
  WQ_CHECK(M && P && out && P->mesh == M, WQ_EINVAL, "gauss_setup: bad arguments");
  WQ_CHECK(!want_laplacian || P->has_lap, WQ_EINVAL, "gauss_setup: Laplacians need build_points(want_laplacian=1)");
  hipStream_t st = (hipStream_t)stream;
  wq_gauss* g = new wq_gauss();
  g->pts = P;
  g->has_lap = want_laplacian != 0;
  g->dim = M->dim;
  const size_t ng = 16 * (size_t)P->n_cfn;
  wq_status s = dalloc_n<double>(g->GN, ng);
  if (s == WQ_OK) s = dalloc_n<double>(g->GX, ng);
  if (s == WQ_OK) s = dalloc_n<double>(g->GY, ng);
  if (s == WQ_OK && g->dim == 3) s = dalloc_n<double>(g->GZ, ng);
  if (s == WQ_OK && g->has_lap) s = dalloc_n<double>(g->GL, ng);
  if (s == WQ_OK) s = dalloc_n<double>(g->gw, 16 * (size_t)P->ncell);
  if (s == WQ_OK) s = dalloc_n<double>(g->gx, 16 * (size_t)g->dim * P->ncell);
  if (s == WQ_OK) s = dalloc_n<int64_t>(g->pbase, (size_t)P->n_cfn);
  if (s == WQ_OK) s = dalloc_n<int64_t>(g->pslot, (size_t)P->n_cfn);
  DBuf bad;
  if (s == WQ_OK) s = dalloc_n<int>(bad, 1);
  if (s == WQ_OK && hipMemsetAsync(bad.p, 0, sizeof(int), st) != hipSuccess) s = WQ_EDEVICE;
  if (s == WQ_OK)
    s = gauss_basis(M, P, g->GN.as<double>(), g->GX.as<double>(), g->GY.as<double>(), g->GZ.as<double>(),
                    g->has_lap ? g->GL.as<double>() : nullptr, g->gw.as<double>(), g->gx.as<double>(), st);
  if (s == WQ_OK && P->ncell > 0) {
    k_gq_pairs<<<P->ncell, 64, 0, st>>>(P->ncell, P->cfn_ptr.as<int64_t>(), P->cfn.as<int32_t>(),
                                         P->supp_ptr.as<int64_t>(), P->supp_cell.as<int32_t>(),
                                         P->soff.as<int64_t>(), P->row_ptr.as<int64_t>(), g->pbase.as<int64_t>(),
                                         g->pslot.as<int64_t>(), bad.as<int>());
    if (hipGetLastError() != hipSuccess) s = WQ_EDEVICE;
  }
  int hbad = 0;
  if (s == WQ_OK && (hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
                     hipStreamSynchronize(st) != hipSuccess))
    s = WQ_EDEVICE;
  dfree(bad);
  if (s == WQ_OK && hbad) {
    set_error("gauss_setup: a cell function's row does not list the cell in its support");
    s = WQ_EDEVICE;
  }
  if (s != WQ_OK) {
    wq_gauss_destroy(g);
    return s;
  }
  *out = g;
  return WQ_OK;
}

extern "C" void wq_gauss_destroy(wq_gauss* g) {
  if (!g) return;
  DBuf* all[] = {&g->GN, &g->GX, &g->GY, &g->GZ, &g->GL, &g->gw, &g->gx, &g->pbase, &g->pslot};
  dfree_many(all, sizeof(all) / sizeof(all[0]));
  delete g;
}

extern "C" int64_t wq_gauss_size(const wq_gauss* g) { return g ? 16 * (int64_t)g->pts->ncell : -1; }

extern "C" wq_status wq_gauss_get_x(const wq_gauss* g, double* dst, wq_stream stream) {
  WQ_CHECK(g && dst, WQ_EINVAL, "wq_gauss_get_x: bad arguments");
  WQ_HIP(hipMemcpyAsync(dst, g->gx.p, g->gx.bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return WQ_OK;
}

extern "C" wq_status assemble_gauss(const wq_gauss* g, wq_gauss_kind kind, const double* coef_at_gauss,
                                    double* vals, wq_stream stream) {
  WQ_CHECK(g && vals, WQ_EINVAL, "assemble_gauss: bad arguments");
  WQ_CHECK(kind == WQ_GQ_MASS || kind == WQ_GQ_STIFFNESS || kind == WQ_GQ_BIHARMONIC, WQ_EINVAL,
           "assemble_gauss: unknown kind");
  WQ_CHECK(kind != WQ_GQ_BIHARMONIC || g->has_lap, WQ_EINVAL,
           "assemble_gauss: the biharmonic kind needs gauss_setup(want_laplacian=1)");
  const wq_points* P = g->pts;
  hipStream_t st = (hipStream_t)stream;
  if (P->nnz > 0) {
    k_zero<<<nblocks(P->nnz, 256), 256, 0, st>>>(vals, P->nnz);
    WQ_HIP(hipGetLastError());
  }
  if (P->ncell == 0) return WQ_OK;
  const char* name = kind == WQ_GQ_MASS ? "k_gq_assemble_mass"
                     : kind == WQ_GQ_STIFFNESS ? "k_gq_assemble_stiffness"
                                               : "k_gq_assemble_biharmonic";
  KTimer tm(name, 16LL * P->ncell, st);
  const int64_t* cp = P->cfn_ptr.as<int64_t>();
  const int64_t* pb = g->pbase.as<int64_t>();
  const int64_t* ps = g->pslot.as<int64_t>();
  const uint8_t* sl = P->slot.as<uint8_t>();
  if (kind == WQ_GQ_STIFFNESS && g->dim == 3)
    k_gq_assemble<3><<<P->ncell, 64, 0, st>>>(cp, g->GX.as<double>(), g->GY.as<double>(), g->GZ.as<double>(),
                                              g->gw.as<double>(), coef_at_gauss, pb, ps, sl, vals);
  else if (kind == WQ_GQ_STIFFNESS)
    k_gq_assemble<2><<<P->ncell, 64, 0, st>>>(cp, g->GX.as<double>(), g->GY.as<double>(), nullptr,
                                              g->gw.as<double>(), coef_at_gauss, pb, ps, sl, vals);
  else
    k_gq_assemble<1><<<P->ncell, 64, 0, st>>>(
        cp, kind == WQ_GQ_MASS ? g->GN.as<double>() : g->GL.as<double>(), nullptr, nullptr, g->gw.as<double>(),
        coef_at_gauss, pb, ps, sl, vals);
  tm.stop();
  WQ_HIP(hipGetLastError());
  return WQ_OK;
}
