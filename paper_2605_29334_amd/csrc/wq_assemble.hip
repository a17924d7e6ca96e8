// Row-wise WQ assembly (Eqs. (9), (11), (12)); Section 6.1 forms the matrix row by row.
#include "wq_internal.h"

using namespace wq;

namespace {

constexpr int GROUP = 16;  // lanes per row
constexpr int BS = 256;    // 16 rows per block

// K = 0 mass, 1 stiffness, 2 biharmonic, 3 mass + stiffness.
// Row i is owned by one 16-lane group. For every cell c of supp N_i (ascending) and every
// cell function k (one lane each): v_k = sum_{points q of c} w_iq coef_q D_k(x_q), then
// acc[slot_k] += v_k. Lanes of a group own distinct slots at every step, so there are no
// atomics and the summation order is fixed.
template <int K>
__global__ void __launch_bounds__(BS) k_assemble(int64_t n, int max_row, const int64_t* __restrict__ sptr,
                                                 const int32_t* __restrict__ scell, const int64_t* __restrict__ cfn_ptr,
                                                 const int64_t* __restrict__ cell_pt_off, const int64_t* __restrict__ dptr,
                                                 const int64_t* __restrict__ soff, const uint8_t* __restrict__ slot,
                                                 const int64_t* __restrict__ row_ptr, const int64_t* __restrict__ qptr,
                                                 const double* __restrict__ W0, const double* __restrict__ W1,
                                                 const double* __restrict__ W2, const double* __restrict__ D0,
                                                 const double* __restrict__ D1, const double* __restrict__ D2,
                                                 const double* __restrict__ c0, const double* __restrict__ c1,
                                                 double* __restrict__ out0, double* __restrict__ out1) {
  extern __shared__ double sh[];
  constexpr int NACC = (K == 3) ? 2 : 1;
  const int grp = threadIdx.x / GROUP;
  const int lane = threadIdx.x % GROUP;
  const int64_t i = (int64_t)blockIdx.x * (BS / GROUP) + grp;
  double* acc = sh + (size_t)grp * NACC * max_row;
  const bool active = i < n;
  for (int t = lane; t < NACC * max_row; t += GROUP) acc[t] = 0.0;
  __syncthreads();
  if (active) {
    int64_t qo = qptr[i];
    for (int64_t p = sptr[i]; p < sptr[i + 1]; ++p) {
      const int32_t c = scell[p];
      const int64_t f0 = cfn_ptr[c];
      const int m = (int)(cfn_ptr[c + 1] - f0);
      const int64_t pt0 = cell_pt_off[c];
      const int np = (int)(cell_pt_off[c + 1] - pt0);
      const int64_t d0 = dptr[c];
      const uint8_t* sl = slot + soff[p];
      for (int k = lane; k < m; k += GROUP) {
        double va = 0.0, vb = 0.0;
        for (int q = 0; q < np; ++q) {
          const int64_t dq = d0 + (int64_t)q * m + k;
          if (K == 0 || K == 2) {
            const double cq = c0 ? c0[pt0 + q] : 1.0;
            va += (W0[qo + q] * cq) * D0[dq];
          } else if (K == 1) {
            const double kq = c0 ? c0[pt0 + q] : 1.0;
            va += kq * (W1[qo + q] * D1[dq] + W2[qo + q] * D2[dq]);
          } else {
            const double cq = c0 ? c0[pt0 + q] : 1.0;
            const double kq = c1 ? c1[pt0 + q] : 1.0;
            va += (W0[qo + q] * cq) * D0[dq];
            vb += kq * (W1[qo + q] * D1[dq] + W2[qo + q] * D2[dq]);
          }
        }
        const int sk = sl[k];
        acc[sk] += va;
        if (K == 3) acc[max_row + sk] += vb;
      }
      qo += np;
    }
  }
  __syncthreads();
  if (active) {
    const int64_t r0 = row_ptr[i];
    const int ni = (int)(row_ptr[i + 1] - r0);
    for (int t = lane; t < ni; t += GROUP) {
      out0[r0 + t] = acc[t];
      if (K == 3) out1[r0 + t] = acc[max_row + t];
    }
  }
}

template <int K>
wq_status launch(const wq_points* P, const wq_weights* w, const double* c0, const double* c1, double* o0, double* o1,
                 hipStream_t st) {
  constexpr int NACC = (K == 3) ? 2 : 1;
  const size_t lds = (size_t)(BS / GROUP) * NACC * P->max_row * sizeof(double);
  const double* W0 = w->W[0].as<double>();
  const double* W1 = w->W[1].as<double>();
  const double* W2 = w->W[2].as<double>();
  const double* D0 = P->DN.as<double>();
  if (K == 2) {
    W0 = w->W[3].as<double>();
    D0 = P->DL.as<double>();
  }
  static const char* names[4] = {"k_assemble_mass", "k_assemble_stiffness", "k_assemble_biharmonic",
                                  "k_assemble_mass_stiffness"};
  KTimer tm(names[K], P->n_rows, st);
  k_assemble<K><<<nblocks(P->n_rows, BS / GROUP), BS, lds, st>>>(
      P->n_rows, P->max_row, P->supp_ptr.as<int64_t>(), P->supp_cell.as<int32_t>(), P->cfn_ptr.as<int64_t>(),
      P->cell_pt_off.as<int64_t>(), P->dptr.as<int64_t>(), P->soff.as<int64_t>(), P->slot.as<uint8_t>(),
      P->row_ptr.as<int64_t>(), P->qptr.as<int64_t>(), W0, W1, W2, D0, P->DX.as<double>(), P->DY.as<double>(), c0,
      c1, o0, o1);
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

}  // namespace

extern "C" wq_status assemble_mass(const wq_points* P, const wq_weights* w, const double* c, void* vals,
                                   wq_precision prec, wq_stream stream) {
  WQ_TRY(check(P, w, WQ_FAM_MASS, vals, prec));
  return launch<0>(P, w, c, nullptr, (double*)vals, nullptr, (hipStream_t)stream);
}

extern "C" wq_status assemble_stiffness(const wq_points* P, const wq_weights* w, const double* k, void* vals,
                                        wq_precision prec, wq_stream stream) {
  WQ_TRY(check(P, w, WQ_FAM_DX | WQ_FAM_DY, vals, prec));
  return launch<1>(P, w, k, nullptr, (double*)vals, nullptr, (hipStream_t)stream);
}

extern "C" wq_status assemble_biharmonic(const wq_points* P, const wq_weights* w, const double* d, void* vals,
                                         wq_precision prec, wq_stream stream) {
  WQ_TRY(check(P, w, WQ_FAM_LAP, vals, prec));
  WQ_CHECK(P->has_lap, WQ_EINVAL, "assemble_biharmonic: build_points without Laplacians");
  return launch<2>(P, w, d, nullptr, (double*)vals, nullptr, (hipStream_t)stream);
}

extern "C" wq_status assemble_mass_stiffness(const wq_points* P, const wq_weights* w, const double* c,
                                             const double* k, void* mv, void* kv, wq_precision prec,
                                             wq_stream stream) {
  WQ_TRY(check(P, w, WQ_FAM_MASS | WQ_FAM_DX | WQ_FAM_DY, mv, prec));
  WQ_CHECK(kv, WQ_EINVAL, "assemble_mass_stiffness: null stiffness output");
  return launch<3>(P, w, c, k, (double*)mv, (double*)kv, (hipStream_t)stream);
}
