// Batched form: many independent meshes processed by one set of launches. The meshes
// are joined into one disjoint union (vertex, face and function ids offset per mesh):
// every step of the method is local to a function's support, so each mesh's rows,
// points, weights and matrix values are those it gets alone, while the uneven weight
// systems of all meshes share the size buckets of one TSVD launch per bucket and the
// assembly tiles run in one launch. The repeated assembly can be captured in a HIP graph
// and replayed. An autotuner picks the assembly's tile shape (the cap on a tile's work) and
// XCD run length by measurement.
#include "wq_internal.h"

#include <algorithm>
#include <vector>

using namespace wq;

struct wq_batch {
  int32_t n_meshes = 0;
  std::vector<int32_t> face0, fn0;   // per mesh + 1: first face, first function
  std::vector<int64_t> nnz0, pt0;    // per mesh + 1: first CSR entry, first point
  wq_mesh* mesh = nullptr;
  wq_points* pts = nullptr;
  wq_weights* w = nullptr;
  // captured assembly graph and the arguments it was captured with
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* g_args[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int g_prec = -1;
  int64_t g_gen = -1;  // tile generation of the points when captured
  hipStream_t g_stream = nullptr;
};

static void drop_graph(wq_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

extern "C" wq_status wq_batch_create(const wq_mesh_desc* meshes, int32_t n_meshes, wq_batch** out) {
  WQ_CHECK(meshes && out && n_meshes > 0, WQ_EINVAL, "wq_batch_create: need at least one mesh");
  int64_t nv = 0, nf = 0, nfn = 0, next = 0, ncoef = 0;
  for (int32_t k = 0; k < n_meshes; ++k) {
    const wq_mesh_desc& d = meshes[k];
    WQ_CHECK(d.nv > 0 && d.nf > 0 && d.n_fn > 0 && d.face_vtx && d.split && d.ext_ptr && d.ext_fn && d.coef_ptr &&
                 d.coef && d.ctrl,
             WQ_EINVAL, "wq_batch_create: incomplete mesh " + std::to_string(k));
    WQ_CHECK(d.dim == 0 || d.dim == 2, WQ_EINVAL, "wq_batch_create: planar meshes only (mesh " + std::to_string(k) + ")");
    nv += d.nv;
    nf += d.nf;
    nfn += d.n_fn;
    next += d.ext_ptr[d.nf];
    ncoef += d.coef_ptr[d.nf];
  }
  WQ_CHECK(nv < INT32_MAX && nf < INT32_MAX && nfn < INT32_MAX, WQ_EINVAL, "wq_batch_create: batch too large");
  std::vector<int32_t> face_vtx(4 * nf), ext_fn(next);
  std::vector<uint8_t> split(nf);
  std::vector<int64_t> ext_ptr(nf + 1), coef_ptr(nf + 1);
  std::vector<double> coef(ncoef), ctrl(2 * nfn);
  wq_batch* b = new wq_batch();
  b->n_meshes = n_meshes;
  b->face0.assign(n_meshes + 1, 0);
  b->fn0.assign(n_meshes + 1, 0);
  int64_t v0 = 0, f0 = 0, j0 = 0, e0 = 0, c0 = 0;
  for (int32_t k = 0; k < n_meshes; ++k) {
    const wq_mesh_desc& d = meshes[k];
    b->face0[k] = (int32_t)f0;
    b->fn0[k] = (int32_t)j0;
    for (int64_t t = 0; t < 4LL * d.nf; ++t) face_vtx[4 * f0 + t] = (int32_t)(d.face_vtx[t] + v0);
    for (int32_t f = 0; f < d.nf; ++f) {
      split[f0 + f] = d.split[f];
      ext_ptr[f0 + f] = e0 + d.ext_ptr[f];
      coef_ptr[f0 + f] = c0 + d.coef_ptr[f];
    }
    for (int64_t t = 0; t < d.ext_ptr[d.nf]; ++t) ext_fn[e0 + t] = (int32_t)(d.ext_fn[t] + j0);
    std::copy(d.coef, d.coef + d.coef_ptr[d.nf], coef.begin() + c0);
    std::copy(d.ctrl, d.ctrl + 2 * (int64_t)d.n_fn, ctrl.begin() + 2 * j0);
    v0 += d.nv;
    f0 += d.nf;
    j0 += d.n_fn;
    e0 += d.ext_ptr[d.nf];
    c0 += d.coef_ptr[d.nf];
  }
  ext_ptr[nf] = e0;
  coef_ptr[nf] = c0;
  b->face0[n_meshes] = (int32_t)f0;
  b->fn0[n_meshes] = (int32_t)j0;
  wq_mesh_desc u{(int32_t)nv, (int32_t)nf, (int32_t)nfn, face_vtx.data(), split.data(), ext_ptr.data(),
                 ext_fn.data(), coef_ptr.data(), coef.data(), ctrl.data()};
  const wq_status s = wq_mesh_create(&u, &b->mesh);
  if (s != WQ_OK) {
    delete b;
    return s;
  }
  *out = b;
  return WQ_OK;
}

extern "C" wq_status wq_batch_build(wq_batch* b, unsigned fam_mask, double tau, wq_stream stream,
                                    wq_solve_report* report) {
  WQ_CHECK(b && b->mesh, WQ_EINVAL, "wq_batch_build: null batch");
  drop_graph(b);
  wq_weights_destroy(b->w);
  wq_points_destroy(b->pts);
  b->w = nullptr;
  b->pts = nullptr;
  int64_t n = 0, nnz = 0, np = 0;
  WQ_TRY(build_points(b->mesh, (fam_mask & WQ_FAM_LAP) ? 1 : 0, stream, &b->pts, &n, &nnz, &np));
  WQ_TRY(solve_weights(b->mesh, b->pts, fam_mask, tau, stream, &b->w, report));
  // per-mesh ranges: rows are function ranges; CSR entries and points follow
  const wq_points* P = b->pts;
  std::vector<int64_t> row_ptr(n + 1), pt_off(P->ncell + 1);
  std::vector<int32_t> cell_face(P->ncell);
  WQ_HIP(hipMemcpy(row_ptr.data(), P->row_ptr.p, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
  WQ_HIP(hipMemcpy(pt_off.data(), P->cell_pt_off.p, (P->ncell + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
  WQ_HIP(hipMemcpy(cell_face.data(), P->cell_face.p, P->ncell * sizeof(int32_t), hipMemcpyDeviceToHost));
  b->nnz0.assign(b->n_meshes + 1, 0);
  b->pt0.assign(b->n_meshes + 1, 0);
  for (int32_t k = 0; k <= b->n_meshes; ++k) {
    b->nnz0[k] = row_ptr[b->fn0[k]];
    const int64_t c = std::lower_bound(cell_face.begin(), cell_face.end(), b->face0[k]) - cell_face.begin();
    b->pt0[k] = pt_off[c];
  }
  return WQ_OK;
}

extern "C" wq_status wq_batch_info(const wq_batch* b, int32_t k, int64_t* row0, int64_t* n_rows, int64_t* nnz0,
                                   int64_t* nnz, int64_t* pt0, int64_t* n_points) {
  WQ_CHECK(b && b->pts && k >= 0 && k < b->n_meshes, WQ_EINVAL, "wq_batch_info: bad batch or mesh index");
  if (row0) *row0 = b->fn0[k];
  if (n_rows) *n_rows = b->fn0[k + 1] - b->fn0[k];
  if (nnz0) *nnz0 = b->nnz0[k];
  if (nnz) *nnz = b->nnz0[k + 1] - b->nnz0[k];
  if (pt0) *pt0 = b->pt0[k];
  if (n_points) *n_points = b->pt0[k + 1] - b->pt0[k];
  return WQ_OK;
}

extern "C" wq_points* wq_batch_points(wq_batch* b) { return b ? b->pts : nullptr; }
extern "C" wq_weights* wq_batch_weights(wq_batch* b) { return b ? b->w : nullptr; }

extern "C" wq_status wq_batch_graph_assemble(wq_batch* b, const double* c, const double* k, void* mass_vals,
                                             void* stiff_vals, wq_precision prec, wq_stream stream) {
  WQ_CHECK(b && b->pts && b->w, WQ_EINVAL, "wq_batch_graph_assemble: batch not built");
  hipStream_t st = (hipStream_t)stream;
  WQ_CHECK(st != nullptr, WQ_EINVAL, "wq_batch_graph_assemble: capture needs a created stream, not the null stream");
  const void* args[5] = {c, k, mass_vals, stiff_vals, nullptr};
  bool same = b->exec && b->g_prec == (int)prec && b->g_stream == st && b->g_gen == b->pts->t2_gen;
  for (int t = 0; t < 4; ++t) same = same && args[t] == b->g_args[t];
  if (!same) {
    drop_graph(b);
    // eager call first: validates the arguments and performs one-time work (basis data
    // conversion for the low-precision forms) outside the capture
    WQ_TRY(assemble_mass_stiffness(b->pts, b->w, c, k, mass_vals, stiff_vals, prec, stream));
    WQ_HIP(hipStreamSynchronize(st));
    const bool timing = timing_enabled();  // no timing events inside the graph
    wq_timing_enable(0);
    WQ_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const wq_status s = assemble_mass_stiffness(b->pts, b->w, c, k, mass_vals, stiff_vals, prec, stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    wq_timing_enable(timing ? 1 : 0);
    if (s != WQ_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      WQ_TRY(s);
      WQ_HIP(e);
    }
    b->graph = g;
    WQ_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    for (int t = 0; t < 4; ++t) b->g_args[t] = args[t];
    b->g_prec = (int)prec;
    b->g_stream = st;
    b->g_gen = b->pts->t2_gen;
  }
  WQ_HIP(hipGraphLaunch(b->exec, st));
  return WQ_OK;
}

extern "C" void wq_batch_destroy(wq_batch* b) {
  if (!b) return;
  drop_graph(b);
  wq_weights_destroy(b->w);
  wq_points_destroy(b->pts);
  wq_mesh_destroy(b->mesh);
  delete b;
}

// ------------------------------------------------------------------ autotuner
namespace {

// Median time (ms) of the FP64 mass + stiffness assembly on P for each candidate XCD run
// length (powers of two from 4 to 1024 below one contiguous band of tiles per XCD, then
// the band); sets P->asm_chunk to the fastest and returns it with its time.
wq_status tune_chunk(wq_points* P, const wq_weights* w, hipStream_t st, double* M, double* K, int* best,
                     double* best_t) {
  const int band = (int)((P->n_t2 + 7) / 8);
  std::vector<int> cand;
  for (int c = 4; c < band && c <= 1024; c *= 2) cand.push_back(c);
  cand.push_back(std::max(band, 1));
  hipEvent_t e0, e1;
  WQ_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    set_error("autotune: hipEventCreate failed");
    return WQ_EDEVICE;
  }
  const int keep = P->asm_chunk;
  *best = keep;
  *best_t = 1e300;
  wq_status s = WQ_OK;
  for (int c : cand) {
    P->asm_chunk = c;
    std::vector<float> ts;
    for (int rep = 0; rep < 6 && s == WQ_OK; ++rep) {
      if (hipEventRecord(e0, st) != hipSuccess) s = WQ_EDEVICE;
      if (s == WQ_OK) s = assemble_mass_stiffness(P, w, nullptr, nullptr, M, K, WQ_FP64, (wq_stream)st);
      float ms = 0.f;
      if (s == WQ_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        s = WQ_EDEVICE;
      if (rep > 0) ts.push_back(ms);  // first run warms caches
    }
    if (s != WQ_OK) break;
    std::sort(ts.begin(), ts.end());
    const double med = ts[ts.size() / 2];
    if (med < *best_t) {
      *best_t = med;
      *best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P->asm_chunk = s == WQ_OK ? *best : keep;
  return s;
}

}  // namespace

extern "C" wq_status wq_autotune_assembly(wq_points* P, const wq_weights* w, wq_stream stream, int32_t* chosen,
                                          double* best_ms) {
  WQ_CHECK(P && w && w->pts == P, WQ_EINVAL, "wq_autotune_assembly: bad arguments");
  DBuf M, K;
  WQ_TRY(dalloc_n<double>(M, P->nnz));
  WQ_TRY(dalloc_n<double>(K, P->nnz));
  int best = P->asm_chunk;
  double best_t = 0.0;
  const wq_status s = tune_chunk(P, w, (hipStream_t)stream, M.as<double>(), K.as<double>(), &best, &best_t);
  ++P->t2_gen;  // the schedule changed
  DBuf* tmp[] = {&M, &K};
  dfree_many(tmp, 2);
  if (chosen) *chosen = P->asm_chunk;
  if (best_ms) *best_ms = best_t;
  return s;
}

extern "C" wq_status wq_autotune_tiles(wq_points* P, const wq_weights* w, wq_stream stream, int32_t* chosen_stepcap,
                                       int32_t* chosen_chunk, double* best_ms) {
  WQ_CHECK(P && w && w->pts == P, WQ_EINVAL, "wq_autotune_tiles: bad arguments");
  hipStream_t st = (hipStream_t)stream;
  DBuf M, K;
  WQ_TRY(dalloc_n<double>(M, P->nnz));
  WQ_TRY(dalloc_n<double>(K, P->nnz));
  // candidate caps on a tile's summed row steps (blocks of four points of its rows' support
  // cells): from about four regular rows up to none (the row and CSR-entry limits alone)
  const int caps[] = {64, 96, 128, 192, 256, 1 << 30};
  const int keep_cap = P->t2_stepcap, keep_chunk = P->asm_chunk;
  int best_cap = keep_cap, best_chunk = keep_chunk;
  double best_t = 1e300;
  wq_status s = WQ_OK;
  for (int cap : caps) {
    P->t2_stepcap = cap;
    s = rebuild_tiles2(P, st);
    int ch = 0;
    double t = 0.0;
    if (s == WQ_OK) s = tune_chunk(P, w, st, M.as<double>(), K.as<double>(), &ch, &t);
    if (s != WQ_OK) break;
    if (t < best_t) {
      best_t = t;
      best_cap = cap;
      best_chunk = ch;
    }
  }
  // keep the fastest (or, after an error, what the handle had)
  P->t2_stepcap = s == WQ_OK ? best_cap : keep_cap;
  const wq_status s2 = rebuild_tiles2(P, st);
  P->asm_chunk = s == WQ_OK ? best_chunk : keep_chunk;
  DBuf* tmp[] = {&M, &K};
  dfree_many(tmp, 2);
  if (s == WQ_OK && s2 != WQ_OK) s = s2;
  if (chosen_stepcap) *chosen_stepcap = P->t2_stepcap;
  if (chosen_chunk) *chosen_chunk = P->asm_chunk;
  if (best_ms) *best_ms = best_t;
  return s;
}
