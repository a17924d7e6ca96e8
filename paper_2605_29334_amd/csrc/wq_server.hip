// Served nonlinear heat transfer: a request loop that runs whole WQ solves (points,
// weights, Newton time steps of Section 5.2) for meshes as they arrive. Requests are
// admitted in arrival order when a slot is free and their HBM estimate fits the budget;
// each slot is a host thread with its own non-blocking stream, so admitted requests
// overlap on the device. All state of a request stays on the device until its final
// temperature is copied out. The setup of a domain (mesh, points, weights: computed once
// per fixed domain) stays on the device after its request; a later request on an
// identical domain takes it over instead of recomputing it. With joining on, requests
// queued together with the same parameters run as one union of their meshes: one set of
// launches for the setup and for every Newton and Krylov step of all of them.
#include "wq_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

using namespace wq;

namespace {

// f = dT*/dt - div(k(T*) grad T*) for T* = (1 - e^{-lam t}) sin(pi x) sin(pi y), with
// div(k grad u) = k'(u) |grad u|^2 + k(u) Lap u.
__global__ void k_manufactured_source(int64_t np, const double* __restrict__ x, double t, double lam,
                                      wq_conductivity kc, double* __restrict__ f) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= np) return;
  const double PI = 3.141592653589793;
  const double e = exp(-lam * t), s = 1.0 - e;
  const double sx = sin(PI * x[2 * q]), sy = sin(PI * x[2 * q + 1]);
  const double cx = cos(PI * x[2 * q]), cy = cos(PI * x[2 * q + 1]);
  const double u = s * sx * sy;
  const double ux = s * PI * cx * sy, uy = s * PI * sx * cy;
  const double lap = -2.0 * PI * PI * u;
  double k, dk;
  switch (kc.kind) {
    case WQ_K_LINEAR: k = kc.a + kc.b * u; dk = kc.b; break;
    case WQ_K_QUADRATIC: k = kc.a + kc.b * u * u; dk = 2.0 * kc.b * u; break;
    case WQ_K_EXP: k = kc.a * exp(kc.b * u); dk = kc.b * k; break;
    default: k = kc.a * sin(kc.b * u); dk = kc.a * kc.b * cos(kc.b * u); break;
  }
  f[q] = lam * e * sx * sy - (dk * (ux * ux + uy * uy) + k * lap);
}

// A domain's setup on the device. Its request's HBM estimate stays charged to the budget
// while it is held (running or idle); busy = in use by a running request (the points
// handle carries per-call Newton scratch, so a setup serves one request at a time).
struct Setup {
  std::vector<int32_t> face_vtx, ext_fn;
  std::vector<uint8_t> split;
  std::vector<int64_t> ext_ptr, coef_ptr;
  std::vector<double> coef, ctrl;
  int32_t nv = 0;
  wq_mesh* mesh = nullptr;
  wq_points* pts = nullptr;
  wq_weights* w = nullptr;
  size_t bytes = 0;
  bool busy = false;
  int64_t last_used = 0;
  void release() {
    wq_weights_destroy(w);
    wq_points_destroy(pts);
    wq_mesh_destroy(mesh);
    w = nullptr;
    pts = nullptr;
    mesh = nullptr;
  }
};

struct Request {
  int64_t id = 0;
  // deep copies of the host inputs
  std::vector<int32_t> face_vtx, ext_fn;
  std::vector<uint8_t> split, dirichlet;
  std::vector<int64_t> ext_ptr, coef_ptr;
  std::vector<double> coef, ctrl;
  wq_mesh_desc desc{};
  wq_heat_params heat{};
  int32_t n_steps = 0, source = 0;
  double lambda = 0;
  bool reuse = true;  // may take over a held setup of its domain and leave its own held
  double* T_out = nullptr;
  size_t est = 0;
  wq_result res{};
  bool done = false;
  Setup* setup = nullptr;  // a held setup of the same domain taken over at admission
};

bool same_domain(const Setup& a, const Request& r) {
  return a.nv == r.desc.nv && a.face_vtx == r.face_vtx && a.split == r.split && a.ext_ptr == r.ext_ptr &&
         a.ext_fn == r.ext_fn && a.coef_ptr == r.coef_ptr && a.coef == r.coef && a.ctrl == r.ctrl;
}

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct wq_server {
  int device = 0;
  size_t budget = 0, in_use = 0;  // in_use: running requests and held setups
  std::vector<Setup*> setups;     // held setups (busy or idle)
  int64_t clock = 0;              // admission counter (least recently used setup first)
  bool stopping = false;
  int64_t next_id = 1;
  int32_t join = 1;         // most requests run as one union (1: each request alone)
  int64_t join_rows = 0;    // most rows of a union (functions of its meshes)
  std::deque<Request*> queue;
  std::map<int64_t, Request*> all;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::vector<std::thread> workers;
  std::chrono::steady_clock::time_point t0;
};

namespace {

// HBM estimate of one request from its input sizes: per face of the control mesh about
// 4 points x (basis values of ~16 functions x 3 arrays + weights x 3) + CSR values and
// pattern + tile records, bounded generously, plus the Newton/PCG vectors.
size_t hbm_estimate(const wq_mesh_desc& d) {
  return (size_t)16384 * (size_t)d.nf + (size_t)256 * (size_t)d.n_fn + ((size_t)8 << 20);
}

// The time steps from T = Tdot = 0 (already cleared) on a points/weights pair whose rows
// form nseg segments, one request each (parameters from r): the manufactured source at
// t_{n+1}, then one heat step of every segment as if alone; iteration counts add up in
// *res[k], and seg_status[k] receives segment k's first failure. The steps end once
// every segment has failed or the device fails (the call's status).
wq_status time_steps(const Request& r, wq_points* pts, wq_weights* w, int64_t np, const DBuf& dir, const DBuf& T,
                     const DBuf& Td, const DBuf& S, const DBuf& f, hipStream_t st, int32_t nseg, const int64_t* row0,
                     wq_result* const* res, wq_status* seg_status) {
  std::vector<wq_heat_report> reps(nseg);
  std::vector<wq_status> ss(nseg);
  for (int32_t k = 0; k < nseg; ++k) seg_status[k] = WQ_OK;
  wq_status s = WQ_OK;
  bool live = true;
  for (int step = 0; s == WQ_OK && live && step < r.n_steps; ++step) {
    const double t1 = r.heat.dt * (step + 1);
    if (r.source) {
      k_manufactured_source<<<nblocks(np, 256), 256, 0, st>>>(np, pts->x.as<double>(), t1, r.lambda, r.heat.k,
                                                               f.as<double>());
      if (hipGetLastError() != hipSuccess) s = WQ_EDEVICE;
    }
    if (s == WQ_OK)
      s = heat_step_segments(pts, w, &r.heat, dir.as<uint8_t>(), nullptr, r.source ? f.as<double>() : nullptr,
                             T.as<double>(), Td.as<double>(), S.as<double>(), nseg, row0, reps.data(), ss.data(), st);
    if (s != WQ_OK) break;
    live = false;
    for (int32_t k = 0; k < nseg; ++k) {
      res[k]->newton_iters += reps[k].newton_iters;
      res[k]->cg_iters += reps[k].cg_iters;
      res[k]->residual = reps[k].residual;
      if (seg_status[k] == WQ_OK) seg_status[k] = ss[k];
      live = live || seg_status[k] == WQ_OK;
    }
  }
  return s;
}

// Requests that may share launches: the same heat parameters, step count and source.
bool joinable(const Request& a, const Request& b) {
  const wq_heat_params &p = a.heat, &q = b.heat;
  return p.dt == q.dt && p.theta == q.theta && p.k.kind == q.k.kind && p.k.a == q.k.a && p.k.b == q.k.b &&
         p.tol == q.tol && p.max_newton == q.max_newton && p.cg_rtol == q.cg_rtol && p.max_cg == q.max_cg &&
         p.tangent == q.tangent && a.n_steps == b.n_steps && a.source == b.source &&
         (!a.source || a.lambda == b.lambda);
}

// Runs several requests as one: their meshes joined into a disjoint union (wq_batch), the
// points and weights built once over it (every system binned with the others by size),
// and every time step one heat step over the union with one segment per mesh (the
// tangent is block diagonal): shared launches, each mesh solved as if alone, so every
// request's temperature, iteration counts and residual are those it gets alone. No setup
// is held afterwards.
wq_status run_joined(const std::vector<Request*>& g, hipStream_t st) {
  const int m = (int)g.size();
  std::vector<wq_mesh_desc> descs(m);
  for (int k = 0; k < m; ++k) descs[k] = g[k]->desc;
  wq_batch* b = nullptr;
  wq_status s = wq_batch_create(descs.data(), m, &b);
  if (s == WQ_OK) s = wq_batch_build(b, WQ_FAM_MASS | WQ_FAM_DX | WQ_FAM_DY, 1e-12, (wq_stream)st, nullptr);
  wq_points* pts = s == WQ_OK ? wq_batch_points(b) : nullptr;
  wq_weights* w = s == WQ_OK ? wq_batch_weights(b) : nullptr;
  const int64_t n = pts ? pts->n_rows : 0, nnz = pts ? pts->nnz : 0, np = pts ? pts->n_points : 0;
  DBuf T, Td, S, dir, f;
  if (s == WQ_OK) s = dalloc_n<double>(T, n);
  if (s == WQ_OK) s = dalloc_n<double>(Td, n);
  if (s == WQ_OK) s = dalloc_n<double>(S, nnz);
  if (s == WQ_OK) s = dalloc_n<uint8_t>(dir, n);
  if (s == WQ_OK && g[0]->source) s = dalloc_n<double>(f, np);
  std::vector<int64_t> row0(m), nr(m), nz(m);
  for (int k = 0; k < m && s == WQ_OK; ++k) s = wq_batch_info(b, k, &row0[k], &nr[k], nullptr, &nz[k], nullptr, nullptr);
  if (s == WQ_OK) {
    if (hipMemsetAsync(T.p, 0, n * sizeof(double), st) != hipSuccess ||
        hipMemsetAsync(Td.p, 0, n * sizeof(double), st) != hipSuccess)
      s = WQ_EDEVICE;
    for (int k = 0; k < m && s == WQ_OK; ++k)
      if (hipMemcpyAsync(dir.as<uint8_t>() + row0[k], g[k]->dirichlet.data(), nr[k], hipMemcpyHostToDevice, st) !=
          hipSuccess)
        s = WQ_EDEVICE;
  }
  std::vector<int64_t> seg(m + 1, n);
  std::vector<wq_result*> res(m);
  std::vector<wq_status> ss(m, WQ_OK);
  for (int k = 0; k < m; ++k) {
    seg[k] = row0[k];
    res[k] = &g[k]->res;
    res[k]->n_rows = nr[k];
    res[k]->nnz = nz[k];
    res[k]->joined = m;
  }
  if (s == WQ_OK) s = time_steps(*g[0], pts, w, np, dir, T, Td, S, f, st, m, seg.data(), res.data(), ss.data());
  for (int k = 0; k < m && s == WQ_OK; ++k)
    if (ss[k] == WQ_OK && g[k]->T_out &&
        hipMemcpyAsync(g[k]->T_out, T.as<double>() + row0[k], nr[k] * sizeof(double), hipMemcpyDeviceToHost, st) !=
            hipSuccess)
      s = WQ_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess && s == WQ_OK) s = WQ_EDEVICE;
  for (int k = 0; k < m; ++k) g[k]->res.status = s != WQ_OK ? s : ss[k];
  DBuf* bufs[5] = {&T, &Td, &S, &dir, &f};
  dfree_many(bufs, 5);
  wq_batch_destroy(b);
  return s;
}

// Runs one request. With r->setup, its mesh, points and weights are reused; otherwise
// they are built and returned in *built (nullptr on failure) for the server to hold.
wq_status run_request(Request* r, hipStream_t st, Setup** built) {
  wq_mesh* mesh = r->setup ? r->setup->mesh : nullptr;
  wq_points* pts = r->setup ? r->setup->pts : nullptr;
  wq_weights* w = r->setup ? r->setup->w : nullptr;
  DBuf T, Td, S, dir, f;
  wq_status s = WQ_OK;
  int64_t n = 0, nnz = 0, np = 0;
  if (r->setup) {
    n = pts->n_rows;
    nnz = pts->nnz;
    np = pts->n_points;
  } else {
    s = wq_mesh_create(&r->desc, &mesh);
    if (s == WQ_OK) s = build_points(mesh, 0, st, &pts, &n, &nnz, &np);
    if (s == WQ_OK) s = solve_weights(mesh, pts, WQ_FAM_MASS | WQ_FAM_DX | WQ_FAM_DY, 1e-12, st, &w, nullptr);
  }
  if (s == WQ_OK) s = dalloc_n<double>(T, n);
  if (s == WQ_OK) s = dalloc_n<double>(Td, n);
  if (s == WQ_OK) s = dalloc_n<double>(S, nnz);
  if (s == WQ_OK) s = dalloc_n<uint8_t>(dir, n);
  if (s == WQ_OK && r->source) s = dalloc_n<double>(f, np);
  if (s == WQ_OK) {
    if (hipMemsetAsync(T.p, 0, n * sizeof(double), st) != hipSuccess ||
        hipMemsetAsync(Td.p, 0, n * sizeof(double), st) != hipSuccess ||
        hipMemcpyAsync(dir.p, r->dirichlet.data(), n, hipMemcpyHostToDevice, st) != hipSuccess)
      s = WQ_EDEVICE;
  }
  r->res.n_rows = n;
  r->res.nnz = nnz;
  r->res.joined = 1;
  if (s == WQ_OK) {
    const int64_t seg[2] = {0, n};
    wq_result* res = &r->res;
    wq_status ss = WQ_OK;
    s = time_steps(*r, pts, w, np, dir, T, Td, S, f, st, 1, seg, &res, &ss);
    if (s == WQ_OK) s = ss;
  }
  if (s == WQ_OK && r->T_out) {
    if (hipMemcpyAsync(r->T_out, T.p, n * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      s = WQ_EDEVICE;
  }
  (void)hipStreamSynchronize(st);
  dfree(T);
  dfree(Td);
  dfree(S);
  dfree(dir);
  dfree(f);
  *built = nullptr;
  if (!r->setup) {
    if (s == WQ_OK && r->reuse) {
      Setup* h = new Setup();
      h->face_vtx = r->face_vtx;
      h->ext_fn = r->ext_fn;
      h->split = r->split;
      h->ext_ptr = r->ext_ptr;
      h->coef_ptr = r->coef_ptr;
      h->coef = r->coef;
      h->ctrl = r->ctrl;
      h->nv = r->desc.nv;
      h->mesh = mesh;
      h->pts = pts;
      h->w = w;
      h->bytes = r->est;
      *built = h;
    } else {
      wq_weights_destroy(w);
      wq_points_destroy(pts);
      wq_mesh_destroy(mesh);
    }
  }
  return s;
}

void worker(wq_server* sv) {
  (void)hipSetDevice(sv->device);
  hipStream_t st = nullptr;
  const bool have_stream = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
  for (;;) {
    Request* r = nullptr;
    std::vector<Request*> group;  // r and the requests joined to it
    std::vector<Setup*> evicted;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      // FIFO admission: the oldest request starts as soon as an idle setup of its domain
      // is held, or its estimate fits once idle setups are released (least recently used
      // first)
      auto idle_match = [&](const Request& q) -> Setup* {
        if (!q.reuse) return nullptr;
        for (Setup* h : sv->setups)
          if (!h->busy && same_domain(*h, q)) return h;
        return nullptr;
      };
      auto idle_bytes = [&]() {
        size_t b = 0;
        for (Setup* h : sv->setups)
          if (!h->busy) b += h->bytes;
        return b;
      };
      sv->cv_work.wait(lk, [&] {
        if (sv->queue.empty()) return sv->stopping;
        const Request& q = *sv->queue.front();
        return idle_match(q) != nullptr || sv->in_use - idle_bytes() + q.est <= sv->budget;
      });
      if (sv->queue.empty()) break;
      r = sv->queue.front();
      sv->queue.pop_front();
      r->setup = idle_match(*r);
      if (r->setup) {
        r->setup->busy = true;  // its bytes are already charged
      } else {
        while (sv->in_use + r->est > sv->budget) {
          Setup* lru = nullptr;
          for (Setup* h : sv->setups)
            if (!h->busy && (!lru || h->last_used < lru->last_used)) lru = h;
          sv->setups.erase(std::find(sv->setups.begin(), sv->setups.end(), lru));
          sv->in_use -= lru->bytes;
          evicted.push_back(lru);
        }
        sv->in_use += r->est;
      }
      group.push_back(r);
      // joining: later queued requests with r's parameters that have no idle setup to
      // take over and fit next to it in the budget (no further setups are released)
      if (!r->setup && sv->join > 1) {
        int64_t rows = r->desc.n_fn;
        for (auto it = sv->queue.begin(); it != sv->queue.end() && (int)group.size() < sv->join;) {
          Request* q = *it;
          if (joinable(*r, *q) && !idle_match(*q) && sv->in_use + q->est <= sv->budget &&
              rows + q->desc.n_fn <= sv->join_rows) {
            sv->in_use += q->est;
            rows += q->desc.n_fn;
            group.push_back(q);
            it = sv->queue.erase(it);
          } else {
            ++it;
          }
        }
      }
      for (Request* q : group) {
        q->res.setup_reused = q->setup ? 1 : 0;
        q->res.started = now_s(sv->t0);
      }
    }
    for (Setup* h : evicted) {  // device frees outside the lock
      h->release();
      delete h;
    }
    Setup* built = nullptr;
    const wq_status s = !have_stream        ? WQ_EDEVICE
                        : group.size() == 1 ? run_request(r, st, &built)
                                            : run_joined(group, st);
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      if (r->setup) {
        r->setup->busy = false;
        r->setup->last_used = ++sv->clock;
      } else if (built) {
        built->last_used = ++sv->clock;
        sv->setups.push_back(built);  // r->est stays charged for the held setup
      } else {
        sv->in_use -= r->est;
      }
      for (size_t k = 1; k < group.size(); ++k) sv->in_use -= group[k]->est;
      for (Request* q : group) {
        if (group.size() == 1 || !have_stream) q->res.status = s;  // (else run_joined set each one's own)
        q->res.finished = now_s(sv->t0);
        q->done = true;
      }
    }
    sv->cv_done.notify_all();
    sv->cv_work.notify_all();
  }
  if (have_stream) (void)hipStreamDestroy(st);
}

}  // namespace

extern "C" wq_status wq_server_start(size_t hbm_budget_bytes, int32_t slots, wq_server** out) {
  WQ_CHECK(out && slots >= 1 && slots <= 16 && hbm_budget_bytes > 0, WQ_EINVAL,
           "wq_server_start: need 1..16 slots and a positive budget");
  wq_server* sv = new wq_server();
  WQ_HIP(hipGetDevice(&sv->device));
  sv->budget = hbm_budget_bytes;
  sv->t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < slots; ++i) sv->workers.emplace_back(worker, sv);
  *out = sv;
  return WQ_OK;
}

extern "C" wq_status wq_server_set_join(wq_server* sv, int32_t max_meshes, int64_t max_rows) {
  WQ_CHECK(sv && max_meshes >= 1 && max_meshes <= 4096 && max_rows >= 0, WQ_EINVAL,
           "wq_server_set_join: need 1..4096 meshes and max_rows >= 0");
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->join = max_meshes;
    sv->join_rows = max_rows;
  }
  sv->cv_work.notify_all();
  return WQ_OK;
}

extern "C" wq_status wq_server_submit(wq_server* sv, const wq_request* q, double* T_out, int64_t* ticket) {
  WQ_CHECK(sv && q && ticket, WQ_EINVAL, "wq_server_submit: null argument");
  const wq_mesh_desc& d = q->mesh;
  WQ_CHECK(d.nf > 0 && d.n_fn > 0 && d.face_vtx && d.split && d.ext_ptr && d.ext_fn && d.coef_ptr && d.coef && d.ctrl &&
               q->dirichlet,
           WQ_EINVAL, "wq_server_submit: incomplete request");
  WQ_CHECK(d.dim == 0 || d.dim == 2, WQ_EINVAL, "wq_server_submit: the heat solve is planar (dim 2)");
  WQ_CHECK(q->n_steps >= 0 && q->heat.dt > 0 && q->heat.theta > 0 && q->heat.theta <= 1, WQ_EINVAL,
           "wq_server_submit: bad time stepping");
  Request* r = new Request();
  r->face_vtx.assign(d.face_vtx, d.face_vtx + 4 * (size_t)d.nf);
  r->split.assign(d.split, d.split + d.nf);
  r->ext_ptr.assign(d.ext_ptr, d.ext_ptr + d.nf + 1);
  r->ext_fn.assign(d.ext_fn, d.ext_fn + d.ext_ptr[d.nf]);
  r->coef_ptr.assign(d.coef_ptr, d.coef_ptr + d.nf + 1);
  r->coef.assign(d.coef, d.coef + d.coef_ptr[d.nf]);
  r->ctrl.assign(d.ctrl, d.ctrl + 2 * (size_t)d.n_fn);
  r->dirichlet.assign(q->dirichlet, q->dirichlet + d.n_fn);
  r->desc = d;
  r->desc.face_vtx = r->face_vtx.data();
  r->desc.split = r->split.data();
  r->desc.ext_ptr = r->ext_ptr.data();
  r->desc.ext_fn = r->ext_fn.data();
  r->desc.coef_ptr = r->coef_ptr.data();
  r->desc.coef = r->coef.data();
  r->desc.ctrl = r->ctrl.data();
  r->heat = q->heat;
  r->n_steps = q->n_steps;
  r->source = q->source;
  r->lambda = q->lambda;
  r->reuse = q->reuse_setup != 0;
  r->T_out = T_out;
  r->est = hbm_estimate(d);
  r->res.hbm_estimate = r->est;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stopping || r->est > sv->budget) {
      const bool too_big = r->est > sv->budget;
      delete r;
      WQ_CHECK(!too_big, WQ_ENOMEM, "wq_server_submit: the request's HBM estimate exceeds the whole budget");
      WQ_CHECK(false, WQ_EINVAL, "wq_server_submit: server is stopping");
    }
    r->id = sv->next_id++;
    r->res.submitted = now_s(sv->t0);
    sv->all[r->id] = r;
    sv->queue.push_back(r);
    *ticket = r->id;
  }
  sv->cv_work.notify_all();
  return WQ_OK;
}

extern "C" int wq_server_poll(wq_server* sv, int64_t ticket, int wait, wq_result* out) {
  if (!sv || !out) return WQ_EINVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end()) return WQ_EINVAL;
  Request* r = it->second;
  if (wait) sv->cv_done.wait(lk, [&] { return r->done; });
  if (!r->done) return 0;
  *out = r->res;
  sv->all.erase(it);
  delete r;
  return 1;
}

extern "C" void wq_server_stop(wq_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stopping = true;
  }
  sv->cv_work.notify_all();
  for (auto& t : sv->workers) t.join();
  for (auto& kv : sv->all) delete kv.second;
  for (Setup* h : sv->setups) {
    h->release();
    delete h;
  }
  delete sv;
}
