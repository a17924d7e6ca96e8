// Errors, device buffers, scans and the mesh handle.
#include "wq_internal.h"

#include <atomic>

#include <cstring>
#include <mutex>
#include <unordered_map>

namespace wq {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

namespace {

constexpr int CACHE_DEVS = 64;
constexpr size_t CACHE_LIMIT = size_t(8) << 30;  // cached bytes kept per device

struct DevCache {
  std::mutex mu;
  std::unordered_map<size_t, std::vector<void*>> ready;  // size class -> free blocks
  size_t bytes = 0;
};

DevCache* cache_of(int dev) {
  static DevCache caches[CACHE_DEVS];
  return dev >= 0 && dev < CACHE_DEVS ? &caches[dev] : nullptr;
}

size_t size_class(size_t b) {
  if (b <= (size_t(1) << 20)) return (b + 511) & ~size_t(511);
  size_t g = size_t(1) << 20;  // an eighth of the largest power of two not above b
  while ((g << 4) <= b) g <<= 1;
  return (b + g - 1) / g * g;
}

// Hands the (idle) blocks of bufs on device dev to its cache, or back to the runtime
// past the cache's limit. The caller has synchronised that device.
void cache_put(int dev, DBuf* const* bufs, size_t n) {
  DevCache* c = cache_of(dev);
  for (size_t k = 0; k < n; ++k) {
    DBuf& b = *bufs[k];
    if (!b.p || b.dev != dev) continue;
    if (c) {
      std::lock_guard<std::mutex> lk(c->mu);
      if (c->bytes + b.cap <= CACHE_LIMIT) {
        c->ready[b.cap].push_back(b.p);
        c->bytes += b.cap;
        b.p = nullptr;
      }
    }
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = b.cap = 0;
  }
}

// Returns every cached block of the current device dev to the runtime.
void cache_trim(int dev) {
  DevCache* c = cache_of(dev);
  if (!c) return;
  std::lock_guard<std::mutex> lk(c->mu);
  for (auto& kv : c->ready)
    for (void* q : kv.second) (void)hipFree(q);
  c->ready.clear();
  c->bytes = 0;
}

}  // namespace

wq_status dalloc(DBuf& b, size_t bytes) {
  dfree(b);
  if (bytes == 0) bytes = 8;  // keep pointers valid for empty arrays
  const size_t cls = size_class(bytes);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  if (DevCache* c = cache_of(dev)) {
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->ready.find(cls);
    if (it != c->ready.end() && !it->second.empty()) {
      b.p = it->second.back();
      it->second.pop_back();
      c->bytes -= cls;
      b.bytes = bytes;
      b.cap = cls;
      b.dev = dev;
      return WQ_OK;
    }
  }
  hipError_t e = hipMalloc(&b.p, cls);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    cache_trim(dev);
    e = hipMalloc(&b.p, cls);
  }
  if (e != hipSuccess) {
    b.p = nullptr;
    set_error(std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
    return WQ_ENOMEM;
  }
  b.bytes = bytes;
  b.cap = cls;
  b.dev = dev;
  return WQ_OK;
}

void dfree_many(DBuf* const* bufs, size_t n) {
  // one synchronisation per device that holds any of the blocks
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) cur = 0;
  int done[8];
  int nd = 0;
  for (size_t k = 0; k < n; ++k) {
    if (!bufs[k]->p) continue;
    const int dev = bufs[k]->dev;
    bool seen = false;
    for (int q = 0; q < nd; ++q) seen = seen || done[q] == dev;
    if (seen) continue;
    if (dev != cur) (void)hipSetDevice(dev);
    (void)hipDeviceSynchronize();
    cache_put(dev, bufs, n);
    if (dev != cur) (void)hipSetDevice(cur);
    if (nd < 8) done[nd++] = dev;
  }
}

void dfree(DBuf& b) {
  DBuf* one = &b;
  dfree_many(&one, 1);
  b.p = nullptr;
  b.bytes = b.cap = 0;
}

// ------------------------------------------------------------------ exclusive scan
// Blocks of 1024 values (256 threads x 4); block totals are scanned by one block.
static constexpr int SCAN_BS = 256;
static constexpr int SCAN_PER = 4;
static constexpr int SCAN_TILE = SCAN_BS * SCAN_PER;

__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t* sh, int64_t* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_BS; off <<= 1) {
    int64_t add = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  int64_t incl = sh[t];
  *total = sh[SCAN_BS - 1];
  __syncthreads();
  return incl - v;
}

__global__ void k_scan_tiles(int64_t* d, int64_t n, int64_t* aux) {
  __shared__ int64_t sh[SCAN_BS];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER;
  int64_t v[SCAN_PER];
  int64_t sum = 0;
  for (int k = 0; k < SCAN_PER; ++k) {
    v[k] = (base + k < n) ? d[base + k] : 0;
    sum += v[k];
  }
  int64_t tot;
  int64_t ex = block_exclusive_scan(sum, sh, &tot);
  for (int k = 0; k < SCAN_PER; ++k) {
    if (base + k < n) d[base + k] = ex;
    ex += v[k];
  }
  if (threadIdx.x == 0) aux[blockIdx.x] = tot;
}

__global__ void k_scan_aux(int64_t* aux, int64_t nb, int64_t* total) {
  __shared__ int64_t sh[SCAN_BS];
  int64_t carry = 0;
  for (int64_t start = 0; start < nb; start += SCAN_BS) {
    int64_t i = start + threadIdx.x;
    int64_t v = (i < nb) ? aux[i] : 0;
    int64_t tot;
    int64_t ex = block_exclusive_scan(v, sh, &tot);
    if (i < nb) aux[i] = ex + carry;
    carry += tot;
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scan_add(int64_t* d, int64_t n, const int64_t* aux) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER;
  const int64_t a = aux[blockIdx.x];
  for (int k = 0; k < SCAN_PER; ++k)
    if (base + k < n) d[base + k] += a;
}

wq_status exclusive_scan_i64(int64_t* d, int64_t n, int64_t* total, hipStream_t st) {
  const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  DBuf aux;
  WQ_TRY(dalloc_n<int64_t>(aux, (size_t)nb + 1));
  int64_t* dtot = aux.as<int64_t>() + nb;
  if (n > 0) {
    k_scan_tiles<<<(unsigned)nb, SCAN_BS, 0, st>>>(d, n, aux.as<int64_t>());
    k_scan_aux<<<1, SCAN_BS, 0, st>>>(aux.as<int64_t>(), nb, dtot);
    k_scan_add<<<(unsigned)nb, SCAN_BS, 0, st>>>(d, n, aux.as<int64_t>());
  } else {
    WQ_HIP(hipMemsetAsync(dtot, 0, sizeof(int64_t), st));
  }
  // the total is the exclusive prefix at the last index: callers pass count + 1 entries
  // whose last entry is never read as an input
  hipError_t e = n > 0 ? hipMemcpyAsync(total, d + (n - 1), sizeof(int64_t), hipMemcpyDeviceToHost, st)
                       : hipMemcpyAsync(total, dtot, sizeof(int64_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  dfree(aux);
  WQ_HIP(e);
  return WQ_OK;
}

// ------------------------------------------------------------------ side streams
static std::atomic<int> g_side{4};
int side_streams() { return g_side.load(); }

// ------------------------------------------------------------------ kernel timing
static bool g_timing = false;
struct TRec {
  std::string name;
  hipEvent_t a, b;
  int64_t work;
};
static std::vector<TRec> g_trecs;

bool timing_enabled() { return g_timing; }

KTimer::KTimer(const char* n, int64_t w, hipStream_t s) : st(s), name(n), work(w) {
  if (!g_timing || !n) return;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    a = b = nullptr;
    return;
  }
  (void)hipEventRecord(a, st);
}

void KTimer::stop() {
  if (!a) return;
  (void)hipEventRecord(b, st);
  g_trecs.push_back({name, a, b, work});
  a = b = nullptr;
}

}  // namespace wq

using namespace wq;

extern "C" void wq_timing_enable(int on) { g_timing = on != 0; }

extern "C" wq_status wq_set_side_streams(int32_t n) {
  WQ_CHECK(n >= 1 && n <= 8, WQ_EINVAL, "wq_set_side_streams: need 1..8 streams");
  g_side.store(n);
  return WQ_OK;
}

extern "C" int wq_timings(wq_timing* out, int cap) {
  int n = 0;
  for (auto& r : g_trecs) {
    float ms = -1.0f;
    if (hipEventSynchronize(r.b) == hipSuccess) (void)hipEventElapsedTime(&ms, r.a, r.b);
    if (out && n < cap) {
      std::memset(out[n].name, 0, sizeof(out[n].name));
      std::strncpy(out[n].name, r.name.c_str(), sizeof(out[n].name) - 1);
      out[n].ms = ms;
      out[n].work = r.work;
      ++n;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_trecs.clear();
  return n;
}

// ------------------------------------------------------------------ errors (C ABI)
extern "C" const char* wq_strerror(wq_status s) {
  switch (s) {
    case WQ_OK: return "ok";
    case WQ_EINVAL: return "invalid argument";
    case WQ_ENOMEM: return "device allocation failed";
    case WQ_EILLPOSED: return "ill-posed weight system (r_i < n_i)";
    case WQ_ESVD: return "Jacobi SVD did not converge";
    case WQ_ENOCONV: return "iterative solve did not converge";
    case WQ_EDEVICE: return "HIP runtime error";
  }
  return "unknown status";
}

extern "C" const char* wq_last_error(void) { return g_last_error.c_str(); }

// ------------------------------------------------------------------ mesh handle
template <class T>
static wq_status upload(DBuf& b, const T* h, size_t n) {
  WQ_TRY(dalloc_n<T>(b, n));
  if (n) WQ_HIP(hipMemcpy(b.p, h, n * sizeof(T), hipMemcpyHostToDevice));
  return WQ_OK;
}

static void release_mesh(wq_mesh* m) {
  DBuf* all[] = {&m->face_vtx, &m->split, &m->ext_ptr, &m->ext_fn, &m->coef_ptr, &m->coef, &m->ctrl};
  dfree_many(all, sizeof(all) / sizeof(all[0]));
}

extern "C" wq_status wq_mesh_create(const wq_mesh_desc* d, wq_mesh** out) {
  WQ_CHECK(d && out, WQ_EINVAL, "wq_mesh_create: null argument");
  WQ_CHECK(d->nv > 0 && d->nf > 0 && d->n_fn > 0, WQ_EINVAL, "wq_mesh_create: empty mesh");
  WQ_CHECK(d->face_vtx && d->split && d->ext_ptr && d->ext_fn && d->coef_ptr && d->coef && d->ctrl,
           WQ_EINVAL, "wq_mesh_create: null array");
  const int dim = d->dim == 0 ? 2 : d->dim;
  WQ_CHECK(dim == 2 || dim == 3, WQ_EINVAL, "wq_mesh_create: dim must be 2 or 3");
  // host-side validation of the descriptor (cheap, O(size))
  for (int64_t i = 0; i < 4LL * d->nf; ++i)
    WQ_CHECK(d->face_vtx[i] >= 0 && d->face_vtx[i] < d->nv, WQ_EINVAL, "face_vtx out of range");
  WQ_CHECK(d->ext_ptr[0] == 0 && d->coef_ptr[0] == 0, WQ_EINVAL, "ext_ptr/coef_ptr must start at 0");
  for (int32_t f = 0; f < d->nf; ++f) {
    const int64_t m = d->ext_ptr[f + 1] - d->ext_ptr[f];
    WQ_CHECK(m >= 0 && m <= 255, WQ_EINVAL, "functions per face must be in [0,255]");
    const int64_t nsub = d->split[f] ? 4 : 1;
    WQ_CHECK(d->coef_ptr[f + 1] - d->coef_ptr[f] == nsub * m * 16, WQ_EINVAL,
             "coef_ptr inconsistent with ext_ptr/split");
    for (int64_t k = d->ext_ptr[f]; k < d->ext_ptr[f + 1]; ++k) {
      WQ_CHECK(d->ext_fn[k] >= 0 && d->ext_fn[k] < d->n_fn, WQ_EINVAL, "ext_fn out of range");
      if (k > d->ext_ptr[f]) WQ_CHECK(d->ext_fn[k] > d->ext_fn[k - 1], WQ_EINVAL, "ext_fn not ascending");
    }
  }
  wq_mesh* m = new wq_mesh();
  WQ_HIP(hipGetDevice(&m->device));
  m->nv = d->nv;
  m->nf = d->nf;
  m->n_fn = d->n_fn;
  m->dim = dim;
  m->n_ext = d->ext_ptr[d->nf];
  m->n_coef = d->coef_ptr[d->nf];
  m->h_ext_ptr.assign(d->ext_ptr, d->ext_ptr + d->nf + 1);
  wq_status s = WQ_OK;
  if (s == WQ_OK) s = upload(m->face_vtx, d->face_vtx, 4 * (size_t)d->nf);
  if (s == WQ_OK) s = upload(m->split, d->split, (size_t)d->nf);
  if (s == WQ_OK) s = upload(m->ext_ptr, d->ext_ptr, (size_t)d->nf + 1);
  if (s == WQ_OK) s = upload(m->ext_fn, d->ext_fn, (size_t)m->n_ext);
  if (s == WQ_OK) s = upload(m->coef_ptr, d->coef_ptr, (size_t)d->nf + 1);
  if (s == WQ_OK) s = upload(m->coef, d->coef, (size_t)m->n_coef);
  if (s == WQ_OK) s = upload(m->ctrl, d->ctrl, (size_t)dim * d->n_fn);
  if (s != WQ_OK) {
    release_mesh(m);
    delete m;
    return s;
  }
  *out = m;
  return WQ_OK;
}

extern "C" void wq_mesh_destroy(wq_mesh* m) {
  if (!m) return;
  release_mesh(m);
  delete m;
}
