// Serving loop over independent tangent solves (declared in mbddc.h).
//
// Host runtime above the solver library: a FIFO queue, admission by the
// estimated device footprint, and a pool of worker threads, each driving one
// request at a time on its own HIP stream and its own handle through the public
// C ABI. Requests that run at the same time overlap on the device; a request's
// arithmetic does not depend on what else runs. Device memory comes from one
// caching pool (mbddc_set_allocator), so that a warm server serves requests
// without hipMalloc / hipFree (a hipFree waits for the whole device).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <unordered_map>
#include <new>
#include <thread>
#include <vector>

#include "mbddc.h"

namespace {

struct Job {
  int64_t ticket = 0;
  std::vector<double> coords;
  std::vector<int32_t> elem_nodes, elem_part, dirichlet;
  std::vector<uint32_t> tags;
  mbddc_mesh mesh{};
  mbddc_options opt{};
  int n_steps = 0, nrhs = 0, lagged = 0;
  int64_t ke_total = 0, n_dofs = 0;
  const double* K = nullptr;
  const double* rhs = nullptr;
  double* x = nullptr;
  mbddc_material material{};         // on-device Newton (K == nullptr)
  const double* frames = nullptr;
  const double* u0 = nullptr;
  const double* f_ext = nullptr;
  size_t footprint = 0;
  bool done = false;
  mbddc_request_result res{};
};

// Caching device-memory pool shared by the workers' handles. Sizes are rounded (4 KiB up to
// 1 MiB, 2 MiB above) and blocks kept by rounded size after they are returned; an allocation
// takes a cached block of exactly its rounded size, else a new hipMalloc. Exact classes make
// reuse predictable: once a request has run, a request with the same allocation sizes finds all
// of its blocks cached (a larger block taken for a smaller size could starve a later
// allocation). When a hipMalloc fails, or the cache would hold more than `cap` bytes, cached
// blocks are freed.
struct Pool {
  int device = 0;
  size_t cap = 0;
  std::mutex mu;
  std::multimap<size_t, void*> cache;          // free blocks by size
  std::unordered_map<void*, size_t> in_use;    // block -> size
  size_t bytes_in_use = 0, bytes_cached = 0;
  int64_t mallocs = 0, frees = 0;

  static size_t round(size_t b) {
    const size_t big = size_t(2) << 20;
    return b > (size_t(1) << 20) ? (b + big - 1) / big * big : (b + 4095) / 4096 * 4096;
  }
  // frees cached blocks, largest first, until at most `keep` bytes stay cached (lock held)
  void trim(size_t keep) {
    while (bytes_cached > keep && !cache.empty()) {
      auto it = std::prev(cache.end());
      (void)hipFree(it->second);
      frees++;
      bytes_cached -= it->first;
      cache.erase(it);
    }
  }
  void* alloc(size_t b) {
    b = round(b);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(b);
    if (it != cache.end()) {
      void* p = it->second;
      const size_t sz = it->first;
      cache.erase(it);
      bytes_cached -= sz;
      in_use[p] = sz;
      bytes_in_use += sz;
      return p;
    }
    (void)hipSetDevice(device);
    void* p = nullptr;
    if (hipMalloc(&p, b) != hipSuccess) {
      (void)hipGetLastError();
      trim(0);
      if (hipMalloc(&p, b) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
    }
    mallocs++;
    in_use[p] = b;
    bytes_in_use += b;
    return p;
  }
  void release(void* p) {
    std::lock_guard<std::mutex> lk(mu);
    auto it = in_use.find(p);
    if (it == in_use.end()) return;
    const size_t sz = it->second;
    in_use.erase(it);
    bytes_in_use -= sz;
    cache.emplace(sz, p);
    bytes_cached += sz;
    if (bytes_cached > cap) trim(cap / 2);
  }
};

void* pool_alloc(size_t bytes, void* user) { return static_cast<Pool*>(user)->alloc(bytes); }
void pool_free(void* p, void* user) { static_cast<Pool*>(user)->release(p); }

}  // namespace

struct mbddc_server {
  int device = 0;
  Pool pool;
  size_t budget = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job*> queue;
  std::map<int64_t, Job*> jobs;
  int active = 0;
  size_t admitted = 0;
  bool stop = false;
  int64_t next_ticket = 0;
  std::vector<std::thread> workers;
  std::chrono::steady_clock::time_point t0;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

// Newton iteration with the tangents and internal forces computed on the device.
int run_newton(Job* j, mbddc_ctx* h) {
  mbddc_request_result& r = j->res;
  int st = mbddc_set_material(h, &j->material, j->frames);
  const int64_t n = j->n_dofs;
  std::vector<double> u(j->u0, j->u0 + n), f(n), b(n), du(n);
  std::vector<uint8_t> clamped(n, 0);
  for (int32_t d : j->dirichlet) clamped[d] = 1;
  for (int k = 0; !st && k < j->n_steps; ++k) {
    st = mbddc_set_displacement(h, u.data(), 0, f.data(), 0);
    if (!st && (k == 0 || !j->lagged)) st = mbddc_factor(h);
    if (st) break;
    double nr = 0.0;
    for (int64_t d = 0; d < n; ++d) {
      b[d] = clamped[d] ? 0.0 : j->f_ext[d] - f[d];
      nr += b[d] * b[d];
    }
    r.newton_res[k] = std::sqrt(nr);
    mbddc_info info{};
    st = mbddc_solve(h, 1, b.data(), du.data(), 0, &info);
    r.iterations[k] = info.iterations;
    r.rel_res_true = std::max(r.rel_res_true, info.rel_res_true);
    for (int64_t d = 0; d < n; ++d) u[d] += du[d];
    std::copy(u.begin(), u.end(), j->x + (int64_t)k * n);
    r.n_steps = k + 1;
  }
  return st;
}

void run_job(mbddc_server* s, Job* j, mbddc_ctx* h) {
  mbddc_request_result& r = j->res;
  int st = mbddc_setup_symbolic(h, &j->mesh, &j->opt);
  if (!st && !j->K) {
    st = run_newton(j, h);
    r.status = st;
    const int st2 = mbddc_release(h);
    if (r.status == MBDDC_OK) r.status = st2;
    return;
  }
  for (int k = 0; !st && k < j->n_steps; ++k) {
    st = mbddc_set_tangent(h, j->K + (int64_t)k * j->ke_total, 0);
    if (!st && (k == 0 || !j->lagged)) st = mbddc_factor(h);
    mbddc_info info{};
    if (!st)
      st = mbddc_solve(h, j->nrhs, j->rhs + (int64_t)k * j->nrhs * j->n_dofs,
                       j->x + (int64_t)k * j->nrhs * j->n_dofs, 0, &info);
    r.iterations[k] = info.iterations;
    r.rel_res_true = std::max(r.rel_res_true, info.rel_res_true);
    r.n_steps = k + 1;
  }
  r.status = st;
  const int st2 = mbddc_release(h);   // buffers back to the pool; the handle serves the next request
  if (r.status == MBDDC_OK) r.status = st2;
}

void worker(mbddc_server* s) {
  (void)hipSetDevice(s->device);
  hipStream_t stream = nullptr;
  mbddc_ctx* h = nullptr;
  bool ready = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess;
  ready = ready && mbddc_create(&h, s->device, stream) == MBDDC_OK;
  ready = ready && mbddc_set_allocator(h, pool_alloc, pool_free, &s->pool) == MBDDC_OK;
  for (;;) {
    Job* j = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] {
        if (s->queue.empty()) return s->stop;
        return s->admitted + s->queue.front()->footprint <= s->budget;
      });
      if (s->queue.empty()) break;   // stop requested and nothing left
      j = s->queue.front();
      s->queue.pop_front();
      s->admitted += j->footprint;
      s->active++;
      j->res.t_admit_ms = s->now_ms();
    }
    if (ready) {
      run_job(s, j, h);
    } else {
      j->res.status = MBDDC_ERR_DEVICE;
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->admitted -= j->footprint;
      s->active--;
      j->res.t_done_ms = s->now_ms();
      j->done = true;
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
  }
  if (h) mbddc_destroy(h);
  if (stream) (void)hipStreamDestroy(stream);
}

}  // namespace

extern "C" {

int mbddc_server_create(mbddc_server** out, int hip_device, size_t hbm_budget, int max_active) {
  if (!out || hbm_budget == 0 || max_active < 1 || max_active > 64) return MBDDC_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return MBDDC_ERR_DEVICE;
  if (hip_device < 0 || hip_device >= ndev) return MBDDC_ERR_ARG;
  mbddc_server* s = new (std::nothrow) mbddc_server();
  if (!s) return MBDDC_ERR_OOM;
  s->device = hip_device;
  s->budget = hbm_budget;
  s->pool.device = hip_device;
  s->pool.cap = hbm_budget;
  s->t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < max_active; ++i) s->workers.emplace_back(worker, s);
  *out = s;
  return MBDDC_OK;
}

int mbddc_server_submit(mbddc_server* s, const mbddc_request* q, int64_t* ticket) {
  if (!s || !q || !ticket || q->n_steps < 1 || q->n_steps > 16 || q->nrhs < 1 || q->nrhs > 8 || !q->x)
    return MBDDC_ERR_ARG;
  const bool newton = !q->elem_K;
  if (newton ? (!q->material || !q->u0 || !q->f_ext || q->nrhs != 1 || !q->mesh.coords) : !q->rhs)
    return MBDDC_ERR_ARG;
  const mbddc_mesh& m = q->mesh;
  const int npe = m.elem_type == MBDDC_HEX8 ? 8 : (m.elem_type == MBDDC_HEX27 ? 27 : 0);
  if (!npe || m.n_nodes <= 0 || m.n_elems <= 0 || !m.elem_nodes || !m.elem_part || m.n_dirichlet < 0 ||
      (m.n_dirichlet > 0 && !m.dirichlet_dofs))
    return MBDDC_ERR_ARG;
  size_t fp = 0;
  int st = mbddc_estimate_footprint(1, &m, &q->opt, q->nrhs, &fp);
  if (st) return st;
  if (fp > s->budget) return MBDDC_ERR_OOM;
  Job* j = new (std::nothrow) Job();
  if (!j) return MBDDC_ERR_OOM;
  j->elem_nodes.assign(m.elem_nodes, m.elem_nodes + (int64_t)m.n_elems * npe);
  j->elem_part.assign(m.elem_part, m.elem_part + m.n_elems);
  if (m.coords) j->coords.assign(m.coords, m.coords + 3LL * m.n_nodes);
  if (m.node_tags) j->tags.assign(m.node_tags, m.node_tags + m.n_nodes);
  if (m.n_dirichlet > 0) j->dirichlet.assign(m.dirichlet_dofs, m.dirichlet_dofs + m.n_dirichlet);
  j->mesh = m;
  j->mesh.coords = m.coords ? j->coords.data() : nullptr;
  j->mesh.elem_nodes = j->elem_nodes.data();
  j->mesh.elem_part = j->elem_part.data();
  j->mesh.node_tags = m.node_tags ? j->tags.data() : nullptr;
  j->mesh.dirichlet_dofs = j->dirichlet.empty() ? nullptr : j->dirichlet.data();
  j->opt = q->opt;
  j->opt.tune_table = nullptr;
  j->n_steps = q->n_steps;
  j->nrhs = q->nrhs;
  j->lagged = q->lagged;
  j->ke_total = (int64_t)m.n_elems * (3 * npe) * (3 * npe);
  j->n_dofs = 3LL * m.n_nodes;
  j->K = q->elem_K;
  j->rhs = q->rhs;
  j->x = q->x;
  if (newton) {
    j->material = *q->material;
    j->frames = q->frames;
    j->u0 = q->u0;
    j->f_ext = q->f_ext;
  }
  j->footprint = fp;
  j->res.footprint = fp;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      delete j;
      return MBDDC_ERR_STATE;
    }
    j->ticket = s->next_ticket++;
    j->res.t_submit_ms = s->now_ms();
    s->jobs[j->ticket] = j;
    s->queue.push_back(j);
    *ticket = j->ticket;
  }
  s->cv_work.notify_all();
  return MBDDC_OK;
}

int mbddc_server_wait(mbddc_server* s, int64_t ticket, mbddc_request_result* res) {
  if (!s || !res) return MBDDC_ERR_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return MBDDC_ERR_ARG;
  Job* j = it->second;
  s->cv_done.wait(lk, [&] { return j->done; });
  *res = j->res;
  s->jobs.erase(it);
  delete j;
  return MBDDC_OK;
}

int mbddc_server_state(mbddc_server* s, int32_t* queued, int32_t* active, size_t* admitted_bytes) {
  if (!s) return MBDDC_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  if (queued) *queued = (int32_t)s->queue.size();
  if (active) *active = s->active;
  if (admitted_bytes) *admitted_bytes = s->admitted;
  return MBDDC_OK;
}

int mbddc_server_destroy(mbddc_server* s) {
  if (!s) return MBDDC_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (std::thread& t : s->workers) t.join();
  for (auto& kv : s->jobs) delete kv.second;
  {
    std::lock_guard<std::mutex> lk(s->pool.mu);
    (void)hipSetDevice(s->device);
    s->pool.trim(0);
    for (auto& kv : s->pool.in_use) (void)hipFree(kv.first);   // none once every handle is gone
  }
  delete s;
  return MBDDC_OK;
}

int mbddc_server_pool_stats(mbddc_server* s, int64_t* device_mallocs, int64_t* device_frees, size_t* bytes_in_use,
                            size_t* bytes_cached) {
  if (!s) return MBDDC_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->pool.mu);
  if (device_mallocs) *device_mallocs = s->pool.mallocs;
  if (device_frees) *device_frees = s->pool.frees;
  if (bytes_in_use) *bytes_in_use = s->pool.bytes_in_use;
  if (bytes_cached) *bytes_cached = s->pool.bytes_cached;
  return MBDDC_OK;
}

}  // extern "C"
