// Serving loop over independent tangent solves (declared in mbddc.h).
//
// Host runtime above the solver library: a FIFO queue, admission by the
// estimated device footprint, and a pool of worker threads, each driving one
// request at a time on its own HIP stream through the public C ABI. Requests
// that run at the same time overlap on the device; each request owns its
// handle, so its arithmetic does not depend on what else runs.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
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
  size_t footprint = 0;
  bool done = false;
  mbddc_request_result res{};
};

}  // namespace

struct mbddc_server {
  int device = 0;
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

void run_job(mbddc_server* s, Job* j, hipStream_t stream) {
  mbddc_request_result& r = j->res;
  mbddc_ctx* h = nullptr;
  int st = mbddc_create(&h, s->device, stream);
  if (!st) st = mbddc_setup_symbolic(h, &j->mesh, &j->opt);
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
  if (h) mbddc_destroy(h);
}

void worker(mbddc_server* s) {
  (void)hipSetDevice(s->device);
  hipStream_t stream = nullptr;
  const bool have_stream = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess;
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
    if (have_stream) {
      run_job(s, j, stream);
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
  s->t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < max_active; ++i) s->workers.emplace_back(worker, s);
  *out = s;
  return MBDDC_OK;
}

int mbddc_server_submit(mbddc_server* s, const mbddc_request* q, int64_t* ticket) {
  if (!s || !q || !ticket || q->n_steps < 1 || q->n_steps > 16 || q->nrhs < 1 || q->nrhs > 8 || !q->elem_K ||
      !q->rhs || !q->x)
    return MBDDC_ERR_ARG;
  const mbddc_mesh& m = q->mesh;
  const int npe = m.elem_type == MBDDC_HEX8 ? 8 : (m.elem_type == MBDDC_HEX27 ? 27 : 0);
  if (!npe || m.n_nodes <= 0 || m.n_elems <= 0 || !m.elem_nodes || !m.elem_part || m.n_dirichlet < 0 ||
      (m.n_dirichlet > 0 && !m.dirichlet_dofs))
    return MBDDC_ERR_ARG;
  size_t fp = 0;
  int st = mbddc_estimate_footprint(1, &m, &q->opt, &fp);
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
  delete s;
  return MBDDC_OK;
}

}  // extern "C"
