// Serving loop for energy-density jobs (rpa_server_* in rpa.h).
//
// A job is (cell, one frequency, a block of coarse points, N_l).  Worker
// threads each own a HIP stream and, per cell, a handle whose workspaces are
// released after every job; the dispatcher admits the oldest waiting job that
// fits the HBM budget as soon as a worker is idle, so jobs that arrive while
// others run start as slots and memory free up, and the kernels of
// concurrent jobs overlap on the device.  Batching of start vectors happens
// inside one job only, so a job's result does not depend on what else runs.
#include "rpa.h"
#include "internal.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct CellDef {
  rpa_setup_params prm;           // pointers below refer to the server's copies
  std::vector<double> eps;
  std::vector<int64_t> proj_ptr, proj_idx;   // host copies of the projectors
  std::vector<double> proj_val, proj_gamma;
  double* v = nullptr;            // device copies (real executor only)
  double* psi = nullptr;
  long long N = 0;
  int nocc = 0;
};

struct Job {
  int64_t id = 0;
  int cell = 0;
  double omega = 0.0;
  std::vector<int64_t> pts;
  int n_lanczos = 0;
  double* out = nullptr;
  uint64_t footprint = 0;
  rpa_job_info info{};
  bool done = false;
};

// Workspace bytes a job needs: exactly the buffers lanczos_energy_density
// allocates for a batch of start vectors (the engine computes them from the
// same launch shape it will use), plus a margin for the HIP runtime.
uint64_t job_footprint(const CellDef& c, int n_pts, int n_lanczos, int num_cu, int device_ok) {
  const int B = std::min(c.prm.batch > 0 ? c.prm.batch : 64, n_pts);
  return rpa::lanczos_workspace_bytes(c.prm, B, n_lanczos, num_cu, device_ok != 0) + (16ULL << 20);
}

}  // namespace

struct rpa_server_s {
  rpa_server_params prm{};
  std::vector<std::unique_ptr<CellDef>> cells;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job*> waiting;
  std::map<int64_t, std::unique_ptr<Job>> jobs;
  int64_t next_id = 1;
  uint64_t in_use = 0;
  uint64_t resident = 0;
  uint64_t high_water = 0;       // max of resident + in_use since creation
  int idle = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  std::string err;
  int num_cu = 256;              // compute units of the device (fake executor: 256)
  int device_ok = 0;             // a HIP device backs the workers
};

namespace {

void worker_main(rpa_server_s* S, int device) {
  hipStream_t stream = nullptr;
  const bool fake = S->prm.fake_executor_us > 0;
  if (!fake) {
    (void)hipSetDevice(device);
    if (hipStreamCreate(&stream) != hipSuccess) stream = nullptr;   // default priority
  }
  std::map<int, rpa_handle> handles;
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    // admission: oldest job that fits the budget
    Job* job = nullptr;
    for (;;) {
      if (S->stop) break;
      for (auto it = S->waiting.begin(); it != S->waiting.end(); ++it) {
        const uint64_t cap = S->prm.hbm_budget;
        if (cap == 0 || S->resident + S->in_use + (*it)->footprint <= cap) {
          job = *it;
          S->waiting.erase(it);
          break;
        }
      }
      if (job) break;
      ++S->idle;
      S->cv_work.wait(lk);
      --S->idle;
    }
    if (!job) break;
    // the cell table may grow (rpa_server_add_cell) while this job runs:
    // take the cell's address while the lock is held
    const CellDef* cell = S->cells[job->cell].get();
    S->in_use += job->footprint;
    S->high_water = std::max(S->high_water, S->resident + S->in_use);
    job->info.t_start = now_s();
    lk.unlock();

    rpa_status st = RPA_OK;
    rpa_stats js{};
    if (fake) {
      std::this_thread::sleep_for(std::chrono::microseconds(S->prm.fake_executor_us));
      js.n_systems = (int64_t)job->pts.size() * cell->nocc * job->n_lanczos;
    } else {
      rpa_handle h = nullptr;
      auto it = handles.find(job->cell);
      if (it == handles.end()) {
        st = rpa_setup(&cell->prm, stream, &h);
        if (st == RPA_OK) handles[job->cell] = h;
      } else {
        h = it->second;
      }
      if (st == RPA_OK)
        st = lanczos_energy_density(h, 1, &job->omega, (int32_t)job->pts.size(), job->pts.data(),
                                    job->n_lanczos, job->out, &js, stream);
      if (h && st != RPA_E_HIP && st != RPA_E_STATE) rpa_release_workspace(h);
    }

    lk.lock();
    S->in_use -= job->footprint;
    job->info.t_finish = now_s();
    job->info.status = st;
    job->info.stats = js;
    job->done = true;
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
  lk.unlock();
  for (auto& kv : handles) rpa_destroy(kv.second);
  if (stream) (void)hipStreamDestroy(stream);
}

}  // namespace

extern "C" {

rpa_status rpa_server_create(const rpa_server_params* p, rpa_server* out) {
  if (!p || !out) return RPA_E_ARG;
  if (p->n_workers < 1 || p->n_workers > 16 || p->fake_executor_us < 0) return RPA_E_ARG;
  auto* S = new rpa_server_s();
  S->prm = *p;
  int device = 0;
  if (p->fake_executor_us == 0 && hipGetDevice(&device) != hipSuccess) {
    (void)hipGetLastError();
    delete S;
    return RPA_E_HIP;
  }
  if (p->fake_executor_us == 0) {
    S->device_ok = 1;
    if (hipDeviceGetAttribute(&S->num_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
      (void)hipGetLastError();
      S->num_cu = 256;
    }
  }
  for (int i = 0; i < p->n_workers; ++i) S->workers.emplace_back(worker_main, S, device);
  *out = S;
  return RPA_OK;
}

rpa_status rpa_server_add_cell(rpa_server S, const rpa_setup_params* p, int32_t* cell_id) {
  if (!S || !p || !cell_id) return RPA_E_ARG;
  if (p->n_proj < 0 || p->n_proj > rpa::kMaxProj) return RPA_E_ARG;
  auto c = std::make_unique<CellDef>();
  c->prm = *p;
  // serving cells keep the occupied Galerkin space (the extra eigenpairs
  // would need a server copy of their own)
  c->prm.n_extra = 0;
  c->prm.psi_extra = nullptr;
  c->prm.eps_extra = nullptr;
  c->N = (long long)p->n[0] * p->n[1] * p->n[2];
  c->nocc = p->n_occ;
  if (c->N <= 0 || c->nocc < 1 || !p->eps) return RPA_E_ARG;
  c->eps.assign(p->eps, p->eps + p->n_occ);
  c->prm.eps = c->eps.data();
  if (p->n_proj > 0) {
    // the workers' rpa_setup validates the contents; only the extents here
    if (!p->proj_ptr || !p->proj_idx || !p->proj_val || !p->proj_gamma) return RPA_E_ARG;
    const int64_t nnz = p->proj_ptr[p->n_proj];
    if (p->proj_ptr[0] != 0 || nnz < 0) return RPA_E_ARG;
    c->proj_ptr.assign(p->proj_ptr, p->proj_ptr + p->n_proj + 1);
    c->proj_idx.assign(p->proj_idx, p->proj_idx + nnz);
    c->proj_val.assign(p->proj_val, p->proj_val + nnz);
    c->proj_gamma.assign(p->proj_gamma, p->proj_gamma + p->n_proj);
    c->prm.proj_ptr = c->proj_ptr.data();
    c->prm.proj_idx = c->proj_idx.data();
    c->prm.proj_val = c->proj_val.data();
    c->prm.proj_gamma = c->proj_gamma.data();
  }
  // The server keeps V and psi (FP64); each worker's rpa_setup keeps V in FP64
  // and FP32, psi, eps, the nu^1/2 and nu diagonals and the three per-axis
  // eigenbases.
  const uint64_t server_copy = (uint64_t)c->N * 8 * (1 + (uint64_t)c->nocc);
  uint64_t bytes = server_copy + (uint64_t)c->N * (4 + 2 * 8) + (uint64_t)c->nocc * 8;
  for (int d = 0; d < 3; ++d) bytes += (uint64_t)p->n[d] * p->n[d] * 8;
  if (p->n_proj > 0) {
    // both projector layouts: indices, FP32 and FP64 values twice, point pointers
    const uint64_t nnz = (uint64_t)p->proj_ptr[p->n_proj];
    bytes += 2 * nnz * (4 + 4 + 8) + ((uint64_t)c->N + 1) * 4;
  }
  if (S->prm.fake_executor_us == 0) {
    if (!p->v_loc || !p->psi) return RPA_E_ARG;
    if (hipMalloc((void**)&c->v, c->N * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&c->psi, (size_t)c->N * c->nocc * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      if (c->v) (void)hipFree(c->v);
      return RPA_E_OOM;
    }
    if (hipMemcpy(c->v, p->v_loc, c->N * sizeof(double), hipMemcpyDeviceToDevice) != hipSuccess ||
        hipMemcpy(c->psi, p->psi, (size_t)c->N * c->nocc * sizeof(double),
                  hipMemcpyDeviceToDevice) != hipSuccess) {
      (void)hipFree(c->v);
      (void)hipFree(c->psi);
      return RPA_E_HIP;
    }
    c->prm.v_loc = c->v;
    c->prm.psi = c->psi;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  // each worker holds its own resident copy once it has run a job of this cell
  S->resident += server_copy + bytes * (uint64_t)S->prm.n_workers;
  S->high_water = std::max(S->high_water, S->resident + S->in_use);
  S->cells.push_back(std::move(c));
  *cell_id = (int32_t)S->cells.size() - 1;
  return RPA_OK;
}

rpa_status rpa_server_submit(rpa_server S, int32_t cell_id, double omega, int32_t n_pts,
                             const int64_t* pts, int32_t n_lanczos, double* d_out,
                             int64_t* job_id) {
  if (!S || !pts || !job_id || n_pts < 1 || n_lanczos < 1 || n_lanczos > rpa::kMaxLanczosPublic)
    return RPA_E_ARG;
  if (!(omega > 0)) return RPA_E_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  if (cell_id < 0 || cell_id >= (int32_t)S->cells.size()) return RPA_E_ARG;
  if (S->prm.fake_executor_us == 0 && !d_out) return RPA_E_ARG;
  const CellDef& c = *S->cells[cell_id];
  for (int i = 0; i < n_pts; ++i)
    if (pts[i] < 0 || pts[i] >= c.N) return RPA_E_ARG;
  auto j = std::make_unique<Job>();
  j->id = S->next_id++;
  j->cell = cell_id;
  j->omega = omega;
  j->pts.assign(pts, pts + n_pts);
  j->n_lanczos = n_lanczos;
  j->out = d_out;
  j->footprint = job_footprint(c, n_pts, n_lanczos, S->num_cu, S->device_ok);
  if (S->prm.hbm_budget && S->resident + j->footprint > S->prm.hbm_budget) return RPA_E_OOM;
  j->info.t_submit = now_s();
  j->info.footprint = (int64_t)j->footprint;
  j->info.status = -1;
  *job_id = j->id;
  S->waiting.push_back(j.get());
  S->jobs[j->id] = std::move(j);
  S->cv_work.notify_one();
  return RPA_OK;
}

rpa_status rpa_server_wait(rpa_server S, int64_t job_id, rpa_job_info* info) {
  if (!S) return RPA_E_ARG;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->jobs.find(job_id);
  if (it == S->jobs.end()) return RPA_E_ARG;
  Job* j = it->second.get();
  S->cv_done.wait(lk, [&] { return j->done; });
  if (info) *info = j->info;
  return RPA_OK;
}

rpa_status rpa_server_status(rpa_server S, int32_t* waiting, int32_t* running, uint64_t* in_use,
                             uint64_t* high_water) {
  if (!S) return RPA_E_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  if (waiting) *waiting = (int32_t)S->waiting.size();
  if (running) *running = S->prm.n_workers - S->idle - (S->stop ? S->prm.n_workers : 0);
  if (in_use) *in_use = S->in_use;
  if (high_water) *high_water = S->high_water;
  return RPA_OK;
}

rpa_status rpa_server_destroy(rpa_server S) {
  if (!S) return RPA_OK;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->waiting.empty() && S->in_use == 0; });
    S->stop = true;
    S->cv_work.notify_all();
  }
  for (auto& t : S->workers) t.join();
  for (auto& c : S->cells) {
    if (c->v) (void)hipFree(c->v);
    if (c->psi) (void)hipFree(c->psi);
  }
  delete S;
  return RPA_OK;
}

}  // extern "C"
