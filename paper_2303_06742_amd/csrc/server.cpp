// Batched solves and the serving loop, built on the single-problem C ABI.
//
// Batch: one host thread and one stream per problem, so the FGMRES iterations
// of different problems (each with one host synchronisation per iteration)
// overlap on the GPU.  Server: a FIFO of requests; a worker thread admits the
// first queued request whose device footprint fits next to the running and
// resident problems (evicting idle resident hierarchies, least recently used
// first), builds or reuses its hierarchy, solves, and either keeps the
// hierarchy resident under the caller's problem key or frees it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "stgmg.h"

namespace {

using clk = std::chrono::steady_clock;

struct Request {
  uint64_t ticket = 0, key = 0;
  stgmg_params prm{};
  std::vector<double> K, rhs, x;
  double rtol = 1e-8;
  int64_t n = 0, resident = 0, peak = 0;
  int state = 0;  // 0 queued, 1 running, 2 done
  stgmg_status status = STGMG_PENDING;
  std::string message;  // error text of a failed request
  stgmg_info info{};
  clk::time_point t_submit, t_done;
};

struct Resident {
  uint64_t key = 0;
  stgmg_handle* h = nullptr;
  double* rhs = nullptr;
  double* x = nullptr;
  int64_t n = 0, bytes = 0;
  bool busy = false;
  uint64_t last_use = 0;
};

}  // namespace

struct stgmg_server {
  int64_t budget = 0, used = 0;
  int slots = 1, resident_max = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::map<uint64_t, std::unique_ptr<Request>> all;
  std::vector<Resident> res;
  std::set<uint64_t> active_keys;  // keys with a request running: later slabs of that problem wait
  std::vector<std::thread> workers;
  uint64_t next_ticket = 1, clock = 0;
  int running = 0;
  bool stop = false;
};

namespace {

void free_resident(Resident& r) {
  if (r.h) stgmg_destroy(r.h);
  // stream-ordered frees: no device-wide synchronisation while other problems run
  if (r.rhs) (void)hipFreeAsync(r.rhs, nullptr);
  if (r.x) (void)hipFreeAsync(r.x, nullptr);
  r.h = nullptr;
  r.rhs = r.x = nullptr;
}

// Under the lock: find a runnable request (resident and idle, or fitting after
// evicting idle residents).  Returns the request and the resident slot index
// (-1 for a new hierarchy); nullptr if none can start now.
Request* pick(stgmg_server* S, int* slot, std::vector<Resident>* evicted) {
  for (auto it = S->queue.begin(); it != S->queue.end(); ++it) {
    Request* q = *it;
    if (q->key != 0) {
      if (S->active_keys.count(q->key)) continue;  // same problem running: keep its slabs in order
      bool found = false;
      for (size_t i = 0; i < S->res.size(); ++i)
        if (S->res[i].key == q->key) {
          *slot = int(i);
          found = true;
          break;
        }
      if (found) {
        S->queue.erase(it);
        return q;
      }
    }
    int64_t free_b = S->budget - S->used;
    if (q->peak > free_b) {
      // evict idle residents, least recently used first
      std::vector<size_t> idle;
      for (size_t i = 0; i < S->res.size(); ++i)
        if (!S->res[i].busy) idle.push_back(i);
      std::sort(idle.begin(), idle.end(), [&](size_t a, size_t b) { return S->res[a].last_use < S->res[b].last_use; });
      int64_t could = free_b;
      size_t take = 0;
      while (could < q->peak && take < idle.size()) could += S->res[idle[take++]].bytes;
      if (could < q->peak) continue;  // does not fit even after evictions: try a later request
      std::vector<size_t> drop(idle.begin(), idle.begin() + take);
      std::sort(drop.rbegin(), drop.rend());
      for (size_t i : drop) {
        S->used -= S->res[i].bytes;
        evicted->push_back(S->res[i]);
        S->res.erase(S->res.begin() + i);
      }
    }
    S->used += q->peak;
    *slot = -1;
    S->queue.erase(it);
    return q;
  }
  return nullptr;
}

void worker(stgmg_server* S) {
  (void)hipSetDevice(0);
  for (;;) {
    Request* q = nullptr;
    int slot = -1;
    std::vector<Resident> evicted;
    Resident R;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait(lk, [&] {
        if (S->stop && S->queue.empty()) return true;
        q = pick(S, &slot, &evicted);
        return q != nullptr;
      });
      if (!q) return;
      q->state = 1;
      S->running++;
      if (q->key != 0) S->active_keys.insert(q->key);
      if (slot >= 0) {
        // copy the resident entry now: other workers may erase entries (and shift
        // indices) as soon as the lock is released; a busy entry is never evicted
        S->res[slot].busy = true;
        S->res[slot].last_use = ++S->clock;
        R = S->res[slot];
      }
    }
    for (auto& e : evicted) free_resident(e);
    const bool fresh = slot < 0;
    stgmg_status st = STGMG_OK;
    std::string msg;
    auto hip_fail = [&](hipError_t e, const char* what) {
      if (e == hipSuccess) return false;
      msg = std::string(what) + ": " + hipGetErrorString(e);
      return true;
    };
    if (fresh) {
      R.key = q->key;
      R.n = q->n;
      stgmg_params p = q->prm;
      p.K_cells = q->K.empty() ? nullptr : q->K.data();
      // no graph capture: the other workers issue null-stream copies at any time, which the
      // runtime rejects (and which break the capture) while a stream is capturing
      p.graph = 0;
      st = stgmg_setup(&p, nullptr, &R.h);
      if (st != STGMG_OK) msg = std::string("setup: ") + stgmg_last_error();
      if (st == STGMG_OK &&
          (hip_fail(hipMallocAsync(reinterpret_cast<void**>(&R.rhs), q->n * sizeof(double), nullptr), "hipMallocAsync") ||
           hip_fail(hipMallocAsync(reinterpret_cast<void**>(&R.x), q->n * sizeof(double), nullptr), "hipMallocAsync")))
        st = STGMG_ERR_OOM;
      R.bytes = q->resident;
    }
    if (st == STGMG_OK) {
      if (hip_fail(hipMemcpy(R.rhs, q->rhs.data(), q->n * sizeof(double), hipMemcpyHostToDevice), "rhs upload") ||
          hip_fail(hipMemset(R.x, 0, q->n * sizeof(double)), "x0 clear"))
        st = STGMG_ERR_HIP;
    }
    if (st == STGMG_OK) {
      st = stgmg_solve(R.h, R.rhs, R.x, q->rtol, 30, 1000, &q->info);
      if (st != STGMG_OK && st != STGMG_NOT_CONVERGED) msg = std::string("solve: ") + stgmg_last_error();
    }
    if (st == STGMG_OK || st == STGMG_NOT_CONVERGED) {
      q->x.resize(q->n);
      if (hip_fail(hipMemcpy(q->x.data(), R.x, q->n * sizeof(double), hipMemcpyDeviceToHost), "x download"))
        st = STGMG_ERR_HIP;
    }
    std::vector<double>().swap(q->rhs);
    bool keep = false;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      q->status = st;
      q->message = msg;
      q->state = 2;
      q->t_done = clk::now();
      S->running--;
      if (q->key != 0) S->active_keys.erase(q->key);
      if (fresh) {
        S->used -= q->peak;  // setup temporaries are gone; the hierarchy holds `resident`
        keep = st == STGMG_OK && q->key != 0 && int(S->res.size()) < S->resident_max;
        if (keep) {
          R.busy = false;
          R.last_use = ++S->clock;
          S->used += R.bytes;
          S->res.push_back(R);
        }
      } else {
        for (auto& r : S->res)
          if (r.key == R.key) r.busy = false;
        keep = true;
      }
    }
    if (!keep) free_resident(R);
    S->cv.notify_all();
  }
}

}  // namespace

extern "C" {

stgmg_status stgmg_solve_batch(int32_t count, stgmg_handle* const* handles, const double* const* rhs_dev,
                               double* const* x_dev, double rtol, int32_t restart, int32_t max_iters,
                               stgmg_info* infos, stgmg_status* statuses) {
  if (count < 0 || (count > 0 && (!handles || !rhs_dev || !x_dev))) return STGMG_ERR_INVALID_ARG;
  std::vector<stgmg_status> st(count, STGMG_OK);
  std::atomic<int> next(0);
  auto run = [&] {
    (void)hipSetDevice(0);
    for (int i; (i = next++) < count;)
      st[i] = stgmg_solve(handles[i], rhs_dev[i], x_dev[i], rtol, restart, max_iters, infos ? &infos[i] : nullptr);
  };
  const int nt = std::min(count, 16);
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(run);
  if (count > 0) run();
  for (auto& t : th) t.join();
  stgmg_status out = STGMG_OK;
  for (int i = 0; i < count; ++i) {
    if (statuses) statuses[i] = st[i];
    if (st[i] != STGMG_OK && out == STGMG_OK) out = st[i];
  }
  return out;
}

stgmg_status stgmg_server_create(int64_t hbm_budget, int32_t max_slots, int32_t resident_max, stgmg_server** out) {
  if (!out || hbm_budget <= 0 || max_slots < 1 || max_slots > 64 || resident_max < 0) return STGMG_ERR_INVALID_ARG;
  auto* S = new stgmg_server();
  S->budget = hbm_budget;
  S->slots = max_slots;
  S->resident_max = resident_max;
  for (int i = 0; i < max_slots; ++i) S->workers.emplace_back(worker, S);
  *out = S;
  return STGMG_OK;
}

stgmg_status stgmg_server_submit(stgmg_server* S, const stgmg_params* params, uint64_t problem_key,
                                 const double* rhs_host, double rtol, uint64_t* ticket) {
  if (!S || !params || !rhs_host || !ticket) return STGMG_ERR_INVALID_ARG;
  auto q = std::make_unique<Request>();
  int64_t n = 0, resident = 0, peak = 0;
  stgmg_status st = stgmg_footprint(params, 30, &n, &resident, &peak);
  if (st != STGMG_OK) return st;
  const int64_t io = 2 * n * int64_t(sizeof(double));
  q->n = n;
  q->resident = resident + io;
  q->peak = peak + io;
  if (q->peak > S->budget) return STGMG_ERR_OOM;
  q->key = problem_key;
  q->prm = *params;
  if (params->K_cells) {
    int64_t nc = 1;
    for (int a = 0; a < params->dim; ++a) nc *= int64_t(params->coarse_cells) << (params->levels - 1);
    q->K.assign(params->K_cells, params->K_cells + nc);
  }
  q->prm.K_cells = nullptr;
  q->rhs.assign(rhs_host, rhs_host + n);
  q->rtol = rtol;
  q->t_submit = clk::now();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    q->ticket = S->next_ticket++;
    *ticket = q->ticket;
    S->queue.push_back(q.get());
    S->all[q->ticket] = std::move(q);
  }
  S->cv.notify_all();
  return STGMG_OK;
}

stgmg_status stgmg_server_poll(stgmg_server* S, uint64_t ticket, double* x_host, stgmg_info* info,
                               double* latency_ms) {
  if (!S) return STGMG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return STGMG_ERR_INVALID_ARG;
  Request* q = it->second.get();
  if (q->state != 2) return STGMG_PENDING;
  if (x_host && !q->x.empty()) std::copy(q->x.begin(), q->x.end(), x_host);
  if (info) *info = q->info;
  if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(q->t_done - q->t_submit).count();
  return q->status;
}

const char* stgmg_server_message(stgmg_server* S, uint64_t ticket) {
  if (!S) return "";
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end() || it->second->state != 2) return "";
  return it->second->message.c_str();
}

stgmg_status stgmg_server_destroy(stgmg_server* S) {
  if (!S) return STGMG_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  for (auto& t : S->workers) t.join();
  for (auto& r : S->res) free_resident(r);
  delete S;
  return STGMG_OK;
}

}  // extern "C"
