// server.hip -- served mode: many registered factors, a stream of requests
// (update or downdate of one factor by a caller-owned V), continuous batching
// onto one GPU.
//
// A worker thread forms batches of at most one request per factor (the
// oldest not yet launched; requests of one factor run in arrival order, in
// successive batches, which the single stream keeps ordered) and enqueues
// each batch with the batched schedule.  Two batch slots, each with its own
// workspace, info words and staging buffer, let the next batch be enqueued
// while the previous one runs.  Admission: a request whose batch workspace
// would exceed the slot's workspace waits for the next batch; a request that
// cannot fit even alone fails with CHOLMOD_ERR_ARG.  A request completes when
// the step that ends its factor's work in the batch has run: after that
// step's launch the worker enqueues the copy of those factors' info words
// and an event, so small factors batched with large ones complete early.  A
// request's latency is the host time from its submission to the worker
// seeing that event.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <functional>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/cholmod_mi355x.h"
#include "internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  int32_t factor;
  const void* V;
  int64_t k;
  int32_t sigma;
  Clock::time_point t_submit;
  bool done = false;
  int status = 0;
  double latency = 0.0;
};

struct Factor {
  void* L;
  int64_t n, ldl;
  int32_t dtype;
  std::deque<uint64_t> queue;  // tickets not yet launched, in arrival order
};

// Requests of a batch that complete together: those whose factors end at
// the same step.
constexpr int kMaxGroups = 32;

struct Group {
  hipEvent_t ev = nullptr;
  std::vector<size_t> idx;  // positions in the slot's batch
};

struct Slot {
  void* ws = nullptr;
  int64_t* d_info = nullptr;
  int64_t* h_info = nullptr;  // pinned
  void* stage = nullptr;      // pinned
  size_t stage_bytes = 0;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<uint64_t> tickets;
  std::vector<int64_t> ks;
  std::vector<char> retired;  // per position in the batch
  Group groups[kMaxGroups];
  int ngroups = 0, next_group = 0;
};

}  // namespace

struct cholmod_server {
  cholmod_server_cfg cfg{};
  int device = 0;
  hipStream_t stream = nullptr;
  Slot slots[2];
  std::mutex mu;
  std::condition_variable cv;
  std::vector<Factor> factors;
  std::unordered_map<uint64_t, Request> reqs;
  uint64_t next_ticket = 1;
  size_t rr = 0;  // round-robin start over factors
  int64_t in_queue = 0, in_flight = 0;
  std::atomic<bool> stop{false};
  std::atomic<int> fatal{0};
  std::thread worker;

  int init_slots() {
    const size_t cap = cfg.max_batch > 0 ? (size_t)cfg.max_batch : 256;
    for (Slot& s : slots) {
      if (hipMalloc(&s.ws, cfg.ws_bytes) != hipSuccess) return CHOLMOD_ERR_HIP;
      if (hipMalloc((void**)&s.d_info, cap * sizeof(int64_t)) != hipSuccess) return CHOLMOD_ERR_HIP;
      if (hipHostMalloc((void**)&s.h_info, cap * sizeof(int64_t), hipHostMallocDefault) !=
          hipSuccess)
        return CHOLMOD_ERR_HIP;
      if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess)
        return CHOLMOD_ERR_HIP;
      for (Group& g : s.groups)
        if (hipEventCreateWithFlags(&g.ev, hipEventDisableTiming) != hipSuccess)
          return CHOLMOD_ERR_HIP;
    }
    return CHOLMOD_OK;
  }

  void release() {
    for (Slot& s : slots) {
      if (s.ws) hipFree(s.ws);
      if (s.d_info) hipFree(s.d_info);
      if (s.h_info) hipHostFree(s.h_info);
      if (s.stage) hipHostFree(s.stage);
      if (s.done) hipEventDestroy(s.done);
      for (Group& g : s.groups)
        if (g.ev) hipEventDestroy(g.ev);
      s = Slot{};
    }
    if (stream) hipStreamDestroy(stream);
    stream = nullptr;
  }

  // Request at position i of slot s gets its status and latency.
  void retire_one(Slot& s, size_t i, Clock::time_point now) {
    if (s.retired[i]) return;
    s.retired[i] = 1;
    --in_flight;
    auto it = reqs.find(s.tickets[i]);
    if (it == reqs.end()) return;
    Request& r = it->second;
    r.status = cholmod_decode_info(s.h_info[i], s.ks[i], nullptr, nullptr);
    r.latency = std::chrono::duration<double>(now - r.t_submit).count();
    r.done = true;
  }

  // Groups whose events have fired, in step order; then the whole slot.
  bool poll_slot(Slot& s) {
    bool progress = false;
    while (s.next_group < s.ngroups && hipEventQuery(s.groups[s.next_group].ev) == hipSuccess) {
      const Clock::time_point now = Clock::now();
      for (size_t i : s.groups[s.next_group].idx) retire_one(s, i, now);
      ++s.next_group;
      progress = true;
    }
    if (hipEventQuery(s.done) == hipSuccess) {
      const Clock::time_point now = Clock::now();
      for (size_t i = 0; i < s.tickets.size(); ++i) retire_one(s, i, now);
      s.tickets.clear();
      s.ks.clear();
      s.retired.clear();
      s.ngroups = s.next_group = 0;
      s.busy = false;
      progress = true;
    }
    return progress;
  }

  // Build and enqueue one batch into slot `s` (lock held).  Returns false
  // if there was nothing to launch.
  bool launch(Slot& s) {
    const size_t cap = cfg.max_batch > 0 ? (size_t)cfg.max_batch : 256;
    std::vector<cholmod_desc> descs;
    std::vector<uint64_t> tickets;
    const size_t nf = factors.size();
    for (size_t c = 0; c < nf && descs.size() < cap; ++c) {
      const size_t f = (rr + c) % nf;
      Factor& F = factors[f];
      if (F.queue.empty()) continue;
      const uint64_t t = F.queue.front();
      Request& r = reqs[t];
      cholmod_desc d;
      d.L = F.L;
      d.V = r.V;
      d.n = F.n;
      d.k = r.k;
      d.ldl = F.ldl;
      d.sigma = r.sigma;
      d.dtype = F.dtype;
      descs.push_back(d);
      const size_t need = chm::batch_workspace_bytes(descs.data(), (int64_t)descs.size());
      if (need == 0 || need > cfg.ws_bytes) {
        descs.pop_back();
        if (need == 0 || descs.empty()) {
          // rejected by the planner, or cannot run even alone: it fails
          // here rather than staying at the head of its factor's queue
          F.queue.pop_front();
          --in_queue;
          r.status = CHOLMOD_ERR_ARG;
          r.latency = std::chrono::duration<double>(Clock::now() - r.t_submit).count();
          r.done = true;
        }
        continue;
      }
      F.queue.pop_front();
      --in_queue;
      tickets.push_back(t);
    }
    rr = nf ? (rr + 1) % nf : 0;
    if (descs.empty()) return false;
    const int64_t count = (int64_t)descs.size();
    const size_t tb = chm::batch_table_bytes(descs.data(), count);
    if (s.stage_bytes < tb) {
      if (s.stage) hipHostFree(s.stage);
      s.stage = nullptr;
      s.stage_bytes = 0;
      if (hipHostMalloc(&s.stage, tb, hipHostMallocDefault) != hipSuccess) {
        fatal = CHOLMOD_ERR_HIP;
        return false;
      }
      s.stage_bytes = tb;
    }
    // completion groups: the requests whose factors end at the same step
    // (factors without steps are final after the preparation launch, so with
    // those of step 0); beyond kMaxGroups - 1 distinct steps the rest
    // complete with the slot
    std::vector<int64_t> last(count);
    std::vector<int64_t> ends;
    for (int64_t i = 0; i < count; ++i) {
      const int64_t st_i = chm::batch_steps_of(descs[i]);
      last[i] = st_i > 0 ? st_i - 1 : 0;
      ends.push_back(last[i]);
    }
    std::sort(ends.begin(), ends.end());
    ends.erase(std::unique(ends.begin(), ends.end()), ends.end());
    if ((int)ends.size() > kMaxGroups - 1) ends.resize(kMaxGroups - 1);
    s.ngroups = (int)ends.size();
    s.next_group = 0;
    for (int g = 0; g < s.ngroups; ++g) s.groups[g].idx.clear();
    for (int64_t i = 0; i < count; ++i) {
      const auto it = std::lower_bound(ends.begin(), ends.end(), last[i]);
      if (it != ends.end() && *it == last[i]) s.groups[it - ends.begin()].idx.push_back((size_t)i);
    }
    int g_next = 0;
    const std::function<int(int64_t)> after_step = [&](int64_t step) -> int {
      while (g_next < s.ngroups && ends[g_next] == step) {
        for (size_t i : s.groups[g_next].idx)
          if (hipMemcpyAsync(s.h_info + i, s.d_info + i, sizeof(int64_t), hipMemcpyDeviceToHost,
                             stream) != hipSuccess)
            return CHOLMOD_ERR_HIP;
        if (hipEventRecord(s.groups[g_next].ev, stream) != hipSuccess) return CHOLMOD_ERR_HIP;
        ++g_next;
      }
      return CHOLMOD_OK;
    };
    int rc = chm::enqueue_batch(descs.data(), count, s.ws, cfg.ws_bytes, s.d_info, stream,
                                s.stage, s.stage_bytes, &after_step);
    // groups never reached (a stopped enqueue) complete with the slot
    s.ngroups = g_next;
    if (rc == CHOLMOD_OK &&
        hipMemcpyAsync(s.h_info, s.d_info, count * sizeof(int64_t), hipMemcpyDeviceToHost,
                       stream) != hipSuccess)
      rc = CHOLMOD_ERR_HIP;
    if (rc == CHOLMOD_OK && hipEventRecord(s.done, stream) != hipSuccess) rc = CHOLMOD_ERR_HIP;
    if (rc != CHOLMOD_OK) {
      for (uint64_t t : tickets) {
        Request& r = reqs[t];
        r.status = rc;
        r.done = true;
      }
      if (rc == CHOLMOD_ERR_HIP) fatal = rc;
      return true;
    }
    s.tickets = std::move(tickets);
    s.ks.clear();
    for (const cholmod_desc& d : descs) s.ks.push_back(d.k);
    s.retired.assign(s.tickets.size(), 0);
    s.busy = true;
    in_flight += count;
    return true;
  }

  void run() {
    hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (!stop) {
      bool progress = false;
      for (Slot& s : slots) {
        if (s.busy) progress |= poll_slot(s);
      }
      if (in_queue > 0 && !fatal) {
        for (Slot& s : slots) {
          if (!s.busy && in_queue > 0) progress |= launch(s);
        }
      }
      cv.notify_all();  // drain() and destroy() wait on the counters
      if (!progress) {
        if (in_flight > 0) {
          // a batch is running: look again shortly
          lk.unlock();
          std::this_thread::sleep_for(std::chrono::microseconds(20));
          lk.lock();
        } else {
          cv.wait(lk, [&] { return stop.load() || in_queue > 0; });
        }
      }
    }
  }
};

extern "C" {

int cholmod_server_create(const cholmod_server_cfg* cfg, cholmod_server** out) {
  if (cfg == nullptr || out == nullptr) return CHOLMOD_ERR_ARG;
  if (cfg->ws_bytes < 4096 || cfg->max_batch < 0 || cfg->max_batch > 65535)
    return CHOLMOD_ERR_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess) return CHOLMOD_ERR_HIP;
  if (cfg->device < 0 || cfg->device >= ndev) return CHOLMOD_ERR_ARG;
  cholmod_server* s = new cholmod_server();
  s->cfg = *cfg;
  s->cfg.ws_bytes = cfg->ws_bytes / 256 * 256;
  s->device = cfg->device;
  int prev = 0;
  hipGetDevice(&prev);
  int rc = CHOLMOD_OK;
  if (hipSetDevice(s->device) != hipSuccess ||
      hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
    rc = CHOLMOD_ERR_HIP;
  if (rc == CHOLMOD_OK) rc = s->init_slots();
  hipSetDevice(prev);
  if (rc != CHOLMOD_OK) {
    s->release();
    delete s;
    return rc;
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return CHOLMOD_OK;
}

int cholmod_server_add_factor(cholmod_server* s, void* L, int64_t n, int64_t ldl, int dtype,
                              int32_t* id) {
  if (s == nullptr || id == nullptr) return CHOLMOD_ERR_ARG;
  if (n < 0 || ldl < (n > 1 ? n : 1) || (n > 0 && L == nullptr)) return CHOLMOD_ERR_ARG;
  if (dtype != CHOLMOD_F64 && dtype != CHOLMOD_F32S) return CHOLMOD_ERR_ARG;
  // the batch planner's own checks (n * ldl must have a byte count)
  cholmod_desc d;
  d.L = L;
  d.V = nullptr;
  d.n = n;
  d.k = 0;
  d.ldl = ldl;
  d.sigma = 1;
  d.dtype = dtype;
  if (chm::batch_workspace_bytes(&d, 1) == 0) return CHOLMOD_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->factors.size() >= 0x7fffffff) return CHOLMOD_ERR_ARG;
  Factor F;
  F.L = L;
  F.n = n;
  F.ldl = ldl;
  F.dtype = dtype;
  s->factors.push_back(F);
  *id = (int32_t)(s->factors.size() - 1);
  return CHOLMOD_OK;
}

int cholmod_server_submit(cholmod_server* s, int32_t id, const void* V, int64_t k, int sigma,
                          uint64_t* ticket) {
  if (s == nullptr || ticket == nullptr) return CHOLMOD_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->fatal) return s->fatal;
  if (id < 0 || (size_t)id >= s->factors.size()) return CHOLMOD_ERR_ARG;
  Factor& F = s->factors[id];
  if (k < 0 || (sigma != 1 && sigma != -1) || (F.n > 0 && k > 0 && V == nullptr))
    return CHOLMOD_ERR_ARG;
  // the batch planner's own checks (sizes whose byte counts overflow)
  cholmod_desc d;
  d.L = F.L;
  d.V = V;
  d.n = F.n;
  d.k = k;
  d.ldl = F.ldl;
  d.sigma = sigma;
  d.dtype = F.dtype;
  if (chm::batch_workspace_bytes(&d, 1) == 0) return CHOLMOD_ERR_ARG;
  const uint64_t t = s->next_ticket++;
  Request r;
  r.factor = id;
  r.V = V;
  r.k = k;
  r.sigma = sigma;
  r.t_submit = Clock::now();
  s->reqs.emplace(t, r);
  F.queue.push_back(t);
  ++s->in_queue;
  *ticket = t;
  s->cv.notify_all();
  return CHOLMOD_OK;
}

int cholmod_server_poll(cholmod_server* s, uint64_t ticket, int* status, double* latency_s) {
  if (s == nullptr) return CHOLMOD_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return CHOLMOD_ERR_ARG;
  if (!it->second.done) return 1;
  if (status) *status = it->second.status;
  if (latency_s) *latency_s = it->second.latency;
  s->reqs.erase(it);
  return CHOLMOD_OK;
}

int cholmod_server_drain(cholmod_server* s) {
  if (s == nullptr) return CHOLMOD_ERR_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv.wait(lk, [&] { return s->fatal != 0 || (s->in_queue == 0 && s->in_flight == 0); });
  return s->fatal;
}

int cholmod_server_destroy(cholmod_server* s) {
  if (s == nullptr) return CHOLMOD_ERR_ARG;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.wait(lk, [&] { return s->fatal != 0 || (s->in_queue == 0 && s->in_flight == 0); });
    s->stop = true;
    s->cv.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  int prev = 0;
  hipGetDevice(&prev);
  hipSetDevice(s->device);
  hipStreamSynchronize(s->stream);
  s->release();
  hipSetDevice(prev);
  delete s;
  return CHOLMOD_OK;
}

}  // extern "C"
