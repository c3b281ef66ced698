// server.hip -- served mode: many registered factors, a stream of requests
// (update or downdate of one factor by a caller-owned V), continuous batching
// onto one GPU.
//
// Admission by HBM footprint.  The server owns one device arena of
// cfg->ws_bytes bytes (its HBM budget besides the factors).  A worker thread
// forms a batch from the waiting requests, oldest first, at most one per
// factor and none of a factor whose previous request is still running (a
// factor's requests run in submission order), taking each request whose
// workspace (its private copy of V, its rotation records and block maps) still fits
// into the free part of the arena; a request that could not fit even into
// an empty arena fails with CHOLMOD_ERR_ARG.  The batch takes its arena
// range, one of the server's streams and runs as one persistent launch (the
// queued batch of cholmod_update_batched, so each result is bit for bit the
// single-factor result).
//
// Overlap.  Up to cfg->streams batches are in flight at once, each on its own
// stream: a batch formed while others run is launched at once, and its
// workgroups take the compute units that the running batches' workgroups
// leave (a launch holds at most one workgroup per unit of work, so a small
// batch runs beside a large one, and a new batch fills the tail of an old
// one).
//
// Completion.  The last workgroup to finish a factor of the batch writes
// the factor's info word into host-mapped memory; the worker sees it and
// completes that request while the rest of the batch still runs, and the
// factor can take its next request at once.  A request's latency is the
// host time from its submission to that point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/cholmod_mi355x.h"
#include "internal.h"

namespace {

using Clock = std::chrono::steady_clock;
constexpr size_t kAlign = 256;
constexpr int kMaxStreams = 16;
constexpr int64_t kDoneEmpty = INT64_MIN;  // a done word not yet written

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

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
  bool busy = false;  // a request of this factor is in flight
};

// First-fit allocator over the arena's byte range.
class Arena {
 public:
  void reset(size_t bytes) {
    free_.clear();
    if (bytes) free_[0] = bytes;
  }
  size_t largest() const {
    size_t m = 0;
    for (const auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;  // offset -> bytes
};

// One stream with the batch that runs on it.
struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;  // the batch's launches and info copy have run
  int64_t* h_info = nullptr;  // pinned: info words copied back after the batch
  int64_t* h_done = nullptr;  // pinned, mapped: per-factor done words
  int64_t* d_done = nullptr;  // device address of h_done
  void* stage = nullptr;      // pinned: the batch tables
  size_t stage_bytes = 0;
  bool busy = false;
  size_t off = 0, bytes = 0;  // arena range
  std::vector<uint64_t> tickets;
  std::vector<int64_t> ks;
  std::vector<char> retired;
  size_t left = 0;  // requests not yet retired
};

}  // namespace

struct cholmod_server {
  cholmod_server_cfg cfg{};
  int device = 0;
  size_t cap = 256;  // requests per batch
  int nslots = 4;
  char* arena_base = nullptr;
  Arena arena;
  Slot slots[kMaxStreams];
  std::mutex mu;
  std::condition_variable cv;
  std::vector<Factor> factors;
  std::unordered_map<uint64_t, Request> reqs;
  std::deque<uint64_t> queue;  // waiting tickets, oldest first
  uint64_t next_ticket = 1;
  int64_t in_flight = 0;
  std::atomic<bool> stop{false};
  std::atomic<int> fatal{0};
  std::thread worker;

  int init() {
    if (hipMalloc((void**)&arena_base, cfg.ws_bytes) != hipSuccess) return CHOLMOD_ERR_HIP;
    arena.reset(cfg.ws_bytes);
    for (int i = 0; i < nslots; ++i) {
      Slot& s = slots[i];
      if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess)
        return CHOLMOD_ERR_HIP;
      if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess)
        return CHOLMOD_ERR_HIP;
      if (hipHostMalloc((void**)&s.h_info, cap * sizeof(int64_t), hipHostMallocDefault) !=
          hipSuccess)
        return CHOLMOD_ERR_HIP;
      if (hipHostMalloc((void**)&s.h_done, cap * sizeof(int64_t),
                        hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
        return CHOLMOD_ERR_HIP;
      if (hipHostGetDevicePointer((void**)&s.d_done, s.h_done, 0) != hipSuccess)
        return CHOLMOD_ERR_HIP;
    }
    return CHOLMOD_OK;
  }

  void release() {
    for (Slot& s : slots) {
      if (s.h_info) hipHostFree(s.h_info);
      if (s.h_done) hipHostFree(s.h_done);
      if (s.stage) hipHostFree(s.stage);
      if (s.done) hipEventDestroy(s.done);
      if (s.stream) hipStreamDestroy(s.stream);
      s = Slot{};
    }
    if (arena_base) hipFree(arena_base);
    arena_base = nullptr;
  }

  void finish(Request& r, int status, Clock::time_point now) {
    r.status = status;
    r.latency = std::chrono::duration<double>(now - r.t_submit).count();
    r.done = true;
  }

  // Request at position i of slot s completes with the raw info word `info`.
  void retire_one(Slot& s, size_t i, int64_t info, Clock::time_point now) {
    if (s.retired[i]) return;
    s.retired[i] = 1;
    --s.left;
    --in_flight;
    auto it = reqs.find(s.tickets[i]);
    if (it == reqs.end()) return;
    Request& r = it->second;
    factors[r.factor].busy = false;
    finish(r, cholmod_decode_info(info, s.ks[i], nullptr, nullptr), now);
  }

  // Factors whose done word has been written; then the whole batch.
  bool poll_slot(Slot& s) {
    bool progress = false;
    const Clock::time_point now = Clock::now();
    for (size_t i = 0; i < s.tickets.size(); ++i) {
      if (s.retired[i]) continue;
      const int64_t w = __atomic_load_n(&s.h_done[i], __ATOMIC_ACQUIRE);
      if (w != kDoneEmpty) {
        retire_one(s, i, w, now);
        progress = true;
      }
    }
    if (hipEventQuery(s.done) == hipSuccess) {
      for (size_t i = 0; i < s.tickets.size(); ++i) retire_one(s, i, s.h_info[i], now);
      arena.release(s.off, s.bytes);
      s.tickets.clear();
      s.ks.clear();
      s.retired.clear();
      s.busy = false;
      progress = true;
    }
    return progress;
  }

  // Form a batch from the waiting requests and launch it on slot `s` (lock
  // held).  Returns false if nothing was launched.
  bool launch(Slot& s) {
    std::vector<cholmod_desc> descs;
    std::vector<uint64_t> tickets;
    std::vector<int32_t> taken;
    const size_t room = arena.largest();
    size_t need = 0;
    const Clock::time_point now = Clock::now();
    for (auto it = queue.begin(); it != queue.end() && descs.size() < cap;) {
      Request& r = reqs[*it];
      Factor& F = factors[r.factor];
      if (F.busy || std::find(taken.begin(), taken.end(), r.factor) != taken.end()) {
        ++it;
        continue;
      }
      cholmod_desc d;
      d.L = F.L;
      d.V = r.V;
      d.n = F.n;
      d.k = r.k;
      d.ldl = F.ldl;
      d.sigma = r.sigma;
      d.dtype = F.dtype;
      descs.push_back(d);
      const size_t plan = chm::batch_workspace_bytes(descs.data(), (int64_t)descs.size());
      const size_t total = plan ? align_up(plan) + align_up(descs.size() * sizeof(int64_t)) : 0;
      if (total == 0 || total > room) {
        descs.pop_back();
        cholmod_desc alone = d;
        const size_t one = chm::batch_workspace_bytes(&alone, 1);
        if (one == 0 || align_up(one) + kAlign > cfg.ws_bytes) {
          // it can never run: it fails rather than blocking its factor
          it = queue.erase(it);
          finish(r, CHOLMOD_ERR_ARG, now);
          continue;
        }
        ++it;  // waits for memory to free up; smaller requests may go first
        continue;
      }
      need = total;
      taken.push_back(r.factor);
      tickets.push_back(*it);
      it = queue.erase(it);
    }
    if (descs.empty()) return false;
    const int64_t count = (int64_t)descs.size();
    size_t off = 0;
    if (!arena.alloc(need, &off)) {  // cannot happen: need <= largest free range
      for (uint64_t t : tickets) queue.push_front(t);
      return false;
    }
    char* ws = arena_base + off;
    const size_t plan = chm::batch_workspace_bytes(descs.data(), count);
    int64_t* d_info = (int64_t*)(ws + align_up(plan));
    const size_t tb = chm::batch_table_bytes(descs.data(), count);
    int rc = CHOLMOD_OK;
    if (s.stage_bytes < tb) {
      if (s.stage) hipHostFree(s.stage);
      s.stage = nullptr;
      s.stage_bytes = 0;
      if (hipHostMalloc(&s.stage, tb, hipHostMallocDefault) != hipSuccess) rc = CHOLMOD_ERR_HIP;
      else s.stage_bytes = tb;
    }
    for (int64_t i = 0; i < count; ++i) s.h_done[i] = kDoneEmpty;
    if (rc == CHOLMOD_OK) {
      // the tuned launch shape of such a batch, always the queued schedule
      // (its factors report completion one by one)
      cholmod_plan lp = chm::select_plan(descs.data(), count);
      lp.schedule = CHOLMOD_SCHED_QUEUED;
      rc = chm::enqueue_batch(descs.data(), count, ws, plan, d_info, s.stream, s.stage,
                              s.stage_bytes, nullptr, s.d_done, &lp);
    }
    if (rc == CHOLMOD_OK &&
        hipMemcpyAsync(s.h_info, d_info, count * sizeof(int64_t), hipMemcpyDeviceToHost,
                       s.stream) != hipSuccess)
      rc = CHOLMOD_ERR_HIP;
    if (rc == CHOLMOD_OK && hipEventRecord(s.done, s.stream) != hipSuccess) rc = CHOLMOD_ERR_HIP;
    if (rc != CHOLMOD_OK) {
      // nothing may still run on this range if enqueueing failed part way
      hipStreamSynchronize(s.stream);
      arena.release(off, need);
      for (uint64_t t : tickets) finish(reqs[t], rc, now);
      if (rc == CHOLMOD_ERR_HIP) fatal = rc;
      return true;
    }
    s.off = off;
    s.bytes = need;
    s.tickets = std::move(tickets);
    s.ks.clear();
    for (const cholmod_desc& d : descs) s.ks.push_back(d.k);
    s.retired.assign(s.tickets.size(), 0);
    s.left = s.tickets.size();
    for (int32_t f : taken) factors[f].busy = true;
    s.busy = true;
    in_flight += count;
    return true;
  }

  void run() {
    hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (!stop) {
      bool progress = false;
      for (int i = 0; i < nslots; ++i)
        if (slots[i].busy) progress |= poll_slot(slots[i]);
      if (!queue.empty() && !fatal) {
        for (int i = 0; i < nslots && !queue.empty(); ++i)
          if (!slots[i].busy) progress |= launch(slots[i]);
      }
      cv.notify_all();  // drain() and destroy() wait on the counters
      if (!progress) {
        if (in_flight > 0) {
          // batches are running: look again shortly
          lk.unlock();
          std::this_thread::sleep_for(std::chrono::microseconds(20));
          lk.lock();
        } else {
          // wake on a submission; requests waiting for memory or for their
          // factor always have a batch in flight ahead of them
          cv.wait(lk, [&] { return stop.load() || (!queue.empty() && in_flight == 0); });
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
  if (cfg->streams < 0 || cfg->streams > kMaxStreams) return CHOLMOD_ERR_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess) return CHOLMOD_ERR_HIP;
  if (cfg->device < 0 || cfg->device >= ndev) return CHOLMOD_ERR_ARG;
  cholmod_server* s = new cholmod_server();
  s->cfg = *cfg;
  s->cfg.ws_bytes = cfg->ws_bytes / kAlign * kAlign;
  s->device = cfg->device;
  s->cap = cfg->max_batch > 0 ? (size_t)cfg->max_batch : 256;
  s->nslots = cfg->streams > 0 ? cfg->streams : 4;
  int prev = 0;
  hipGetDevice(&prev);
  int rc = hipSetDevice(s->device) == hipSuccess ? s->init() : CHOLMOD_ERR_HIP;
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
  s->queue.push_back(t);
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
  s->cv.wait(lk, [&] { return s->fatal != 0 || (s->queue.empty() && s->in_flight == 0); });
  return s->fatal;
}

int cholmod_server_destroy(cholmod_server* s) {
  if (s == nullptr) return CHOLMOD_ERR_ARG;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.wait(lk, [&] { return s->fatal != 0 || (s->queue.empty() && s->in_flight == 0); });
    s->stop = true;
    s->cv.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  int prev = 0;
  hipGetDevice(&prev);
  hipSetDevice(s->device);
  for (int i = 0; i < s->nslots; ++i)
    if (s->slots[i].stream) hipStreamSynchronize(s->slots[i].stream);
  s->release();
  hipSetDevice(prev);
  delete s;
  return CHOLMOD_OK;
}

}  // extern "C"
