// Serving runtime: a request loop that runs fast-multiply requests of
// different sizes as they arrive.  Requests wait in a FIFO queue; the
// admission controller admits the head request when a slot (a HIP stream) is
// free and the HBM it needs - operands, output and temporaries - fits as one
// block in the server's device arena (first fit).  An admitted request
// generates its operands in its block on the device from its seed, runs
// mf_fastmm_ws with the plan chosen by a pure function of (n, dtype), all on
// its slot's stream; requests on different slots overlap on the device, and a
// block is released when its request's completion is observed.  A worker
// thread admits and polls completions; an optional replay thread submits
// requests at given arrival times.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <thread>

#include "mf_internal.h"

namespace mf {

hipError_t launch_fill_uniform(void* p, int64_t count, int elem, uint64_t seed, hipStream_t s);

// Host-side bookkeeping of a device arena [0, size): first-fit allocation of
// 256-byte aligned blocks, coalescing on release.
class Arena {
 public:
  explicit Arena(size_t size) : size_(size) {
    if (size_ > 0) free_[0] = size_;
  }
  bool alloc(size_t need, size_t* off) {
    need = (need + 255) / 256 * 256;
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= need) {
        *off = it->first;
        const size_t rest = it->second - need, at = it->first + need;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += need;
        return true;
      }
    return false;
  }
  void release(size_t off, size_t need) {
    need = (need + 255) / 256 * 256;
    used_ -= need;
    auto it = free_.emplace(off, need).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  size_t size_;
  size_t used_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length
};

// FIFO admission by free slots and HBM (host only).  A request is admitted
// when a slot is free and its memory fits, as one block, in the arena of
// budget bytes; the same policy drives the server and the simulation.
class Admission {
 public:
  Admission(int slots, size_t budget, bool overtake) : slots_(slots), arena_(budget), overtake_(overtake) {}
  void arrive(int64_t id, size_t need) { queue_.push_back({id, need, 0}); }
  // Admits what fits now, in arrival order; returns (id, arena offset) pairs.
  std::vector<std::pair<int64_t, size_t>> admit() {
    std::vector<std::pair<int64_t, size_t>> out;
    for (auto it = queue_.begin(); it != queue_.end();) {
      if (busy_ >= slots_) break;
      size_t off = 0;
      if (arena_.alloc(it->need, &off)) {
        ++busy_;
        it->off = off;
        held_.push_back(*it);
        out.push_back({it->id, off});
        it = queue_.erase(it);
      } else if (overtake_) {
        ++it;
      } else {
        break;
      }
    }
    return out;
  }
  void release(int64_t id) {
    for (auto it = held_.begin(); it != held_.end(); ++it)
      if (it->id == id) {
        arena_.release(it->off, it->need);
        --busy_;
        held_.erase(it);
        return;
      }
  }
  size_t used() const { return arena_.used(); }
  int busy() const { return busy_; }
  size_t waiting() const { return queue_.size(); }

 private:
  struct Item {
    int64_t id;
    size_t need;
    size_t off;
  };
  int slots_;
  Arena arena_;
  bool overtake_;
  int busy_ = 0;
  std::deque<Item> queue_;
  std::vector<Item> held_;
};

}  // namespace mf

using namespace mf;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Req {
  int64_t id;
  int64_t n;
  int dtype;
  uint64_t seed;
  void* host_out;  // pinned host buffer for C, or NULL
  // caller-owned device operands (NULL: A and B generated from the seed in
  // the request's arena block, C there too)
  const void* A_user = nullptr;
  const void* B_user = nullptr;
  void* C_user = nullptr;
  size_t need = 0;
  int depth = 0;
  double t_arrive = 0, t_admit = 0, t_done = 0;
  int slot = -1;
  size_t off = 0;  // of its memory in the arena
  mf_status status = MF_OK;
  bool done = false;
  double device_ms = -1;  // from the request's first launch to its completion, on its stream
  // the same interval on the device timeline: ms since the server's origin
  // event (recorded when the server started)
  double device_start = -1, device_end = -1;
};

size_t round256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

struct mf_server {
  mf_server_config cfg;
  const mf_algo* algo = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;        // completion, per slot
  std::vector<hipEvent_t> start_events;  // start of the request's device work, per slot
  hipEvent_t origin = nullptr;           // device time 0 of the per-request intervals
  char* arena = nullptr;                 // hbm_budget bytes of device memory for admitted requests
  std::vector<int64_t> slot_req;  // request id per slot, -1 if free
  std::mutex mu;
  std::condition_variable cv;
  std::vector<Req> reqs;  // by id
  Admission adm;
  std::thread worker;
  std::thread replayer;
  std::atomic<bool> stop{false};
  int device = 0;
  double t0 = 0;
  int64_t completed = 0;
  explicit mf_server(const mf_server_config& c)
      : cfg(c), adm(c.max_slots, c.hbm_budget, c.allow_overtake != 0) {}
};

namespace {

// Depth policy: a pure function of (n, dtype), so a request's result is the
// same alone and among others.
int depth_for(const mf_server* s, int64_t n, int dtype) {
  if (!s->algo) return 0;
  const bool f64 = (dtype & 0xff) == MF_F64;
  const int64_t* th = f64 ? s->cfg.depth_min_n_f64 : s->cfg.depth_min_n_f32;
  int d = 0;
  for (int k = 0; k < 4; ++k)
    if (th[k] > 0 && n >= th[k]) d = k + 1;
  return d;
}

// HBM a request is admitted against: A, B and C (unless the caller owns them)
// and the workspace of its plan.
mf_status need_bytes(const mf_server* s, int64_t n, int dtype, int depth, bool own_operands, size_t* bytes) {
  size_t ws = 0;
  if (depth > 0) {
    mf_status st = mf_workspace_bytes(s->algo, depth, 0, n, dtype, &ws);
    if (st != MF_OK) return st;
  }
  const size_t elem = (dtype & 0xff) == MF_F64 ? 8 : 4;
  *bytes = (own_operands ? 3 * round256((size_t)n * (size_t)n * elem) : 0) + round256(ws);
  return MF_OK;
}

// Enqueues the whole request on its slot's stream.
mf_status launch_request(mf_server* s, Req& r) {
  hipStream_t st = s->streams[r.slot];
  const size_t elem = (r.dtype & 0xff) == MF_F64 ? 8 : 4;
  const bool own = r.A_user == nullptr;
  const size_t mat = own ? round256((size_t)r.n * (size_t)r.n * elem) : 0;
  if (hipEventRecord(s->start_events[r.slot], st) != hipSuccess) return fail(MF_ERR_HIP, "start event failed");
  char* mem = s->arena + r.off;  // reserved by admission until the completion is observed
  const void* A = own ? static_cast<const void*>(mem) : r.A_user;
  const void* B = own ? static_cast<const void*>(mem + mat) : r.B_user;
  void* C = own ? static_cast<void*>(mem + 2 * mat) : r.C_user;
  void* ws = mem + 3 * mat;
  const int64_t cnt = r.n * r.n;
  mf_status res = MF_OK;
  if (own && (launch_fill_uniform(const_cast<void*>(A), cnt, (int)elem, r.seed * 2 + 0, st) != hipSuccess ||
              launch_fill_uniform(const_cast<void*>(B), cnt, (int)elem, r.seed * 2 + 1, st) != hipSuccess))
    res = fail(MF_ERR_HIP, "operand generation launch failed");
  if (res == MF_OK) {
    if (r.depth > 0)
      res = mf_fastmm_ws(s->algo, r.depth, 0, A, B, C, r.n, r.dtype, ws, r.need - 3 * mat, st);
    else
      res = mf_classical_mm(A, B, C, r.n, r.dtype, st);
  }
  if (res == MF_OK && r.host_out &&
      hipMemcpyAsync(r.host_out, C, (size_t)cnt * elem, hipMemcpyDeviceToHost, st) != hipSuccess)
    res = fail(MF_ERR_HIP, "result copy failed");
  if (hipEventRecord(s->events[r.slot], st) != hipSuccess && res == MF_OK)
    res = fail(MF_ERR_HIP, "completion event failed");
  return res;
}

void worker_loop(mf_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    // completions
    bool any_busy = false;
    for (size_t k = 0; k < s->slot_req.size(); ++k) {
      const int64_t id = s->slot_req[k];
      if (id < 0) continue;
      any_busy = true;
      const hipError_t q = hipEventQuery(s->events[k]);
      if (q == hipErrorNotReady) continue;
      Req& r = s->reqs[id];
      r.t_done = now_s() - s->t0;
      if (q != hipSuccess && r.status == MF_OK) r.status = MF_ERR_HIP;
      float ms = 0.f, t_start = 0.f, t_end = 0.f;
      if (q == hipSuccess && hipEventElapsedTime(&ms, s->start_events[k], s->events[k]) == hipSuccess)
        r.device_ms = ms;
      if (q == hipSuccess && hipEventElapsedTime(&t_start, s->origin, s->start_events[k]) == hipSuccess &&
          hipEventElapsedTime(&t_end, s->origin, s->events[k]) == hipSuccess) {
        r.device_start = t_start;
        r.device_end = t_end;
      }
      r.done = true;
      s->adm.release(id);
      s->slot_req[k] = -1;
      ++s->completed;
      s->cv.notify_all();
    }
    // admissions
    for (const auto& adm : s->adm.admit()) {
      const int64_t id = adm.first;
      Req& r = s->reqs[id];
      r.off = adm.second;
      int slot = -1;
      for (size_t k = 0; k < s->slot_req.size(); ++k)
        if (s->slot_req[k] < 0) {
          slot = (int)k;
          break;
        }
      r.slot = slot;
      r.t_admit = now_s() - s->t0;
      s->slot_req[slot] = id;
      r.status = launch_request(s, r);
      any_busy = true;
    }
    if (s->stop && !any_busy && s->adm.waiting() == 0) break;
    if (any_busy) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    } else {
      s->cv.wait_for(lk, std::chrono::milliseconds(1));
    }
  }
}

}  // namespace

extern "C" {

mf_status mf_server_create(const mf_server_config* cfg, const mf_algo* algo, mf_server** out) {
  clear_error();
  if (!cfg || !out) return fail(MF_ERR_ARG, "NULL argument");
  *out = nullptr;
  if (cfg->max_slots < 1 || cfg->max_slots > 64) return fail(MF_ERR_ARG, "max_slots must be in [1, 64]");
  if (cfg->hbm_budget == 0) return fail(MF_ERR_ARG, "hbm_budget must be > 0");
  mf_server* s = new (std::nothrow) mf_server(*cfg);
  if (!s) return fail(MF_ERR_NOMEM, "host allocation failed");
  s->algo = algo;
  (void)hipGetDevice(&s->device);
  // One device arena of hbm_budget bytes holds every admitted request's
  // memory; admission places a request in it (first fit), so requests never
  // allocate or map device memory while the server runs.
  if (hipMalloc(reinterpret_cast<void**>(&s->arena), cfg->hbm_budget) != hipSuccess) {
    (void)hipGetLastError();
    s->arena = nullptr;
    mf_server_free(s);
    return fail(MF_ERR_NOMEM, "the HBM budget cannot be allocated on the device");
  }
  for (int k = 0; k < cfg->max_slots; ++k) {
    hipStream_t st;
    hipEvent_t ev, ev0;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&ev) != hipSuccess || hipEventCreate(&ev0) != hipSuccess) {
      (void)hipGetLastError();
      mf_server_free(s);
      return fail(MF_ERR_HIP, "stream creation failed");
    }
    s->streams.push_back(st);
    s->events.push_back(ev);
    s->start_events.push_back(ev0);
    s->slot_req.push_back(-1);
  }
  if (hipEventCreate(&s->origin) != hipSuccess || hipEventRecord(s->origin, s->streams[0]) != hipSuccess ||
      hipEventSynchronize(s->origin) != hipSuccess) {
    (void)hipGetLastError();
    mf_server_free(s);
    return fail(MF_ERR_HIP, "origin event failed");
  }
  s->t0 = now_s();
  s->worker = std::thread(worker_loop, s);
  *out = s;
  return MF_OK;
}

mf_status mf_server_need_bytes(const mf_server* s, int64_t n, int dtype, size_t* bytes) {
  clear_error();
  if (!s || !bytes || n < 1) return fail(MF_ERR_ARG, "invalid argument");
  if ((dtype & 0xff) != MF_F64 && (dtype & 0xff) != MF_F32) return fail(MF_ERR_ARG, "unknown dtype");
  return need_bytes(s, n, dtype, depth_for(s, n, dtype), true, bytes);
}

}  // extern "C"

namespace {

mf_status enqueue(mf_server* s, Req r, int64_t* id) {
  r.depth = depth_for(s, r.n, r.dtype);
  mf_status st = need_bytes(s, r.n, r.dtype, r.depth, r.A_user == nullptr, &r.need);
  if (st != MF_OK) return st;
  if (r.need > s->cfg.hbm_budget) return fail(MF_ERR_NOMEM, "request needs more HBM than the whole budget");
  std::lock_guard<std::mutex> lk(s->mu);
  r.id = (int64_t)s->reqs.size();
  r.t_arrive = now_s() - s->t0;
  s->reqs.push_back(r);
  s->adm.arrive(r.id, r.need);
  s->cv.notify_all();
  if (id) *id = r.id;
  return MF_OK;
}

bool serving_dtype(int dtype) {
  return (dtype & ~0xff) == 0 && ((dtype & 0xff) == MF_F64 || (dtype & 0xff) == MF_F32);
}

}  // namespace

extern "C" {

mf_status mf_server_submit(mf_server* s, int64_t n, int dtype, uint64_t seed, void* host_out, int64_t* id) {
  clear_error();
  if (!s || n < 1 || n > (1 << 16)) return fail(MF_ERR_ARG, "invalid argument");
  if (!serving_dtype(dtype)) return fail(MF_ERR_ARG, "serving takes MF_F64 or MF_F32 (native leaves)");
  Req r{};
  r.n = n;
  r.dtype = dtype;
  r.seed = seed;
  r.host_out = host_out;
  return enqueue(s, r, id);
}

mf_status mf_server_submit_operands(mf_server* s, int64_t n, int dtype, const void* A, const void* B, void* C,
                                    int64_t* id) {
  clear_error();
  if (!s || n < 1 || n > (1 << 16)) return fail(MF_ERR_ARG, "invalid argument");
  if (!serving_dtype(dtype)) return fail(MF_ERR_ARG, "serving takes MF_F64 or MF_F32 (native leaves)");
  if (!A || !B || !C) return fail(MF_ERR_ARG, "A, B and C must be non-NULL");
  const size_t elem = (dtype & 0xff) == MF_F64 ? 8 : 4;
  if ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B) | reinterpret_cast<uintptr_t>(C)) &
      (elem - 1))
    return fail(MF_ERR_ARG, "A, B and C must be aligned to the element size");
  const size_t bytes = (size_t)n * (size_t)n * elem;
  if (overlaps(C, bytes, A, bytes) || overlaps(C, bytes, B, bytes)) return fail(MF_ERR_ARG, "C overlaps A or B");
  Req r{};
  r.n = n;
  r.dtype = dtype;
  r.host_out = nullptr;
  r.A_user = A;
  r.B_user = B;
  r.C_user = C;
  return enqueue(s, r, id);
}

mf_status mf_server_replay(mf_server* s, int count, const double* t_arrive, const int64_t* n, const int* dtype,
                           const uint64_t* seed) {
  clear_error();
  if (!s || count < 0 || (count > 0 && (!t_arrive || !n || !dtype || !seed))) return fail(MF_ERR_ARG, "invalid argument");
  if (s->replayer.joinable()) s->replayer.join();
  std::vector<double> t(t_arrive, t_arrive + count);
  std::vector<int64_t> nn(n, n + count);
  std::vector<int> dt(dtype, dtype + count);
  std::vector<uint64_t> sd(seed, seed + count);
  s->replayer = std::thread([s, t, nn, dt, sd]() {
    (void)hipSetDevice(s->device);
    const double base = now_s();
    for (size_t k = 0; k < t.size(); ++k) {
      const double wait = base + t[k] - now_s();
      if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
      (void)mf_server_submit(s, nn[k], dt[k], sd[k], nullptr, nullptr);
    }
  });
  return MF_OK;
}

mf_status mf_server_drain(mf_server* s) {
  clear_error();
  if (!s) return fail(MF_ERR_ARG, "server is NULL");
  if (s->replayer.joinable()) s->replayer.join();
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv.wait(lk, [&]() { return s->completed == (int64_t)s->reqs.size(); });
  for (const Req& r : s->reqs)
    if (r.status != MF_OK) return fail(r.status, "a request failed");
  return MF_OK;
}

mf_status mf_server_stats(mf_server* s, int64_t* count, double* t_arrive, double* t_admit, double* t_done,
                          int64_t* n, int* depth) {
  clear_error();
  if (!s) return fail(MF_ERR_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  if (count) *count = (int64_t)s->reqs.size();
  for (size_t k = 0; k < s->reqs.size(); ++k) {
    const Req& r = s->reqs[k];
    if (t_arrive) t_arrive[k] = r.t_arrive;
    if (t_admit) t_admit[k] = r.t_admit;
    if (t_done) t_done[k] = r.done ? r.t_done : -1.0;
    if (n) n[k] = r.n;
    if (depth) depth[k] = r.depth;
  }
  return MF_OK;
}

void mf_server_free(mf_server* s) {
  if (!s) return;
  if (s->replayer.joinable()) s->replayer.join();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  for (auto& st : s->streams) (void)hipStreamSynchronize(st);
  for (auto& e : s->events) (void)hipEventDestroy(e);
  for (auto& e : s->start_events) (void)hipEventDestroy(e);
  if (s->origin) (void)hipEventDestroy(s->origin);
  for (auto& st : s->streams) (void)hipStreamDestroy(st);
  if (s->arena) (void)hipFree(s->arena);
  delete s;
}

mf_status mf_server_device_ms(mf_server* s, double* ms) {
  clear_error();
  if (!s || !ms) return fail(MF_ERR_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  for (size_t k = 0; k < s->reqs.size(); ++k) ms[k] = s->reqs[k].device_ms;
  return MF_OK;
}

mf_status mf_server_device_interval(mf_server* s, double* start_ms, double* end_ms) {
  clear_error();
  if (!s || !start_ms || !end_ms) return fail(MF_ERR_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  for (size_t k = 0; k < s->reqs.size(); ++k) {
    start_ms[k] = s->reqs[k].device_start;
    end_ms[k] = s->reqs[k].device_end;
  }
  return MF_OK;
}

mf_status mf_fill_uniform(void* p, int64_t count, int dtype, uint64_t seed, mf_stream stream) {
  clear_error();
  if (count < 0 || (count > 0 && !p)) return fail(MF_ERR_ARG, "invalid argument");
  if (dtype != MF_F64 && dtype != MF_F32) return fail(MF_ERR_ARG, "dtype must be MF_F64 or MF_F32");
  const int elem = dtype == MF_F64 ? 8 : 4;
  if (reinterpret_cast<uintptr_t>(p) & (elem - 1)) return fail(MF_ERR_ARG, "misaligned pointer");
  if (launch_fill_uniform(p, count, elem, seed, static_cast<hipStream_t>(stream)) != hipSuccess)
    return fail(MF_ERR_HIP, "fill launch failed");
  return MF_OK;
}

mf_status mf_admission_simulate(int count, const double* t_arrive, const double* service, const size_t* need,
                                int slots, size_t budget, int allow_overtake, double* t_admit, double* t_done,
                                size_t* peak_used) {
  clear_error();
  if (count < 0 || slots < 1 || (count > 0 && (!t_arrive || !service || !need || !t_admit || !t_done)))
    return fail(MF_ERR_ARG, "invalid argument");
  for (int k = 0; k < count; ++k)
    if (need[k] > budget) return fail(MF_ERR_NOMEM, "a request needs more than the whole budget");
  Admission adm(slots, budget, allow_overtake != 0);
  std::vector<std::pair<double, int>> running;  // (finish time, id)
  int next = 0, finished = 0;
  double now = 0;
  size_t peak = 0;
  while (finished < count) {
    // next event: an arrival or a completion
    double t_arr = next < count ? t_arrive[next] : 1e300;
    double t_fin = 1e300;
    for (auto& rf : running) t_fin = std::min(t_fin, rf.first);
    if (t_arr <= t_fin) {
      now = t_arr;
      adm.arrive(next, need[next]);
      ++next;
    } else {
      now = t_fin;
      for (auto it = running.begin(); it != running.end();) {
        if (it->first <= now) {
          t_done[it->second] = it->first;
          adm.release(it->second);
          ++finished;
          it = running.erase(it);
        } else {
          ++it;
        }
      }
    }
    for (const auto& a : adm.admit()) {
      t_admit[a.first] = now;
      running.push_back({now + service[a.first], (int)a.first});
    }
    peak = std::max(peak, adm.used());
  }
  if (peak_used) *peak_used = peak;
  return MF_OK;
}

}  // extern "C"
