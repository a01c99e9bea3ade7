// serve.hip -- continuous-batching solve server (C ABI in mg_serve.h).
//
// One worker thread drives every batch.  Each pass of its loop:
//   1. takes new submissions into the pending queue;
//   2. completes retirements whose copies have landed (slot freed, completion queued);
//   3. admits pending requests into free slots of their size's batch, creating a batch
//      when the HBM budget allows (releasing idle batches, least recently used first);
//   4. keeps one chunk of replays in flight per busy batch (see inflight_from_env) and, when
//      the oldest chunk's flag copy has landed, retires every slot that finished in it.
// A slot's flags are trusted only from chunks launched after the slot was admitted,
// and a slot is reused only after its retirement copy has been observed, so the host
// never confuses two occupants of one slot.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "batch.h"
#include "mg_serve.h"

namespace {

// Chunks of replays a busy batch keeps in flight: one (MG_SERVE_INFLIGHT=2: two).  A
// request admitted to a batch waits for the chunks already in flight on the batch's
// stream, and batches of a size group share a stream, so one chunk in flight per batch
// keeps that wait short.  Measured at half load (400 requests, sizes 65^2 .. 2049^2,
// chunks of two steps): p50 / p99 13.4 / 18.1 ms with two in flight, 8.0 / 12.3 ms with
// one, and the saturated rate rose from 2516 to 2849 requests/s.
// Read once per server, when it is created.
int inflight_from_env() {
  const char *e = getenv("MG_SERVE_INFLIGHT");
  return e != nullptr && atoi(e) == 2 ? 2 : 1;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Req {
  long long tag = 0;
  int n = 0;
  const double *f = nullptr;
  double *u = nullptr;
  double t_submit = 0.0, t_admit = 0.0;
};

enum SlotState { kFree = 0, kRunning = 1, kRetiring = 2 };

struct Batch {
  int n = 0, slots = 0;
  mg_ctx *ctx = nullptr;
  hipStream_t stream = nullptr;
  bool own_stream = true;             // false: a group stream of the server
  size_t bytes = 0;
  std::vector<int> state;             // SlotState per slot
  std::vector<Req> req;               // occupant per slot
  std::vector<long long> admitted_at; // chunks launched before the admission
  std::vector<hipEvent_t> retire_ev;
  mgb::SlotFlags *flags[2] = {nullptr, nullptr};  // pinned, one buffer per chunk in flight (up to two)
  mgk::DevState *states = nullptr;                // pinned, retirement copies
  hipEvent_t chunk_ev[2] = {nullptr, nullptr};
  long long chunk_seq[2] = {0, 0};
  int inflight = 0, oldest = 0;
  long long launched = 0;
  double last_used = 0.0;

  int busy() const {
    int b = 0;
    for (int s : state) b += s != kFree;
    return b;
  }
  int running() const {
    int b = 0;
    for (int s : state) b += s == kRunning;
    return b;
  }
  int free_slot() const {
    for (int k = 0; k < slots; ++k)
      if (state[k] == kFree) return k;
    return -1;
  }
};

}  // namespace

struct mg_server_s {
  mg_server_config cfg{};
  int device = 0;
  int max_inflight = 1;  // chunks in flight per busy batch, 1 or 2
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req> incoming;
  std::deque<mg_completion> done;
  bool stop = false;
  bool failed = false;
  std::string error;
  mg_server_stats stats{};
  std::thread worker;
  // worker-owned
  std::deque<Req> pending;
  std::map<int, std::unique_ptr<Batch>> batches;
  hipStream_t group_stream[3] = {nullptr, nullptr, nullptr};  // stream_groups > 0
};

namespace {

mg_config config_for(const mg_config &base, int n) {
  mg_config c = base;
  c.n = n;
  return c;
}

void free_batch(Batch *b) {
  if (b->ctx) mgb::destroy(b->ctx);  // waits for the batch stream
  for (auto &e : b->retire_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto &e : b->chunk_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto &p : b->flags)
    if (p) (void)hipHostFree(p);
  if (b->states) (void)hipHostFree(b->states);
  if (b->stream && b->own_stream) (void)hipStreamDestroy(b->stream);
  b->ctx = nullptr;
}

class Worker {
 public:
  explicit Worker(mg_server_s *s) : s_(s) {}
  void run();

 private:
  mg_server_s *s_;
  bool fail(const std::string &msg) {
    std::lock_guard<std::mutex> g(s_->mu);
    s_->failed = true;
    s_->error = msg;
    s_->cv_done.notify_all();
    return false;
  }
  bool hip_ok(hipError_t e, const char *what) {
    if (e == hipSuccess) return true;
    return fail(std::string(what) + ": " + hipGetErrorString(e));
  }
  bool mg_ok(mg_status st, const char *what) {
    if (st == MG_OK) return true;
    return fail(std::string(what) + ": " + mg_last_error());
  }
  size_t held() const {
    size_t b = 0;
    for (auto &kv : s_->batches) b += kv.second->bytes;
    return b;
  }
  bool release_idle(size_t need);
  Batch *create_batch(int n, bool *ok);
  bool admit_pending(bool *progress);
  bool complete_retirements(bool *progress);
  bool drive(Batch *b, bool *progress);
};

bool Worker::release_idle(size_t need) {
  const size_t budget = s_->cfg.hbm_budget;
  while (held() + need > budget) {
    Batch *victim = nullptr;
    int key = 0;
    for (auto &kv : s_->batches) {
      Batch *b = kv.second.get();
      if (b->busy() == 0 && b->inflight == 0 && (!victim || b->last_used < victim->last_used)) {
        victim = b;
        key = kv.first;
      }
    }
    if (!victim) return false;
    free_batch(victim);
    s_->batches.erase(key);
    std::lock_guard<std::mutex> g(s_->mu);
    s_->stats.batches_released++;
    s_->stats.batches = (int)s_->batches.size();
    s_->stats.bytes_held = held();
  }
  return true;
}

Batch *Worker::create_batch(int n, bool *ok) {
  *ok = true;
  const mg_config cfg = config_for(s_->cfg.base, n);
  const size_t one = mgb::footprint(&cfg, 1), two = mgb::footprint(&cfg, 2);
  const size_t per_slot = two - one, fixed = one - per_slot;
  if (!release_idle(one)) return nullptr;
  const size_t avail = s_->cfg.hbm_budget - held();
  const int slots = (int)std::min<size_t>((size_t)s_->cfg.max_slots, (avail - fixed) / per_slot);
  if (slots < 1) return nullptr;
  auto b = std::make_unique<Batch>();
  b->n = n;
  b->slots = slots;
  b->bytes = mgb::footprint(&cfg, slots);
  const int groups = s_->cfg.stream_groups;
  if (groups > 0) {  // a stream shared by the sizes of one group, created on first use
    const int g = groups == 1 ? 0 : (groups == 2 ? (n <= 1025 ? 0 : 1) : (n <= 257 ? 0 : (n <= 1025 ? 1 : 2)));
    if (!s_->group_stream[g] &&
        !hip_ok(hipStreamCreateWithFlags(&s_->group_stream[g], hipStreamNonBlocking), "hipStreamCreate")) {
      *ok = false;
      return nullptr;
    }
    b->stream = s_->group_stream[g];
    b->own_stream = false;
  } else if (!hip_ok(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking), "hipStreamCreate")) {
    *ok = false;
    return nullptr;
  }
  mg_status st = mgb::create(&cfg, slots, b->stream, &b->ctx);
  if (st != MG_OK) {
    free_batch(b.get());
    if (st == MG_ENOMEM) return nullptr;  // the device is fuller than the budget: wait
    *ok = mg_ok(st, "batch setup");
    return nullptr;
  }
  b->state.assign(slots, kFree);
  b->req.assign(slots, Req{});
  b->admitted_at.assign(slots, 0);
  b->retire_ev.assign(slots, nullptr);
  bool good = true;
  for (auto &e : b->retire_ev)
    good = good && hip_ok(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
  for (auto &e : b->chunk_ev)
    good = good && hip_ok(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
  for (auto &p : b->flags)
    good = good && hip_ok(hipHostMalloc((void **)&p, sizeof(mgb::SlotFlags) * slots, hipHostMallocDefault),
                          "hipHostMalloc");
  good = good && hip_ok(hipHostMalloc((void **)&b->states, sizeof(mgk::DevState) * slots, hipHostMallocDefault),
                        "hipHostMalloc");
  if (!good) {
    free_batch(b.get());
    *ok = false;
    return nullptr;
  }
  b->last_used = now_s();
  Batch *raw = b.get();
  s_->batches[n] = std::move(b);
  std::lock_guard<std::mutex> g(s_->mu);
  s_->stats.batches_created++;
  s_->stats.batches = (int)s_->batches.size();
  s_->stats.bytes_held = held();
  s_->stats.peak_bytes_held = std::max(s_->stats.peak_bytes_held, s_->stats.bytes_held);
  return raw;
}

bool Worker::admit_pending(bool *progress) {
  bool may_create = true;  // once the oldest waiting request is blocked on memory, later
                           // requests only use batches that exist
  for (auto it = s_->pending.begin(); it != s_->pending.end();) {
    Batch *b = nullptr;
    auto bi = s_->batches.find(it->n);
    if (bi != s_->batches.end()) b = bi->second.get();
    if (!b && may_create) {
      bool ok = true;
      b = create_batch(it->n, &ok);
      if (!ok) return false;
      if (!b) may_create = false;
    }
    const int k = b ? b->free_slot() : -1;
    if (k < 0) {
      ++it;
      continue;
    }
    if (!mg_ok(mgb::admit(b->ctx, k, it->f), "admission")) return false;
    b->state[k] = kRunning;
    b->req[k] = *it;
    b->req[k].t_admit = now_s();
    b->admitted_at[k] = b->launched;
    b->last_used = b->req[k].t_admit;
    it = s_->pending.erase(it);
    *progress = true;
    std::lock_guard<std::mutex> g(s_->mu);
    s_->stats.queued--;
    s_->stats.active++;
    s_->stats.peak_active = std::max(s_->stats.peak_active, s_->stats.active);
  }
  return true;
}

bool Worker::complete_retirements(bool *progress) {
  for (auto &kv : s_->batches) {
    Batch *b = kv.second.get();
    for (int k = 0; k < b->slots; ++k) {
      if (b->state[k] != kRetiring) continue;
      const hipError_t e = hipEventQuery(b->retire_ev[k]);
      if (e == hipErrorNotReady) continue;
      if (!hip_ok(e, "retirement copy")) return false;
      mg_completion c;
      std::memset(&c, 0, sizeof(c));
      c.tag = b->req[k].tag;
      c.n = b->n;
      c.t_submit = b->req[k].t_submit;
      c.t_admit = b->req[k].t_admit;
      c.t_done = now_s();
      mg_status outcome = MG_OK;
      mgb::result(b->ctx, b->states[k], &c.result, &outcome);
      c.status = outcome;
      b->state[k] = kFree;
      b->last_used = c.t_done;
      *progress = true;
      std::lock_guard<std::mutex> g(s_->mu);
      s_->done.push_back(c);
      s_->stats.completed++;
      s_->stats.active--;
      s_->cv_done.notify_all();
    }
  }
  return true;
}

bool Worker::drive(Batch *b, bool *progress) {
  // launch while fewer than max_inflight chunks are in flight and some slot is running
  while (b->inflight < s_->max_inflight && b->running() > 0) {
    const int buf = (b->oldest + b->inflight) & 1;
    if (!mg_ok(mgb::step(b->ctx, s_->cfg.chunk_steps), "replay")) return false;
    if (!mg_ok(mgb::read_flags(b->ctx, b->flags[buf]), "flag copy")) return false;
    if (!hip_ok(hipEventRecord(b->chunk_ev[buf], b->stream), "hipEventRecord")) return false;
    b->chunk_seq[buf] = ++b->launched;
    b->inflight++;
    *progress = true;
    std::lock_guard<std::mutex> g(s_->mu);
    s_->stats.replays += s_->cfg.chunk_steps;
  }
  if (b->inflight == 0) return true;
  const int buf = b->oldest;
  const hipError_t e = hipEventQuery(b->chunk_ev[buf]);
  if (e == hipErrorNotReady) return true;
  if (!hip_ok(e, "chunk")) return false;
  const mgb::SlotFlags *fl = b->flags[buf];
  for (int k = 0; k < b->slots; ++k) {
    if (b->state[k] != kRunning || b->admitted_at[k] >= b->chunk_seq[buf] || !fl[k].done) continue;
    if (!mg_ok(mgb::retire(b->ctx, k, b->req[k].u, &b->states[k]), "retirement")) return false;
    if (!hip_ok(hipEventRecord(b->retire_ev[k], b->stream), "hipEventRecord")) return false;
    b->state[k] = kRetiring;
  }
  b->oldest ^= 1;
  b->inflight--;
  *progress = true;
  return true;
}

void Worker::run() {
  if (!hip_ok(hipSetDevice(s_->device), "hipSetDevice")) return;
  int idle_spins = 0;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(s_->mu);
      if (s_->stop) break;
      const bool busy = !s_->pending.empty() ||
                        std::any_of(s_->batches.begin(), s_->batches.end(), [](auto &kv) {
                          return kv.second->busy() > 0 || kv.second->inflight > 0;
                        });
      if (!busy && s_->incoming.empty()) {
        s_->cv_work.wait(lk, [&] { return s_->stop || !s_->incoming.empty(); });
        if (s_->stop) break;
      }
      while (!s_->incoming.empty()) {
        s_->pending.push_back(s_->incoming.front());
        s_->incoming.pop_front();
      }
    }
    bool progress = false;
    if (!complete_retirements(&progress)) return;
    if (!admit_pending(&progress)) return;
    for (auto &kv : s_->batches)
      if (!drive(kv.second.get(), &progress)) return;
    if (progress) {
      idle_spins = 0;
    } else if (++idle_spins > 64) {
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    } else {
      std::this_thread::yield();
    }
  }
}

}  // namespace

extern "C" {

double mg_server_clock(void) { return now_s(); }

size_t mg_serve_batch_bytes(const mg_config *base, int n, int slots) {
  if (!base || slots < 1 || base->dim != 2) return 0;
  const mg_config c = config_for(*base, n);
  return mgb::footprint(&c, slots);
}

mg_status mg_server_create(const mg_server_config *cfg, mg_server *out) {
  if (!out) return MG_EINVAL;
  *out = nullptr;
  if (!cfg || cfg->base.dim != 2 || cfg->max_slots < 1 || cfg->max_slots > 1024 ||
      cfg->chunk_steps < 1 || cfg->chunk_steps > 64 || cfg->hbm_budget == 0 || cfg->stream_groups < 0 ||
      cfg->stream_groups > 3)
    return MG_EINVAL;
  // the base configuration must be valid at its own size
  if (mgb::footprint(&cfg->base, 1) == 0) return MG_EINVAL;
  auto s = std::make_unique<mg_server_s>();
  s->cfg = *cfg;
  s->max_inflight = inflight_from_env();
  if (hipGetDevice(&s->device) != hipSuccess) return MG_EDEVICE;
  mg_server_s *raw = s.release();
  raw->worker = std::thread([raw] { Worker(raw).run(); });
  *out = raw;
  return MG_OK;
}

mg_status mg_server_submit(mg_server s, long long tag, int n, const double *f, double *u) {
  if (!s || !f || !u) return MG_EINVAL;
  const mg_config c = config_for(s->cfg.base, n);
  const size_t one = mgb::footprint(&c, 1);
  if (one == 0) return MG_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  if (s->failed) {
    mgb::set_error(s->error);
    return MG_EDEVICE;
  }
  if (one > s->cfg.hbm_budget) {
    s->stats.rejected++;
    return MG_ENOMEM;
  }
  Req r;
  r.tag = tag;
  r.n = n;
  r.f = f;
  r.u = u;
  r.t_submit = now_s();
  s->incoming.push_back(r);
  s->stats.submitted++;
  s->stats.queued++;
  s->cv_work.notify_one();
  return MG_OK;
}

int mg_server_poll(mg_server s, mg_completion *out, int max, double timeout_s) {
  if (!s || (max > 0 && !out) || max < 0) return -1;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && timeout_s > 0.0 && !s->failed)
    s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s),
                        [&] { return !s->done.empty() || s->failed; });
  int k = 0;
  while (k < max && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  if (k == 0 && s->failed) {
    mgb::set_error(s->error);
    return -MG_EDEVICE;
  }
  return k;
}

mg_status mg_server_stats_get(mg_server s, mg_server_stats *out) {
  if (!s || !out) return MG_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  *out = s->stats;
  return MG_OK;
}

mg_status mg_server_destroy(mg_server s) {
  if (!s) return MG_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->device);
  for (auto &kv : s->batches) free_batch(kv.second.get());
  s->batches.clear();
  for (auto &st : s->group_stream)
    if (st) (void)hipStreamDestroy(st);
  delete s;
  return MG_OK;
}

}  // extern "C"
