// Serving runtime: continuous batching of k-NN requests over resident clouds, with deletions
// applied between batches (Sec. 4.3) and per-request latency stamps.
//
// Clients submit requests (cloud, device queries, k, m, device outputs, optional pinned host
// outputs) and deletion batches; every operation gets a ticket.  A scheduler thread keeps a
// FIFO of pending operations and a few stream slots.  Whenever a slot is free it forms a wave
// from the pending requests, in arrival order, as long as the wave's queries fit the slot's
// share of the device pool -- admission by memory footprint -- and launches it as one
// batched launch (mknn_batch_plan_run, a replayed hipGraph).  Requests that arrive while
// waves run wait only until the next slot frees, and waves on different slots overlap on
// the GPU.  A wave's completion event follows the copies of its results to host memory, and
// the time the scheduler observes it is the request's completion time.
//
// Deletions on one cloud run one at a time, in arrival order.  A worker thread edits the
// host lists (Alg. 3) while waves keep running.  The device delta (copy-on-write list
// segments and a descriptor switch) is then enqueued on a deletion stream after the events
// of the in-flight waves that read that cloud, and later waves on that cloud wait for the
// delta's event.  Waves launched before the switch answer on the old lists, later ones on
// the new lists.  Two orders are offered.  By default a request sees exactly the deletions
// submitted before it: a deletion starts only once no earlier request on its cloud is still
// waiting, and later requests on that cloud wait until it is applied.  With
// MKNN_SERVER_BIND_AT_ADMISSION a request binds to the lists current when its wave is
// launched, so requests never wait for the host part of a deletion.
//
// Insertion batches (points appended as new ranks) are update batches of the same kind:
// they share the per-cloud order, the worker threads, the delta path and the counts of
// update batches a request saw.  Below, "deletion" stands for either kind.
//
// In plain mode (the baseline) every request is its own mknn_knn launch.  All of them go,
// in FIFO order and back to back, onto one stream; up to kPlainSlots are in flight, each
// with its own completion event, and the requests in flight hold at most the pool.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <condition_variable>
#include <deque>
#include <list>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "device_common.h"

namespace mknn {

static double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct ServerOp {
  uint64_t ticket = 0;
  bool is_update = false;           // a list update batch: a deletion, or an insertion
  bool is_insert = false;
  mknn_request req{};
  int32_t *h_idx = nullptr;
  float *h_dist = nullptr;
  mknn_cloud *cloud = nullptr;
  std::vector<int32_t> ranks;       // deletion
  std::vector<float> xyz;           // insertion, [count][3]
  DeviceDelta delta;
  double t_submit = 0, t_launch = 0, t_done = 0;
  int64_t seen = 0;                 // update batches applied to the cloud at launch
  mknn_status status = MKNN_OK;
  std::string err;
  bool done = false;
};
using OpPtr = std::shared_ptr<ServerOp>;

constexpr int kPlainSlots = 64;

struct Slot {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipEvent_t ev = nullptr;
  mknn_batch_plan *plan = nullptr;
  bool busy = false;
  std::vector<OpPtr> ops;
  std::unordered_set<mknn_cloud *> clouds;
  int64_t queries = 0;
};

struct Applying {   // a deletion whose device delta is on the deletion stream
  OpPtr op;
  hipEvent_t ev;
};

}  // namespace mknn

using namespace mknn;

struct mknn_server {
  int device = 0;
  bool plain = false;
  bool strict = true;               // requests see exactly the deletions submitted before them
  int64_t slot_queries = 0;         // largest wave (queries) one slot takes
  int64_t pool_queries = 0;
  int64_t inflight_queries = 0;     // plain mode: queries of the requests in flight
  int32_t max_wave = 0;
  std::vector<Slot> slots;
  hipStream_t del_stream = nullptr;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done, cv_work;
  std::atomic<bool> dirty{false};   // new operations or finished host work since the last pass
  std::deque<int> plain_order;      // plain mode: busy slots in launch order (one stream)
  std::list<OpPtr> pending;         // arrival order
  int64_t pending_updates = 0;
  std::unordered_map<uint64_t, OpPtr> ops;
  std::unordered_set<mknn_cloud *> blocked;   // a deletion is in its host or device part
  std::unordered_map<mknn_cloud *, int64_t> applied;   // deletion batches applied per cloud
  std::unordered_map<mknn_cloud *, hipEvent_t> ready_ev;
  std::deque<OpPtr> del_queue, del_done;
  std::vector<Applying> applying;
  std::vector<hipEvent_t> free_events;
  std::vector<std::thread> workers;
  std::thread sched;
  bool stop = false;
  uint64_t next_ticket = 1;
  int64_t waves = 0, wave_requests = 0;
  // seconds the scheduler spent launching waves, applying deltas and freeing old arenas,
  // and host seconds of the workers' deletion work (printed at destroy if MKNN_SERVER_TRACE)
  double t_launch = 0, t_apply = 0, t_release = 0, t_prepare = 0;
  int64_t repacks = 0;
};

namespace mknn {

static void wake_scheduler(mknn_server *s) {
  s->dirty.store(true, std::memory_order_release);
  s->cv_sched.notify_one();
}

static hipEvent_t take_event(mknn_server *s) {
  if (!s->free_events.empty()) {
    hipEvent_t e = s->free_events.back();
    s->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

static void finish_op(mknn_server *s, const OpPtr &op, mknn_status st, const std::string &err) {
  op->status = st;
  op->err = err;
  op->t_done = now_s();
  op->done = true;
  s->cv_done.notify_all();
}

// Launch one wave of requests on slot x (mu held).
static void launch_wave(mknn_server *s, int x, std::vector<OpPtr> &wave) {
  Slot &sl = s->slots[x];
  sl.ops = wave;
  sl.clouds.clear();
  const double t_launch = now_s();
  for (const OpPtr &op : wave) {
    op->t_launch = t_launch;
    sl.clouds.insert(op->cloud);
    auto it = s->applied.find(op->cloud);
    op->seen = it == s->applied.end() ? 0 : it->second;
    // a prefix beyond the lists the request runs on (possible when bound at admission
    // while an insertion of its submitter was pending) covers them all
    if (op->req.m > op->cloud->dev_n) op->req.m = 0;
  }
  for (mknn_cloud *c : sl.clouds) {
    auto it = s->ready_ev.find(c);
    if (it != s->ready_ev.end()) (void)hipStreamWaitEvent(sl.stream, it->second, 0);
  }
  mknn_status st = MKNN_OK;
  if (s->plain) {
    const mknn_request &r = wave[0]->req;
    st = mknn_knn(r.cloud, r.d_q, r.nq, r.k, r.m == 0 ? (int32_t)r.cloud->dev_n : r.m, r.d_idx,
                  r.d_dist, sl.stream);
  } else {
    std::vector<mknn_request> reqs;
    reqs.reserve(wave.size());
    for (const OpPtr &op : wave) reqs.push_back(op->req);
    st = mknn_batch_plan_run(sl.plan, reqs.data(), (int32_t)reqs.size(), sl.stream);
  }
  const std::string err = st == MKNN_OK ? "" : mknn_last_error();
  for (const OpPtr &op : wave) {
    if (st != MKNN_OK) continue;
    const mknn_request &r = op->req;
    const size_t cnt = (size_t)r.nq * (size_t)r.k;
    if (cnt && op->h_idx)
      (void)hipMemcpyAsync(op->h_idx, r.d_idx, cnt * sizeof(int32_t), hipMemcpyDeviceToHost, sl.stream);
    if (cnt && op->h_dist)
      (void)hipMemcpyAsync(op->h_dist, r.d_dist, cnt * sizeof(float), hipMemcpyDeviceToHost, sl.stream);
  }
  if (st != MKNN_OK) {
    for (const OpPtr &op : wave) finish_op(s, op, st, err);
    sl.ops.clear();
    return;
  }
  (void)hipEventRecord(sl.ev, sl.stream);
  sl.busy = true;
  if (s->plain) s->plain_order.push_back(x);
  for (const OpPtr &op : wave) sl.queries += op->req.nq;
  s->inflight_queries += sl.queries;
  ++s->waves;
  s->wave_requests += (int64_t)wave.size();
}

static void worker_loop(mknn_server *s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_work.wait(lk, [&] { return s->stop || !s->del_queue.empty(); });
    if (s->del_queue.empty()) {
      if (s->stop) return;
      continue;
    }
    OpPtr op = s->del_queue.front();
    s->del_queue.pop_front();
    lk.unlock();
    // host part of Alg. 3, or of an insertion
    const double t0 = now_s();
    op->status = op->is_insert
                     ? insert_prepare(op->cloud, op->xyz.data(), (int64_t)op->xyz.size() / 3, &op->delta)
                     : delete_prepare(op->cloud, op->ranks.data(), (int64_t)op->ranks.size(), &op->delta);
    if (op->status != MKNN_OK) op->err = mknn_last_error();
    const double dt = now_s() - t0;
    lk.lock();
    s->t_prepare += dt;
    s->del_done.push_back(op);
    wake_scheduler(s);
  }
}

static bool server_idle(const mknn_server *s) {
  bool idle = s->pending.empty() && s->blocked.empty() && s->applying.empty();
  for (const Slot &sl : s->slots) idle &= !sl.busy;
  return idle;
}

// The scheduler thread owns the slots and the list of deltas being applied; it polls their
// completion events without the lock, so submitters and waiters are not starved, and takes
// the lock only when something finished or new work arrived.
static void scheduler_loop(mknn_server *s) {
  (void)hipSetDevice(s->device);
  std::vector<int> done_slots;
  std::vector<size_t> done_apps;
  for (;;) {
    done_slots.clear();
    done_apps.clear();
    bool inflight = !s->applying.empty();
    if (s->plain) {
      // one stream: requests complete in launch order
      for (int x : s->plain_order) {
        if (hipEventQuery(s->slots[x].ev) != hipSuccess) break;
        done_slots.push_back(x);
      }
      inflight |= !s->plain_order.empty();
    } else {
      for (int x = 0; x < (int)s->slots.size(); ++x) {
        if (!s->slots[x].busy) continue;
        inflight = true;
        if (hipEventQuery(s->slots[x].ev) == hipSuccess) done_slots.push_back(x);
      }
    }
    for (size_t t = 0; t < s->applying.size(); ++t)
      if (hipEventQuery(s->applying[t].ev) == hipSuccess) done_apps.push_back(t);
    const bool fresh = s->dirty.exchange(false, std::memory_order_acq_rel);
    if (done_slots.empty() && done_apps.empty() && !fresh) {
      if (inflight) {
        std::this_thread::yield();
        continue;
      }
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->stop && server_idle(s)) break;
      s->cv_sched.wait_for(lk, std::chrono::milliseconds(2),
                           [&] { return s->stop || s->dirty.load(std::memory_order_acquire); });
      continue;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    // ---- completions of waves
    for (int x : done_slots) {
      Slot &sl = s->slots[x];
      for (const OpPtr &op : sl.ops) finish_op(s, op, MKNN_OK, "");
      sl.ops.clear();
      sl.clouds.clear();
      s->inflight_queries -= sl.queries;
      sl.queries = 0;
      sl.busy = false;
      if (s->plain) s->plain_order.pop_front();
    }
    // ---- completions of applied deletions (indices ascending: erase from the back)
    for (size_t t = done_apps.size(); t-- > 0;) {
      Applying &ap = s->applying[done_apps[t]];
      if (ap.op->delta.old_ent) {
        const double t0 = now_s();
        release_old_arena(&ap.op->delta);
        s->t_release += now_s() - t0;
      }
      finish_op(s, ap.op, MKNN_OK, "");
      s->free_events.push_back(ap.ev);
      s->applying.erase(s->applying.begin() + (std::ptrdiff_t)done_apps[t]);
    }
    // ---- deletions whose host part finished: order the device delta after the waves that
    //      still read the cloud, then release the cloud
    while (!s->del_done.empty()) {
      OpPtr op = s->del_done.front();
      s->del_done.pop_front();
      mknn_cloud *c = op->cloud;
      if (op->status == MKNN_OK && op->delta.on_device) {
        // the in-flight waves on this cloud finish before the switch (and before a replaced
        // arena is freed, when the applied event completes)
        for (Slot &sl : s->slots)
          if (sl.busy && sl.clouds.count(c)) (void)hipStreamWaitEvent(s->del_stream, sl.ev, 0);
        const double t0 = now_s();
        op->t_launch = t0;
        s->repacks += op->delta.repack ? 1 : 0;
        mknn_status st = apply_delta(c, &op->delta, s->del_stream);
        s->t_apply += now_s() - t0;
        if (st != MKNN_OK) {
          op->status = st;
          op->err = mknn_last_error();
        }
      }
      s->blocked.erase(c);
      if (op->status != MKNN_OK) {
        finish_op(s, op, op->status, op->err);
        continue;
      }
      ++s->applied[c];
      hipEvent_t &rev = s->ready_ev[c];
      if (!rev) rev = take_event(s);
      hipEvent_t done_ev = take_event(s);
      (void)hipEventRecord(rev, s->del_stream);
      (void)hipEventRecord(done_ev, s->del_stream);
      s->applying.push_back({op, done_ev});
    }
    // ---- form waves on the free slots, in arrival order
    for (int x = 0; x < (int)s->slots.size(); ++x) {
      if (s->slots[x].busy) continue;
      std::unordered_set<mknn_cloud *> held;   // strict order: clouds with an earlier waiting op
      std::vector<OpPtr> wave;
      int64_t wq = 0;
      for (auto it = s->pending.begin(); it != s->pending.end();) {
        const OpPtr &op = *it;
        mknn_cloud *c = op->cloud;
        if (op->is_update || (s->strict && (s->blocked.count(c) || held.count(c)))) {
          if (s->strict) held.insert(c);
          ++it;
          continue;
        }
        const int64_t nq = op->req.nq;
        const bool fits = s->plain ? wave.empty() && s->inflight_queries + nq <= s->pool_queries
                                   : (int64_t)wave.size() < s->max_wave && wq + nq <= s->slot_queries;
        if (!fits) break;   // later requests wait for the next wave, in arrival order
        wave.push_back(op);
        wq += nq;
        it = s->pending.erase(it);
      }
      if (wave.empty()) break;   // the other free slots would find the same
      const double t0 = now_s();
      launch_wave(s, x, wave);
      s->t_launch += now_s() - t0;
    }
    // ---- start deletions: one at a time per cloud, in arrival order; in strict order only
    //      once no earlier request on the cloud is still waiting
    if (s->pending_updates > 0) {
      std::unordered_set<mknn_cloud *> held, del_held;
      for (auto it = s->pending.begin(); it != s->pending.end();) {
        const OpPtr &op = *it;
        mknn_cloud *c = op->cloud;
        if (!op->is_update) {
          held.insert(c);
          ++it;
          continue;
        }
        if (!s->blocked.count(c) && !del_held.count(c) && !(s->strict && held.count(c))) {
          s->blocked.insert(c);
          s->del_queue.push_back(op);
          --s->pending_updates;
          s->cv_work.notify_one();
          it = s->pending.erase(it);
        } else {
          del_held.insert(c);
          ++it;
        }
      }
    }
    if (s->stop && server_idle(s)) break;
  }
}

}  // namespace mknn

extern "C" {

double mknn_server_now(void) { return now_s(); }

mknn_status mknn_server_create(int64_t pool_queries, int32_t nstreams, int32_t max_wave_requests,
                               int32_t flags, mknn_server **out) {
  clear_error();
  if (!out) return set_error(MKNN_EINVAL, "mknn_server_create: out is NULL");
  *out = nullptr;
  const bool plain = (flags & MKNN_SERVER_PLAIN) != 0;
  const bool strict = (flags & MKNN_SERVER_BIND_AT_ADMISSION) == 0;
  if (nstreams < 1 || nstreams > 8 || pool_queries < 1 || max_wave_requests < 1)
    return set_error(MKNN_EINVAL, "mknn_server_create: bad capacity");
  mknn_server *s = new (std::nothrow) mknn_server();
  if (!s) return set_error(MKNN_ENOMEM, "mknn_server_create: out of host memory");
  s->plain = plain;
  s->strict = strict;
  s->pool_queries = pool_queries;
  s->slot_queries = plain ? pool_queries : std::max<int64_t>(1, pool_queries / nstreams);
  s->max_wave = plain ? 1 : max_wave_requests;
  hipError_t e = hipGetDevice(&s->device);
  s->slots.resize(plain ? kPlainSlots : nstreams);
  for (Slot &sl : s->slots) {
    if (e == hipSuccess && (!plain || &sl == &s->slots[0])) {
      e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
      sl.own_stream = true;
    } else if (plain) {
      sl.stream = s->slots[0].stream;
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
    if (e == hipSuccess && !plain) {
      if (mknn_batch_plan_create(s->max_wave, s->slot_queries, 16, 0, &sl.plan) != MKNN_OK) {
        const std::string msg = mknn_last_error();
        mknn_server_destroy(s);
        return set_error(MKNN_ENOMEM, "mknn_server_create: " + msg);
      }
    }
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->del_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    mknn_server_destroy(s);
    return set_error(MKNN_EHIP, std::string("mknn_server_create: ") + hipGetErrorName(e));
  }
  const unsigned hw = std::thread::hardware_concurrency();
  const int nworkers = (int)std::max(1u, std::min(8u, hw > 2 ? hw / 2 : 1u));
  for (int w = 0; w < nworkers; ++w) s->workers.emplace_back(worker_loop, s);
  s->sched = std::thread(scheduler_loop, s);
  *out = s;
  return MKNN_OK;
}

mknn_status mknn_server_submit(mknn_server *s, const mknn_request *req, int32_t *h_idx,
                               float *h_dist, uint64_t *ticket) {
  clear_error();
  if (!s || !req || !ticket) return set_error(MKNN_EINVAL, "mknn_server_submit: NULL argument");
  const mknn_request &r = *req;
  if (!r.cloud || !r.cloud->d_ent)
    return set_error(MKNN_EINVAL, "mknn_server_submit: cloud missing or never uploaded");
  if (r.k > MKNN_KMAX) return set_error(MKNN_EUNSUPPORTED, "mknn_server_submit: k above MKNN_KMAX");
  if (r.k < 1 || r.m < 0 || r.m > r.cloud->n || r.nq < 0)
    return set_error(MKNN_EINVAL, "mknn_server_submit: k, m or nq out of range");
  if (r.nq > 0 && (!r.d_q || !r.d_idx || !r.d_dist))
    return set_error(MKNN_EINVAL, "mknn_server_submit: NULL buffer");
  if (r.nq > s->slot_queries)
    return set_error(MKNN_EBUSY, "mknn_server_submit: request larger than a stream slot's pool");
  OpPtr op = std::make_shared<ServerOp>();
  op->req = r;
  op->h_idx = h_idx;
  op->h_dist = h_dist;
  op->cloud = const_cast<mknn_cloud *>(r.cloud);
  op->t_submit = now_s();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return set_error(MKNN_EINVAL, "mknn_server_submit: server is stopping");
  op->ticket = s->next_ticket++;
  *ticket = op->ticket;
  s->ops[op->ticket] = op;
  if (r.nq == 0) {
    finish_op(s, op, MKNN_OK, "");
    return MKNN_OK;
  }
  s->pending.push_back(op);
  wake_scheduler(s);
  return MKNN_OK;
}

mknn_status mknn_server_delete(mknn_server *s, mknn_cloud *c, const int32_t *ranks, int64_t count,
                               uint64_t *ticket) {
  clear_error();
  if (!s || !c || !ticket || count < 0 || (count > 0 && !ranks))
    return set_error(MKNN_EINVAL, "mknn_server_delete: bad argument");
  OpPtr op = std::make_shared<ServerOp>();
  op->is_update = true;
  op->cloud = c;
  op->ranks.assign(ranks, ranks + count);
  op->t_submit = now_s();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return set_error(MKNN_EINVAL, "mknn_server_delete: server is stopping");
  op->ticket = s->next_ticket++;
  *ticket = op->ticket;
  s->ops[op->ticket] = op;
  s->pending.push_back(op);
  ++s->pending_updates;
  wake_scheduler(s);
  return MKNN_OK;
}

mknn_status mknn_server_insert(mknn_server *s, mknn_cloud *c, const float *xyz, int64_t count,
                               uint64_t *ticket) {
  clear_error();
  if (!s || !c || !ticket || count < 0 || (count > 0 && !xyz))
    return set_error(MKNN_EINVAL, "mknn_server_insert: bad argument");
  OpPtr op = std::make_shared<ServerOp>();
  op->is_update = true;
  op->is_insert = true;
  op->cloud = c;
  op->xyz.assign(xyz, xyz + 3 * count);
  op->t_submit = now_s();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return set_error(MKNN_EINVAL, "mknn_server_insert: server is stopping");
  op->ticket = s->next_ticket++;
  *ticket = op->ticket;
  s->ops[op->ticket] = op;
  s->pending.push_back(op);
  ++s->pending_updates;
  wake_scheduler(s);
  return MKNN_OK;
}

mknn_status mknn_server_poll(mknn_server *s, uint64_t ticket, int32_t *done) {
  clear_error();
  if (!s || !done) return set_error(MKNN_EINVAL, "mknn_server_poll: NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->ops.find(ticket);
  if (it == s->ops.end()) return set_error(MKNN_ENOTFOUND, "mknn_server_poll: unknown ticket");
  *done = it->second->done ? 1 : 0;
  return MKNN_OK;
}

mknn_status mknn_server_wait(mknn_server *s, uint64_t ticket, double *times,
                             int64_t *updates_seen) {
  clear_error();
  if (!s) return set_error(MKNN_EINVAL, "mknn_server_wait: server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->ops.find(ticket);
  if (it == s->ops.end()) return set_error(MKNN_ENOTFOUND, "mknn_server_wait: unknown ticket");
  OpPtr op = it->second;
  s->cv_done.wait(lk, [&] { return op->done; });
  s->ops.erase(ticket);
  if (times) {
    times[0] = op->t_submit;
    times[1] = op->t_launch;
    times[2] = op->t_done;
  }
  if (updates_seen) *updates_seen = op->seen;
  if (op->status != MKNN_OK) return set_error(op->status, op->err);
  return MKNN_OK;
}

mknn_status mknn_server_stats(mknn_server *s, int64_t *waves, int64_t *wave_requests) {
  clear_error();
  if (!s) return set_error(MKNN_EINVAL, "mknn_server_stats: server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  if (waves) *waves = s->waves;
  if (wave_requests) *wave_requests = s->wave_requests;
  return MKNN_OK;
}

void mknn_server_destroy(mknn_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    wake_scheduler(s);
  }
  if (s->sched.joinable()) s->sched.join();
  if (std::getenv("MKNN_SERVER_TRACE"))
    std::fprintf(stderr,
                 "[mknn server] waves %lld (requests %lld): launch %.3f s, apply %.3f s "
                 "(%lld re-packs), arena release %.3f s, deletion host work %.3f s\n",
                 (long long)s->waves, (long long)s->wave_requests, s->t_launch, s->t_apply,
                 (long long)s->repacks, s->t_release, s->t_prepare);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->cv_work.notify_all();
  }
  for (std::thread &t : s->workers)
    if (t.joinable()) t.join();
  for (Slot &sl : s->slots) {
    if (sl.stream && sl.own_stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.plan) mknn_batch_plan_destroy(sl.plan);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
  }
  for (Slot &sl : s->slots) {
    if (sl.stream && sl.own_stream) (void)hipStreamDestroy(sl.stream);
  }
  if (s->del_stream) {
    (void)hipStreamSynchronize(s->del_stream);
    (void)hipStreamDestroy(s->del_stream);
  }
  for (auto &kv : s->ready_ev)
    if (kv.second) (void)hipEventDestroy(kv.second);
  for (hipEvent_t e : s->free_events) (void)hipEventDestroy(e);
  delete s;
}

}  // extern "C"
