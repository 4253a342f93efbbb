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
// With MKNN_SERVER_LAZY_DELETE the order is the strict one, but no request waits for the
// host part of a deletion.  A deletion batch gets the next epoch of its cloud and is marked
// at once in the cloud's device epoch array (a kernel on a marking stream; later waves on
// the cloud wait for it).  A request filters the marks of the epochs submitted before it:
// it walks k + 16 neighbours on the lists it finds and keeps the first k unmarked ones,
// exact whenever the walk holds k of them (Sec. 4.3's lists are not needed for that).  The
// device delta of a deletion (or insertion) is applied once every request submitted before
// it has completed, so those requests never see its lists.  A request with a row the walk
// could not certify is queued again and answered once the deletions it saw are applied.
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
#include <map>
#include <memory>
#include <set>
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
  // lazy deletion: an update's sequence number on its cloud, or for a request the number of
  // update batches submitted on its cloud before it; a deletion's epoch, or for a request
  // the number of deletion epochs before it
  int64_t seq = 0;
  uint32_t epoch = 0;
  bool marked = false;              // a deletion's marks are enqueued
  bool rerun = false;               // a request answered again after an uncertified row
  uint32_t *old_dead = nullptr;     // an insertion's replaced epoch array
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

// Lazy deletion: the order of one cloud's updates and requests.
struct CloudView {
  int64_t updates = 0;              // update batches submitted so far
  uint32_t epochs = 0;              // deletion epochs handed out so far
  std::set<uint32_t> marked_epochs; // deletions marked, delta not yet enqueued
  int64_t live = 0;                 // live points once the marked deletions are applied
  int64_t inserting = -1;           // sequence number of an insertion in progress
  bool grown = false;               // an insertion replaced the epoch array since the last mark
  std::unordered_set<int32_t> marked;        // ranks marked, not yet applied
  std::map<int64_t, int64_t> outstanding;    // requests waiting or in flight, by `seq`
  std::vector<int64_t> failed;               // sequence numbers of failed update batches
  std::deque<OpPtr> gated;          // host part done; the delta waits for earlier requests
};

}  // namespace mknn

using namespace mknn;

struct mknn_server {
  int device = 0;
  bool plain = false;
  bool strict = true;               // requests see exactly the deletions submitted before them
  bool lazy = false;                // strict order by marking deletions (MKNN_SERVER_LAZY_DELETE)
  hipStream_t mark_stream = nullptr;
  std::unordered_map<mknn_cloud *, CloudView> views;
  std::unordered_map<mknn_cloud *, hipEvent_t> mark_ev;   // after the cloud's last marks
  int64_t reruns = 0;
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

// Lazy deletion: whether a request whose view holds the deletion epochs 1 .. epoch still
// finds some of them marked and not yet applied on the device lists.
static bool needs_filter(const CloudView &v, uint32_t epoch) {
  return !v.marked_epochs.empty() && *v.marked_epochs.begin() <= epoch;
}

// Lazy deletion: a request no longer holds back the deltas of later updates on its cloud.
static void release_outstanding(mknn_server *s, const OpPtr &op) {
  auto &o = s->views[op->cloud].outstanding;
  auto it = o.find(op->seq);
  if (it != o.end() && --it->second == 0) o.erase(it);
}

// Lazy deletion: queue a request again, at its place in arrival order (mu held).
static void requeue(mknn_server *s, const OpPtr &op) {
  op->rerun = true;
  ++s->reruns;
  auto it = s->pending.begin();
  while (it != s->pending.end() && (*it)->ticket < op->ticket) ++it;
  s->pending.insert(it, op);
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
    if (s->lazy) {
      // every update batch before the request is in its view, the failed ones aside
      const CloudView &v = s->views[op->cloud];
      op->seen = op->seq - (int64_t)std::count_if(v.failed.begin(), v.failed.end(),
                                                  [&](int64_t u) { return u < op->seq; });
    } else {
      auto it = s->applied.find(op->cloud);
      op->seen = it == s->applied.end() ? 0 : it->second;
    }
    // a prefix beyond the lists the request runs on (possible when bound at admission
    // while an insertion of its submitter was pending) covers them all
    if (op->req.m > op->cloud->dev_n) op->req.m = 0;
  }
  for (mknn_cloud *c : sl.clouds) {
    auto it = s->ready_ev.find(c);
    if (it != s->ready_ev.end()) (void)hipStreamWaitEvent(sl.stream, it->second, 0);
    auto im = s->mark_ev.find(c);
    if (im != s->mark_ev.end()) (void)hipStreamWaitEvent(sl.stream, im->second, 0);
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
    if (s->lazy) {
      // filter the marks of the deletions before each request, unless all are applied
      std::vector<uint32_t> ep;
      ep.reserve(wave.size());
      for (const OpPtr &op : wave)
        ep.push_back(needs_filter(s->views[op->cloud], op->epoch) ? op->epoch : 0u);
      st = batch_plan_run_pending(sl.plan, reqs.data(), (int32_t)reqs.size(), sl.stream, ep.data());
    } else {
      st = mknn_batch_plan_run(sl.plan, reqs.data(), (int32_t)reqs.size(), sl.stream);
    }
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
    for (const OpPtr &op : wave) {
      if (s->lazy) release_outstanding(s, op);
      finish_op(s, op, st, err);
    }
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

// Enqueue the device delta of an update whose host part finished (mu held): ordered after
// the in-flight waves that read the cloud (and before a replaced arena is freed, when the
// applied event completes); then the cloud's next update may start.
static void enqueue_delta(mknn_server *s, const OpPtr &op) {
  mknn_cloud *c = op->cloud;
  if (op->status == MKNN_OK && op->delta.on_device) {
    for (Slot &sl : s->slots)
      if (sl.busy && sl.clouds.count(c)) (void)hipStreamWaitEvent(s->del_stream, sl.ev, 0);
    const double t0 = now_s();
    op->t_launch = t0;
    s->repacks += op->delta.repack ? 1 : 0;
    mknn_status st = apply_delta(c, &op->delta, s->del_stream);
    if (st == MKNN_OK && s->lazy && op->is_insert && c->d_dead && c->dead_cap < c->n) {
      // the epoch array grows with the cloud (the old one is freed with the old arena)
      st = ensure_epochs_async(c, c->n, s->del_stream, &op->old_dead);
      s->views[c].grown = true;
    }
    s->t_apply += now_s() - t0;
    if (st != MKNN_OK) {
      op->status = st;
      op->err = mknn_last_error();
    }
  }
  s->blocked.erase(c);
  if (s->lazy) {
    CloudView &v = s->views[c];
    if (op->is_insert) {
      v.inserting = -1;
    } else {
      v.marked_epochs.erase(op->epoch);
      for (int32_t r : op->ranks) v.marked.erase(r);
    }
    if (op->status != MKNN_OK) {
      v.failed.push_back(op->seq);
      v.live = c->nlive - (int64_t)v.marked.size();
    } else if (op->is_insert) {
      v.live += (int64_t)op->xyz.size() / 3;
    }
  }
  if (op->status != MKNN_OK) {
    finish_op(s, op, op->status, op->err);
    return;
  }
  ++s->applied[c];
  hipEvent_t &rev = s->ready_ev[c];
  if (!rev) rev = take_event(s);
  hipEvent_t done_ev = take_event(s);
  (void)hipEventRecord(rev, s->del_stream);
  (void)hipEventRecord(done_ev, s->del_stream);
  s->applying.push_back({op, done_ev});
}

// Lazy deletion: the deltas whose earlier requests have all completed, in order (mu held).
static void apply_gated(mknn_server *s) {
  for (auto &kv : s->views) {
    CloudView &v = kv.second;
    while (!v.gated.empty()) {
      const OpPtr op = v.gated.front();
      // a request with seq <= op->seq was submitted before the update
      if (!v.outstanding.empty() && v.outstanding.begin()->first <= op->seq) break;
      v.gated.pop_front();
      enqueue_delta(s, op);
    }
  }
}

// Lazy deletion: mark the waiting deletion batches, in arrival order per cloud, once no
// insertion before them is still to be applied (mu held).  A batch is checked as
// mknn_delete checks it; a bad one fails whole and marks nothing.
static void mark_deletions(mknn_server *s) {
  std::unordered_set<mknn_cloud *> ins_held;
  for (auto it = s->pending.begin(); it != s->pending.end();) {
    const OpPtr op = *it;
    mknn_cloud *c = op->cloud;
    if (!op->is_update || op->marked) {
      ++it;
      continue;
    }
    if (op->is_insert) {
      ins_held.insert(c);
      ++it;
      continue;
    }
    CloudView &v = s->views[c];
    if (ins_held.count(c) || v.inserting >= 0) {
      ++it;
      continue;
    }
    // no insertion runs on the cloud now, so its size and live flags hold still; the
    // ranks of earlier marked batches are in v.marked (their live flags may be changing)
    mknn_status st = MKNN_OK;
    std::string err;
    std::vector<int32_t> sorted(op->ranks);
    std::sort(sorted.begin(), sorted.end());
    for (size_t t = 0; t < sorted.size() && st == MKNN_OK; ++t) {
      const int32_t r = sorted[t];
      if (r < 0 || r >= c->n || v.marked.count(r) || !c->live[r] || (t && sorted[t - 1] == r)) {
        st = MKNN_ENOTFOUND;
        err = "mknn_server_delete: rank " + std::to_string(r) +
              " is unknown, deleted, pending or repeated";
      }
    }
    if (st == MKNN_OK && v.live - (int64_t)sorted.size() < 1) {
      st = MKNN_EINVAL;
      err = "mknn_server_delete: a cloud must keep at least one point";
    }
    if (st == MKNN_OK && !sorted.empty()) {
      if (v.grown) {
        // an insertion replaced the array on the deletion stream
        auto ie = s->ready_ev.find(c);
        if (ie != s->ready_ev.end()) (void)hipStreamWaitEvent(s->mark_stream, ie->second, 0);
        v.grown = false;
      }
      uint32_t *old = nullptr;
      st = ensure_epochs_async(c, c->n, s->mark_stream, &old);
      if (st == MKNN_OK && old) {
        // only before the first marks of this server can the array be too small: no wave
        // reads the old one
        (void)hipStreamSynchronize(s->mark_stream);
        (void)hipFree(old);
      }
      if (st == MKNN_OK) st = mark_deleted_async(c, op->ranks.data(), (int64_t)op->ranks.size(),
                                                 op->epoch, s->mark_stream);
      if (st != MKNN_OK) err = mknn_last_error();
    }
    if (st != MKNN_OK) {
      v.failed.push_back(op->seq);
      --s->pending_updates;
      it = s->pending.erase(it);
      finish_op(s, op, st, err);
      continue;
    }
    v.live -= (int64_t)sorted.size();
    v.marked.insert(sorted.begin(), sorted.end());
    if (!sorted.empty()) v.marked_epochs.insert(op->epoch);
    hipEvent_t &mev = s->mark_ev[c];
    if (!mev) mev = take_event(s);
    (void)hipEventRecord(mev, s->mark_stream);
    op->marked = true;
    op->t_launch = now_s();
    ++it;
  }
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
      const uint32_t *ovf = s->lazy && sl.plan ? batch_plan_overflow(sl.plan) : nullptr;
      for (size_t i = 0; i < sl.ops.size(); ++i) {
        const OpPtr &op = sl.ops[i];
        if (ovf && ovf[i] != 0) {
          requeue(s, op);   // a row could not be certified: answer again on applied lists
          continue;
        }
        if (s->lazy) release_outstanding(s, op);
        finish_op(s, op, MKNN_OK, "");
      }
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
      if (ap.op->old_dead) {
        (void)hipFree(ap.op->old_dead);
        ap.op->old_dead = nullptr;
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
      if (s->lazy)
        s->views[op->cloud].gated.push_back(op);   // after the requests submitted before it
      else
        enqueue_delta(s, op);
    }
    if (s->lazy) {
      apply_gated(s);
      mark_deletions(s);
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
        if (s->lazy) {
          // held: behind a deletion not yet marked or an insertion not yet applied, or
          // (answered again) until the deletions in its view are applied
          if (op->is_update) {
            if (op->is_insert || !op->marked) held.insert(c);
            ++it;
            continue;
          }
          const CloudView &v = s->views[c];
          if (held.count(c) || (v.inserting >= 0 && op->seq > v.inserting) ||
              (op->rerun && needs_filter(v, op->epoch))) {
            ++it;
            continue;
          }
        } else if (op->is_update || (s->strict && (s->blocked.count(c) || held.count(c)))) {
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
        bool start = !s->blocked.count(c) && !del_held.count(c);
        if (s->lazy)   // a deletion once marked; an insertion once no earlier request waits
          start = start && (op->is_insert ? !held.count(c) : op->marked);
        else
          start = start && !(s->strict && held.count(c));
        if (start) {
          if (s->lazy && op->is_insert) s->views[c].inserting = op->seq;
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

// Lazy deletion: the view of a cloud, made at the cloud's first operation (mu held).  The
// cloud must have no deletions pending from mknn_delete_lazy.
static mknn_status take_view(mknn_server *s, mknn_cloud *c, const char *who) {
  if (s->views.count(c)) return MKNN_OK;
  if (!c->lazy.empty())
    return set_error(MKNN_EINVAL, std::string(who) + ": the cloud has deletions pending from "
                                                     "mknn_delete_lazy (apply them first)");
  CloudView &v = s->views[c];
  v.live = c->nlive;
  v.epochs = c->lazy_epoch;          // above the epochs already in the cloud's array
  return MKNN_OK;
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
  const bool lazy = (flags & MKNN_SERVER_LAZY_DELETE) != 0;
  if (nstreams < 1 || nstreams > 8 || pool_queries < 1 || max_wave_requests < 1)
    return set_error(MKNN_EINVAL, "mknn_server_create: bad capacity");
  if (lazy && (plain || !strict))
    return set_error(MKNN_EINVAL, "mknn_server_create: MKNN_SERVER_LAZY_DELETE is a form of the "
                                  "strict order of the batched server");
  mknn_server *s = new (std::nothrow) mknn_server();
  if (!s) return set_error(MKNN_ENOMEM, "mknn_server_create: out of host memory");
  s->plain = plain;
  s->strict = strict;
  s->lazy = lazy;
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
  if (e == hipSuccess && lazy) e = hipStreamCreateWithFlags(&s->mark_stream, hipStreamNonBlocking);
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
  if (s->lazy) {
    mknn_status st = take_view(s, op->cloud, "mknn_server_submit");
    if (st != MKNN_OK) return st;
  }
  op->ticket = s->next_ticket++;
  *ticket = op->ticket;
  s->ops[op->ticket] = op;
  if (r.nq == 0) {
    finish_op(s, op, MKNN_OK, "");
    return MKNN_OK;
  }
  if (s->lazy) {
    CloudView &v = s->views[op->cloud];
    op->seq = v.updates;
    op->epoch = v.epochs;
    ++v.outstanding[op->seq];
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
  if (s->lazy) {
    mknn_status st = take_view(s, c, "mknn_server_delete");
    if (st != MKNN_OK) return st;
    CloudView &v = s->views[c];
    op->seq = v.updates++;
    op->epoch = ++v.epochs;
  }
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
  if (s->lazy) {
    mknn_status st = take_view(s, c, "mknn_server_insert");
    if (st != MKNN_OK) return st;
    op->seq = s->views[c].updates++;
  }
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
                 "(%lld re-packs), arena release %.3f s, deletion host work %.3f s, "
                 "requests answered again %lld\n",
                 (long long)s->waves, (long long)s->wave_requests, s->t_launch, s->t_apply,
                 (long long)s->repacks, s->t_release, s->t_prepare, (long long)s->reruns);
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
  if (s->mark_stream) {
    (void)hipStreamSynchronize(s->mark_stream);
    (void)hipStreamDestroy(s->mark_stream);
  }
  for (auto &kv : s->mark_ev)
    if (kv.second) (void)hipEventDestroy(kv.second);
  for (auto &kv : s->ready_ev)
    if (kv.second) (void)hipEventDestroy(kv.second);
  for (hipEvent_t e : s->free_events) (void)hipEventDestroy(e);
  delete s;
}

}  // extern "C"
