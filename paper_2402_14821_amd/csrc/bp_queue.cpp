// bp_queue.cpp -- served feasibility checks with continuous batching.
//
// A serving thread owns two pipeline contexts, each with its own stream and
// workspaces.  Requests are copied at submit and admitted against an HBM
// budget and a slot limit.  Whenever a context is idle the thread launches
// every admitted request that has not started yet as one batch on it, so
// arrivals during a running batch join the next launch on the other context
// and the two batches overlap on the device.  Finished batches release their
// budget and publish one result per request.
//
// Test hook: BP_TEST_FAIL_LAUNCH=n makes the n-th batch launch (1-based)
// fail on the host without touching the device; its requests complete with
// BP_ERR_DEVICE.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "bp_ctx.h"
#include "bp_internal.h"

using namespace bpi;

namespace {

constexpr uint64_t kQueueMagic = 0x6270717565756531ull;
constexpr int kMaxBatch = 8192;

double now_us() {
  using namespace std::chrono;
  return (double)duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count() * 1e-3;
}

struct Req {
  uint64_t ticket = 0, tag = 0;
  int32_t C = 0, m = 0;
  int64_t n = 0;
  uint32_t flags = 0;
  std::vector<int32_t> residual, unpacked;
  double submit_us = 0;
  size_t bytes = 0;
};

struct Slot {
  Ctx ctx;
  bool ready = false;
  bool busy = false;
  double start_us = 0;
  std::vector<Req> reqs;
};

// Device bytes a request occupies while admitted: its inputs, the sorted
// sizes, prefix sums and stream records, and its per-instance records.
size_t request_bytes(int64_t n, int64_t m) {
  const int64_t r = n + m;
  return (size_t)(4 * r + 4 * r + 8 * (r + 1) + 4 * r) + sizeof(InstPlan) +
         sizeof(InstState) + kNB * 8 + sizeof(bp_bounds) + 7 * sizeof(Entry) + 64;
}

struct Queue {
  uint64_t magic = 0;
  int device = 0;
  size_t budget = 0;
  int32_t max_slots = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_space, cv_results;
  std::deque<Req> pending;
  std::deque<bp_result> results;
  size_t bytes_in_use = 0, bytes_peak = 0;
  int64_t admitted = 0;  // submitted and not yet completed
  uint64_t submitted = 0, completed = 0, rejected = 0, batches = 0;
  double busy_us = 0;
  bool shutdown = false;
  uint64_t next_ticket = 1;
  long fail_launch_at = -1;
  Slot slots[2];
  std::thread thr;

  void publish(std::vector<Req> &reqs, const bp_bounds *out, bp_status batch_status, double start) {
    const double t = now_us();
    std::lock_guard<std::mutex> lk(mu);
    for (size_t i = 0; i < reqs.size(); ++i) {
      bp_result res;
      memset(&res, 0, sizeof res);
      res.ticket = reqs[i].ticket;
      res.tag = reqs[i].tag;
      res.submit_us = reqs[i].submit_us;
      res.start_us = start;
      res.done_us = t;
      if (batch_status == BP_OK && out) {
        res.bounds = out[i];
        res.status = out[i].status;
        res.verdict = out[i].verdict;
        res.lb = out[i].lb;
      } else {
        res.status = batch_status;
      }
      results.push_back(res);
      bytes_in_use -= reqs[i].bytes;
      --admitted;
      ++completed;
    }
    reqs.clear();
    cv_results.notify_all();
    cv_space.notify_all();
  }

  bp_status launch(Slot &s, std::vector<Req> &take) {
    std::vector<PlanIn> pin(take.size());
    std::vector<const int32_t *> a(take.size()), b(take.size());
    for (size_t i = 0; i < take.size(); ++i) {
      const Req &q = take[i];
      bp_status st = make_plan_in(q.C, q.m, q.n, q.m, kFormResidual, nullptr, !(q.flags & BP_NO_EARLY_EXIT), &pin[i],
                                  (q.flags & BP_SEGMENTS) != 0);
      if (st) return st;
      a[i] = q.unpacked.data();
      b[i] = q.residual.data();
    }
    return launch_host_batch(&s.ctx, pin, a, b);
  }

  void loop() {
    (void)hipSetDevice(device);
    std::vector<bp_bounds> outbuf;
    for (;;) {
      // 1. finished batches
      for (Slot &s : slots) {
        if (!s.busy) continue;
        if (hipEventQuery(s.ctx.done) == hipErrorNotReady) continue;
        outbuf.resize(s.reqs.size());
        bp_status st = collect_host_batch(&s.ctx, (int64_t)s.reqs.size(), outbuf.data(), false);
        const double t = now_us();
        {
          std::lock_guard<std::mutex> lk(mu);
          busy_us += t - s.start_us;
        }
        publish(s.reqs, outbuf.data(), st, s.start_us);
        s.busy = false;
      }
      // 2. launch what is waiting on an idle context
      Slot *idle = nullptr;
      for (Slot &s : slots)
        if (!s.busy) { idle = &s; break; }
      std::vector<Req> take;
      bool stop = false;
      {
        std::unique_lock<std::mutex> lk(mu);
        if (idle && !pending.empty() && !shutdown) {
          while (!pending.empty() && (int)take.size() < kMaxBatch) {
            take.push_back(std::move(pending.front()));
            pending.pop_front();
          }
        }
        const bool any_busy = slots[0].busy || slots[1].busy;
        if (take.empty()) {
          if (shutdown && !any_busy) stop = true;
          else if (!any_busy) cv_work.wait_for(lk, std::chrono::milliseconds(5));
        }
      }
      if (stop) break;
      if (!take.empty()) {
        ++batches;
        bp_status st;
        if (fail_launch_at > 0 && (long)batches == fail_launch_at) st = fail(BP_ERR_DEVICE, "injected launch failure");
        else st = launch(*idle, take);
        idle->start_us = now_us();
        if (st) {
          publish(take, nullptr, st, idle->start_us);
        } else {
          idle->reqs = std::move(take);
          idle->busy = true;
        }
        continue;
      }
      // a batch is running: poll its completion at a short interval
      if (slots[0].busy || slots[1].busy) {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait_for(lk, std::chrono::microseconds(20));
      }
    }
    // shut down: what never started completes with BP_ERR_STATE
    std::vector<Req> rest;
    {
      std::lock_guard<std::mutex> lk(mu);
      while (!pending.empty()) {
        rest.push_back(std::move(pending.front()));
        pending.pop_front();
      }
    }
    if (!rest.empty()) publish(rest, nullptr, BP_ERR_STATE, now_us());
  }
};

bp_status get_queue(bp_queue *q, Queue **out) {
  Queue *x = (Queue *)q;
  if (!x || x->magic != kQueueMagic) return fail(BP_ERR_STATE, "bad queue");
  *out = x;
  return BP_OK;
}

}  // namespace

bp_status bp_queue_create(bp_ctx *ctx, size_t hbm_budget_bytes, int32_t max_slots, bp_queue **out) {
  if (!out) return fail(BP_ERR_ARG, "out is NULL");
  *out = nullptr;
  Ctx *c = (Ctx *)ctx;
  if (!c || c->magic != kCtxMagic) return fail(BP_ERR_STATE, "bad context");
  if (hbm_budget_bytes == 0 || max_slots < 1) return fail(BP_ERR_ARG, "budget and max_slots must be positive");
  Queue *q = new (std::nothrow) Queue();
  if (!q) return fail(BP_ERR_NOMEM, "queue allocation");
  q->device = c->device;
  q->budget = hbm_budget_bytes;
  q->max_slots = max_slots;
  const char *fl = getenv("BP_TEST_FAIL_LAUNCH");
  if (fl) q->fail_launch_at = atol(fl);
  for (Slot &s : q->slots) {
    bp_status st = s.ctx.init(c->device);
    if (st) {
      for (Slot &t : q->slots) t.ctx.destroy();
      delete q;
      return st;
    }
    s.ctx.magic = kCtxMagic;
    s.ready = true;
  }
  q->magic = kQueueMagic;
  try {
    q->thr = std::thread([q] { q->loop(); });
  } catch (...) {
    for (Slot &t : q->slots) t.ctx.destroy();
    delete q;
    return fail(BP_ERR_NOMEM, "serving thread");
  }
  *out = (bp_queue *)q;
  return BP_OK;
}

bp_status bp_queue_submit(bp_queue *qh, const bp_request *req, int32_t blocking, uint64_t *ticket) {
  Queue *q;
  bp_status st = get_queue(qh, &q);
  if (st) return st;
  if (!req || !ticket) return fail(BP_ERR_ARG, "NULL argument");
  if (req->C < 1 || req->m < 0 || req->n < 0) return fail(BP_ERR_ARG, "bad request sizes");
  if ((req->m > 0 && !req->residual) || (req->n > 0 && !req->unpacked)) return fail(BP_ERR_ARG, "NULL request array");
  if (req->flags & ~(BP_NO_EARLY_EXIT | BP_SEGMENTS)) return fail(BP_ERR_ARG, "unknown flags");
  if (req->n + req->m > kLargeCap) return fail(BP_ERR_LIMIT, "request of %lld items", (long long)(req->n + req->m));
  if ((st = host_validate_items(req->C, req->unpacked, req->n))) return st;
  if ((st = host_validate_items(req->C, req->residual, req->m))) return st;
  Req r;
  r.tag = req->tag;
  r.C = req->C;
  r.m = req->m;
  r.n = req->n;
  r.flags = req->flags;
  r.bytes = request_bytes(req->n, req->m);
  if (r.bytes > q->budget) return fail(BP_ERR_LIMIT, "request needs %zu bytes > budget %zu", r.bytes, q->budget);
  r.residual.assign(req->residual, req->residual + req->m);
  r.unpacked.assign(req->unpacked, req->unpacked + req->n);
  std::unique_lock<std::mutex> lk(q->mu);
  for (;;) {
    if (q->shutdown) return fail(BP_ERR_STATE, "queue is shutting down");
    if (q->bytes_in_use + r.bytes <= q->budget && q->admitted < q->max_slots) break;
    if (!blocking) {
      ++q->rejected;
      return fail(BP_ERR_AGAIN, "no free slot or budget");
    }
    q->cv_space.wait(lk);
  }
  r.ticket = q->next_ticket++;
  r.submit_us = now_us();
  q->bytes_in_use += r.bytes;
  if (q->bytes_in_use > q->bytes_peak) q->bytes_peak = q->bytes_in_use;
  ++q->admitted;
  ++q->submitted;
  *ticket = r.ticket;
  q->pending.push_back(std::move(r));
  q->cv_work.notify_one();
  return BP_OK;
}

bp_status bp_queue_poll(bp_queue *qh, bp_result *out, int32_t max, int32_t *got, int32_t timeout_us) {
  Queue *q;
  bp_status st = get_queue(qh, &q);
  if (st) return st;
  if (!got || (max > 0 && !out) || max < 0) return fail(BP_ERR_ARG, "bad poll arguments");
  std::unique_lock<std::mutex> lk(q->mu);
  if (q->results.empty() && timeout_us > 0)
    q->cv_results.wait_for(lk, std::chrono::microseconds(timeout_us), [q] { return !q->results.empty(); });
  int32_t n = 0;
  while (n < max && !q->results.empty()) {
    out[n++] = q->results.front();
    q->results.pop_front();
  }
  *got = n;
  return BP_OK;
}

bp_status bp_queue_stats_get(bp_queue *qh, bp_queue_stats *out) {
  Queue *q;
  bp_status st = get_queue(qh, &q);
  if (st) return st;
  if (!out) return fail(BP_ERR_ARG, "out is NULL");
  std::lock_guard<std::mutex> lk(q->mu);
  out->submitted = q->submitted;
  out->completed = q->completed;
  out->rejected = q->rejected;
  out->batches = q->batches;
  out->in_flight = (uint64_t)q->admitted;
  out->bytes_in_use = q->bytes_in_use;
  out->bytes_peak = q->bytes_peak;
  out->budget = q->budget;
  out->busy_us = q->busy_us;
  return BP_OK;
}

bp_status bp_queue_destroy(bp_queue *qh) {
  Queue *q;
  bp_status st = get_queue(qh, &q);
  if (st) return st;
  {
    std::lock_guard<std::mutex> lk(q->mu);
    q->shutdown = true;
  }
  q->cv_work.notify_all();
  q->cv_space.notify_all();
  if (q->thr.joinable()) q->thr.join();
  q->magic = 0;
  for (Slot &s : q->slots) s.ctx.destroy();
  delete q;
  return BP_OK;
}
