// bp_queue.cpp -- served feasibility checks with continuous batching and
// incremental node states.
//
// A serving thread owns two pipeline contexts, each with its own stream and
// workspaces.  Requests are copied at submit and admitted against a slot
// limit and a byte allowance.  Whenever a context is idle the thread
// launches every admitted request that has not started yet as one batch on
// it, so arrivals during a running batch join the next launch on the other
// context and the two batches overlap on the device.
//
// A request is a node of the search.  A root (a partial packing) runs the
// full pipeline -- reduction, sort, L2 and the six sweeps -- and, when the
// node-state arena has room, also writes its node state: the per-parameter
// sums of every bound over its reduced items (node_layout).  A child (its
// parent's node plus committed items, Sec. 5) differs from an ancestor whose
// state is complete by a few reduced items: each committed size leaves the
// unpacked items, and its bin's virtual item (Fig. 3) changes from the old
// load to the new one.  Its state is the ancestor's plus those items' terms
// (k_node_delta), O(P) per changed item.  The ancestor may be a node of a
// finished batch (its state kept on the device), a root earlier in the same
// launch (stream order), or a node of a batch running on another context
// (the launch waits for that batch's end event).  A child with no such
// ancestor within the chain limits runs the full pipeline on its instance,
// rebuilt on the host from the nearest ancestor that carries one.
//
// Node states live in one device arena allocated at queue creation (three
// quarters of the budget), least recently used first out; the other quarter
// bounds the bytes charged to admitted requests.
//
// Test hook: BP_TEST_FAIL_LAUNCH=n makes the n-th batch launch (1-based)
// fail on the host without touching the device; its requests complete with
// BP_ERR_DEVICE.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "bp_ctx.h"
#include "bp_internal.h"

using namespace bpi;

#define QTRY(call)                                        \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return hip_fail(e_, #call);     \
  } while (0)

namespace {

constexpr uint64_t kQueueMagic = 0x6270717565756531ull;
constexpr int kMaxBatch = 8192;
// Batches in flight at once, each on a context and stream of its own: a
// batch with roots (full pipelines) does not hold up the children that
// arrive meanwhile.  Three measured no faster than two on the 200k/s
// search stream (smaller batches, same completion rate).
constexpr int kQueueSlots = 2;
constexpr int kChainDepth = 64;       // ancestors a child's base search visits
constexpr int kMaxDelta = 4096;       // changed reduced items a child may be computed from
constexpr int kFlattenEvery = 32;     // a node keeps full loads and unpacked sizes every this many levels

double now_us() {
  using namespace std::chrono;
  return (double)duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count() * 1e-3;
}

// Encoded change of the reduced instance: v > 0 adds a size v - 1, v < 0
// removes a size -v - 1 (NodeTask::delta).
inline int32_t add_item(int32_t w) { return w + 1; }
inline int32_t rem_item(int32_t w) { return -w - 1; }

// Host record of a node of the search.
struct Node {
  uint64_t ticket = 0, parent = 0;
  int32_t C = 0, m = 0;
  int depth = 0;                      // levels since the nearest node holding full loads and sizes
  std::vector<int32_t> load;          // depth 0: every bin's load (C - residual)
  std::vector<int32_t> unpacked;      // depth 0: the unpacked sizes
  std::vector<std::pair<int32_t, int32_t>> changed;  // depth > 0: (bin, new load) of the commits
  std::vector<int32_t> committed;     // depth > 0: sizes committed since the parent
  std::vector<int32_t> delta;         // depth > 0: change of the reduced instance vs the parent
  int64_t r = 0, sumW = 0, n_unp = 0;
  int32_t nbig = 0;
  int64_t slot = -1;                  // node state at arena + slot (elements), when kept
  bool complete = false;              // the state at slot is written and valid
  int in_flight = -1;                 // context index while its batch runs
  bool guaranteed = false;            // in flight with a slot whose state will be complete (no early exit)
  int pins = 0;                       // launches that read its state
  bool in_lru = false;
  std::list<uint64_t>::iterator lru;
};

struct Req {
  uint64_t ticket = 0, tag = 0;
  uint32_t flags = 0;
  double submit_us = 0;
  size_t bytes = 0;
};

// One planned request of a batch.
struct Work {
  Req req;
  bp_status err = BP_OK;     // set when the request cannot run (its record carries it)
  bool full = true;          // full pipeline, else from a base's state
  bool early = false;        // full pipeline with early exit
  std::vector<int32_t> residual, unpacked;  // full: the instance
  uint64_t base = 0;         // child: the base node
  std::vector<int32_t> delta;  // child: change vs the base
  int wait_slot = -1;        // child: the base is in flight on this context
};

struct Slot {
  Ctx ctx;
  bool busy = false;
  double start_us = 0;
  std::vector<Work> work;
  std::vector<uint64_t> pinned;  // nodes whose state this launch reads
  DevBuf node_dev;               // [NodeTask][delta][keys] of the launch's children
  HostBuf node_host;
  HostBuf out_host;
  DevBuf out_dev;
};

size_t state_elems(int32_t C) {
  int64_t off[kNB + 1];
  node_layout(C, off);
  return (size_t)off[kNB];
}

int64_t param_count(int32_t C) {
  int64_t off[kNB + 1];
  node_layout(C, off);
  return off[kNB] - off[kMT];
}

// Bytes charged to an admitted request: for the full pipeline its inputs,
// sorted sizes, stream records, prefix sums, one partial-sum slot per
// parameter and, for an instance the planner prepares from value tables
// (large, c at most kVtRatio times its items), those tables; for a child its
// changed items and task record.
size_t full_bytes(int64_t n, int64_t m, int32_t C) {
  const int64_t r = n + m;
  const bool vt = r > kSmallCap && C <= kVtMaxC && (int64_t)C <= kVtRatio * r;
  const int64_t tables = vt ? 16 * ((int64_t)C + 2) + 32 * (((int64_t)C + 2 + kVtChunk - 1) / kVtChunk) + 8 : 0;
  return (size_t)(4 * (n + m) + 16 * r + 8 * (r + 1) + 8 * param_count(C) + tables) + sizeof(InstPlan) +
         sizeof(InstState) + kNB * 8 + sizeof(bp_bounds) + 8 * sizeof(Entry) + 256;
}
size_t child_bytes(int32_t ncommit) {
  return (size_t)(12 * ncommit) * 4 + sizeof(NodeTask) + kNB * 8 + sizeof(bp_bounds) + 64;
}

struct Queue {
  uint64_t magic = 0;
  int device = 0;
  size_t budget = 0, allowance = 0;
  int32_t max_slots = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_space, cv_results;
  std::deque<Req> pending;
  std::atomic<uint64_t> npending{0};  // pending.size(), readable without mu
  std::deque<bp_result> results;
  size_t bytes_in_use = 0, bytes_peak = 0;
  int64_t admitted = 0;  // submitted and not yet completed
  uint64_t submitted = 0, completed = 0, rejected = 0, batches = 0, n_delta = 0, n_full = 0, evictions = 0;
  double busy_us = 0;
  bool shutdown = false;
  uint64_t next_ticket = 1;
  long fail_launch_at = -1;
  Slot slots[kQueueSlots];
  std::thread thr;

  // node records (guarded by mu)
  std::unordered_map<uint64_t, Node> nodes;
  std::deque<uint64_t> history;  // tickets in submission order, for forgetting old records
  // the requests' instances for the full pipeline, by ticket (guarded by mu)
  std::unordered_map<uint64_t, std::pair<std::vector<int32_t>, std::vector<int32_t>>> instances;

  // node-state arena (serving thread only, with mu held)
  long long *arena = nullptr;
  size_t arena_elems = 0, arena_top = 0;
  std::map<size_t, std::vector<size_t>> free_slots;  // by size in elements
  std::list<uint64_t> lru;                            // kept, complete, unpinned-or-pinned nodes, oldest first
  uint64_t kept = 0;

  // -- node records -----------------------------------------------------------

  Node *find(uint64_t t) {
    auto it = nodes.find(t);
    return it == nodes.end() ? nullptr : &it->second;
  }

  // Load of bin j at node x (walks to the nearest node holding all loads).
  bool load_of(const Node *x, int32_t j, int32_t *out) {
    for (int guard = 0; guard <= kFlattenEvery + 1 && x; ++guard) {
      for (auto it = x->changed.rbegin(); it != x->changed.rend(); ++it)
        if (it->first == j) {
          *out = it->second;
          return true;
        }
      if (x->depth == 0) {
        *out = x->load[(size_t)j];
        return true;
      }
      x = find(x->parent);
    }
    return false;
  }

  // Full loads and unpacked sizes of node x, rebuilt from the nearest node
  // holding them and the commits since.
  bool instance_of(const Node *x, std::vector<int32_t> *load, std::vector<int32_t> *unp) {
    std::vector<const Node *> chain;
    const Node *y = x;
    while (y && y->depth > 0) {
      chain.push_back(y);
      y = find(y->parent);
      if (chain.size() > (size_t)kFlattenEvery + 1) return false;
    }
    if (!y) return false;
    *load = y->load;
    std::vector<int32_t> gone;
    for (auto it = chain.rbegin(); it != chain.rend(); ++it) {
      for (auto &cb : (*it)->changed) (*load)[(size_t)cb.first] = cb.second;
      gone.insert(gone.end(), (*it)->committed.begin(), (*it)->committed.end());
    }
    // the unpacked multiset minus the committed sizes
    std::unordered_map<int32_t, int64_t> cnt;
    for (int32_t w : gone) ++cnt[w];
    unp->clear();
    unp->reserve(y->unpacked.size());
    for (int32_t w : y->unpacked) {
      auto it = cnt.find(w);
      if (it != cnt.end() && it->second > 0) {
        --it->second;
        continue;
      }
      unp->push_back(w);
    }
    for (auto &kv : cnt)
      if (kv.second) return false;  // a committed size the ancestor never had unpacked
    return true;
  }

  void forget_old_nodes() {
    while (history.size() > (size_t)BP_QUEUE_HISTORY) {
      const uint64_t t = history.front();
      Node *x = find(t);
      if (x && (x->pins > 0 || x->in_flight >= 0)) break;  // still needed; retry later
      history.pop_front();
      if (!x) continue;
      if (x->slot >= 0) free_state(*x);
      nodes.erase(t);
    }
  }

  // -- arena ----------------------------------------------------------------

  void free_state(Node &x) {
    if (x.in_lru) {
      lru.erase(x.lru);
      x.in_lru = false;
    }
    if (x.slot >= 0) {
      free_slots[state_elems(x.C)].push_back((size_t)x.slot);
      --kept;
    }
    x.slot = -1;
    x.complete = false;
  }

  // A slot for a node state of capacity C; evicts least recently used
  // complete states that no launch reads.  -1 when nothing fits.
  int64_t alloc_state(int32_t C) {
    const size_t need = state_elems(C);
    for (;;) {
      auto &fl = free_slots[need];
      if (!fl.empty()) {
        const size_t s = fl.back();
        fl.pop_back();
        ++kept;
        return (int64_t)s;
      }
      if (arena_top + need <= arena_elems) {
        const size_t s = arena_top;
        arena_top += need;
        ++kept;
        return (int64_t)s;
      }
      // evict the oldest unpinned state of the same size
      bool freed = false;
      for (auto it = lru.begin(); it != lru.end(); ++it) {
        Node *x = find(*it);
        if (!x || x->pins > 0 || x->in_flight >= 0 || state_elems(x->C) != need) continue;
        free_state(*x);
        ++evictions;
        freed = true;
        break;
      }
      if (!freed) return -1;
    }
  }

  void touch(Node &x) {
    if (!x.in_lru) return;
    lru.splice(lru.end(), lru, x.lru);
  }

  // -- results --------------------------------------------------------------

  void publish(std::vector<Work> &work, const bp_bounds *out, bp_status batch_status, double start, int slot_idx) {
    const double t = now_us();
    std::lock_guard<std::mutex> lk(mu);
    for (size_t i = 0; i < work.size(); ++i) {
      const Req &q = work[i].req;
      bp_result res;
      memset(&res, 0, sizeof res);
      res.ticket = q.ticket;
      res.tag = q.tag;
      res.submit_us = q.submit_us;
      res.start_us = start;
      res.done_us = t;
      res.from_parent = work[i].full ? 0 : 1;
      if (batch_status == BP_OK && out && work[i].err == BP_OK) {
        res.bounds = out[i];
        res.status = out[i].status;
        res.verdict = out[i].verdict;
        res.lb = out[i].lb;
      } else {
        res.status = batch_status != BP_OK ? batch_status : work[i].err;
      }
      Node *x = find(q.ticket);
      if (x && x->in_flight == slot_idx) {
        x->in_flight = -1;
        x->guaranteed = false;
        if (x->slot >= 0) {
          // complete unless an early exit skipped part of the sweeps
          if (res.status == BP_OK && batch_status == BP_OK && !res.bounds.early_exit) {
            x->complete = true;
            x->lru = lru.insert(lru.end(), x->ticket);
            x->in_lru = true;
          } else {
            free_state(*x);
          }
        }
      }
      if (work[i].full) ++n_full; else ++n_delta;
      results.push_back(res);
      bytes_in_use -= q.bytes;
      --admitted;
      ++completed;
    }
    work.clear();
    cv_results.notify_all();
    cv_space.notify_all();
  }

  void unpin(Slot &s) {
    std::lock_guard<std::mutex> lk(mu);
    for (uint64_t t : s.pinned) {
      Node *x = find(t);
      if (x) --x->pins;
    }
    s.pinned.clear();
    forget_old_nodes();
  }

  // -- batch formation (mu held) ----------------------------------------------

  // The work of one admitted request: a base whose state will be complete
  // when this launch reads it, or the full pipeline.
  void plan_work(const Req &q, int slot_idx, std::vector<Work> &batch, std::unordered_map<uint64_t, size_t> &in_batch) {
    Work w;
    w.req = q;
    Node *x = find(q.ticket);
    auto inst = instances.find(q.ticket);
    if (x && x->depth > 0) {
      // walk up, composing the changes, to a usable base
      std::vector<int32_t> delta = x->delta;
      uint64_t cur = x->parent;
      for (int d = 0; d < kChainDepth && (int)delta.size() <= kMaxDelta; ++d) {
        Node *c = find(cur);
        if (!c) break;
        bool usable = false;
        int wait = -1;
        if (c->complete && c->slot >= 0 && c->in_flight < 0) {
          usable = true;
        } else if (c->slot >= 0 && c->in_flight == slot_idx) {
          // a root earlier in this launch: the full pipeline runs before the children
          auto b = in_batch.find(cur);
          usable = b != in_batch.end() && batch[b->second].full;
        } else if (c->slot >= 0 && c->in_flight >= 0 && c->in_flight != slot_idx && c->guaranteed) {
          usable = true;
          wait = c->in_flight;
        }
        if (usable) {
          w.full = false;
          w.base = cur;
          w.wait_slot = wait;
          // cancel an item added and removed along the way
          std::unordered_map<int32_t, int64_t> net;
          for (int32_t v : delta) net[v > 0 ? v - 1 : -v - 1] += v > 0 ? 1 : -1;
          w.delta.clear();
          for (auto &kv : net) {
            for (int64_t k = 0; k < kv.second; ++k) w.delta.push_back(add_item(kv.first));
            for (int64_t k = 0; k > kv.second; --k) w.delta.push_back(rem_item(kv.first));
          }
          ++c->pins;
          slots[slot_idx].pinned.push_back(cur);
          touch(*c);
          break;
        }
        if (c->depth == 0 && c->parent == 0) break;  // a root without a usable state
        delta.insert(delta.begin(), c->delta.begin(), c->delta.end());
        cur = c->parent;
      }
    }
    if (w.full) {
      w.early = !(q.flags & BP_NO_EARLY_EXIT);
      if (inst != instances.end()) {
        w.residual = std::move(inst->second.first);
        w.unpacked = std::move(inst->second.second);
      } else {
        std::vector<int32_t> load;
        if (x && instance_of(x, &load, &w.unpacked)) {
          w.residual.resize(load.size());
          for (size_t j = 0; j < load.size(); ++j) w.residual[j] = x->C - load[j];
        } else {
          w.err = BP_ERR_STATE;  // neither a base state nor an instance to rebuild
        }
      }
    }
    if (inst != instances.end()) instances.erase(inst);
    // the request's own node state
    if (x && w.err == BP_OK) {
      x->slot = alloc_state(x->C);
      x->in_flight = slot_idx;
      x->guaranteed = x->slot >= 0 && !(w.full && w.early);
      x->complete = false;
    } else if (x) {
      x->in_flight = slot_idx;
    }
    in_batch[q.ticket] = batch.size();
    batch.push_back(std::move(w));
  }

  // -- launch -----------------------------------------------------------------

  bool busy_any() const {
    for (const Slot &s : slots)
      if (s.busy) return true;
    return false;
  }

  bp_status launch(int slot_idx) {
    Slot &s = slots[slot_idx];
    Ctx &c = s.ctx;
    std::vector<Work> &work = s.work;
    // full pipeline first (records [0, nfull)), then the children, then the
    // requests that cannot run (their records are set on the host)
    std::stable_partition(work.begin(), work.end(), [](const Work &w) { return w.err == BP_OK; });
    std::stable_partition(work.begin(), work.end(), [](const Work &w) { return w.err == BP_OK && w.full; });
    size_t nfull = 0, nrun = 0;
    while (nfull < work.size() && work[nfull].err == BP_OK && work[nfull].full) ++nfull;
    while (nrun < work.size() && work[nrun].err == BP_OK) ++nrun;
    const size_t total = std::max<size_t>(nrun, 1);
    bp_status st;
    if ((st = c.wait_staging())) return st;
    if ((st = c.reserve_dev(s.out_dev, sizeof(bp_bounds) * total))) return st;
    if ((st = s.out_host.reserve(sizeof(bp_bounds) * total))) return st;
    bp_bounds *out_dev = (bp_bounds *)s.out_dev.p;
    if (nfull) {
      std::vector<PlanIn> pin(nfull);
      int64_t tot = 0;
      for (size_t i = 0; i < nfull; ++i) {
        const Work &w = work[i];
        Node *x;
        {
          std::lock_guard<std::mutex> lk(mu);
          x = find(w.req.ticket);
        }
        if (!x) return fail(BP_ERR_STATE, "node record lost");
        const int32_t C = x->C;
        const bool keep = x->slot >= 0;
        if ((st = make_plan_in(C, (int64_t)w.residual.size(), (int64_t)w.unpacked.size(), (int32_t)w.residual.size(),
                               kFormResidual, nullptr, w.early, &pin[i], (w.req.flags & BP_SEGMENTS) != 0)))
          return st;
        pin[i].state_off = keep ? x->slot : -1;
        pin[i].in_off = tot;
        tot += pin[i].n_in;
        pin[i].res_off = tot;
        tot += pin[i].m_res;
      }
      int64_t ntasks = 0;
      if ((st = c.plan(pin, &ntasks))) return st;
      if ((st = c.in_host.reserve(sizeof(int32_t) * (size_t)std::max<int64_t>(tot, 1)))) return st;
      int32_t *h = (int32_t *)c.in_host.p;
      for (size_t i = 0; i < nfull; ++i) {
        if (pin[i].n_in) memcpy(h + pin[i].in_off, work[i].unpacked.data(), sizeof(int32_t) * (size_t)pin[i].n_in);
        if (pin[i].m_res) memcpy(h + pin[i].res_off, work[i].residual.data(), sizeof(int32_t) * (size_t)pin[i].m_res);
      }
      if ((st = c.run((int64_t)nfull, ntasks, h, tot, nullptr, nullptr, out_dev, c.stream))) return st;
    }
    if (nrun > nfull) {
      const size_t nch = nrun - nfull;
      std::vector<NodeTask> tasks(nch);
      std::vector<int32_t> delta;
      int64_t tiles = 0;
      std::vector<int> waits;
      {
        std::lock_guard<std::mutex> lk(mu);
        for (size_t i = 0; i < nch; ++i) {
          const Work &w = work[nfull + i];
          const Node *x = find(w.req.ticket);
          const Node *b = find(w.base);
          if (!x || !b) return fail(BP_ERR_STATE, "node record lost");
          NodeTask &t = tasks[i];
          memset(&t, 0, sizeof t);
          t.base_off = b->slot;
          t.dst_off = x->slot;
          t.tile_begin = tiles;
          tiles += node_tiles(x->C);
          t.sumW = x->sumW;
          t.r = x->r;
          t.k = x->m;
          t.C = x->C;
          t.nbig = x->nbig;
          t.d_off = (int32_t)delta.size();
          t.nd = (int32_t)w.delta.size();
          t.out_idx = (int32_t)(nfull + i);
          delta.insert(delta.end(), w.delta.begin(), w.delta.end());
          if (w.wait_slot >= 0 && std::find(waits.begin(), waits.end(), w.wait_slot) == waits.end())
            waits.push_back(w.wait_slot);
        }
      }
      const size_t off_delta = (sizeof(NodeTask) * nch + 255) & ~size_t(255);
      const size_t off_keys = off_delta + ((sizeof(int32_t) * std::max<size_t>(delta.size(), 1) + 255) & ~size_t(255));
      const size_t bytes = off_keys + sizeof(unsigned long long) * kNB * nch;
      if ((st = s.node_host.reserve(off_keys))) return st;
      if ((st = c.reserve_dev(s.node_dev, bytes))) return st;
      char *h = (char *)s.node_host.p;
      memcpy(h, tasks.data(), sizeof(NodeTask) * nch);
      if (!delta.empty()) memcpy(h + off_delta, delta.data(), sizeof(int32_t) * delta.size());
      char *dv = (char *)s.node_dev.p;
      // bases in batches running on other contexts are complete when those end
      for (int ws : waits) QTRY(hipStreamWaitEvent(c.stream, slots[ws].ctx.done, 0));
      if (c.any_run) QTRY(hipStreamWaitEvent(c.stream, c.last_run, 0));
      QTRY(hipMemcpyAsync(dv, h, off_keys, hipMemcpyHostToDevice, c.stream));
      QTRY(launch_node_delta((const NodeTask *)dv, (int64_t)nch, tiles, (const int32_t *)(dv + off_delta), arena,
                             (unsigned long long *)(dv + off_keys), out_dev, c.num_cu * 8, c.stream));
    }
    if (nrun) QTRY(hipMemcpyAsync(s.out_host.p, out_dev, sizeof(bp_bounds) * nrun, hipMemcpyDeviceToHost, c.stream));
    QTRY(hipEventRecord(c.done, c.stream));
    return BP_OK;
  }

  void loop() {
    (void)hipSetDevice(device);
    for (;;) {
      // 1. finished batches
      for (int si = 0; si < kQueueSlots; ++si) {
        Slot &s = slots[si];
        if (!s.busy) continue;
        if (hipEventQuery(s.ctx.done) == hipErrorNotReady) continue;
        const hipError_t e = hipEventSynchronize(s.ctx.done);
        const double t = now_us();
        {
          std::lock_guard<std::mutex> lk(mu);
          busy_us += t - s.start_us;
        }
        publish(s.work, (const bp_bounds *)s.out_host.p, e == hipSuccess ? BP_OK : hip_fail(e, "served batch"),
                s.start_us, si);
        unpin(s);
        s.busy = false;
      }
      // 2. launch what is waiting on an idle context
      int idle = -1;
      for (int si = 0; si < kQueueSlots; ++si)
        if (!slots[si].busy) {
          idle = si;
          break;
        }
      bool stop = false, took = false;
      // (with a batch running and nothing to take, the lock is left to the
      // submitters)
      if (!busy_any() || (idle >= 0 && npending.load(std::memory_order_acquire) > 0)) {
        std::unique_lock<std::mutex> lk(mu);
        if (idle >= 0 && !pending.empty() && !shutdown) {
          std::vector<Work> &batch = slots[idle].work;
          batch.clear();
          std::unordered_map<uint64_t, size_t> in_batch;
          while (!pending.empty() && (int)batch.size() < kMaxBatch) {
            plan_work(pending.front(), idle, batch, in_batch);
            pending.pop_front();
            npending.fetch_sub(1, std::memory_order_relaxed);
          }
          took = !batch.empty();
        }
        const bool any_busy = busy_any();
        if (!took) {
          if (shutdown && !any_busy) stop = true;
          else if (!any_busy) cv_work.wait_for(lk, std::chrono::milliseconds(5));
        }
      }
      if (stop) break;
      if (took) {
        Slot &s = slots[idle];
        ++batches;
        bp_status st;
        if (fail_launch_at > 0 && (long)batches == fail_launch_at) st = fail(BP_ERR_DEVICE, "injected launch failure");
        else st = launch(idle);
        s.start_us = now_us();
        if (st) {
          publish(s.work, nullptr, st, s.start_us, idle);
          unpin(s);
        } else {
          s.busy = true;
        }
        continue;
      }
      // a batch is running: poll its end event again (a timed wait of a few
      // microseconds would sleep for the scheduler's timer slack, tens of
      // microseconds, and every served request would wait it out)
      if (busy_any()) std::this_thread::yield();
    }
    // shut down: what never started completes with BP_ERR_STATE
    std::vector<Work> rest;
    {
      std::lock_guard<std::mutex> lk(mu);
      while (!pending.empty()) {
        Work w;
        w.req = pending.front();
        rest.push_back(std::move(w));
        pending.pop_front();
        npending.fetch_sub(1, std::memory_order_relaxed);
      }
    }
    if (!rest.empty()) publish(rest, nullptr, BP_ERR_STATE, now_us(), -2);
  }
};

bp_status get_queue(bp_queue *q, Queue **out) {
  Queue *x = (Queue *)q;
  if (!x || x->magic != kQueueMagic) return fail(BP_ERR_STATE, "bad queue");
  *out = x;
  return BP_OK;
}

void destroy_slots(Queue *q) {
  for (Slot &s : q->slots) {
    s.node_dev.release();
    s.out_dev.release();
    s.node_host.release();
    s.out_host.release();
    s.ctx.destroy();
  }
  if (q->arena) (void)hipFree(q->arena);
  q->arena = nullptr;
}

}  // namespace

bp_status bp_queue_create(bp_ctx *ctx, size_t hbm_budget_bytes, int32_t max_slots, bp_queue **out) {
  if (!out) return fail(BP_ERR_ARG, "out is NULL");
  *out = nullptr;
  Ctx *c = (Ctx *)ctx;
  if (!c || c->magic != kCtxMagic) return fail(BP_ERR_STATE, "bad context");
  if (hbm_budget_bytes < (size_t(1) << 20) || max_slots < 1)
    return fail(BP_ERR_ARG, "budget must be at least 1 MiB and max_slots positive");
  Queue *q = new (std::nothrow) Queue();
  if (!q) return fail(BP_ERR_NOMEM, "queue allocation");
  q->device = c->device;
  q->budget = hbm_budget_bytes;
  q->allowance = hbm_budget_bytes / 4;
  q->max_slots = max_slots;
  const char *fl = getenv("BP_TEST_FAIL_LAUNCH");
  if (fl) q->fail_launch_at = atol(fl);
  hipError_t e = hipSetDevice(c->device);
  const size_t arena_bytes = (hbm_budget_bytes - q->allowance) & ~size_t(255);
  if (e == hipSuccess) e = hipMalloc(&q->arena, arena_bytes);
  if (e != hipSuccess) {
    delete q;
    return fail(BP_ERR_NOMEM, "node-state arena of %zu bytes: %s", arena_bytes, hipGetErrorString(e));
  }
  q->arena_elems = arena_bytes / sizeof(long long);
  for (Slot &s : q->slots) {
    bp_status st = s.ctx.init(c->device);
    if (st) {
      destroy_slots(q);
      delete q;
      return st;
    }
    s.ctx.magic = kCtxMagic;
    s.ctx.nodes = q->arena;
    // a full batch's records and child tasks (with a few changed items each)
    // from the start: a burst that fills a batch then grows no buffer (a
    // growth waits for the context's launches and frees memory mid-stream)
    const size_t nodes = (sizeof(NodeTask) * kMaxBatch + 255) & ~size_t(255);
    const size_t deltas = (sizeof(int32_t) * 16 * kMaxBatch + 255) & ~size_t(255);
    const size_t keys = sizeof(unsigned long long) * kNB * kMaxBatch;
    if (!st) st = s.ctx.reserve_dev(s.out_dev, sizeof(bp_bounds) * kMaxBatch);
    if (!st) st = s.out_host.reserve(sizeof(bp_bounds) * kMaxBatch);
    if (!st) st = s.node_host.reserve(nodes + deltas);
    if (!st) st = s.ctx.reserve_dev(s.node_dev, nodes + deltas + keys);
    if (st) {
      destroy_slots(q);
      delete q;
      return st;
    }
  }
  q->magic = kQueueMagic;
  try {
    q->thr = std::thread([q] { q->loop(); });
  } catch (...) {
    destroy_slots(q);
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
  if (req->flags & ~(BP_NO_EARLY_EXIT | BP_SEGMENTS)) return fail(BP_ERR_ARG, "unknown flags");
  const bool child = req->parent != 0;
  const bool has_inst = !child || req->residual || req->unpacked;
  if (req->C < 1 || req->m < 0 || (has_inst && req->n < 0)) return fail(BP_ERR_ARG, "bad request sizes");
  if (has_inst && ((req->m > 0 && !req->residual) || (req->n > 0 && !req->unpacked)))
    return fail(BP_ERR_ARG, "NULL request array");
  if (child && (req->ncommit < 0 || req->ncommit > BP_MAX_COMMIT || (req->ncommit > 0 && !req->commits)))
    return fail(BP_ERR_ARG, "bad commit list");
  if (has_inst) {
    if (!instance_fits(req->C, req->n + req->m))
      return fail(BP_ERR_LIMIT, "request of %lld items at c = %d", (long long)(req->n + req->m), req->C);
    if ((st = host_validate_items(req->C, req->unpacked, req->n))) return st;
    if ((st = host_validate_items(req->C, req->residual, req->m))) return st;
  }
  Node node;
  node.C = req->C;
  node.m = req->m;
  std::vector<int32_t> residual, unpacked;
  if (has_inst) {
    residual.assign(req->residual, req->residual + req->m);
    unpacked.assign(req->unpacked, req->unpacked + req->n);
  }
  Req r;
  r.tag = req->tag;
  r.flags = req->flags;
  std::unique_lock<std::mutex> lk(q->mu);
  if (child) {
    Node *p = q->find(req->parent);
    if (!p) {
      if (!has_inst) return fail(BP_ERR_STATE, "parent ticket %llu is not known to the queue", (unsigned long long)req->parent);
    } else {
      if (p->C != req->C || p->m != req->m) return fail(BP_ERR_ARG, "a child's C and m must be its parent's");
      node.parent = req->parent;
      node.depth = p->depth + 1;
      node.r = p->r;
      node.sumW = p->sumW;
      node.nbig = p->nbig;
      node.n_unp = p->n_unp - req->ncommit;
      if (node.n_unp < 0) return fail(BP_ERR_RANGE, "more commits than unpacked items");
      for (int32_t i = 0; i < req->ncommit; ++i) {
        const int32_t w = req->commits[i].size, j = req->commits[i].bin;
        if (w < 0 || w > req->C || j < 0 || j >= req->m)
          return fail(BP_ERR_RANGE, "commit %d: size %d or bin %d out of range", i, w, j);
        int32_t old = -1;
        bool found = false;
        for (auto it = node.changed.rbegin(); it != node.changed.rend(); ++it)
          if (it->first == j) {
            old = it->second;
            found = true;
            break;
          }
        if (!found && !q->load_of(p, j, &old))
          return fail(BP_ERR_STATE, "the load of bin %d at ticket %llu is no longer known", j,
                      (unsigned long long)req->parent);
        if ((int64_t)old + w > req->C) return fail(BP_ERR_RANGE, "commit %d overfills bin %d", i, j);
        // the item leaves the unpacked items; the bin's virtual item goes from old to old + w
        node.delta.push_back(rem_item(w));
        if (old > 0) node.delta.push_back(rem_item(old));
        if (old + w > 0) node.delta.push_back(add_item(old + w));
        node.r += -1 - (old > 0 ? 1 : 0) + (old + w > 0 ? 1 : 0);
        node.sumW += -(int64_t)w - old + (old + w);
        node.nbig += -(2ll * w > req->C) - (2ll * old > req->C) + (2ll * (old + w) > req->C);
        node.changed.push_back({j, old + w});
        node.committed.push_back(w);
      }
      if (node.depth >= kFlattenEvery) {
        // keep full loads and sizes here, so that chains stay short
        std::vector<int32_t> load, unp;
        if (q->instance_of(p, &load, &unp)) {
          for (auto &cb : node.changed) load[(size_t)cb.first] = cb.second;
          std::unordered_map<int32_t, int64_t> cnt;
          for (int32_t w : node.committed) ++cnt[w];
          std::vector<int32_t> keep;
          keep.reserve(unp.size());
          for (int32_t w : unp) {
            auto it = cnt.find(w);
            if (it != cnt.end() && it->second > 0) { --it->second; continue; }
            keep.push_back(w);
          }
          node.load = std::move(load);
          node.unpacked = std::move(keep);
          node.depth = 0;
        }
      }
    }
  }
  if (node.parent == 0) {
    // a root, or a child with its own instance whose parent is gone
    node.depth = 0;
    node.load.resize((size_t)req->m);
    node.r = req->n;
    node.sumW = 0;
    node.nbig = 0;
    for (int64_t i = 0; i < req->n; ++i) {
      node.sumW += unpacked[(size_t)i];
      node.nbig += 2ll * unpacked[(size_t)i] > req->C;
    }
    for (int32_t j = 0; j < req->m; ++j) {
      const int32_t ld = req->C - residual[(size_t)j];
      node.load[(size_t)j] = ld;
      node.r += ld > 0;
      node.sumW += ld;
      node.nbig += 2ll * ld > req->C;
    }
    node.unpacked = unpacked;
    node.n_unp = req->n;
  }
  r.bytes = node.parent == 0 || has_inst ? full_bytes(req->n, req->m, req->C) : child_bytes(req->ncommit);
  if (r.bytes > q->allowance) return fail(BP_ERR_LIMIT, "request needs %zu bytes > allowance %zu", r.bytes, q->allowance);
  for (;;) {
    if (q->shutdown) return fail(BP_ERR_STATE, "queue is shutting down");
    if (q->bytes_in_use + r.bytes <= q->allowance && q->admitted < q->max_slots) break;
    if (!blocking) {
      ++q->rejected;
      return fail(BP_ERR_AGAIN, "no free slot or budget");
    }
    q->cv_space.wait(lk);
  }
  r.ticket = q->next_ticket++;
  r.submit_us = now_us();
  node.ticket = r.ticket;
  q->bytes_in_use += r.bytes;
  if (q->bytes_in_use > q->bytes_peak) q->bytes_peak = q->bytes_in_use;
  ++q->admitted;
  ++q->submitted;
  *ticket = r.ticket;
  if (has_inst) q->instances[r.ticket] = {std::move(residual), std::move(unpacked)};
  q->nodes[r.ticket] = std::move(node);
  q->history.push_back(r.ticket);
  q->forget_old_nodes();
  q->pending.push_back(r);
  q->npending.fetch_add(1, std::memory_order_release);
  q->cv_work.notify_one();
  return BP_OK;
}

bp_status bp_queue_replay(bp_queue *qh, bp_request *reqs, const double *arrival_s, const int64_t *parent_index,
                          int64_t n, uint64_t *tickets, int32_t *status, double *lateness_s) {
  Queue *q;
  bp_status st = get_queue(qh, &q);
  if (st) return st;
  if (n < 0 || (n > 0 && (!reqs || !arrival_s || !parent_index || !tickets || !status)))
    return fail(BP_ERR_ARG, "bad replay arguments");
  const double t0 = now_us();
  double late = 0;
  for (int64_t i = 0; i < n; ++i) {
    tickets[i] = 0;
    const int64_t p = parent_index[i];
    if (p >= i) return fail(BP_ERR_ARG, "request %lld names a later parent", (long long)i);
    if (p >= 0) {
      if (tickets[p] == 0) {
        status[i] = BP_ERR_STATE;
        continue;
      }
      reqs[i].parent = tickets[p];
    }
    const double due = t0 + arrival_s[i] * 1e6;
    double now = now_us();
    while (now < due) now = now_us();
    late = std::max(late, now - due);
    status[i] = bp_queue_submit(qh, &reqs[i], 0, &tickets[i]);
    if (status[i] != BP_OK) tickets[i] = 0;
  }
  if (lateness_s) *lateness_s = late * 1e-6;
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
  memset(out, 0, sizeof *out);
  out->submitted = q->submitted;
  out->completed = q->completed;
  out->rejected = q->rejected;
  out->batches = q->batches;
  out->in_flight = (uint64_t)q->admitted;
  out->bytes_in_use = q->bytes_in_use;
  out->bytes_peak = q->bytes_peak;
  out->budget = q->budget;
  out->busy_us = q->busy_us;
  out->from_parent = q->n_delta;
  out->full_sweeps = q->n_full;
  out->nodes_kept = q->kept;
  out->node_evictions = q->evictions;
  out->node_bytes = q->arena_elems * sizeof(long long);
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
  destroy_slots(q);
  delete q;
  return BP_OK;
}
