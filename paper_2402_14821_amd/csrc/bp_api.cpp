// bp_api.cpp -- host side of libbp: validation, planning, workspaces, the
// captured pipeline graph and the C ABI declared in include/bp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "bp_ctx.h"
#include "bp_divide.h"
#include "bp_internal.h"

using namespace bpi;

namespace bpi {

static thread_local std::string g_err;

bp_status fail(bp_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

bp_status hip_fail(hipError_t e, const char *what) {
  return fail(BP_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call)                                     \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return hip_fail(e_, #call);     \
  } while (0)

// Paper's parameter ranges (Sec. 3.1) for integer parameters.
void default_ranges(int32_t C, int64_t lo[kNB], int64_t hi[kNB]) {
  const int64_t c = C;
  lo[kL1] = 0; hi[kL1] = -1;
  lo[kL2] = 0; hi[kL2] = c / 2;
  lo[kMT] = 0; hi[kMT] = c / 2;
  lo[kRAD2] = c / 4 + 1; hi[kRAD2] = c / 3;
  lo[kFS1] = 1; hi[kFS1] = 100;
  lo[kCCM1] = 1; hi[kCCM1] = c / 2;
  lo[kVB2] = 2; hi[kVB2] = c;
  lo[kBJ1] = 1; hi[kBJ1] = c;
}

bp_status DevBuf::reserve(size_t bytes) {
  if (bytes <= cap) return BP_OK;
  size_t want = std::max(bytes, cap + cap / 2);
  want = (want + 4095) & ~size_t(4095);
  if (p) {
    hipError_t e = hipFree(p);
    p = nullptr;
    cap = 0;
    if (e != hipSuccess) return hip_fail(e, "hipFree");
  }
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    p = nullptr;
    return fail(BP_ERR_NOMEM, "hipMalloc(%zu): %s", want, hipGetErrorString(e));
  }
  cap = want;
  return BP_OK;
}

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  cap = 0;
}

bp_status HostBuf::reserve(size_t bytes) {
  if (bytes <= cap) return BP_OK;
  size_t want = std::max(bytes, cap + cap / 2);
  want = (want + 4095) & ~size_t(4095);
  if (p) {
    (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
  }
  hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
  if (e != hipSuccess) {
    p = nullptr;
    return fail(BP_ERR_NOMEM, "hipHostMalloc(%zu): %s", want, hipGetErrorString(e));
  }
  cap = want;
  return BP_OK;
}

void HostBuf::release() {
  if (p) (void)hipHostFree(p);
  p = nullptr;
  cap = 0;
}

// Relative cost of one (item, parameter) evaluation per bound, in issue
// slots of a full-rate VALU instruction (measured rates on gfx950: 32-bit
// add/sub/logic/shift-right issue at twice the rate of multiplies, compares,
// selects and fp64 operations).
static double unit_cost(int b) {
  switch (b) {
    case kMT: return 2.5;
    case kRAD2: return 3.0;
    case kFS1: return 9.0;
    case kCCM1: return 2.0;
    case kVB2: return 2.5;
    case kBJ1: return 4.0;
    default: return 1.0;
  }
}

static int ilog2ceil(int64_t x) {
  int l = 0;
  while ((1ll << l) < x) ++l;
  return l;
}

// Divisors of c in ascending order, by trial division up to sqrt(c), and
// c's prime factorisation with each divisor's place in the lattice of
// exponent vectors (cached per context: a batch or a served stream has few
// distinct capacities).
static const Ctx::DivInfo &divisors_of(Ctx *c, int32_t C) {
  auto it = c->div_cache.find(C);
  if (it != c->div_cache.end()) return it->second;
  if (c->div_cache.size() > 4096) c->div_cache.clear();
  Ctx::DivInfo info;
  std::vector<int32_t> hi;
  for (int64_t i = 1; i * i <= (int64_t)C; ++i) {
    if (C % i) continue;
    info.divs.push_back((int32_t)i);
    if (i * i != (int64_t)C) hi.push_back((int32_t)(C / i));
  }
  info.divs.insert(info.divs.end(), hi.rbegin(), hi.rend());
  std::vector<int64_t> pr;
  std::vector<int32_t> ex;
  int64_t x = C;
  for (int64_t q = 2; q * q <= x; ++q) {
    if (x % q) continue;
    int32_t a = 0;
    while (x % q == 0) {
      x /= q;
      ++a;
    }
    pr.push_back(q);
    ex.push_back(a);
  }
  if (x > 1) {
    pr.push_back(x);
    ex.push_back(1);
  }
  for (int32_t d : info.divs) {
    int64_t bin = 0, stride = 1, y = d;
    for (size_t j = 0; j < pr.size(); ++j) {
      int32_t e = 0;
      while (y % pr[j] == 0) {
        y /= pr[j];
        ++e;
      }
      bin += e * stride;
      stride *= ex[j] + 1;
    }
    info.lattice.push_back((int32_t)bin);
  }
  info.lattice.push_back((int32_t)pr.size());
  for (size_t j = 0; j < pr.size(); ++j) {
    info.lattice.push_back((int32_t)pr[j]);
    info.lattice.push_back(ex[j]);
  }
  // the divisibility-test constants of p_j^e, e = 1..a_j, prime by prime (at
  // most 30 prime powers below 2^31), as (low, high) 32-bit halves
  std::vector<uint64_t> pm;
  for (size_t j = 0; j < pr.size(); ++j) {
    uint64_t q = 1;
    for (int32_t e = 1; e <= ex[j]; ++e) {
      q *= (uint64_t)pr[j];
      pm.push_back(divides_const((uint32_t)q));
    }
  }
  info.lattice.push_back((int32_t)pm.size());
  for (uint64_t m : pm) {
    info.lattice.push_back((int32_t)(uint32_t)m);
    info.lattice.push_back((int32_t)(uint32_t)(m >> 32));
  }
  return c->div_cache.emplace(C, std::move(info)).first->second;
}

// Checks a caller range against the paper's range of that bound.
static bp_status check_sweep(int32_t C, const bp_sweep *sw, int64_t lo[kNB], int64_t hi[kNB]) {
  int64_t dlo[kNB], dhi[kNB];
  default_ranges(C, dlo, dhi);
  for (int b = 0; b < kNB; ++b) {
    if (!sw) {
      lo[b] = dlo[b];
      hi[b] = dhi[b];
      continue;
    }
    lo[b] = sw->lo[b];
    hi[b] = sw->hi[b];
    if (b == kL1) continue;
    if (lo[b] > hi[b]) continue;  // empty by request
    if (lo[b] < dlo[b] || hi[b] > dhi[b])
      return fail(BP_ERR_RANGE, "sweep range of bound %d [%lld, %lld] outside [%lld, %lld] for C=%d", b,
                  (long long)lo[b], (long long)hi[b], (long long)dlo[b], (long long)dhi[b], C);
  }
  if (sw && (sw->flags & ~(BP_SWEEP_PAPER_VB2_CLAMP | BP_SWEEP_SEGMENTS)))
    return fail(BP_ERR_ARG, "unknown bp_sweep flags 0x%x", sw->flags);
  return BP_OK;
}

// ---------------------------------------------------------------------------

bp_status Ctx::init(int dev) {
  device = dev;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (dev < 0 || dev >= ndev) return fail(BP_ERR_ARG, "device %d not in [0, %d)", dev, ndev);
  HIP_TRY(hipSetDevice(dev));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  num_cu = prop.multiProcessorCount;
  HIP_TRY(set_kernel_attrs());
  HIP_TRY(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
  // The stage-timing events only measure time: they skip the system-scope
  // fence (an L2 writeback and invalidation at each record).  The ordering
  // events keep it.
  HIP_TRY(hipEventCreateWithFlags(&staged, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&done, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&last_run, hipEventDisableTiming));
  for (auto &set : tev)
    for (hipEvent_t &e : set) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  bp_status st = counter_buf.reserve(sizeof(unsigned long long) * kQueues * kQueueStride);
  if (st) return st;
  apply_tuning();
  grid_prep_small = num_cu * 2;
  grid_prep_large = std::max(1, num_cu / 4);
  grid_comb = num_cu * 2;
  grid_fin = 64;
  const char *ng = getenv("BP_NO_GRAPH");
  use_graph = !(ng && ng[0] == '1');
  const char *nv = getenv("BP_NO_VALUE_PREP");
  value_prep = !(nv && nv[0] == '1');
  const char *ns = getenv("BP_NO_SMALL_PATH");
  small_path = !(ns && ns[0] == '1');
  if (const char *sw = getenv("BP_SMALL_PATH_WORK")) {
    const long long v = atoll(sw);
    if (v > 0) small_work = v;
  }
  small_grid = std::min(num_cu, kSmallFusedMaxGrid);
  if (const char *sg = getenv("BP_SMALL_GRID")) {
    const int v = atoi(sg);
    if (v > 0 && v <= kSmallFusedMaxGrid) small_grid = v;
  }
  if (const char *sv = getenv("BP_SMALL_WAVES")) {
    const int v = atoi(sv);
    if (v > 0 && v <= 16) small_waves = v;
  }
  if (const char *si = getenv("BP_SMALL_ITEMS")) {
    const int v = atoi(si);
    if (v > 0 && v <= 1024) small_items = v;
  }
  {
    const hipError_t e = hipHostMalloc(&small_out, sizeof(bp_bounds) + 64, hipHostMallocCoherent);
    if (e != hipSuccess) {
      small_out = nullptr;
      return fail(BP_ERR_NOMEM, "hipHostMalloc (coherent, %zu): %s", sizeof(bp_bounds) + 64, hipGetErrorString(e));
    }
    memset(small_out, 0, sizeof(bp_bounds) + 64);
  }
  if ((st = small_keys.reserve(kSmallBufBytes))) return st;
  HIP_TRY(hipMemset(small_keys.p, 0, kSmallBufBytes));  // the one-kernel keys and count start at zero
  // BP_SEGMENT_KCUT=K: segment tiles of BJ1 wherever floor(c / lambda) <= K
  // (0 .. 64) instead of where the cost model puts the cut; same results.
  const char *kc = getenv("BP_SEGMENT_KCUT");
  if (kc && kc[0]) seg_kcut = std::min(std::max(atoi(kc), 0), (int)kSegMaxK);
  if (const char *lk = getenv("BP_LUT_KCUT")) lut_kcut = std::max<long long>(atoll(lk), 0);
  if (const char *lq = getenv("BP_LUT_QCHUNK")) lut_qchunk = std::min(std::max(atoi(lq), 1), 1 << 20);
  return BP_OK;
}

void Ctx::destroy() {
  if (device >= 0) (void)hipSetDevice(device);
  if (stream) (void)hipStreamSynchronize(stream);
  if (last_run && any_run) (void)hipEventSynchronize(last_run);
  drop_graphs();
  for (DevBuf *b : {&stage_buf, &counter_buf, &state_buf, &sorted_buf, &pre_buf, &rec_buf, &keys_buf, &ref_buf,
                    &acc_buf, &out_buf, &red_buf, &bidx_buf, &dcnt_buf, &small_keys, &vraw_buf, &vcnt_buf, &vsum_buf,
                    &vtot_buf, &vlat_buf, &vflag_buf})
    b->release();
  for (HostBuf *b : {&stage_host, &in_host, &out_host, &red_host}) b->release();
  if (small_out) (void)hipHostFree(small_out);
  small_out = nullptr;
  if (staged) (void)hipEventDestroy(staged);
  if (done) (void)hipEventDestroy(done);
  if (last_run) (void)hipEventDestroy(last_run);
  last_run = nullptr;
  for (auto &set : tev)
    for (hipEvent_t &e : set) {
      if (e) (void)hipEventDestroy(e);
      e = nullptr;
    }
  if (stream) (void)hipStreamDestroy(stream);
  staged = done = nullptr;
  stream = nullptr;
}

void Ctx::apply_tuning() { grid_sweep = num_cu * tune.waves_per_cu; }

// Callers make sure no launch of these graphs is still running
// (wait_last_run: every launch goes through run(), which records last_run).
void Ctx::drop_graphs() {
  for (auto &kv : graphs) {
    if (kv.second.ex) (void)hipGraphExecDestroy(kv.second.ex);
    if (kv.second.g) (void)hipGraphDestroy(kv.second.g);
  }
  graphs.clear();
  graph_used.clear();
}

bp_status Ctx::wait_last_run() {
  if (any_run) HIP_TRY(hipEventSynchronize(last_run));
  return BP_OK;
}

// Grows a device workspace; the old allocation may still be read by the
// previous launch, so that launch is waited for before it is freed.
bp_status Ctx::reserve_dev(DevBuf &b, size_t bytes) {
  if (bytes <= b.cap) return BP_OK;
  bp_status st = wait_last_run();
  if (st) return st;
  return b.reserve(bytes);
}

static int pow2_at_least(int64_t x) {
  int p = 1;
  while (p < x && p < (1 << 30)) p <<= 1;
  return p;
}

// Kernels and grids of a launch of `count` instances and `ntasks` sweep
// tasks: each grid is the work it has, rounded up to a power of two (few
// distinct graphs), and at most the machine-filling size.  The persistent
// sweep serves its task queues with any grid; a small launch so avoids
// dispatching thousands of waves that would find no task.
Ctx::LaunchShape Ctx::shape_of(int64_t count, int64_t ntasks) const {
  bool with_large = false, tiny = true;
  for (int64_t i = 0; i < count; ++i) {
    with_large |= plan_vec[i].large == 1;
    tiny &= plan_vec[i].large != 0 || plan_vec[i].r_cap <= kTinyCap;
  }
  LaunchShape sh;
  sh.v = (with_large ? 1 : 0) | (nsplit > 0 ? 2 : 0) | (tiny ? 4 : 0);
  sh.lpl = tune.lanes_params;
  // (the small-instance prep kernel also counts the sizes of value-table instances)
  sh.prep_small = std::min(grid_prep_small, pow2_at_least(std::max<int64_t>(count, vt_list.empty() ? 1 : 64)));
  sh.prep_large = std::min(grid_prep_large, pow2_at_least(std::max<int64_t>(count, 1)));
  sh.vt = vt_list.empty() ? 0 : std::max(1, num_cu);
  sh.sweep = std::min(grid_sweep, std::max(64, pow2_at_least(ntasks)));
  sh.comb = std::min(grid_comb, pow2_at_least(std::max<int64_t>(nsplit, 1)));
  // the value tables' counts are cleared by the finalize grid
  sh.fin = std::min(grid_fin, std::max(vt_list.empty() ? 1 : 16, pow2_at_least((count + 255) / 256)));
  return sh;
}

// Captures the pipeline of one launch shape once; every call with that shape
// replays it.  At most 32 shapes are kept: past that the least recently used
// graph is destroyed, once the launch before this one has finished.
bp_status Ctx::ensure_graph(const LaunchDesc *d_desc, const LaunchShape &sh, hipGraphExec_t *out) {
  auto it = graphs.find(sh);
  if (it != graphs.end()) {
    graph_used[sh] = run_count;
    *out = it->second.ex;
    return BP_OK;
  }
  if (graphs.size() >= 32) {
    bp_status st = wait_last_run();
    if (st) return st;
    auto lru = graph_used.begin();
    for (auto u = graph_used.begin(); u != graph_used.end(); ++u)
      if (u->second < lru->second) lru = u;
    auto g = graphs.find(lru->first);
    if (g->second.ex) (void)hipGraphExecDestroy(g->second.ex);
    if (g->second.g) (void)hipGraphDestroy(g->second.g);
    graphs.erase(g);
    graph_used.erase(lru);
  }
  HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
  hipError_t le =
      launch_pipeline(d_desc, sh.lpl, sh.prep_small, sh.prep_large, sh.vt, sh.sweep, sh.comb, sh.fin, sh.v, stream);
  hipGraph_t g = nullptr;
  hipError_t ee = hipStreamEndCapture(stream, &g);
  if (le != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(le, "capture launch_pipeline");
  }
  if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
  hipGraphExec_t ex = nullptr;
  hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (ie != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(ie, "hipGraphInstantiate");
  }
  graphs[sh] = GraphPair{g, ex};
  graph_used[sh] = run_count;
  *out = ex;
  return BP_OK;
}

// Staging layout (one pinned block, copied to the device in one transfer):
// [LaunchDesc][InstPlan x count][Entry x nentries][input int32 ...], each part
// aligned to 256 bytes.
static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Build InstPlan + Entry tables into the pinned staging block.
bp_status Ctx::plan(const std::vector<PlanIn> &pin, int64_t *ntasks_out) {
  const int64_t count = (int64_t)pin.size();
  std::vector<InstPlan> &pl = plan_vec;
  pl.assign((size_t)count, InstPlan{});
  int64_t ws = 0, pre = 0, bidx = 0, dcnt = 0, vt = 0, vtt = 0, vl = 0;
  div_vec.clear();
  vt_list.clear();
  std::vector<Entry> ent;
  std::vector<double> tile_cost_v;
  std::vector<int64_t> rcap_v;
  ent.reserve((size_t)count * 7);
  double total = 0;
  const int64_t tile = 64 * (int64_t)tune.lanes_params;
  for (int64_t i = 0; i < count; ++i) {
    const PlanIn &q = pin[i];
    InstPlan &p = pl[i];
    memset(&p, 0, sizeof p);
    p.in_off = q.in_off;
    p.res_off = q.res_off;
    p.n_in = q.n_in;
    p.k = q.k;
    p.m_res = q.m_res;
    p.C = q.C;
    p.form = q.form;
    const int64_t rcap = q.n_in + q.m_res;
    if (!instance_fits(q.C, rcap))
      return fail(BP_ERR_LIMIT,
                  "instance %lld: %lld reduced items; more than %d need c <= %d and c <= %lld x the items",
                  (long long)i, (long long)rcap, kLargeCap, kVtMaxC, (long long)kVtRatio);
    p.r_cap = (int32_t)rcap;
    p.large = rcap > kSmallCap ? 1 : 0;  // (above kLargeCap instance_fits leaves only the value tables)
    // Prepared from value tables by kernels over the whole GPU: a large
    // instance whose c is not much above its item count.  (For a few hundred
    // items the one-block prep and the windowed segment sums are faster than
    // tables of c entries, measured at c = 10^3 .. 10^6.)
    if ((value_prep || rcap > kLargeCap) && p.large && q.C <= kVtMaxC && (int64_t)q.C <= kVtRatio * rcap) {
      p.large = 2;
      p.vt_off = vt;
      vt += (int64_t)q.C + 2;
      p.vtt_off = vtt;
      vtt += 4 * (((int64_t)q.C + 2 + kVtChunk - 1) / kVtChunk);
      vt_list.push_back((int32_t)i);
    }
    p.flags = (q.clamp ? kPlanClampVB2 : 0u) | (q.early_exit ? kPlanEarlyExit : 0u);
    p.state_off = q.state_off;
    if (q.state_off >= 0) {
      // node states hold the paper's full ranges, computed by plain tiles
      int64_t dlo[kNB], dhi[kNB];
      default_ranges(q.C, dlo, dhi);
      for (int b = kL2; b < kNB; ++b)
        if (q.lo[b] != dlo[b] || q.hi[b] != dhi[b] || q.clamp)
          return fail(BP_ERR_ARG, "instance %lld: a node state needs the paper's full ranges", (long long)i);
    }
    p.ws_off = ws;
    p.pre_off = pre;
    ws += std::max<int64_t>(rcap, 1);
    pre += rcap + 1;
    // Threshold table of the segment sums: buckets of width 2^bshift over
    // [0, C + 1], about four sizes per bucket when the sizes spread evenly.
    int64_t bw = 1;
    if (q.segments) {
      int32_t sh = 0;
      while (((int64_t)q.C >> sh) > std::max<int64_t>(rcap / 4, 1)) ++sh;
      p.flags |= kPlanSegments;
      p.bshift = sh;
      p.nbk = (int32_t)((((int64_t)q.C + 1) >> sh) + 2);
      p.bidx_off = bidx;
      bidx += p.nbk;
      bw = 1ll << sh;
    }
    for (int b = 0; b < kNB; ++b) {
      p.lo[b] = q.lo[b];
      p.hi[b] = q.hi[b];
    }
    auto push = [&](Entry e, double tc) {
      total += tc * (double)e.ntiles;
      ent.push_back(e);
      tile_cost_v.push_back(tc);
      rcap_v.push_back(rcap);
    };
    const double dens = (double)std::max<int64_t>(rcap, 1) / (double)q.C;  // sizes per unit of capacity
    for (int b = kL2; b < kNB; ++b) {
      if (q.lo[b] > q.hi[b]) continue;
      Entry e;
      memset(&e, 0, sizeof e);
      e.inst = (int32_t)i;
      e.bound = b;
      e.mode = kModeDense;
      if (b == kL2) {
        const int64_t cand = 2 * rcap + 1;
        e.lam0 = 0;
        e.ntiles = (cand + tile - 1) / tile;
        push(e, (double)tile * (2.0 * (ilog2ceil(rcap + 1) + 1) * 4.0 + 20.0));
        if (q.state_off >= 0) {
          // the L2 aggregates of the node state at every lambda in [0, c/2]
          e.mode = kModeL2State;
          e.ntiles = ((int64_t)q.C / 2 + tile) / tile;
          push(e, (double)tile * (2.0 * (ilog2ceil(rcap + 1) + 1) * 4.0 + 20.0));
        }
        continue;
      }
      const double dense_tc = (double)tile * ((double)rcap * unit_cost(b) + 60.0);
      const int64_t ncand = (b == kMT ? 2 : 4) * rcap + 1;
      if (q.segments && (b == kMT || b == kRAD2) && q.state_off < 0 && ncand < q.hi[b] - q.lo[b] + 1) {
        // fewer change points than parameters: tiles over the candidate
        // indices, each a binary search per threshold (2 for MT, 4 for RAD2)
        e.mode = kModeCand;
        e.lam0 = 0;
        e.ntiles = (ncand + tile - 1) / tile;
        push(e, (double)tile * ((b == kMT ? 2.0 : 4.0) * (ilog2ceil(rcap + 1) + 1) * 4.0 + 20.0));
        continue;
      }
      if (q.segments && b == kRAD2) {
        // four windows per tile (128 or 256 thresholds wide)
        e.mode = kModeSegments;
        e.lam0 = q.lo[b];
        e.ntiles = (q.hi[b] - q.lo[b] + tile) / tile;
        push(e, (double)tile * (4.0 * ((double)(2 * tile + bw) * dens * 1.5 + 30.0)) + 400.0);
        continue;
      }
      if (q.segments && b == kMT) {
        // two windows per tile (small sizes around lambda, big ones around
        // c - lambda), each about (tile + bucket) sizes long
        e.mode = kModeSegments;
        e.lam0 = q.lo[b];
        e.ntiles = (q.hi[b] - q.lo[b] + tile) / tile;
        push(e, (double)tile * (2.0 * ((double)(tile + bw) * dens * 2.0 + 30.0)) + 400.0);
        continue;
      }
      if (q.segments && p.large == 2 && (b == kBJ1 || b == kCCM1)) {
        // Value-table instance: lambda with K = floor(c / lambda) (BJ1) or
        // floor(floor(c/2) / lambda) (CCM1) up to kcut read 2K thresholds
        // from the tables, about lut_q slots per q and parameter (measured on
        // MI355X: table gathers are latency-bound) against r dense
        // evaluations; smaller lambda stay dense.  The lookup range is cut
        // into bands [L, 2L), whose tiles are split into q chunks of
        // kLutQPerChunk, so that no task walks a long chain of loads.
        const double lut_q = b == kBJ1 ? 112.0 : 56.0;
        const int64_t knum = b == kBJ1 ? (int64_t)q.C : (int64_t)q.C / 2;
        const int64_t kcut = lut_kcut >= 0 ? lut_kcut : std::max<int64_t>(1, (int64_t)((double)rcap * unit_cost(b) / lut_q));
        const int64_t lstar = std::max<int64_t>(q.lo[b], knum / (kcut + 1) + 1);
        if (lstar > q.lo[b]) {
          e.lam0 = q.lo[b];
          e.ntiles = (std::min(lstar - 1, q.hi[b]) - q.lo[b] + tile) / tile;
          push(e, dense_tc);
        }
        for (int64_t L = lstar; L <= q.hi[b];) {
          // the band's tiles: whole tiles from L, up to about 2L
          const int64_t nt = std::max<int64_t>(1, (L + tile - 1) / tile);
          const int64_t end = std::min(q.hi[b], L + nt * tile - 1);
          const int64_t kfirst = knum / L;
          e.mode = kModeLookup;
          e.lam0 = L;
          e.ntiles = (end - L + tile) / tile;
          e.aux = (int32_t)std::min<int64_t>(64, std::max<int64_t>(1, (kfirst + lut_qchunk - 1) / lut_qchunk));
          push(e, (double)tile * (double)std::max<int64_t>(kfirst, 1) * lut_q + 400.0);
          L = end + 1;
        }
        continue;
      }
      if (q.segments && (b == kBJ1 || b == kCCM1) && (rcap >= kSegWindowMinItems || pin.size() > 1 || seg_kcut >= 0)) {
        // A tile whose smallest parameter is lambda has K = floor(c / lambda)
        // (BJ1) or floor(floor(c/2) / lambda) (CCM1) and 2K windows of about
        // (tile j + bucket) sizes, at about per_size slots per size and
        // parameter; it is cheaper than r dense evaluations while K <= kcut.
        const double per_size = b == kBJ1 ? 1.0 : 1.5;
        const int64_t knum = b == kBJ1 ? (int64_t)q.C : (int64_t)q.C / 2;
        int64_t kcut = 0;
        for (int64_t K = 1; K <= kSegMaxK; ++K) {
          const double seg = 2.0 * (((double)tile * K * K / 2.0 + (double)bw * K) * dens * per_size + 30.0 * K);
          if (seg > (double)rcap * unit_cost(b)) break;
          kcut = K;
        }
        if (seg_kcut >= 0) kcut = seg_kcut;
        const int64_t lstar = kcut > 0 ? knum / (kcut + 1) + 1 : q.hi[b] + 1;  // K(lambda) <= kcut from here
        const int64_t ndense = std::max<int64_t>(0, (std::min(lstar, q.hi[b] + 1) - q.lo[b] + tile - 1) / tile);
        if (ndense > 0) {
          e.lam0 = q.lo[b];
          e.ntiles = ndense;
          push(e, dense_tc);
        }
        const int64_t s0 = q.lo[b] + ndense * tile;
        if (s0 <= q.hi[b]) {
          e.mode = kModeSegments;
          e.lam0 = s0;
          e.ntiles = (q.hi[b] - s0 + tile) / tile;
          const double kmid = std::max(1.0, (double)knum / (0.5 * (double)(s0 + q.hi[b])));
          push(e, (double)tile * (60.0 * kmid + ((double)tile * kmid * kmid + 2.0 * (double)bw * kmid) * dens * per_size) +
                      400.0);
        }
        continue;
      }
      if (q.segments && b == kVB2 && !q.clamp && rcap >= kMirrorMinItems && q.C >= 5) {
        // Mirrored VB2: a dense sum at lambda <= (c - 1)/2 also gives the sum
        // at c - lambda.  N1 = the range's own low parameters, N2 = the
        // mirrors of its high ones; the dense half is their hull.
        const int64_t C = q.C, lo = q.lo[b], hi = q.hi[b];
        const int64_t low_end = (C - 1) / 2, high_start = C - low_end;
        const int64_t a1 = std::max<int64_t>(lo, 1), b1 = std::min(hi, low_end);
        const int64_t a2 = C - std::min(hi, C - 1), b2 = C - std::max(lo, high_start);
        const bool has1 = a1 <= b1, has2 = a2 <= b2;
        const int64_t lm = std::min(has1 ? a1 : a2, has2 ? a2 : a1), mm = std::max(has1 ? b1 : b2, has2 ? b2 : b1);
        const int64_t need = (has1 ? b1 - a1 + 1 : 0) + (has2 ? b2 - a2 + 1 : 0);
        const Ctx::DivInfo &di = divisors_of(this, q.C);
        const std::vector<int32_t> &dv = di.divs;
        if (has1 && has2 && (double)(mm - lm + 1) < 0.75 * (double)need && (int)dv.size() <= kMaxDivs) {
          // the divisors, then the lattice block the prep's multiple counts use
          p.div_off = (int64_t)div_vec.size();
          p.ndiv = (int32_t)dv.size();
          p.dc_off = dcnt;
          div_vec.insert(div_vec.end(), dv.begin(), dv.end());
          div_vec.insert(div_vec.end(), di.lattice.begin(), di.lattice.end());
          dcnt += 2 * (int64_t)dv.size();
          e.mode = kModeMirror;
          e.lam0 = lm;
          e.aux = (int32_t)mm;
          e.ntiles = (mm - lm + tile) / tile;
          push(e, dense_tc);
          // parameters the two halves miss: c/2 (even c) and c
          e.mode = kModeDense;
          e.aux = 0;
          for (int64_t x : {C % 2 == 0 ? C / 2 : (int64_t)-1, C}) {
            if (x < lo || x > hi) continue;
            e.lam0 = x;
            e.ntiles = 1;
            push(e, dense_tc);
          }
          continue;
        }
      }
      const int64_t nl = q.hi[b] - q.lo[b] + 1;
      e.lam0 = q.lo[b];
      e.ntiles = (nl + tile - 1) / tile;
      push(e, dense_tc);
    }
    if (p.large == 2 && p.ndiv > 0) {
      p.vl_off = vl;
      vl += 2 * (int64_t)p.ndiv;
    }
  }
  ws_items = ws;
  vt_items = vt;
  vtt_items = vtt;
  vl_items = vl;
  pre_items = pre;
  bidx_items = bidx;
  dcnt_items = dcnt;
  // Task size: about tasks_per_wave tasks per resident wave over the whole
  // launch.  A tile cheaper than that is grouped with its neighbours; a dearer
  // one is split into item chunks of at least min_chunk items.
  const int64_t min_chunk = tune.min_chunk;
  const double target = std::max(1.0, total / ((double)tune.tasks_per_wave * (double)grid_sweep));
  std::vector<double> task_cost(ent.size());
  // A BJ1 or CCM1 segment tile walks its 2K windows one after another, each a
  // short chain of dependent loads.  When the launch has fewer such tiles
  // than resident waves (one large instance), that chain and not the issue
  // rate sets the sweep's length, so their q range is split into chunks of
  // at most kSegQPerChunk values, each a task of its own; a launch with more
  // tiles keeps them whole (its waves hide the latency, and split tiles cost
  // partial-sum slots).
  int64_t seg_tiles = 0;
  for (const Entry &e : ent)
    if (e.mode == kModeSegments && (e.bound == kBJ1 || e.bound == kCCM1)) seg_tiles += e.ntiles;
  const bool split_seg = seg_tiles < (int64_t)grid_sweep;
  // Partial-sum slots of the split tiles stay under kMaxAccBytes: past it the
  // chunk count of the item-split tiles is halved until they fit (a tile of a
  // huge instance could otherwise ask for 64 chunks of every parameter).
  int64_t max_chunks = 64;
  int64_t acc = 0, cnt = 0;
  for (;;) {
  int64_t slots = 0;
  for (size_t j = 0; j < ent.size(); ++j) {
    Entry &e = ent[j];
    const double tc = tile_cost_v[j];
    if (e.mode == kModeLookup) {
      if (e.aux) {  // chunks of the q range, set by the band (moved once: this loop may run again)
        e.nchunks = e.aux;
        e.aux = 0;
      }
      e.tpt = 1;
      task_cost[j] = tc / e.nchunks;
    } else if (split_seg && e.mode == kModeSegments && (e.bound == kBJ1 || e.bound == kCCM1)) {
      const int64_t C = pin[e.inst].C;
      const int64_t knum = e.bound == kBJ1 ? C : C / 2;
      const int64_t kfirst = knum / std::max<int64_t>(1, e.lam0);  // the entry's largest window count
      e.nchunks = (int32_t)std::min<int64_t>(64, std::max<int64_t>(1, (kfirst + kSegQPerChunk - 1) / kSegQPerChunk));
      e.tpt = 1;
      task_cost[j] = tc / e.nchunks;
    } else if (tc <= target || e.bound == kL2 || e.mode == kModeSegments || e.mode == kModeCand) {
      double tpt = std::floor(target / tc);
      tpt = std::min(std::max(tpt, 1.0), std::min((double)e.ntiles, 1e9));
      e.tpt = (int32_t)tpt;
      e.nchunks = 1;
      task_cost[j] = tc * tpt;
    } else {
      // an entry of a few tiles (FS1's 100 parameters, the single mirrored VB2
      // parameters) would otherwise be a few long chains: chunks down to 256
      // items, but at most 16 of them (the combine adds a tile's chunks in
      // rounds of four dependent loads)
      const int64_t minc = e.ntiles < 4 ? std::min<int64_t>(min_chunk, std::max<int64_t>(256, (rcap_v[j] + 15) / 16))
                                        : min_chunk;
      const int64_t maxch = std::max<int64_t>(1, rcap_v[j] / minc);
      const int64_t want = (int64_t)std::ceil(tc / target);
      e.nchunks = (int32_t)std::min<int64_t>(std::min<int64_t>(want, maxch), max_chunks);
      e.tpt = 1;
      task_cost[j] = tc / e.nchunks;
    }
    if (e.nchunks > 1) slots += e.ntiles * e.nchunks * tile;
  }
  if (slots * (int64_t)sizeof(long long) <= kMaxAccBytes || max_chunks == 1) break;
  max_chunks /= 2;
  }
  std::vector<size_t> order(ent.size());
  for (size_t j = 0; j < order.size(); ++j) order[j] = j;
  // Longest task first, except that L2 tasks and the candidate tiles of MT
  // and RAD2 go first of all: they are cheap in issue slots but wait on
  // chains of dependent loads, and started early they overlap the sweeps of
  // other waves instead of trailing the launch.
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
    const bool la = ent[a].bound == kL2 || ent[a].mode == kModeCand, lb = ent[b].bound == kL2 || ent[b].mode == kModeCand;
    if (la != lb) return la;
    const int32_t ra = order_rank[ent[a].bound], rb = order_rank[ent[b].bound];
    if (ra != rb) return ra < rb;
    return task_cost[a] > task_cost[b];
  });
  std::vector<Entry> seq;
  seq.reserve(ent.size() + 1);
  for (size_t j : order) seq.push_back(ent[j]);
  for (Entry &e : seq) {
    e.split_base = cnt;
    e.slot32 = 0;
    if (e.nchunks > 1) {
      // Item chunks of MT, RAD2, CCM1, VB2 and BJ1 tiles have partial sums of
      // magnitude at most 2 c per item (MT, RAD2, VB2: c; CCM1: 2c / lambda;
      // BJ1: the sizes' sum plus lambda per item), so a chunk of at most
      // ceil(r / chunks) items fits an int32 slot when that times 2c does:
      // half the slot traffic.  FS1 (up to 100 c per item) and the q-range
      // chunks of segment and lookup tiles keep int64.
      const int64_t rcap = plan_vec[(size_t)e.inst].r_cap;
      const int64_t per = (rcap + e.nchunks - 1) / e.nchunks;
      const bool item_split = e.mode == kModeDense || e.mode == kModeMirror;
      const bool bounded = e.bound == kMT || e.bound == kRAD2 || e.bound == kCCM1 || e.bound == kVB2 || e.bound == kBJ1;
      e.slot32 = item_split && bounded && per * 2 * (int64_t)plan_vec[(size_t)e.inst].C < (int64_t(1) << 31) ? 1 : 0;
      const int64_t n = e.ntiles * e.nchunks * tile;
      e.acc_base = acc;
      acc += e.slot32 ? (n + 1) / 2 : n;
      cnt += (e.ntiles + kSegTiles - 1) / kSegTiles;
    }
  }
  acc_len = acc;
  nsplit = cnt;
  entry_vec.resize(std::max<size_t>(seq.size(), 1));
  memset(entry_vec.data(), 0, sizeof(Entry) * entry_vec.size());
  int64_t tb = 0;
  for (size_t j = 0; j < seq.size(); ++j) {
    Entry e = seq[j];
    e.task_begin = tb;
    tb += ((e.ntiles + e.tpt - 1) / e.tpt) * e.nchunks;
    entry_vec[j] = e;
  }
  nentries = (int64_t)seq.size();
  *ntasks_out = tb;
  return BP_OK;
}

// Runs one planned launch.  host_in (optional): input arena to stage with the
// tables (it holds the residuals too); else in_dev and in2_dev are the device
// arenas of the sizes and of the residuals.  out_dev: device result array;
// s: stream to queue on.  The launch is ordered after the previous one of
// this context, whichever stream that went to.
bp_status Ctx::run(int64_t count, int64_t ntasks, const int32_t *host_in, int64_t host_in_len,
                   const int32_t *in_dev, const int32_t *in2_dev, bp_bounds *out_dev, hipStream_t s) {
  bp_status st;
  const size_t off_plan = align256(sizeof(LaunchDesc));
  const size_t off_ent = off_plan + align256(sizeof(InstPlan) * (size_t)count);
  const size_t off_div = off_ent + align256(sizeof(Entry) * entry_vec.size());
  const size_t off_vl = off_div + align256(sizeof(int32_t) * std::max<size_t>(div_vec.size(), 1));
  const size_t off_in = off_vl + align256(sizeof(int32_t) * std::max<size_t>(vt_list.size(), 1));
  const size_t total = off_in + (host_in ? align256(sizeof(int32_t) * (size_t)std::max<int64_t>(host_in_len, 1)) : 0);
  if ((st = stage_host.reserve(total))) return st;
  void *old_dev = stage_buf.p;
  if ((st = reserve_dev(stage_buf, total))) return st;
  if (stage_buf.p != old_dev) drop_graphs();  // the graphs hold the descriptor's address: capture again
  if ((st = reserve_dev(state_buf, sizeof(InstState) * count))) return st;
  if ((st = reserve_dev(sorted_buf, sizeof(int32_t) * ws_items))) return st;
  if ((st = reserve_dev(rec_buf, sizeof(uint32_t) * ws_items))) return st;
  if ((st = reserve_dev(pre_buf, sizeof(int64_t) * pre_items))) return st;
  if ((st = reserve_dev(keys_buf, sizeof(unsigned long long) * kNB * count))) return st;
  if ((st = reserve_dev(ref_buf, sizeof(int32_t) * count))) return st;
  if ((st = reserve_dev(acc_buf, sizeof(long long) * (size_t)std::max<int64_t>(acc_len, 1)))) return st;
  if ((st = reserve_dev(bidx_buf, sizeof(int32_t) * (size_t)std::max<int64_t>(bidx_items, 1)))) return st;
  if ((st = reserve_dev(dcnt_buf, sizeof(int32_t) * (size_t)std::max<int64_t>(dcnt_items, 1)))) return st;
  // value tables: the raw counts, chunk totals, lattice bins, flags and
  // maxima are zero at rest (a new allocation is cleared here, each launch
  // clears what it used)
  bool clear_vt = false;
  if (!vt_list.empty()) {
    const void *old_r = vraw_buf.p, *old_t = vtot_buf.p, *old_l = vlat_buf.p, *old_f = vflag_buf.p;
    if ((st = reserve_dev(vraw_buf, sizeof(int32_t) * (size_t)vt_items))) return st;
    if ((st = reserve_dev(vcnt_buf, sizeof(int32_t) * (size_t)vt_items))) return st;
    if ((st = reserve_dev(vsum_buf, sizeof(long long) * (size_t)vt_items))) return st;
    if ((st = reserve_dev(vtot_buf, sizeof(long long) * (size_t)std::max<int64_t>(vtt_items, 1)))) return st;
    if ((st = reserve_dev(vlat_buf, sizeof(int32_t) * (size_t)std::max<int64_t>(vl_items, 1)))) return st;
    if ((st = reserve_dev(vflag_buf, 2 * sizeof(int32_t) * vt_list.size()))) return st;
    clear_vt = vt_dirty || vraw_buf.p != old_r || vtot_buf.p != old_t || vlat_buf.p != old_l || vflag_buf.p != old_f;
  }
  char *h = (char *)stage_host.p;
  char *dv = (char *)stage_buf.p;
  LaunchDesc *d = (LaunchDesc *)h;
  memset(d, 0, sizeof *d);
  d->in = host_in ? (const int32_t *)(dv + off_in) : in_dev;
  d->in2 = host_in ? (const int32_t *)(dv + off_in) : in2_dev;
  d->plan = (const InstPlan *)(dv + off_plan);
  d->entries = (const Entry *)(dv + off_ent);
  d->state = (InstState *)state_buf.p;
  d->sorted = (int32_t *)sorted_buf.p;
  d->pre = (int64_t *)pre_buf.p;
  d->av = (uint32_t *)rec_buf.p;
  d->keys = (unsigned long long *)keys_buf.p;
  d->refuted = (int32_t *)ref_buf.p;
  d->counter = (unsigned long long *)counter_buf.p;
  d->acc = (long long *)acc_buf.p;
  d->bidx = (int32_t *)bidx_buf.p;
  d->divs = (const int32_t *)(dv + off_div);
  d->dcnt = (int32_t *)dcnt_buf.p;
  d->nodes = nodes;
  d->vraw = (int32_t *)vraw_buf.p;
  d->vcnt = (int32_t *)vcnt_buf.p;
  d->vsum = (long long *)vsum_buf.p;
  d->vtot = (long long *)vtot_buf.p;
  d->vlat = (int32_t *)vlat_buf.p;
  d->vflag = (int32_t *)vflag_buf.p;
  d->vlist = (const int32_t *)(dv + off_vl);
  d->nvt = (int64_t)vt_list.size();
  for (int64_t i = 0; i < count; ++i)
    if (plan_vec[(size_t)i].state_off >= 0 && !nodes)
      return fail(BP_ERR_STATE, "instance %lld asks for a node state but the context has no node arena", (long long)i);
  d->out = out_dev;
  d->count = count;
  d->nentries = nentries;
  d->ntasks = ntasks;
  d->acc_len = acc_len;
  d->nsplit = nsplit;
  memcpy(h + off_plan, plan_vec.data(), sizeof(InstPlan) * (size_t)count);
  memcpy(h + off_ent, entry_vec.data(), sizeof(Entry) * entry_vec.size());
  if (!div_vec.empty()) memcpy(h + off_div, div_vec.data(), sizeof(int32_t) * div_vec.size());
  if (!vt_list.empty()) memcpy(h + off_vl, vt_list.data(), sizeof(int32_t) * vt_list.size());
  if (host_in && host_in_len > 0) memcpy(h + off_in, host_in, sizeof(int32_t) * (size_t)host_in_len);
  if (any_run) HIP_TRY(hipStreamWaitEvent(s, last_run, 0));
  HIP_TRY(hipMemcpyAsync(dv, h, total, hipMemcpyHostToDevice, s));
  HIP_TRY(hipEventRecord(staged, s));
  if (!vt_list.empty()) {
    if (clear_vt) {
      // outside any captured graph: a plain stream operation before the launch
      HIP_TRY(hipMemsetAsync(vraw_buf.p, 0, vraw_buf.cap, s));
      HIP_TRY(hipMemsetAsync(vtot_buf.p, 0, vtot_buf.cap, s));
      HIP_TRY(hipMemsetAsync(vlat_buf.p, 0, vlat_buf.cap, s));
      HIP_TRY(hipMemsetAsync(vflag_buf.p, 0, vflag_buf.cap, s));
    }
    vt_dirty = true;  // until the whole launch is queued
  }
  const LaunchDesc *d_desc = (const LaunchDesc *)dv;
  const LaunchShape sh = shape_of(count, ntasks);
  if (timing) {
    hipEvent_t *ev = nullptr;
    if ((st = timing_slot(&ev))) return st;
    HIP_TRY(launch_pipeline_timed(d_desc, sh.lpl, sh.prep_small, sh.prep_large, sh.vt, sh.sweep, sh.comb, sh.fin, sh.v,
                                  s, ev));
  } else if (use_graph) {
    hipGraphExec_t ex = nullptr;
    if ((st = ensure_graph(d_desc, sh, &ex))) return st;
    HIP_TRY(hipGraphLaunch(ex, s));
  } else {
    HIP_TRY(launch_pipeline(d_desc, sh.lpl, sh.prep_small, sh.prep_large, sh.vt, sh.sweep, sh.comb, sh.fin, sh.v, s));
  }
  HIP_TRY(hipEventRecord(last_run, s));
  any_run = true;
  ++run_count;
  if (!vt_list.empty()) vt_dirty = false;  // queued whole: its finalize clears the tables
  return BP_OK;
}

// The pinned staging buffers may still feed copies of the previous call.
bp_status Ctx::wait_staging() {
  HIP_TRY(hipEventSynchronize(staged));
  return BP_OK;
}

}  // namespace bpi

// ===========================================================================
// C ABI

const char *bp_version(void) { return "libbp 0.1 (gfx950)"; }

const char *bp_last_error(void) { return bpi::g_err.c_str(); }

bp_status bp_default_sweep(int32_t C, int64_t r, int32_t max_w, uint32_t flags, bp_sweep *out) {
  if (!out) return fail(BP_ERR_ARG, "out is NULL");
  if (C < 1) return fail(BP_ERR_ARG, "C = %d < 1", C);
  if (flags & ~(BP_SWEEP_PAPER_VB2_CLAMP | BP_SWEEP_SEGMENTS)) return fail(BP_ERR_ARG, "unknown flags 0x%x", flags);
  if (r < 0 || max_w < 0) return fail(BP_ERR_ARG, "negative r or max_w");
  memset(out, 0, sizeof *out);
  default_ranges(C, out->lo, out->hi);
  out->flags = flags;
  if (flags & BP_SWEEP_PAPER_VB2_CLAMP) {
    const int64_t denom = r * (int64_t)max_w;
    const int64_t cap = denom > 0 ? (int64_t)0xffffffffLL / denom : (int64_t)C;
    if (cap < out->hi[kVB2]) out->hi[kVB2] = cap;
  }
  return BP_OK;
}

bp_status bp_ctx_create(int device, bp_ctx **out) {
  if (!out) return fail(BP_ERR_ARG, "out is NULL");
  *out = nullptr;
  Ctx *c = new (std::nothrow) Ctx();
  if (!c) return fail(BP_ERR_NOMEM, "context allocation");
  bp_status st = c->init(device);
  if (st) {
    c->destroy();
    delete c;
    return st;
  }
  c->magic = kCtxMagic;
  *out = (bp_ctx *)c;
  return BP_OK;
}

bp_status bp_ctx_destroy(bp_ctx *ctx) {
  Ctx *c = (Ctx *)ctx;
  if (!c || c->magic != kCtxMagic) return fail(BP_ERR_STATE, "bad context");
  c->magic = 0;
  c->destroy();
  delete c;
  return BP_OK;
}

static bp_status get_ctx(bp_ctx *ctx, Ctx **c) {
  Ctx *x = (Ctx *)ctx;
  if (!x || x->magic != kCtxMagic) return fail(BP_ERR_STATE, "bad context");
  hipError_t e = hipSetDevice(x->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  *c = x;
  return BP_OK;
}

void Ctx::timing_reset() {
  t_runs = t_folded = 0;
  t_sum[0] = t_sum[1] = t_sum[2] = 0;
}

static bp_status fold_set(hipEvent_t *ev, double sum[3]) {
  HIP_TRY(hipEventSynchronize(ev[3]));
  for (int i = 0; i < 3; ++i) {
    float t = 0;
    HIP_TRY(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
    sum[i] += t;
  }
  return BP_OK;
}

bp_status Ctx::timing_slot(hipEvent_t **ev) {
  if (t_runs - t_folded == kTimingRing) {
    bp_status st = fold_set(tev[t_folded % kTimingRing], t_sum);
    if (st) return st;
    ++t_folded;
  }
  *ev = tev[t_runs % kTimingRing];
  ++t_runs;
  return BP_OK;
}

bp_status Ctx::timing_mean(double ms[3], int64_t *runs) {
  for (; t_folded < t_runs; ++t_folded) {
    bp_status st = fold_set(tev[t_folded % kTimingRing], t_sum);
    if (st) return st;
  }
  if (runs) *runs = t_runs;
  if (t_runs == 0) return fail(BP_ERR_STATE, "no timed call since timing was switched on");
  for (int i = 0; i < 3; ++i) ms[i] = t_sum[i] / (double)t_runs;
  return BP_OK;
}

bp_status bp_ctx_set_timing(bp_ctx *ctx, int32_t enable) {
  Ctx *c;
  bp_status st = get_ctx(ctx, &c);
  if (st) return st;
  c->timing = enable != 0;
  c->timing_reset();
  return BP_OK;
}

static bp_status check_tuning(const bp_tuning *t) {
  if (!t) return fail(BP_ERR_ARG, "tuning is NULL");
  if (t->lanes_params != 1 && t->lanes_params != 2 && t->lanes_params != 4)
    return fail(BP_ERR_ARG, "lanes_params must be 1, 2 or 4");
  if (t->waves_per_cu < 4 || t->waves_per_cu > 32) return fail(BP_ERR_ARG, "waves_per_cu outside [4, 32]");
  if (t->tasks_per_wave < 1 || t->tasks_per_wave > 64) return fail(BP_ERR_ARG, "tasks_per_wave outside [1, 64]");
  if (t->min_chunk < 64 || t->min_chunk > 65536) return fail(BP_ERR_ARG, "min_chunk outside [64, 65536]");
  return BP_OK;
}

bp_status bp_ctx_get_tuning(bp_ctx *ctx, bp_tuning *out) {
  Ctx *c;
  bp_status st = get_ctx(ctx, &c);
  if (st) return st;
  if (!out) return fail(BP_ERR_ARG, "out is NULL");
  *out = c->tune;
  return BP_OK;
}

bp_status bp_ctx_set_tuning(bp_ctx *ctx, const bp_tuning *tuning) {
  Ctx *c;
  bp_status st = get_ctx(ctx, &c);
  if (st) return st;
  if ((st = check_tuning(tuning))) return st;
  if ((st = c->wait_staging())) return st;
  c->tune = *tuning;
  c->apply_tuning();
  return BP_OK;
}

bp_status bp_ctx_set_order(bp_ctx *ctx, const int32_t *order) {
  Ctx *c;
  bp_status st = get_ctx(ctx, &c);
  if (st) return st;
  int32_t rank[kNB] = {};
  if (order) {
    bool seen[kNB] = {};
    for (int i = 0; i < 6; ++i) {
      const int32_t b = order[i];
      if (b < kMT || b > kBJ1 || seen[b]) return fail(BP_ERR_ARG, "order is not a permutation of the six functions");
      seen[b] = true;
      rank[b] = i + 1;
    }
  }
  if ((st = c->wait_staging())) return st;
  memcpy(c->order_rank, rank, sizeof rank);
  return BP_OK;
}

bp_status bp_ctx_stage_times(bp_ctx *ctx, double ms[3], int64_t *runs) {
  Ctx *c;
  bp_status st = get_ctx(ctx, &c);
  if (st) return st;
  if (!ms) return fail(BP_ERR_ARG, "ms is NULL");
  if (!c->timing) return fail(BP_ERR_STATE, "timing is off");
  return c->timing_mean(ms, runs);
}

// ---- reduction ----------------------------------------------------------

static bp_status reduce_common(bp_ctx *ctx, int32_t C, int32_t m, const int32_t *residual, const int32_t *size,
                               const int32_t *bin_of, int64_t n, int32_t *out_items, int64_t *out_r,
                               int32_t *out_residual) {
  Ctx *c;
  bp_status st = get_ctx(ctx, &c);
  if (st) return st;
  if (C < 1 || m < 0 || n < 0 || !out_items || !out_r) return fail(BP_ERR_ARG, "bad reduction arguments");
  if ((n > 0 && !size) || (m > 0 && !bin_of && !residual) || (bin_of && n > 0 && !bin_of))
    return fail(BP_ERR_ARG, "NULL input array");
  if (n + (int64_t)m > BP_MAX_REDUCE_ITEMS)
    return fail(BP_ERR_LIMIT, "n + m = %lld > %d", (long long)(n + m), BP_MAX_REDUCE_ITEMS);
  // host staging: [size n][bin_of n][residual m]
  const size_t in_bytes = sizeof(int32_t) * (size_t)(2 * n + m) + 64;
  if ((st = c->wait_staging())) return st;
  if ((st = c->red_host.reserve(in_bytes + sizeof(int32_t) * (size_t)(n + 2 * (int64_t)m) + 64))) return st;
  int32_t *h = (int32_t *)c->red_host.p;
  if (n) memcpy(h, size, sizeof(int32_t) * n);
  if (bin_of && n) memcpy(h + n, bin_of, sizeof(int32_t) * n);
  if (!bin_of && m) memcpy(h + 2 * n, residual, sizeof(int32_t) * m);
  // device: inputs, loads (u64 m), out (n + m), out_residual (m), out_r, bad
  const size_t dev_bytes = in_bytes + sizeof(uint64_t) * (size_t)(m + 1) + sizeof(int32_t) * (size_t)(n + 2 * (int64_t)m) + 256;
  if ((st = c->reserve_dev(c->red_buf, dev_bytes))) return st;
  char *base = (char *)c->red_buf.p;
  int32_t *d_size = (int32_t *)base;
  int32_t *d_bin = d_size + n;
  int32_t *d_res = d_size + 2 * n;
  size_t off = (sizeof(int32_t) * (size_t)(2 * n + m) + 63) & ~size_t(63);
  unsigned long long *d_loads = (unsigned long long *)(base + off);
  off += (sizeof(uint64_t) * (size_t)(m + 1) + 63) & ~size_t(63);
  int64_t *d_r = (int64_t *)(base + off);
  int32_t *d_bad = (int32_t *)(base + off + 8);
  off += 64;
  int32_t *d_out = (int32_t *)(base + off);
  int32_t *d_outres = d_out + n + m;
  hipStream_t s = c->stream;
  HIP_TRY(hipMemcpyAsync(d_size, h, sizeof(int32_t) * (size_t)(2 * n + m), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(d_loads, 0, sizeof(uint64_t) * (size_t)(m + 1), s));
  HIP_TRY(hipMemsetAsync(d_r, 0, 64, s));
  HIP_TRY(launch_reduce(C, m, bin_of ? nullptr : d_res, d_size, bin_of ? d_bin : nullptr, n, d_loads, d_out, d_r,
                        d_outres, d_bad, s));
  int32_t *ho = h + 2 * n + m;
  HIP_TRY(hipMemcpyAsync(ho, d_out, sizeof(int32_t) * (size_t)(n + 2 * (int64_t)m), hipMemcpyDeviceToHost, s));
  int64_t *hr = (int64_t *)(((uintptr_t)(ho + n + 2 * (int64_t)m) + 15) & ~uintptr_t(15));
  HIP_TRY(hipMemcpyAsync(hr, d_r, 16, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int32_t bad = ((int32_t *)hr)[2];
  if (bad) return fail(BP_ERR_RANGE, "size, bin index or residual out of range, or a bin over capacity");
  const int64_t r = hr[0];
  memcpy(out_items, ho, sizeof(int32_t) * (size_t)r);
  *out_r = r;
  if (out_residual && m) memcpy(out_residual, ho + n + m, sizeof(int32_t) * (size_t)m);
  return BP_OK;
}

bp_status bp_residual_reduce(bp_ctx *ctx, int32_t C, int32_t m, const int32_t *residual, const int32_t *unpacked,
                             int64_t n, int32_t *out_items, int64_t *out_r) {
  if (m > 0 && !residual) return fail(BP_ERR_ARG, "residual is NULL");
  return reduce_common(ctx, C, m, residual, unpacked, nullptr, n, out_items, out_r, nullptr);
}

bp_status bp_assignment_reduce(bp_ctx *ctx, int32_t C, int32_t m, const int32_t *size, const int32_t *bin_of,
                               int64_t n, int32_t *out_items, int64_t *out_r, int32_t *out_residual) {
  if (n > 0 && !bin_of) return fail(BP_ERR_ARG, "bin_of is NULL");
  static const int32_t dummy = 0;
  return reduce_common(ctx, C, m, nullptr, size, bin_of ? bin_of : &dummy, n, out_items, out_r, out_residual);
}

// ---- checks --------------------------------------------------------------

namespace bpi {

// Host-input batch in either form: stage into pinned memory, plan, launch and
// queue the copy of the results back into c->out_host; c->done marks the end.
bp_status launch_host_batch(Ctx *c, std::vector<PlanIn> &pin, const std::vector<const int32_t *> &src_a,
                            const std::vector<const int32_t *> &src_b) {
  bp_status st;
  const int64_t count = (int64_t)pin.size();
  // input arena layout: per instance [a: n_in][b: m_res]
  int64_t tot = 0;
  for (auto &q : pin) {
    q.in_off = tot;
    tot += q.n_in;
    q.res_off = tot;
    tot += q.m_res;
  }
  if ((st = c->wait_staging())) return st;
  int64_t ntasks = 0;
  if ((st = c->plan(pin, &ntasks))) return st;
  if ((st = c->in_host.reserve(sizeof(int32_t) * (size_t)std::max<int64_t>(tot, 1)))) return st;
  if ((st = c->out_host.reserve(sizeof(bp_bounds) * count))) return st;
  if ((st = c->reserve_dev(c->out_buf, sizeof(bp_bounds) * count))) return st;
  int32_t *h = (int32_t *)c->in_host.p;
  for (int64_t i = 0; i < count; ++i) {
    if (pin[i].n_in) memcpy(h + pin[i].in_off, src_a[i], sizeof(int32_t) * (size_t)pin[i].n_in);
    if (pin[i].m_res) memcpy(h + pin[i].res_off, src_b[i], sizeof(int32_t) * (size_t)pin[i].m_res);
  }
  if ((st = c->run(count, ntasks, h, tot, nullptr, nullptr, (bp_bounds *)c->out_buf.p, c->stream))) return st;
  HIP_TRY(hipMemcpyAsync(c->out_host.p, c->out_buf.p, sizeof(bp_bounds) * count, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipEventRecord(c->done, c->stream));
  return BP_OK;
}

// Wait for the batch launched by launch_host_batch and copy its results.
bp_status collect_host_batch(Ctx *c, int64_t count, bp_bounds *out, bool check_status) {
  HIP_TRY(hipEventSynchronize(c->done));
  memcpy(out, c->out_host.p, sizeof(bp_bounds) * count);
  if (!check_status) return BP_OK;
  for (int64_t i = 0; i < count; ++i) {
    if (out[i].status == BP_ERR_RANGE) return fail(BP_ERR_RANGE, "instance %lld: size or residual outside [0, C]", (long long)i);
    if (out[i].status) return fail(out[i].status, "instance %lld: device status %d", (long long)i, out[i].status);
  }
  return BP_OK;
}

bp_status run_host_batch(Ctx *c, std::vector<PlanIn> &pin, const std::vector<const int32_t *> &src_a,
                                const std::vector<const int32_t *> &src_b, bp_bounds *out) {
  bp_status st = launch_host_batch(c, pin, src_a, src_b);
  if (st) return st;
  return collect_host_batch(c, (int64_t)pin.size(), out, true);
}

bp_status make_plan_in(int32_t C, int64_t k, int64_t n_in, int32_t m_res, int32_t form, const bp_sweep *sw,
                       bool early, PlanIn *q, bool segments) {
  if (C < 1) return fail(BP_ERR_ARG, "C = %d < 1", C);
  if (k < 0) return fail(BP_ERR_ARG, "k = %lld < 0", (long long)k);
  if (n_in < 0 || m_res < 0) return fail(BP_ERR_ARG, "negative count");
  if (n_in + m_res > BP_MAX_ITEMS) return fail(BP_ERR_LIMIT, "%lld items > %d", (long long)(n_in + m_res), BP_MAX_ITEMS);
  memset(q, 0, sizeof *q);
  q->state_off = -1;
  q->C = C;
  q->k = k;
  q->n_in = n_in;
  q->m_res = m_res;
  q->form = form;
  q->early_exit = early;
  q->clamp = sw && (sw->flags & BP_SWEEP_PAPER_VB2_CLAMP);
  q->segments = segments || (sw && (sw->flags & BP_SWEEP_SEGMENTS));
  return check_sweep(C, sw, q->lo, q->hi);
}

bp_status host_validate_items(int32_t C, const int32_t *items, int64_t r) {
  for (int64_t i = 0; i < r; ++i)
    if (items[i] < 0 || items[i] > C)
      return fail(BP_ERR_RANGE, "item %lld has size %d outside [0, %d]", (long long)i, items[i], C);
  return BP_OK;
}

}  // namespace bpi

namespace bpi {

// The one-launch path for small checks: the instance goes in the kernel's
// arguments and the record comes back in host memory, so a check costs one
// launch and one wait.  *done is false when the instance is too large for it.
bp_status run_small(Ctx *c, const PlanIn &q, const int32_t *sizes, const int32_t *residual, bp_bounds *out,
                    bool *done) {
  *done = false;
  if (!c->small_path || c->timing) return BP_OK;  // stage timing measures the pipeline
  const int64_t nv = q.n_in + (q.form == kFormResidual ? q.m_res : 0);
  if (nv > kSmallFusedMax) return BP_OK;
  int64_t params = 0;  // L2 and the six functions, before any VB2 cut
  for (int b = kL2; b < kNB; ++b) params += q.lo[b] <= q.hi[b] ? q.hi[b] - q.lo[b] + 1 : 0;
  if (params * std::max<int64_t>(nv, 1) > c->small_work) return BP_OK;
  SmallArgs a;
  memset(&a, 0, offsetof(SmallArgs, v));
  a.C = q.C;
  a.m = q.form == kFormResidual ? q.m_res : 0;
  a.n = (int32_t)q.n_in;
  a.form = q.form;
  a.k = q.k;
  for (int b = 0; b < kNB; ++b) {
    a.lo[b] = q.lo[b];
    a.hi[b] = q.hi[b];
  }
  a.clamp = q.clamp ? 1u : 0u;
  // S lanes per (bound, parameter) pair, each summing every S-th item: about
  // small_items items per lane, and no more lanes than small_waves waves per
  // SIMD hold (four SIMDs per compute unit)
  a.slices = 1;
  while (a.slices < 64 && (int64_t)a.slices * c->small_items < nv &&
         params * a.slices < (int64_t)c->num_cu * 4 * 64 * c->small_waves)
    a.slices <<= 1;
  if (q.n_in) memcpy(a.v, sizes, sizeof(int32_t) * (size_t)q.n_in);
  if (a.m) memcpy(a.v + q.n_in, residual, sizeof(int32_t) * (size_t)a.m);
  bp_bounds *h = (bp_bounds *)c->small_out;
  uint32_t *seq = (uint32_t *)((char *)c->small_out + sizeof(bp_bounds));
  const uint32_t want = ++c->small_seq;
  // a few workgroups of 256: one kernel; else workgroups of 1024 and the final kernel
  const int64_t lanes = params * a.slices;
  const bool one = (lanes + kSmallOneThreads - 1) / kSmallOneThreads <= kSmallOneMaxGrid;
  const int grid = one ? (int)std::max<int64_t>(1, (lanes + kSmallOneThreads - 1) / kSmallOneThreads)
                       : (int)std::min<int64_t>(c->small_grid, (lanes + kSmallFusedThreads - 1) / kSmallFusedThreads);
  HIP_TRY(launch_small_check(a, one, grid, c->small_keys.p, h, seq, want, c->stream));
  // Wait for the kernel's sequence number in host memory; after two seconds
  // without it, let the stream report what went wrong.
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t spin = 0;; ++spin) {
    if (__atomic_load_n(seq, __ATOMIC_ACQUIRE) == want) break;
    if ((spin & 1023u) == 1023u && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
      HIP_TRY(hipStreamSynchronize(c->stream));
      if (__atomic_load_n(seq, __ATOMIC_ACQUIRE) == want) break;
      return fail(BP_ERR_DEVICE, "the small check did not report its record");
    }
  }
  *out = *h;
  *done = true;
  if (out->status == BP_ERR_RANGE) return fail(BP_ERR_RANGE, "size or residual outside [0, C]");
  if (out->status) return fail(out->status, "device status %d", out->status);
  return BP_OK;
}

}  // namespace bpi

bp_status bp_lower_bounds(bp_ctx *ctx, int32_t C, int32_t k, const int32_t *items, int64_t r, const bp_sweep *sweep,
                          bp_bounds *out) {
  Ctx *c;
  bp_status st = get_ctx(ctx, &c);
  if (st) return st;
  if (!out || (r > 0 && !items)) return fail(BP_ERR_ARG, "NULL argument");
  std::vector<PlanIn> pin(1);
  if ((st = make_plan_in(C, k, r, 0, kFormItems, sweep, false, &pin[0]))) return st;
  if ((st = host_validate_items(C, items, r))) return st;
  bool done = false;
  if ((st = run_small(c, pin[0], items, nullptr, out, &done)) || done) return st;
  return run_host_batch(c, pin, {items}, {nullptr}, out);
}

bp_status bp_lower_bounds_dev(bp_ctx *ctx, int32_t C, int32_t k, const int32_t *d_items, int64_t r,
                              const bp_sweep *sweep, bp_bounds *d_out, void *stream) {
  Ctx *c;
  bp_status st = get_ctx(ctx, &c);
  if (st) return st;
  if (!d_out || (r > 0 && !d_items)) return fail(BP_ERR_ARG, "NULL argument");
  std::vector<PlanIn> pin(1);
  if ((st = make_plan_in(C, k, r, 0, kFormItems, sweep, false, &pin[0]))) return st;
  pin[0].in_off = 0;
  if ((st = c->wait_staging())) return st;
  int64_t ntasks = 0;
  if ((st = c->plan(pin, &ntasks))) return st;
  return c->run(1, ntasks, nullptr, 0, d_items, d_items, d_out, (hipStream_t)stream);
}

bp_status bp_feasible(bp_ctx *ctx, int32_t C, int32_t m, const int32_t *residual, const int32_t *unpacked, int64_t n,
                      uint32_t flags, int32_t *verdict, int64_t *lb, bp_bounds *bounds) {
  Ctx *c;
  bp_status st = get_ctx(ctx, &c);
  if (st) return st;
  if ((m > 0 && !residual) || (n > 0 && !unpacked)) return fail(BP_ERR_ARG, "NULL input array");
  if (flags & ~(BP_NO_EARLY_EXIT | BP_SEGMENTS)) return fail(BP_ERR_ARG, "unknown flags 0x%x", flags);
  std::vector<PlanIn> pin(1);
  if ((st = make_plan_in(C, m, n, m, kFormResidual, nullptr, !(flags & BP_NO_EARLY_EXIT), &pin[0],
                         (flags & BP_SEGMENTS) != 0)))
    return st;
  if ((st = host_validate_items(C, unpacked, n))) return st;
  if ((st = host_validate_items(C, residual, m))) return st;
  bp_bounds o;
  bool done = false;
  if ((st = run_small(c, pin[0], unpacked, residual, &o, &done))) return st;
  if (!done && (st = run_host_batch(c, pin, {unpacked}, {residual}, &o))) return st;
  if (verdict) *verdict = o.verdict;
  if (lb) *lb = o.lb;
  if (bounds) *bounds = o;
  return BP_OK;
}

bp_status bp_feasible_dev(bp_ctx *ctx, int32_t C, int32_t m, const int32_t *d_residual, const int32_t *d_unpacked,
                          int64_t n, uint32_t flags, bp_bounds *d_out, void *stream) {
  Ctx *c;
  bp_status st = get_ctx(ctx, &c);
  if (st) return st;
  if (!d_out || (m > 0 && !d_residual) || (n > 0 && !d_unpacked)) return fail(BP_ERR_ARG, "NULL argument");
  if (flags & ~(BP_NO_EARLY_EXIT | BP_SEGMENTS)) return fail(BP_ERR_ARG, "unknown flags 0x%x", flags);
  std::vector<PlanIn> pin(1);
  if ((st = make_plan_in(C, m, n, m, kFormResidual, nullptr, !(flags & BP_NO_EARLY_EXIT), &pin[0],
                         (flags & BP_SEGMENTS) != 0)))
    return st;
  // the sizes and the residuals come from two arenas, each at offset 0
  pin[0].in_off = 0;
  pin[0].res_off = 0;
  if ((st = c->wait_staging())) return st;
  int64_t ntasks = 0;
  if ((st = c->plan(pin, &ntasks))) return st;
  return c->run(1, ntasks, nullptr, 0, d_unpacked, d_residual, d_out, (hipStream_t)stream);
}

// ---- allocation-free check -------------------------------------------------

bp_status bp_feasible_dev_noalloc(int32_t C, int32_t m, const int32_t *d_residual, const int32_t *d_unpacked,
                                  int64_t n, uint32_t flags, bp_bounds *d_out, void *stream) {
  if (!d_out || (m > 0 && !d_residual) || (n > 0 && !d_unpacked)) return fail(BP_ERR_ARG, "NULL argument");
  if (flags & ~BP_NO_EARLY_EXIT)
    return fail(BP_ERR_ARG, "flags 0x%x: the allocation-free check takes BP_NO_EARLY_EXIT only", flags);
  if (n < 0 || m < 0) return fail(BP_ERR_ARG, "negative count");
  if (n + (int64_t)m > BP_NOALLOC_MAX_ITEMS)
    return fail(BP_ERR_LIMIT, "n + m = %lld exceeds BP_NOALLOC_MAX_ITEMS = %d", (long long)(n + m),
                BP_NOALLOC_MAX_ITEMS);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  unsigned char *base = nullptr;
  HIP_TRY(noalloc_scratch(dev, &base));
  // Host-side planning tables only (no device memory): a planner per host
  // thread, set up for the device's compute-unit count and the default shape.
  thread_local Ctx planner;
  thread_local int planner_dev = -1;
  if (planner_dev != dev) {
    int cu = 0;
    HIP_TRY(hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev));
    planner.num_cu = cu;
    planner.grid_prep_small = cu * 2;
    planner.grid_prep_large = std::max(1, cu / 4);
    planner.grid_comb = cu * 2;
    planner.grid_fin = 64;
    planner_dev = dev;
  }
  planner.tune = bp_tuning{2, 32, 32, 2048};
  planner.apply_tuning();
  planner.value_prep = false;  // no value tables in the static workspace
  std::vector<PlanIn> pin(1);
  bp_status st = make_plan_in(C, m, n, m, kFormResidual, nullptr, !(flags & BP_NO_EARLY_EXIT), &pin[0], false);
  if (st) return st;
  pin[0].in_off = 0;
  pin[0].res_off = 0;
  int64_t ntasks = 0;
  if ((st = planner.plan(pin, &ntasks))) return st;
  if (planner.acc_len > kNaAccSlots) {
    // more partial-sum slots than the array holds: tiles split only where a
    // bound has fewer than four tiles
    planner.tune.min_chunk = 65536;
    if ((st = planner.plan(pin, &ntasks))) return st;
    if (planner.acc_len > kNaAccSlots)
      return fail(BP_ERR_LIMIT, "%lld partial-sum slots exceed the %lld of the static workspace",
                  (long long)planner.acc_len, (long long)kNaAccSlots);
  }
  if (planner.nentries > kNoAllocMaxEntries)
    return fail(BP_ERR_LIMIT, "%lld schedule entries > %d", (long long)planner.nentries, kNoAllocMaxEntries);
  NoAllocTables t;
  memset(&t, 0, sizeof t);
  LaunchDesc &d = t.d;
  d.in = d_unpacked;
  d.in2 = d_residual;
  d.plan = (const InstPlan *)(base + offsetof(NoAllocTables, p));
  d.entries = (const Entry *)(base + offsetof(NoAllocTables, e));
  d.state = (InstState *)(base + kNaState);
  d.sorted = (int32_t *)(base + kNaSorted);
  d.pre = (int64_t *)(base + kNaPre);
  d.av = (uint32_t *)(base + kNaAv);
  d.keys = (unsigned long long *)(base + kNaKeys);
  d.refuted = (int32_t *)(base + kNaRefuted);
  d.counter = (unsigned long long *)(base + kNaCounter);
  d.acc = (long long *)(base + kNaAcc);
  d.bidx = (int32_t *)(base + kNaCounter);  // no segment tables in this variant: never read
  d.divs = (const int32_t *)(base + kNaCounter);
  d.dcnt = (int32_t *)(base + kNaCounter);
  d.out = d_out;
  d.count = 1;
  d.nentries = planner.nentries;
  d.ntasks = ntasks;
  d.acc_len = planner.acc_len;
  d.nsplit = planner.nsplit;
  t.p = planner.plan_vec[0];
  for (int64_t j = 0; j < planner.nentries; ++j) t.e[j] = planner.entry_vec[(size_t)j];
  const Ctx::LaunchShape sh = planner.shape_of(1, ntasks);
  HIP_TRY(launch_noalloc(t, base, sh.lpl, sh.prep_small, sh.prep_large, sh.sweep, sh.comb, sh.fin, sh.v,
                         (hipStream_t)stream));
  return BP_OK;
}

static bp_status check_batch(const bp_batch *b) {
  if (!b || b->count < 0 || (b->count > 0 && (!b->off || !b->C || !b->k)))
    return fail(BP_ERR_ARG, "bad batch descriptor");
  if (b->count > BP_MAX_BATCH) return fail(BP_ERR_LIMIT, "batch of %d > %d", b->count, BP_MAX_BATCH);
  if (b->count > 0 && b->off[0] != 0) return fail(BP_ERR_ARG, "off[0] != 0");
  for (int32_t i = 0; i < b->count; ++i)
    if (b->off[i + 1] < b->off[i]) return fail(BP_ERR_ARG, "off not non-decreasing at %d", i);
  return BP_OK;
}

static bp_status batch_plan_in(const bp_batch *b, const bp_sweep *per, bool early, std::vector<PlanIn> &pin) {
  pin.resize(b->count);
  for (int32_t i = 0; i < b->count; ++i) {
    bp_status st = make_plan_in(b->C[i], b->k[i], b->off[i + 1] - b->off[i], 0, kFormItems, per ? &per[i] : nullptr,
                                early, &pin[i]);
    if (st) return st;
  }
  return BP_OK;
}

bp_status bp_lower_bounds_batch(bp_ctx *ctx, const bp_batch *batch, const bp_sweep *per_inst, bp_bounds *out) {
  Ctx *c;
  bp_status st = get_ctx(ctx, &c);
  if (st) return st;
  if ((st = check_batch(batch))) return st;
  if (batch->count == 0) return BP_OK;
  if (!out || !batch->items) return fail(BP_ERR_ARG, "NULL argument");
  std::vector<PlanIn> pin;
  if ((st = batch_plan_in(batch, per_inst, false, pin))) return st;
  std::vector<const int32_t *> a(batch->count), b(batch->count, nullptr);
  for (int32_t i = 0; i < batch->count; ++i) {
    a[i] = batch->items + batch->off[i];
    if ((st = host_validate_items(batch->C[i], a[i], pin[i].n_in))) return st;
  }
  return run_host_batch(c, pin, a, b, out);
}

bp_status bp_lower_bounds_batch_dev(bp_ctx *ctx, const bp_batch *batch, const int32_t *d_items,
                                    const bp_sweep *per_inst, bp_bounds *d_out, void *stream) {
  Ctx *c;
  bp_status st = get_ctx(ctx, &c);
  if (st) return st;
  if ((st = check_batch(batch))) return st;
  if (batch->count == 0) return BP_OK;
  if (!d_out || !d_items) return fail(BP_ERR_ARG, "NULL argument");
  std::vector<PlanIn> pin;
  if ((st = batch_plan_in(batch, per_inst, false, pin))) return st;
  for (int32_t i = 0; i < batch->count; ++i) {
    pin[i].in_off = batch->off[i];
    pin[i].res_off = batch->off[i];
  }
  if ((st = c->wait_staging())) return st;
  int64_t ntasks = 0;
  if ((st = c->plan(pin, &ntasks))) return st;
  return c->run(batch->count, ntasks, nullptr, 0, d_items, d_items, d_out, (hipStream_t)stream);
}

bp_status bp_feasible_batch(bp_ctx *ctx, const bp_batch *batch, uint32_t flags, int32_t *verdict, int64_t *lb,
                            bp_bounds *bounds) {
  Ctx *c;
  bp_status st = get_ctx(ctx, &c);
  if (st) return st;
  if ((st = check_batch(batch))) return st;
  if (flags & ~(BP_NO_EARLY_EXIT | BP_SEGMENTS)) return fail(BP_ERR_ARG, "unknown flags 0x%x", flags);
  if (batch->count == 0) return BP_OK;
  if (!batch->items) return fail(BP_ERR_ARG, "NULL items");
  std::vector<PlanIn> pin;
  if ((st = batch_plan_in(batch, nullptr, !(flags & BP_NO_EARLY_EXIT), pin))) return st;
  for (PlanIn &q : pin) q.segments = (flags & BP_SEGMENTS) != 0;
  std::vector<const int32_t *> a(batch->count), b(batch->count, nullptr);
  for (int32_t i = 0; i < batch->count; ++i) {
    a[i] = batch->items + batch->off[i];
    if ((st = host_validate_items(batch->C[i], a[i], pin[i].n_in))) return st;
  }
  std::vector<bp_bounds> o(batch->count);
  if ((st = run_host_batch(c, pin, a, b, o.data()))) return st;
  for (int32_t i = 0; i < batch->count; ++i) {
    if (verdict) verdict[i] = o[i].verdict;
    if (lb) lb[i] = o[i].lb;
  }
  if (bounds) memcpy(bounds, o.data(), sizeof(bp_bounds) * (size_t)batch->count);
  return BP_OK;
}

// ---- autotuner ---------------------------------------------------------------

bp_status bp_autotune_batch(bp_ctx *ctx, const bp_batch *batch, const bp_sweep *per_inst, int32_t reps,
                            bp_tuning *best, double *best_ms) {
  Ctx *c;
  bp_status st = get_ctx(ctx, &c);
  if (st) return st;
  if ((st = check_batch(batch))) return st;
  if (batch->count == 0 || !batch->items) return fail(BP_ERR_ARG, "empty batch");
  if (reps < 1) reps = 1;
  std::vector<PlanIn> pin;
  if ((st = batch_plan_in(batch, per_inst, false, pin))) return st;
  std::vector<const int32_t *> a(batch->count), b(batch->count, nullptr);
  for (int32_t i = 0; i < batch->count; ++i) {
    a[i] = batch->items + batch->off[i];
    if ((st = host_validate_items(batch->C[i], a[i], pin[i].n_in))) return st;
  }
  const bool was_timing = c->timing;
  c->timing = true;
  std::vector<bp_bounds> out(batch->count);
  auto measure = [&](const bp_tuning &t, double *ms) -> bp_status {
    c->tune = t;
    c->apply_tuning();
    double bestv = 1e300;
    for (int32_t r = 0; r < reps; ++r) {
      c->timing_reset();
      std::vector<PlanIn> p2 = pin;
      bp_status s2 = launch_host_batch(c, p2, a, b);
      if (s2) return s2;
      if ((s2 = collect_host_batch(c, batch->count, out.data(), true))) return s2;
      double t_ms[3];
      if ((s2 = c->timing_mean(t_ms, nullptr))) return s2;
      bestv = std::min(bestv, t_ms[1]);
    }
    *ms = bestv;
    return BP_OK;
  };
  bp_tuning cur = c->tune;
  double cur_ms = 0;
  if ((st = measure(cur, &cur_ms))) { c->timing = was_timing; return st; }
  const int32_t lpls[] = {1, 2, 4};
  const int32_t waves[] = {8, 16, 24, 32};
  const int32_t tasks[] = {1, 2, 4, 8, 16, 32, 64};
  const int32_t chunks[] = {128, 384, 1024, 4096};
  for (int knob = 0; knob < 4; ++knob) {
    const int32_t *vals = knob == 0 ? lpls : knob == 1 ? waves : knob == 2 ? tasks : chunks;
    const int nv = knob == 0 ? 3 : knob == 1 ? 4 : knob == 2 ? 7 : 4;
    for (int v = 0; v < nv; ++v) {
      bp_tuning t = cur;
      int32_t *field = knob == 0 ? &t.lanes_params : knob == 1 ? &t.waves_per_cu : knob == 2 ? &t.tasks_per_wave : &t.min_chunk;
      if (*field == vals[v]) continue;
      *field = vals[v];
      double ms = 0;
      if ((st = measure(t, &ms))) { c->timing = was_timing; return st; }
      if (ms < cur_ms) {
        cur_ms = ms;
        cur = t;
      }
    }
  }
  c->timing = was_timing;
  c->timing_reset();
  c->tune = cur;
  c->apply_tuning();
  if (best) *best = cur;
  if (best_ms) *best_ms = cur_ms;
  return BP_OK;
}

static int64_t pow2_ceil64(int64_t x) {
  int64_t p = 1;
  while (p < x && p < (int64_t(1) << 62)) p <<= 1;
  return p;
}

// Shape key of a batch for the tuning cache (no spaces).
static std::string batch_key(const bp_batch *b, const bp_sweep *per) {
  std::vector<int64_t> caps;
  for (int32_t i = 0; i < b->count; ++i) {
    const int64_t c = pow2_ceil64(b->C[i]);
    if (std::find(caps.begin(), caps.end(), c) == caps.end()) caps.push_back(c);
  }
  std::sort(caps.begin(), caps.end());
  if (caps.size() > 8) caps.resize(8);
  uint32_t flags = 0;
  if (per)
    for (int32_t i = 0; i < b->count; ++i) flags |= per[i].flags;
  char buf[64];
  std::string key = "n" + std::to_string(pow2_ceil64(b->count)) + ".r" +
                    std::to_string(pow2_ceil64(b->count ? b->off[b->count] : 0)) + ".c";
  for (size_t i = 0; i < caps.size(); ++i) key += (i ? "-" : "") + std::to_string(caps[i]);
  snprintf(buf, sizeof buf, ".f%u", flags);
  return key + buf;
}

bp_status bp_autotune_batch_cached(bp_ctx *ctx, const bp_batch *batch, const bp_sweep *per_inst, int32_t reps,
                                   const char *cache_path, bp_tuning *best, double *best_ms, int32_t *from_cache) {
  Ctx *c;
  bp_status st = get_ctx(ctx, &c);
  if (st) return st;
  if ((st = check_batch(batch))) return st;
  if (batch->count == 0 || !batch->items) return fail(BP_ERR_ARG, "empty batch");
  const std::string key = batch_key(batch, per_inst);
  if (from_cache) *from_cache = 0;
  if (cache_path) {
    FILE *f = fopen(cache_path, "r");
    if (f) {
      char line[512];
      bp_tuning t;
      double ms = 0;
      bool found = false;
      while (fgets(line, sizeof line, f)) {
        char k[256];
        bp_tuning u;
        double v = 0;
        if (sscanf(line, "%255s %d %d %d %d %lf", k, &u.lanes_params, &u.waves_per_cu, &u.tasks_per_wave,
                   &u.min_chunk, &v) == 6 &&
            key == k && check_tuning(&u) == BP_OK) {
          t = u;  // the last matching line wins
          ms = v;
          found = true;
        }
      }
      fclose(f);
      if (found) {
        if ((st = c->wait_staging())) return st;
        c->tune = t;
        c->apply_tuning();
        if (best) *best = t;
        if (best_ms) *best_ms = ms;
        if (from_cache) *from_cache = 1;
        return BP_OK;
      }
    }
  }
  bp_tuning t;
  double ms = 0;
  if ((st = bp_autotune_batch(ctx, batch, per_inst, reps, &t, &ms))) return st;
  if (best) *best = t;
  if (best_ms) *best_ms = ms;
  if (cache_path) {
    FILE *f = fopen(cache_path, "a");
    if (!f) return fail(BP_ERR_ARG, "cannot append to the tuning cache %s", cache_path);
    fprintf(f, "%s %d %d %d %d %.6f\n", key.c_str(), t.lanes_params, t.waves_per_cu, t.tasks_per_wave, t.min_chunk, ms);
    fclose(f);
  }
  return BP_OK;
}

// ---- self test --------------------------------------------------------------

int64_t bp_selftest_division(uint32_t d_lo, uint32_t d_hi, uint32_t n_hi, uint32_t mode) {
  if (d_lo < 1 || d_hi < d_lo || d_hi >= 0x80000000u || n_hi >= 0x80000000u) return BP_ERR_ARG;
  int64_t bad = 0;
  if (mode == 0) {
    // floor(n / d) for n < 2^31 by family (1)
    for (uint64_t d = d_lo; d <= d_hi; ++d) {
      const MagicU31 g = magic_u31((uint32_t)d);
      auto one = [&](uint64_t n) {
        if (n >= 0x80000000ull) return;
        if (div_u31((uint32_t)(2 * n), g.m, g.s) != (uint32_t)(n / d)) ++bad;
      };
      for (uint64_t n = 0; n <= n_hi; ++n) one(n);
      for (uint64_t k = 1; k <= 64; ++k) {
        const uint64_t mult = d * k;
        one(mult - 1);
        one(mult);
        one(mult + 1);
      }
      const uint64_t q = 0x7fffffffull / d;
      for (int64_t t = -2; t <= 2; ++t) {
        one(q * d + t);
        one(0x7fffffffull - (uint64_t)(t + 2));
      }
    }
  } else if (mode == 1) {
    // ceil(a lam / c) - 1 by family (2): c in [d_lo, d_hi], lam in [1, c], a in [1, c] (a capped at n_hi + edges)
    for (uint64_t c = d_lo; c <= d_hi; ++c) {
      const uint64_t lam_step = c > 4096 ? c / 4096 : 1;
      for (uint64_t lam = 1; lam <= c; lam += (lam < 64 || c - lam < 64) ? 1 : lam_step) {
        const uint64_t R = vb2_recip((uint32_t)lam, (uint32_t)c);
        auto one = [&](uint64_t a) {
          if (a < 1 || a > c) return;
          const unsigned __int128 p = (unsigned __int128)a * lam;
          const uint64_t want = (uint64_t)((p + c - 1) / c) - 1;
          if (vb2_part((uint32_t)a, (uint32_t)R, (uint32_t)(R >> 32)) != want) ++bad;
        };
        for (uint64_t a = 1; a <= std::min<uint64_t>(c, n_hi); ++a) one(a);
        for (uint64_t a = c > 64 ? c - 64 : 1; a <= c; ++a) one(a);
        // a where a lam / c is an integer or just past one
        for (uint64_t k = 1; k <= 32; ++k) {
          const unsigned __int128 t = (unsigned __int128)k * c;
          if (t % lam == 0) {
            const uint64_t a = (uint64_t)(t / lam);
            one(a - 1);
            one(a);
            one(a + 1);
          } else {
            const uint64_t a = (uint64_t)(t / lam);
            one(a);
            one(a + 1);
          }
        }
      }
    }
  } else if (mode == 2) {
    // d | n by family (3): d in [d_lo, d_hi], n in [0, n_hi], around multiples of d and below 2^31
    for (uint64_t d = d_lo; d <= d_hi; ++d) {
      const uint64_t M = divides_const((uint32_t)d);
      auto one = [&](uint64_t n) {
        if (n >= 0x80000000ull) return;
        if (divides_u32((uint32_t)n, M) != (n % d == 0)) ++bad;
      };
      for (uint64_t n = 0; n <= n_hi; ++n) one(n);
      for (uint64_t k = 1; k <= 64; ++k) {
        one(d * k - 1);
        one(d * k);
        one(d * k + 1);
      }
      const uint64_t q = 0x7fffffffull / d;
      for (uint64_t t = 0; t <= 4; ++t) {
        one(q * d + t - 2);
        one(0x7fffffffull - t);
      }
    }
  } else if (mode == 3) {
    // floor(n / d) by family (4): every d in [d_lo, d_hi], n in [0, n_hi], around multiples of d and below 2^31
    for (uint64_t d = d_lo; d <= d_hi; ++d) {
      const double rd = 1.0 / (double)d;
      auto one = [&](uint64_t n) {
        if (n >= 0x80000000ull) return;
        if (fdiv_u31((uint32_t)n, (uint32_t)d, rd) != (uint32_t)(n / d)) ++bad;
      };
      for (uint64_t n = 0; n <= n_hi; ++n) one(n);
      for (uint64_t k = 1; k <= 64; ++k) {
        one(d * k - 1);
        one(d * k);
        one(d * k + 1);
      }
      const uint64_t q = 0x7fffffffull / d;
      for (uint64_t t = 0; t <= 4; ++t) {
        one(q * d + t - 2);
        one(0x7fffffffull - t);
      }
    }
  } else if (mode == 4) {
    // floor(N / c) by family (4) for N = a lam - 1 < c^2: c in [d_lo, d_hi], lam and a near 1, near c and
    // where a lam is a multiple of c or one off
    for (uint64_t c = d_lo; c <= d_hi; ++c) {
      const double rc = 1.0 / (double)c;
      auto one = [&](uint64_t a, uint64_t lam) {
        if (a < 1 || a > c || lam < 1 || lam > c) return;
        const int64_t N = (int64_t)(a * lam) - 1;
        if (fdiv_u62(N, (int64_t)c, rc) != N / (int64_t)c) ++bad;
      };
      const uint64_t lams[] = {1, 2, 3, c / 3 + 1, c / 2, c / 2 + 1, c - 2, c - 1, c};
      for (uint64_t lam : lams) {
        if (lam < 1 || lam > c) continue;
        for (uint64_t a = 1; a <= std::min<uint64_t>(c, n_hi); ++a) one(a, lam);
        for (uint64_t a = c > 64 ? c - 64 : 1; a <= c; ++a) one(a, lam);
        for (uint64_t k = 1; k <= 64; ++k) {
          const uint64_t a = (k * c) / lam;
          one(a, lam);
          one(a + 1, lam);
          if (a > 1) one(a - 1, lam);
        }
      }
    }
  } else if (mode == 5) {
    // floor(n / d) by family (5a) where n d <= 2^32: every d in [max(d_lo, 2), d_hi], n in [0, n_hi] under
    // that limit, the multiples of d around it and the limit itself
    for (uint64_t d = std::max<uint64_t>(d_lo, 2); d <= d_hi; ++d) {
      const uint32_t m = magic_short((uint32_t)d);
      const uint64_t lim = (1ull << 32) / d;  // the largest n with n d <= 2^32
      auto one = [&](uint64_t n) {
        if (n > lim) return;
        if (div_short((uint32_t)n, m) != (uint32_t)(n / d)) ++bad;
      };
      for (uint64_t n = 0; n <= n_hi; ++n) one(n);
      for (uint64_t k = 1; k <= 64; ++k) {
        one(d * k - 1);
        one(d * k);
        one(d * k + 1);
      }
      const uint64_t q = lim / d;
      for (uint64_t t = 0; t <= 4; ++t) {
        if (q * d + t >= 2) one(q * d + t - 2);
        if (q >= t && (q - t) * d > 0) {
          one((q - t) * d - 1);
          one((q - t) * d);
        }
        if (lim >= t) one(lim - t);
      }
    }
  } else if (mode == 6) {
    // ceil(a lam / c) - 1 by family (5b) where a c <= 2^32: c in [d_lo, d_hi], lam as in mode 1, a up to
    // that limit (capped at n_hi, plus the top of the range and a where a lam / c is an integer or one off)
    for (uint64_t c = d_lo; c <= d_hi; ++c) {
      const uint64_t alim = std::min<uint64_t>(c, (1ull << 32) / c);
      const uint64_t lam_step = c > 4096 ? c / 4096 : 1;
      for (uint64_t lam = 1; lam <= c; lam += (lam < 64 || c - lam < 64) ? 1 : lam_step) {
        const uint64_t R = vb2_recip((uint32_t)lam, (uint32_t)c);
        auto one = [&](uint64_t a) {
          if (a < 1 || a > alim) return;
          const unsigned __int128 p = (unsigned __int128)a * lam;
          const uint64_t want = (uint64_t)((p + c - 1) / c) - 1;
          if (vb2_part_short((uint32_t)a, (uint32_t)(R >> 32)) != want) ++bad;
        };
        for (uint64_t a = 1; a <= std::min<uint64_t>(alim, n_hi); ++a) one(a);
        for (uint64_t a = alim > 64 ? alim - 64 : 1; a <= alim; ++a) one(a);
        for (uint64_t k = 1; k <= 64; ++k) {
          const unsigned __int128 t = (unsigned __int128)k * c;
          const uint64_t a = (uint64_t)(t / lam);
          one(a);
          one(a + 1);
          if (a > 1) one(a - 1);
          // the same near the limit
          const uint64_t kk = (uint64_t)(((unsigned __int128)alim * lam) / c);
          if (kk >= k) {
            const uint64_t b = (uint64_t)(((unsigned __int128)(kk - k + 1) * c) / lam);
            one(b);
            one(b + 1);
            if (b > 1) one(b - 1);
          }
        }
      }
    }
  } else {
    return BP_ERR_ARG;
  }
  return bad;
}

