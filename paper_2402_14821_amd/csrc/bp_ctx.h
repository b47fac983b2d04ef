// bp_ctx.h -- host-side context of libbp (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <unordered_map>
#include <vector>

#include "bp_internal.h"

namespace bpi {

constexpr uint64_t kCtxMagic = 0x6270637478303031ull;

bp_status fail(bp_status st, const char *fmt, ...);
bp_status hip_fail(hipError_t e, const char *what);
void default_ranges(int32_t C, int64_t lo[kNB], int64_t hi[kNB]);

// kernels (bp_kernels.hip)
hipError_t set_kernel_attrs();
hipError_t launch_pipeline(const LaunchDesc *d_desc, int lpl, int grid_prep_small, int grid_prep_large, int grid_vt,
                           int grid_sweep, int grid_comb, int grid_fin, int v, hipStream_t s);
hipError_t launch_pipeline_timed(const LaunchDesc *d_desc, int lpl, int grid_prep_small, int grid_prep_large,
                                 int grid_vt, int grid_sweep, int grid_comb, int grid_fin, int v, hipStream_t s,
                                 hipEvent_t ev[4]);
hipError_t launch_node_delta(const NodeTask *tasks, int64_t ntasks, int64_t ntiles, const int32_t *delta,
                             long long *nodes, unsigned long long *keys, bp_bounds *out, int grid, hipStream_t s);
hipError_t launch_small_check(const SmallArgs &a, bool one, int grid, void *buf, bp_bounds *out, uint32_t *seq_out,
                              uint32_t seq, hipStream_t s);
hipError_t noalloc_scratch(int device, unsigned char **out);
hipError_t launch_noalloc(const NoAllocTables &t, unsigned char *base, int lpl, int grid_prep_small,
                          int grid_prep_large, int grid_sweep, int grid_comb, int grid_fin, int v, hipStream_t s);
hipError_t launch_reduce(int32_t C, int32_t m, const int32_t *residual, const int32_t *size, const int32_t *bin_of,
                         int64_t n, unsigned long long *loads, int32_t *out, int64_t *out_r, int32_t *out_residual,
                         int32_t *bad, hipStream_t s);

struct DevBuf {
  void *p = nullptr;
  size_t cap = 0;
  bp_status reserve(size_t bytes);
  void release();
};

struct HostBuf {
  void *p = nullptr;
  size_t cap = 0;
  bp_status reserve(size_t bytes);
  void release();
};

// One instance as the planner sees it.
struct PlanIn {
  int64_t in_off, res_off, n_in, k;
  int64_t lo[kNB], hi[kNB];
  int32_t m_res, C, form;
  bool early_exit, clamp, segments;
  int64_t state_off;  // >= 0: write the node state there (served requests); -1: none
};

struct Ctx {
  uint64_t magic = 0;
  int device = -1;
  int num_cu = 0;
  hipStream_t stream = nullptr;
  hipEvent_t staged = nullptr;  // staging buffers consumed by the device
  hipEvent_t done = nullptr;
  // End of the last launch queued by run(), on whatever stream it went to.
  // The next run() makes its stream wait for it before rewriting the
  // descriptor, the tables and the workspaces the launch still reads, and
  // the host waits for it before a workspace is reallocated or a captured
  // graph destroyed.
  hipEvent_t last_run = nullptr;
  bool any_run = false;
  bool use_graph = true;
  int seg_kcut = -1;  // BJ1 segment tiles for K <= seg_kcut; -1: chosen by the cost model
  int64_t lut_kcut = -1;  // lookup tiles for K <= lut_kcut (BP_LUT_KCUT); -1: chosen by the cost model
  int lut_qchunk = kLutQPerChunk;  // q values per chunk of a lookup tile (BP_LUT_QCHUNK)
  bool timing = false;
  // Stage timing: one set of 4 events per timed run, reused round-robin; a
  // set is folded into the sums (waiting for it) before it is reused.
  static constexpr int kTimingRing = 64;
  hipEvent_t tev[kTimingRing][4] = {};
  int64_t t_runs = 0, t_folded = 0;
  double t_sum[3] = {0, 0, 0};
  // Grids and kernels of one launch: variant bit 0 = large-instance prep
  // block, bit 1 = combine, bit 2 = the short small-instance prep; vt = grid
  // of the value-table prep (0: none);
  // each grid at most the machine-filling size of its kernel.
  struct LaunchShape {
    int v, lpl, prep_small, prep_large, vt, sweep, comb, fin;
    bool operator<(const LaunchShape &o) const {
      const int a[8] = {v, lpl, prep_small, prep_large, vt, sweep, comb, fin};
      const int b[8] = {o.v, o.lpl, o.prep_small, o.prep_large, o.vt, o.sweep, o.comb, o.fin};
      for (int i = 0; i < 8; ++i)
        if (a[i] != b[i]) return a[i] < b[i];
      return false;
    }
  };
  struct GraphPair {
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
  };
  std::map<LaunchShape, GraphPair> graphs;  // captured pipelines by shape
  std::map<LaunchShape, uint64_t> graph_used;  // last use (run counter) of each cached graph
  uint64_t run_count = 0;
  bp_tuning tune = {2, 32, 32, 2048};  // parameters per lane, waves per CU, tasks per wave, min chunk
  int32_t order_rank[kNB] = {};         // schedule rank of each function (bp_ctx_set_order); all 0: longest first
  int grid_sweep = 0, grid_prep_small = 0, grid_prep_large = 0, grid_comb = 0, grid_fin = 0;
  void drop_graphs();
  LaunchShape shape_of(int64_t count, int64_t ntasks) const;
  int64_t ws_items = 0, pre_items = 0, bidx_items = 0, dcnt_items = 0, nentries = 0, acc_len = 0, nsplit = 0;
  // value-table prep (InstPlan::large == 2): table entries, chunk words and
  // lattice bins of this launch, its instances, and whether the planner may
  // choose it (BP_NO_VALUE_PREP=1 at context creation: never)
  int64_t vt_items = 0, vtt_items = 0, vl_items = 0;
  std::vector<int32_t> vt_list;
  bool value_prep = true;
  bool vt_dirty = false;  // a launch with value tables was not queued whole: clear them before the next
  std::vector<int32_t> div_vec;  // divisor lists of this launch (staged with the plan)
  // divisors of c by c, and c's divisor lattice: per divisor its bin
  // sum_j e_j stride_j (e_j its exponent of the j-th prime of c, stride_j =
  // prod_{i<j} (a_i + 1)), then the prime count and (prime, exponent) pairs,
  // then the prime-power count and each prime power's divisibility-test
  // constant as (low, high) halves
  struct DivInfo {
    std::vector<int32_t> divs, lattice;
  };
  std::unordered_map<int32_t, DivInfo> div_cache;
  std::vector<InstPlan> plan_vec;
  std::vector<Entry> entry_vec;

  DevBuf stage_buf, counter_buf, state_buf, sorted_buf, pre_buf, rec_buf, keys_buf, ref_buf, acc_buf, out_buf,
      red_buf, bidx_buf, dcnt_buf, vraw_buf, vcnt_buf, vsum_buf, vtot_buf, vlat_buf, vflag_buf;
  HostBuf stage_host, in_host, out_host, red_host;
  // The one-launch small check writes its record, then its sequence number,
  // to this coherent host memory: [bp_bounds][uint32 sequence].
  void *small_out = nullptr;
  uint32_t small_seq = 0;
  DevBuf small_keys;  // the small check's per-workgroup maxima and head (kSmallBufBytes)
  bool small_path = true;  // BP_NO_SMALL_PATH=1 at context creation turns the one-launch path off
  int64_t small_work = kSmallFusedWork;  // BP_SMALL_PATH_WORK=<evals> at context creation overrides
  int small_grid = 0;                    // at most this many workgroups (default: one per compute unit; BP_SMALL_GRID)
  int small_items = 8;                   // BP_SMALL_ITEMS=<items per lane>
  int small_waves = 4;                   // BP_SMALL_WAVES=<waves per SIMD the lanes may fill>

  bp_status init(int dev);
  void destroy();
  bp_status ensure_graph(const LaunchDesc *d_desc, const LaunchShape &sh, hipGraphExec_t *ex);
  bp_status plan(const std::vector<PlanIn> &pin, int64_t *ntasks_out);
  long long *nodes = nullptr;  // node-state arena for plans with state_off >= 0 (owned by a served queue)
  bp_status run(int64_t count, int64_t ntasks, const int32_t *host_in, int64_t host_in_len, const int32_t *in_dev,
                const int32_t *in2_dev, bp_bounds *out_dev, hipStream_t s);
  bp_status wait_last_run();
  bp_status reserve_dev(DevBuf &b, size_t bytes);
  bp_status wait_staging();
  void apply_tuning();
  void timing_reset();
  bp_status timing_slot(hipEvent_t **ev);
  bp_status timing_mean(double ms[3], int64_t *runs);
};

bp_status run_small(Ctx *c, const PlanIn &q, const int32_t *sizes, const int32_t *residual, bp_bounds *out,
                    bool *done);
bp_status make_plan_in(int32_t C, int64_t k, int64_t n_in, int32_t m_res, int32_t form, const bp_sweep *sw,
                       bool early, PlanIn *q, bool segments = false);
bp_status host_validate_items(int32_t C, const int32_t *items, int64_t r);
bp_status launch_host_batch(Ctx *c, std::vector<PlanIn> &pin, const std::vector<const int32_t *> &src_a,
                            const std::vector<const int32_t *> &src_b);
bp_status collect_host_batch(Ctx *c, int64_t count, bp_bounds *out, bool check_status);
bp_status run_host_batch(Ctx *c, std::vector<PlanIn> &pin, const std::vector<const int32_t *> &src_a,
                         const std::vector<const int32_t *> &src_b, bp_bounds *out);

}  // namespace bpi
