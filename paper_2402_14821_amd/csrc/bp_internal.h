// bp_internal.h -- data layout shared by the host planner and the gfx950 kernels.
//
// One "launch" checks a batch of instances (a single check is a batch of one).
// Everything a kernel needs is reached from one device-resident LaunchDesc,
// so the captured HIP graph of the pipeline is reused for every call: the
// host rewrites the descriptor and the inputs, then replays the graph.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/bp.h"

namespace bpi {

enum : int { kL1 = 0, kL2, kMT, kRAD2, kFS1, kCCM1, kVB2, kBJ1, kNB };

constexpr int kWave = 64;
// Task counters of the persistent sweep: kQueues of them, kQueueStride
// 64-bit words (256 bytes) apart so that each sits in its own cache line and
// memory channel.
constexpr int kQueues = 8;
constexpr int kQueueStride = 32;
// Split tiles are combined in segments of kSegTiles consecutive tiles of one
// entry, a block (one wave per tile) per segment.
constexpr int kSegTiles = 8;
// Largest K = floor(c / lambda) a segment tile of BJ1 handles (2K windows).
constexpr int kSegMaxK = 64;
constexpr int kSegQPerChunk = 8;  // q values per chunk of a split BJ1/CCM1 segment tile
// Windowed BJ1/CCM1 segment tiles in a single check only for instances of
// at least this many items: below it their chains of dependent loads take
// longer than the dense tiles' fuller machine (measured at c = 10^6 with
// r = 366 and 1 335: BJ1 142 vs 123 us, 226 vs 213 us; CCM1 104 vs 73 us,
// 126 vs 98 us).  A launch of several instances keeps them: there the total
// work decides (the uneven batch of 4 096 checks: 0.085 s against 0.19 s).
constexpr int64_t kSegWindowMinItems = 8192;
constexpr int kSmallThreads = 256;      // prep block for small instances
constexpr int kSmallCap = 8192;         // items per small-instance prep block (LDS resident)
constexpr int kTinyCap = 2048;          // the same block's short form, for launches whose small instances fit it
constexpr int kLargeThreads = 1024;      // prep block for one large instance
constexpr int kLargeCap = 16384;        // items per large-instance prep block (LDS resident)
static_assert(kLargeCap <= BP_MAX_ITEMS, "the block prep's capacity is within the check's item limit");
// Value-table prep (two kernels over the whole GPU instead of one
// block): a count per size value, suffix-scanned into #{w >= v} and
// sum{w : w >= v}, from which the sorted sizes, their prefix sums, the class
// bounds and the threshold tables are read off, and which the lookup tiles
// of BJ1 and CCM1 read.  Used for c at most kVtMaxC when the instance is
// large and c is at most kVtRatio times its reduced count (the tables hold
// c + 2 entries).
constexpr int kVtChunk = 2048;           // values per block of the suffix scan (2^kVtChunkLog)
constexpr int kVtThreads = 512;
constexpr int32_t kVtMaxC = 1 << 21;
constexpr int64_t kVtRatio = 16;
constexpr int kVtMaxChunks = (kVtMaxC + 2 + kVtChunk - 1) / kVtChunk;
// An instance of r reduced items fits a check when the block prep takes it
// (r <= kLargeCap) or the value-table prep does (c <= kVtMaxC, c <= kVtRatio r),
// up to BP_MAX_ITEMS.
inline bool instance_fits(int32_t C, int64_t r) {
  return r <= kLargeCap || (r <= BP_MAX_ITEMS && C <= kVtMaxC && (int64_t)C <= kVtRatio * r);
}
// most bytes of split-tile partial sums one launch may use
constexpr int64_t kMaxAccBytes = int64_t(1) << 30;

// Input form of an instance.
enum : int32_t { kFormItems = 0, kFormResidual = 1 };

// Per-instance plan, written by the host, read-only on the device.
struct InstPlan {
  int64_t in_off;    // items form: offset of items[]; residual form: offset of unpacked[]
  int64_t res_off;   // residual form: offset of residual[] (int32) in the residual arena (LaunchDesc::in2)
  int64_t n_in;      // items form: r; residual form: number of unpacked items
  int64_t k;         // bins
  int64_t ws_off;    // offset of this instance's slice of the per-item workspaces
  int64_t pre_off;   // offset of this instance's prefix-sum slice (r_cap + 1 entries)
  int64_t lo[kNB];   // parameter ranges (lo > hi: empty)
  int64_t hi[kNB];
  int32_t m_res;     // residual form: number of bins given as residuals
  int32_t C;
  int32_t form;
  int32_t r_cap;     // n_in + m_res: upper bound of the reduced count
  uint32_t flags;    // kPlanClampVB2 | kPlanEarlyExit | kPlanSegments
  int32_t large;     // 1: prepared by the large-instance block; 2: by the value-table kernels
  int32_t bshift;    // kPlanSegments: bucket width 2^bshift of the threshold table
  int32_t nbk;       // kPlanSegments: entries of the threshold table
  int64_t bidx_off;  // kPlanSegments: offset of the threshold table
  int64_t div_off;   // ndiv > 0: offset of the divisors of c (ascending) in the divisor list
  int64_t dc_off;    // ndiv > 0: offset of the multiple counts [small x ndiv][big x ndiv]
  int32_t ndiv;      // divisors of c listed for the mirrored VB2 tiles (0: none)
  int32_t pad2;
  int64_t state_off; // >= 0: the instance's node state (see node_layout) at LaunchDesc::nodes + state_off
  int64_t vt_off;    // large == 2: offset of the c + 2 value-table entries (LaunchDesc::vraw, vcnt, vsum)
  int64_t vtt_off;   // large == 2: offset of the chunk totals, then the chunk offsets (2 x 2 x chunks, LaunchDesc::vtot)
  int64_t vl_off;    // large == 2, ndiv > 0: offset of the 2 x ndiv lattice bins (LaunchDesc::vlat)
};
constexpr uint32_t kPlanClampVB2 = 1u;
constexpr uint32_t kPlanEarlyExit = 2u;
constexpr uint32_t kPlanSegments = 4u;

// How an entry's tiles compute their sums: one evaluation per (item,
// parameter), or threshold sums over windows of the sorted sizes.
// kModeMirror (VB2): each lane's dense sum at lambda also gives the sum at
// c - lambda.
// kModeL2State: tiles over every lambda in [0, c/2] that store the L2
// aggregates of the node state (no maximum).
// kModeLookup (BJ1, CCM1 of value-table instances): each lane walks its own
// thresholds q lambda and c - q lambda and reads #{w >= t} and sum{w >= t}
// from the value tables.
// kModeCand (MT, RAD2): tiles over candidate indices, as L2's: the range's
// first parameter and the points where a size crosses one of the function's
// thresholds, each evaluated from counts and prefix sums of the sorted sizes.
enum : int32_t { kModeDense = 0, kModeSegments = 1, kModeMirror = 2, kModeL2State = 3, kModeLookup = 4,
                 kModeCand = 5 };
constexpr int kVtChunkLog = 11;  // kVtChunk = 2^kVtChunkLog
constexpr int kLutQPerChunk = 8;  // q values per chunk of a split lookup tile (each a chain of table loads)
constexpr int kMaxDivs = 256;         // most divisors of c a mirrored instance may have
constexpr int kMirrorMinItems = 256;  // fewer items: the per-parameter gcd outweighs the saved half

// Per-instance state, written by the prep kernel.
struct InstState {
  int64_t sumW;      // sum of all reduced sizes
  int64_t sumBig;    // sum over big, not full items (c/2 < w < c)
  int64_t sumNZ;     // sum over items with 0 < w < c
  int64_t hiEff[kNB];// effective upper ends (the VB2 cut applied)
  int32_t r;         // reduced item count
  int32_t nf;        // [0, nf) items of size c
  int32_t nb;        // [nf, nb) big: c/2 < w < c
  int32_t nm;        // [nb, nm) mid: 2w = c
  int32_t nz;        // [nm, nz) small: 0 < 2w < c ; [nz, r) zero
  int32_t maxw;
  int32_t status;    // BP_OK or an error found on the device
  int32_t pad;
  unsigned long long evals_skipped;  // (item, parameter) evaluations of the tiles an early exit skipped
};

// One (instance, bound) entry of the sweep schedule.  Its parameter range is
// cut into tiles of 64 x (parameters per lane) parameters.  A task is either
// tpt consecutive tiles over all items (nchunks = 1) or one of nchunks item
// chunks of one tile ("split" tile), whose per-parameter partial sums go to a
// slot of their own and are added up by the combine kernel.
struct Entry {
  int64_t task_begin;   // prefix of task counts over entries (schedule order)
  int64_t lam0;         // first parameter of the entry
  int64_t ntiles;
  int64_t acc_base;     // nchunks > 1: first partial-sum slot, laid out [tile][chunk][parameter]
  int64_t split_base;   // combine segments of the entries before this one
  int32_t inst;
  int32_t bound;        // kL2 .. kBJ1
  int32_t tpt;          // tiles per task
  int32_t nchunks;      // item chunks per tile
  int32_t mode;         // kModeDense, kModeSegments, kModeMirror, ...
  int32_t aux;          // kModeMirror: last parameter of the dense half
  int32_t slot32;       // nchunks > 1: the slots hold int32 (every chunk's partial sum fits), else int64
  int32_t pad;
};

struct LaunchDesc {
  // inputs
  const int32_t *in;        // input arena: items, or the unpacked sizes of residual-form instances
  const int32_t *in2;       // residual arena: the residual capacities of residual-form instances
  const InstPlan *plan;
  const Entry *entries;
  // workspaces
  InstState *state;
  int32_t *sorted;          // per-item, descending sizes
  int64_t *pre;             // prefix sums of sorted sizes
  uint32_t *av;             // per item: c - w for big items, w otherwise
  unsigned long long *keys; // [count][kNB] packed (value, parameter) maxima
  int32_t *refuted;         // [count] early-exit flags
  unsigned long long *counter; // kQueues task counters of the persistent sweep, kQueueStride apart
  long long *acc;           // partial sums of split tiles, one slot per (tile, chunk, parameter)
  int32_t *bidx;            // threshold tables: bidx[b] = #{sorted sizes >= b 2^bshift}
  const int32_t *divs;      // per mirrored instance: divisors of c (ascending), their lattice bins, prime count, (prime, exponent) pairs, prime-power count, test constants
  int32_t *dcnt;            // per divisor d: #{small sizes divisible by d}, then the same for big sizes
  long long *nodes;         // node-state arena of served requests (InstPlan::state_off)
  int32_t *vraw;            // value tables (large == 2): count per size value; zero between launches
  int32_t *vcnt;            //   #{w >= v} within the chunk of kVtChunk values (written whole by each launch)
  long long *vsum;          //   sum{w >= v} within the chunk (likewise)
  long long *vtot;          //   per chunk: (count, sum) totals, then (count, sum) of the chunks above it; zero between launches
  int32_t *vlat;            //   divisor-lattice bins of the mirrored VB2; zero between launches
  int32_t *vflag;           //   per listed instance: [an input outside [0, c] was seen, largest size]; zero between launches
  const int32_t *vlist;     //   the instances prepared this way
  int64_t nvt;
  bp_bounds *out;           // [count] results
  int64_t count;            // instances
  int64_t nentries;
  int64_t ntasks;
  int64_t acc_len;
  int64_t nsplit;           // combine segments (kSegTiles split tiles each) over all entries
};

// Node state of a served request (incremental serving): everything the
// bounds of the collection need, as sums over the reduced items that are
// additive in the items, so that a node one commit away from another has
// its state from the other's plus the changed items' terms.  Per bound, in
// the order L2, MT, RAD2, FS1, CCM1, VB2, BJ1, over the paper's ranges
// (Sec. 3.1), int64:
//   L2    lambda in [0, c/2]: n1(lambda) = #{w > c - lambda}, then
//         T(lambda) = sum of the sizes in W2 and W3 (c/2 < w <= c - lambda,
//         or lambda <= w <= c/2); L2(I, lambda) = nbig + max(0, ceil((T -
//         c (nbig - n1)) / c)) with nbig = #{2w > c};
//   DFF f S_f(lambda) = sum_w f(w, lambda) for lambda in its range.
// node_len(C, b) is the number of elements of bound b, node_off(C, b) its
// first element; node_layout fills off[b] = node_off(C, b), off[kNB] = the
// length.  (No arrays in the functions the kernels call: a runtime-indexed
// array would be placed in per-lane scratch memory.)
__host__ __device__ inline int64_t node_len(int32_t C, int b) {
  const int64_t c = C;
  switch (b) {
    case kL2: return 2 * (c / 2 + 1);
    case kMT: return c / 2 + 1;
    case kRAD2: return c / 3 > c / 4 ? c / 3 - c / 4 : 0;
    case kFS1: return 100;
    case kCCM1: return c / 2;
    case kVB2: return c > 1 ? c - 1 : 0;
    case kBJ1: return c;
    default: return 0;
  }
}

__host__ __device__ inline int64_t node_off(int32_t C, int bound) {
  int64_t o = 0;
  for (int b = kL2; b < bound; ++b) o += node_len(C, b);
  return o;
}

__host__ __device__ inline void node_layout(int32_t C, int64_t off[kNB + 1]) {
  off[0] = 0;
  for (int b = 0; b < kNB; ++b) off[b + 1] = off[b] + node_len(C, b);
}

// A served request computed from another node's state (the base) and the
// items by which its reduced instance differs from the base's.
struct NodeTask {
  int64_t base_off;    // node state of the base (LaunchDesc::nodes + base_off)
  int64_t dst_off;     // where this request's node state goes (-1: not kept)
  int64_t tile_begin;  // prefix of node_tiles() over the tasks of the launch
  int64_t sumW;        // total size of the request's reduced items
  int64_t r;           // their count
  int64_t k;           // bins
  int32_t C;
  int32_t nbig;        // #{2w > c} among them
  int32_t d_off;       // changed items: delta[d_off .. d_off + nd), v > 0 adds a size v - 1,
  int32_t nd;          //   v < 0 removes a size -v - 1
  int32_t out_idx;     // record index in the launch's output
  int32_t pad;
};

// Parameters handled by one block of the served-child kernel, and the
// per-bound tile counts: tb[b] is the first tile of bound b, tb[kNB] the
// total (L2 tiles cover lambda in [0, c/2], both aggregates).
constexpr int kNodeTile = 256;
// Parameters of bound b in one node state (L2: lambda in [0, c/2]).
__host__ __device__ inline int64_t node_params(int32_t C, int b) {
  return b == kL2 ? node_len(C, b) / 2 : node_len(C, b);
}

__host__ __device__ inline int64_t node_tile_count(int32_t C, int b) {
  return (node_params(C, b) + kNodeTile - 1) / kNodeTile;
}

__host__ __device__ inline int64_t node_tiles(int32_t C) {
  int64_t n = 0;
  for (int b = kL2; b < kNB; ++b) n += node_tile_count(C, b);
  return n;
}

// Small checks in one launch (k_small_check, then k_small_final): the
// instance travels in the kernel arguments, the workgroups split the (bound,
// parameter) pairs and write their maxima, and a one-workgroup kernel after
// them writes the record to host memory.  Used for at most kSmallFusedMax
// input values and at most Ctx::small_work (item, parameter) evaluations.
constexpr int kSmallFusedMax = 960;
constexpr int64_t kSmallFusedWork = int64_t(1) << 26;  // below the pipeline's time up to about 1e8 evaluations
constexpr int kSmallFusedThreads = 1024;  // per workgroup
constexpr int kSmallFusedMaxGrid = 2048;
// what workgroup 0 of k_small_check leaves for k_small_final
struct SmallHead {
  uint64_t tot_w;  // sum of the reduced sizes
  int64_t evals;   // r x the DFF parameters after any VB2 cut
  int32_t r;
  int32_t bad;     // a size or residual outside [0, C]
};
// Checks whose pairs fit in kSmallOneMaxGrid workgroups of kSmallOneThreads
// fold their maxima by atomics in one kernel (k_small_check<true>); larger
// ones run workgroups of kSmallFusedThreads and add k_small_final.
constexpr int kSmallOneThreads = 256;
constexpr int kSmallOneMaxGrid = 64;
// the buffer: kNB keys per workgroup, the head, then the one-kernel keys and
// count (kNB + 1 words, zero between calls)
constexpr size_t kSmallBufBytes =
    sizeof(unsigned long long) * kNB * kSmallFusedMaxGrid + sizeof(SmallHead) + sizeof(unsigned long long) * (kNB + 1);
struct SmallArgs {
  int32_t C;
  int32_t m;       // residual form: bins given as residuals (after the n sizes)
  int32_t n;       // sizes
  int32_t form;    // kFormResidual or kFormItems
  int64_t k;
  int64_t lo[kNB];
  int64_t hi[kNB];
  uint32_t clamp;  // the paper's VB2 cut
  int32_t slices;  // lanes per (bound, parameter) pair: a power of two, 1 .. 64
  int32_t v[kSmallFusedMax];  // the n sizes, then (residual form) the m residuals
};
static_assert(sizeof(SmallArgs) <= 4096, "kernel arguments are limited to 4 KiB");

// Allocation-free check (bp_feasible_dev_noalloc): the tables and every
// workspace of a one-instance launch inside one file-scope device array per
// GPU, at the fixed offsets below.  The rest of the array holds the partial
// sums of split tiles.
constexpr size_t kNoAllocScratchBytes = size_t(BP_NOALLOC_SCRATCH_BYTES);
constexpr int kNoAllocMaxEntries = 8;  // one instance, dense sweeps: L2 + six functions
constexpr int kNoAllocMaxDevices = 64;
struct NoAllocTables {
  LaunchDesc d;
  InstPlan p;
  Entry e[kNoAllocMaxEntries];
};
constexpr size_t na_align(size_t x) { return (x + 255) & ~size_t(255); }
constexpr size_t kNaState = na_align(sizeof(NoAllocTables));
constexpr size_t kNaKeys = kNaState + na_align(sizeof(InstState));
constexpr size_t kNaRefuted = kNaKeys + na_align(sizeof(unsigned long long) * kNB);
constexpr size_t kNaCounter = kNaRefuted + na_align(sizeof(int32_t));
constexpr size_t kNaSorted = kNaCounter + na_align(sizeof(unsigned long long) * kQueues * kQueueStride);
constexpr size_t kNaAv = kNaSorted + na_align(sizeof(int32_t) * size_t(BP_NOALLOC_MAX_ITEMS));
constexpr size_t kNaPre = kNaAv + na_align(sizeof(uint32_t) * size_t(BP_NOALLOC_MAX_ITEMS));
constexpr size_t kNaAcc = kNaPre + na_align(sizeof(int64_t) * (size_t(BP_NOALLOC_MAX_ITEMS) + 1));
constexpr int64_t kNaAccSlots = int64_t((kNoAllocScratchBytes - kNaAcc) / sizeof(long long));
static_assert(kNaAcc < kNoAllocScratchBytes / 2, "the partial-sum slots keep most of the array");
static_assert(BP_NOALLOC_MAX_ITEMS <= kLargeCap, "the prep kernels bound the item count");

}  // namespace bpi
