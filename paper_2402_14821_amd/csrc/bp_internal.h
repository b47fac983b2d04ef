// bp_internal.h -- data layout shared by the host planner and the gfx950 kernels.
//
// One "launch" checks a batch of instances (a single check is a batch of one).
// Everything a kernel needs is reached from one device-resident LaunchDesc,
// so the captured HIP graph of the pipeline is reused for every call: the
// host rewrites the descriptor and the inputs, then replays the graph.
#pragma once

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
constexpr int kSmallThreads = 256;      // prep block for small instances
constexpr int kSmallCap = 8192;         // items per small-instance prep block (LDS resident)
constexpr int kLargeThreads = 1024;      // prep block for one large instance
constexpr int kLargeCap = 16384;        // items per large-instance prep block (LDS resident)
static_assert(kLargeCap == BP_MAX_ITEMS, "the check's item limit is the large prep block's capacity");

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
  int32_t large;     // 1: prepared by the large-instance block
  int32_t bshift;    // kPlanSegments: bucket width 2^bshift of the threshold table
  int32_t nbk;       // kPlanSegments: entries of the threshold table
  int64_t bidx_off;  // kPlanSegments: offset of the threshold table
  int64_t div_off;   // ndiv > 0: offset of the divisors of c (ascending) in the divisor list
  int64_t dc_off;    // ndiv > 0: offset of the multiple counts [small x ndiv][big x ndiv]
  int32_t ndiv;      // divisors of c listed for the mirrored VB2 tiles (0: none)
  int32_t pad2;
};
constexpr uint32_t kPlanClampVB2 = 1u;
constexpr uint32_t kPlanEarlyExit = 2u;
constexpr uint32_t kPlanSegments = 4u;

// How an entry's tiles compute their sums: one evaluation per (item,
// parameter), or threshold sums over windows of the sorted sizes.
// kModeMirror (VB2): each lane's dense sum at lambda also gives the sum at
// c - lambda.
enum : int32_t { kModeDense = 0, kModeSegments = 1, kModeMirror = 2 };
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
  int32_t mode;         // kModeDense, kModeSegments or kModeMirror (the last two never split into chunks)
  int32_t aux;          // kModeMirror: last parameter of the dense half
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
  const int32_t *divs;      // per mirrored instance: divisors of c (ascending), their lattice bins, prime count, (prime, exponent) pairs
  int32_t *dcnt;            // per divisor d: #{small sizes divisible by d}, then the same for big sizes
  bp_bounds *out;           // [count] results
  int64_t count;            // instances
  int64_t nentries;
  int64_t ntasks;
  int64_t acc_len;
  int64_t nsplit;           // combine segments (kSegTiles split tiles each) over all entries
};

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
