// bp_kernels.hip -- gfx950 kernels of the bin_packing feasibility check.
//
// Pipeline of one launch (a batch; a single check is a batch of one):
//   k_prep  one block per instance (persistent over the batch): reduce the
//       partial packing to one capacity (Sec. 3, Fig. 3), validate, LSD radix
//       sort by decreasing size in LDS, int64 prefix sums (DPP wave scans),
//       class boundaries and sums, the class-sorted item stream.  Three
//       forms: 256 threads for up to 2 048 or 8 192 items, 1 024 threads for
//       up to 16 384.  The 256-thread form also builds the histogram of the
//       value-table instances (vt_hist).
//   k_vt_emit  value-table prep of large instances over the whole GPU: the
//       sorted sizes, prefix sums and class bounds read off per-value counts.
//   k_sweep  persistent: each wave runs task (its index) first, then claims
//       tasks (instance, bound, run of parameter tiles, or one item chunk of
//       a tile) from eight queues, its own XCD's first, in longest-first
//       order.  A tile gives each lane LPL parameters; the wave reads the
//       item stream with scalar loads (every lane uses the same item) and
//       accumulates sum_w f(w, lambda) per lane (Alg. 2's inner loop, Alg.
//       4's per-thread loop), then ceil(sum / f(c, lambda)) and a DPP wave
//       max of packed (bound, parameter) keys, one 64-bit atomic max per
//       tile.  An item chunk stores its partial sums in a slot of its own.
//       L2 tiles evaluate L2(I, lambda) at the parameters where it can
//       change (Sec. 3.1); the segment forms read threshold sums.
//   k_combine  adds the chunk slots of each split tile and finalises it.
//   k_finalize  per instance: L1, the maximum over the collection, verdict;
//       clears the value tables the launch used.
// Beside the pipeline: k_small_check (a whole small check in one launch),
// k_node_* (served children from their base's sums), k_reduce_one /
// k_bin_loads (the reductions alone), and the allocation-free variant's
// tables kernel.
//
// Class split used by the sweeps (sizes sorted decreasing):
//   [0, nf) w = c ; [nf, nb) c/2 < w < c ; [nb, nm) 2w = c ;
//   [nm, nz) 0 < 2w < c ; [nz, r) w = 0.
// Items of size c add exactly f(c, lambda) to every sum, so they add exactly 1
// to every bound and are counted, not streamed.  Zero sizes add 0 to every
// function.  Mid items (2w = c) take one fixed value per parameter.  For the
// big and small classes each function reduces to per-lane arithmetic on a
// scalar operand, written out per function below.  The quotients of CCM1,
// VB2 and BJ1 take one high multiply where the product is at most 2^32 and a
// multiply-shift or a 64-bit reciprocal otherwise; within each sorted class
// range the short form covers a prefix or a suffix (bp_divide.h).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "bp_divide.h"
#include "bp_internal.h"

namespace bpi {

// Address spaces.  Every pointer reaches the kernels through the descriptor in
// device memory, so it arrives as a generic pointer, and the compiler must
// treat loads through generic pointers as per-lane (they could address
// scratch).  Data that a kernel only reads is therefore read through the
// constant address space (scalar loads when the address is wave-uniform),
// per-lane data through the global one.
#if defined(__HIP_DEVICE_COMPILE__)
#define BP_CONST __attribute__((address_space(4)))
#define BP_GLOBAL __attribute__((address_space(1)))
#else
#define BP_CONST
#define BP_GLOBAL
#endif

template <typename T>
__device__ __forceinline__ const BP_CONST T *as_const(const T *p) {
  return (const BP_CONST T *)p;
}

template <typename T>
__device__ __forceinline__ const BP_GLOBAL T *as_global(const T *p) {
  return (const BP_GLOBAL T *)p;
}

// ---------------------------------------------------------------------------
// Wave-level primitives (wave64, DPP).

template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWMASK, 0xf, true);
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
  uint32_t lo = dpp32<CTRL, ROWMASK>((uint32_t)v);
  uint32_t hi = dpp32<CTRL, ROWMASK>((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Inclusive scan (sum) over the 64 lanes: row_shr 1,2,4,8 within rows of 16,
// then row_bcast15 / row_bcast31 across rows.  Lanes shifted in from outside
// a row read 0 (bound_ctrl).
__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v) {
  v += dpp64<0x111, 0xf>(v);
  v += dpp64<0x112, 0xf>(v);
  v += dpp64<0x114, 0xf>(v);
  v += dpp64<0x118, 0xf>(v);
  v += dpp64<0x142, 0xa>(v);
  v += dpp64<0x143, 0xc>(v);
  return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
  v += dpp32<0x111, 0xf>(v);
  v += dpp32<0x112, 0xf>(v);
  v += dpp32<0x114, 0xf>(v);
  v += dpp32<0x118, 0xf>(v);
  v += dpp32<0x142, 0xa>(v);
  v += dpp32<0x143, 0xc>(v);
  return v;
}

__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }

// Maximum over the 64 lanes (same DPP pattern; lane 63 ends with the maximum).
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  v = umax64(v, dpp64<0x111, 0xf>(v));
  v = umax64(v, dpp64<0x112, 0xf>(v));
  v = umax64(v, dpp64<0x114, 0xf>(v));
  v = umax64(v, dpp64<0x118, 0xf>(v));
  v = umax64(v, dpp64<0x142, 0xa>(v));
  v = umax64(v, dpp64<0x143, 0xc>(v));
  uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// |a - b| + acc in one instruction (v_sad_u32).
// a is wave-uniform (an item size) and is passed in an SGPR.
__device__ __forceinline__ uint32_t sad_u32(uint32_t a, uint32_t b, uint32_t acc) {
  uint32_t r;
  asm("v_sad_u32 %0, %1, %2, %3" : "=v"(r) : "s"(a), "v"(b), "v"(acc));
  return r;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  uint32_t l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Packed maximum key: bound value in the high word, (2^32 - 1 - lambda) in the
// low word, so that the maximum key carries the largest value and, among
// equal values, the smallest parameter.  0 means "nothing evaluated".
__device__ __forceinline__ uint64_t pack_key(int64_t value, int64_t lam) {
  uint64_t v = value > 0xffffffffLL ? 0xffffffffull : (uint64_t)value;
  return (v << 32) | (uint64_t)(0xffffffffu - (uint32_t)lam);
}

// ---------------------------------------------------------------------------
// Prep: reduction, validation, radix sort, prefix sums, classes, stream.

template <int NT, int CAP>
struct PrepSmem {
  uint32_t keys[2][CAP];
  uint32_t hist[256];
  uint32_t wcnt[NT / 64][256];  // per (wave, digit): counts, then offsets
  uint64_t wtot[NT / 64];
  unsigned long long sums[3];  // sizes of all, of the big and of the non-zero non-full items
  int32_t flags[8];
};

// Rows of 64 keys per wave when n keys are spread evenly over the NW waves
// (at most K = CAP / NT): wave w owns the keys [w 64 R, (w + 1) 64 R).
template <int NW, int K>
__device__ __forceinline__ int rows_per_wave(int n) {
  return min(K, (((n + 63) >> 6) + NW - 1) / NW);
}

// Stable LSD radix sort (8-bit digits) of n keys in LDS, ascending.  Wave w
// owns the keys [w 64 R, (w + 1) 64 R), R = rows_per_wave(n), and holds them
// in registers, key k of a lane at w 64 R + 64 k + lane.  Per digit pass each
// wave ranks its keys in that order: a key's peers (lanes with the same
// digit) come from ballots over the digit's bits, its rank is the wave's
// running count of the digit plus the peers below it.  One block-wide scan
// over (digit, wave) counts then gives every key its place.  The digits are
// those of key - kmin, kmin the smallest key, so the passes cover only the
// bits of kmax - kmin (all keys equal or n = 0: no pass).  Returns the buffer
// index holding the result.
template <int NT, int CAP>
__device__ int lds_radix_sort(PrepSmem<NT, CAP> &sm, int n) {
  constexpr int NW = NT / 64;
  constexpr int K = CAP / NT;
  static_assert(K * NT == CAP, "capacity must be a multiple of the block size");
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int R = rows_per_wave<NW, K>(n);
  const int wbase = wave * 64 * R;
  // number of key rows of this wave that hold any key (wave-uniform)
  const int rows = n > wbase ? min(R, (n - wbase + 63) >> 6) : 0;
  // key range: per-wave minimum and maximum, then every thread combines them
  uint32_t kmin = 0xffffffffu, kmax = 0u;
  for (int k = 0; k < rows; ++k) {
    const int i = wbase + 64 * k + lane;
    if (i < n) {
      const uint32_t v = sm.keys[0][i];
      kmin = min(kmin, v);
      kmax = max(kmax, v);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, off));
    kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, off));
  }
  if (lane == 0) sm.wtot[wave] = ((uint64_t)kmax << 32) | (uint64_t)kmin;
  __syncthreads();
  kmin = 0xffffffffu;
  kmax = 0u;
  for (int w = 0; w < NW; ++w) {
    const uint64_t mm = sm.wtot[w];
    kmin = min(kmin, (uint32_t)mm);
    kmax = max(kmax, (uint32_t)(mm >> 32));
  }
  const int bits = kmax > kmin ? 32 - __clz((int)(kmax - kmin)) : 0;
  int src = 0;
  for (int sh = 0; sh < bits; sh += 8) {
    const uint32_t *a = sm.keys[src];
    uint32_t *b = sm.keys[src ^ 1];
    const int dbits = min(8, bits - sh);
    for (int i = lane; i < 256; i += 64) sm.wcnt[wave][i] = 0;
    uint32_t key[K], rank[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      key[k] = 0;
      rank[k] = 0;
      if (k < rows) {
        const int i = wbase + 64 * k + lane;
        const bool valid = i < n;
        key[k] = valid ? a[i] : kmin;
        const uint32_t d = ((key[k] - kmin) >> sh) & 255u;
        // peers: the valid lanes whose digit equals this lane's, one ballot
        // per digit bit; a lane keeps the lanes that agree with it on the bit
        // (~(m ^ s) is m where its bit is set, ~m where it is clear)
        uint64_t peers = ballot64(valid);
        for (int bit = 0; bit < dbits; ++bit) {
          const uint32_t s32 = (uint32_t)__builtin_amdgcn_sbfe((int)d, (unsigned)bit, 1u);  // 0 or all ones
          const uint64_t m = ballot64(s32 != 0u);
          const uint64_t s64 = ((uint64_t)s32 << 32) | (uint64_t)s32;
          peers &= ~(m ^ s64);
        }
        const uint32_t below = (uint32_t)__popcll(peers & lanemask_lt());
        // the wave's LDS accesses complete in program order: every lane reads
        // the count before the group's lowest lane writes the new one
        const uint32_t prior = valid ? sm.wcnt[wave][d] : 0u;
        rank[k] = prior + below;
        if (valid && below == 0) sm.wcnt[wave][d] = prior + (uint32_t)__popcll(peers);
      }
    }
    __syncthreads();
    // offsets, digit-major then wave, written over the counts
    for (int dg = tid; dg < 256; dg += NT) {
      uint32_t run = 0;
      for (int w = 0; w < NW; ++w) {
        const uint32_t c = sm.wcnt[w][dg];
        sm.wcnt[w][dg] = run;
        run += c;
      }
      sm.hist[dg] = run;
    }
    __syncthreads();
    if (tid < 64) {
      const uint32_t c0 = sm.hist[4 * tid], c1 = sm.hist[4 * tid + 1], c2 = sm.hist[4 * tid + 2],
                     c3 = sm.hist[4 * tid + 3];
      const uint32_t tot = c0 + c1 + c2 + c3;
      const uint32_t excl = wave_incl_scan_u32(tot) - tot;
      sm.hist[4 * tid] = excl;
      sm.hist[4 * tid + 1] = excl + c0;
      sm.hist[4 * tid + 2] = excl + c0 + c1;
      sm.hist[4 * tid + 3] = excl + c0 + c1 + c2;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (k < rows && wbase + 64 * k + lane < n) {
        const uint32_t d = ((key[k] - kmin) >> sh) & 255u;
        b[sm.hist[d] + sm.wcnt[wave][d] + rank[k]] = key[k];
      }
    }
    __syncthreads();
    src ^= 1;
  }
  return src;
}

// Exclusive prefix sums of the sorted sizes into pre[0..n], block-wide, in
// the same wave-striped layout as the sort: each wave first sums its keys,
// then scans them row by row from its offset.
template <int NT, int CAP>
__device__ void block_prefix(PrepSmem<NT, CAP> &sm, const uint32_t *sizes, int n, int64_t *pre, bool narrow) {
  constexpr int NW = NT / 64;
  constexpr int K = CAP / NT;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int R = rows_per_wave<NW, K>(n);
  const int wbase = wave * 64 * R;
  const int rows = n > wbase ? min(R, (n - wbase + 63) >> 6) : 0;
  uint64_t mine = 0;
  for (int k = 0; k < rows; ++k) {
    const int i = wbase + 64 * k + lane;
    mine += i < n ? sizes[i] : 0u;
  }
  const uint64_t tot = wave_incl_scan_u64(mine);
  if (lane == 63) sm.wtot[wave] = tot;
  __syncthreads();
  uint64_t carry = 0;
  for (int w = 0; w < wave; ++w) carry += sm.wtot[w];
  if (tid == 0) pre[0] = 0;
  if (narrow) {
    // every size < 2^26, so a row of 64 sums below 2^32: 32-bit row scans,
    // the 64-bit carry added after
    for (int k = 0; k < rows; ++k) {
      const int i = wbase + 64 * k + lane;
      const uint32_t v = i < n ? sizes[i] : 0u;
      const uint32_t incl32 = wave_incl_scan_u32(v);
      if (i < n) pre[i + 1] = (int64_t)(carry + incl32);
      carry += (uint32_t)__builtin_amdgcn_readlane((int)incl32, 63);
    }
  } else {
    for (int k = 0; k < rows; ++k) {
      const int i = wbase + 64 * k + lane;
      const uint64_t v = i < n ? sizes[i] : 0u;
      const uint64_t incl = wave_incl_scan_u64(v) + carry;
      if (i < n) pre[i + 1] = (int64_t)incl;
      carry = (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)incl, 63) |
              ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(incl >> 32), 63) << 32);
    }
  }
  (void)NW;
}

// floor(UINT32_MAX / denom) for denom > 0 (the VB2 cut of Sec. 4), in
// 32-bit arithmetic: 0 once denom exceeds UINT32_MAX.
__device__ __forceinline__ int64_t vb2_cut_cap(int64_t denom) {
  return denom > (int64_t)0xffffffffLL ? 0 : (int64_t)(0xffffffffu / (uint32_t)denom);
}

// L1 = ceil(sumW / c) > k for r items of sizes at most c, without a 64-bit
// division: never when k >= r (then L1 <= r), else sumW > k c (k c < 2^52).
__device__ __forceinline__ bool l1_exceeds(int64_t sumW, int64_t r, int64_t C, int64_t k) {
  return k < r && sumW > k * C;
}

template <int NT, int CAP>
__device__ void prep_instance(const LaunchDesc &d, int64_t inst, PrepSmem<NT, CAP> &sm) {
  const BP_CONST InstPlan &p = as_const(d.plan)[inst];
  InstState *st = &d.state[inst];
  const int tid = threadIdx.x;
  const int32_t C = p.C;
  const uint32_t uC = (uint32_t)C;
  int64_t r = 0;
  int32_t status = BP_OK;
  int32_t maxw = 0;   // (thread 0)
  int64_t sumW = 0;   // (thread 0)
  if (tid < 8) sm.flags[tid] = 0;
  __syncthreads();
  if (p.r_cap > CAP) {
    status = BP_ERR_LIMIT;
  } else {
    // Reduction into LDS: sort key = c - w (ascending key = decreasing size).
    // Inputs are read in the wave-striped layout of the sort, every load of a
    // lane issued before the first store, so the block waits for one memory
    // round trip per array rather than one per row.
    constexpr int K = CAP / NT;
    const int wave = tid >> 6, lane = tid & 63;
    const int wbase = wave * 64 * K;
    const BP_GLOBAL int32_t *in = as_global(d.in + p.in_off);
    const int n_in = (int)p.n_in;
    {
      int32_t v[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int i = wbase + 64 * k + lane;
        v[k] = i < n_in ? in[i] : 0;
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int i = wbase + 64 * k + lane;
        if (i < n_in) {
          int32_t w = v[k];
          if (w < 0 || w > C) { sm.flags[0] = 1; w = 0; }
          sm.keys[0][i] = uC - (uint32_t)w;
        }
      }
    }
    int64_t nfill = 0;
    if (p.form == kFormResidual) {
      // one virtual item of size c - residual per bin with residual < c
      // (Fig. 3), appended in bin order: a stable compaction of the loaded bins
      const BP_GLOBAL int32_t *res = as_global(d.in2 + p.res_off);
      const int m = p.m_res;
      int32_t rv[K];
      uint32_t pos[K];
      uint32_t takes = 0;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int j = wbase + 64 * k + lane;
        rv[k] = j < m ? res[j] : C;
      }
      uint32_t run = 0;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int j = wbase + 64 * k + lane;
        int32_t rj = rv[k];
        if (j < m && (rj < 0 || rj > C)) { sm.flags[0] = 1; rj = C; }
        rv[k] = rj;
        const bool take = j < m && rj < C;
        const uint64_t bal = ballot64(take);
        pos[k] = run + (uint32_t)__popcll(bal & lanemask_lt());
        run += (uint32_t)__popcll(bal);
        takes |= (uint32_t)take << k;
      }
      if (lane == 0) sm.wcnt[0][wave] = run;
      __syncthreads();
      uint32_t off = 0, tot = 0;
      for (int w = 0; w < NT / 64; ++w) {
        const uint32_t c = sm.wcnt[0][w];
        off += w < wave ? c : 0u;
        tot += c;
      }
#pragma unroll
      for (int k = 0; k < K; ++k)
        if ((takes >> k) & 1u) sm.keys[0][n_in + off + pos[k]] = (uint32_t)rv[k];  // key = c - load = residual
      nfill = tot;
    }
    r = n_in + nfill;
    __syncthreads();
    if (sm.flags[0]) {
      status = BP_ERR_RANGE;
      r = 0;
    }
    const int res_buf = lds_radix_sort<NT, CAP>(sm, (int)r);
    uint32_t *keys = sm.keys[res_buf];
    uint32_t *sz = sm.keys[res_buf ^ 1];
    for (int i = tid; i < r; i += NT) sz[i] = uC - keys[i];
    __syncthreads();
    if (p.flags & kPlanSegments) {
      // threshold table of the segment sums: bidx[b] = #{sizes >= b 2^bshift},
      // a binary search over the decreasing sizes in LDS per entry
      int32_t *bidx = d.bidx + p.bidx_off;
      const int sh = p.bshift;
      for (int b = tid; b < p.nbk; b += NT) {
        const uint64_t v = (uint64_t)b << sh;
        int lo = 0, hi = (int)r;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if ((uint64_t)sz[mid] >= v) lo = mid + 1; else hi = mid;
        }
        bidx[b] = lo;
      }
    }
    // class boundaries on the decreasing sizes, and the class sums
    if (tid < 8) sm.flags[tid] = 0;
    if (tid < 3) sm.sums[tid] = 0ull;
    __syncthreads();
    uint32_t c_full = 0, c_big = 0, c_bm = 0, c_nz = 0;
    uint64_t s_all = 0, s_big = 0, s_nz = 0;
    for (int i = tid; i < r; i += NT) {
      const uint32_t w = sz[i];
      c_full += w == uC;
      c_big += 2ull * w > uC;
      c_bm += 2ull * w >= uC;
      c_nz += w > 0;
      s_all += w;
      s_big += (2ull * w > uC && w < uC) ? w : 0u;
      s_nz += (w > 0 && w < uC) ? w : 0u;
    }
    c_full = wave_incl_scan_u32(c_full);
    c_big = wave_incl_scan_u32(c_big);
    c_bm = wave_incl_scan_u32(c_bm);
    c_nz = wave_incl_scan_u32(c_nz);
    s_all = wave_incl_scan_u64(s_all);
    s_big = wave_incl_scan_u64(s_big);
    s_nz = wave_incl_scan_u64(s_nz);
    if ((tid & 63) == 63) {
      atomicAdd(&sm.flags[1], (int)c_full);
      atomicAdd(&sm.flags[2], (int)c_big);
      atomicAdd(&sm.flags[3], (int)c_bm);
      atomicAdd(&sm.flags[4], (int)c_nz);
      atomicAdd(&sm.sums[0], (unsigned long long)s_all);
      atomicAdd(&sm.sums[1], (unsigned long long)s_big);
      atomicAdd(&sm.sums[2], (unsigned long long)s_nz);
    }
    __syncthreads();
    const int nf = sm.flags[1], nb = sm.flags[2], nm = sm.flags[3], nz = sm.flags[4];
    int32_t *sorted = d.sorted + p.ws_off;
    uint32_t *av = d.av + p.ws_off;
    for (int i = tid; i < r; i += NT) {
      const uint32_t w = sz[i];
      sorted[i] = (int32_t)w;
      av[i] = (2ull * w > uC) ? uC - w : w;  // c - w for big items, w otherwise
    }
    int64_t *pre = d.pre + p.pre_off;
    block_prefix<NT, CAP>(sm, sz, (int)r, pre, uC < (1u << 26));
    __syncthreads();
    if (p.ndiv > 0) {
      // mirrored VB2: per divisor d of c, the small and the big sizes that d
      // divides.  With c = prod p_j^a_j, d | w iff every exponent of d is at
      // most min(v_pj(w), a_j).  Each size adds 1 to the lattice bin of its
      // capped exponent vector (about two multiply-compare divisibility tests
      // of bp_divide.h per prime, family 3); superset sums along each prime's
      // axis then turn the bins into the count of multiples of every divisor.
      // wcnt[0..1] hold the small and the big class; the sort's key buffer is
      // free here and holds the test constants of p_j^e, e = 1..a_j (laid
      // out by the host after the (p_j, a_j) pairs).
      const int nd = p.ndiv;  // = number of lattice bins
      const BP_GLOBAL int32_t *dv = as_global(d.divs + p.div_off);
      const BP_GLOBAL int32_t *dbin = dv + nd;
      const int np = dv[2 * nd];
      const BP_GLOBAL int32_t *pa = dv + 2 * nd + 1;  // (p_j, a_j) pairs
      uint64_t *pmul = reinterpret_cast<uint64_t *>(keys);
      {
        const int npp = pa[2 * np];
        const BP_GLOBAL int32_t *m = pa + 2 * np + 1;
        for (int k = tid; k < npp; k += NT)
          pmul[k] = (uint64_t)(uint32_t)m[2 * k] | ((uint64_t)(uint32_t)m[2 * k + 1] << 32);
      }
      for (int k = tid; k < 256; k += NT) {
        sm.wcnt[0][k] = 0;
        sm.wcnt[1][k] = 0;
      }
      __syncthreads();
      for (int i = tid; i < r; i += NT) {
        const int cls = (i >= nf && i < nb) ? 1 : ((i >= nm && i < nz) ? 0 : -1);
        if (cls < 0) continue;
        const uint32_t w = sz[i];
        int bin = 0, stride = 1, o = 0;
        for (int j = 0; j < np; ++j) {
          const int aj = pa[2 * j + 1];
          int e = 0;
          while (e < aj && divides_u32(w, pmul[o + e])) ++e;
          bin += e * stride;
          stride *= aj + 1;
          o += aj;
        }
        atomicAdd(&sm.wcnt[cls][bin], 1u);
      }
      __syncthreads();
      {
        int stride = 1;
        for (int j = 0; j < np; ++j) {
          const int aj = pa[2 * j + 1];
          for (int e = aj - 1; e >= 0; --e) {
            // bins whose j-th exponent is e take the sums of the bins one step up
            for (int b = tid; b < nd; b += NT) {
              if ((b / stride) % (aj + 1) == e) {
                sm.wcnt[0][b] += sm.wcnt[0][b + stride];
                sm.wcnt[1][b] += sm.wcnt[1][b + stride];
              }
            }
            __syncthreads();
          }
          stride *= aj + 1;
        }
      }
      int32_t *dc = d.dcnt + p.dc_off;
      for (int k = tid; k < nd; k += NT) {
        const int bk = dbin[k];
        dc[k] = (int32_t)sm.wcnt[0][bk];
        dc[nd + k] = (int32_t)sm.wcnt[1][bk];
      }
      __syncthreads();
    }
    if (tid == 0) {
      maxw = r > 0 ? (int32_t)sz[0] : 0;
      sumW = (int64_t)sm.sums[0];
      st->r = (int32_t)r;
      st->nf = nf;
      st->nb = nb;
      st->nm = nm;
      st->nz = nz;
      st->maxw = maxw;
      st->sumW = sumW;
      st->sumBig = (int64_t)sm.sums[1];
      st->sumNZ = (int64_t)sm.sums[2];
    }
  }
  // the rest of the state from what this block holds (no read-back of the
  // global workspaces): status, effective ranges, cleared results
  if (tid < kNB) d.keys[inst * kNB + tid] = 0ull;
  if (tid == 0) {
    st->status = status;
    if (status != BP_OK) {
      r = 0;
      st->r = 0; st->nf = st->nb = st->nm = st->nz = 0; st->maxw = 0;
      st->sumW = st->sumBig = st->sumNZ = 0;
    }
    for (int b = 0; b < kNB; ++b) st->hiEff[b] = p.hi[b];
    if ((p.flags & kPlanClampVB2) && status == BP_OK) {
      const int64_t denom = r * (int64_t)maxw;
      const int64_t cap = denom > 0 ? vb2_cut_cap(denom) : (int64_t)p.C;
      if (cap < st->hiEff[kVB2]) st->hiEff[kVB2] = cap;
    }
    st->evals_skipped = 0ull;
    int refuted = 0;
    if ((p.flags & kPlanEarlyExit) && status == BP_OK && r > 0) refuted = l1_exceeds(sumW, r, p.C, p.k);
    d.refuted[inst] = refuted;
  }
}

// Clears the task counters of the sweep that follows (run by the
// small-instance prep grid).
__device__ void clear_sweep_state(const LaunchDesc &d) {
  if (blockIdx.x == 0 && threadIdx.x < kQueues) d.counter[threadIdx.x * kQueueStride] = 0ull;
}

// ---------------------------------------------------------------------------
// Value-table prep of large instances (InstPlan::large == 2), over the whole
// GPU instead of one block, in two steps:
//   vt_hist    (in the small-instance prep kernel, which runs first) every
//              reduced size adds 1 to the raw count of its value; per block
//              in LDS, then one atomic per touched entry: each chunk's
//              (count, sum) totals, and for a mirrored VB2 each size's
//              divisor-lattice bin; the largest size and the input flag;
//   k_vt_emit  the chunks' offsets (suffix sums of the totals, in LDS), then
//              per chunk the suffix sums of the counts and of count x value
//              within the chunk (the tables the lookup tiles read), and every
//              value v present fills its run of sorted positions
//              [#{w > v}, #{w >= v}) with v, av and the prefix sums; the
//              class bounds, the threshold table and the instance state are
//              written by the threads holding their values, the multiple
//              counts of the mirrored VB2 from the lattice bins.
// The raw counts, chunk totals, lattice bins and per-instance flag and
// maximum are zero at the start of a launch: the allocation clears them and
// k_finalize clears what a launch used.  The chunk-local tables are written
// whole by every launch.

// LDS of vt_hist, over the prep kernel's own (used before its instance loop).
struct VtHistSmem {
  unsigned long long csum[kVtMaxChunks];
  unsigned long long pmul[32];
  uint32_t ccnt[kVtMaxChunks];
  uint32_t lat[2][kMaxDivs];
  int32_t pa[64];
  int32_t np;
  int32_t maxw;
  int32_t bad;
};
static_assert(sizeof(VtHistSmem) <= sizeof(PrepSmem<kSmallThreads, kTinyCap>), "vt_hist fits the prep LDS");

// The divisor-lattice bin of a size w: its class (0 small, 0 < 2w < c; 1
// big, c/2 < w < c; -1 neither) and sum_j e_j stride_j, e_j the exponent of
// the j-th prime of c in gcd(w, c).
__device__ __forceinline__ int vt_lattice_bin(uint32_t uw, uint32_t uC, const VtHistSmem &sm, int *bin) {
  const int cls = (2ull * uw > uC && uw < uC) ? 1 : ((uw > 0 && 2ull * uw < uC) ? 0 : -1);
  if (cls < 0) return cls;
  int b = 0, stride = 1, o = 0;
  for (int j = 0; j < sm.np; ++j) {
    const int aj = sm.pa[2 * j + 1];
    int e = 0;
    while (e < aj && divides_u32(uw, sm.pmul[o + e])) ++e;
    b += e * stride;
    stride *= aj + 1;
    o += aj;
  }
  *bin = b;
  return cls;
}

__device__ void vt_hist(const LaunchDesc &d, VtHistSmem &sm) {
  const int64_t gsz = (int64_t)gridDim.x * blockDim.x;
  for (int64_t jj = 0; jj < d.nvt; ++jj) {
    const int64_t inst = d.vlist[jj];
    const BP_CONST InstPlan &p = as_const(d.plan)[inst];
    const int32_t C = p.C;
    const int64_t tot = p.n_in + (p.form == kFormResidual ? p.m_res : 0);
    const int64_t first = blockIdx.x * (int64_t)blockDim.x;
    if (first >= tot) continue;  // no items in this block (block-uniform)
    const int64_t nch = ((int64_t)C + 2 + kVtChunk - 1) >> kVtChunkLog;
    const int nd = p.ndiv;
    __syncthreads();  // the previous instance's LDS has been flushed
    for (int64_t c = threadIdx.x; c < nch; c += blockDim.x) {
      sm.ccnt[c] = 0u;
      sm.csum[c] = 0ull;
    }
    for (int k = threadIdx.x; k < nd; k += blockDim.x) {
      sm.lat[0][k] = 0u;
      sm.lat[1][k] = 0u;
    }
    if (threadIdx.x == 0) {
      sm.maxw = 0;
      sm.bad = 0;
    }
    if (nd > 0) {
      // the primes of c with their exponents, then the test constants of each
      // prime power p_j^e, e = 1..a_j (laid out by the host)
      const BP_GLOBAL int32_t *dv = as_global(d.divs + p.div_off) + 2 * nd;
      const int np = dv[0];
      const int npp = dv[1 + 2 * np];
      if ((int)threadIdx.x < 2 * np) sm.pa[threadIdx.x] = dv[1 + threadIdx.x];
      if ((int)threadIdx.x < npp) {
        const BP_GLOBAL int32_t *m = dv + 2 + 2 * np + 2 * threadIdx.x;
        sm.pmul[threadIdx.x] = (unsigned long long)(uint32_t)m[0] | ((unsigned long long)(uint32_t)m[1] << 32);
      }
      if (threadIdx.x == 0) sm.np = np;
    }
    __syncthreads();
    int32_t *raw = d.vraw + p.vt_off;
    bool bad = false;
    int32_t mx = 0;
    for (int64_t i = first + threadIdx.x; i < tot; i += gsz) {
      int32_t w;
      if (i < p.n_in) {
        w = d.in[p.in_off + i];
        if (w < 0 || w > C) {
          bad = true;
          continue;
        }
      } else {
        const int32_t res = d.in2[p.res_off + (i - p.n_in)];
        if (res < 0 || res > C) {
          bad = true;
          continue;
        }
        if (res == C) continue;  // an empty bin adds no virtual item (Fig. 3)
        w = C - res;
      }
      atomicAdd(&raw[w], 1);
      const int c = w >> kVtChunkLog;
      atomicAdd(&sm.ccnt[c], 1u);
      atomicAdd(&sm.csum[c], (unsigned long long)w);
      mx = max(mx, w);
      if (nd > 0) {
        int bin;
        const int cls = vt_lattice_bin((uint32_t)w, (uint32_t)C, sm, &bin);
        if (cls >= 0) atomicAdd(&sm.lat[cls][bin], 1u);
      }
    }
    const uint64_t wmx = wave_max_u64((uint64_t)(uint32_t)mx);
    if ((threadIdx.x & 63) == 0) atomicMax(&sm.maxw, (int32_t)wmx);
    if (bad) atomicOr(&sm.bad, 1);
    __syncthreads();
    unsigned long long *ctot = (unsigned long long *)(d.vtot + p.vtt_off);
    for (int64_t c = threadIdx.x; c < nch; c += blockDim.x) {
      const uint32_t n = sm.ccnt[c];
      if (!n) continue;
      atomicAdd(&ctot[2 * c], (unsigned long long)n);
      atomicAdd(&ctot[2 * c + 1], sm.csum[c]);
    }
    for (int k = threadIdx.x; k < nd; k += blockDim.x) {
      if (sm.lat[0][k]) atomicAdd(&d.vlat[p.vl_off + k], (int32_t)sm.lat[0][k]);
      if (sm.lat[1][k]) atomicAdd(&d.vlat[p.vl_off + nd + k], (int32_t)sm.lat[1][k]);
    }
    if (threadIdx.x == 0) {
      if (sm.bad) atomicOr(&d.vflag[2 * jj], 1);
      if (sm.maxw > 0) atomicMax(&d.vflag[2 * jj + 1], sm.maxw);
    }
  }
  if (d.nvt > 0) __syncthreads();  // before the instance loop reuses the LDS
}

template <int NT, int CAP, int LARGE>
__global__ __launch_bounds__(NT) void k_prep(const LaunchDesc *__restrict__ dp) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  PrepSmem<NT, CAP> &sm = *reinterpret_cast<PrepSmem<NT, CAP> *>(smem_raw);
  const LaunchDesc d = *as_const(dp);
  if (!LARGE) {
    clear_sweep_state(d);
    vt_hist(d, *reinterpret_cast<VtHistSmem *>(smem_raw));
  }
  for (int64_t inst = blockIdx.x; inst < d.count; inst += gridDim.x) {
    if (as_const(d.plan)[inst].large != LARGE) continue;
    prep_instance<NT, CAP>(d, inst, sm);
    __syncthreads();
  }
}

// Block-wide inclusive scan of two 64-bit sums (kVtThreads threads); also
// returns the block totals.  Uses red[2][kVtThreads / 64].
__device__ __forceinline__ void vt_block_scan(uint64_t a, uint64_t b, uint64_t (*red)[kVtThreads / 64],
                                              uint64_t *ia, uint64_t *ib, uint64_t *ta, uint64_t *tb) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t sa = wave_incl_scan_u64(a), sb = wave_incl_scan_u64(b);
  __syncthreads();
  if (lane == 63) {
    red[0][wave] = sa;
    red[1][wave] = sb;
  }
  __syncthreads();
  uint64_t pa = 0, pb = 0, xa = 0, xb = 0;
  for (int w = 0; w < kVtThreads / 64; ++w) {
    pa += w < wave ? red[0][w] : 0ull;
    pb += w < wave ? red[1][w] : 0ull;
    xa += red[0][w];
    xb += red[1][w];
  }
  *ia = sa + pa;
  *ib = sb + pb;
  *ta = xa;
  *tb = xb;
}

__global__ __launch_bounds__(kVtThreads) void k_vt_emit(const LaunchDesc *__restrict__ dp) {
  __shared__ long long offc[kVtMaxChunks + 1], offs[kVtMaxChunks + 1];
  __shared__ uint64_t red[2][kVtThreads / 64];
  __shared__ uint32_t lat[2][kMaxDivs];
  // runs longer than kVtShortRun, filled by the whole block: (value, first
  // position, length, sum of the sizes above), at most one per value of the
  // chunk
  constexpr int kVtShortRun = 16;
  constexpr int PER = kVtChunk / kVtThreads;
  __shared__ int32_t lrun_v[kVtChunk], lrun_s[kVtChunk], lrun_n[kVtChunk];
  __shared__ long long lrun_a[kVtChunk];
  // the chunk's #{w >= v} and sum{w >= v} within the chunk, by value
  __shared__ int32_t lge[kVtChunk + 1];
  __shared__ long long lsge[kVtChunk];
  __shared__ int32_t nlong;
  const LaunchDesc d = *as_const(dp);
  for (int64_t jj = 0; jj < d.nvt; ++jj) {
    const int64_t inst = d.vlist[jj];
    const BP_CONST InstPlan &p = as_const(d.plan)[inst];
    const int64_t C = p.C;
    const int64_t nv = C + 2;
    const int64_t nch = (nv + kVtChunk - 1) / kVtChunk;
    const int32_t *raw = d.vraw + p.vt_off;
    int32_t *cnt = d.vcnt + p.vt_off;
    long long *sum = d.vsum + p.vt_off;
    const long long *tot = d.vtot + p.vtt_off;
    const bool ok = d.vflag[2 * jj] == 0;
    const int32_t maxw = d.vflag[2 * jj + 1];
    const int64_t nfull = raw[C];  // items of size c
    // this block's first chunk of raw counts, loaded with the totals (one
    // memory round trip for both)
    const int64_t v0_first = (int64_t)blockIdx.x * kVtChunk + (int64_t)threadIdx.x * PER;
    uint32_t cn[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int64_t v = v0_first + k;
      cn[k] = ((int64_t)blockIdx.x < nch && v < nv) ? (uint32_t)raw[v] : 0u;
    }
    // offsets of the chunks: the totals of the chunks above each, a block scan
    // of up to E totals per thread
    uint64_t all_c, all_s;
    {
      const int E = (int)((nch + kVtThreads - 1) / kVtThreads);
      const int64_t c0 = (int64_t)threadIdx.x * E;
      uint64_t mc = 0, ms = 0;
      for (int k = 0; k < E; ++k)
        if (c0 + k < nch) {
          mc += (uint64_t)tot[2 * (c0 + k)];
          ms += (uint64_t)tot[2 * (c0 + k) + 1];
        }
      uint64_t ic, is;
      vt_block_scan(mc, ms, red, &ic, &is, &all_c, &all_s);
      uint64_t rc = all_c - ic, rs = all_s - is;
      for (int k = E - 1; k >= 0; --k) {
        const int64_t c = c0 + k;
        if (c < nch) {
          offc[c] = (long long)rc;
          offs[c] = (long long)rs;
          if (c % gridDim.x == blockIdx.x) {
            // for the lookup tiles of the sweep, after the totals
            d.vtot[p.vtt_off + 2 * nch + 2 * c] = (long long)rc;
            d.vtot[p.vtt_off + 2 * nch + 2 * c + 1] = (long long)rs;
          }
          rc += (uint64_t)tot[2 * c];
          rs += (uint64_t)tot[2 * c + 1];
        }
      }
    }
    InstState *st = &d.state[inst];
    int32_t *sorted = d.sorted + p.ws_off;
    uint32_t *av = d.av + p.ws_off;
    int64_t *pre = d.pre + p.pre_off;
    const bool seg = (p.flags & kPlanSegments) != 0;
    const int64_t bmask = ((int64_t)1 << p.bshift) - 1;
    // position i of value v's run: the size, av and the prefix sum through i
    auto put = [&](int64_t v, int64_t i, int64_t above, int64_t sum_above) {
      sorted[i] = (int32_t)v;
      av[i] = (2 * v > C) ? (uint32_t)(C - v) : (uint32_t)v;
      pre[i + 1] = sum_above + (i + 1 - above) * v;
    };
    if (ok && blockIdx.x == 0 && threadIdx.x == 0) pre[0] = 0;
    for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
      if (threadIdx.x == 0) nlong = 0;
      const int64_t v0 = c * kVtChunk + (int64_t)threadIdx.x * PER;
      uint64_t mc = 0, ms = 0;
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int64_t v = v0 + k;
        if (c != (int64_t)blockIdx.x) cn[k] = v < nv ? (uint32_t)raw[v] : 0u;
        mc += cn[k];
        ms += (uint64_t)cn[k] * (uint64_t)v;
      }
      uint64_t ic, is, tc, ts;
      vt_block_scan(mc, ms, red, &ic, &is, &tc, &ts);  // (its barriers also order the nlong reset)
      // #{w >= v} and sum{w >= v} within the chunk: everything held by the
      // threads after this one, then this thread's values downwards
      uint64_t rc = tc - ic, rs = ts - is;
#pragma unroll
      for (int k = PER - 1; k >= 0; --k) {
        const int64_t v = v0 + k;
        rc += cn[k];
        rs += (uint64_t)cn[k] * (uint64_t)v;
        lge[threadIdx.x * PER + k] = (int32_t)rc;
        lsge[threadIdx.x * PER + k] = (long long)rs;
        if (v < nv) {
          cnt[v] = (int32_t)rc;
          sum[v] = (long long)rs;
        }
      }
      if (threadIdx.x == 0) lge[kVtChunk] = 0;
      __syncthreads();
      if (ok) {
        const long long oc = offc[c], os = offs[c];
        // (a rolled loop over this thread's values, read back from LDS: one
        // copy of its body)
#pragma unroll 1
        for (int k = 0; k < PER; ++k) {
          const int64_t v = v0 + k;
          if (v >= nv) break;
          const int li = threadIdx.x * PER + k;
          const int64_t n = lge[li] - lge[li + 1], cge = lge[li] + oc, sgev = lsge[li] + os;
          // the class bounds and sums of the state, by the thread holding the value
          if (v == C) st->nf = (int32_t)cge;
          if (v == C / 2 + 1) {
            st->nb = (int32_t)cge;
            st->sumBig = sgev - C * nfull;  // sizes c/2 < w < c
          }
          if (v == (C + 1) / 2) st->nm = (int32_t)cge;
          if (v == 1) {
            st->nz = (int32_t)cge;
            st->sumNZ = sgev - C * nfull;  // sizes 0 < w < c
          }
          if (seg && (v & bmask) == 0) d.bidx[p.bidx_off + (v >> p.bshift)] = (int32_t)cge;
          if (n == 0) continue;
          const int64_t gt = cge - n, sgt = sgev - n * v;
          if (n <= kVtShortRun) {
            for (int64_t i = gt; i < cge; ++i) put(v, i, gt, sgt);
          } else {
            const int slot = atomicAdd(&nlong, 1);
            lrun_v[slot] = (int32_t)v;
            lrun_s[slot] = (int32_t)gt;
            lrun_n[slot] = (int32_t)n;
            lrun_a[slot] = sgt;
          }
        }
      }
      __syncthreads();
      if (ok) {
        for (int q = 0; q < nlong; ++q) {
          const int64_t v = lrun_v[q], gt = lrun_s[q], sgt = lrun_a[q];
          for (int64_t i = gt + threadIdx.x; i < gt + lrun_n[q]; i += blockDim.x) put(v, i, gt, sgt);
        }
      }
      __syncthreads();
    }
    if (blockIdx.x != jj % gridDim.x) continue;
    // one block per instance: the multiple counts of the mirrored VB2, the
    // threshold-table entries past c + 1, and the rest of the state
    const int nd = p.ndiv;
    if (nd > 0 && ok) {
      const BP_GLOBAL int32_t *dv = as_global(d.divs + p.div_off);
      const BP_GLOBAL int32_t *dbin = dv + nd;
      const int np = dv[2 * nd];
      const BP_GLOBAL int32_t *pa = dv + 2 * nd + 1;
      for (int k = threadIdx.x; k < nd; k += blockDim.x) {
        lat[0][k] = (uint32_t)d.vlat[p.vl_off + k];
        lat[1][k] = (uint32_t)d.vlat[p.vl_off + nd + k];
      }
      __syncthreads();
      // superset sums along each prime's axis: bin e takes bin e + 1's count
      int stride = 1;
      for (int j = 0; j < np; ++j) {
        const int aj = pa[2 * j + 1];
        for (int e = aj - 1; e >= 0; --e) {
          for (int b = threadIdx.x; b < nd; b += blockDim.x) {
            if ((b / stride) % (aj + 1) == e) {
              lat[0][b] += lat[0][b + stride];
              lat[1][b] += lat[1][b + stride];
            }
          }
          __syncthreads();
        }
        stride *= aj + 1;
      }
      int32_t *dc = d.dcnt + p.dc_off;
      for (int k = threadIdx.x; k < nd; k += blockDim.x) {
        const int bk = dbin[k];
        dc[k] = (int32_t)lat[0][bk];
        dc[nd + k] = (int32_t)lat[1][bk];
      }
    }
    if (seg && ok)
      for (int64_t b = ((C + 1) >> p.bshift) + 1 + threadIdx.x; b < p.nbk; b += blockDim.x)
        d.bidx[p.bidx_off + b] = 0;
    if (threadIdx.x == 0) {
      const int64_t r = (int64_t)all_c;
      if (ok) {
        st->status = BP_OK;
        st->r = (int32_t)r;
        st->maxw = maxw;
        st->sumW = (int64_t)all_s;
      } else {
        st->status = BP_ERR_RANGE;
        st->r = 0;
        st->nf = st->nb = st->nm = st->nz = 0;
        st->maxw = 0;
        st->sumW = st->sumBig = st->sumNZ = 0;
      }
      for (int b = 0; b < kNB; ++b) st->hiEff[b] = p.hi[b];
      if ((p.flags & kPlanClampVB2) && ok && r > 0) {
        const int64_t denom = r * (int64_t)st->maxw;
        const int64_t cap = denom > 0 ? vb2_cut_cap(denom) : (int64_t)p.C;
        if (cap < st->hiEff[kVB2]) st->hiEff[kVB2] = cap;
      }
      for (int b = 0; b < kNB; ++b) d.keys[inst * kNB + b] = 0ull;
      st->evals_skipped = 0ull;
      int refuted = 0;
      if ((p.flags & kPlanEarlyExit) && ok && r > 0) refuted = l1_exceeds((int64_t)all_s, r, p.C, p.k);
      d.refuted[inst] = refuted;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Sweep tiles.  Each lane holds LPL parameters lam = lam0 + lane + 64 j;
// lanes past the end of the range compute with lam = lo and are dropped.
//
// A tile's items may be split into chunks run by different waves.  Every
// function's per-parameter sum is an instance constant plus a part that is a
// plain sum over the streamed items, so a chunk computes that part exactly
// (int64) over its items and stores it in a slot of its own; after the sweep
// the combine kernel adds a tile's slots and finalises the tile.  Split BJ1
// and CCM1 segment tiles divide their q range instead of the items, the
// instance constant going with chunk 0.
// Streamed items are [nf, nz); functions with a class split stream
// [nf, nb) (big) and [nm, nz) (small) and count the mid items.

struct TileArgs {
  const BP_CONST uint32_t *wv;     // sizes, decreasing (scalar stream)
  const BP_CONST uint32_t *av;     // c - w for big items, w otherwise (scalar stream)
  const BP_GLOBAL int32_t *sorted; // sizes again, for per-lane binary search
  const BP_GLOBAL int64_t *pre;
  int64_t lo, hi;        // effective range of the bound
  int64_t lam0;          // first parameter of the tile
  int64_t k;
  int32_t C, r, nf, nb, nm, nz;
  int32_t i0, i1;        // streamed item range of this chunk, inside [nf, nz)
  int64_t sumBig, sumNZ;
  const BP_CONST int32_t *bidx;  // threshold table (segment entries)
  const BP_CONST int64_t *prec;  // prefix sums again, for scalar loads
  int32_t bsh;                   // bucket width 2^bsh of the table
  int32_t ndiv;                  // mirrored VB2: divisors of c
  int32_t qc, qn;                // BJ1/CCM1 segment tiles: this chunk of qn takes its share of the q range
  const BP_GLOBAL int32_t *divs; // ascending
  const BP_GLOBAL int32_t *dcnt; // [small x ndiv][big x ndiv] multiple counts
  long long *node;               // served request: this bound's block of the node state, indexed by lambda - lo
  const BP_GLOBAL int32_t *vc;   // value tables (lookup tiles): #{w >= v} and sum{w >= v} within each chunk,
  const BP_GLOBAL long long *vs; //   plus the chunk's offsets vo[2 chunk], vo[2 chunk + 1]
  const BP_GLOBAL long long *vo;
};

// Largest number of items whose per-item increments, each at most maxinc,
// can be summed in 32 bits.
__device__ __forceinline__ int chunk_len(uint64_t maxinc) {
  if (maxinc == 0) return 1 << 30;
  uint64_t l = 0xffffffffull / maxinc;
  return l > (1ull << 30) ? (1 << 30) : (int)l;
}

// ceil(a / b) for 0 <= a < 2^53 and b >= 1 without a 64-bit integer division:
// the correctly rounded fp64 quotient is within 2 of a / b, and the exact
// remainder a - q b (no overflow: q b <= a + 2b, and q > 0 only when b <= a)
// moves q to floor(a / b).  Every bound's numerator here is such a sum.
__device__ __forceinline__ int64_t ceil_div_small(int64_t a, int64_t b) {
  int64_t q = (int64_t)((double)a / (double)b);
  int64_t r = a - q * b;
  while (r < 0) { --q; r += b; }
  while (r >= b) { ++q; r -= b; }
  return q + (r != 0);
}

// Items per scalar block of the dense sweeps: 16 (one s_load_dwordx16, the
// next 16 in flight) with two or four parameters per lane; 8 with one, whose
// wave would otherwise spill.
template <int LPL>
constexpr int kStreamBlock = LPL >= 2 ? 16 : 8;

// Calls f(p[i]) for i in [i0, i1) in order.  Every lane uses the same item,
// so items are read with scalar loads, U at a time, and the next block's
// loads are issued before the current block is processed: the stream is
// larger than the scalar cache, and this hides the latency of its misses.
template <int U = 8, typename F>
__device__ __forceinline__ void stream_u32(const BP_CONST uint32_t *p, int i0, int i1, F &&f) {
  int i = i0;
  if (i1 - i >= U) {
    uint32_t cur[U];
#pragma unroll
    for (int u = 0; u < U; ++u) cur[u] = p[i + u];
    i += U;
    for (; i + U <= i1; i += U) {
      uint32_t nxt[U];
#pragma unroll
      for (int u = 0; u < U; ++u) nxt[u] = p[i + u];
#pragma unroll
      for (int u = 0; u < U; ++u) f(cur[u]);
#pragma unroll
      for (int u = 0; u < U; ++u) cur[u] = nxt[u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) f(cur[u]);
  }
  for (; i < i1; ++i) f(p[i]);
}

// The sub-range of [i0, i1) whose values are at most lim, for a monotone
// range (the sorted sizes of one class, or their complements): it is a
// prefix or a suffix, [*s0, *s1), and the rest of the range is the other
// end.  Two scalar loads decide the common cases (all or none); a range
// that straddles lim takes a binary search.
__device__ __forceinline__ void small_part(const BP_CONST uint32_t *p, int i0, int i1, uint32_t lim, int *s0,
                                           int *s1) {
  *s0 = *s1 = i0;
  if (i0 >= i1) return;
  const bool a = p[i0] <= lim, b = p[i1 - 1] <= lim;
  if (a == b) {
    if (a) *s1 = i1;
    return;
  }
  // the first index whose test differs from the first item's, in (i0, i1 - 1]
  int lo = i0 + 1, hi = i1 - 1;
  while (lo < hi) {
    const int mid = lo + ((hi - lo) >> 1);
    if ((p[mid] <= lim) == a) lo = mid + 1;
    else hi = mid;
  }
  if (a) {
    *s1 = lo;  // [i0, lo) passes
  } else {
    *s0 = lo;  // [lo, i1) passes
    *s1 = i1;
  }
}

// Sums over [i0, i1) in segments of at most L items so that 32-bit partial
// sums cannot wrap; flushes each segment into the 64-bit totals.
template <int LPL, typename F>
__device__ __forceinline__ void stream_chunked(const BP_CONST uint32_t *p, int i0, int i1, int L,
                                               uint64_t tot[LPL], F &&f) {
  for (int a = i0; a < i1;) {
    const int e = a + min(i1 - a, L);  // a + L could overflow int
    uint32_t s[LPL] = {};
    stream_u32<kStreamBlock<LPL>>(p, a, e, [&](uint32_t x) { f(x, s); });
    for (int j = 0; j < LPL; ++j) tot[j] += s[j];
    a = e;
  }
}

// stream_chunked over a monotone range with two bodies: fs for the items
// at most lim (small_part), ff for the others.  Integer sums: the order of
// the two parts does not change them.
template <int LPL, typename FS, typename FF>
__device__ __forceinline__ void stream_chunked_two(const BP_CONST uint32_t *p, int i0, int i1, int L, uint32_t lim,
                                                   uint64_t tot[LPL], FS &&fs, FF &&ff) {
  int s0, s1;
  small_part(p, i0, i1, lim, &s0, &s1);
  stream_chunked<LPL>(p, s0, s1, L, tot, fs);
  // the other items: one end of the range
  if (s0 > i0) stream_chunked<LPL>(p, i0, s0, L, tot, ff);
  else stream_chunked<LPL>(p, s1, i1, L, tot, ff);
}

template <int LPL>
__device__ __forceinline__ void tile_lams(const TileArgs &t, int64_t lam_out[LPL], uint32_t lam[LPL]) {
  for (int j = 0; j < LPL; ++j) {
    const int64_t L = t.lam0 + lane_id() + 64 * j;
    lam_out[j] = L;
    lam[j] = (uint32_t)(L <= t.hi ? L : t.lo);
  }
}

// Class-split item ranges of this chunk.
__device__ __forceinline__ void split_ranges(const TileArgs &t, int &b0, int &b1, int &s0, int &s1) {
  b0 = max(t.i0, t.nf);
  b1 = min(t.i1, t.nb);
  s0 = max(t.i0, t.nm);
  s1 = min(t.i1, t.nz);
}

// f_MT.  part = sum_big [c - w < lambda] (c - w) + sum_small [w >= lambda] w;
// S = sum_big w + n_mid c/2 + part.  The conditions are sign bits of 32-bit
// differences (all operands < 2^31), turned into masks: no compare, no select.
template <int LPL>
__device__ void part_mt(const TileArgs &t, const uint32_t lam[LPL], int64_t part[LPL]) {
  int b0, b1, s0, s1;
  split_ranges(t, b0, b1, s0, s1);
  uint32_t lm1[LPL];
  for (int j = 0; j < LPL; ++j) lm1[j] = lam[j] - 1u;  // lambda - 1 (wraps to -1 for lambda = 0)
  uint64_t acc[LPL] = {};
  const int L = chunk_len((uint64_t)t.C / 2 + 1);
  stream_chunked<LPL>(t.av, b0, b1, L, acc, [&](uint32_t a, uint32_t *s) {
    for (int j = 0; j < LPL; ++j) s[j] += (uint32_t)((int32_t)(a - lam[j]) >> 31) & a;
  });
  stream_chunked<LPL>(t.wv, s0, s1, L, acc, [&](uint32_t w, uint32_t *s) {
    for (int j = 0; j < LPL; ++j) s[j] += (uint32_t)((int32_t)(lm1[j] - w) >> 31) & w;
  });
  for (int j = 0; j < LPL; ++j) part[j] = (int64_t)acc[j];
}

// S_MT(lambda) over the streamed items (sizes c excluded); f_MT(c) = c.
__device__ __forceinline__ int64_t sum_mt(const TileArgs &t, int64_t lam, int64_t part) {
  return t.sumBig + (int64_t)(t.nm - t.nb) * (int64_t)(t.C / 2) + part;
}

// f_RAD2 (c/4 < lambda <= c/3), from counts of threshold crossings:
//   small: c3 [w >= lambda] + (c2 - c3) [w > c - 2 lambda]
//   big:   c2 + (c - c2 - c3) [w >= 2 lambda] + c3 [w > c - lambda]
//   mid:   c2
// part = the count terms; S = (n_big + n_mid) c2 + part.
template <int LPL>
__device__ void part_rad2(const TileArgs &t, const uint32_t lam[LPL], int64_t part[LPL]) {
  int b0, b1, s0, s1;
  split_ranges(t, b0, b1, s0, s1);
  // w >= t  <=>  (t - 1) - w < 0: count the sign bits (thresholds <= c, sizes < 2^31)
  uint32_t u1[LPL], u2[LPL], u3[LPL], u4[LPL];
  for (int j = 0; j < LPL; ++j) {
    u1[j] = lam[j] - 1u;                        // w >= lambda
    u2[j] = (uint32_t)t.C - 2u * lam[j];        // w >= c - 2 lambda + 1
    u3[j] = 2u * lam[j] - 1u;                   // w >= 2 lambda
    u4[j] = (uint32_t)t.C - lam[j];             // w >= c - lambda + 1
  }
  uint32_t n1[LPL] = {}, n2[LPL] = {}, n3[LPL] = {}, n4[LPL] = {};
  stream_u32<kStreamBlock<LPL>>(t.wv, s0, s1, [&](uint32_t w) {
    for (int j = 0; j < LPL; ++j) {
      n1[j] += (u1[j] - w) >> 31;
      n2[j] += (u2[j] - w) >> 31;
    }
  });
  stream_u32<kStreamBlock<LPL>>(t.wv, b0, b1, [&](uint32_t w) {
    for (int j = 0; j < LPL; ++j) {
      n3[j] += (u3[j] - w) >> 31;
      n4[j] += (u4[j] - w) >> 31;
    }
  });
  const int64_t C = t.C, c3 = C / 3, c2 = C / 2;
  for (int j = 0; j < LPL; ++j)
    part[j] = c3 * n1[j] + (c2 - c3) * n2[j] + (C - c2 - c3) * n3[j] + c3 * n4[j];
}

__device__ __forceinline__ int64_t sum_rad2(const TileArgs &t, int64_t lam, int64_t part) {
  return (int64_t)(t.nm - t.nf) * (int64_t)(t.C / 2) + part;
}

// f_FS1 (1 <= lambda <= 100): with n = w (lambda + 1) and q = floor(n / c),
// f = q c - w [c divides n].  Evaluated in fp64, exact: n < 2^38, and
// q = floor((n + 0.5) / c) is computed from (n + 0.5) * (1/c) whose relative
// error (2^-52) is below the distance 0.5/c of (n + 0.5)/c to an integer;
// the remainder fma(-q, c, n) is exact.  part = S = c sum q - sum_{c | n} w.
template <int LPL>
__device__ void part_fs1(const TileArgs &t, const uint32_t lam[LPL], int64_t part[LPL]) {
  double l1[LPL];
  for (int j = 0; j < LPL; ++j) l1[j] = (double)(lam[j] + 1u);
  const double Cd = (double)t.C;
  const double rc = 1.0 / Cd;
  double Q[LPL] = {}, D[LPL] = {};
  stream_u32(t.wv, max(t.i0, t.nf), min(t.i1, t.nz), [&](uint32_t wi) {
    const double w = (double)wi;
    for (int j = 0; j < LPL; ++j) {
      const double n = w * l1[j];
      const double q = floor((n + 0.5) * rc);
      const double rem = fma(-q, Cd, n);
      Q[j] += q;
      D[j] += rem == 0.0 ? w : 0.0;
    }
  });
  for (int j = 0; j < LPL; ++j) part[j] = (int64_t)Q[j] * (int64_t)t.C - (int64_t)D[j];
}

__device__ __forceinline__ int64_t sum_fs1(const TileArgs &t, int64_t lam, int64_t part) { return part; }

// f_CCM1 (1 <= lambda <= c/2), K = floor(c / lambda):
//   big 2K - 2 floor((c - w)/lambda), mid K, small 2 floor(w / lambda).
// part = 2 (sum_small floor(w/lambda) - sum_big floor((c-w)/lambda));
// S = 2K n_big + K n_mid + part.
template <int LPL>
__device__ void part_ccm1(const TileArgs &t, const uint32_t lam[LPL], int64_t part[LPL]) {
  int b0, b1, s0, s1;
  split_ranges(t, b0, b1, s0, s1);
  uint32_t mg[LPL], sh[LPL], ms[LPL];
  for (int j = 0; j < LPL; ++j) {
    const MagicU31 g = magic_u31(lam[j]);
    mg[j] = g.m;
    sh[j] = g.s;
    ms[j] = magic_short(lam[j]);
  }
  const uint32_t lmin = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)max(t.lo, t.lam0));
  const uint32_t lmax = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)min(t.hi, t.lam0 + (64 * LPL) - 1));
  // a lambda <= 2^32 for every lane (and lambda >= 2): one high multiply
  const uint32_t lim = lmin >= 2 ? 0xffffffffu / lmax : 0u;
  uint64_t hb[LPL] = {}, hs[LPL] = {};
  const int L = chunk_len(((uint64_t)t.C / 2) / lmin + 1);
  auto body = [&](uint32_t a, uint32_t *s) {
    const uint32_t a2 = 2u * a;
    for (int j = 0; j < LPL; ++j) s[j] += div_u31(a2, mg[j], sh[j]);
  };
  auto body_short = [&](uint32_t a, uint32_t *s) {
    for (int j = 0; j < LPL; ++j) s[j] += div_short(a, ms[j]);
  };
  stream_chunked_two<LPL>(t.av, b0, b1, L, lim, hb, body_short, body);
  stream_chunked_two<LPL>(t.av, s0, s1, L, lim, hs, body_short, body);
  for (int j = 0; j < LPL; ++j) part[j] = 2 * ((int64_t)hs[j] - (int64_t)hb[j]);
}

__device__ __forceinline__ int64_t sum_ccm1(const TileArgs &t, int64_t lam, int64_t part) {
  const int64_t K = (int64_t)((uint32_t)t.C / (uint32_t)lam);
  return 2 * K * (t.nb - t.nf) + K * (t.nm - t.nb) + part;
}

// f_VB2 (2 <= lambda <= c), h(a) = ceil(a lambda / c) - 1 for a >= 1:
//   big 2(lambda - 1) - 2 h(c - w), mid lambda - 1, small 2 h(w).
// part = 2 (sum_small h(w) - sum_big h(c - w));
// S = 2 (lambda - 1) n_big + (lambda - 1) n_mid + part.
template <int LPL>
__device__ void part_vb2(const TileArgs &t, const uint32_t lam[LPL], int64_t part[LPL]) {
  int b0, b1, s0, s1;
  split_ranges(t, b0, b1, s0, s1);
  uint32_t rlo[LPL], rhi[LPL];
  for (int j = 0; j < LPL; ++j) {
    const uint64_t R = vb2_recip(lam[j], (uint32_t)t.C);
    rlo[j] = (uint32_t)R;
    rhi[j] = (uint32_t)(R >> 32);
  }
  const uint32_t lmax = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)min(t.hi, t.lam0 + (64 * LPL) - 1));
  uint64_t hb[LPL] = {}, hs[LPL] = {};
  // h(a) <= a lambda / c <= lambda / 2 for a <= c/2
  const int L = chunk_len((uint64_t)lmax / 2 + 1);
  // a c <= 2^32: one high multiply by R's high word
  const uint32_t lim = 0xffffffffu / (uint32_t)t.C;
  auto body = [&](uint32_t a, uint32_t *s) {
    for (int j = 0; j < LPL; ++j) s[j] += vb2_part(a, rlo[j], rhi[j]);
  };
  auto body_short = [&](uint32_t a, uint32_t *s) {
    for (int j = 0; j < LPL; ++j) s[j] += vb2_part_short(a, rhi[j]);
  };
  stream_chunked_two<LPL>(t.av, b0, b1, L, lim, hb, body_short, body);
  stream_chunked_two<LPL>(t.av, s0, s1, L, lim, hs, body_short, body);
  for (int j = 0; j < LPL; ++j) part[j] = 2 * ((int64_t)hs[j] - (int64_t)hb[j]);
}

__device__ __forceinline__ int64_t sum_vb2(const TileArgs &t, int64_t lam, int64_t part) {
  const int64_t K = lam - 1;
  return 2 * K * (t.nb - t.nf) + K * (t.nm - t.nb) + part;
}

// f_BJ1 (1 <= lambda <= c), p = c mod lambda, q = floor(w / lambda),
// rem = w - q lambda:  f = q (lambda - p) + max(0, rem - p)
//                        = q (lambda - p) + (rem - p + |rem - p|) / 2.
// Per item the lane keeps Q += q and A += |w - (q lambda + p)| = |rem - p|.
// Over items 2S = (lambda - 2p) Q + A + W - n p with W = sum w, n = #items,
// so part = (lambda - 2p) Q + A and S = (part + W - n p) / 2.
template <int LPL>
__device__ void part_bj1(const TileArgs &t, const uint32_t lam[LPL], int64_t part[LPL]) {
  uint32_t ms[LPL], pm[LPL];
  for (int j = 0; j < LPL; ++j) {
    ms[j] = magic_short(lam[j]);
    pm[j] = (uint32_t)t.C % lam[j];
  }
  const uint32_t lmin = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)max(t.lo, t.lam0));
  const uint32_t lmax = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)min(t.hi, t.lam0 + (64 * LPL) - 1));
  const int a0 = max(t.i0, t.nf), a1 = min(t.i1, t.nz);
  if (2ull * lmin > (uint64_t)(uint32_t)t.C) {
    // Every lane's lambda exceeds c/2: floor(c / lambda) = 1 and p = c - lambda,
    // so for 0 < w < c f = clamp(w - p, 0, 2 lambda - c)
    // = (|w - p| - |w - lambda| + 2 lambda - c) / 2, two v_sad_u32 per item.
    // part = 2S - W + n p = A1 - A2 + n lambda - W over the streamed items,
    // A1 = sum |w - p|, A2 = sum |w - lambda| (each term below c).
    uint64_t A1[LPL] = {}, A2[LPL] = {};
    const int L = chunk_len((uint64_t)(uint32_t)t.C);
    for (int i0 = a0; i0 < a1;) {
      const int e = i0 + min(a1 - i0, L);  // i0 + L could overflow int
      uint32_t s1[LPL] = {}, s2[LPL] = {};
      stream_u32<kStreamBlock<LPL>>(t.wv, i0, e, [&](uint32_t w) {
        for (int j = 0; j < LPL; ++j) {
          s1[j] = sad_u32(w, pm[j], s1[j]);
          s2[j] = sad_u32(w, lam[j], s2[j]);
        }
      });
      for (int j = 0; j < LPL; ++j) {
        A1[j] += s1[j];
        A2[j] += s2[j];
      }
      i0 = e;
    }
    const int64_t n = a1 > a0 ? a1 - a0 : 0;
    const int64_t W = a1 > a0 ? t.prec[a1] - t.prec[a0] : 0;
    for (int j = 0; j < LPL; ++j) part[j] = (int64_t)A1[j] - (int64_t)A2[j] + n * (int64_t)lam[j] - W;
    return;
  }
  // w lambda <= 2^32 for every lane (and lambda >= 2): one high multiply
  const uint32_t lim = lmin >= 2 ? 0xffffffffu / lmax : 0u;
  uint64_t Q[LPL] = {}, A[LPL] = {};
  const uint64_t inc = max((uint64_t)((uint32_t)t.C / lmin), (uint64_t)lmax) + 1;
  const int L = chunk_len(inc);
  // sums over [x0, x1) in segments of at most L items, q from quot(w, j)
  auto run = [&](int x0, int x1, auto &&quot) {
    for (int i0 = x0; i0 < x1;) {
      const int e = i0 + min(x1 - i0, L);  // i0 + L could overflow int
      uint32_t sq[LPL] = {}, sa[LPL] = {};
      stream_u32<kStreamBlock<LPL>>(t.wv, i0, e, [&](uint32_t w) {
        for (int j = 0; j < LPL; ++j) {
          const uint32_t q = quot(w, j);
          const uint32_t v = q * lam[j] + pm[j];
          sq[j] += q;
          sa[j] = sad_u32(w, v, sa[j]);
        }
      });
      for (int j = 0; j < LPL; ++j) {
        Q[j] += sq[j];
        A[j] += sa[j];
      }
      i0 = e;
    }
  };
  int s0, s1;
  small_part(t.wv, a0, a1, lim, &s0, &s1);
  run(s0, s1, [&](uint32_t w, int j) { return div_short(w, ms[j]); });
  // the other items (one end of the range), by the two-step quotient
  const int f0 = s0 > a0 ? a0 : s1, f1 = s0 > a0 ? s0 : a1;
  if (f0 < f1) {
    uint32_t mg[LPL], sh[LPL];
    for (int j = 0; j < LPL; ++j) {
      const MagicU31 g = magic_u31(lam[j]);
      mg[j] = g.m;
      sh[j] = g.s;
    }
    run(f0, f1, [&](uint32_t w, int j) { return div_u31(2u * w, mg[j], sh[j]); });
  }
  for (int j = 0; j < LPL; ++j)
    part[j] = ((int64_t)lam[j] - 2 * (int64_t)pm[j]) * (int64_t)Q[j] + (int64_t)A[j];
}

__device__ __forceinline__ int64_t sum_bj1(const TileArgs &t, int64_t lam, int64_t part) {
  const int64_t p = (int64_t)((uint32_t)t.C % (uint32_t)lam);
  const int64_t n = t.nz - t.nf;
  return (part + t.sumNZ - n * p) >> 1;  // the sum is even and >= 0
}

// ---------------------------------------------------------------------------
// Segment sums.  The table bidx[b] = #{sizes >= b B}, B = 2^bsh, over the
// decreasing sizes bounds where a threshold falls: every size before
// pos_ge(v) is >= v, every size from pos_lt(v) on is < v.  A tile's
// parameters are consecutive, so for each threshold family the thresholds
// of its lanes lie in one window [tlo, thi], and only the sizes between
// pos_ge(thi + 1) and pos_lt(tlo + 1) need a per-lane test; the sizes
// before count in full, those after not at all.

__device__ __forceinline__ int32_t seg_pos_ge(const TileArgs &t, int64_t v) {
  return t.bidx[(v + (1ll << t.bsh) - 1) >> t.bsh];
}

__device__ __forceinline__ int32_t seg_pos_lt(const TileArgs &t, int64_t v) { return t.bidx[v >> t.bsh]; }

__device__ __forceinline__ int32_t clamp32(int32_t x, int32_t lo, int32_t hi) { return min(max(x, lo), hi); }

__device__ __forceinline__ int64_t uniform64(int64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// U(t) = sum over sizes [i0, i1) of max(0, w - t), for each lane threshold
// th[j] in [tlo, thi].  Sizes before p0 exceed every threshold and add
// w - t; in [p0, p1) max(0, w - t) = ((w - t) + |w - t|) / 2, with |w - t|
// summed per lane (v_sad_u32); sizes from p1 on add 0.  So
// 2 U = (H0 - N0 t) + (H1 - N1 t) + sum_[p0,p1) |w - t| with H, N the sum
// and count of [i0, p0) and [i0, p1).
template <int LPL>
__device__ void seg_u(const TileArgs &t, int32_t i0, int32_t i1, int64_t tlo, int64_t thi, const uint32_t th[LPL],
                      int64_t u[LPL]) {
  const int32_t p0 = __builtin_amdgcn_readfirstlane(clamp32(seg_pos_ge(t, thi + 1), i0, i1));
  const int32_t p1 = __builtin_amdgcn_readfirstlane(clamp32(seg_pos_lt(t, tlo + 1), p0, i1));
  const int64_t base = t.prec[i0];
  const int64_t h = (t.prec[p0] - base) + (t.prec[p1] - base);
  const int64_t n = (int64_t)(p0 - i0) + (int64_t)(p1 - i0);
  uint64_t sad[LPL] = {};
  stream_chunked<LPL>(t.wv, p0, p1, chunk_len((uint64_t)t.C), sad, [&](uint32_t w, uint32_t *s) {
    for (int j = 0; j < LPL; ++j) s[j] = sad_u32(w, th[j], s[j]);
  });
  for (int j = 0; j < LPL; ++j) u[j] = (h - n * (int64_t)th[j] + (int64_t)sad[j]) >> 1;
}

// f_BJ1 by segments.  Over the sizes 0 < w < c, with K = floor(c / lambda)
// and p = c mod lambda, grouping the sizes by q = floor(w / lambda) turns
// sum_w f_BJ1(w, lambda) into the telescoping form
//   S = sum_{m=1..K} U(c - m lambda) - sum_{j=1..K} U(j lambda),
// 2K threshold sums.  Lanes whose K is below the tile's largest mask the
// extra terms.  Returns the same part as part_bj1 (part = 2S - W + n p).
template <int LPL>
__device__ void part_bj1_seg(const TileArgs &t, const int64_t lam_out[LPL], int64_t part[LPL]) {
  const int64_t C = t.C;
  const int64_t l0 = uniform64(max(t.lo, t.lam0));
  const int64_t l1 = uniform64(min(t.hi, t.lam0 + 64 * LPL - 1));
  uint32_t lam[LPL];
  int32_t K[LPL];
  for (int j = 0; j < LPL; ++j) {
    lam[j] = (uint32_t)min(max(lam_out[j], l0), l1);
    K[j] = (int32_t)((uint32_t)C / lam[j]);
  }
  const int32_t kmax = (int32_t)(C / l0);
  // chunk qc of qn takes q in [1 + floor(kmax qc / qn), floor(kmax (qc + 1) / qn)]
  const int32_t qa = 1 + (int32_t)((int64_t)kmax * t.qc / t.qn);
  const int32_t qb = (int32_t)((int64_t)kmax * (t.qc + 1) / t.qn);
  int64_t acc[LPL] = {};
  for (int32_t q = qa; q <= qb; ++q) {
    uint32_t th[LPL];
    int64_t u[LPL];
    {
      const int64_t tlo = (int64_t)q * l0, thi = min(C, (int64_t)q * l1);
      for (int j = 0; j < LPL; ++j) th[j] = (uint32_t)min(max((int64_t)q * lam[j], tlo), thi);
      seg_u<LPL>(t, t.nf, t.nz, tlo, thi, th, u);
      for (int j = 0; j < LPL; ++j) acc[j] -= q <= K[j] ? u[j] : 0;
    }
    {
      const int64_t tlo = max((int64_t)0, C - (int64_t)q * l1), thi = C - (int64_t)q * l0;
      for (int j = 0; j < LPL; ++j) th[j] = (uint32_t)min(max(C - (int64_t)q * lam[j], tlo), thi);
      seg_u<LPL>(t, t.nf, t.nz, tlo, thi, th, u);
      for (int j = 0; j < LPL; ++j) acc[j] += q <= K[j] ? u[j] : 0;
    }
  }
  // the instance constant goes with chunk 0 only, so the chunks' parts add up
  const int64_t n = t.nz - t.nf;
  for (int j = 0; j < LPL; ++j)
    part[j] = 2 * acc[j] - (t.qc == 0 ? t.sumNZ - n * (int64_t)((uint32_t)C % lam[j]) : 0);
}

// #{w in [i0, i1) : w >= th[j]} for thresholds in [tlo, thi], 1 <= tlo:
// sizes before p0 are >= thi, sizes from p1 on are < tlo; in between one
// sign bit per size and parameter.
template <int LPL>
__device__ void seg_count(const TileArgs &t, int32_t i0, int32_t i1, int64_t tlo, int64_t thi, const uint32_t th[LPL],
                          int64_t cnt[LPL]) {
  const int32_t p0 = __builtin_amdgcn_readfirstlane(clamp32(seg_pos_ge(t, thi), i0, i1));
  const int32_t p1 = __builtin_amdgcn_readfirstlane(clamp32(seg_pos_lt(t, tlo), p0, i1));
  uint32_t tm1[LPL], n[LPL];
  for (int j = 0; j < LPL; ++j) {
    tm1[j] = th[j] - 1u;
    n[j] = 0;
  }
  stream_u32(t.wv, p0, p1, [&](uint32_t w) {
    for (int j = 0; j < LPL; ++j) n[j] += (tm1[j] - w) >> 31;
  });
  for (int j = 0; j < LPL; ++j) cnt[j] = (int64_t)(p0 - i0) + (int64_t)n[j];
}

// f_CCM1 by segments: sum_small floor(w / lambda) = sum_{q >= 1} #{small
// w >= q lambda} and sum_big floor((c - w) / lambda) = sum_{q >= 1} #{big
// w <= c - q lambda}.  Thresholds past the reach of a class give exact
// zeros (small) or full counts (big), so they are clamped to the class
// edge and no lane is masked.  Returns the same part as part_ccm1.
template <int LPL>
__device__ void part_ccm1_seg(const TileArgs &t, const int64_t lam_out[LPL], int64_t part[LPL]) {
  const int64_t C = t.C;
  const int64_t l0 = uniform64(max(t.lo, t.lam0));
  const int64_t l1 = uniform64(min(t.hi, t.lam0 + 64 * LPL - 1));
  uint32_t lam[LPL];
  for (int j = 0; j < LPL; ++j) lam[j] = (uint32_t)min(max(lam_out[j], l0), l1);
  const int64_t half = C / 2;
  const int64_t scap = (C - 1) / 2 + 1;  // every small size is below it
  const int64_t bfloor = half + 1;       // every big size reaches it
  const int64_t nbig = t.nb - t.nf;
  const int32_t qmax = (int32_t)(half / l0);
  // chunk qc of qn takes q in [1 + floor(qmax qc / qn), floor(qmax (qc + 1) / qn)]
  const int32_t qa = 1 + (int32_t)((int64_t)qmax * t.qc / t.qn);
  const int32_t qb = (int32_t)((int64_t)qmax * (t.qc + 1) / t.qn);
  int64_t acc[LPL] = {};
  for (int32_t q = qa; q <= qb; ++q) {
    uint32_t th[LPL];
    int64_t c[LPL];
    {
      const int64_t tlo = min((int64_t)q * l0, scap), thi = min((int64_t)q * l1, scap);
      for (int j = 0; j < LPL; ++j) th[j] = (uint32_t)min((int64_t)q * lam[j], scap);
      seg_count<LPL>(t, t.nm, t.nz, tlo, thi, th, c);
      for (int j = 0; j < LPL; ++j) acc[j] += c[j];
    }
    {
      const int64_t tlo = max(C - (int64_t)q * l1 + 1, bfloor), thi = max(C - (int64_t)q * l0 + 1, bfloor);
      for (int j = 0; j < LPL; ++j) th[j] = (uint32_t)max(C - (int64_t)q * lam[j] + 1, bfloor);
      seg_count<LPL>(t, t.nf, t.nb, tlo, thi, th, c);
      for (int j = 0; j < LPL; ++j) acc[j] -= nbig - c[j];
    }
  }
  for (int j = 0; j < LPL; ++j) part[j] = 2 * acc[j];
}

// #{w >= v} and sum{w >= v} over all reduced sizes, 0 <= v <= c + 1, from
// the value tables.
__device__ __forceinline__ void lut_ge(const TileArgs &t, int64_t v, int64_t &cnt, int64_t &sum) {
  const int64_t c = v >> kVtChunkLog;
  cnt = (int64_t)t.vc[v] + (int64_t)t.vo[2 * c];
  sum = (int64_t)t.vs[v] + (int64_t)t.vo[2 * c + 1];
}

// U(th) = sum over the sizes 0 < w < c of max(0, w - th), 0 <= th <= c:
// sum{w >= th} - th #{w >= th} over all sizes, less the nf sizes c.
__device__ __forceinline__ int64_t lut_u(const TileArgs &t, int64_t th) {
  int64_t n, s;
  lut_ge(t, th, n, s);
  return s - th * n - (int64_t)t.nf * ((int64_t)t.C - th);
}

// f_BJ1 by lookups: the telescoping form of part_bj1_seg,
//   S = sum_{q=1..K} U(c - q lambda) - U(q lambda),
// each lane over its own K = floor(c / lambda), this chunk's share of the q
// range.  Returns the same part as part_bj1 (part = 2S - W + n p).
template <int LPL>
__device__ void part_bj1_lut(const TileArgs &t, const int64_t lam_out[LPL], int64_t part[LPL]) {
  const int64_t C = t.C;
  const int64_t l0 = uniform64(max(t.lo, t.lam0));
  const int64_t l1 = uniform64(min(t.hi, t.lam0 + 64 * LPL - 1));
  int64_t lam[LPL], acc[LPL];
  int32_t K[LPL];
  for (int j = 0; j < LPL; ++j) {
    lam[j] = min(max(lam_out[j], l0), l1);
    K[j] = (int32_t)((uint32_t)C / (uint32_t)lam[j]);  // 32-bit: c < 2^31
    acc[j] = 0;
  }
  const int64_t kmax = (int64_t)((uint32_t)C / (uint32_t)l0);
  const int64_t qa = 1 + (int64_t)((uint64_t)kmax * (uint32_t)t.qc / (uint32_t)t.qn),
                qb = (int64_t)((uint64_t)kmax * (uint32_t)(t.qc + 1) / (uint32_t)t.qn);
  // one parameter slot at a time (few registers: this runs inside the sweep
  // kernel's 64-register budget), two q per step with their loads in flight
  for (int j = 0; j < LPL; ++j) {
    const int64_t qe = min(qb, K[j]);
    int64_t a0 = 0, a1 = 0;
    int64_t q = qa;
    for (; q + 1 <= qe; q += 2) {
      a0 += lut_u(t, C - q * lam[j]) - lut_u(t, q * lam[j]);
      a1 += lut_u(t, C - (q + 1) * lam[j]) - lut_u(t, (q + 1) * lam[j]);
    }
    if (q <= qe) a0 += lut_u(t, C - q * lam[j]) - lut_u(t, q * lam[j]);
    acc[j] = a0 + a1;
  }
  const int64_t n = t.nz - t.nf;
  for (int j = 0; j < LPL; ++j)
    part[j] = 2 * acc[j] - (t.qc == 0 ? t.sumNZ - n * (int64_t)((uint32_t)C % (uint32_t)lam[j]) : 0);
}

// f_CCM1 by lookups: the counts of part_ccm1_seg, sum_{q >= 1} #{small w >=
// q lambda} - #{big w <= c - q lambda}, each lane over its own q <= floor(c/2)
// / lambda (larger q add nothing), this chunk's share of the q range.
template <int LPL>
__device__ void part_ccm1_lut(const TileArgs &t, const int64_t lam_out[LPL], int64_t part[LPL]) {
  const int64_t C = t.C;
  const int64_t l0 = uniform64(max(t.lo, t.lam0));
  const int64_t l1 = uniform64(min(t.hi, t.lam0 + 64 * LPL - 1));
  const int64_t half = C / 2;
  const int64_t scap = (C - 1) / 2 + 1;  // the small sizes are those below it (and above 0)
  const int64_t nbig = t.nb - t.nf;
  int64_t ns, ss;
  lut_ge(t, scap, ns, ss);  // #{w >= scap}
  int64_t lam[LPL], acc[LPL];
  int32_t Q[LPL];
  for (int j = 0; j < LPL; ++j) {
    lam[j] = min(max(lam_out[j], l0), l1);
    Q[j] = (int32_t)((uint32_t)half / (uint32_t)lam[j]);  // 32-bit: c < 2^31
    acc[j] = 0;
  }
  const int64_t qmax = (int64_t)((uint32_t)half / (uint32_t)l0);
  const int64_t qa = 1 + (int64_t)((uint64_t)qmax * (uint32_t)t.qc / (uint32_t)t.qn),
                qb = (int64_t)((uint64_t)qmax * (uint32_t)(t.qc + 1) / (uint32_t)t.qn);
  // one parameter slot at a time, two q per step (as part_bj1_lut)
  auto term = [&](int64_t q, int64_t l) {
    int64_t a, b, s;
    lut_ge(t, q * l, a, s);          // small sizes >= q lambda: #{w >= q lambda} - #{w >= scap}
    lut_ge(t, C - q * l + 1, b, s);  // big sizes >= c - q lambda + 1, less the nf sizes c
    return (a - ns) - (nbig - (b - t.nf));
  };
  for (int j = 0; j < LPL; ++j) {
    const int64_t qe = min(qb, Q[j]);
    int64_t a0 = 0, a1 = 0;
    int64_t q = qa;
    for (; q + 1 <= qe; q += 2) {
      a0 += term(q, lam[j]);
      a1 += term(q + 1, lam[j]);
    }
    if (q <= qe) a0 += term(q, lam[j]);
    acc[j] = a0 + a1;
  }
  for (int j = 0; j < LPL; ++j) part[j] = 2 * acc[j];
}

// f_RAD2 by segments: the four threshold counts of part_rad2 (small sizes
// >= lambda and >= c - 2 lambda + 1, big sizes >= 2 lambda and
// >= c - lambda + 1), one window each per tile.  Same part as part_rad2.
template <int LPL>
__device__ void part_rad2_seg(const TileArgs &t, const int64_t lam_out[LPL], int64_t part[LPL]) {
  const int64_t C = t.C;
  const int64_t l0 = uniform64(max(t.lo, t.lam0));
  const int64_t l1 = uniform64(min(t.hi, t.lam0 + 64 * LPL - 1));
  uint32_t lam[LPL], th[LPL];
  for (int j = 0; j < LPL; ++j) lam[j] = (uint32_t)min(max(lam_out[j], l0), l1);
  int64_t n1[LPL], n2[LPL], n3[LPL], n4[LPL];
  for (int j = 0; j < LPL; ++j) th[j] = lam[j];
  seg_count<LPL>(t, t.nm, t.nz, l0, l1, th, n1);
  for (int j = 0; j < LPL; ++j) th[j] = (uint32_t)(C - 2 * (int64_t)lam[j] + 1);
  seg_count<LPL>(t, t.nm, t.nz, C - 2 * l1 + 1, C - 2 * l0 + 1, th, n2);
  for (int j = 0; j < LPL; ++j) th[j] = 2u * lam[j];
  seg_count<LPL>(t, t.nf, t.nb, 2 * l0, 2 * l1, th, n3);
  for (int j = 0; j < LPL; ++j) th[j] = (uint32_t)(C - (int64_t)lam[j] + 1);
  seg_count<LPL>(t, t.nf, t.nb, C - l1 + 1, C - l0 + 1, th, n4);
  const int64_t c3 = C / 3, c2 = C / 2;
  for (int j = 0; j < LPL; ++j)
    part[j] = c3 * n1[j] + (c2 - c3) * n2[j] + (C - c2 - c3) * n3[j] + c3 * n4[j];
}

// f_MT by segments: the small sizes with w >= lambda and the big ones with
// c - w < lambda (w >= c - lambda + 1) are prefixes of their classes; each
// class has one window per tile.  Returns the same part as part_mt.
template <int LPL>
__device__ void part_mt_seg(const TileArgs &t, const int64_t lam_out[LPL], int64_t part[LPL]) {
  const int64_t C = t.C;
  const int64_t l0 = uniform64(max(t.lo, t.lam0));
  const int64_t l1 = uniform64(min(t.hi, t.lam0 + 64 * LPL - 1));
  uint32_t lam[LPL], lm1[LPL];
  for (int j = 0; j < LPL; ++j) {
    lam[j] = (uint32_t)min(max(lam_out[j], l0), l1);
    lm1[j] = lam[j] - 1u;  // wraps to -1 for lambda = 0: every size counts
  }
  const int32_t ps0 = __builtin_amdgcn_readfirstlane(clamp32(seg_pos_ge(t, l1), t.nm, t.nz));
  const int32_t ps1 = __builtin_amdgcn_readfirstlane(clamp32(seg_pos_lt(t, l0), ps0, t.nz));
  const int32_t pb0 = __builtin_amdgcn_readfirstlane(clamp32(seg_pos_ge(t, C - l0 + 1), t.nf, t.nb));
  const int32_t pb1 = __builtin_amdgcn_readfirstlane(clamp32(seg_pos_lt(t, C - l1 + 1), pb0, t.nb));
  uint64_t acc[LPL] = {};
  const int L = chunk_len((uint64_t)C / 2 + 1);
  stream_chunked<LPL>(t.av, pb0, pb1, L, acc, [&](uint32_t a, uint32_t *s) {
    for (int j = 0; j < LPL; ++j) s[j] += (uint32_t)((int32_t)(a - lam[j]) >> 31) & a;
  });
  stream_chunked<LPL>(t.wv, ps0, ps1, L, acc, [&](uint32_t w, uint32_t *s) {
    for (int j = 0; j < LPL; ++j) s[j] += (uint32_t)((int32_t)(lm1[j] - w) >> 31) & w;
  });
  const int64_t base = (int64_t)(pb0 - t.nf) * C - (t.prec[pb0] - t.prec[t.nf]) + (t.prec[ps0] - t.prec[t.nm]);
  for (int j = 0; j < LPL; ++j) part[j] = base + (int64_t)acc[j];
}

// sum over the streamed items (sizes c excluded) of f(w, lambda), from a
// tile's part
__device__ __forceinline__ int64_t sum_bound(int bound, const TileArgs &t, int64_t lam, int64_t part) {
  switch (bound) {
    case kMT: return sum_mt(t, lam, part);
    case kRAD2: return sum_rad2(t, lam, part);
    case kFS1: return sum_fs1(t, lam, part);
    case kCCM1: return sum_ccm1(t, lam, part);
    case kVB2: return sum_vb2(t, lam, part);
    default: return sum_bj1(t, lam, part);
  }
}

// f(c, lambda) of each function (Sec. 3.1): c (MT, RAD2), c lambda (FS1),
// 2 floor(c / lambda) (CCM1), 2 (lambda - 1) (VB2), floor(c / lambda)
// (lambda - c mod lambda) (BJ1).
__device__ __forceinline__ int64_t fc_bound(int bound, int32_t C, int64_t lam) {
  const uint32_t c32 = (uint32_t)C, l32 = (uint32_t)lam;
  switch (bound) {
    case kMT: case kRAD2: return C;
    case kFS1: return (int64_t)C * lam;
    case kCCM1: return 2 * (int64_t)(c32 / l32);
    case kVB2: return 2 * (lam - 1);
    default: return (int64_t)(c32 / l32) * (lam - (int64_t)(c32 % l32));
  }
}

// The bound at lambda without the items of size c (each adds exactly 1):
// ceil(S / f(c, lambda)).
__device__ __forceinline__ int64_t fin_bound(int bound, const TileArgs &t, int64_t lam, int64_t part) {
  return ceil_div_small(sum_bound(bound, t, lam, part), fc_bound(bound, t.C, lam));
}

// Node state of a served request: S(lambda) over all reduced items, the
// nf items of size c included (each adds f(c, lambda)).
__device__ __forceinline__ void store_state(int bound, const TileArgs &t, int64_t lam, int64_t part) {
  t.node[lam - t.lo] = (long long)(sum_bound(bound, t, lam, part) + (int64_t)t.nf * fc_bound(bound, t.C, lam));
}

template <int LPL>
__device__ __forceinline__ void store_state_lanes(int bound, const TileArgs &t, const int64_t lam[LPL],
                                                  const int64_t part[LPL]) {
  for (int j = 0; j < LPL; ++j)
    if (lam[j] >= t.lo && lam[j] <= t.hi) store_state(bound, t, lam[j], part[j]);
}

// Parameters of the range [lo, hi] inside [a, b].
__device__ __forceinline__ int64_t overlap(int64_t a, int64_t b, int64_t lo, int64_t hi) {
  const int64_t x = max(a, lo), y = min(b, hi);
  return y >= x ? y - x + 1 : 0;
}

// Parameters of the bound's range a tile of entry e evaluates (a mirrored
// VB2 tile: its dense half's lambdas and their mirrors c - lambda), for the
// count of skipped work.
template <int LPL>
__device__ __forceinline__ int64_t tile_params(int32_t mode, int32_t aux, const TileArgs &t, int64_t lam0) {
  const int64_t lam1 = lam0 + 64 * LPL - 1;
  if (mode != kModeMirror) return overlap(lam0, lam1, t.lo, t.hi);
  const int64_t b = min(lam1, (int64_t)aux);
  return overlap(lam0, b, t.lo, t.hi) + overlap(lam0, b, (int64_t)t.C - t.hi, (int64_t)t.C - t.lo);
}

// L2 (Sec. 3.1) evaluated at the parameters where it can change: the range's
// first parameter and w + 1, c - w + 1 for every size.  Candidate index
// c = 0 is lo; c = 1 + 2i is w_i + 1; c = 2 + 2i is c - w_i + 1.
// With nbig = #{2w > c} (every big item is in W1 or W2):
//   n1 = #{w > c - lambda}, n2 = nbig - n1, sum W2 = pre[nbig] - pre[n1],
//   W3 = {lambda <= w <= c/2} = sorted[nbig, j3) with j3 = #{w >= lambda},
//   L2(lambda) = nbig + max(0, ceil((sum W3 - (c n2 - sum W2)) / c)).
// The counts #{w > x} over the decreasing sizes are found by binary lifting
// with a fixed number of steps, all 2 LPL searches of a lane in lockstep, so
// that their loads are in flight together.
template <int LPL>
__device__ void tile_l2(const TileArgs &t, int64_t lam_out[LPL], int64_t lbp[LPL], bool ok[LPL]) {
  const int64_t C = t.C;
  const int32_t nbig = t.nb;  // includes the items of size c
  const int32_t r = t.r;
  int64_t x1[LPL], x3[LPL];
  int32_t p1[LPL], p3[LPL];
  for (int j = 0; j < LPL; ++j) {
    const int64_t cidx = t.lam0 + lane_id() + 64 * j;
    int64_t lam = -1;
    if (cidx == 0) lam = t.lo;
    else if (cidx <= 2 * (int64_t)r) {
      const int64_t i = (cidx - 1) >> 1;
      const int64_t w = t.sorted[i];
      lam = ((cidx - 1) & 1) ? C - w + 1 : w + 1;
    }
    ok[j] = lam >= t.lo && lam <= t.hi;
    if (!ok[j]) lam = t.lo;
    lam_out[j] = lam;
    x1[j] = C - lam;  // n1 = #{w > c - lambda}
    x3[j] = lam - 1;  // j3 = #{w > lambda - 1}
    p1[j] = 0;
    p3[j] = 0;
  }
  for (int32_t step = r > 0 ? (int32_t)(1u << (31 - __clz(r))) : 0; step > 0; step >>= 1) {
    for (int j = 0; j < LPL; ++j) {
      const int32_t q1 = p1[j] + step, q3 = p3[j] + step;
      const int64_t v1 = t.sorted[min(q1, r) - 1];
      const int64_t v3 = t.sorted[min(q3, r) - 1];
      if (q1 <= r && v1 > x1[j]) p1[j] = q1;
      if (q3 <= r && v3 > x3[j]) p3[j] = q3;
    }
  }
  for (int j = 0; j < LPL; ++j) {
    const int32_t n1 = p1[j], j3 = p3[j];
    const int64_t n2 = nbig - n1;
    const int64_t s2 = t.pre[nbig] - t.pre[n1];
    const int64_t s3 = j3 > nbig ? t.pre[j3] - t.pre[nbig] : 0;
    const int64_t x = s3 - (C * n2 - s2);
    lbp[j] = nbig + (x > 0 ? ceil_div_small(x, C) : 0);
  }
}

// #{w > x[k]} over the decreasing sizes for NT thresholds, by binary
// lifting with a fixed number of steps, the NT searches in lockstep so that
// their loads are in flight together.
template <int NT>
__device__ __forceinline__ void count_above(const TileArgs &t, const int64_t (&x)[NT], int32_t (&n)[NT]) {
  const int32_t r = t.r;
  for (int k = 0; k < NT; ++k) n[k] = 0;
  for (int32_t step = r > 0 ? (int32_t)(1u << (31 - __clz(r))) : 0; step > 0; step >>= 1) {
    for (int k = 0; k < NT; ++k) {
      const int32_t q = n[k] + step;
      const int64_t v = t.sorted[min(q, r) - 1];
      if (q <= r && v > x[k]) n[k] = q;
    }
  }
}

// f_MT over its change points (Sec. 3.1; the candidate set of L2): lo and,
// for every size w, w + 1 and c - w + 1.  Between them every size keeps its
// case, so S(lambda) is constant there and the smallest parameter of each
// piece is a candidate.  With n1 = #{w > c - lambda} (value c each) and
// j3 = #{w >= lambda}, the sizes [n1, j3) of the sorted order count w:
//   S = c n1 + pre[j3] - pre[n1],  L = ceil(S / c) = n1 + ceil((pre[j3] - pre[n1]) / c);
// lbp leaves out the nf sizes c (k_finalize adds them back, as for every DFF).
template <int LPL>
__device__ void tile_mt_cand(const TileArgs &t, int64_t lam_out[LPL], int64_t lbp[LPL], bool ok[LPL]) {
  const int64_t C = t.C;
  const int32_t r = t.r;
  for (int j = 0; j < LPL; ++j) {
    const int64_t cidx = t.lam0 + lane_id() + 64 * j;
    int64_t lam = -1;
    if (cidx == 0) lam = t.lo;
    else if (cidx <= 2 * (int64_t)r) {
      const int64_t w = t.sorted[(cidx - 1) >> 1];
      lam = ((cidx - 1) & 1) ? C - w + 1 : w + 1;
    }
    ok[j] = lam >= t.lo && lam <= t.hi;
    if (!ok[j]) lam = t.lo;
    lam_out[j] = lam;
    const int64_t x[2] = {C - lam, lam - 1};  // n1 = #{w > c - lambda}, j3 = #{w > lambda - 1}
    int32_t n[2];
    count_above<2>(t, x, n);
    const int32_t n1 = n[0], j3 = max(n[1], n1);
    lbp[j] = (int64_t)(n1 - t.nf) + ceil_div_small(t.pre[j3] - t.pre[n1], C);
  }
}

// f_RAD2 over its change points (Sec. 3.1): lo and, for every size w, w + 1,
// c - w + 1, floor((c - w)/2) + 1 and floor(w/2) + 1, where w crosses lambda,
// c - lambda, c - 2 lambda or 2 lambda.  For c/4 < lambda <= c/3 the cases
// are, with a = #{w >= lambda}, b = #{w > c - 2 lambda}, g = #{w >= 2 lambda},
// e = #{w > c - lambda} (a >= b >= g >= e):
//   lambda <= w <= c - 2 lambda        (a - b sizes)  floor(c/3)
//   c - 2 lambda < w < 2 lambda        (b - g)        floor(c/2)
//   2 lambda <= w <= c - lambda        (g - e)        c - floor(c/3)
//   w > c - lambda                     (e)            c
// and f(c, lambda) = c; lbp leaves out the nf sizes c.
template <int LPL>
__device__ void tile_rad2_cand(const TileArgs &t, int64_t lam_out[LPL], int64_t lbp[LPL], bool ok[LPL]) {
  const int64_t C = t.C;
  const int32_t r = t.r;
  const int64_t f3 = C / 3, f2 = C / 2;
  for (int j = 0; j < LPL; ++j) {
    const int64_t cidx = t.lam0 + lane_id() + 64 * j;
    int64_t lam = -1;
    if (cidx == 0) lam = t.lo;
    else if (cidx <= 4 * (int64_t)r) {
      const int64_t w = t.sorted[(cidx - 1) >> 2];
      switch ((cidx - 1) & 3) {
        case 0: lam = w + 1; break;
        case 1: lam = C - w + 1; break;
        case 2: lam = (C - w) / 2 + 1; break;
        default: lam = w / 2 + 1; break;
      }
    }
    ok[j] = lam >= t.lo && lam <= t.hi;
    if (!ok[j]) lam = t.lo;
    lam_out[j] = lam;
    const int64_t x[4] = {lam - 1, C - 2 * lam, 2 * lam - 1, C - lam};
    int32_t n[4];
    count_above<4>(t, x, n);
    const int64_t a = n[0], b = n[1], g = n[2], e = n[3];
    const int64_t S = f3 * (a - b) + f2 * (b - g) + (C - f3) * (g - e) + C * e;
    lbp[j] = ceil_div_small(S, C) - t.nf;
  }
}

// L2 aggregates of the node state at every lambda of the tile, lambda in
// [0, c/2]: n1 = #{w > c - lambda} and T = sum W2 + sum W3, from the sorted
// sizes (binary lifting, as tile_l2) and their prefix sums.
template <int LPL>
__device__ void tile_l2_state(const TileArgs &t) {
  const int64_t C = t.C;
  const int32_t nbig = t.nb;
  const int32_t r = t.r;
  const int64_t half = C / 2;
  int64_t lam[LPL], x1[LPL], x3[LPL];
  int32_t p1[LPL], p3[LPL];
  for (int j = 0; j < LPL; ++j) {
    lam[j] = t.lam0 + lane_id() + 64 * j;
    const int64_t l = lam[j] <= half ? lam[j] : half;
    x1[j] = C - l;
    x3[j] = l - 1;
    p1[j] = 0;
    p3[j] = 0;
  }
  for (int32_t step = r > 0 ? (int32_t)(1u << (31 - __clz(r))) : 0; step > 0; step >>= 1) {
    for (int j = 0; j < LPL; ++j) {
      const int32_t q1 = p1[j] + step, q3 = p3[j] + step;
      const int64_t v1 = t.sorted[min(q1, r) - 1];
      const int64_t v3 = t.sorted[min(q3, r) - 1];
      if (q1 <= r && v1 > x1[j]) p1[j] = q1;
      if (q3 <= r && v3 > x3[j]) p3[j] = q3;
    }
  }
  for (int j = 0; j < LPL; ++j) {
    if (lam[j] > half) continue;
    const int32_t n1 = p1[j], j3 = p3[j];
    const int64_t s2 = t.pre[nbig] - t.pre[n1];
    const int64_t s3 = j3 > nbig ? t.pre[j3] - t.pre[nbig] : 0;
    t.node[lam[j]] = n1;
    t.node[half + 1 + lam[j]] = s2 + s3;
  }
}

// Largest packed key of a tile (0 if no lane holds a parameter of the range),
// valid in every lane.
template <int LPL>
__device__ __forceinline__ uint64_t tile_max(const int64_t lam[LPL], const int64_t lbp[LPL], const bool ok[LPL]) {
  uint64_t key = 0;
  for (int j = 0; j < LPL; ++j)
    if (ok[j]) key = umax64(key, pack_key(lbp[j], lam[j]));
  return wave_max_u64(key);
}

// Greatest common divisor (Euclid).
__device__ __forceinline__ uint32_t gcd_u32(uint32_t a, uint32_t b) {
  while (b) {
    const uint32_t r = a % b;
    a = b;
    b = r;
  }
  return a;
}

// Mirrored VB2.  For a >= 1, h(a, c - lambda) = a - 1 - h(a, lambda) - [c | a
// lambda], and c | a lambda iff d | a with d = c / gcd(c, lambda).  Over a
// class with n sizes summing (as a) to A, the sum at c - lambda is
// A - n - (sum at lambda) - #{d | a}; the counts per divisor of c come from
// prep (for the big class a = c - w, and d | c - w iff d | w).  Returns the
// packed maximum over the lanes' keys at lambda and at c - lambda, each kept
// when inside the bound's range [t.lo, t.hi]; lam[j] <= mm marks a lane in
// the dense half.
template <int LPL>
__device__ uint64_t vb2_mirror_key(const TileArgs &t, int64_t mm, const int64_t lam[LPL], const int64_t part[LPL]) {
  const int64_t C = t.C;
  const int64_t nsm = t.nz - t.nm, nbg = t.nb - t.nf;
  const int64_t sum_small = t.sumNZ - t.sumBig - (int64_t)(t.nm - t.nb) * (C / 2);
  const int64_t base = (sum_small - nsm) - (nbg * C - t.sumBig - nbg);  // (A - n) small minus (A - n) big
  uint64_t key = 0;  // this lane's largest key, folded as each one is made
  for (int j = 0; j < LPL; ++j) {
    const bool in = lam[j] >= 1 && lam[j] <= mm;
    const uint32_t lj = in ? (uint32_t)lam[j] : 1u;
    const uint32_t dd = (uint32_t)C / gcd_u32((uint32_t)C, lj);
    int lo = 0, hi = t.ndiv - 1;  // dd is a divisor of c: find it
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if ((uint32_t)t.divs[mid] < dd) lo = mid + 1; else hi = mid;
    }
    const int64_t dsm = t.dcnt[lo], dbg = t.dcnt[t.ndiv + lo];
    const int64_t part2 = 2 * (base - dsm + dbg) - part[j];
    const int64_t l1 = lam[j], l2 = C - lam[j];
    if (in && l1 >= t.lo && l1 <= t.hi) {
      key = umax64(key, pack_key(fin_bound(kVB2, t, l1, part[j]), l1));
      if (t.node) store_state(kVB2, t, l1, part[j]);
    }
    if (in && l2 >= t.lo && l2 <= t.hi) {
      key = umax64(key, pack_key(fin_bound(kVB2, t, l2, part2), l2));
      if (t.node) store_state(kVB2, t, l2, part2);
    }
  }
  return wave_max_u64(key);
}

// Folds a key into the instance's maximum for the bound and raises the
// early-exit flag when the bound refutes the instance.  Keys only grow: a key
// that does not beat the current one leaves it alone.
__device__ __forceinline__ void publish_key(const LaunchDesc &d, int64_t inst, int bound, const TileArgs &t,
                                            uint64_t key, bool early) {
  if (!key) return;
  unsigned long long *kp = &d.keys[inst * kNB + bound];
  if (key > __hip_atomic_load(kp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(kp, (unsigned long long)key);
  if (early) {
    const int64_t v = (int64_t)(key >> 32) + (bound == kL2 ? 0 : t.nf);
    if (v > t.k) __hip_atomic_store(&d.refuted[inst], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <int LPL>
__device__ __forceinline__ void flush_tile(const LaunchDesc &d, int64_t inst, int bound, const TileArgs &t,
                                           const int64_t lam[LPL], const int64_t lbp[LPL], const bool ok[LPL],
                                           bool early) {
  const uint64_t wmax = tile_max<LPL>(lam, lbp, ok);
  if (lane_id() == 0) publish_key(d, inst, bound, t, wmax, early);
}

__device__ __forceinline__ int64_t find_entry(const BP_CONST Entry *e, int64_t n, uint64_t task) {
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if ((uint64_t)e[mid].task_begin <= task) lo = mid; else hi = mid - 1;
  }
  return lo;
}


// The tile arguments of one (instance, bound) entry; false when the
// instance failed in prep.
__device__ __forceinline__ bool entry_args(const LaunchDesc &d, const BP_CONST Entry &e, TileArgs &t, bool &early) {
  const int64_t inst = e.inst;
  const BP_CONST InstState &st = as_const(d.state)[inst];
  if (st.status != BP_OK) return false;
  const BP_CONST InstPlan &p = as_const(d.plan)[inst];
  const int bound = e.bound;
  t.wv = as_const((const uint32_t *)d.sorted + p.ws_off);
  t.av = as_const((const uint32_t *)d.av + p.ws_off);
  t.sorted = as_global(d.sorted + p.ws_off);
  t.pre = as_global(d.pre + p.pre_off);
  t.lo = p.lo[bound];
  t.hi = st.hiEff[bound];
  t.k = p.k;
  t.C = p.C;
  t.r = st.r;
  t.nf = st.nf;
  t.nb = st.nb;
  t.nm = st.nm;
  t.nz = st.nz;
  t.sumBig = st.sumBig;
  t.sumNZ = st.sumNZ;
  t.bidx = as_const(d.bidx + p.bidx_off);
  t.prec = as_const(d.pre + p.pre_off);
  t.bsh = p.bshift;
  t.ndiv = p.ndiv;
  t.divs = as_global(d.divs + p.div_off);
  t.dcnt = as_global(d.dcnt + p.dc_off);
  t.node = p.state_off >= 0 ? d.nodes + p.state_off + node_off(p.C, bound) : nullptr;
  if (p.large == 2) {
    t.vc = as_global(d.vcnt + p.vt_off);
    t.vs = as_global(d.vsum + p.vt_off);
    t.vo = as_global(d.vtot + p.vtt_off + 2 * (((int64_t)p.C + 2 + kVtChunk - 1) / kVtChunk));
  }
  early = (p.flags & kPlanEarlyExit) != 0;
  return true;
}

__device__ __forceinline__ bool refuted_now(const LaunchDesc &d, int64_t inst) {
  return __builtin_amdgcn_readfirstlane(
             __hip_atomic_load(&d.refuted[inst], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0;
}

template <int LPL>
__device__ void run_task(const LaunchDesc &d, uint64_t task) {
  const BP_CONST Entry &e = as_const(d.entries)[find_entry(as_const(d.entries), d.nentries, task)];
  const int64_t inst = e.inst;
  const int bound = e.bound;
  TileArgs t;
  bool early;
  if (!entry_args(d, e, t, early)) return;
  const int64_t local = (int64_t)task - e.task_begin;
  const int32_t nch = e.nchunks;
  const int64_t tile0 = (local / nch) * e.tpt;
  const int32_t chunk = (int32_t)(local % nch);
  // this chunk's share of the streamed items [nf, nz)
  const int64_t span = (int64_t)t.nz - t.nf;
  t.i0 = t.nf + (int32_t)(span * chunk / nch);
  t.i1 = t.nf + (int32_t)(span * (chunk + 1) / nch);
  // a split BJ1/CCM1 segment tile divides its q range instead
  t.qc = chunk;
  t.qn = nch;
  const int64_t tile1 = min(e.ntiles, tile0 + e.tpt);
  for (int64_t tl = tile0; tl < tile1; ++tl) {
    if (early && refuted_now(d, inst)) {
      if (bound != kL2 && e.mode != kModeCand) {
        // the work left out: this chunk's share of the r items (the shares
        // of a tile's chunks add up to r) for each remaining tile's parameters
        const uint32_t r32 = (uint32_t)t.r;
        const uint64_t share = (uint64_t)(r32 * (uint32_t)(chunk + 1) / (uint32_t)nch - r32 * (uint32_t)chunk / (uint32_t)nch);
        uint64_t skipped = 0;
        for (int64_t u = tl; u < tile1; ++u)
          skipped += (uint64_t)tile_params<LPL>(e.mode, e.aux, t, e.lam0 + u * (64 * LPL)) * share;
        if (skipped && lane_id() == 0) atomicAdd(&d.state[inst].evals_skipped, (unsigned long long)skipped);
      }
      return;
    }
    t.lam0 = e.lam0 + tl * (64 * LPL);
    int64_t lam[LPL], lbp[LPL];
    bool ok[LPL];
    if (e.mode == kModeL2State) {
      tile_l2_state<LPL>(t);
      continue;
    }
    if (bound == kL2) {
      // tiles of L2 run over candidate indices, not parameters
      tile_l2<LPL>(t, lam, lbp, ok);
      flush_tile<LPL>(d, inst, kL2, t, lam, lbp, ok, early);
      continue;
    }
    if (e.mode == kModeCand) {
      // so do the candidate tiles of MT and RAD2
      if (bound == kMT) tile_mt_cand<LPL>(t, lam, lbp, ok);
      else tile_rad2_cand<LPL>(t, lam, lbp, ok);
      flush_tile<LPL>(d, inst, bound, t, lam, lbp, ok, early);
      continue;
    }
    if (t.lam0 > t.hi) return;
    // the dense half of a mirrored VB2 entry runs over [1, aux]
    TileArgs tv = t;
    if (e.mode == kModeMirror) {
      tv.lo = 1;
      tv.hi = e.aux;
    }
    uint32_t l32[LPL];
    tile_lams<LPL>(tv, lam, l32);
    int64_t part[LPL];
    if (e.mode == kModeLookup) {
      if (bound == kCCM1) part_ccm1_lut<LPL>(t, lam, part);
      else part_bj1_lut<LPL>(t, lam, part);
    } else if (e.mode == kModeSegments) {
      if (bound == kMT) part_mt_seg<LPL>(t, lam, part);
      else if (bound == kCCM1) part_ccm1_seg<LPL>(t, lam, part);
      else if (bound == kRAD2) part_rad2_seg<LPL>(t, lam, part);
      else part_bj1_seg<LPL>(t, lam, part);
    } else switch (bound) {
      case kMT: part_mt<LPL>(t, l32, part); break;
      case kRAD2: part_rad2<LPL>(t, l32, part); break;
      case kFS1: part_fs1<LPL>(t, l32, part); break;
      case kCCM1: part_ccm1<LPL>(t, l32, part); break;
      case kVB2: part_vb2<LPL>(tv, l32, part); break;
      default: part_bj1<LPL>(t, l32, part); break;
    }
    if (nch > 1) {
      // A chunk of a split tile: store its partial sums in its own slot (no
      // other wave touches it) and move on; the combine kernel adds the
      // chunks of the tile once the sweep is over.
      const int64_t at = (tl * nch + chunk) * (64 * LPL);
      if (e.slot32) {
        int32_t *slot = (int32_t *)(d.acc + e.acc_base) + at;
        for (int j = 0; j < LPL; ++j) slot[lane_id() + 64 * j] = (int32_t)part[j];
      } else {
        long long *slot = d.acc + e.acc_base + at;
        for (int j = 0; j < LPL; ++j) slot[lane_id() + 64 * j] = (long long)part[j];
      }
      continue;
    }
    if (e.mode == kModeMirror) {
      const uint64_t key = vb2_mirror_key<LPL>(t, e.aux, lam, part);
      if (lane_id() == 0) publish_key(d, inst, bound, t, key, early);
      continue;
    }
    if (t.node) store_state_lanes<LPL>(bound, t, lam, part);
    for (int j = 0; j < LPL; ++j) {
      ok[j] = lam[j] >= t.lo && lam[j] <= t.hi;
      lbp[j] = ok[j] ? fin_bound(bound, t, lam[j], part[j]) : 0;
    }
    flush_tile<LPL>(d, inst, bound, t, lam, lbp, ok, early);
  }
}

// Split tiles, in segments of kSegTiles consecutive tiles of one entry: a
// block per segment, a wave per tile.  A wave adds the chunks' partial sums
// of its tile (in chunk order; integer sums, so the order does not change
// them) and finalises the tile; the block takes the maximum of its waves and
// publishes it once, so the tiles of one bound do not queue on its key.
// Tiles whose chunks did not all run -- the instance failed in prep, was
// refuted early, or the tile lies past the effective range -- are skipped by
// the same tests the sweep applied.
template <int LPL>
__global__ __launch_bounds__(64 * kSegTiles) void k_combine(const LaunchDesc *__restrict__ dp) {
  __shared__ unsigned long long wkey[kSegTiles];
  const LaunchDesc d = *as_const(dp);
  const int wave = threadIdx.x >> 6;
  for (int64_t sg = blockIdx.x; sg < d.nsplit; sg += gridDim.x) {
    // the entry holding segment sg: the last one with split_base <= sg (an
    // entry without split tiles shares its split_base with the next entry
    // that has some, so the search always lands on a split entry)
    const BP_CONST Entry *es = as_const(d.entries);
    int64_t lo = 0, hi = d.nentries - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (es[mid].split_base <= sg) lo = mid; else hi = mid - 1;
    }
    const BP_CONST Entry &e = es[lo];
    TileArgs t;
    bool early;
    if (!entry_args(d, e, t, early)) continue;  // the same for the whole block
    const int64_t tl = (sg - e.split_base) * kSegTiles + wave;
    t.lam0 = e.lam0 + tl * (64 * LPL);
    uint64_t key = 0;
    if (tl < e.ntiles && t.lam0 <= t.hi && !(early && refuted_now(d, e.inst))) {
      const int32_t nch = e.nchunks;
      int64_t lam[LPL], lbp[LPL], part[LPL];
      bool ok[LPL];
      uint32_t l32[LPL];
      TileArgs tv = t;
      if (e.mode == kModeMirror) {
        tv.lo = 1;
        tv.hi = e.aux;
      }
      tile_lams<LPL>(tv, lam, l32);
      for (int j = 0; j < LPL; ++j) part[j] = 0;
      // four chunks' loads in flight at a time
      auto add_slots = [&](const auto *slots) {
        int32_t c = 0;
        for (; c + 4 <= nch; c += 4) {
          int64_t v[4][LPL];
#pragma unroll
          for (int u = 0; u < 4; ++u)
            for (int j = 0; j < LPL; ++j) v[u][j] = slots[(c + u) * (64 * LPL) + lane_id() + 64 * j];
#pragma unroll
          for (int u = 0; u < 4; ++u)
            for (int j = 0; j < LPL; ++j) part[j] += v[u][j];
        }
        for (; c < nch; ++c)
          for (int j = 0; j < LPL; ++j) part[j] += slots[c * (64 * LPL) + lane_id() + 64 * j];
      };
      if (e.slot32)
        add_slots((const int32_t *)(d.acc + e.acc_base) + tl * nch * (64 * LPL));
      else
        add_slots(d.acc + e.acc_base + tl * nch * (64 * LPL));
      if (e.mode == kModeMirror) {
        key = vb2_mirror_key<LPL>(t, e.aux, lam, part);
      } else {
        if (t.node) store_state_lanes<LPL>(e.bound, t, lam, part);
        for (int j = 0; j < LPL; ++j) {
          ok[j] = lam[j] >= t.lo && lam[j] <= t.hi;
          lbp[j] = ok[j] ? fin_bound(e.bound, t, lam[j], part[j]) : 0;
        }
        key = tile_max<LPL>(lam, lbp, ok);
      }
    }
    if (lane_id() == 0) wkey[wave] = key;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t m = 0;
      for (int w = 0; w < kSegTiles; ++w) m = umax64(m, wkey[w]);
      publish_key(d, e.inst, e.bound, t, m, early);
    }
    __syncthreads();
  }
}

// Persistent sweep.  Wave b runs task b first; the tasks past the grid are
// dealt round-robin to kQueues queues (task grid + q + kQueues c is claim c
// of queue q), each with its own counter.  A wave claims from the queue of
// its own XCD first (blocks are dispatched to the XCDs round-robin) and from
// the others once that one is exhausted, so no single counter serialises
// every claim of the launch.  Every wave leaves when all queues are empty.
// One and two parameters per lane fit 64 VGPRs (eight waves per SIMD); four
// hold twice the per-lane sums and constants and get four waves per SIMD
// rather than spill.
template <int LPL>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(LPL == 4 ? 4 : 8))) void k_sweep(const LaunchDesc *__restrict__ dp) {
  const LaunchDesc d = *as_const(dp);
  const uint64_t ntasks = (uint64_t)d.ntasks;
  const uint64_t grid = gridDim.x;
  const int home = (int)(blockIdx.x % kQueues);
  uint32_t empty = 0;  // queues this wave found exhausted
  uint64_t task = blockIdx.x;
  while (task < ntasks) {
    run_task<LPL>(d, task);
    task = ntasks;
    for (int k = 0; k < kQueues; ++k) {
      const int q = (home + k) % kQueues;
      if ((empty >> q) & 1u) continue;
      unsigned long long c = 0;
      if (lane_id() == 0) c = atomicAdd(&d.counter[q * kQueueStride], 1ull);
      c = (unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)c) |
          ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(c >> 32)) << 32);
      const uint64_t t = grid + (uint64_t)q + (uint64_t)kQueues * c;
      if (t < ntasks) {
        task = t;
        break;
      }
      empty |= 1u << q;
    }
  }
}

// ---------------------------------------------------------------------------
// Finalize: one thread per instance.

__global__ __launch_bounds__(256) void k_finalize(const LaunchDesc *__restrict__ dp) {
  const LaunchDesc d = *as_const(dp);
  for (int64_t inst = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; inst < d.count;
       inst += (int64_t)gridDim.x * blockDim.x) {
    const BP_CONST InstPlan &p = as_const(d.plan)[inst];
    const InstState &st = d.state[inst];
    bp_bounds o;
    o.k = p.k;
    o.r = st.r;
    o.status = st.status;
    o.early_exit = 0;
    int64_t P = 0;
    for (int b = 0; b < kNB; ++b) {
      o.value[b] = 0;
      o.argmax_lambda[b] = -1;
      if (b >= kMT && st.hiEff[b] >= p.lo[b]) P += st.hiEff[b] - p.lo[b] + 1;
    }
    o.evals = (int64_t)st.r * P;
    o.evals_done = o.evals - (int64_t)st.evals_skipped;
    if (st.status == BP_OK) {
      o.value[kL1] = (st.sumW + p.C - 1) / p.C;
      for (int b = kL2; b < kNB; ++b) {
        const uint64_t key = d.keys[inst * kNB + b];
        if (key) {
          o.value[b] = (int64_t)(key >> 32) + (b == kL2 ? 0 : st.nf);
          o.argmax_lambda[b] = (int64_t)(0xffffffffu - (uint32_t)key);
        }
      }
      if (p.flags & kPlanEarlyExit) o.early_exit = d.refuted[inst];
    }
    int64_t lb = -1;
    int32_t arg = 0;
    for (int b = 0; b < kNB; ++b)
      if (o.value[b] > lb) { lb = o.value[b]; arg = b; }
    o.lb = lb;
    o.lb_arg = arg;
    o.verdict = lb <= p.k ? 1 : 0;
    d.out[inst] = o;
  }
  // the value tables' raw counts, chunk totals and offsets, lattice bins,
  // flag and maximum back to zero for the next launch
  const int64_t gsz = (int64_t)gridDim.x * blockDim.x, gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int64_t jj = 0; jj < d.nvt; ++jj) {
    const BP_CONST InstPlan &p = as_const(d.plan)[d.vlist[jj]];
    const int64_t nv = (int64_t)p.C + 2, nch = (nv + kVtChunk - 1) / kVtChunk;
    for (int64_t v = gt; v < nv; v += gsz) d.vraw[p.vt_off + v] = 0;
    // (the chunk offsets too: another launch may place its totals there)
    for (int64_t k = gt; k < 4 * nch; k += gsz) d.vtot[p.vtt_off + k] = 0;
    for (int64_t k = gt; k < 2 * (int64_t)p.ndiv; k += gsz) d.vlat[p.vl_off + k] = 0;
    if (gt < 2) d.vflag[2 * jj + gt] = 0;
  }
}

// ---------------------------------------------------------------------------
// Served requests from another node's state (incremental serving).  Every
// quantity of the node state is a sum over the reduced items, so a request
// whose reduced instance differs from its base's by a few items has
//   S_f(lambda) = S_f,base(lambda) + sum_added f(w, lambda) - sum_removed f(w, lambda)
// and likewise n1 and T of L2: O(P) work per changed item instead of O(P r).
// The per-item terms are the functions of Sec. 3.1 evaluated exactly for one
// size and the lane's parameter.

// Per-lane constants of one parameter lambda.
struct LamConst {
  uint32_t lam, K, p;   // lambda, floor(c / lambda), c mod lambda
  double rl;            // 1 / lambda
};

__device__ __forceinline__ LamConst lam_const(uint32_t C, uint32_t lam) {
  LamConst k;
  k.lam = lam;
  k.rl = 1.0 / (double)(lam ? lam : 1u);
  k.K = lam ? fdiv_u31(C, lam, k.rl) : 0;
  k.p = lam ? C - k.K * lam : 0;
  return k;
}

// f(w, lambda) for 0 <= w <= c, lambda in the function's range (Sec. 3.1);
// rc = 1 / c.
template <int BOUND>
__device__ __forceinline__ int64_t dff_term_b(uint32_t C, uint32_t w, const LamConst &k, double rc) {
  const uint32_t lam = k.lam;
  switch (BOUND) {
    case kMT:  // c if w > c - lambda; w if lambda <= w <= c - lambda; 0 if w < lambda
      if (w > C - lam) return C;
      return w >= lam ? (int64_t)w : 0;
    case kRAD2:  // 0 | c/3 | c/2 | c - f(c - w), the last one level deep
      if (w < lam) return 0;
      if (w <= C - 2 * lam) return C / 3;
      if (w < 2 * lam) return C / 2;
      return (int64_t)C - (C - w >= lam ? (int64_t)(C / 3) : 0);
    case kFS1: {  // w lambda if c divides n = w (lambda + 1), else floor(n / c) c
      // n < 2^38: q = floor((n + 0.5) / c) from the fp64 product is exact (the
      // relative error 2^-52 stays below the distance 0.5 / c to an integer),
      // and fma(-q, c, n) is the exact remainder
      const double n = (double)w * (double)(lam + 1u);
      const double q = floor((n + 0.5) * rc);
      const double rem = fma(-q, (double)C, n);
      return rem == 0.0 ? (int64_t)w * lam : (int64_t)q * C;
    }
    case kCCM1:  // 2 K - 2 floor((c - w) / lambda) | K | 2 floor(w / lambda)
      if (2ull * w > C) return 2 * ((int64_t)k.K - (int64_t)fdiv_u31(C - w, lam, k.rl));
      if (2ull * w == C) return k.K;
      return 2 * (int64_t)fdiv_u31(w, lam, k.rl);
    case kVB2: {  // with h(a) = max(0, ceil(a lambda / c) - 1) = floor((a lambda - 1) / c) for a >= 1:
                  // 2 (lambda - 1) - 2 h(c - w) | lambda - 1 | 2 h(w)
      if (2ull * w > C) {
        const int64_t a = C - w;
        return 2 * ((int64_t)lam - 1) - 2 * (a ? fdiv_u62(a * lam - 1, C, rc) : 0);
      }
      if (2ull * w == C) return (int64_t)lam - 1;
      return 2 * (w ? fdiv_u62((int64_t)w * lam - 1, C, rc) : 0);
    }
    default: {  // BJ1: floor(w / lambda) (lambda - p) + max(0, (w mod lambda) - p)
      const uint32_t q = fdiv_u31(w, lam, k.rl);
      const uint32_t rem = w - q * lam;
      return (int64_t)q * (lam - k.p) + (rem > k.p ? (int64_t)(rem - k.p) : 0);
    }
  }
}

__device__ __forceinline__ int64_t dff_term(int bound, uint32_t C, uint32_t w, const LamConst &k, double rc) {
  switch (bound) {
    case kMT: return dff_term_b<kMT>(C, w, k, rc);
    case kRAD2: return dff_term_b<kRAD2>(C, w, k, rc);
    case kFS1: return dff_term_b<kFS1>(C, w, k, rc);
    case kCCM1: return dff_term_b<kCCM1>(C, w, k, rc);
    case kVB2: return dff_term_b<kVB2>(C, w, k, rc);
    default: return dff_term_b<kBJ1>(C, w, k, rc);
  }
}

__device__ __forceinline__ int64_t default_lo(int bound, int32_t C) {
  switch (bound) {
    case kL2: case kMT: return 0;
    case kRAD2: return C / 4 + 1;
    case kVB2: return 2;
    default: return 1;
  }
}

__device__ __forceinline__ int64_t find_node_task(const BP_CONST NodeTask *t, int64_t n, int64_t tile) {
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (t[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Clears the packed maxima of the launch's child requests.
__global__ __launch_bounds__(256) void k_node_begin(unsigned long long *keys, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * kNB; i += (int64_t)gridDim.x * blockDim.x)
    keys[i] = 0ull;
}

// One block of kNodeTile threads per (child, bound, run of kNodeTile
// parameters): each thread updates its parameter's state from the base,
// stores it (when kept) and takes its bound value; one packed-key maximum
// per block.
__global__ __launch_bounds__(kNodeTile) void k_node_delta(const NodeTask *__restrict__ tasks, int64_t ntasks,
                                                       int64_t ntiles, const int32_t *__restrict__ delta,
                                                       long long *__restrict__ nodes, unsigned long long *keys) {
  __shared__ unsigned long long wkey[kNodeTile / 64];
  const BP_CONST NodeTask *tk = as_const(tasks);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t ti = find_node_task(tk, ntasks, tile);
    const BP_CONST NodeTask &t = tk[ti];
    const int32_t C = t.C;
    // the bound and first parameter of this tile
    int64_t local = tile - t.tile_begin;
    int bound = kL2;
    while (bound + 1 < kNB && local >= node_tile_count(C, bound)) {
      local -= node_tile_count(C, bound);
      ++bound;
    }
    const int64_t len = node_params(C, bound);
    const int64_t boff = node_off(C, bound);
    const int64_t idx = local * kNodeTile + threadIdx.x;
    const bool valid = idx < len;
    const int64_t lam = default_lo(bound, C) + idx;
    uint64_t key = 0;
    if (valid) {
      const long long *base = nodes + t.base_off + boff;
      long long *dst = t.dst_off >= 0 ? nodes + t.dst_off + boff : nullptr;
      const BP_CONST int32_t *dl = as_const(delta + t.d_off);
      const uint32_t uC = (uint32_t)C;
      if (bound == kL2) {
        const int64_t half = C / 2;
        int64_t n1 = base[idx], T = base[half + 1 + idx];
        for (int32_t j = 0; j < t.nd; ++j) {
          const int32_t v = dl[j];
          const int64_t sg = v > 0 ? 1 : -1;
          const int64_t w = v > 0 ? v - 1 : -(int64_t)v - 1;
          if (w > C - lam) n1 += sg;
          const bool w2 = 2 * w > C && w <= C - lam;   // c/2 < w <= c - lambda
          const bool w3 = w >= lam && 2 * w <= C;      // lambda <= w <= c/2
          if (w2 || w3) T += sg * w;
        }
        if (dst) {
          dst[idx] = n1;
          dst[half + 1 + idx] = T;
        }
        const int64_t x = T - (int64_t)C * ((int64_t)t.nbig - n1);
        key = pack_key(t.nbig + (x > 0 ? ceil_div_small(x, C) : 0), lam);
      } else {
        const LamConst kc = lam_const(uC, (uint32_t)lam);
        const double rc = 1.0 / (double)C;
        int64_t S = base[idx];
        for (int32_t j = 0; j < t.nd; ++j) {
          const int32_t v = dl[j];
          const uint32_t w = v > 0 ? (uint32_t)(v - 1) : (uint32_t)(-(int64_t)v - 1);
          const int64_t f = dff_term(bound, uC, w, kc, rc);
          S += v > 0 ? f : -f;
        }
        if (dst) dst[idx] = S;
        key = pack_key(ceil_div_small(S, fc_bound(bound, C, lam)), lam);
      }
    }
    const uint64_t wm = wave_max_u64(key);
    if (lane_id() == 0) wkey[threadIdx.x >> 6] = wm;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t m = 0;
      for (int w = 0; w < kNodeTile / 64; ++w) m = umax64(m, wkey[w]);
      if (m) atomicMax(&keys[ti * kNB + bound], (unsigned long long)m);
    }
    __syncthreads();
  }
}

// The records of the launch's child requests: L1 from the total size, the
// other bounds from the packed maxima, lb, verdict (Alg. 1).
__global__ __launch_bounds__(256) void k_node_finalize(const NodeTask *__restrict__ tasks, int64_t ntasks,
                                                    const unsigned long long *__restrict__ keys, bp_bounds *out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ntasks; i += (int64_t)gridDim.x * blockDim.x) {
    const NodeTask &t = tasks[i];
    const int64_t P = node_off(t.C, kNB) - node_off(t.C, kMT);
    bp_bounds o;
    o.k = t.k;
    o.r = t.r;
    o.status = BP_OK;
    o.early_exit = 0;
    o.evals = t.r * P;
    o.evals_done = (int64_t)t.nd * P;
    o.value[kL1] = (t.sumW + t.C - 1) / t.C;
    o.argmax_lambda[kL1] = -1;
    for (int b = kL2; b < kNB; ++b) {
      const uint64_t key = keys[i * kNB + b];
      o.value[b] = key ? (int64_t)(key >> 32) : 0;
      o.argmax_lambda[b] = key ? (int64_t)(0xffffffffu - (uint32_t)key) : -1;
    }
    int64_t lb = -1;
    int32_t arg = 0;
    for (int b = 0; b < kNB; ++b)
      if (o.value[b] > lb) { lb = o.value[b]; arg = b; }
    o.lb = lb;
    o.lb_arg = arg;
    o.verdict = lb <= t.k ? 1 : 0;
    out[t.out_idx] = o;
  }
}

// ---------------------------------------------------------------------------
// Small checks in one launch.  Every workgroup rebuilds the reduced instance
// of Fig. 3 in its LDS (sizes, then one virtual item per loaded bin) from the
// kernel arguments, with its totals, then takes its share of the (bound,
// parameter) pairs, S lanes per pair: the exact f of Sec. 3.1 summed over
// the items, or L2(I, lambda) from its three classes.  Each workgroup writes
// its packed maxima to its own slots with plain stores (no atomics, no
// fences: a device-scope fence or atomic per workgroup costs more than the
// sums at these sizes); k_small_final, next on the stream, takes the maxima
// over the workgroups, writes the record to `out` (host memory) and then
// publishes `seq`.

// The record of a small check from the packed maxima of L2 .. BJ1 and the
// instance totals, written to host memory, then its sequence number.
__device__ void small_record(const unsigned long long *keys, uint64_t tot_w, int64_t evals, int32_t r, int32_t bad,
                             uint32_t C, int64_t k, bp_bounds *out, uint32_t *seq_out, uint32_t seq) {
  bp_bounds o;
  o.k = k;
  o.r = r;
  o.status = bad ? BP_ERR_RANGE : BP_OK;
  o.early_exit = 0;
  o.evals = evals;
  o.evals_done = evals;
  o.value[kL1] = r > 0 ? (int64_t)((tot_w + C - 1) / C) : 0;
  o.argmax_lambda[kL1] = -1;
  for (int q = kL2; q < kNB; ++q) {
    const unsigned long long gk = keys[q];
    o.value[q] = gk ? (int64_t)(gk >> 32) : 0;
    o.argmax_lambda[q] = gk ? (int64_t)(0xffffffffu - (uint32_t)gk) : -1;
  }
  int64_t lb = -1;
  int32_t arg = 0;
  for (int q = 0; q < kNB; ++q)
    if (o.value[q] > lb) { lb = o.value[q]; arg = q; }
  o.lb = lb;
  o.lb_arg = arg;
  o.verdict = lb <= k ? 1 : 0;
  *out = o;
  // the record is visible to the host before the sequence number that announces it
  __threadfence_system();
  __hip_atomic_store(seq_out, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ONE (at most kSmallOneMaxGrid workgroups of kSmallOneThreads): the
// workgroups fold their maxima into one set of keys by atomics and the last
// one to finish writes the record (a few dozen device-scope atomics and
// fences cost less than a second launch); otherwise (workgroups of
// kSmallFusedThreads) each writes its own slots for k_small_final.
template <bool ONE, int NT>
__global__ __launch_bounds__(NT) void k_small_check(SmallArgs a, unsigned long long *part,
                                                                   SmallHead *head, unsigned long long *onek,
                                                                   bp_bounds *out, uint32_t *seq_out, uint32_t seq) {
  __shared__ uint32_t w[kSmallFusedMax];
  __shared__ uint32_t wsum[NT / 64];
  __shared__ unsigned long long key[kNB];
  __shared__ unsigned long long tot_w;
  __shared__ int32_t nbig_s, maxw_s, bad_s, last_s;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const uint32_t C = (uint32_t)a.C;
  if (tid < kNB) key[tid] = 0ull;
  if (tid == 0) {
    tot_w = 0ull;
    nbig_s = 0;
    maxw_s = 0;
    bad_s = 0;
  }
  // the sizes, validated
  for (int i = tid; i < a.n; i += NT) {
    int32_t x = a.v[i];
    if (x < 0 || x > a.C) { bad_s = 1; x = 0; }
    w[i] = (uint32_t)x;
  }
  int32_t r = a.n;
  if (a.form == kFormResidual) {
    // one virtual item of size c - residual per bin with residual < c, in bin order
    uint32_t base = 0;
    for (int j0 = 0; j0 < a.m; j0 += NT) {
      const int j = j0 + tid;
      const bool in = j < a.m;
      int32_t res = in ? a.v[a.n + j] : a.C;
      if (in && (res < 0 || res > a.C)) { bad_s = 1; res = a.C; }
      const bool take = in && res < a.C;
      const uint64_t bal = ballot64(take);
      __syncthreads();
      if ((tid & 63) == 0) wsum[wave] = (uint32_t)__popcll(bal);
      __syncthreads();
      uint32_t off = 0, tot = 0;
      for (int v = 0; v < NT / 64; ++v) {
        off += v < wave ? wsum[v] : 0u;
        tot += wsum[v];
      }
      if (take) w[a.n + base + off + (uint32_t)__popcll(bal & lanemask_lt())] = C - (uint32_t)res;
      base += tot;
    }
    r = a.n + (int32_t)base;
  }
  __syncthreads();
  if (bad_s) r = 0;
  // totals: sum, count of big sizes, largest size
  for (int i = tid; i < r; i += NT) {
    const uint32_t x = w[i];
    atomicAdd(&tot_w, (unsigned long long)x);
    if (2ull * x > C) atomicAdd(&nbig_s, 1);
    atomicMax(&maxw_s, (int32_t)x);
  }
  __syncthreads();
  const int64_t nbig = nbig_s;
  int64_t hi[kNB];
  for (int b = 0; b < kNB; ++b) hi[b] = a.hi[b];
  if (a.clamp) {
    const int64_t denom = (int64_t)r * maxw_s;
    const int64_t cap = denom > 0 ? vb2_cut_cap(denom) : (int64_t)a.C;
    if (cap < hi[kVB2]) hi[kVB2] = cap;
  }
  // this workgroup's (bound, parameter) pairs: a group of S consecutive
  // lanes per pair, each lane summing every S-th item, the group's partial
  // sums added by shuffles
  int64_t total = 0;
  for (int b = kL2; b < kNB; ++b) total += a.lo[b] <= hi[b] ? hi[b] - a.lo[b] + 1 : 0;
  const double rc = 1.0 / (double)C;
  const int S = a.slices;
  const int sh = __builtin_ctz((unsigned)S);
  const int sl = tid & (S - 1);
  unsigned long long best[kNB] = {};
  for (int64_t gt = (int64_t)blockIdx.x * NT + tid; gt < total * S;
       gt += (int64_t)gridDim.x * NT) {
    int b = kL2;
    int64_t idx = gt >> sh;
    for (; b < kNB; ++b) {
      const int64_t len = a.lo[b] <= hi[b] ? hi[b] - a.lo[b] + 1 : 0;
      if (idx < len) break;
      idx -= len;
    }
    const int64_t lam = a.lo[b] + idx;
    int64_t p0 = 0, p1 = 0;  // L2: n1 and T; a function: its partial sum
    if (b == kL2) {
      for (int32_t i = sl; i < r; i += S) {
        const int64_t x = w[i];
        p0 += x > (int64_t)C - lam;
        const bool in2 = 2 * x > (int64_t)C && x <= (int64_t)C - lam;
        const bool in3 = x >= lam && 2 * x <= (int64_t)C;
        p1 += (in2 || in3) ? x : 0;
      }
    } else {
      const LamConst kc = lam_const(C, (uint32_t)lam);
      auto sum = [&](auto term) {
        for (int32_t i = sl; i < r; i += S) p0 += term(w[i]);
      };
      switch (b) {
        case kMT: sum([&](uint32_t x) { return dff_term_b<kMT>(C, x, kc, rc); }); break;
        case kRAD2: sum([&](uint32_t x) { return dff_term_b<kRAD2>(C, x, kc, rc); }); break;
        case kFS1: sum([&](uint32_t x) { return dff_term_b<kFS1>(C, x, kc, rc); }); break;
        case kCCM1: sum([&](uint32_t x) { return dff_term_b<kCCM1>(C, x, kc, rc); }); break;
        case kVB2: sum([&](uint32_t x) { return dff_term_b<kVB2>(C, x, kc, rc); }); break;
        default: sum([&](uint32_t x) { return dff_term_b<kBJ1>(C, x, kc, rc); }); break;
      }
    }
    for (int o = 1; o < S; o <<= 1) {
      p0 += __shfl_xor(p0, o, 64);
      p1 += __shfl_xor(p1, o, 64);
    }
    if (sl == 0) {
      int64_t v;
      if (b == kL2) {
        const int64_t y = p1 - (int64_t)C * (nbig - p0);
        v = nbig + (y > 0 ? ceil_div_small(y, (int64_t)C) : 0);
      } else {
        v = ceil_div_small(p0, fc_bound(b, a.C, lam));
      }
      for (int q = kL2; q < kNB; ++q)
        if (q == b) best[q] = umax64(best[q], pack_key(v, lam));
    }
  }
  for (int q = kL2; q < kNB; ++q) {
    const uint64_t m = wave_max_u64(best[q]);
    if (lane_id() == 0 && m) atomicMax(&key[q], (unsigned long long)m);
  }
  __syncthreads();
  int64_t P = 0;
  for (int b = kMT; b < kNB; ++b) P += a.lo[b] <= hi[b] ? hi[b] - a.lo[b] + 1 : 0;
  if (ONE) {
    if (tid < kNB && key[tid]) atomicMax(&onek[tid], key[tid]);
    __threadfence();
    __syncthreads();
    if (tid == 0) last_s = atomicAdd(&onek[kNB], 1ull) == (unsigned long long)(gridDim.x - 1) ? 1 : 0;
    __syncthreads();
    if (!last_s) return;
    __threadfence();
    if (tid < kNB) key[tid] = __hip_atomic_load(&onek[tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    // clean for the next call (every other workgroup is done with the keys)
    if (tid <= kNB) __hip_atomic_store(&onek[tid], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tid == 0) small_record(key, tot_w, (int64_t)r * P, r, bad_s, C, a.k, out, seq_out, seq);
    return;
  }
  if (tid < kNB) part[(size_t)blockIdx.x * kNB + tid] = key[tid];
  if (blockIdx.x == 0 && tid == 0) {
    SmallHead h;
    h.tot_w = tot_w;
    h.evals = (int64_t)r * P;
    h.r = r;
    h.bad = bad_s;
    *head = h;
  }
}

__global__ __launch_bounds__(256) void k_small_final(const unsigned long long *part, int grid,
                                                      const SmallHead *head, uint32_t C, int64_t k, bp_bounds *out,
                                                      uint32_t *seq_out, uint32_t seq) {
  __shared__ unsigned long long red[256];
  const int tid = threadIdx.x;
  const int b = tid & (kNB - 1);
  unsigned long long mx = 0ull;
  for (int g = tid / kNB; g < grid; g += 256 / kNB) mx = umax64(mx, part[(size_t)g * kNB + b]);
  red[tid] = mx;
  __syncthreads();
  for (int st = 128; st >= kNB; st >>= 1) {
    if (tid < st) red[tid] = umax64(red[tid], red[tid + st]);
    __syncthreads();
  }
  if (tid == 0) {
    const SmallHead h = *head;
    small_record(red, h.tot_w, h.evals, h.r, h.bad, C, k, out, seq_out, seq);
  }
}

hipError_t launch_small_check(const SmallArgs &a, bool one, int grid, void *buf, bp_bounds *out, uint32_t *seq_out,
                              uint32_t seq, hipStream_t s) {
  if (grid < 1 || grid > kSmallFusedMaxGrid) return hipErrorInvalidValue;
  unsigned long long *part = (unsigned long long *)buf;
  SmallHead *head = (SmallHead *)(part + (size_t)kNB * kSmallFusedMaxGrid);
  unsigned long long *onek = (unsigned long long *)(head + 1);
  if (one) {
    if (grid > kSmallOneMaxGrid) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_small_check<true, kSmallOneThreads>), dim3(grid), dim3(kSmallOneThreads), 0, s, a, part,
                       head, onek, out, seq_out, seq);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_small_check<false, kSmallFusedThreads>), dim3(grid), dim3(kSmallFusedThreads), 0, s, a, part,
                     head, onek, out, seq_out, seq);
  hipLaunchKernelGGL(k_small_final, dim3(1), dim3(256), 0, s, (const unsigned long long *)part, grid,
                     (const SmallHead *)head, (uint32_t)a.C, a.k, out, seq_out, seq);
  return hipGetLastError();
}

hipError_t launch_node_delta(const NodeTask *tasks, int64_t ntasks, int64_t ntiles, const int32_t *delta,
                             long long *nodes, unsigned long long *keys, bp_bounds *out, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_node_begin, dim3(std::max<int64_t>(1, std::min<int64_t>(64, (ntasks * kNB + 255) / 256))),
                     dim3(256), 0, s, keys, ntasks);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ntiles > 0) {
    hipLaunchKernelGGL(k_node_delta, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(grid, ntiles))),
                       dim3(kNodeTile), 0, s, tasks, ntasks, ntiles, delta, nodes, keys);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_node_finalize, dim3(std::max<int64_t>(1, std::min<int64_t>(64, (ntasks + 255) / 256))),
                     dim3(256), 0, s, tasks, ntasks, keys, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Standalone reduction (bp_residual_reduce / bp_assignment_reduce).

// loads[j] += size of every item assigned to bin j (int64 atomics).
__global__ __launch_bounds__(256) void k_bin_loads(const int32_t *size, const int32_t *bin_of, int64_t n,
                                                   int32_t m, int32_t C, unsigned long long *loads,
                                                   int32_t *bad) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t w = size[i], b = bin_of[i];
    if (w < 0 || w > C || b < -1 || b >= m) { *bad = 1; continue; }
    if (b >= 0) atomicAdd(&loads[b], (unsigned long long)w);
  }
}

// One block: out = unpacked items (those with bin_of < 0 when bin_of != NULL),
// then one item C - residual per bin with residual < C, in bin order.  With
// loads != NULL the residuals are C - loads.
__global__ __launch_bounds__(1024) void k_reduce_one(int32_t C, int32_t m, const int32_t *residual,
                                                     const unsigned long long *loads, const int32_t *items,
                                                     const int32_t *bin_of, int64_t n, int32_t *out,
                                                     int64_t *out_r, int32_t *out_residual, int32_t *bad) {
  __shared__ uint32_t wsum[16];
  const int tid = threadIdx.x, wave = tid >> 6;
  int64_t pos = 0;
  for (int pass = 0; pass < 2; ++pass) {
    const int64_t cnt = pass == 0 ? n : m;
    for (int64_t base = 0; base < cnt; base += 1024) {
      const int64_t i = base + tid;
      bool take = false;
      int32_t v = 0;
      if (i < cnt) {
        if (pass == 0) {
          v = items[i];
          if (v < 0 || v > C) { *bad = 1; v = 0; }
          take = bin_of ? bin_of[i] < 0 : true;
        } else {
          int64_t res;
          if (loads) {
            const unsigned long long ld = loads[i];
            if (ld > (unsigned long long)C) { *bad = 1; res = C; } else res = C - (int64_t)ld;
          } else {
            res = residual[i];
            if (res < 0 || res > C) { *bad = 1; res = C; }
          }
          if (out_residual) out_residual[i] = (int32_t)res;
          take = res < C;
          v = (int32_t)(C - res);
        }
      }
      const uint64_t bal = ballot64(take);
      const uint32_t below = (uint32_t)__popcll(bal & lanemask_lt());
      if ((tid & 63) == 0) wsum[wave] = (uint32_t)__popcll(bal);
      __syncthreads();
      uint32_t off = 0, tot = 0;
      for (int w = 0; w < 16; ++w) {
        if (w < wave) off += wsum[w];
        tot += wsum[w];
      }
      if (take) out[pos + off + below] = v;
      pos += tot;
      __syncthreads();
    }
  }
  if (tid == 0) *out_r = pos;
}

// ---------------------------------------------------------------------------
// Host-side launch helpers (C++ linkage inside the library).

size_t prep_smem_small() { return sizeof(PrepSmem<kSmallThreads, kSmallCap>); }
size_t prep_smem_tiny() { return sizeof(PrepSmem<kSmallThreads, kTinyCap>); }
size_t prep_smem_large() { return sizeof(PrepSmem<kLargeThreads, kLargeCap>); }

hipError_t set_kernel_attrs() {
  hipError_t e = hipFuncSetAttribute((const void *)k_prep<kSmallThreads, kSmallCap, 0>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)prep_smem_small());
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)k_prep<kSmallThreads, kTinyCap, 0>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)prep_smem_tiny());
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void *)k_prep<kLargeThreads, kLargeCap, 1>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)prep_smem_large());
}

static hipError_t launch_sweep(const LaunchDesc *d_desc, int lpl, int grid_sweep, hipStream_t s) {
  switch (lpl) {
    case 1: hipLaunchKernelGGL(k_sweep<1>, dim3(grid_sweep), dim3(64), 0, s, d_desc); break;
    case 4: hipLaunchKernelGGL(k_sweep<4>, dim3(grid_sweep), dim3(64), 0, s, d_desc); break;
    default: hipLaunchKernelGGL(k_sweep<2>, dim3(grid_sweep), dim3(64), 0, s, d_desc); break;
  }
  return hipGetLastError();
}

static hipError_t launch_combine(const LaunchDesc *d_desc, int lpl, int grid_comb, hipStream_t s) {
  switch (lpl) {
    case 1: hipLaunchKernelGGL(k_combine<1>, dim3(grid_comb), dim3(64 * kSegTiles), 0, s, d_desc); break;
    case 4: hipLaunchKernelGGL(k_combine<4>, dim3(grid_comb), dim3(64 * kSegTiles), 0, s, d_desc); break;
    default: hipLaunchKernelGGL(k_combine<2>, dim3(grid_comb), dim3(64 * kSegTiles), 0, s, d_desc); break;
  }
  return hipGetLastError();
}

// The small-instance prep in its short form (kTinyCap items per block: a
// quarter of the unrolled code) when every block-prepared instance is that
// small (variant bit 4).
static hipError_t launch_prep(const LaunchDesc *d_desc, int grid_prep_small, int grid_prep_large, int grid_vt,
                              int v, hipStream_t s) {
  if (v & 4)
    hipLaunchKernelGGL((k_prep<kSmallThreads, kTinyCap, 0>), dim3(grid_prep_small), dim3(kSmallThreads),
                       prep_smem_tiny(), s, d_desc);
  else
    hipLaunchKernelGGL((k_prep<kSmallThreads, kSmallCap, 0>), dim3(grid_prep_small), dim3(kSmallThreads),
                       prep_smem_small(), s, d_desc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (v & 1) {
    hipLaunchKernelGGL((k_prep<kLargeThreads, kLargeCap, 1>), dim3(grid_prep_large), dim3(kLargeThreads),
                       prep_smem_large(), s, d_desc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (grid_vt > 0) {
    hipLaunchKernelGGL(k_vt_emit, dim3(grid_vt), dim3(kVtThreads), 0, s, d_desc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Variant bits v: 1 = the launch holds a large instance prepared by one
// block, 2 = it has split tiles, 4 = its small instances fit the short prep.
// The large-instance prep runs only with bit 1 (the block form) or grid_vt >
// 0 (the value-table kernels), the combine only with bit 2 (either would find
// no work); the small-instance prep always runs, as it clears the sweep's
// task counters.
hipError_t launch_pipeline(const LaunchDesc *d_desc, int lpl, int grid_prep_small, int grid_prep_large, int grid_vt,
                           int grid_sweep, int grid_comb, int grid_fin, int v, hipStream_t s) {
  hipError_t e = launch_prep(d_desc, grid_prep_small, grid_prep_large, grid_vt, v, s);
  if (e != hipSuccess) return e;
  if ((e = launch_sweep(d_desc, lpl, grid_sweep, s)) != hipSuccess) return e;
  if ((v & 2) && (e = launch_combine(d_desc, lpl, grid_comb, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_finalize, dim3(grid_fin), dim3(256), 0, s, d_desc);
  return hipGetLastError();
}

// The same launches with events around the stages (diagnostic timing).
hipError_t launch_pipeline_timed(const LaunchDesc *d_desc, int lpl, int grid_prep_small, int grid_prep_large,
                                 int grid_vt, int grid_sweep, int grid_comb, int grid_fin, int v, hipStream_t s,
                                 hipEvent_t ev[4]) {
  hipError_t e = hipEventRecord(ev[0], s);
  if (e != hipSuccess) return e;
  if ((e = launch_prep(d_desc, grid_prep_small, grid_prep_large, grid_vt, v, s)) != hipSuccess) return e;
  if ((e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
  if ((e = launch_sweep(d_desc, lpl, grid_sweep, s)) != hipSuccess) return e;
  if ((e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
  if ((v & 2) && (e = launch_combine(d_desc, lpl, grid_comb, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_finalize, dim3(grid_fin), dim3(256), 0, s, d_desc);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return hipEventRecord(ev[3], s);
}

// ---------------------------------------------------------------------------
// The allocation-free check.  Its tables and workspaces are this file-scope
// array; each GPU holds its own copy, whose address hipGetSymbolAddress
// gives with that GPU current.  Host code uses that address, never the
// array's name (a host-side stand-in).

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static unsigned char *g_scratch_ptr[kNoAllocMaxDevices] = {};

// Set-up, once per device: the address of that device's array (the caller
// has made `device` current).
hipError_t noalloc_scratch(int device, unsigned char **out) {
  if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = (unsigned char *)p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

// Writes the launch tables (passed by value, so no copy from host memory is
// needed) to the start of the array.
__global__ __launch_bounds__(64) void k_noalloc_tables(NoAllocTables t, NoAllocTables *dst) {
  if (threadIdx.x == 0) *dst = t;
}

// The tables' kernel, then the pipeline reading its descriptor from `base`
// (the array's device address).
hipError_t launch_noalloc(const NoAllocTables &t, unsigned char *base, int lpl, int grid_prep_small,
                          int grid_prep_large, int grid_sweep, int grid_comb, int grid_fin, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_noalloc_tables, dim3(1), dim3(64), 0, s, t, (NoAllocTables *)base);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_pipeline((const LaunchDesc *)base, lpl, grid_prep_small, grid_prep_large, 0, grid_sweep, grid_comb,
                         grid_fin, v, s);
}

hipError_t launch_reduce(int32_t C, int32_t m, const int32_t *residual, const int32_t *size, const int32_t *bin_of,
                         int64_t n, unsigned long long *loads, int32_t *out, int64_t *out_r, int32_t *out_residual,
                         int32_t *bad, hipStream_t s) {
  if (bin_of) {
    hipLaunchKernelGGL(k_bin_loads, dim3(256), dim3(256), 0, s, size, bin_of, n, m, C, loads, bad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_reduce_one, dim3(1), dim3(1024), 0, s, C, m, residual,
                     (const unsigned long long *)(bin_of ? loads : nullptr), size, bin_of, n, out, out_r,
                     out_residual, bad);
  return hipGetLastError();
}

}  // namespace bpi
