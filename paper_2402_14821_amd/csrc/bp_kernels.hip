// bp_kernels.hip -- gfx950 kernels of the bin_packing feasibility check.
//
// Pipeline of one launch (a batch; a single check is a batch of one):
//   k_prep_small / k_prep_large  one block per instance (persistent over the
//       batch): reduce the partial packing to one capacity (Sec. 3, Fig. 3),
//       validate, LSD radix sort by decreasing size in LDS, int64 prefix sums
//       (DPP wave scans), class boundaries and the class-sorted item stream.
//   k_sweep  persistent: waves pull tasks (instance, bound, run of parameter
//       tiles) from one atomic counter, in longest-first order.  A tile gives
//       each lane kLPL parameters; the wave reads the item stream with scalar
//       loads (every lane uses the same item) and accumulates
//       sum_w f(w, lambda) per lane (Alg. 2's inner loop, Alg. 4's per-thread
//       loop), then ceil(sum / f(c, lambda)) and a DPP wave max of packed
//       (bound, parameter) keys, one 64-bit atomic max per tile.  L2 tiles
//       evaluate L2(I, lambda) at the parameters where it can change, from
//       the sorted sizes and prefix sums by binary search (Sec. 3.1).
//   k_finalize  per instance: L1, the maximum over the collection, verdict.
//
// Class split used by the sweeps (sizes sorted decreasing):
//   [0, nf) w = c ; [nf, nb) c/2 < w < c ; [nb, nm) 2w = c ;
//   [nm, nz) 0 < 2w < c ; [nz, r) w = 0.
// Items of size c add exactly f(c, lambda) to every sum, so they add exactly 1
// to every bound and are counted, not streamed.  Zero sizes add 0 to every
// function.  Mid items (2w = c) take one fixed value per parameter.  For the
// big and small classes each function reduces to per-lane arithmetic on a
// scalar operand, written out per function below.
#include <hip/hip_runtime.h>
#include <stdint.h>

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
  uint32_t wcnt[NT / 64][256];
  uint32_t woff[NT / 64][256];
  uint64_t wtot[NT / 64];
  int32_t flags[8];
};

// Stable LSD radix sort (8-bit digits) of n keys in LDS, ascending.  Each
// round places NT keys: a key's rank among equal digits of its wave comes
// from eight ballots (the lanes that share its digit), the offset of earlier
// waves and earlier rounds from per-(wave, digit) counts.  Returns the buffer
// index holding the result.
template <int NT, int CAP>
__device__ int lds_radix_sort(PrepSmem<NT, CAP> &sm, int n, int bits) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  int src = 0;
  for (int sh = 0; sh < bits; sh += 8) {
    uint32_t *a = sm.keys[src];
    uint32_t *b = sm.keys[src ^ 1];
    for (int i = tid; i < 256; i += NT) sm.hist[i] = 0;
    for (int i = tid; i < NW * 256; i += NT) (&sm.wcnt[0][0])[i] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += NT) atomicAdd(&sm.hist[(a[i] >> sh) & 255u], 1u);
    __syncthreads();
    // exclusive scan of the 256 digit counts by wave 0 (4 digits per lane)
    if (tid < 64) {
      uint32_t c0 = sm.hist[4 * tid], c1 = sm.hist[4 * tid + 1], c2 = sm.hist[4 * tid + 2], c3 = sm.hist[4 * tid + 3];
      uint32_t tot = c0 + c1 + c2 + c3;
      uint32_t excl = wave_incl_scan_u32(tot) - tot;
      sm.hist[4 * tid] = excl;
      sm.hist[4 * tid + 1] = excl + c0;
      sm.hist[4 * tid + 2] = excl + c0 + c1;
      sm.hist[4 * tid + 3] = excl + c0 + c1 + c2;
    }
    __syncthreads();
    for (int base = 0; base < n; base += NT) {
      const int i = base + tid;
      const bool valid = i < n;
      const uint32_t key = valid ? a[i] : 0u;
      const uint32_t d = (key >> sh) & 255u;
      uint64_t peers = ballot64(valid);
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        const bool set = (d >> bit) & 1u;
        const uint64_t m = ballot64(valid && set);
        peers &= set ? m : ~m;
      }
      const uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt());
      if (valid && rank == 0) sm.wcnt[wave][d] = (uint32_t)__popcll(peers);
      __syncthreads();
      // per digit: offsets of the waves of this round, then advance the digit base
      for (int dg = tid; dg < 256; dg += NT) {
        uint32_t run = sm.hist[dg];
        for (int w = 0; w < NW; ++w) {
          uint32_t c = sm.wcnt[w][dg];
          sm.woff[w][dg] = run;
          sm.wcnt[w][dg] = 0;
          run += c;
        }
        sm.hist[dg] = run;
      }
      __syncthreads();
      if (valid) b[sm.woff[wave][d] + rank] = key;
      __syncthreads();
    }
    src ^= 1;
  }
  return src;
}

// Exclusive prefix sums of the sorted sizes into pre[0..n], block-wide.
template <int NT, int CAP>
__device__ void block_prefix(PrepSmem<NT, CAP> &sm, const uint32_t *sizes, int n, int64_t *pre) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  uint64_t carry = 0;
  if (tid == 0) pre[0] = 0;
  for (int base = 0; base < n; base += NT) {
    const int i = base + tid;
    const uint64_t v = i < n ? sizes[i] : 0u;
    const uint64_t incl = wave_incl_scan_u64(v);
    if ((tid & 63) == 63) sm.wtot[wave] = incl;
    __syncthreads();
    uint64_t before = carry;
    for (int w = 0; w < wave; ++w) before += sm.wtot[w];
    if (i < n) pre[i + 1] = (int64_t)(before + incl);
    uint64_t all = 0;
    for (int w = 0; w < NW; ++w) all += sm.wtot[w];
    carry += all;
    __syncthreads();
  }
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
  if (tid < 8) sm.flags[tid] = 0;
  __syncthreads();
  if (p.r_cap > CAP) {
    status = BP_ERR_LIMIT;
  } else {
    // Reduction into LDS: sort key = c - w (ascending key = decreasing size).
    const BP_GLOBAL int32_t *in = as_global(d.in + p.in_off);
    const int64_t n_in = p.n_in;
    for (int64_t i = tid; i < n_in; i += NT) {
      int32_t w = in[i];
      if (w < 0 || w > C) { sm.flags[0] = 1; w = 0; }
      sm.keys[0][i] = uC - (uint32_t)w;
    }
    int64_t nfill = 0;
    if (p.form == kFormResidual) {
      // one virtual item of size c - residual per bin with residual < c (Fig. 3)
      const BP_GLOBAL int32_t *res = as_global(d.in + p.res_off);
      for (int base = 0; base < p.m_res; base += NT) {
        const int j = base + tid;
        int32_t rj = j < p.m_res ? res[j] : C;
        if (rj < 0 || rj > C) { sm.flags[0] = 1; rj = C; }
        const bool take = rj < C;
        // stable compaction of the loaded bins, in bin order
        const uint64_t bal = ballot64(take);
        const uint32_t below = (uint32_t)__popcll(bal & lanemask_lt());
        if ((tid & 63) == 0) sm.wcnt[0][tid >> 6] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t off = 0;
        for (int w = 0; w < (tid >> 6); ++w) off += sm.wcnt[0][w];
        uint32_t tot = 0;
        for (int w = 0; w < NT / 64; ++w) tot += sm.wcnt[0][w];
        if (take) sm.keys[0][n_in + nfill + off + below] = (uint32_t)rj;  // key = c - load = residual
        nfill += tot;
        __syncthreads();
      }
    }
    r = n_in + nfill;
    __syncthreads();
    if (sm.flags[0]) {
      status = BP_ERR_RANGE;
      r = 0;
    }
    const int bits = 32 - __clz((int)uC);  // keys are <= c
    const int res_buf = lds_radix_sort<NT, CAP>(sm, (int)r, bits);
    uint32_t *keys = sm.keys[res_buf];
    uint32_t *sz = sm.keys[res_buf ^ 1];
    for (int i = tid; i < r; i += NT) sz[i] = uC - keys[i];
    __syncthreads();
    // class boundaries on the decreasing sizes
    if (tid < 8) sm.flags[tid] = 0;
    __syncthreads();
    int c_full = 0, c_big = 0, c_bm = 0, c_nz = 0;
    for (int i = tid; i < r; i += NT) {
      const uint32_t w = sz[i];
      c_full += w == uC;
      c_big += 2ull * w > uC;
      c_bm += 2ull * w >= uC;
      c_nz += w > 0;
    }
    if (c_full) atomicAdd(&sm.flags[1], c_full);
    if (c_big) atomicAdd(&sm.flags[2], c_big);
    if (c_bm) atomicAdd(&sm.flags[3], c_bm);
    if (c_nz) atomicAdd(&sm.flags[4], c_nz);
    __syncthreads();
    const int nf = sm.flags[1], nb = sm.flags[2], nm = sm.flags[3], nz = sm.flags[4];
    int32_t *sorted = d.sorted + p.ws_off;
    ItemRec *rec = d.rec + p.ws_off;
    for (int i = tid; i < r; i += NT) {
      const uint32_t w = sz[i];
      sorted[i] = (int32_t)w;
      const uint32_t a = (2ull * w > uC) ? uC - w : w;
      ItemRec ir;
      ir.w = w;
      ir.a = a;
      ir.a2 = 2u * a;
      ir.w2 = 2u * w;
      rec[i] = ir;
    }
    int64_t *pre = d.pre + p.pre_off;
    block_prefix<NT, CAP>(sm, sz, (int)r, pre);
    __syncthreads();
    if (tid == 0) {
      st->r = (int32_t)r;
      st->nf = nf;
      st->nb = nb;
      st->nm = nm;
      st->nz = nz;
      st->maxw = r > 0 ? (int32_t)sz[0] : 0;
    }
  }
  __syncthreads();
  if (tid == 0) {
    st->status = status;
    if (status != BP_OK) {
      st->r = 0; st->nf = st->nb = st->nm = st->nz = 0; st->maxw = 0;
    }
  }
}

// Second half of prep (thread 0): sums, effective ranges, cleared results.
__device__ void prep_finish(const LaunchDesc &d, int64_t inst) {
  const BP_CONST InstPlan &p = as_const(d.plan)[inst];
  InstState *st = &d.state[inst];
  const int64_t *pre = d.pre + p.pre_off;
  const int32_t r = st->r;
  st->sumW = r > 0 ? pre[r] : 0;
  st->sumBig = r > 0 ? pre[st->nb] - pre[st->nf] : 0;
  st->sumNZ = r > 0 ? pre[st->nz] - pre[st->nf] : 0;
  for (int b = 0; b < kNB; ++b) st->hiEff[b] = p.hi[b];
  if ((p.flags & kPlanClampVB2) && st->status == BP_OK) {
    const int64_t denom = (int64_t)r * (int64_t)st->maxw;
    const int64_t cap = denom > 0 ? (int64_t)0xffffffffLL / denom : (int64_t)p.C;
    if (cap < st->hiEff[kVB2]) st->hiEff[kVB2] = cap;
  }
  for (int b = 0; b < kNB; ++b) d.keys[inst * kNB + b] = 0ull;
  int refuted = 0;
  if ((p.flags & kPlanEarlyExit) && st->status == BP_OK && r > 0) {
    const int64_t l1 = (st->sumW + p.C - 1) / p.C;
    refuted = l1 > p.k;
  }
  d.refuted[inst] = refuted;
}

template <int NT, int CAP, int LARGE>
__global__ __launch_bounds__(NT) void k_prep(const LaunchDesc *__restrict__ dp) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  PrepSmem<NT, CAP> &sm = *reinterpret_cast<PrepSmem<NT, CAP> *>(smem_raw);
  const LaunchDesc d = *as_const(dp);
  if (blockIdx.x == 0 && threadIdx.x == 0 && !LARGE) *d.counter = 0ull;
  for (int64_t inst = blockIdx.x; inst < d.count; inst += gridDim.x) {
    if (as_const(d.plan)[inst].large != LARGE) continue;
    prep_instance<NT, CAP>(d, inst, sm);
    __syncthreads();
    if (threadIdx.x == 0) prep_finish(d, inst);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Sweep tiles.  Each lane holds kLPL parameters lam = lam0 + lane + 64 j.
// Lanes past the end of the range compute with lam = lo and are dropped.

struct TileArgs {
  const BP_CONST ItemRec *rec;
  const BP_GLOBAL int32_t *sorted;
  const BP_GLOBAL int64_t *pre;
  int64_t lo, hi;        // effective range of the bound
  int64_t lam0;          // first parameter of the tile
  int64_t k;
  int32_t C, r, nf, nb, nm, nz;
  int64_t sumBig, sumNZ;
};

// Largest number of items whose per-item increments, each at most maxinc,
// can be summed in 32 bits.
__device__ __forceinline__ int chunk_len(uint64_t maxinc) {
  if (maxinc == 0) return 1 << 30;
  uint64_t l = 0xffffffffull / maxinc;
  return l > (1ull << 30) ? (1 << 30) : (int)l;
}

__device__ __forceinline__ int64_t ceil_div_i64(int64_t a, int64_t b) { return a / b + (a % b != 0); }

// f_MT: big items add c when c - w < lambda (else w, summed in sumBig);
// mid items add c/2; small items add w when w >= lambda.
__device__ void tile_mt(const TileArgs &t, int64_t lam_out[kLPL], int64_t lbp[kLPL]) {
  uint32_t lam[kLPL];
  for (int j = 0; j < kLPL; ++j) {
    int64_t L = t.lam0 + lane_id() + 64 * j;
    lam_out[j] = L;
    lam[j] = (uint32_t)(L <= t.hi ? L : t.lo);
  }
  uint64_t acc[kLPL] = {};
  const int L = chunk_len((uint64_t)t.C / 2 + 1);
  for (int i0 = t.nf; i0 < t.nb;) {
    const int e = i0 + min(t.nb - i0, L);  // i0 + L could overflow int
    uint32_t s[kLPL] = {};
#pragma unroll 8
    for (int i = i0; i < e; ++i) {
      const uint32_t a = t.rec[i].a;
      for (int j = 0; j < kLPL; ++j) s[j] += a < lam[j] ? a : 0u;
    }
    for (int j = 0; j < kLPL; ++j) acc[j] += s[j];
    i0 = e;
  }
  for (int i0 = t.nm; i0 < t.nz;) {
    const int e = i0 + min(t.nz - i0, L);  // i0 + L could overflow int
    uint32_t s[kLPL] = {};
#pragma unroll 8
    for (int i = i0; i < e; ++i) {
      const uint32_t w = t.rec[i].w;
      for (int j = 0; j < kLPL; ++j) s[j] += w >= lam[j] ? w : 0u;
    }
    for (int j = 0; j < kLPL; ++j) acc[j] += s[j];
    i0 = e;
  }
  const int64_t nmid = t.nm - t.nb;
  for (int j = 0; j < kLPL; ++j) {
    const int64_t S = t.sumBig + (int64_t)acc[j] + nmid * (int64_t)(t.C / 2);
    lbp[j] = ceil_div_i64(S, (int64_t)t.C);
  }
}

// f_RAD2 (c/4 < lambda <= c/3), counts of threshold crossings:
//   small: c3 [w >= lambda] + (c2 - c3) [w > c - 2 lambda]
//   big:   c2 + (c - c2 - c3) [w >= 2 lambda] + c3 [w > c - lambda]
//   mid:   c2
__device__ void tile_rad2(const TileArgs &t, int64_t lam_out[kLPL], int64_t lbp[kLPL]) {
  uint32_t t1[kLPL], t2[kLPL], t3[kLPL], t4[kLPL];
  for (int j = 0; j < kLPL; ++j) {
    int64_t L = t.lam0 + lane_id() + 64 * j;
    lam_out[j] = L;
    const uint32_t l = (uint32_t)(L <= t.hi ? L : t.lo);
    t1[j] = l;
    t2[j] = (uint32_t)t.C - 2u * l + 1u;
    t3[j] = 2u * l;
    t4[j] = (uint32_t)t.C - l + 1u;
  }
  uint32_t n1[kLPL] = {}, n2[kLPL] = {}, n3[kLPL] = {}, n4[kLPL] = {};
#pragma unroll 8
  for (int i = t.nm; i < t.nz; ++i) {
    const uint32_t w = t.rec[i].w;
    for (int j = 0; j < kLPL; ++j) {
      n1[j] += w >= t1[j];
      n2[j] += w >= t2[j];
    }
  }
#pragma unroll 8
  for (int i = t.nf; i < t.nb; ++i) {
    const uint32_t w = t.rec[i].w;
    for (int j = 0; j < kLPL; ++j) {
      n3[j] += w >= t3[j];
      n4[j] += w >= t4[j];
    }
  }
  const int64_t C = t.C, c3 = C / 3, c2 = C / 2;
  const int64_t nbig = t.nb - t.nf, nmid = t.nm - t.nb;
  for (int j = 0; j < kLPL; ++j) {
    const int64_t S = (nbig + nmid) * c2 + c3 * n1[j] + (c2 - c3) * n2[j] + (C - c2 - c3) * n3[j] + c3 * n4[j];
    lbp[j] = ceil_div_i64(S, C);
  }
}

// f_FS1 (1 <= lambda <= 100): with n = w (lambda + 1) and q = floor(n / c),
// f = q c - w [c divides n].  Evaluated in fp64, exact: n < 2^38, and
// q = floor((n + 0.5) / c) is computed from (n + 0.5) * (1/c) whose relative
// error (2^-52) is below the distance 0.5/c of (n + 0.5)/c to an integer;
// the remainder fma(-q, c, n) is exact.
__device__ void tile_fs1(const TileArgs &t, int64_t lam_out[kLPL], int64_t lbp[kLPL]) {
  double l1[kLPL];
  for (int j = 0; j < kLPL; ++j) {
    int64_t L = t.lam0 + lane_id() + 64 * j;
    lam_out[j] = L;
    l1[j] = (double)((L <= t.hi ? L : t.lo) + 1);
  }
  const double Cd = (double)t.C;
  const double rc = 1.0 / Cd;
  double Q[kLPL] = {}, D[kLPL] = {};
#pragma unroll 4
  for (int i = t.nf; i < t.nz; ++i) {
    const double w = (double)t.rec[i].w;
    for (int j = 0; j < kLPL; ++j) {
      const double n = w * l1[j];
      const double q = floor((n + 0.5) * rc);
      const double rem = fma(-q, Cd, n);
      Q[j] += q;
      D[j] += rem == 0.0 ? w : 0.0;
    }
  }
  for (int j = 0; j < kLPL; ++j) {
    const int64_t lam = (int64_t)l1[j] - 1;
    const int64_t S = (int64_t)Q[j] * (int64_t)t.C - (int64_t)D[j];
    lbp[j] = ceil_div_i64(S, (int64_t)t.C * lam);
  }
}

// f_CCM1 (1 <= lambda <= c/2), K = floor(c / lambda):
//   big 2K - 2 floor((c - w)/lambda), mid K, small 2 floor(w / lambda).
__device__ void tile_ccm1(const TileArgs &t, int64_t lam_out[kLPL], int64_t lbp[kLPL]) {
  uint32_t mg[kLPL], sh[kLPL], lmin = 0xffffffffu;
  for (int j = 0; j < kLPL; ++j) {
    int64_t L = t.lam0 + lane_id() + 64 * j;
    lam_out[j] = L;
    const uint32_t l = (uint32_t)(L <= t.hi ? L : t.lo);
    const MagicU31 g = magic_u31(l);
    mg[j] = g.m;
    sh[j] = g.s;
    lmin = min(lmin, l);
  }
  lmin = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)max((int64_t)t.lo, t.lam0));
  uint64_t hb[kLPL] = {}, hs[kLPL] = {};
  const int L = chunk_len(((uint64_t)t.C / 2) / lmin + 1);
  for (int i0 = t.nf; i0 < t.nb;) {
    const int e = i0 + min(t.nb - i0, L);  // i0 + L could overflow int
    uint32_t s[kLPL] = {};
#pragma unroll 8
    for (int i = i0; i < e; ++i) {
      const uint32_t a2 = t.rec[i].a2;
      for (int j = 0; j < kLPL; ++j) s[j] += div_u31(a2, mg[j], sh[j]);
    }
    for (int j = 0; j < kLPL; ++j) hb[j] += s[j];
    i0 = e;
  }
  for (int i0 = t.nm; i0 < t.nz;) {
    const int e = i0 + min(t.nz - i0, L);  // i0 + L could overflow int
    uint32_t s[kLPL] = {};
#pragma unroll 8
    for (int i = i0; i < e; ++i) {
      const uint32_t a2 = t.rec[i].a2;
      for (int j = 0; j < kLPL; ++j) s[j] += div_u31(a2, mg[j], sh[j]);
    }
    for (int j = 0; j < kLPL; ++j) hs[j] += s[j];
    i0 = e;
  }
  const int64_t nbig = t.nb - t.nf, nmid = t.nm - t.nb;
  for (int j = 0; j < kLPL; ++j) {
    const int64_t lam = lam_out[j] <= t.hi ? lam_out[j] : t.lo;
    const int64_t K = (int64_t)t.C / lam;
    const int64_t S = 2 * K * nbig - 2 * (int64_t)hb[j] + K * nmid + 2 * (int64_t)hs[j];
    lbp[j] = ceil_div_i64(S, 2 * K);
  }
}

// f_VB2 (2 <= lambda <= c), h(a) = ceil(a lambda / c) - 1 for a >= 1:
//   big 2(lambda - 1) - 2 h(c - w), mid lambda - 1, small 2 h(w).
__device__ void tile_vb2(const TileArgs &t, int64_t lam_out[kLPL], int64_t lbp[kLPL]) {
  uint32_t rlo[kLPL], rhi[kLPL];
  uint32_t lmax = 0;
  for (int j = 0; j < kLPL; ++j) {
    int64_t L = t.lam0 + lane_id() + 64 * j;
    lam_out[j] = L;
    const uint32_t l = (uint32_t)(L <= t.hi ? L : t.lo);
    const uint64_t R = vb2_recip(l, (uint32_t)t.C);
    rlo[j] = (uint32_t)R;
    rhi[j] = (uint32_t)(R >> 32);
  }
  lmax = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)min(t.hi, t.lam0 + kTile - 1));
  uint64_t hb[kLPL] = {}, hs[kLPL] = {};
  // h(a) <= a lambda / c <= lambda / 2 for a <= c/2
  const int L = chunk_len((uint64_t)lmax / 2 + 1);
  for (int i0 = t.nf; i0 < t.nb;) {
    const int e = i0 + min(t.nb - i0, L);  // i0 + L could overflow int
    uint32_t s[kLPL] = {};
#pragma unroll 8
    for (int i = i0; i < e; ++i) {
      const uint32_t a = t.rec[i].a;
      for (int j = 0; j < kLPL; ++j) s[j] += vb2_part(a, rlo[j], rhi[j]);
    }
    for (int j = 0; j < kLPL; ++j) hb[j] += s[j];
    i0 = e;
  }
  for (int i0 = t.nm; i0 < t.nz;) {
    const int e = i0 + min(t.nz - i0, L);  // i0 + L could overflow int
    uint32_t s[kLPL] = {};
#pragma unroll 8
    for (int i = i0; i < e; ++i) {
      const uint32_t a = t.rec[i].a;
      for (int j = 0; j < kLPL; ++j) s[j] += vb2_part(a, rlo[j], rhi[j]);
    }
    for (int j = 0; j < kLPL; ++j) hs[j] += s[j];
    i0 = e;
  }
  const int64_t nbig = t.nb - t.nf, nmid = t.nm - t.nb;
  for (int j = 0; j < kLPL; ++j) {
    const int64_t lam = lam_out[j] <= t.hi ? lam_out[j] : t.lo;
    const int64_t K = lam - 1;
    const int64_t S = 2 * K * nbig - 2 * (int64_t)hb[j] + K * nmid + 2 * (int64_t)hs[j];
    lbp[j] = ceil_div_i64(S, 2 * K);
  }
}

// f_BJ1 (1 <= lambda <= c), p = c mod lambda, q = floor(w / lambda),
// rem = w - q lambda:  f = q (lambda - p) + max(0, rem - p)
//                        = q (lambda - p) + (rem - p + |rem - p|) / 2.
// Per item the lane keeps Q += q and A += |w - (q lambda + p)| = |rem - p|;
// then  S = (lambda - p) Q + (W - lambda Q - n p + A) / 2  with W = sum w.
__device__ void tile_bj1(const TileArgs &t, int64_t lam_out[kLPL], int64_t lbp[kLPL]) {
  uint32_t mg[kLPL], sh[kLPL], lam[kLPL], pm[kLPL];
  for (int j = 0; j < kLPL; ++j) {
    int64_t L = t.lam0 + lane_id() + 64 * j;
    lam_out[j] = L;
    const uint32_t l = (uint32_t)(L <= t.hi ? L : t.lo);
    const MagicU31 g = magic_u31(l);
    mg[j] = g.m;
    sh[j] = g.s;
    lam[j] = l;
    pm[j] = (uint32_t)t.C % l;
  }
  const uint32_t lmin = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)max((int64_t)t.lo, t.lam0));
  const uint32_t lmax = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)min(t.hi, t.lam0 + kTile - 1));
  uint64_t Q[kLPL] = {}, A[kLPL] = {};
  const uint64_t inc = max((uint64_t)((uint32_t)t.C / lmin), (uint64_t)lmax) + 1;
  const int L = chunk_len(inc);
  for (int i0 = t.nf; i0 < t.nz;) {
    const int e = i0 + min(t.nz - i0, L);  // i0 + L could overflow int
    uint32_t sq[kLPL] = {}, sa[kLPL] = {};
    // unrolled by hand: the inline v_sad_u32 keeps the compiler from unrolling
    int i = i0;
    for (; i + 4 <= e; i += 4) {
      ItemRec it[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) it[u] = t.rec[i + u];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        for (int j = 0; j < kLPL; ++j) {
          const uint32_t q = div_u31(it[u].w2, mg[j], sh[j]);
          const uint32_t v = q * lam[j] + pm[j];
          sq[j] += q;
          sa[j] = sad_u32(it[u].w, v, sa[j]);
        }
      }
    }
    for (; i < e; ++i) {
      const ItemRec it = t.rec[i];
      for (int j = 0; j < kLPL; ++j) {
        const uint32_t q = div_u31(it.w2, mg[j], sh[j]);
        const uint32_t v = q * lam[j] + pm[j];
        sq[j] += q;
        sa[j] = sad_u32(it.w, v, sa[j]);
      }
    }
    for (int j = 0; j < kLPL; ++j) {
      Q[j] += sq[j];
      A[j] += sa[j];
    }
    i0 = e;
  }
  const int64_t n = t.nz - t.nf;
  for (int j = 0; j < kLPL; ++j) {
    const int64_t l = lam[j], p = pm[j];
    const int64_t q = (int64_t)Q[j];
    const int64_t S = (l - p) * q + (t.sumNZ - l * q - n * p + (int64_t)A[j]) / 2;
    const int64_t fc = ((int64_t)t.C / l) * (l - p);
    lbp[j] = ceil_div_i64(S, fc);
  }
}

// First index of the decreasing array s[0..r) whose value is <= x.
__device__ __forceinline__ int32_t first_le(const BP_GLOBAL int32_t *s, int32_t r, int64_t x) {
  int32_t lo = 0, hi = r;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if ((int64_t)s[mid] > x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// L2 (Sec. 3.1) evaluated at the parameters where it can change: the range's
// first parameter and w + 1, c - w + 1 for every size.  Candidate index
// c = 0 is lo; c = 1 + 2i is w_i + 1; c = 2 + 2i is c - w_i + 1.
// With nbig = #{2w > c} (every big item is in W1 or W2):
//   n1 = #{w > c - lambda}, n2 = nbig - n1, sum W2 = pre[nbig] - pre[n1],
//   W3 = {lambda <= w <= c/2} = sorted[nbig, j3) with j3 = #{w >= lambda},
//   L2(lambda) = nbig + max(0, ceil((sum W3 - (c n2 - sum W2)) / c)).
__device__ void tile_l2(const TileArgs &t, int64_t lam_out[kLPL], int64_t lbp[kLPL], bool ok[kLPL]) {
  const int64_t C = t.C;
  const int32_t nbig = t.nb;  // includes the items of size c
  for (int j = 0; j < kLPL; ++j) {
    const int64_t cidx = t.lam0 + lane_id() + 64 * j;
    int64_t lam = -1;
    if (cidx == 0) lam = t.lo;
    else if (cidx <= 2 * (int64_t)t.r) {
      const int64_t i = (cidx - 1) >> 1;
      const int64_t w = t.sorted[i];
      lam = ((cidx - 1) & 1) ? C - w + 1 : w + 1;
    }
    ok[j] = lam >= t.lo && lam <= t.hi;
    if (!ok[j]) lam = t.lo;
    lam_out[j] = lam;
    const int32_t n1 = first_le(t.sorted, t.r, C - lam);
    const int32_t j3 = first_le(t.sorted, t.r, lam - 1);
    const int64_t n2 = nbig - n1;
    const int64_t s2 = t.pre[nbig] - t.pre[n1];
    const int64_t s3 = j3 > nbig ? t.pre[j3] - t.pre[nbig] : 0;
    const int64_t x = s3 - (C * n2 - s2);
    lbp[j] = nbig + (x > 0 ? ceil_div_i64(x, C) : 0);
  }
}

__device__ __forceinline__ void flush_tile(const LaunchDesc &d, int64_t inst, int bound, const TileArgs &t,
                                           const int64_t lam[kLPL], const int64_t lbp[kLPL], const bool *okp) {
  uint64_t key = 0;
  int64_t best = -1;
  for (int j = 0; j < kLPL; ++j) {
    const bool ok = okp ? okp[j] : (lam[j] >= t.lo && lam[j] <= t.hi);
    if (ok) {
      const uint64_t kk = pack_key(lbp[j], lam[j]);
      key = umax64(key, kk);
      best = max(best, lbp[j]);
    }
  }
  const uint64_t wmax = wave_max_u64(key);
  if (lane_id() == 0 && wmax) {
    atomicMax(&d.keys[inst * kNB + bound], (unsigned long long)wmax);
    if (as_const(d.plan)[inst].flags & kPlanEarlyExit) {
      const int64_t v = (int64_t)(wmax >> 32) + (bound == kL2 ? 0 : t.nf);
      if (v > t.k) d.refuted[inst] = 1;
    }
  }
  (void)best;
}

__device__ __forceinline__ int64_t find_entry(const BP_CONST Entry *e, int64_t n, uint64_t task) {
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if ((uint64_t)e[mid].task_begin <= task) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(64) void k_sweep(const LaunchDesc *__restrict__ dp) {
  const LaunchDesc d = *as_const(dp);
  const BP_CONST Entry *entries = as_const(d.entries);
  const BP_CONST InstState *states = as_const(d.state);
  const BP_CONST InstPlan *plans = as_const(d.plan);
  for (;;) {
    unsigned long long task = 0;
    if (lane_id() == 0) task = atomicAdd(d.counter, 1ull);
    task = (unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)task) |
           ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(task >> 32)) << 32);
    if (task >= (unsigned long long)d.ntasks) return;
    const int64_t ei = find_entry(entries, d.nentries, task);
    const BP_CONST Entry &e = entries[ei];
    const int64_t inst = e.inst;
    const BP_CONST InstState &st = states[inst];
    if (st.status != BP_OK) continue;
    const BP_CONST InstPlan &p = plans[inst];
    TileArgs t;
    t.rec = as_const(d.rec + p.ws_off);
    t.sorted = as_global(d.sorted + p.ws_off);
    t.pre = as_global(d.pre + p.pre_off);
    t.lo = p.lo[e.bound];
    t.hi = st.hiEff[e.bound];
    t.k = p.k;
    t.C = p.C;
    t.r = st.r;
    t.nf = st.nf;
    t.nb = st.nb;
    t.nm = st.nm;
    t.nz = st.nz;
    t.sumBig = st.sumBig;
    t.sumNZ = st.sumNZ;
    const bool early = (p.flags & kPlanEarlyExit) != 0;
    const int64_t tile0 = ((int64_t)task - e.task_begin) * e.tpt;
    const int64_t tile1 = min(e.ntiles, tile0 + e.tpt);
    for (int64_t tl = tile0; tl < tile1; ++tl) {
      if (early && __builtin_amdgcn_readfirstlane(*(volatile int32_t *)&d.refuted[inst])) break;
      t.lam0 = e.lam0 + tl * kTile;
      int64_t lam[kLPL], lbp[kLPL];
      bool ok[kLPL];
      if (e.bound == kL2) {
        // tiles of L2 run over candidate indices, not parameters
        tile_l2(t, lam, lbp, ok);
        flush_tile(d, inst, kL2, t, lam, lbp, ok);
        continue;
      }
      if (t.lam0 > t.hi) break;
      switch (e.bound) {
        case kMT: tile_mt(t, lam, lbp); break;
        case kRAD2: tile_rad2(t, lam, lbp); break;
        case kFS1: tile_fs1(t, lam, lbp); break;
        case kCCM1: tile_ccm1(t, lam, lbp); break;
        case kVB2: tile_vb2(t, lam, lbp); break;
        default: tile_bj1(t, lam, lbp); break;
      }
      flush_tile(d, inst, e.bound, t, lam, lbp, nullptr);
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
size_t prep_smem_large() { return sizeof(PrepSmem<kLargeThreads, kLargeCap>); }

hipError_t set_kernel_attrs() {
  hipError_t e = hipFuncSetAttribute((const void *)k_prep<kSmallThreads, kSmallCap, 0>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)prep_smem_small());
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void *)k_prep<kLargeThreads, kLargeCap, 1>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)prep_smem_large());
}

hipError_t launch_pipeline(const LaunchDesc *d_desc, int grid_prep_small, int grid_prep_large, int grid_sweep,
                           int grid_fin, hipStream_t s) {
  hipLaunchKernelGGL((k_prep<kSmallThreads, kSmallCap, 0>), dim3(grid_prep_small), dim3(kSmallThreads),
                     prep_smem_small(), s, d_desc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (grid_prep_large > 0) {
    hipLaunchKernelGGL((k_prep<kLargeThreads, kLargeCap, 1>), dim3(grid_prep_large), dim3(kLargeThreads),
                       prep_smem_large(), s, d_desc);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_sweep, dim3(grid_sweep), dim3(64), 0, s, d_desc);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_finalize, dim3(grid_fin), dim3(256), 0, s, d_desc);
  return hipGetLastError();
}

// The same four launches with events around the stages (diagnostic timing).
hipError_t launch_pipeline_timed(const LaunchDesc *d_desc, int grid_prep_small, int grid_prep_large, int grid_sweep,
                                 int grid_fin, hipStream_t s, hipEvent_t ev[4]) {
  hipError_t e = hipEventRecord(ev[0], s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_prep<kSmallThreads, kSmallCap, 0>), dim3(grid_prep_small), dim3(kSmallThreads),
                     prep_smem_small(), s, d_desc);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((k_prep<kLargeThreads, kLargeCap, 1>), dim3(grid_prep_large), dim3(kLargeThreads),
                     prep_smem_large(), s, d_desc);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_sweep, dim3(grid_sweep), dim3(64), 0, s, d_desc);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_finalize, dim3(grid_fin), dim3(256), 0, s, d_desc);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return hipEventRecord(ev[3], s);
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
