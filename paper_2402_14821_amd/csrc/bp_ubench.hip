// bp_ubench.hip -- VALU issue-rate microbenchmark for gfx950.
//
// Measures, per opcode used by the inner loops of the sweep kernel, how many
// lane-operations per second the whole device sustains when every wave
// issues nothing but that opcode on eight independent dependency chains.
// The result, divided by the full rate (256 CUs x 4 SIMDs x 16 lanes x the
// clock), tells whether an opcode occupies a full VALU issue slot (ratio
// ~1) or less.  These ratios are the weights of the sweep's roofline
// accounting.  Separate library (libbp_ubench.so): not part of the check.
//
// Every instruction under test is written in inline asm so that the
// compiler cannot fold, combine or strength-reduce it; the chains' final
// values are stored, so no chain is dead.  No memory is read inside the
// timed loops.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

enum Op : int {
  kAddU32 = 0, kSubU32, kAndB32, kXorB32, kLshrB32, kAshrI32, kAdd3U32, kSadU32, kMulLoU32, kMulHiU32,
  kMadU64U32, kCndmask, kMaxU32, kAddCoU32, kCmpLtU32, kFmaF64, kAddF64, kMulF64, kCvtF64U32, kBfeI32,
  kMadU32U24, kMulU32U24, kMulHiU32U24, kLshlAddU32, kNumOps
};

const char *const kNames[kNumOps] = {
  "v_add_u32", "v_sub_u32", "v_and_b32", "v_xor_b32", "v_lshrrev_b32", "v_ashrrev_i32", "v_add3_u32",
  "v_sad_u32", "v_mul_lo_u32", "v_mul_hi_u32", "v_mad_u64_u32", "v_cndmask_b32", "v_max_u32",
  "v_add_co_u32", "v_cmp_lt_u32", "v_fma_f64", "v_add_f64", "v_mul_f64", "v_cvt_f64_u32", "v_bfe_i32",
  "v_mad_u32_u24", "v_mul_u32_u24", "v_mul_hi_u32_u24", "v_lshl_add_u32"};

constexpr int kChains = 8;
constexpr int kUnroll = 16;  // steps of each chain per loop iteration (one asm block of kChains * kUnroll instructions)

// One block: the opcode under test kUnroll times on each of the eight
// chains, in a single asm statement (separate statements would get a
// hazard-guard s_nop between them).  Scalar outputs (carry, compare mask) go to one SGPR pair,
// overwritten by every instruction and folded into the stored value once at
// the end, so that no scalar instruction runs per step.
#define BPU_ROW(F) F(0) F(1) F(2) F(3) F(4) F(5) F(6) F(7)
#define BPU_L8(F)                                                                                         \
  BPU_ROW(F) BPU_ROW(F) BPU_ROW(F) BPU_ROW(F) BPU_ROW(F) BPU_ROW(F) BPU_ROW(F) BPU_ROW(F) BPU_ROW(F) \
      BPU_ROW(F) BPU_ROW(F) BPU_ROW(F) BPU_ROW(F) BPU_ROW(F) BPU_ROW(F) BPU_ROW(F)
#define BPU_X8 "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]), "+v"(x[6]), "+v"(x[7])

#define BPU_ADD(i) "v_add_u32 %" #i ", %" #i ", %8\n\t"
#define BPU_SUB(i) "v_sub_u32 %" #i ", %" #i ", %8\n\t"
#define BPU_AND(i) "v_and_b32 %" #i ", %" #i ", %8\n\t"
#define BPU_XOR(i) "v_xor_b32 %" #i ", %" #i ", %8\n\t"
#define BPU_LSHR(i) "v_lshrrev_b32 %" #i ", %8, %" #i "\n\t"
#define BPU_ASHR(i) "v_ashrrev_i32 %" #i ", %8, %" #i "\n\t"
#define BPU_ADD3(i) "v_add3_u32 %" #i ", %" #i ", %8, %8\n\t"
#define BPU_SAD(i) "v_sad_u32 %" #i ", %8, %" #i ", %" #i "\n\t"
#define BPU_MULLO(i) "v_mul_lo_u32 %" #i ", %" #i ", %8\n\t"
#define BPU_MULHI(i) "v_mul_hi_u32 %" #i ", %" #i ", %8\n\t"
#define BPU_MAX(i) "v_max_u32 %" #i ", %" #i ", %8\n\t"
#define BPU_BFE(i) "v_bfe_i32 %" #i ", %" #i ", %8, 1\n\t"
#define BPU_MAD24(i) "v_mad_u32_u24 %" #i ", %" #i ", %8, %8\n\t"
#define BPU_MUL24(i) "v_mul_u32_u24 %" #i ", %" #i ", %8\n\t"
#define BPU_MULHI24(i) "v_mul_hi_u32_u24 %" #i ", %" #i ", %8\n\t"
#define BPU_LSHLADD(i) "v_lshl_add_u32 %" #i ", %" #i ", 1, %8\n\t"
#define BPU_CND(i) "v_cndmask_b32_e64 %" #i ", %" #i ", %8, %9\n\t"
#define BPU_ADDCO(i) "v_add_co_u32_e64 %" #i ", %8, %" #i ", %9\n\t"
#define BPU_CMP(i) "v_cmp_lt_u32_e64 %8, %" #i ", %9\n\t"
// v_mad_u64_u32: each chain x_i = a_i * b + x_i through the 64-bit addend
// (a_i a fixed 32-bit operand, %10 .. %17)
#define BPU_MADI(i, a) "v_mad_u64_u32 %" #i ", %8, %" #a ", %9, %" #i "\n\t"
#define BPU_MADROW                                                                                      \
  BPU_MADI(0, 10) BPU_MADI(1, 11) BPU_MADI(2, 12) BPU_MADI(3, 13) BPU_MADI(4, 14) BPU_MADI(5, 15) \
      BPU_MADI(6, 16) BPU_MADI(7, 17)
#define BPU_FMA(i) "v_fma_f64 %" #i ", %" #i ", %8, %8\n\t"
#define BPU_ADDF(i) "v_add_f64 %" #i ", %" #i ", %8\n\t"
#define BPU_MULF(i) "v_mul_f64 %" #i ", %" #i ", %8\n\t"
#define BPU_CVT(i) "v_cvt_f64_u32 %" #i ", %8\n\t"

template <int OP>
__device__ __forceinline__ void row32(uint32_t (&x)[kChains], uint32_t b, uint64_t m, uint64_t &c) {
  if constexpr (OP == kAddU32) asm volatile(BPU_L8(BPU_ADD) : BPU_X8 : "v"(b));
  else if constexpr (OP == kSubU32) asm volatile(BPU_L8(BPU_SUB) : BPU_X8 : "v"(b));
  else if constexpr (OP == kAndB32) asm volatile(BPU_L8(BPU_AND) : BPU_X8 : "v"(b));
  else if constexpr (OP == kXorB32) asm volatile(BPU_L8(BPU_XOR) : BPU_X8 : "v"(b));
  else if constexpr (OP == kLshrB32) asm volatile(BPU_L8(BPU_LSHR) : BPU_X8 : "v"(b));
  else if constexpr (OP == kAshrI32) asm volatile(BPU_L8(BPU_ASHR) : BPU_X8 : "v"(b));
  else if constexpr (OP == kAdd3U32) asm volatile(BPU_L8(BPU_ADD3) : BPU_X8 : "v"(b));
  else if constexpr (OP == kSadU32) asm volatile(BPU_L8(BPU_SAD) : BPU_X8 : "v"(b));
  else if constexpr (OP == kMulLoU32) asm volatile(BPU_L8(BPU_MULLO) : BPU_X8 : "v"(b));
  else if constexpr (OP == kMulHiU32) asm volatile(BPU_L8(BPU_MULHI) : BPU_X8 : "v"(b));
  else if constexpr (OP == kMaxU32) asm volatile(BPU_L8(BPU_MAX) : BPU_X8 : "v"(b));
  else if constexpr (OP == kBfeI32) asm volatile(BPU_L8(BPU_BFE) : BPU_X8 : "v"(b));
  else if constexpr (OP == kMadU32U24) asm volatile(BPU_L8(BPU_MAD24) : BPU_X8 : "v"(b));
  else if constexpr (OP == kMulU32U24) asm volatile(BPU_L8(BPU_MUL24) : BPU_X8 : "v"(b));
  else if constexpr (OP == kMulHiU32U24) asm volatile(BPU_L8(BPU_MULHI24) : BPU_X8 : "v"(b));
  else if constexpr (OP == kLshlAddU32) asm volatile(BPU_L8(BPU_LSHLADD) : BPU_X8 : "v"(b));
  else if constexpr (OP == kCndmask) asm volatile(BPU_L8(BPU_CND) : BPU_X8 : "v"(b), "s"(m));
  else if constexpr (OP == kAddCoU32) asm volatile(BPU_L8(BPU_ADDCO) : BPU_X8, "=s"(c) : "v"(b));
  else if constexpr (OP == kCmpLtU32) asm volatile(BPU_L8(BPU_CMP) : BPU_X8, "=s"(c) : "v"(b));
}

template <int OP>
__device__ __forceinline__ void row64(uint64_t (&x)[kChains], uint32_t b, const uint32_t (&a)[kChains],
                                      uint64_t &c) {
  asm volatile(BPU_MADROW BPU_MADROW BPU_MADROW BPU_MADROW BPU_MADROW BPU_MADROW BPU_MADROW BPU_MADROW
                   BPU_MADROW BPU_MADROW BPU_MADROW BPU_MADROW BPU_MADROW BPU_MADROW BPU_MADROW BPU_MADROW
               : BPU_X8, "=s"(c)
               : "v"(b), "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(a[4]), "v"(a[5]), "v"(a[6]), "v"(a[7]));
}

template <int OP>
__device__ __forceinline__ void rowf(double (&x)[kChains], double b) {
  if constexpr (OP == kFmaF64) asm volatile(BPU_L8(BPU_FMA) : BPU_X8 : "v"(b));
  else if constexpr (OP == kAddF64) asm volatile(BPU_L8(BPU_ADDF) : BPU_X8 : "v"(b));
  else if constexpr (OP == kMulF64) asm volatile(BPU_L8(BPU_MULF) : BPU_X8 : "v"(b));
}

// v_cvt_f64_u32: eight doubles from eight fixed integers (a throughput test
// with no chain: each result is overwritten by the next row).
__device__ __forceinline__ void rowcvt(double (&x)[kChains], uint32_t b) {
  asm volatile(BPU_L8(BPU_CVT) : BPU_X8 : "v"(b));
}

template <int OP>
__global__ __launch_bounds__(256) void k_rate(uint32_t *out, int iters) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t b = (tid & 7u) | 1u;
  const uint64_t m = 0x5555555555555555ull ^ (uint64_t)blockIdx.x;
  uint64_t c64 = 0;
  uint32_t res = 0;
  if constexpr (OP == kMadU64U32) {
    uint64_t x[kChains];
    uint32_t a[kChains];
    for (int c = 0; c < kChains; ++c) {
      x[c] = tid + c;
      a[c] = tid * 2654435761u + c;
    }
    for (int i = 0; i < iters; ++i)
      row64<OP>(x, b, a, c64);
    for (int c = 0; c < kChains; ++c) res ^= (uint32_t)x[c] ^ (uint32_t)(x[c] >> 32);
  } else if constexpr (OP == kFmaF64 || OP == kAddF64 || OP == kMulF64 || OP == kCvtF64U32) {
    double x[kChains];
    const double bd = 1.0 + 1e-9 * (double)(tid & 15u);
    for (int c = 0; c < kChains; ++c) x[c] = (double)(tid + c) * 1e-3;
    for (int i = 0; i < iters; ++i)
    {
      if constexpr (OP == kCvtF64U32) rowcvt(x, b + (uint32_t)i);
      else rowf<OP>(x, bd);
    }
    for (int c = 0; c < kChains; ++c) res ^= (uint32_t)(int64_t)x[c];
  } else {
    uint32_t x[kChains];
    for (int c = 0; c < kChains; ++c) x[c] = tid * 2654435761u + c;
    for (int i = 0; i < iters; ++i)
      row32<OP>(x, b, m, c64);
    for (int c = 0; c < kChains; ++c) res ^= x[c];
  }
  out[tid] = res ^ (uint32_t)c64 ^ (uint32_t)(c64 >> 32);
}

template <int OP>
hipError_t launch_op(uint32_t *out, int blocks, int iters, hipStream_t s) {
  hipLaunchKernelGGL(k_rate<OP>, dim3(blocks), dim3(256), 0, s, out, iters);
  return hipGetLastError();
}

using Launcher = hipError_t (*)(uint32_t *, int, int, hipStream_t);

template <int... OPS>
struct Table {
  static constexpr Launcher fns[sizeof...(OPS)] = {&launch_op<OPS>...};
};

template <int N, int... OPS>
struct MakeTable : MakeTable<N - 1, N - 1, OPS...> {};
template <int... OPS>
struct MakeTable<0, OPS...> {
  using type = Table<OPS...>;
};

using OpTable = MakeTable<kNumOps>::type;

}  // namespace

extern "C" {

int bpu_num_ops(void) { return kNumOps; }

const char *bpu_op_name(int op) { return (op >= 0 && op < kNumOps) ? kNames[op] : ""; }

// Runs opcode `op` on blocks_per_cu * (CU count) blocks of 4 waves, `iters`
// loop iterations of kChains * kUnroll instructions per lane, `reps` timed
// launches after one warm-up.  *lane_ops_per_s receives the sustained rate
// over the best launch, *ms its duration, *insts_per_lane the instructions
// under test per lane.  Returns 0 or a HIP error code.
int bpu_valu_rate(int device, int op, int blocks_per_cu, int iters, int reps, double *lane_ops_per_s, double *ms,
                  double *insts_per_lane) {
  if (op < 0 || op >= kNumOps || blocks_per_cu < 1 || iters < 1 || reps < 1 || !lane_ops_per_s || !ms)
    return (int)hipErrorInvalidValue;
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return (int)e;
  int cu = 0;
  if ((e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device)) != hipSuccess) return (int)e;
  const int blocks = cu * blocks_per_cu;
  uint32_t *out = nullptr;
  if ((e = hipMalloc(&out, sizeof(uint32_t) * (size_t)blocks * 256)) != hipSuccess) return (int)e;
  hipEvent_t a = nullptr, b = nullptr;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  const Launcher fn = OpTable::fns[op];
  double best = 1e300;
  e = fn(out, blocks, iters, nullptr);
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    (void)hipEventRecord(a, nullptr);
    e = fn(out, blocks, iters, nullptr);
    (void)hipEventRecord(b, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    if (e == hipSuccess && t < best) best = t;
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipFree(out);
  if (e != hipSuccess) return (int)e;
  const double per_lane = (double)iters * kChains * kUnroll;
  *ms = best;
  *lane_ops_per_s = per_lane * (double)blocks * 256.0 / (best * 1e-3);
  if (insts_per_lane) *insts_per_lane = per_lane;
  return 0;
}

}  // extern "C"
