// bp_divide.h -- exact integer division by multiplication, for the sweep kernels.
//
// Each form is exact for every input the kernels feed it (proofs inline; the
// host self-test bp_selftest_division checks them against '/').
//
// (1) Division by a per-lane parameter d (1 <= d < 2^31) of a numerator
//     n < 2^31.  Granlund & Montgomery, "Division by invariant integers using
//     multiplication" (PLDI 1994), Theorem 4.2 with N = 31: with
//     s = ceil(log2 d) and m = ceil(2^(31+s) / d), the product satisfies
//     2^(31+s) <= m d < 2^(31+s) + d <= 2^(31+s) + 2^s, hence
//     floor(n / d) = floor(m n / 2^(31+s)) for 0 <= n < 2^31.  Feeding 2n
//     (< 2^32) to a 32x32 high multiply gives floor(m 2n / 2^32) >> s =
//     floor(m n / 2^(31+s)).  m < 2^32 for every d < 2^31 (m = 2^31 when d is a
//     power of two).  Cost: one v_mul_hi_u32 and one shift.
//
// (2) ceil(a * lam / c) - 1 for 1 <= a < 2^31, 1 <= lam <= c < 2^31 (the
//     building block of f_VB2).  With the 64-bit per-lane constant
//     R = ceil(lam 2^64 / c) - 1 we have lam 2^64 / c - 1 <= R < lam 2^64 / c,
//     so v = a R / 2^64 lies in [a lam / c - 2^-33, a lam / c).  If a lam / c
//     is an integer q, floor(v) = q - 1; otherwise its fraction is at least
//     1/c > 2^-31 > 2^-33 and floor(v) = floor(a lam / c).  Both equal
//     ceil(a lam / c) - 1.  floor(a R / 2^64) is the high word of
//     a * R_hi + mulhi(a, R_lo) (no overflow: < 2^63 + 2^32).  Cost: one
//     v_mul_hi_u32 and one v_mad_u64_u32.
//
// (3) Divisibility of n < 2^32 by d, 1 <= d < 2^31 (Lemire, Kaser, Kurz,
//     "Faster remainder by direct computation", 2019).  With M = ceil(2^64 / d)
//     = (2^64 + e) / d, 0 <= e < d, and n = q d + t (0 <= t < d), n M =
//     q 2^64 + q e + t M, so n M mod 2^64 = q e + t M as long as that is below
//     2^64.  If t = 0 it is q e < (2^32 / d) d = 2^32 <= M; if t >= 1 it is at
//     least M and below 2^32 + (d - 1)(2^64 / d + 1) < 2^64 (d < 2^31).  Hence
//     d | n iff n M mod 2^64 <= M - 1.  For d = 1, M wraps to 0 and the test
//     reads n 0 <= 2^64 - 1, true.  Cost: a 64-bit product by a 32-bit value
//     and a 64-bit compare.
//
// (5) Short forms of (1) and (2) for small products, one v_mul_hi_u32 each.
//     (a) floor(n / d) for 2 <= d < 2^31 and n d <= 2^32: with
//         m = ceil(2^32 / d) = (2^32 + e) / d, 0 <= e < d (m <= 2^31), and
//         n = q d + t (0 <= t < d), n m / 2^32 = q + (t + n e / 2^32) / d;
//         n e < n d <= 2^32 keeps t + n e / 2^32 below t + 1 <= d, so
//         floor(n m / 2^32) = q.  m = floor((2^32 - 1) / d) + 1 (equal to
//         ceil(2^32 / d) whether or not d divides 2^32).
//     (b) ceil(a lam / c) - 1 for 1 <= a, 1 <= lam <= c and a c <= 2^32,
//         from R_hi, the high word of (2)'s R: R_hi = floor((lam 2^32 - 1) / c)
//         (no multiple of c lies strictly between lam 2^32 - 1 and
//         lam 2^32 - 2^-32), so lam 2^32 / c - 1 <= R_hi < lam 2^32 / c and
//         v = a R_hi / 2^32 lies in [a lam / c - a / 2^32, a lam / c).  If
//         a lam / c is an integer q, floor(v) = q - 1 (a / 2^32 <= 1);
//         otherwise its fraction is at least 1/c >= a / 2^32 and floor(v) =
//         floor(a lam / c).  Both equal ceil(a lam / c) - 1.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace bpi {

struct MagicU31 {
  uint32_t m;
  uint32_t s;
};

__host__ __device__ inline uint32_t ceil_log2_u32(uint32_t d) {
#if defined(__HIP_DEVICE_COMPILE__)
  return d <= 1 ? 0u : 32u - (uint32_t)__clz((int)(d - 1));
#else
  return d <= 1 ? 0u : 32u - (uint32_t)__builtin_clz(d - 1);
#endif
}

// Constants of family (1) for divisor d in [1, 2^31).
__host__ __device__ inline MagicU31 magic_u31(uint32_t d) {
  uint32_t s = ceil_log2_u32(d);
  uint64_t num = 1ull << (31 + s);
  uint64_t m = (num + d - 1) / d;
  return {(uint32_t)m, s};
}

// floor(n / d) given n2 = 2n (n < 2^31).
__host__ __device__ inline uint32_t div_u31(uint32_t n2, uint32_t m, uint32_t s) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umulhi(n2, m) >> s;
#else
  return (uint32_t)(((uint64_t)n2 * m) >> 32) >> s;
#endif
}

// Constant of family (2): ceil(lam 2^64 / c) - 1 for 1 <= lam <= c < 2^31.
__host__ __device__ inline uint64_t vb2_recip(uint32_t lam, uint32_t c) {
  if (lam >= c) return ~0ull;  // lam = c: 2^64 - 1
  uint64_t x = (uint64_t)lam << 32;  // < 2^63
  uint64_t q1 = x / c, r1 = x % c;   // q1 < 2^32 because lam < c
  uint64_t y = r1 << 32;             // r1 < c < 2^31
  uint64_t q2 = y / c, r2 = y % c;   // q2 < 2^32
  uint64_t fl = (q1 << 32) | q2;     // floor(lam 2^64 / c), >= 1
  return r2 ? fl : fl - 1;
}

// ceil(a lam / c) - 1 for 1 <= a < 2^31 from R = vb2_recip(lam, c).
__host__ __device__ inline uint32_t vb2_part(uint32_t a, uint32_t r_lo, uint32_t r_hi) {
#if defined(__HIP_DEVICE_COMPILE__)
  uint32_t t = __umulhi(a, r_lo);
#else
  uint32_t t = (uint32_t)(((uint64_t)a * r_lo) >> 32);
#endif
  uint64_t s = (uint64_t)a * r_hi + t;
  return (uint32_t)(s >> 32);
}

// (4) Floors through an fp64 reciprocal, for per-lane divisors with no
//     precomputed constant.  For 0 <= n < 2^31 and 1 <= d < 2^31 the product
//     n * fl(1/d) (two roundings, relative error below 2^-52) is within
//     2^31 * 2^-52 < 1 of n / d, so its truncation is floor(n / d) or one
//     off, and the exact integer remainder n - q d moves it back.  The 62-bit
//     form takes N < c^2 (N = a lambda - 1 with a, lambda <= c < 2^31): the
//     quotient is below 2^31, N's own rounding to 53 bits and the two others
//     keep the estimate within 2^31 * 3 2^-53 < 1, and one step of the
//     correction loops suffices.
__host__ __device__ inline uint32_t fdiv_u31(uint32_t n, uint32_t d, double rd) {
  uint32_t q = (uint32_t)((double)n * rd);
  const int64_t r = (int64_t)n - (int64_t)q * d;
  if (r < 0) --q;
  else if (r >= (int64_t)d) ++q;
  return q;
}

__host__ __device__ inline int64_t fdiv_u62(int64_t N, int64_t c, double rc) {
  int64_t q = (int64_t)((double)N * rc);
  int64_t r = N - q * c;
  while (r < 0) { --q; r += c; }
  while (r >= c) { ++q; r -= c; }
  return q;
}

// Constant of family (5a) for 2 <= d < 2^31: ceil(2^32 / d); 0 for d = 1
// (which (5a) does not cover).
__host__ __device__ inline uint32_t magic_short(uint32_t d) { return d >= 2 ? 0xffffffffu / d + 1u : 0u; }

// floor(n / d) from m = magic_short(d), for n d <= 2^32 (family (5a)).
__host__ __device__ inline uint32_t div_short(uint32_t n, uint32_t m) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umulhi(n, m);
#else
  return (uint32_t)(((uint64_t)n * m) >> 32);
#endif
}

// ceil(a lam / c) - 1 from the high word of vb2_recip(lam, c), for a >= 1
// and a c <= 2^32 (family (5b)).
__host__ __device__ inline uint32_t vb2_part_short(uint32_t a, uint32_t r_hi) { return div_short(a, r_hi); }

// Constant of family (3) for divisor d in [1, 2^31): ceil(2^64 / d) mod 2^64.
__host__ __device__ inline uint64_t divides_const(uint32_t d) { return ~0ull / d + 1ull; }

// d | n from M = divides_const(d).
__host__ __device__ inline bool divides_u32(uint32_t n, uint64_t M) { return (uint64_t)n * M <= M - 1ull; }

}  // namespace bpi
