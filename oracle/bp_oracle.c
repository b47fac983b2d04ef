/*
 * bp_oracle.c -- plain, slow CPU oracle for the bin_packing feasibility check.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke entry and the bench's
 * CPU-baseline leg may load this library.  It shares no code, header, table or
 * helper with the HIP library: it is written from the paper's definitions,
 * in exact int64 arithmetic, with no blocking, fusion or reordering beyond what
 * the definitions state.
 *
 * Paper: Tardivo, Michel, Pontelli, "Constraint Propagation on GPU: A Case
 * Study for the Bin Packing Constraint" (arXiv 2402.14821).
 *
 * Numeric range: 1 <= C <= 2^31-1, item sizes in [0, C], r <= 2^24.  The
 * largest intermediate is C*lambda <= 2^62 (VB2) and the largest sum is
 * r * C * 100 < 2^62 (FS1), so int64 is exact throughout.
 *
 * Parity pins: every function here is pinned by tests that do not reuse its
 * arithmetic (hand-worked fixtures, brute-force optimum, dual-feasibility by
 * dynamic programming, closed forms); the list is in the test files.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef int64_t i64;

/* Order of the bound collection, as in the sequential DFF algorithm
 * (Alg. 2 iterates MT, RAD2, FS1, CCM1, VB2, BJ1) preceded by L1 and L2. */
enum { OR_L1 = 0, OR_L2, OR_MT, OR_RAD2, OR_FS1, OR_CCM1, OR_VB2, OR_BJ1, OR_NB };

#define OR_OK 0
#define OR_ERR_ARG -1
#define OR_ERR_RANGE -2
#define OR_ERR_NOMEM -3

#define OR_MAX_C 2147483647LL
#define OR_MAX_R (1LL << 24)

/* ceil(a / b) for a >= 0, b > 0. */
static i64 ceil_div(i64 a, i64 b) { return a / b + (a % b != 0); }

/* ------------------------------------------------------------------------- */
/* Reduction (Sec. 3, "Feasibility check" paragraph, and Fig. 3): the residual
 * instance keeps every unpacked item and adds one virtual item per bin whose
 * size is the load already packed in that bin.  A bin with remaining capacity
 * res has load C - res; an empty bin (load 0) adds nothing, as in Fig. 3,
 * where the fourth, empty bin has no virtual item. */
int oracle_residual_reduce(i64 C, i64 m, const i64 *residual, const i64 *unpacked, i64 n,
                           i64 *out_items, i64 *out_r) {
  if (C < 1 || C > OR_MAX_C || m < 0 || n < 0 || !out_r) return OR_ERR_ARG;
  if ((m > 0 && !residual) || (n > 0 && !unpacked)) return OR_ERR_ARG;
  i64 r = 0;
  for (i64 i = 0; i < n; i++) {
    if (unpacked[i] < 0 || unpacked[i] > C) return OR_ERR_RANGE;
    if (out_items) out_items[r] = unpacked[i];
    r++;
  }
  for (i64 j = 0; j < m; j++) {
    if (residual[j] < 0 || residual[j] > C) return OR_ERR_RANGE;
    i64 load = C - residual[j];
    if (load > 0) {
      if (out_items) out_items[r] = load;
      r++;
    }
  }
  *out_r = r;
  return OR_OK;
}

/* Same reduction from the constraint's own variables (Sec. 3, the CP model
 * bin_packing(X, W, L)): bin_of[i] in [0, m) means item i is packed there,
 * -1 means unpacked.  out_residual (optional) receives C - load_j. */
int oracle_assignment_reduce(i64 C, i64 m, const i64 *size, const i64 *bin_of, i64 n,
                             i64 *out_items, i64 *out_r, i64 *out_residual) {
  if (C < 1 || C > OR_MAX_C || m < 0 || n < 0 || !out_r) return OR_ERR_ARG;
  if (n > 0 && (!size || !bin_of)) return OR_ERR_ARG;
  i64 *load = (i64 *)calloc((size_t)(m > 0 ? m : 1), sizeof(i64));
  if (!load) return OR_ERR_NOMEM;
  i64 r = 0;
  for (i64 i = 0; i < n; i++) {
    if (size[i] < 0 || size[i] > C || bin_of[i] < -1 || bin_of[i] >= m) { free(load); return OR_ERR_RANGE; }
    if (bin_of[i] < 0) {
      if (out_items) out_items[r] = size[i];
      r++;
    } else {
      load[bin_of[i]] += size[i];
      if (load[bin_of[i]] > C) { free(load); return OR_ERR_RANGE; }
    }
  }
  for (i64 j = 0; j < m; j++) {
    if (out_residual) out_residual[j] = C - load[j];
    if (load[j] > 0) {
      if (out_items) out_items[r] = load[j];
      r++;
    }
  }
  free(load);
  *out_r = r;
  return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* L1 (Sec. 3.1, first equation): ceil(sum of sizes / c). */
i64 oracle_l1(i64 C, const i64 *W, i64 r) {
  i64 s = 0;
  for (i64 i = 0; i < r; i++) s += W[i];
  return ceil_div(s, C);
}

/* L2(I, lambda) (Sec. 3.1, Martello-Toth bound): with
 *   W1 = { w : c - lambda < w },
 *   W2 = { w : c/2 < w <= c - lambda },
 *   W3 = { w : lambda <= w <= c/2 },
 * L2(I, lambda) = |W1| + |W2| + max(0, ceil((sum W3 - (c|W2| - sum W2)) / c)).
 * "c/2 < w" and "w <= c/2" are taken as 2w > c and 2w <= c (exact for odd c). */
i64 oracle_l2_at(i64 C, const i64 *W, i64 r, i64 lam) {
  i64 n1 = 0, n2 = 0, s2 = 0, s3 = 0;
  for (i64 i = 0; i < r; i++) {
    i64 w = W[i];
    if (C - lam < w) n1++;
    if (2 * w > C && w <= C - lam) { n2++; s2 += w; }
    if (lam <= w && 2 * w <= C) s3 += w;
  }
  i64 x = s3 - (C * n2 - s2);
  i64 extra = x > 0 ? ceil_div(x, C) : 0; /* max(0, ceil(x / c)) */
  return n1 + n2 + extra;
}

/* L2 = max over integer 0 <= lambda <= c/2, by visiting every lambda. */
i64 oracle_l2_dense(i64 C, const i64 *W, i64 r, i64 *argmax) {
  i64 best = -1, arg = -1;
  for (i64 lam = 0; lam <= C / 2; lam++) {
    i64 v = oracle_l2_at(C, W, r, lam);
    if (v > best) { best = v; arg = lam; }
  }
  if (argmax) *argmax = arg;
  return best;
}

/* ------------------------------------------------------------------------- */
/* The six dual feasible functions of Sec. 3.1, in the paper's integer form.
 * Each takes the capacity C, a size w in [0, C] and the integer parameter. */

/* f_MT (Sec. 3.1, Fig. 4 and the equation below it), 0 <= lambda <= c/2. */
i64 oracle_f_mt(i64 C, i64 w, i64 lam) {
  if (C - lam < w) return C;
  if (lam <= w && w <= C - lam) return w;
  return 0; /* w < lambda */
}

/* f_RAD2, c/4 < lambda <= c/3.  The last case refers back to the function at
 * c - w, which is at most c - 2*lambda and so lands in the first two cases. */
i64 oracle_f_rad2(i64 C, i64 w, i64 lam) {
  if (w < lam) return 0;
  if (lam <= w && w <= C - 2 * lam) return C / 3;
  if (C - 2 * lam < w && w < 2 * lam) return C / 2;
  return C - oracle_f_rad2(C, C - w, lam); /* 2*lambda <= w */
}

/* f_FS1, 1 <= lambda <= 100: w*lambda when w(lambda+1)/c is a natural number,
 * else floor(w(lambda+1)/c) * c. */
i64 oracle_f_fs1(i64 C, i64 w, i64 lam) {
  i64 num = w * (lam + 1);
  if (num % C == 0) return w * lam;
  return (num / C) * C;
}

/* f_CCM1, 1 <= lambda <= c/2. */
i64 oracle_f_ccm1(i64 C, i64 w, i64 lam) {
  if (2 * w > C) return 2 * (C / lam) - 2 * ((C - w) / lam);
  if (2 * w == C) return C / lam;
  return 2 * (w / lam); /* 2w < c */
}

/* max(0, ceil(a / c) - 1), the building block of f_VB2 (a >= 0). */
static i64 vb2_part(i64 a, i64 C) {
  i64 v = ceil_div(a, C) - 1;
  return v > 0 ? v : 0;
}

/* f_VB2, 2 <= lambda <= c; the printed ceil(c*lambda/c) is kept as written. */
i64 oracle_f_vb2(i64 C, i64 w, i64 lam) {
  if (2 * w > C) return 2 * vb2_part(C * lam, C) - 2 * vb2_part(C * lam - w * lam, C);
  if (2 * w == C) return vb2_part(C * lam, C);
  return 2 * vb2_part(w * lam, C); /* 2w < c */
}

/* f_BJ1, 1 <= lambda <= c. */
i64 oracle_f_bj1(i64 C, i64 w, i64 lam) {
  i64 cm = C % lam, wm = w % lam, q = w / lam;
  if (wm <= cm) return q * (lam - cm);
  return q * (lam - cm) + wm - cm;
}

i64 oracle_f(int id, i64 C, i64 w, i64 lam) {
  switch (id) {
    case OR_MT: return oracle_f_mt(C, w, lam);
    case OR_RAD2: return oracle_f_rad2(C, w, lam);
    case OR_FS1: return oracle_f_fs1(C, w, lam);
    case OR_CCM1: return oracle_f_ccm1(C, w, lam);
    case OR_VB2: return oracle_f_vb2(C, w, lam);
    case OR_BJ1: return oracle_f_bj1(C, w, lam);
    default: return -1;
  }
}

/* Parameter range of each function (the subscripts of Sec. 3.1) for integer
 * lambda:  MT [0, floor(c/2)], RAD2 [floor(c/4)+1, floor(c/3)], FS1 [1, 100],
 * CCM1 [1, floor(c/2)], VB2 [2, c], BJ1 [1, c].  An empty range has lo > hi.
 * L2 uses [0, floor(c/2)].  With clamp_vb2 set, the upper end of VB2 is cut to
 * floor(UINT_MAX / (r * max w)) as in Sec. 4, "Implementation details". */
int oracle_default_range(int id, i64 C, i64 r, i64 maxw, int clamp_vb2, i64 *lo, i64 *hi) {
  switch (id) {
    case OR_L1: *lo = 0; *hi = -1; return OR_OK;
    case OR_L2: case OR_MT: *lo = 0; *hi = C / 2; return OR_OK;
    case OR_RAD2: *lo = C / 4 + 1; *hi = C / 3; return OR_OK;
    case OR_FS1: *lo = 1; *hi = 100; return OR_OK;
    case OR_CCM1: *lo = 1; *hi = C / 2; return OR_OK;
    case OR_VB2:
      *lo = 2; *hi = C;
      if (clamp_vb2) {
        i64 denom = r * maxw;
        i64 cap = denom > 0 ? (i64)4294967295LL / denom : C;
        if (cap < *hi) *hi = cap;
      }
      return OR_OK;
    case OR_BJ1: *lo = 1; *hi = C; return OR_OK;
    default: return OR_ERR_ARG;
  }
}

/* The DFF bound over lambda in [lo, hi] (Alg. 2, inner two loops):
 *   L_f = max over lambda of ceil( sum_{w in W_R} f(w, lambda) / f(c, lambda) ),
 * 0 for an empty range.  argmax = smallest lambda attaining L_f, -1 if empty. */
i64 oracle_dff_bound(int id, i64 C, const i64 *W, i64 r, i64 lo, i64 hi, i64 *argmax) {
  i64 best = 0, arg = -1;
  for (i64 lam = lo; lam <= hi; lam++) {
    i64 sum = 0;
    for (i64 i = 0; i < r; i++) sum += oracle_f(id, C, W[i], lam);
    i64 lbp = ceil_div(sum, oracle_f(id, C, C, lam));
    if (arg < 0 || lbp > best) { best = lbp; arg = lam; }
  }
  if (argmax) *argmax = arg;
  return best;
}

/* ------------------------------------------------------------------------- */
/* Piece-start evaluation, for capacities too large to visit every lambda.
 * L2(I, lambda), f_MT and f_RAD2 depend on lambda only through comparisons of
 * each size w with lambda, c - lambda, c - 2*lambda and 2*lambda (and, for
 * RAD2's reflected case, of c - w with lambda); f(c, lambda) is c for MT and
 * RAD2.  Going from lambda - 1 to lambda can change one of those comparisons
 * only at lambda = w + 1, c - w + 1, floor((c - w)/2) + 1 or floor(w/2) + 1.
 * Between such points the per-lambda value is constant, so the maximum over
 * the range equals the maximum over {lo} and those points inside [lo, hi].
 * The per-lambda value is the same definition as above. */
static int cmp_i64(const void *a, const void *b) {
  i64 x = *(const i64 *)a, y = *(const i64 *)b;
  return (x > y) - (x < y);
}

static i64 collect_points(int kind, i64 C, const i64 *W, i64 r, i64 lo, i64 hi, i64 *pts) {
  i64 np = 0;
  pts[np++] = lo;
  for (i64 i = 0; i < r; i++) {
    i64 w = W[i];
    i64 cand[4] = {w + 1, C - w + 1, (C - w) / 2 + 1, w / 2 + 1};
    int nc = kind == OR_RAD2 ? 4 : 2;
    for (int j = 0; j < nc; j++)
      if (cand[j] > lo && cand[j] <= hi) pts[np++] = cand[j];
  }
  qsort(pts, (size_t)np, sizeof(i64), cmp_i64);
  return np;
}

/* kind = OR_L2, OR_MT or OR_RAD2. Returns -1 on allocation failure. */
i64 oracle_piecewise_bound(int kind, i64 C, const i64 *W, i64 r, i64 lo, i64 hi, i64 *argmax) {
  if (lo > hi) { if (argmax) *argmax = -1; return 0; }
  i64 *pts = (i64 *)malloc(sizeof(i64) * (size_t)(4 * r + 1));
  if (!pts) return -1;
  i64 np = collect_points(kind, C, W, r, lo, hi, pts);
  i64 best = -1, arg = -1;
  for (i64 j = 0; j < np; j++) {
    i64 lam = pts[j];
    if (j > 0 && lam == pts[j - 1]) continue;
    i64 v;
    if (kind == OR_L2) {
      v = oracle_l2_at(C, W, r, lam);
    } else {
      i64 sum = 0;
      for (i64 i = 0; i < r; i++) sum += oracle_f(kind, C, W[i], lam);
      v = ceil_div(sum, oracle_f(kind, C, C, lam));
    }
    if (v > best) { best = v; arg = lam; }
  }
  free(pts);
  if (argmax) *argmax = arg;
  return best;
}

/* ------------------------------------------------------------------------- */
/* The whole check (Alg. 1's feasibility check with Alg. 2's bound collection,
 * extended by L1 and L2): every bound, lb = their maximum, FAIL iff lb > k.
 *
 *   lo/hi      per-bound lambda ranges (index OR_L1.. OR_BJ1), or NULL for the
 *              paper's ranges; entries for L1 are ignored.
 *   l2_dense   1: visit every lambda for L2; 0: piece starts (same maximum).
 *   value, argmax: arrays of OR_NB; lb, lb_arg (first bound attaining lb),
 *   verdict (1 = PASS, lb <= k; 0 = FAIL). */
int oracle_bounds(i64 C, i64 k, const i64 *W, i64 r, const i64 *lo, const i64 *hi, int l2_dense,
                  i64 *value, i64 *argmax, i64 *lb, i64 *lb_arg, i64 *verdict) {
  if (C < 1 || C > OR_MAX_C || r < 0 || r > OR_MAX_R || k < 0) return OR_ERR_ARG;
  if (r > 0 && !W) return OR_ERR_ARG;
  for (i64 i = 0; i < r; i++)
    if (W[i] < 0 || W[i] > C) return OR_ERR_RANGE;
  i64 maxw = 0;
  for (i64 i = 0; i < r; i++)
    if (W[i] > maxw) maxw = W[i];
  i64 rlo[OR_NB], rhi[OR_NB];
  for (int b = 0; b < OR_NB; b++) {
    if (lo && hi) { rlo[b] = lo[b]; rhi[b] = hi[b]; }
    else oracle_default_range(b, C, r, maxw, 0, &rlo[b], &rhi[b]);
  }
  value[OR_L1] = oracle_l1(C, W, r);
  argmax[OR_L1] = -1;
  if (rlo[OR_L2] > rhi[OR_L2]) { value[OR_L2] = 0; argmax[OR_L2] = -1; }
  else if (l2_dense) {
    /* dense over the requested range */
    i64 best = -1, arg = -1;
    for (i64 lam = rlo[OR_L2]; lam <= rhi[OR_L2]; lam++) {
      i64 v = oracle_l2_at(C, W, r, lam);
      if (v > best) { best = v; arg = lam; }
    }
    value[OR_L2] = best; argmax[OR_L2] = arg;
  } else {
    value[OR_L2] = oracle_piecewise_bound(OR_L2, C, W, r, rlo[OR_L2], rhi[OR_L2], &argmax[OR_L2]);
    if (value[OR_L2] < 0) return OR_ERR_NOMEM;
  }
  for (int b = OR_MT; b <= OR_BJ1; b++)
    value[b] = oracle_dff_bound(b, C, W, r, rlo[b], rhi[b], &argmax[b]);
  i64 best = -1, barg = 0;
  for (int b = 0; b < OR_NB; b++)
    if (value[b] > best) { best = value[b]; barg = b; }
  *lb = best;
  *lb_arg = barg;
  *verdict = best <= k ? 1 : 0;
  return OR_OK;
}

/* Range-restricted DFF bound for sampling: evaluates lambda = lo, lo+step, ...
 * <= hi and returns the number of (item, lambda) evaluations made in *evals.
 * Used to time the oracle on a bounded slice of a large sweep. */
i64 oracle_dff_bound_strided(int id, i64 C, const i64 *W, i64 r, i64 lo, i64 hi, i64 step,
                             i64 *argmax, i64 *evals) {
  i64 best = 0, arg = -1, ev = 0;
  for (i64 lam = lo; lam <= hi; lam += step) {
    i64 sum = 0;
    for (i64 i = 0; i < r; i++) sum += oracle_f(id, C, W[i], lam);
    ev += r;
    i64 lbp = ceil_div(sum, oracle_f(id, C, C, lam));
    if (arg < 0 || lbp > best) { best = lbp; arg = lam; }
  }
  if (argmax) *argmax = arg;
  if (evals) *evals = ev;
  return best;
}

/* ------------------------------------------------------------------------- */
/* Event sweep of f_CCM1 and f_BJ1 (Sec. 3.1) over [lo, hi], for capacities
 * too large to visit every lambda.  Same result as oracle_dff_bound: the
 * maximum of ceil(sum_w f(w, lambda) / f(c, lambda)) and its smallest
 * maximiser.
 *
 * Both functions read lambda only through Q = floor(c / lambda) and, per size,
 * floor-quotients by lambda.  On a run of lambda with Q fixed:
 *   CCM1  each case of the definition is an integer combination of Q and of
 *         t = floor(v / lambda) with v = w (small item) or v = c - w (big
 *         item); t holds until lambda passes floor(v / t), so the item's value
 *         is constant until floor(v / t) + 1 (for ever once t = 0);
 *   BJ1   writing c mod lambda = c - Q lambda and w mod lambda = w - q lambda
 *         with q = floor(w / lambda), the definition reads
 *           f = q ((Q + 1) lambda - c) + max(0, (w - c) + (Q - q) lambda),
 *         linear in lambda while q holds (until floor(w / q) + 1) and the
 *         max keeps its case; with Q - q >= 0 the second term can only turn
 *         positive as lambda grows, at floor((c - w) / (Q - q)) + 1.
 * f(c, lambda) is the same expression at w = c (2Q for CCM1, Q((Q + 1)
 * lambda - c) >= Q > 0 for BJ1).  Between two consecutive change points of
 * any item the sum and f(c, .) are linear in lambda, the denominator is
 * positive, so their ratio is monotone and so is its ceiling: the stretch's
 * maximum is at one of its ends, and when the ceiling rises along the
 * stretch its smallest maximiser is found by bisection.  Items are visited
 * in the order of their next change point (a binary heap); every item is
 * re-read when Q changes.  Sums are held as A + B lambda in 128-bit integers.
 *
 * Needs 1 <= lo and hi <= c (where both functions are defined).  Returns -1
 * on a bad argument or allocation failure. */
typedef __int128 i128;

#define EV_NEVER INT64_MAX

/* Item w's value on lambda's stretch (Q = floor(c / lambda) fixed):
 * a + b * lambda up to next - 1. */
static void ev_piece(int id, i64 C, i64 w, i64 lam, i64 Q, i128 *a, i128 *b, i64 *next) {
  if (id == OR_CCM1) {
    *b = 0;
    if (2 * w > C) {
      i64 u = C - w, t = u / lam;
      *a = 2 * Q - 2 * t;
      *next = t > 0 ? u / t + 1 : EV_NEVER;
    } else if (2 * w == C) {
      *a = Q;
      *next = EV_NEVER;
    } else {
      i64 t = w / lam;
      *a = 2 * t;
      *next = t > 0 ? w / t + 1 : EV_NEVER;
    }
    return;
  }
  /* BJ1 */
  i64 q = w / lam, d = Q - q;
  int on = (w - C) + d * lam > 0;
  *a = -(i128)q * C + (on ? (w - C) : 0);
  *b = (i128)q * (Q + 1) + (on ? d : 0);
  i64 nq = q > 0 ? w / q + 1 : EV_NEVER;
  i64 nk = (!on && d > 0) ? (C - w) / d + 1 : EV_NEVER;
  *next = nq < nk ? nq : nk;
}

static i64 ev_ceil(i128 s, i128 f) { return (i64)(s / f + (s % f != 0)); }

static void ev_sift(i64 *heap, i64 n, const i64 *key, i64 at) {
  for (;;) {
    i64 l = 2 * at + 1, m = at;
    if (l < n && key[heap[l]] < key[heap[m]]) m = l;
    if (l + 1 < n && key[heap[l + 1]] < key[heap[m]]) m = l + 1;
    if (m == at) return;
    i64 t = heap[at]; heap[at] = heap[m]; heap[m] = t;
    at = m;
  }
}

i64 oracle_event_bound(int id, i64 C, const i64 *W, i64 r, i64 lo, i64 hi, i64 *argmax) {
  if ((id != OR_CCM1 && id != OR_BJ1) || C < 1 || C > OR_MAX_C || r < 0 || (r > 0 && !W)) return -1;
  if (lo > hi) { if (argmax) *argmax = -1; return 0; }
  if (lo < 1 || hi > C) return -1;
  size_t nr = (size_t)(r > 0 ? r : 1);
  i128 *a = (i128 *)malloc(sizeof(i128) * nr), *b = (i128 *)malloc(sizeof(i128) * nr);
  i64 *next = (i64 *)malloc(sizeof(i64) * nr), *heap = (i64 *)malloc(sizeof(i64) * nr);
  if (!a || !b || !next || !heap) { free(a); free(b); free(next); free(heap); return -1; }
  i64 best = 0, arg = -1;
  for (i64 lam = lo; lam <= hi;) {
    i64 Q = C / lam, qend = C / Q;
    if (qend > hi) qend = hi;
    i128 D, E, A = 0, B = 0;
    i64 unused;
    ev_piece(id, C, C, lam, Q, &D, &E, &unused);
    for (i64 i = 0; i < r; i++) {
      ev_piece(id, C, W[i], lam, Q, &a[i], &b[i], &next[i]);
      A += a[i];
      B += b[i];
      heap[i] = i;
    }
    for (i64 i = r / 2 - 1; i >= 0; i--) ev_sift(heap, r, next, i);
    for (i64 cur = lam;;) {
      i64 stop = r > 0 ? next[heap[0]] : EV_NEVER;
      if (stop > qend + 1) stop = qend + 1;
      /* the stretch [cur, stop - 1] */
      i64 x = cur, y = stop - 1;
      i64 gx = ev_ceil(A + B * x, D + E * x), gy = ev_ceil(A + B * y, D + E * y), m, at;
      if (gx >= gy) {
        m = gx;
        at = x;
      } else {
        m = gy;
        i64 l2 = x + 1, h2 = y;
        while (l2 < h2) {
          i64 mid = l2 + (h2 - l2) / 2;
          if (ev_ceil(A + B * mid, D + E * mid) >= m) h2 = mid;
          else l2 = mid + 1;
        }
        at = l2;
      }
      if (arg < 0 || m > best) { best = m; arg = at; }
      if (stop > qend) break;
      while (next[heap[0]] == stop) {
        i64 i = heap[0];
        A -= a[i];
        B -= b[i];
        ev_piece(id, C, W[i], stop, Q, &a[i], &b[i], &next[i]);
        A += a[i];
        B += b[i];
        ev_sift(heap, r, next, 0);
      }
      cur = stop;
    }
    lam = qend + 1;
  }
  free(a); free(b); free(next); free(heap);
  if (argmax) *argmax = arg;
  return best;
}
