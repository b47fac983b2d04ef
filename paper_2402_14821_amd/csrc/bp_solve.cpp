// bp_solve.cpp -- the propagator around the feasibility check and the search
// that drives it (Sec. 3 Alg. 1, Sec. 5 resolution procedure).
//
// Decision version: pack n items into k bins of capacity c.  The resolution
// procedure (Sec. 5) starts k at the root's lower bound and increases it
// until an attempt finds a packing.  An attempt is a depth-first search with
// decreasing best fit: the largest unpacked item goes to the bin of its
// domain with the smallest residual capacity that holds it (left branch),
// or leaves that bin's domain (right branch).  On the right branch the two
// symmetry-breaking rules of Sec. 5 apply: the bin leaves the domain of
// every unpacked item of the same size, and so does every bin with the same
// load.  Before branching, two dominance rules (Sec. 5) pack an item that
// fills a bin exactly, and the heaviest item that fits a bin into which no
// two items fit together.
//
// Propagation at every node follows Alg. 1 with load variables [lmin, lmax]
// per bin, restated from the rule descriptions that come with Alg. 1:
//   - load coherence: a bin holds at least the total weight minus what the
//     other bins can hold at most, and at most the total minus what they
//     hold at least;
//   - basic load tightening: a bin's load lies between its packed weight and
//     its packed weight plus every item that may still go there;
//   - basic item elimination and commitment: an item leaves a bin it would
//     overfill, and goes to a bin that cannot reach its minimum load without
//     it (or to the only bin left in its domain);
//   - knapsack reasoning (bin packability, load tightening, item elimination
//     and commitment) with an approximate subset-sum test, subset_sum_gap
//     below;
// repeated to a fixpoint, then the feasibility check: the lower bound of the
// reduced instance (Fig. 3) against k.  The check is the library's (the DFF
// bound collection, or L1 and L2 only) or a caller's function.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>
#include <vector>

#include "bp_ctx.h"
#include "bp_internal.h"

using namespace bpi;

namespace {

constexpr int64_t kInf = INT64_MAX / 4;

// The sizes a subset-sum test runs over: x[0..n) sorted by decreasing size
// with prefix sums from both ends, optionally without the item at index t
// (the knapsack item rules ask about every candidate but one).
struct SumView {
  const int32_t *x = nullptr;
  int32_t n = 0;
  const int64_t *asc = nullptr;   // asc[m]: the m smallest sizes
  const int64_t *desc = nullptr;  // desc[q]: the q largest sizes
  int32_t t = -1;                 // the item left out, or -1

  int32_t size() const { return t < 0 ? n : n - 1; }
  int64_t smallest(int32_t m) const {
    if (t < 0 || m <= n - 1 - t) return asc[m];
    return asc[m + 1] - x[t];
  }
  int64_t largest(int32_t q) const {
    if (t < 0 || q <= t) return desc[q];
    return desc[q + 1] - x[t];
  }
};

void prefix_sums(const int32_t *x, int32_t n, std::vector<int64_t> &asc, std::vector<int64_t> &desc) {
  asc.assign((size_t)n + 1, 0);
  desc.assign((size_t)n + 1, 0);
  for (int32_t q = 0; q < n; ++q) {
    asc[(size_t)q + 1] = asc[(size_t)q] + x[n - 1 - q];
    desc[(size_t)q + 1] = desc[(size_t)q] + x[q];
  }
}

// The approximate subset-sum test of the knapsack reasoning.  Returns true
// when it proves that no subset of the view's sizes sums into [alpha, beta];
// then every subset sum is <= *below or >= *above.  false: no proof (a sum
// may or may not exist).
//
// The argument: take the q largest sizes (sum G_q) and the largest set L of
// smallest sizes with G_q + sum(L) < alpha.  A subset with at most q items
// outside L sums to at most G_q + sum(L); one with q + 1 or more items
// outside L sums to at least the q + 1 smallest sizes outside L.  When that
// second figure exceeds beta for some q, no subset sums into [alpha, beta].
// Every q that proves it gives a gap containing [alpha, beta]; the gaps
// overlap, so their union is reported.  Cost: O(Q log n) for the Q values of
// q with G_q < alpha.
bool subset_sum_gap(const SumView &v, int64_t alpha, int64_t beta, int64_t *below, int64_t *above) {
  if (alpha > beta || beta < 0 || alpha <= 0) return false;  // (the empty set sums to 0)
  const int32_t n = v.size();
  const int64_t tot = v.smallest(n);
  if (alpha > tot) {
    *below = tot;
    *above = kInf;
    return true;
  }
  bool found = false;
  int64_t lo = kInf, hi = -1;
  int32_t kp = 0, top = n;  // |L|: the largest m with G_q + smallest(m) < alpha
  while (kp < top) {
    const int32_t mid = kp + (top - kp + 1) / 2;
    if (v.smallest(mid) < alpha) kp = mid;
    else top = mid - 1;
  }
  for (int32_t q = 0; q <= n; ++q) {
    const int64_t G = v.largest(q);
    if (G >= alpha) break;
    while (kp > 0 && G + v.smallest(kp) >= alpha) --kp;  // shrinks as G grows
    // alpha <= tot makes q + 1 items outside L exist (else every sum < alpha)
    const int64_t B = (kp + q + 1 <= n) ? v.smallest(kp + q + 1) - v.smallest(kp) : kInf;
    if (B > beta) {
      found = true;
      lo = std::min(lo, G + v.smallest(kp));
      hi = std::max(hi, B);
    }
  }
  if (found) {
    *below = lo;
    *above = hi;
  }
  return found;
}

struct Limits {
  int64_t max_nodes = 0;  // per attempt, 0 = none
  double deadline = 0;    // seconds since the start, 0 = none
};

struct State {
  std::vector<int64_t> load;        // packed weight per bin
  std::vector<int64_t> lmin, lmax;  // bounds on the bin's final load
  std::vector<int32_t> bin_of;      // per item (sorted order), -1 unpacked
  std::vector<uint64_t> dom;        // per item, k bits
};

struct Solver {
  bp_ctx *ctx = nullptr;
  int32_t C = 0, n = 0, k = 0, words = 0;
  int64_t total = 0;              // weight of all items
  std::vector<int32_t> w;         // sizes, decreasing
  const bp_solve_opts *opt = nullptr;
  bp_solve_result *res = nullptr;
  std::chrono::steady_clock::time_point t0;
  Limits lim;
  int64_t attempt_nodes = 0;
  bool stopped = false;
  std::vector<int32_t> best;      // a packing found (sorted order)
  bp_status err = BP_OK;
  std::vector<int32_t> res_buf, unp_buf, red_buf;
  std::vector<int32_t> cand, cand_w;  // scratch of the knapsack pass
  std::vector<int64_t> asc, desc;
  std::vector<int32_t> last_w, verdicts;  // the item rules' answers for the last bin
  int64_t last_a = 0, last_b = 0;
  bool last_valid = false;

  double elapsed() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  bool rule(uint32_t off_flag) const { return !(opt->disable & off_flag); }

  bool has(const State &s, int32_t i, int32_t j) const {
    return (s.dom[(size_t)i * words + (j >> 6)] >> (j & 63)) & 1ull;
  }
  void drop(State &s, int32_t i, int32_t j) const { s.dom[(size_t)i * words + (j >> 6)] &= ~(1ull << (j & 63)); }

  int32_t dom_count(const State &s, int32_t i, int32_t *only) const {
    int32_t cnt = 0;
    for (int32_t t = 0; t < words; ++t) {
      const uint64_t x = s.dom[(size_t)i * words + t];
      if (x && only) *only = t * 64 + __builtin_ctzll(x);
      cnt += __builtin_popcountll(x);
    }
    return cnt;
  }

  void pack(State &s, int32_t i, int32_t j) const {
    s.bin_of[(size_t)i] = j;
    s.load[(size_t)j] += w[(size_t)i];
  }

  // Removes bin j from item i's domain and packs i when one bin is left.
  // false: the domain is empty.
  bool eliminate(State &s, int32_t i, int32_t j) const {
    drop(s, i, j);
    int32_t only = -1;
    const int32_t cnt = dom_count(s, i, &only);
    if (cnt == 0) return false;
    if (cnt == 1) pack(s, i, only);
    return true;
  }

  // The lower bound of the node's reduced instance (Fig. 3): 1 = feasible
  // (lb <= k), 0 = refuted, -1 = error (err set).
  int check(const State &s, int64_t *lb_out) {
    res_buf.resize((size_t)k);
    unp_buf.clear();
    for (int32_t j = 0; j < k; ++j) res_buf[(size_t)j] = (int32_t)(C - s.load[(size_t)j]);
    for (int32_t i = 0; i < n; ++i)
      if (s.bin_of[(size_t)i] < 0) unp_buf.push_back(w[(size_t)i]);
    const auto tc = std::chrono::steady_clock::now();
    int64_t lb = 0;
    bp_status st;
    if (opt->check) {
      st = opt->check(opt->user, C, k, res_buf.data(), unp_buf.data(), (int64_t)unp_buf.size(), &lb);
      if (st) st = fail(st, "the caller's check returned %d", st);
    } else if (opt->mode == BP_SOLVE_L2) {
      // L1 and L2 only: every DFF range empty
      red_buf = unp_buf;
      for (int32_t j = 0; j < k; ++j)
        if (s.load[(size_t)j] > 0) red_buf.push_back((int32_t)s.load[(size_t)j]);
      bp_sweep sw;
      st = bp_default_sweep(C, 0, 0, 0, &sw);
      for (int b = BP_MT; b < BP_NB && st == BP_OK; ++b) {
        sw.lo[b] = 1;
        sw.hi[b] = 0;
      }
      bp_bounds o;
      if (!st) st = bp_lower_bounds(ctx, C, k, red_buf.data(), (int64_t)red_buf.size(), &sw, &o);
      lb = o.lb;
    } else {
      int32_t verdict = 0;
      st = bp_feasible(ctx, C, k, res_buf.data(), unp_buf.data(), (int64_t)unp_buf.size(), opt->check_flags,
                       &verdict, &lb, nullptr);
    }
    res->check_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - tc).count();
    ++res->checks;
    if (st) {
      err = st;
      return -1;
    }
    if (lb_out) *lb_out = lb;
    if (lb > k) {
      ++res->check_fails;
      return 0;
    }
    return 1;
  }

  // One pass of the basic rules over every bin.  false: the node fails.
  bool basic_pass(State &s, bool *changed) {
    int64_t sum_lo = 0, sum_hi = 0;
    for (int32_t j = 0; j < k; ++j) {
      sum_lo += s.lmin[(size_t)j];
      sum_hi += s.lmax[(size_t)j];
    }
    for (int32_t j = 0; j < k; ++j) {
      int64_t cand_sum = 0;
      for (int32_t i = 0; i < n; ++i)
        if (s.bin_of[(size_t)i] < 0 && has(s, i, j)) cand_sum += w[(size_t)i];
      int64_t &lo = s.lmin[(size_t)j], &hi = s.lmax[(size_t)j];
      const int64_t p = s.load[(size_t)j];
      const int64_t nlo = std::max({lo, p, total - (sum_hi - hi)});
      const int64_t nhi = std::min({hi, p + cand_sum, total - (sum_lo - lo)});
      if (nlo > nhi) return false;
      if (nlo != lo || nhi != hi) {
        sum_lo += nlo - lo;
        sum_hi += nhi - hi;
        lo = nlo;
        hi = nhi;
        *changed = true;
      }
      // p + cand_sum stays an upper bound on what the bin can reach while
      // candidates move into it or leave it
      for (int32_t i = 0; i < n; ++i) {
        if (s.bin_of[(size_t)i] >= 0 || !has(s, i, j)) continue;
        if (s.load[(size_t)j] + w[(size_t)i] > hi) {
          if (!eliminate(s, i, j)) return false;
          *changed = true;
        } else if (p + cand_sum - w[(size_t)i] < lo) {
          pack(s, i, j);
          *changed = true;
        }
      }
      if (s.load[(size_t)j] > hi) return false;
    }
    return true;
  }

  // One pass of the knapsack rules over every bin: bin packability and load
  // tightening, and with items set, item elimination and commitment.  Each
  // bin reads the state as it is when its turn comes.  The item rules of a
  // bin all run on the candidates and packed weight it started with: items
  // that leave the bin meanwhile only add subsets, and an item committed to
  // it lies in every subset that counts, so a gap proved on that view holds
  // in the new state too.  false: the node fails.
  bool knapsack_pass(State &s, bool items, bool *changed) {
    last_valid = false;
    for (int32_t j = 0; j < k; ++j) {
      cand.clear();
      cand_w.clear();
      for (int32_t i = 0; i < n; ++i)
        if (s.bin_of[(size_t)i] < 0 && has(s, i, j)) {
          cand.push_back(i);
          cand_w.push_back(w[(size_t)i]);
        }
      const int32_t nc = (int32_t)cand.size();
      const int64_t p = s.load[(size_t)j];
      const int64_t a = s.lmin[(size_t)j] - p, b = s.lmax[(size_t)j] - p;
      prefix_sums(cand_w.data(), nc, asc, desc);
      SumView view{cand_w.data(), nc, asc.data(), desc.data(), -1};
      int64_t below, above;
      // bin packability
      if (subset_sum_gap(view, a, b, &below, &above)) return false;
      // load tightening
      if (subset_sum_gap(view, a, a, &below, &above)) {
        s.lmin[(size_t)j] = p + above;
        *changed = true;
      }
      if (subset_sum_gap(view, b, b, &below, &above)) {
        s.lmax[(size_t)j] = p + below;
        *changed = true;
      }
      if (s.lmin[(size_t)j] > s.lmax[(size_t)j]) return false;
      if (s.lmin[(size_t)j] != p + a || s.lmax[(size_t)j] != p + b) continue;
      if (!items || a <= 0) continue;  // elimination and commitment need a positive minimum
      // item elimination and commitment, once per distinct size (items of one
      // size get the same answer).  The answers depend on a, b and the
      // candidates' sizes only; bins in a row often share them (empty bins
      // differ only by index), so the previous bin's answers are reused.
      const bool same = last_valid && a == last_a && b == last_b && cand_w == last_w;
      if (!same) {
        verdicts.clear();
        for (int32_t t = 0; t < nc; ++t) {
          const int32_t v = cand_w[(size_t)t];
          if (t > 0 && cand_w[(size_t)t - 1] == v) continue;
          SumView rest = view;
          rest.t = t;
          if (v < a && subset_sum_gap(rest, a - v, b - v, &below, &above)) verdicts.push_back(v);
          else if (subset_sum_gap(rest, a, b, &below, &above)) verdicts.push_back(-v);
        }
        last_valid = true;
        last_a = a;
        last_b = b;
        last_w = cand_w;
      }
      // a positive entry v: items of size v leave the bin; -v: they go there
      for (int32_t verdict : verdicts) {
        const int32_t v = verdict > 0 ? verdict : -verdict;
        for (int32_t u = 0; u < nc; ++u) {
          const int32_t i = cand[(size_t)u];
          if (cand_w[(size_t)u] != v || s.bin_of[(size_t)i] >= 0) continue;
          if (verdict > 0) {
            if (!eliminate(s, i, j)) return false;
          } else {
            pack(s, i, j);
          }
          *changed = true;
        }
      }
    }
    return true;
  }

  // Alg. 1: the filtering rules to a fixpoint, then the feasibility check.
  // false: the node fails (or the search stops).
  bool propagate(State &s) {
    for (;;) {
      bool changed = false;
      if (!basic_pass(s, &changed)) return filter_failed();
      if (changed) continue;
      if (!rule(BP_SOLVE_OFF_KNAPSACK)) break;
      // the item rules, the dearest, run once the bin-level rules are quiet
      if (!knapsack_pass(s, false, &changed)) return filter_failed();
      if (changed) continue;
      if (!knapsack_pass(s, true, &changed)) return filter_failed();
      if (!changed) break;
    }
    if (opt->mode == BP_SOLVE_NO_CHECK && !opt->check) return true;
    const int r = check(s, nullptr);
    if (r < 0) stopped = true;
    return r == 1;
  }
  bool filter_failed() {
    ++res->filter_fails;
    return false;
  }

  bool out_of_limits() {
    if (lim.max_nodes && attempt_nodes >= lim.max_nodes) return true;
    if (lim.deadline > 0 && (attempt_nodes & 63) == 0 && elapsed() > lim.deadline) return true;
    return false;
  }

  // A move that a dominance rule forces: the node's only child.
  bool forced(const State &s, int32_t i, int32_t j) {
    State t = s;
    pack(t, i, j);
    if (propagate(t) && dfs(t)) return true;
    if (!stopped) ++res->fails;
    return false;
  }

  bool dfs(State &s) {
    if (stopped) return false;
    if (out_of_limits()) {
      stopped = true;
      res->limit_reached = 1;
      return false;
    }
    ++attempt_nodes;
    ++res->nodes;
    int32_t i = 0;
    while (i < n && s.bin_of[(size_t)i] >= 0) ++i;
    if (i == n) {
      best = s.bin_of;
      return true;
    }
    const int32_t wi = w[(size_t)i];
    // dominance: a bin the item fills exactly
    if (rule(BP_SOLVE_OFF_FILL))
      for (int32_t j = 0; j < k; ++j)
        if (has(s, i, j) && s.load[(size_t)j] + wi == C) return forced(s, i, j);
    // dominance: a bin into which no two of its candidates fit together takes
    // the heaviest one that fits
    if (rule(BP_SOLVE_OFF_SINGLE))
      for (int32_t j = 0; j < k; ++j) {
        const int64_t room = C - s.load[(size_t)j];
        int32_t heavy = -1, s1 = -1, s2 = -1;  // s1, s2: the two smallest that fit, w[s1] >= w[s2]
        for (int32_t u = 0; u < n; ++u) {
          if (s.bin_of[(size_t)u] >= 0 || !has(s, u, j) || w[(size_t)u] > room) continue;
          if (heavy < 0) heavy = u;
          s1 = s2;
          s2 = u;
        }
        if (heavy >= 0 && (s1 < 0 || (int64_t)w[(size_t)s1] + w[(size_t)s2] > room)) return forced(s, heavy, j);
      }
    // decreasing best fit: the bin of the domain with the smallest residual that holds the item
    int32_t jb = -1;
    for (int32_t j = 0; j < k; ++j)
      if (has(s, i, j) && s.load[(size_t)j] + wi <= s.lmax[(size_t)j] &&
          (jb < 0 || s.load[(size_t)j] > s.load[(size_t)jb]))
        jb = j;
    if (jb < 0) {
      ++res->fails;
      return false;
    }
    {
      State t = s;
      pack(t, i, jb);
      if (propagate(t) && dfs(t)) return true;
      if (stopped) return false;
    }
    // the item stays out of jb; symmetry: jb and every bin with its load leave
    // the domains of the unpacked items of the same size
    State t = s;
    const int64_t lj = s.load[(size_t)jb];
    bool ok = eliminate(t, i, jb);
    if (rule(BP_SOLVE_OFF_SYMMETRY))
      for (int32_t i2 = i; ok && i2 < n && w[(size_t)i2] == wi; ++i2)  // sizes are sorted decreasing
        for (int32_t j = 0; ok && j < k; ++j)
          if (t.bin_of[(size_t)i2] < 0 && has(t, i2, j) && s.load[(size_t)j] == lj) ok = eliminate(t, i2, j);
    if (!ok) ++res->filter_fails;
    if (ok && propagate(t) && dfs(t)) return true;
    if (!stopped) ++res->fails;
    return false;
  }

  // One attempt with k bins: 1 found, 0 none exists, -1 stopped.
  int attempt(int32_t kk) {
    k = kk;
    words = (k + 63) / 64;
    State s;
    s.load.assign((size_t)k, 0);
    s.lmin.assign((size_t)k, 0);
    s.lmax.assign((size_t)k, C);
    s.bin_of.assign((size_t)n, -1);
    s.dom.assign((size_t)n * words, 0);
    for (int32_t i = 0; i < n; ++i)
      for (int32_t j = 0; j < k; ++j) s.dom[(size_t)i * words + (j >> 6)] |= 1ull << (j & 63);
    attempt_nodes = 0;
    stopped = false;
    if (!propagate(s)) return stopped ? -1 : 0;
    if (dfs(s)) return 1;
    return stopped ? -1 : 0;
  }
};

// First fit decreasing: a packing, so an upper bound on the optimum.
int32_t first_fit_decreasing(const std::vector<int32_t> &w, int32_t C, std::vector<int32_t> *bin_of) {
  std::vector<int64_t> load;
  bin_of->assign(w.size(), -1);
  for (size_t i = 0; i < w.size(); ++i) {
    size_t j = 0;
    while (j < load.size() && load[j] + w[i] > C) ++j;
    if (j == load.size()) load.push_back(0);
    load[j] += w[i];
    (*bin_of)[i] = (int32_t)j;
  }
  return (int32_t)load.size();
}

}  // namespace

int32_t bp_subset_sum_gap(const int32_t *x, int32_t n, int64_t alpha, int64_t beta, int64_t *below,
                          int64_t *above) {
  if (n < 0 || (n > 0 && !x) || !below || !above) return fail(BP_ERR_ARG, "NULL argument or n < 0");
  for (int32_t i = 0; i < n; ++i)
    if (x[i] < 0 || (i > 0 && x[i] > x[i - 1])) return fail(BP_ERR_ARG, "sizes must be >= 0 and non-increasing");
  std::vector<int64_t> asc, desc;
  prefix_sums(x, n, asc, desc);
  return subset_sum_gap(SumView{x, n, asc.data(), desc.data(), -1}, alpha, beta, below, above) ? 1 : 0;
}

bp_status bp_solve(bp_ctx *ctx, int32_t C, int64_t n, const int32_t *sizes, const bp_solve_opts *opts,
                   int32_t *bin_of, bp_solve_result *out) {
  if (!opts || !out || (n > 0 && !sizes)) return fail(BP_ERR_ARG, "NULL argument");
  if (C < 1 || n < 0) return fail(BP_ERR_ARG, "bad capacity or count");
  if (n > kLargeCap) return fail(BP_ERR_LIMIT, "%lld items > %d", (long long)n, kLargeCap);
  if (!opts->check && opts->mode != BP_SOLVE_NO_CHECK && !ctx)
    return fail(BP_ERR_ARG, "the library's check needs a context");
  if (opts->mode != BP_SOLVE_DFFS && opts->mode != BP_SOLVE_L2 && opts->mode != BP_SOLVE_NO_CHECK)
    return fail(BP_ERR_ARG, "unknown mode %d", opts->mode);
  bp_status st = host_validate_items(C, sizes, n);
  if (st) return st;
  memset(out, 0, sizeof *out);
  Solver sv;
  sv.ctx = ctx;
  sv.C = C;
  sv.n = (int32_t)n;
  sv.opt = opts;
  sv.res = out;
  sv.t0 = std::chrono::steady_clock::now();
  sv.lim.max_nodes = opts->max_nodes;
  sv.lim.deadline = opts->time_limit_s;
  std::vector<int32_t> order((size_t)n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return sizes[a] > sizes[b]; });
  sv.w.resize((size_t)n);
  for (int64_t i = 0; i < n; ++i) sv.w[(size_t)i] = sizes[order[(size_t)i]];
  for (int32_t x : sv.w) sv.total += x;
  std::vector<int32_t> ffd;
  const int32_t ub = first_fit_decreasing(sv.w, C, &ffd);
  // the root's lower bound: every item unpacked, as many empty bins as first fit decreasing uses
  int32_t lower = 0;
  {
    State s;
    sv.k = std::max(ub, 1);
    s.load.assign((size_t)sv.k, 0);
    s.bin_of.assign((size_t)n, -1);
    int64_t lb = 0;
    if (opts->check || opts->mode != BP_SOLVE_NO_CHECK) {
      if (sv.check(s, &lb) < 0) return sv.err;
    } else {
      lb = (sv.total + C - 1) / C;  // L1
    }
    lower = (int32_t)std::max<int64_t>(lb, n > 0 ? 1 : 0);
  }
  out->lower = lower;
  out->upper = ub;
  std::vector<int32_t> sol = ffd;
  int32_t bins = ub;
  out->status = BP_SOLVE_OPTIMAL;
  for (int32_t k = lower; k < ub; ++k) {
    const int r = sv.attempt(k);
    if (sv.err) return sv.err;
    ++out->attempts;
    if (r == 1) {
      sol = sv.best;
      bins = k;
      break;
    }
    if (r < 0) {
      out->status = BP_SOLVE_LIMIT;
      break;
    }
  }
  out->bins = bins;
  out->seconds = sv.elapsed();
  if (bin_of)
    for (int64_t i = 0; i < n; ++i) bin_of[order[(size_t)i]] = sol[(size_t)i];
  return BP_OK;
}
