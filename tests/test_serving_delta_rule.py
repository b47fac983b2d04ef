"""CPU pins of the change rule behind incremental serving.

A node of the search reached by committing items (Sec. 5) has a reduced
instance (Sec. 3, Fig. 3) that differs from its parent's by: each committed
size leaving the unpacked items, and its bin's virtual item changing from
the bin's old load to the new one (none for a load of 0).  The served
queue computes a child from that change; here the rule is checked against
the oracle's reduction of the two explicit instances, and the simulated
search's requests against their parents."""
import collections
import random

import numpy as np

import oracle as O
from paper_2402_14821_amd import workloads as W


def changed_items(C, residual, commits):
    """(removed, added) reduced sizes when (size, bin) commits are applied in order."""
    load = [C - int(x) for x in residual]
    rem, add = [], []
    for w, j in commits:
        old = load[j]
        rem.append(w)
        if old > 0:
            rem.append(old)
        if old + w > 0:
            add.append(old + w)
        load[j] = old + w
    return rem, add


def test_change_rule_matches_the_reductions():
    rng = random.Random(31)
    for t in range(400):
        C = rng.randint(1, 60)
        m = rng.randint(1, 6)
        load = [0] * m
        for j in range(m):
            if rng.random() < 0.5:
                load[j] = rng.randint(0, C)
        unp = [rng.randint(0, C) for _ in range(rng.randint(0, 10))]
        residual = [C - x for x in load]
        # commit up to three unpacked items where they fit (a bin may take several)
        commits, left, cur = [], list(unp), list(load)
        for _ in range(rng.randint(0, 3)):
            if not left:
                break
            w = left[rng.randrange(len(left))]
            fits = [j for j in range(m) if cur[j] + w <= C]
            if not fits:
                break
            j = rng.choice(fits)
            commits.append((w, j))
            left.remove(w)
            cur[j] += w
        child_res = [C - x for x in cur]
        parent_items = collections.Counter(O.residual_reduce(C, residual, unp).tolist())
        child_items = collections.Counter(O.residual_reduce(C, child_res, left).tolist())
        rem, add = changed_items(C, residual, commits)
        # signed counts: a bin taking two items gains a virtual item that the second commit removes again
        got = collections.Counter(parent_items)
        got.subtract(collections.Counter(rem))
        got.update(collections.Counter(add))
        assert min(got.values(), default=0) >= 0, (C, load, unp, commits)
        assert +got == +child_items, (C, load, unp, commits)
        # every bound is a function of the multiset: equal records
        k = m
        a = O.bounds(C, k, list(child_items.elements()))
        b = O.bounds(C, k, list(got.elements()))
        assert np.array_equal(a["value"], b["value"])


def test_simulated_search_children_follow_their_parents():
    for seed in (3, 4):
        reqs = W.dfs_requests(seed, rate=200_000.0, duration=1.0, max_requests=400)
        kinds = collections.Counter()
        for i, r in enumerate(reqs):
            assert r.parent < i
            if r.parent < 0:
                kinds["root"] += 1
                continue
            p = reqs[r.parent]
            res = p.residual.astype(np.int64).copy()
            unp = list(p.unpacked.tolist())
            for w, j in r.commits:
                assert res[j] >= w
                res[j] -= w
                unp.remove(w)
            assert np.array_equal(res, r.residual) and sorted(unp) == sorted(r.unpacked.tolist())
            kinds["child" if r.commits else "revisit"] += 1
        assert kinds["root"] > 0 and kinds["child"] > 0 and kinds["revisit"] > 0
