"""Served checks: continuous batching through bp_queue_* on the GPU.

A request's result must be the same whether it runs alone (bp_feasible) or
inside a mix of overlapping batches; the admission limits and the injected
launch failure are forced from the host."""
import sys
import time

import numpy as np
import pytest

import oracle as O
import oracle_par
import paper_2402_14821_amd as bp
from paper_2402_14821_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = bp.Context(0)
    yield c
    c.close()


def drain(q, n, deadline_s=60.0):
    out = {}
    t0 = time.time()
    while len(out) < n:
        assert time.time() - t0 < deadline_s, f"only {len(out)} of {n} results"
        for r in q.poll(256, timeout_us=20000):
            out[r.ticket] = r
    return out


def fields(b):
    return (list(b.value), list(b.argmax_lambda), b.lb, b.lb_arg, b.verdict, b.r, b.status)


def test_alone_equals_in_mix(ctx):
    reqs = W.dfs_requests(3, rate=20000, duration=1.0, max_requests=80)
    say("queue mix of", len(reqs))
    q = bp.Queue(ctx, 8 << 30, 4096)
    tickets = {}
    for i, r in enumerate(reqs):
        tickets[q.submit(r.C, r.residual, r.unpacked, tag=i, flags=bp.BP_NO_EARLY_EXIT)] = i
    res = drain(q, len(reqs))
    st = q.stats()
    q.close()
    assert st["completed"] == len(reqs) and st["batches"] >= 1
    for t, r in res.items():
        i = tickets[t]
        assert r.tag == i and r.status == 0
        alone = ctx.feasible(reqs[i].C, reqs[i].residual, reqs[i].unpacked, flags=bp.BP_NO_EARLY_EXIT)
        assert fields(r.bounds) == (list(alone["value"]), list(alone["argmax"]), alone["lb"], alone["lb_arg"],
                                    alone["verdict"], alone["r"], 0), i
        assert r.submit_us <= r.start_us <= r.done_us
    # the oracle on the smallest few
    small = sorted(range(len(reqs)), key=lambda i: len(reqs[i].unpacked))[:2]
    for i in small:
        items = O.residual_reduce(reqs[i].C, reqs[i].residual, reqs[i].unpacked)
        want = O.bounds(reqs[i].C, len(reqs[i].residual), items)
        got = [r for r in res.values() if r.tag == i][0].bounds
        assert list(got.value) == want["value"].tolist() and got.verdict == want["verdict"]


def test_early_exit_verdicts_in_mix(ctx):
    reqs = W.dfs_requests(4, rate=200000, duration=1.0, max_requests=60)
    say("queue early exit", len(reqs))
    q = bp.Queue(ctx, 8 << 30, 4096)
    tickets = {q.submit(r.C, r.residual, r.unpacked, tag=i): i for i, r in enumerate(reqs)}
    res = drain(q, len(reqs))
    q.close()
    for t, r in res.items():
        i = tickets[t]
        full = ctx.feasible(reqs[i].C, reqs[i].residual, reqs[i].unpacked, flags=bp.BP_NO_EARLY_EXIT)
        assert r.verdict == full["verdict"]
        if r.verdict == 1:
            assert r.lb == full["lb"]
        else:
            assert r.lb > len(reqs[i].residual)


def _tight_twin(r):
    """The same node with empty bins dropped until ceil(total / C) - 1 bins
    remain (or only the loaded ones): a node the check must refute."""
    total = int(np.sum(r.unpacked, dtype=np.int64)) + int(np.sum(r.C - r.residual.astype(np.int64)))
    want_m = max(int((r.residual < r.C).sum()), -(-total // r.C) - 1)
    keep = list(np.flatnonzero(r.residual < r.C))
    empty = list(np.flatnonzero(r.residual == r.C))
    keep += empty[: max(0, want_m - len(keep))]
    return W.Request(r.t, r.C, r.residual[sorted(keep)].copy(), r.unpacked.copy(), r.node)


def test_served_requests_match_oracle(ctx):
    # 48 requests of the simulated search, 24 from each arrival-rate stream,
    # and their tightened twins, served in one mix twice over: exhaustive
    # (every field against the oracle) and with early exit (verdict against
    # the oracle; a passing request's whole record, a failing one's lb above
    # its bin count)
    picks = []
    for seed, rate in ((3, 20_000.0), (4, 200_000.0)):
        reqs = W.dfs_requests(seed, rate=rate, duration=1.0, max_requests=600)
        idx = np.linspace(0, len(reqs) - 1, 24).astype(int)
        picks += [reqs[i] for i in idx]
    picks += [_tight_twin(r) for r in picks]
    items = [O.residual_reduce(r.C, r.residual, r.unpacked) for r in picks]
    want = O.bounds_many([(r.C, len(r.residual), it) for r, it in zip(picks, items)],
                         threads=oracle_par.pool_threads(), l2_dense=True)
    say("served mix vs oracle,", len(picks), "requests x 2")
    q = bp.Queue(ctx, 8 << 30, 4096)
    tickets = {}
    for i, r in enumerate(picks):
        tickets[q.submit(r.C, r.residual, r.unpacked, tag=2 * i, flags=bp.BP_NO_EARLY_EXIT)] = (i, False)
        tickets[q.submit(r.C, r.residual, r.unpacked, tag=2 * i + 1)] = (i, True)
    res = drain(q, len(tickets))
    q.close()
    refuted_early = 0
    for t, got in res.items():
        i, early = tickets[t]
        w, m = want[i], len(picks[i].residual)
        assert got.status == 0 and got.bounds.r == len(items[i])
        assert got.verdict == w["verdict"], (i, early)
        if not early or w["verdict"] == 1:
            assert list(got.bounds.value) == w["value"].tolist(), (i, early)
            assert list(got.bounds.argmax_lambda) == w["argmax"].tolist(), (i, early)
            assert (got.lb, got.bounds.lb_arg) == (w["lb"], w["lb_arg"]), (i, early)
        else:
            assert got.lb > m, (i, got.lb, m)
            refuted_early += got.bounds.early_exit
    verdicts = [w["verdict"] for w in want]
    assert 0 < sum(verdicts) < len(verdicts)  # both kinds of nodes
    assert refuted_early == len(verdicts) - sum(verdicts)


def submit_stream(q, reqs, root_flags=bp.BP_NO_EARLY_EXIT, child_flags=bp.BP_NO_EARLY_EXIT, with_instance=False,
                  wave=None, results=None):
    """Roots as partial packings, children as (parent ticket, commits); with
    `wave`, the results of each wave of that many requests are drained into
    `results` before the next wave goes in."""
    tickets, by_ticket = {}, {}
    for i, r in enumerate(reqs):
        if wave and i and i % wave == 0:
            results.update(drain(q, wave))
        if r.parent < 0 or r.parent not in tickets:
            t = q.submit(r.C, r.residual, r.unpacked, tag=i, flags=root_flags)
        else:
            kw = dict(residual=r.residual, unpacked=r.unpacked) if with_instance else {}
            t = q.submit_child(r.C, len(r.residual), tickets[r.parent], r.commits, tag=i, flags=child_flags, **kw)
        tickets[i] = t
        by_ticket[t] = i
    return tickets, by_ticket


def check_against_full_path(ctx, reqs, res, by_ticket, what):
    for t, got in res.items():
        i = by_ticket[t]
        r = reqs[i]
        assert got.status == 0, (what, i, got.status)
        alone = ctx.feasible(r.C, r.residual, r.unpacked, flags=bp.BP_NO_EARLY_EXIT)
        assert fields(got.bounds) == (list(alone["value"]), list(alone["argmax"]), alone["lb"], alone["lb_arg"],
                                      alone["verdict"], alone["r"], 0), (what, i, got.from_parent)
        assert got.bounds.evals == alone["evals"]


def test_child_requests_from_parent_sums(ctx):
    # children submitted as (parent ticket, commits) without their instances:
    # every record equals the full check of the node, and the oracle's on a sample
    for seed, rate in ((3, 20_000.0), (4, 200_000.0)):
        reqs = W.dfs_requests(seed, rate=rate, duration=1.0, max_requests=240)
        say("served children from parent sums, seed", seed)
        q = bp.Queue(ctx, 8 << 30, 4096)
        tickets, by_ticket = submit_stream(q, reqs)
        res = drain(q, len(reqs))
        st = q.stats()
        q.close()
        assert st["from_parent"] > len(reqs) // 2, st
        assert st["from_parent"] + st["full_sweeps"] == len(reqs)
        check_against_full_path(ctx, reqs, res, by_ticket, ("seed", seed))
        by_index = {by_ticket[t]: g for t, g in res.items()}
        # the oracle on every 10th request
        idx = list(range(0, len(reqs), 10))
        want = O.bounds_many([(reqs[i].C, len(reqs[i].residual), O.residual_reduce(reqs[i].C, reqs[i].residual,
                                                                                   reqs[i].unpacked)) for i in idx],
                             threads=oracle_par.pool_threads(), l2_dense=True)
        for i, w in zip(idx, want):
            got = by_index[i]
            assert list(got.bounds.value) == w["value"].tolist(), i
            assert list(got.bounds.argmax_lambda) == w["argmax"].tolist(), i
            assert (got.lb, got.bounds.lb_arg, got.verdict) == (w["lb"], w["lb_arg"], w["verdict"]), i
        # a child computed from sums did O(P) work per changed item
        kids = [g for g in res.values() if g.from_parent]
        assert kids and all(0 <= g.bounds.evals_done < g.bounds.evals for g in kids)


def test_child_requests_with_evictions_and_early_exit_roots(ctx):
    # a 16 MiB budget keeps a few dozen node states (C = 10 000): evicted
    # ancestors send children to the full sweeps on instances rebuilt from
    # the commits; roots with early exit are bases only once they finished
    reqs = W.dfs_requests(3, rate=200_000.0, duration=1.0, max_requests=320)
    for root_flags in (bp.BP_NO_EARLY_EXIT, 0):
        say("served children, small budget, root flags", root_flags)
        q = bp.Queue(ctx, 16 << 20, 4096)
        res = {}
        tickets, by_ticket = submit_stream(q, reqs, root_flags=root_flags, wave=40, results=res)
        res.update(drain(q, len(reqs) - len(res)))
        st = q.stats()
        q.close()
        assert st["node_evictions"] > 0 and st["from_parent"] > 0, st
        assert st["completed"] == len(reqs) == len(res)
        check_against_full_path(ctx, reqs, res, by_ticket, ("small budget", root_flags))


def test_child_request_errors(ctx):
    C, m, res, unp = W.small_partial_packing(seed=3)
    q = bp.Queue(ctx, 64 << 20, 64)
    say("served child errors")
    root = q.submit(C, res, unp, flags=bp.BP_NO_EARLY_EXIT)
    w = int(unp[0])
    fits = [j for j in range(m) if res[j] >= w]
    with pytest.raises(bp.BpError) as e:
        q.submit_child(C, m, 10**12, [(w, fits[0])])
    assert e.value.status == bp.BP_ERR_STATE
    with pytest.raises(bp.BpError) as e:
        q.submit_child(C, m, root, [(w, m)])
    assert e.value.status == bp.BP_ERR_RANGE
    full = [j for j in range(m) if res[j] < w]
    if full:
        with pytest.raises(bp.BpError) as e:
            q.submit_child(C, m, root, [(w, full[0])])
        assert e.value.status == bp.BP_ERR_RANGE
    with pytest.raises(bp.BpError) as e:
        q.submit_child(C, m + 1, root, [(w, fits[0])])
    assert e.value.status == bp.BP_ERR_ARG
    kid = q.submit_child(C, m, root, [(w, fits[0])], flags=bp.BP_NO_EARLY_EXIT)
    out = drain(q, 2)
    q.close()
    res2 = res.copy()
    res2[fits[0]] -= w
    unp2 = list(unp)
    unp2.remove(w)
    want = O.bounds(C, m, O.residual_reduce(C, res2, unp2), l2_dense=True)
    assert list(out[kid].bounds.value) == want["value"].tolist()
    assert list(out[kid].bounds.argmax_lambda) == want["argmax"].tolist()


def test_open_loop_replay(ctx):
    # bp_queue_replay submits at the arrival times from native code, children
    # through their parents' tickets; every record equals the node's full check
    import ctypes
    reqs = W.dfs_requests(4, rate=50_000.0, duration=1.0, max_requests=300)
    say("open-loop replay of", len(reqs))
    keep, structs = [], []
    for i, r in enumerate(reqs):
        if r.parent < 0:
            res = np.ascontiguousarray(r.residual, dtype=np.int32)
            unp = np.ascontiguousarray(r.unpacked, dtype=np.int32)
            keep.append((res, unp))
            structs.append(bp.bp_request(r.C, len(res), len(unp), res.ctypes.data_as(bp._P32),
                                         unp.ctypes.data_as(bp._P32), i, bp.BP_NO_EARLY_EXIT, 0, 0, None, 0, 0))
        else:
            cm = (bp.bp_commit * max(1, len(r.commits)))(*[bp.bp_commit(w, b) for w, b in r.commits])
            keep.append(cm)
            structs.append(bp.bp_request(r.C, len(r.residual), 0, None, None, i, bp.BP_NO_EARLY_EXIT, 0, 0, cm,
                                         len(r.commits), 0))
    n = len(reqs)
    arr = (bp.bp_request * n)(*structs)
    arrival = np.ascontiguousarray([r.t for r in reqs], dtype=np.float64)
    parent = np.ascontiguousarray([r.parent for r in reqs], dtype=np.int64)
    tickets = np.zeros(n, dtype=np.uint64)
    status = np.zeros(n, dtype=np.int32)
    late = ctypes.c_double(0)
    q = bp.Queue(ctx, 8 << 30, 4096)
    lib = bp.load()
    st = lib.bp_queue_replay(q.handle, ctypes.cast(arr, ctypes.c_void_p), arrival.ctypes.data_as(ctypes.c_void_p),
                             parent.ctypes.data_as(ctypes.c_void_p), n, tickets.ctypes.data_as(ctypes.c_void_p),
                             status.ctypes.data_as(ctypes.c_void_p), ctypes.byref(late))
    assert st == 0 and (status == 0).all() and (tickets > 0).all()
    res = drain(q, n)
    stats = q.stats()
    q.close()
    assert stats["from_parent"] > n // 2
    by_ticket = {int(t): i for i, t in enumerate(tickets)}
    check_against_full_path(ctx, reqs, res, by_ticket, "replay")


def test_admission_limits(ctx):
    C, m, res, unp = W.large_residual(1)
    with pytest.raises(bp.BpError) as e:
        bp.Queue(ctx, 1000, 4)  # below the 1 MiB minimum
    assert e.value.status == bp.BP_ERR_ARG
    q = bp.Queue(ctx, 4 << 20, 4)
    say("request larger than the budget's admission share")
    with pytest.raises(bp.BpError) as e:
        q.submit(C, res, unp)
    assert e.value.status == bp.BP_ERR_LIMIT
    q.close()
    q = bp.Queue(ctx, 1 << 30, 1)
    t1 = q.submit(C, res, unp, flags=bp.BP_NO_EARLY_EXIT)
    rejected = 0
    t2 = None
    t0 = time.time()
    while t2 is None:
        t2 = q.try_submit(150, [10, 20], [100, 50])
        if t2 is None:
            rejected += 1
            time.sleep(0.0002)
        assert time.time() - t0 < 30
    out = drain(q, 2)
    assert q.stats()["rejected"] == rejected
    q.close()
    assert out[t1].status == 0 and out[t2].status == 0
    alone = ctx.feasible(150, [10, 20], [100, 50], flags=bp.BP_NO_EARLY_EXIT)
    assert out[t2].lb == alone["lb"]


def test_injected_launch_failure(ctx, monkeypatch):
    monkeypatch.setenv("BP_TEST_FAIL_LAUNCH", "1")
    q = bp.Queue(ctx, 1 << 30, 64)
    monkeypatch.delenv("BP_TEST_FAIL_LAUNCH")
    say("injected failure")
    t1 = q.submit(150, [10], [100, 60])
    r1 = drain(q, 1)[t1]
    assert r1.status == bp.BP_ERR_DEVICE
    t2 = q.submit(150, [10], [100, 60], flags=bp.BP_NO_EARLY_EXIT)
    r2 = drain(q, 1)[t2]
    q.close()
    assert r2.status == 0
    assert r2.lb == ctx.feasible(150, [10], [100, 60], flags=bp.BP_NO_EARLY_EXIT)["lb"]


def test_destroy_while_busy(ctx):
    C, m, res, unp = W.large_residual(2)
    q = bp.Queue(ctx, 1 << 30, 64)
    for i in range(6):
        q.submit(C, res, unp, tag=i)
    say("destroy while busy")
    q.close()  # must finish or drain without hanging
