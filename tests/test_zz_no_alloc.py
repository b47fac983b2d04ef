"""The allocation-free check (bp_feasible_dev_noalloc) through the C ABI.

Its records must equal those of bp_feasible_dev (the context-owning entry
point it varies) field by field, and the oracle's, on two calls in a row
that share the static workspace, the second on a smaller instance; then the
same pair again with early exit, and the size limit."""
import sys

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


def record(t):
    return bp.bounds_to_dict(np.frombuffer(t.cpu().numpy().tobytes(), dtype=bp.BOUNDS_DTYPE)[0])


def same(got, want, what):
    assert got["status"] == 0, (what, got)
    for f in ("value", "argmax"):
        assert np.array_equal(got[f], want[f]), (what, f, got[f], want[f])
    for f in ("lb", "lb_arg", "verdict"):
        assert got[f] == want[f], (what, f, got[f], want[f])


def test_noalloc_equals_feasible_dev_on_two_calls():
    torch = pytest.importorskip("torch")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    C1, m1, res1, unp1, items1, want1 = oracle_par.large_residual_record(1)
    C2, m2, res2, unp2 = W.small_partial_packing(seed=7)
    items2 = O.residual_reduce(C2, res2, unp2)
    want2 = O.bounds(C2, m2, items2, l2_dense=True)
    cases = [("large residual instance", C1, m1, res1, unp1, want1),
             ("small partial packing", C2, m2, res2, unp2, want2)]
    with bp.Context(0) as ctx:
        for flags in (bp.BP_NO_EARLY_EXIT, 0):
            for name, C, m, res, unp, want in cases:
                say("noalloc", name, "flags", flags)
                d_res = torch.from_numpy(np.ascontiguousarray(res, dtype=np.int32)).to(dev)
                d_unp = torch.from_numpy(np.ascontiguousarray(unp, dtype=np.int32)).to(dev)
                out_ref = torch.zeros(bp.BOUNDS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
                out_na = torch.full((bp.BOUNDS_DTYPE.itemsize,), 0xAB, dtype=torch.uint8, device=dev)
                ctx.feasible_dev(C, m, d_res.data_ptr(), len(unp), d_unp.data_ptr(), out_ref.data_ptr(), stream,
                                 flags=flags)
                bp.feasible_dev_noalloc(C, m, d_res.data_ptr(), len(unp), d_unp.data_ptr(), out_na.data_ptr(),
                                        stream, flags=flags)
                torch.cuda.synchronize()
                ref, got = record(out_ref), record(out_na)
                assert bytes(out_na.cpu().numpy()) == bytes(out_ref.cpu().numpy()), (name, flags, got, ref)
                assert got["r"] == ref["r"] and got["evals"] == ref["evals"] and got["k"] == m
                if flags == bp.BP_NO_EARLY_EXIT or want["verdict"] == 1:
                    same(got, want, (name, flags))
                else:
                    assert got["verdict"] == 0 and got["lb"] > m


def test_noalloc_rejects_oversized_and_bad_flags():
    torch = pytest.importorskip("torch")
    dev = torch.device("cuda:0")
    d = torch.zeros(bp.BP_NOALLOC_MAX_ITEMS + 1, dtype=torch.int32, device=dev)
    out = torch.zeros(bp.BOUNDS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    say("noalloc limits")
    with pytest.raises(bp.BpError) as e:
        bp.feasible_dev_noalloc(100, 1, d.data_ptr(), bp.BP_NOALLOC_MAX_ITEMS, d.data_ptr(), out.data_ptr(), 0)
    assert e.value.status == bp.BP_ERR_LIMIT
    with pytest.raises(bp.BpError) as e:
        bp.feasible_dev_noalloc(100, 1, d.data_ptr(), 4, d.data_ptr(), out.data_ptr(), 0, flags=bp.BP_SEGMENTS)
    assert e.value.status == bp.BP_ERR_ARG
