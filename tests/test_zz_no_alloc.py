"""pperm_run_batch_noalloc: the batched epoch step with the launch entries in
the library's own scratch array.  Through the C ABI it must give exactly the
bits of pperm_run_batch (its caller-workspace twin) on the same problems, call
after call, including a second call with fewer problems than the first (the
scratch keeps the first call's entries; nothing of them may leak)."""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _make(mix):
    from paper_2002_03000_amd import ParallelFlatPERM
    return [ParallelFlatPERM(p.dim, p.n_max, p.n_sequences, p.seed, stream_id=p.stream) for p in mix]


def _epoch_state(g):
    import torch
    torch.cuda.synchronize()
    n1 = g.n_max + 1
    rec = g.records("L")[:, :n1]
    return (rec["m"].copy(), rec["e"].copy(), rec["h"].copy(),
            g.view("m").cpu().numpy().view(np.uint32).copy(),
            g.view("t").cpu().numpy().view(np.uint64).copy(),
            g.sequence_stats())


def _pooled_state(g):
    import torch
    torch.cuda.synchronize()
    n1 = g.n_max + 1
    rec = g.records("G")[:n1]
    return (rec["m"].copy(), rec["e"].copy(), g.view("HG").cpu().numpy().view(np.uint64)[:n1].copy(),
            g.view("MG").cpu().numpy().view(np.uint64).copy())


def _assert_same(a, b, label):
    for k, (x, y) in enumerate(zip(a, b)):
        if x.dtype.names:
            for f in x.dtype.names:
                assert np.array_equal(x[f], y[f]), f"{label}: field {k}.{f}"
        else:
            assert np.array_equal(x, y), f"{label}: field {k}"


def test_noalloc_batch_matches_workspace_batch_two_calls():
    from paper_2002_03000_amd import Batch, run_batch_noalloc
    mix = workloads.batched_mix()[:10]          # 2D and 3D, n_max 64..2048, N 64..1024
    ref, dut = _make(mix), _make(mix)
    b = Batch(len(mix))
    # first call: every problem; second call: the first four only (smaller input)
    calls = [(list(range(len(mix))), 0), (list(range(4)), 1)]
    for c, (which, epoch) in enumerate(calls):
        tours = [mix[i].schedule()[epoch] for i in which]
        b.run_tours([ref[i] for i in which], tours)
        run_batch_noalloc([dut[i] for i in which], tours)
        for i in which:
            _assert_same(_epoch_state(ref[i]), _epoch_state(dut[i]), f"call {c} problem {i} epoch sums")
            ref[i].merge_epoch()
            dut[i].merge_epoch()
            _assert_same(_pooled_state(ref[i]), _pooled_state(dut[i]), f"call {c} problem {i} pooled")
        print(f"no-alloc call {c}: {len(which)} problems bit-identical to the workspace batch", flush=True)
    # estimates through the same calls agree bit for bit
    for i in range(4):
        a, ha, ta = ref[i].estimates()
        d, hd, td = dut[i].estimates()
        assert np.array_equal(a.view(np.uint64), d.view(np.uint64)) and np.array_equal(ha, hd) and ta == td


def test_noalloc_batch_rejects_more_problems_than_its_scratch():
    from paper_2002_03000_amd import _abi
    lib = _abi.load()
    count = _abi.NOALLOC_MAX_PROBLEMS + 1
    ctxs = (ctypes.c_void_p * count)()
    tours = (ctypes.c_uint32 * count)(*([1] * count))
    assert lib.pperm_run_batch_noalloc(ctxs, count, tours, None) == -1      # PPERM_EINVAL
