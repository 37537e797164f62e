"""Observables through the ratio estimator of eqn (5): <R^2_n>.

The device keeps, beside every weight sum, the sum of W * R^2 over the same
samples and merges it through the same pairwise tree.  Every per-sequence and
pooled record must equal the oracle's bit for bit, and the ratio read through
the C-ABI must equal the oracle's ratio."""
import ctypes

import numpy as np
import pytest

import oracle
from parity_util import MODE_CODES, assert_epoch_equal, assert_pooled_equal

pytestmark = pytest.mark.gpu


def _pair(dim, n_max, N, seed, mode="shared", **kw):
    from paper_2002_03000_amd import ParallelFlatPERM
    g = ParallelFlatPERM(dim, n_max, N, seed, mode=mode, observables=True, **kw)
    o = oracle.Oracle(dim, n_max, N, seed, mode=MODE_CODES[mode], observables=True)
    return g, o


def _assert_records(rec, ref, label):
    for f in ("m", "e"):
        if not np.array_equal(rec[f], ref[f]):
            idx = np.argwhere(rec[f] != ref[f])[:5]
            raise AssertionError(f"{label}.{f} differs at {idx.tolist()}")


def _assert_ratio(a, b):
    nan = np.isnan(b)
    assert np.array_equal(np.isnan(a), nan)
    assert np.array_equal(a[~nan].view(np.uint64), b[~nan].view(np.uint64))


@pytest.mark.parametrize("dim,n_max,N,seed,mode", [
    (2, 60, 100, 11, "shared"),       # two merge passes, ragged last chunk
    (3, 45, 130, 12, "shared"),       # three 64-row chunks
    (2, 40, 1, 13, "shared"),         # a single sequence
    (3, 30, 70, 14, "rosenbluth"),    # no prune/enrich: plain Rosenbluth weights
])
def test_r2_sums_match_oracle_every_epoch(dim, n_max, N, seed, mode):
    g, o = _pair(dim, n_max, N, seed, mode)
    n1 = n_max + 1
    for T in (1, 1, 2, 4):
        g.run_tours(T)
        o.run_tours(T)
        assert_epoch_equal(g, o, label="observable epoch")
        _assert_records(g.records("obs_L")[:, :n1], o.LR, "LR")
        g.merge_epoch()
        o.merge_epoch()
        assert_pooled_equal(g, o, "observable merge")
        _assert_records(g.records("obs_G")[:n1], o.GR, "GR")
        assert not g.records("obs_L")["m"].any()
        _assert_ratio(g.observable_r2(), o.observable_r2())
    r2 = g.observable_r2()
    assert r2[0] == 0.0 and r2[1] == 1.0


def test_observables_leave_the_walks_unchanged():
    from paper_2002_03000_amd import ParallelFlatPERM
    a = ParallelFlatPERM(3, 80, 96, 21, observables=True)
    b = ParallelFlatPERM(3, 80, 96, 21)
    for T in (1, 1, 2):
        for g in (a, b):
            g.run_tours(T)
            g.merge_epoch()
    la, ha, ma = a.estimates()
    lb, hb, mb = b.estimates()
    assert np.array_equal(la.view(np.uint64), lb.view(np.uint64)) and np.array_equal(ha, hb) and ma == mb
    sa, sb = a.sequence_stats(), b.sequence_stats()
    assert all(np.array_equal(sa[f], sb[f]) for f in sa.dtype.names)


def test_r2_at_long_lengths_matches_oracle():
    # a 2D problem at n_max = 1000 (deep copy stacks, records beyond the LDS
    # part of the stack), compared on every length
    g, o = _pair(2, 1000, 192, 31)
    for T in (1, 1, 2):
        g.run_tours(T)
        o.run_tours(T)
        g.merge_epoch()
        o.merge_epoch()
    assert_pooled_equal(g, o, "long observable merge")
    _assert_records(g.records("obs_G")[:1001], o.GR, "GR")
    _assert_ratio(g.observable_r2(), o.observable_r2())


def test_epoch_graph_replays_carry_the_observable():
    g, o = _pair(2, 50, 80, 41)
    g.run_tours(1)
    o.run_tours(1)
    g.merge_epoch()
    o.merge_epoch()
    graph = g.epoch_graph(2)
    for _ in range(3):
        graph.launch()
        g.sync()
        o.run_tours(2)
        o.merge_epoch()
        _assert_records(g.records("obs_G")[:51], o.GR, "GR")
        _assert_ratio(g.observable_r2(), o.observable_r2())


def test_observable_contexts_stay_out_of_batches_and_jobs():
    from paper_2002_03000_amd import ParallelFlatPERM, _abi
    import torch
    lib = _abi.load()
    g = ParallelFlatPERM(2, 30, 8, 51, observables=True)
    plain = ParallelFlatPERM(2, 30, 8, 52)
    ctxs = (ctypes.c_void_p * 2)(g._ctx, plain._ctx)
    tours = (ctypes.c_uint32 * 2)(1, 1)
    need = ctypes.c_size_t()
    _abi.check(lib.pperm_batch_workspace_bytes(2, ctypes.byref(need)), "batch bytes")
    ws = torch.empty(need.value + 256, dtype=torch.uint8, device="cuda")
    rc = lib.pperm_run_batch(ctxs, 2, tours, ctypes.c_void_p(ws.data_ptr()), need.value, None)
    assert rc == -1
    # without the flag the estimator is refused
    out = np.zeros(31)
    assert lib.pperm_observable_r2(plain._ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 31) == -1
    # before any merge: call out of order
    rc = lib.pperm_observable_r2(g._ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 31)
    assert rc == -4                       # PPERM_ESTATE
