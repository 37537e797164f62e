"""Checkpoint between epochs and resume.

A run stopped after a merge and resumed from its checkpoint in a fresh
context (with the same or another launch shape) continues bit for bit as the
uninterrupted run and as the oracle; a checkpoint is refused by a context of
another problem and while tours are unmerged."""
import ctypes

import numpy as np
import pytest

import oracle
from parity_util import MODE_CODES, assert_pooled_equal, gpu_pooled_state

pytestmark = pytest.mark.gpu


def _same_state(a, b, label):
    ra, ha, ma = gpu_pooled_state(a)
    rb, hb, mb = gpu_pooled_state(b)
    for name, x, y in (("G.m", ra["m"], rb["m"]), ("G.e", ra["e"], rb["e"]), ("HG", ha, hb), ("MG", ma, mb)):
        assert np.array_equal(x, y), f"{label}: {name} differs"
    sa, sb = a.sequence_stats(), b.sequence_stats()
    for f in sa.dtype.names:
        assert np.array_equal(sa[f], sb[f]), f"{label}: stats {f} differ"


@pytest.mark.parametrize("dim,n_max,N,seed,mode,shape", [
    (2, 80, 100, 61, "shared", dict(walks_per_wave=4)),
    (3, 60, 70, 62, "shared", dict(hash_slots=512)),
    (2, 50, 40, 63, "independent", dict()),
    (3, 40, 64, 64, "shared", dict(sums_global=True)),
])
def test_resume_from_checkpoint_is_bit_identical(dim, n_max, N, seed, mode, shape):
    from paper_2002_03000_amd import ParallelFlatPERM
    full = ParallelFlatPERM(dim, n_max, N, seed, mode=mode, group_stats=True)
    part = ParallelFlatPERM(dim, n_max, N, seed, mode=mode, group_stats=True)
    sched = (1, 1, 2, 4, 4)
    for T in sched[:3]:
        for g in (full, part):
            g.run_tours(T)
            g.merge_epoch()
    blob = part.checkpoint()
    part.close()
    # resume in a fresh context, with another launch shape
    resumed = ParallelFlatPERM(dim, n_max, N, seed, mode=mode, group_stats=True, **shape)
    resumed.restore(blob)
    _same_state(full, resumed, "restored")
    for T in sched[3:]:
        for g in (full, resumed):
            g.run_tours(T)
            g.merge_epoch()
    _same_state(full, resumed, "continued")
    ra, rb = resumed.error_estimate()[0], full.error_estimate()[0]
    assert ra == rb or (np.isinf(ra) and np.isinf(rb))
    o = oracle.Oracle(dim, n_max, N, seed, mode=MODE_CODES[mode])
    for T in sched:
        o.run_tours(T)
        o.merge_epoch()
    assert_pooled_equal(resumed, o, "resumed vs oracle")
    la, ha, ma = full.estimates()
    lb, hb, mb = resumed.estimates()
    assert np.array_equal(la.view(np.uint64), lb.view(np.uint64)) and ma == mb


def test_checkpoint_carries_observables():
    from paper_2002_03000_amd import ParallelFlatPERM
    a = ParallelFlatPERM(2, 40, 32, 71, observables=True)
    for T in (1, 1):
        a.run_tours(T)
        a.merge_epoch()
    b = ParallelFlatPERM(2, 40, 32, 71, observables=True)
    b.restore(a.checkpoint())
    for g in (a, b):
        g.run_tours(2)
        g.merge_epoch()
    x, y = a.observable_r2(), b.observable_r2()
    assert np.array_equal(np.isnan(x), np.isnan(y))
    assert np.array_equal(x[~np.isnan(x)].view(np.uint64), y[~np.isnan(y)].view(np.uint64))


def test_checkpoint_refusals():
    from paper_2002_03000_amd import ParallelFlatPERM, _abi
    lib = _abi.load()
    a = ParallelFlatPERM(2, 30, 16, 81)
    a.run_tours(1)
    n = ctypes.c_size_t()
    assert lib.pperm_checkpoint_bytes(a._ctx, ctypes.byref(n)) == 0
    buf = ctypes.create_string_buffer(n.value)
    assert lib.pperm_checkpoint_save(a._ctx, buf, n.value) == -4       # unmerged tours: ESTATE
    a.merge_epoch()
    assert lib.pperm_checkpoint_save(a._ctx, buf, n.value - 1) == -1   # short buffer
    blob = a.checkpoint()
    other = ParallelFlatPERM(2, 30, 16, 82)                           # another seed
    ob = ctypes.create_string_buffer(blob, len(blob))
    assert lib.pperm_checkpoint_load(other._ctx, ob, len(blob)) == -1
    junk = ctypes.create_string_buffer(len(blob))
    assert lib.pperm_checkpoint_load(a._ctx, junk, len(blob)) == -1    # not a checkpoint
    busy = ParallelFlatPERM(2, 30, 16, 81)
    busy.run_tours(1)
    assert lib.pperm_checkpoint_load(busy._ctx, ob, len(blob)) == -4   # unmerged tours
