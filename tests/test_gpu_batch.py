"""Batched launches: every problem of a mixed batch gives exactly the bits it
gives alone, and (for small problems) exactly the oracle's."""
import numpy as np
import pytest

import oracle
import workloads
from parity_util import assert_epoch_equal, assert_pooled_equal, gpu_epoch_state, gpu_pooled_state

pytestmark = pytest.mark.gpu


def _mix():
    # d, n_max, N, seed, mode: small and large tables, 2D and 3D, ragged N
    return [(2, 30, 7, 11, "shared"), (3, 25, 64, 12, "shared"), (2, 200, 100, 13, "shared"),
            (3, 300, 33, 14, "independent"), (2, 64, 1, 15, "rosenbluth"), (3, 1500, 20, 16, "shared"),
            (2, 2000, 9, 17, "shared"), (3, 60, 130, 18, "shared")]


def _make(specs):
    from paper_2002_03000_amd import ParallelFlatPERM
    return [ParallelFlatPERM(d, n, N, sd, mode=mode, stream_id=i) for i, (d, n, N, sd, mode) in enumerate(specs)]


def _state(g):
    rec, m, t, st = gpu_epoch_state(g)
    grec, hg, mg = gpu_pooled_state(g)
    return rec, m, t, st, grec, hg, mg


def _equal(a, b):
    for x, y in zip(a, b):
        if x.dtype.names:
            for f in x.dtype.names:
                if not np.array_equal(x[f], y[f]):
                    return False
        elif not np.array_equal(x, y):
            return False
    return True


def test_batch_matches_each_problem_alone():
    from paper_2002_03000_amd import Batch
    specs = _mix()
    sched = [[1, 2, 3], [2, 0, 1], [1, 1, 1], [3, 1, 0], [4, 4, 4], [1, 1, 1], [1, 1, 2], [2, 2, 2]]
    batched = _make(specs)
    alone = _make(specs)
    b = Batch(len(specs))
    for e in range(3):
        tours = [s[e] for s in sched]
        b.run_tours(batched, tours)
        for g, a, t in zip(batched, alone, tours):
            if t:
                a.run_tours(t)
        for i, (g, a, t) in enumerate(zip(batched, alone, tours)):
            assert _equal(_state(g), _state(a)), f"problem {i} epoch {e}: batch != alone"
            if t:
                g.merge_epoch()
                a.merge_epoch()
    for i, (g, a) in enumerate(zip(batched, alone)):
        assert _equal(_state(g), _state(a)), f"problem {i}: batch != alone after merges"


def test_batch_matches_oracle_small_problems():
    from paper_2002_03000_amd import Batch
    specs = [(2, 40, 17, 21, "shared"), (3, 30, 40, 22, "shared"), (2, 50, 5, 23, "independent")]
    gs = _make(specs)
    os_ = [oracle.Oracle(d, n, N, sd, mode={"shared": 0, "independent": 1}[mode], stream=i)
           for i, (d, n, N, sd, mode) in enumerate(specs)]
    b = Batch(len(specs))
    for tours in ([1, 1, 2], [2, 3, 1], [4, 1, 1]):
        b.run_tours(gs, tours)
        for o, t in zip(os_, tours):
            o.run_tours(t)
        for i, (g, o) in enumerate(zip(gs, os_)):
            assert_epoch_equal(g, o, label=f"batch problem {i}")
            g.merge_epoch()
            o.merge_epoch()
            assert_pooled_equal(g, o, f"batch problem {i} merge")


def test_batched_mix_first_epochs_subset():
    # the first problems of the 256-problem mix, their first two epochs, batched
    # versus alone (shape coverage: n_max up to 2048, 64..1024 sequences)
    from paper_2002_03000_amd import Batch, ParallelFlatPERM
    mix = workloads.batched_mix()[:24]
    mk = lambda: [ParallelFlatPERM(p.dim, p.n_max, p.n_sequences, p.seed, stream_id=p.stream) for p in mix]
    batched, alone = mk(), mk()
    b = Batch(len(mix))
    for e in range(2):
        tours = [p.schedule()[e] for p in mix]
        b.run_tours(batched, tours)
        for a, t in zip(alone, tours):
            a.run_tours(t)
        for i, (g, a) in enumerate(zip(batched, alone)):
            assert _equal(_state(g), _state(a)), f"mix problem {i} epoch {e}"
            g.merge_epoch()
            a.merge_epoch()
        print(f"mix epoch {e} identical", flush=True)


def test_long_walk_contexts_batch_beside_in_lds_ones():
    # contexts whose sums stay in global memory (a long walk, and shorter walks
    # with the launch option) run in classes of their own, next to in-LDS
    # contexts: each bit-identical to itself alone and to the oracle.  (The
    # long walk runs only its first two one-tour epochs: its third would start
    # a cascade of enrichment at lengths no sequence has reached, 1e7-8e7
    # steps, past the default step cap of a call.)
    from paper_2002_03000_amd import Batch, ParallelFlatPERM
    specs = [(2, 6000, 6, 71, True), (3, 400, 24, 72, True), (2, 300, 40, 73, False),
             (3, 900, 20, 74, False), (2, 120, 33, 75, True)]
    mk = lambda: [ParallelFlatPERM(d, n, N, sd, stream_id=i, sums_global=sg)
                  for i, (d, n, N, sd, sg) in enumerate(specs)]
    batched, alone = mk(), mk()
    os_ = [oracle.Oracle(d, n, N, sd, stream=i) for i, (d, n, N, sd, sg) in enumerate(specs)]
    b = Batch(len(specs))
    for e, tours in enumerate(([1] * 5, [1, 2, 1, 2, 3], [0, 1, 3, 1, 2])):
        b.run_tours(batched, tours)
        for a, o, t in zip(alone, os_, tours):
            if t:
                a.run_tours(t)
                assert not o.run_tours(t)
        for i, (g, a, o) in enumerate(zip(batched, alone, os_)):
            if not tours[i]:
                continue
            assert _equal(_state(g), _state(a)), f"problem {i} epoch {e}: batch != alone"
            assert_epoch_equal(g, o, label=f"long batch problem {i} epoch {e}")
            g.merge_epoch()
            a.merge_epoch()
            o.merge_epoch()
            assert_pooled_equal(g, o, f"long batch problem {i} merge {e}")
        print(f"long-walk batch epoch {e} identical", flush=True)
