"""Captured epochs (HIP graphs) and the launch-shape autotuner."""
import numpy as np
import pytest

import oracle
from parity_util import assert_pooled_equal, assert_stats_equal, gpu_pooled_state, make_pair

pytestmark = pytest.mark.gpu


def _pooled(g):
    rec, hg, mg = gpu_pooled_state(g)
    return rec["m"].copy(), rec["e"].copy(), hg.copy(), mg.copy(), g.sequence_stats()


def _same(a, b, label):
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y), label
    for f in a[4].dtype.names:
        assert np.array_equal(a[4][f], b[4][f]), f"{label}: {f}"


def test_graph_replays_match_eager_calls_and_the_oracle():
    from paper_2002_03000_amd import ParallelFlatPERM
    for d, n, N, seed in ((2, 60, 100, 61), (3, 40, 33, 62)):
        g_graph = ParallelFlatPERM(d, n, N, seed)
        g_eager, o = make_pair(d, n, N, seed)
        graph = g_graph.epoch_graph(2)
        for rep in range(5):
            graph.launch()
            g_eager.run_tours(2)
            g_eager.merge_epoch()
            o.run_tours(2)
            o.merge_epoch()
            # the program's own eager work between replays
            g_graph.estimates()
            a, b = _pooled(g_graph), _pooled(g_eager)
            _same(a, b, f"replay {rep}")
            assert_pooled_equal(g_graph, o, f"graph replay {rep}")
            assert_stats_equal(g_graph.sequence_stats(), o.stats)
            if rep == 2:
                for g in (g_graph, g_eager):
                    g.run_tours(3)
                    g.merge_epoch()
                o.run_tours(3)
                o.merge_epoch()
        graph.close()


def test_graph_needs_a_merged_context():
    from paper_2002_03000_amd import ParallelFlatPERM, PPermError
    g = ParallelFlatPERM(2, 20, 8, 63)
    g.run_tours(1)
    with pytest.raises(PPermError, match="ESTATE"):
        g.epoch_graph(1)


def test_autotune_picks_a_fitting_shape_with_identical_results():
    from paper_2002_03000_amd import ParallelFlatPERM, autotune
    best, table = autotune(2, 120, 256, trial=(1, 1, 2))
    print(table, flush=True)
    assert best in table and len(table) >= 2
    assert any(r["sums_global"] for r in table)
    tuned = ParallelFlatPERM(2, 120, 256, 64, hash_slots=best["hash_slots"], walks_per_wave=best["walks_per_wave"],
                             sums_global=best["sums_global"])
    plain = ParallelFlatPERM(2, 120, 256, 64)
    for g in (tuned, plain):
        for T in (1, 1, 2, 4):
            g.run_tours(T)
            g.merge_epoch()
    _same(_pooled(tuned), _pooled(plain), "autotuned shape")
