"""HIP path vs the CPU oracle, through the C ABI, on seeded inputs.

Bar: walk trajectories (via the per-step digest), every per-sequence sum and
counter, and the pooled sums after each merge are bit-identical; the reported
log c_n agree to 1e-12 relative (host-side log conversion only).
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from parity_util import (assert_epoch_equal, assert_pooled_equal, gpu_epoch_state, make_pair)

pytestmark = pytest.mark.gpu


def _run_schedule(g, o, schedule, label):
    """schedule: list of tours-per-call; 'M' means merge."""
    for i, step in enumerate(schedule):
        if step == "M":
            g.merge_epoch()
            o.merge_epoch()
            assert_pooled_equal(g, o, f"{label} merge@{i}")
        else:
            g.run_tours(step)
            capped = o.run_tours(step)
            assert not capped
            assert_epoch_equal(g, o, label=f"{label} run@{i}")


def _check_estimates(g, o):
    lc, hist, tours = g.estimates()
    olc = o.log_estimates()
    if o.mode == oracle.MODE_INDEPENDENT:
        assert tours == int(o.MG.sum())
        assert np.array_equal(hist, o.HG.sum(axis=0))
    else:
        assert tours == int(o.MG[0])
        assert np.array_equal(hist, o.HG)
    fin = np.isfinite(olc)
    assert np.array_equal(fin, np.isfinite(lc))
    np.testing.assert_allclose(lc[fin], olc[fin], rtol=1e-12, atol=0)


def test_plain_flatperm_square_n20():
    # plain flatPERM: one sequence, n_max = 20, 10^5 tours, seed 1
    p = workloads.PLAIN_2D
    g, o = make_pair(p.dim, p.n_max, p.n_sequences, p.seed)
    _run_schedule(g, o, [p.tours_per_epoch, "M"], "plain2d")
    _check_estimates(g, o)
    # and the estimates are close to the exact counts
    lc, _, _ = g.estimates()
    exact = oracle.saw_counts(2, 20).astype(float)
    assert np.all(np.abs(np.exp(lc) / exact - 1) < 1e-2)


@pytest.mark.parametrize("dim,n_max,N,seed", [
    (2, 60, 100, 7),      # ragged: N not a multiple of the walks per wave or of 64
    (2, 120, 300, 8),
    (3, 50, 70, 9),
    (3, 90, 129, 10),
])
def test_parallel_epochs_bitwise(dim, n_max, N, seed):
    g, o = make_pair(dim, n_max, N, seed)
    _run_schedule(g, o, [5, "M", 3, 4, "M", 6, "M"], f"par{dim}d")
    _check_estimates(g, o)


@pytest.mark.parametrize("mode", ["independent", "rosenbluth"])
@pytest.mark.parametrize("dim", [2, 3])
def test_other_modes_bitwise(mode, dim):
    g, o = make_pair(dim, 40, 37, 21, mode=mode)
    _run_schedule(g, o, [6, "M", 5, "M"], f"{mode}{dim}d")
    _check_estimates(g, o)


@pytest.mark.parametrize("dim,wpw", [(2, 1), (2, 2), (2, 4), (2, 8), (2, 16),
                                     (3, 1), (3, 2), (3, 4), (3, 8)])
def test_launch_shape_never_changes_results(dim, wpw):
    g, o = make_pair(dim, 64, 45, 33, walks_per_wave=wpw)
    _run_schedule(g, o, [4, "M", 4, "M"], f"wpw{wpw}")
    # a larger table too
    g2, o2 = make_pair(dim, 64, 45, 33, walks_per_wave=wpw, hash_slots=512)
    _run_schedule(g2, o2, [4, "M"], f"wpw{wpw}-slots")


def test_edge_shapes():
    # shortest walks, a single sequence and a single tour, stream ids
    for dim, n_max, N, tours, sid in [(2, 1, 1, 1, 0), (3, 1, 3, 2, 0), (2, 2, 5, 3, 1),
                                      (3, 3, 64, 2, 7), (2, 4, 65, 3, 0)]:
        g, o = make_pair(dim, n_max, N, 100 + N, stream_id=sid)
        _run_schedule(g, o, [tours, "M", tours, "M"], f"edge{dim}/{n_max}/{N}")
        _check_estimates(g, o)


def test_exact_small_lengths_on_gpu():
    # c_1..c_3 exact for any seed and schedule (every weight at n <= 3 is equal)
    from paper_2002_03000_amd import ParallelFlatPERM
    for dim in (2, 3):
        g = ParallelFlatPERM(dim, 30, 500, 4242)
        for _ in range(3):
            g.run_tours(3)
            g.merge_epoch()
        lc, _, tours = g.estimates()
        q = 2 * dim
        assert tours == 4500
        for n, c in ((1, q), (2, q * (q - 1)), (3, q * (q - 1) ** 2)):
            assert abs(math.exp(lc[n]) / c - 1) < 1e-14


def test_parallel_square_full_shape_epochs():
    # 4096 sequences, n_max = 500: the warm-up epochs (1, 1, 2, 4, 8 tours) in
    # full, merges included, then the next epoch on sampled sequences.
    p = workloads.PARALLEL_2D
    sched = p.schedule()
    assert sched[:7] == [1, 1, 2, 4, 8, 16, 32] and sum(sched) == 38 * 64
    g, o = make_pair(p.dim, p.n_max, p.n_sequences, p.seed)
    for i, T in enumerate(sched[:5]):
        g.run_tours(T)
        o.run_tours(T)
        assert_epoch_equal(g, o, label=f"C2 epoch{i}")
        g.merge_epoch()
        o.merge_epoch()
        assert_pooled_equal(g, o, f"C2 merge{i}")
        print(f"C2 epoch {i} ({T} tours) bit-identical", flush=True)
    rng = np.random.default_rng(11)
    rows = np.sort(rng.choice(p.n_sequences, size=96, replace=False))
    rows[0], rows[-1] = 0, p.n_sequences - 1
    g.run_tours(sched[5])
    o.run_tours(sched[5], ids=rows)
    assert_epoch_equal(g, o, rows=rows, label="C2 epoch5 sampled")


def test_parallel_cubic_full_shape_sampled():
    # 16384 sequences, n_max = 1000: warm-up epochs of 1, 1, 2 tours in full,
    # then a 32-tour epoch on sampled sequences.
    p = workloads.PARALLEL_3D
    g, o = make_pair(p.dim, p.n_max, p.n_sequences, p.seed)
    for i, T in enumerate([1, 1, 2]):
        g.run_tours(T)
        o.run_tours(T)
        assert_epoch_equal(g, o, label=f"C3 epoch{i}")
        g.merge_epoch()
        o.merge_epoch()
        assert_pooled_equal(g, o, f"C3 merge{i}")
        print(f"C3 epoch {i} ({T} tours) bit-identical", flush=True)
    rng = np.random.default_rng(12)
    rows = np.sort(rng.choice(p.n_sequences, size=64, replace=False))
    rows[0], rows[-1] = 0, p.n_sequences - 1
    g.run_tours(p.tours_per_epoch)
    o.run_tours(p.tours_per_epoch, ids=rows)
    assert_epoch_equal(g, o, rows=rows, label="C3 epoch3 sampled")
    # properties of the whole epoch: one record at n = 0 per tour, steps = sum of H
    rec, m, t, st = gpu_epoch_state(g)
    H = rec["h"]
    assert (m == p.tours_per_epoch).all() and (H[:, 0] == p.tours_per_epoch).all()
    g.merge_epoch()
    lc, hist, tours = g.estimates()
    assert tours == p.n_sequences * (4 + p.tours_per_epoch)
    assert abs(math.exp(lc[3]) / 150 - 1) < 1e-14


def test_step_cap_reports_overflow():
    from paper_2002_03000_amd import ParallelFlatPERM, PPermError
    g = ParallelFlatPERM(2, 100, 10, 5, step_cap=50)
    g.run_tours(100)
    g.merge_epoch()
    with pytest.raises(PPermError) as ei:
        g.estimates()
    assert "EOVERFLOW" in str(ei.value)
    st = g.sequence_stats()
    assert (st["capped"] == 1).all() and (st["steps"] == 50).all()
    o = oracle.Oracle(2, 100, 10, 5, step_cap=50)
    assert o.run_tours(100)
    assert np.array_equal(st["digest"], o.stats["digest"])


def test_call_order_errors():
    from paper_2002_03000_amd import ParallelFlatPERM, PPermError
    g = ParallelFlatPERM(2, 10, 4, 1)
    with pytest.raises(PPermError) as ei:
        g.estimates()          # nothing merged yet
    assert "ESTATE" in str(ei.value)
    with pytest.raises(PPermError):
        g.run_tours(0)
