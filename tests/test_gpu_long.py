"""Long walks (n_max ~ 10^4): the per-length sums stay in global memory.

Parity with the oracle bit for bit at n_max = 10^4 in two and three
dimensions, with and without observables, and the launch-shape rules of the
long layout."""
import ctypes

import numpy as np
import pytest

import oracle
from parity_util import assert_epoch_equal, assert_pooled_equal, make_pair

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim,n_max,N,seed,tours", [
    (2, 10000, 100, 5, (1, 1)),
    (3, 10000, 70, 6, (1, 1, 2)),
    (2, 6000, 130, 7, (1, 2)),
])
def test_long_walks_match_oracle(dim, n_max, N, seed, tours):
    g, o = make_pair(dim, n_max, N, seed)
    shape = g.launch_shape()
    print(f"d={dim} n_max={n_max} N={N}: {shape}", flush=True)
    for T in tours:
        g.run_tours(T)
        o.run_tours(T)
        assert_epoch_equal(g, o, label=f"long epoch T={T}")
        g.merge_epoch()
        o.merge_epoch()
        assert_pooled_equal(g, o, f"long merge T={T}")
    lc, hist, M = g.estimates()
    olc = o.log_estimates()
    fin = np.isfinite(olc)
    assert np.array_equal(fin, np.isfinite(lc)) and fin[n_max]
    np.testing.assert_allclose(lc[fin], olc[fin], rtol=1e-12, atol=0)


def test_long_walk_layout():
    from paper_2002_03000_amd import ParallelFlatPERM
    g = ParallelFlatPERM(3, 10000, 8, 1)
    # 2^14 slots (5/8 full at most) of 8-byte keys: one workgroup per CU
    assert g.launch_shape()["hash_slots"] == 16384
    g2 = ParallelFlatPERM(2, 10000, 8, 1)
    assert g2.launch_shape()["hash_slots"] == 32768


def test_long_walk_observables_match_oracle():
    from paper_2002_03000_amd import ParallelFlatPERM
    g = ParallelFlatPERM(2, 8000, 90, 8, observables=True)
    o = oracle.Oracle(2, 8000, 90, 8, observables=True)
    for T in (1, 1):
        g.run_tours(T)
        o.run_tours(T)
        g.merge_epoch()
        o.merge_epoch()
    assert_pooled_equal(g, o, "long observables")
    rec = g.records("obs_G")[:8001]
    assert np.array_equal(rec["m"], o.GR["m"]) and np.array_equal(rec["e"], o.GR["e"])
    a, b = g.observable_r2(), o.observable_r2()
    nan = np.isnan(b)
    assert np.array_equal(np.isnan(a), nan)
    assert np.array_equal(a[~nan].view(np.uint64), b[~nan].view(np.uint64))


def test_long_contexts_batch_and_chain():
    # a long walk (sums in global memory) runs in a batched launch, in a class
    # of its own, and in the chained launch beside in-LDS problems, with the
    # bits it gives alone epoch by epoch, and the oracle's
    from paper_2002_03000_amd import Batch, ParallelFlatPERM, job_report, run_job
    g = ParallelFlatPERM(2, 9000, 4, 9)
    a = ParallelFlatPERM(2, 9000, 4, 9)
    Batch(1).run_tours([g], [1])
    a.run_tours(1)
    rg, ra = g.records("L"), a.records("L")
    assert np.array_equal(rg["m"], ra["m"]) and np.array_equal(rg["e"], ra["e"]) and np.array_equal(rg["h"], ra["h"])
    assert np.array_equal(g.sequence_stats()["digest"], a.sequence_stats()["digest"])

    # chained: a long square walk, a long cubic walk with sums in global memory
    # by choice, and an in-LDS problem (the long square walk stops before the
    # epoch whose enrichment cascade would pass the default step cap)
    specs = [(2, 7000, 3, 91, False), (3, 600, 5, 92, True), (2, 200, 20, 93, False)]
    sched = [[1, 1, 2, 4], [1, 1, 2], [1, 2, 4]]
    chained = [ParallelFlatPERM(d, n, N, sd, stream_id=i, sums_global=sg) for i, (d, n, N, sd, sg) in enumerate(specs)]
    alone = [ParallelFlatPERM(d, n, N, sd, stream_id=i, sums_global=sg) for i, (d, n, N, sd, sg) in enumerate(specs)]
    ws = run_job(chained, sched)
    rep = job_report(ws)
    print(f"chained with long walks: {rep}", flush=True)
    assert rep["problems_finished"] == len(specs) and rep["problems_failed"] == 0 and rep["problems_incomplete"] == 0
    for i, (x, y) in enumerate(zip(chained, alone)):
        for T in sched[i]:
            y.run_tours(T)
            y.merge_epoch()
        lx, hx, mx = x.estimates()
        ly, hy, my = y.estimates()
        assert mx == my and np.array_equal(hx, hy), f"problem {i}"
        assert np.array_equal(lx.view(np.uint64), ly.view(np.uint64)), f"problem {i}: chained != alone"
        a_, b_ = x.sequence_stats(), y.sequence_stats()
        assert all(np.array_equal(a_[f], b_[f]) for f in a_.dtype.names), f"problem {i}: stats"
    d, n, N, sd, sg = specs[0]
    o = oracle.Oracle(d, n, N, sd, stream=0)
    for T in sched[0]:
        assert not o.run_tours(T)
        o.merge_epoch()
    assert_pooled_equal(chained[0], o, "chained long walk")


def test_log_c10000_agrees_with_the_long_run_value():
    # Algorithm 2 on the square lattice up to n = 10^4 (256 sequences, 98304
    # tours): the estimate of log c_10000 must fall within 1 of the value a
    # very long flatPERM run gives (eqn (8)), the band Tables 1 and 2 show for
    # Algorithm 2 once a few thousand walks have been started
    import workloads
    from paper_2002_03000_amd import ParallelFlatPERM
    p = workloads.LONG_2D
    g = ParallelFlatPERM(p.dim, p.n_max, p.n_sequences, p.seed, group_stats=True)
    for T in p.schedule():
        g.run_tours(T)
        g.merge_epoch()
    lc, hist, M = g.estimates()
    rel, _ = g.error_estimate()
    print(f"log c_10000 = {lc[10000]:.4f} after {M} tours (relative error estimate {rel:.3g})", flush=True)
    assert M == p.total_tours
    assert abs(lc[10000] - 9704.14) < 1.0


@pytest.mark.parametrize("dim,n_max,N,seed", [(3, 1000, 200, 21), (2, 500, 130, 22)])
def test_sums_in_global_memory_change_no_bit(dim, n_max, N, seed):
    # the tuning flag that keeps the per-length sums out of LDS (more walks per
    # compute unit) runs the long-walk walker at ordinary lengths: same bits as
    # the oracle and as the default layout
    from paper_2002_03000_amd import ParallelFlatPERM
    g = ParallelFlatPERM(dim, n_max, N, seed, sums_global=True)
    h = ParallelFlatPERM(dim, n_max, N, seed)
    o = oracle.Oracle(dim, n_max, N, seed)
    for T in (1, 1, 2):
        for x in (g, h, o):
            x.run_tours(T)
        assert_epoch_equal(g, o, label=f"sums in global memory T={T}")
        for x in (g, h, o):
            x.merge_epoch()
        assert_pooled_equal(g, o, "sums in global memory")
    a, b = g.sequence_stats(), h.sequence_stats()
    assert all(np.array_equal(a[f], b[f]) for f in a.dtype.names)


def test_global_sums_walker_independent_and_rosenbluth_batched():
    # Algorithm 1 (each sequence with its own sums) and plain Rosenbluth runs
    # through the walker that keeps the sums in global memory, in one batched
    # launch with one-tour and longer epochs: each problem bit-identical to the
    # oracle.  Each sequence of Algorithm 1 meets its own enrichment cascade on
    # its second tour, so every context gets the step watchdog of a 64-tour
    # epoch.
    from paper_2002_03000_amd import Batch, ParallelFlatPERM
    specs = [(2, 700, 5, 31, "independent"), (3, 500, 4, 32, "independent"),
             (2, 600, 6, 33, "rosenbluth"), (3, 300, 7, 34, "shared")]
    gs = [ParallelFlatPERM(d, n, N, sd, mode=mode, stream_id=i, sums_global=True,
                           step_cap=4096 * 64 * (n + 1))
          for i, (d, n, N, sd, mode) in enumerate(specs)]
    os_ = [oracle.Oracle(d, n, N, sd, mode={"shared": 0, "independent": 1, "rosenbluth": 2}[mode], stream=i)
           for i, (d, n, N, sd, mode) in enumerate(specs)]
    b = Batch(len(specs))
    for e, tours in enumerate(([1, 1, 1, 1], [1, 1, 2, 1], [2, 1, 1, 2], [4, 2, 0, 4])):
        print(f"global-sums batch epoch {e}: tours {tours}", flush=True)
        b.run_tours(gs, tours)
        for i, (g, o, t) in enumerate(zip(gs, os_, tours)):
            if not t:
                continue
            assert not o.run_tours(t)
            assert_epoch_equal(g, o, label=f"global sums problem {i} ({specs[i][4]}) epoch {e}")
            g.merge_epoch()
            o.merge_epoch()
            assert_pooled_equal(g, o, f"global sums problem {i} merge {e}")
    for g, o in zip(gs, os_):
        lc, _, _ = g.estimates()
        olc = o.log_estimates()
        fin = np.isfinite(olc)
        assert np.array_equal(fin, np.isfinite(lc))
        np.testing.assert_allclose(lc[fin], olc[fin], rtol=1e-12, atol=0)


def test_one_and_a_half_power_of_two_tables_change_no_bit():
    # occupancy tables of 3 * 2^k slots (hash by the high word of hash * S,
    # probe positions wrapped by one subtraction), with the sums in LDS and in
    # global memory, batched and chained: the oracle's bits and the default
    # shape's
    from paper_2002_03000_amd import Batch, ParallelFlatPERM, run_job
    specs = [(2, 150, 30, 41, 384, False), (3, 300, 50, 42, 768, False),
             (2, 700, 40, 43, 1536, False), (3, 1000, 64, 44, 1536, True)]
    sched = [1, 1, 2, 4]
    mk = lambda slots: [ParallelFlatPERM(d, n, N, sd, stream_id=i, hash_slots=(hs if slots else 0), sums_global=sg)
                        for i, (d, n, N, sd, hs, sg) in enumerate(specs)]
    batched, default, chained = mk(True), mk(False), mk(True)
    for g, (d, n, N, sd, hs, sg) in zip(batched, specs):
        assert g.launch_shape()["hash_slots"] == hs
    b = Batch(len(specs))
    for T in sched:
        b.run_tours(batched, [T] * len(specs))
        for g in batched:
            g.merge_epoch()
        for g in default:
            g.run_tours(T)
            g.merge_epoch()
    run_job(chained, [sched] * len(specs))
    for i, (x, y, z) in enumerate(zip(batched, default, chained)):
        lx, hx, mx = x.estimates()
        for other, label in ((y, "default shape"), (z, "chained")):
            lo, ho, mo = other.estimates()
            assert mx == mo and np.array_equal(hx, ho), f"problem {i} vs {label}"
            assert np.array_equal(lx.view(np.uint64), lo.view(np.uint64)), f"problem {i} vs {label}"
            a_, b_ = x.sequence_stats(), other.sequence_stats()
            assert all(np.array_equal(a_[f], b_[f]) for f in a_.dtype.names), f"problem {i} vs {label}: stats"
        d, n, N, sd, hs, sg = specs[i]
        o = oracle.Oracle(d, n, N, sd, stream=i)
        for T in sched:
            assert not o.run_tours(T)
            o.merge_epoch()
        assert_pooled_equal(x, o, f"{hs}-slot table, problem {i}")
        print(f"problem {i}: {hs} slots, d={d}, n_max={n}: identical", flush=True)
