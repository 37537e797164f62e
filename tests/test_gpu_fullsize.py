"""The HIP path against the oracle at the benchmarked shapes, bit for bit.

* square lattice, N = 4096, n_max = 500 (the 38-epoch job): every warm-up
  epoch and the first two 64-tour epochs in full, then a later 64-tour epoch
  on sampled sequences;
* cubic lattice, N = 16384, n_max = 1000: the warm-up epochs and the first
  32-tour epoch in full, with the per-length sums in LDS and in global memory,
  then the next 32-tour epoch on sampled sequences;
* problems of the 256-problem mix with n_max above 1000 and N = 1024, through
  the chained launch (whole epochs, pooled state compared) and then the
  batched launch (a later epoch, sampled sequences);
* served jobs of the stream's shape (N = 256, T = 16, warm-up epochs, n_max
  up to 2000) replayed by the oracle to the epoch at which they stopped.

The oracle runs every sequence of every epoch that a later epoch depends on
(the pooled sums are a function of all of them); only the last epoch of a
comparison may be restricted to sampled sequences.
"""
import numpy as np
import pytest

import oracle
import workloads
from parity_util import assert_epoch_equal, assert_pooled_equal, make_pair

pytestmark = pytest.mark.gpu


def _sample_rows(N, k, seed):
    rng = np.random.default_rng(seed)
    rows = np.sort(rng.choice(N, size=k, replace=False))
    rows[0], rows[-1] = 0, N - 1
    return rows


def _epochs_in_full(g, o, sched, label):
    for i, T in enumerate(sched):
        g.run_tours(T)
        assert not o.run_tours(T)
        assert_epoch_equal(g, o, label=f"{label} epoch {i}")
        g.merge_epoch()
        o.merge_epoch()
        assert_pooled_equal(g, o, f"{label} merge {i}")
        print(f"{label}: epoch {i} ({T} tours) bit-identical", flush=True)


def test_square_n500_steady_state_epochs():
    p = workloads.PARALLEL_2D
    sched = p.schedule()
    assert sched[:9] == [1, 1, 2, 4, 8, 16, 32, 64, 64]
    g, o = make_pair(p.dim, p.n_max, p.n_sequences, p.seed)
    _epochs_in_full(g, o, sched[:9], "C2")
    # the tenth epoch (64 tours) on sampled sequences
    rows = _sample_rows(p.n_sequences, 128, 21)
    g.run_tours(sched[9])
    o.run_tours(sched[9], ids=rows)
    assert_epoch_equal(g, o, rows=rows, label="C2 epoch 9 sampled")
    st = g.sequence_stats()
    # the deep copy stacks of the steady state reach global memory
    print(f"C2: deepest copy stack {int(st['max_depth'].max())}", flush=True)
    assert int(st["max_depth"].max()) > 32


@pytest.mark.parametrize("sums_global", [False, True])
def test_cubic_n1000_steady_state_epochs(sums_global):
    p = workloads.PARALLEL_3D
    sched = p.schedule()
    assert sched[:7] == [1, 1, 2, 4, 8, 16, 32]
    g, o = make_pair(p.dim, p.n_max, p.n_sequences, p.seed, sums_global=sums_global)
    _epochs_in_full(g, o, sched[:7], f"C3 sums_global={sums_global}")
    rows = _sample_rows(p.n_sequences, 64, 22)
    g.run_tours(sched[7])
    o.run_tours(sched[7], ids=rows)
    assert_epoch_equal(g, o, rows=rows, label="C3 epoch 7 sampled")


# (index in the mix, epochs run chained and compared in full)
MIX_BIG = [(0, 7), (27, 7), (166, 4), (164, 5)]


def test_mix_long_problems_chained_then_batched():
    from paper_2002_03000_amd import Batch, ParallelFlatPERM, run_job
    mix = workloads.batched_mix()
    probs = [mix[i] for i, _ in MIX_BIG]
    for p in probs:
        assert p.n_max > 1000 and p.n_sequences == 1024
    gs = [ParallelFlatPERM(p.dim, p.n_max, p.n_sequences, p.seed, stream_id=p.stream) for p in probs]
    os_ = [oracle.Oracle(p.dim, p.n_max, p.n_sequences, p.seed, stream=p.stream) for p in probs]
    heads = [p.schedule()[:k] for p, (_, k) in zip(probs, MIX_BIG)]
    ws = run_job(gs, heads)
    for k, (g, o, head) in enumerate(zip(gs, os_, heads)):
        for T in head:
            assert not o.run_tours(T)
            o.merge_epoch()
        assert_pooled_equal(g, o, f"mix problem {MIX_BIG[k][0]} chained")
        assert np.array_equal(g.view("t").cpu().numpy().view(np.uint64), o.t)
        st = g.sequence_stats()
        for f in ("steps", "events", "enrich", "copies", "prunes", "traps", "tours", "digest"):
            assert np.array_equal(st[f], o.stats[f]), (MIX_BIG[k][0], f)
        print(f"mix problem {MIX_BIG[k][0]} (d={probs[k].dim}, n_max={probs[k].n_max}): "
              f"{len(head)} chained epochs bit-identical, deepest stack {int(st['max_depth'].max())}",
              flush=True)
    del ws
    # the next epoch of every problem in one batched launch, sampled sequences
    b = Batch(len(gs))
    nxt = [p.schedule()[k] for p, (_, k) in zip(probs, MIX_BIG)]
    b.run_tours(gs, nxt)
    for k, (g, o, T) in enumerate(zip(gs, os_, nxt)):
        rows = _sample_rows(o.N, 48, 30 + k)
        o.run_tours(T, ids=rows)
        assert_epoch_equal(g, o, rows=rows, label=f"mix problem {MIX_BIG[k][0]} batched epoch")


# (dim, n_max, seed, target relative error, tour cap): the served stream's shape
C5_JOBS = [(2, 2000, 7001, 1e-3, 65536), (3, 1999, 7002, 1e-3, 65536),
           (2, 1200, 7003, 1e-3, 32768), (2, 60, 7004, 2e-2, 10 ** 6)]


def test_served_stream_shaped_jobs_match_oracle_replay():
    from paper_2002_03000_amd import Server
    N, T = 256, 16
    srv = Server(2 << 30, 1 << 16)
    ids = [srv.submit(d, n, N, sd, T, cap, tgt, stream_id=100 + i)
           for i, (d, n, sd, tgt, cap) in enumerate(C5_JOBS)]
    done, steps = set(), 0
    while len(done) < len(ids):
        done.update(srv.step())
        steps += 1
        assert steps < 5000
    for i, (jid, (d, n, sd, tgt, cap)) in enumerate(zip(ids, C5_JOBS)):
        info = srv.info(jid)
        assert info["state"] == "done", info
        lc, hist = srv.result(jid)
        sched = workloads.Problem(d, n, N, T, info["epochs"] + 8, sd, stream=100 + i).schedule()
        o = oracle.Oracle(d, n, N, sd, stream=100 + i, group_stats=True)
        tours, stop_at = 0, None
        for e, t in enumerate(sched):
            assert not o.run_tours(t)
            o.merge_epoch()
            tours += N * t
            if o.error_estimate() <= tgt:
                stop_at = (e + 1, 1)
                break
            if tours >= cap:
                stop_at = (e + 1, 2)
                break
        assert stop_at == (info["epochs"], info["stop"]), (i, stop_at, info)
        assert tours == info["tours"] and o.walk_steps() == info["steps"]
        assert np.array_equal(hist, o.HG)
        olc = o.log_estimates()
        fin = np.isfinite(olc)
        assert np.array_equal(fin, np.isfinite(lc))
        np.testing.assert_allclose(lc[fin], olc[fin], rtol=1e-12, atol=0)
        print(f"served job {i} (d={d}, n_max={n}): {info['epochs']} epochs, stop {info['stop']}, "
              f"{info['steps']} walk-steps, bit-identical to the oracle's replay", flush=True)
        srv.release(jid)
    srv.close()
