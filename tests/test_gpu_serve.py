"""Serving: continuous batching of sampling jobs through the library's server.

Each served job's result (estimates, sample counts, epochs run, stop reason,
error estimate, walk-steps) is the same alone and in the mix, whatever the
pool pressure; served jobs agree with the oracle replaying the epochs the
server ran, including the epoch at which the stop rule fired."""
import numpy as np
import pytest

import oracle
import workloads
from parity_util import assert_epoch_equal, assert_pooled_equal, make_pair

pytestmark = pytest.mark.gpu

MB = 1 << 20


def _jobs():
    # (dim, n_max, N, seed, T, tour_cap, target): mixed d and n_max, some stop
    # on the error target, the rest on the tour cap
    return [(2, 40, 32, 101, 4, 4000, 0.02), (3, 30, 16, 102, 8, 3000, 0.05),
            (2, 120, 64, 103, 2, 2500, 1e-4), (3, 200, 32, 104, 4, 2000, 1e-4),
            (2, 25, 16, 105, 16, 20000, 0.01), (3, 60, 48, 106, 3, 5000, 0.03),
            (2, 300, 16, 107, 4, 1000, 0.0), (2, 10, 16, 108, 1, 3000, 0.005),
            (3, 15, 64, 109, 5, 6000, 0.01), (2, 80, 32, 110, 6, 3000, 0.05)]


def _job_bytes(spec):
    import ctypes
    from paper_2002_03000_amd import _abi
    d, n, N, sd, T, cap, tgt = spec
    cfg = _abi.Config(ctypes.sizeof(_abi.Config), d, n, N, sd, 0, 0, 0, 1, 0, _abi.FLAG_GROUP_STATS)
    nb = ctypes.c_size_t()
    _abi.check(_abi.load().pperm_workspace_bytes(ctypes.byref(cfg), ctypes.byref(nb)), "workspace")
    return (nb.value + 255) // 256 * 256


def _serve(specs, stream_ids=None, pool_bytes=256 * MB, max_seq=4096, slice_us=None):
    from paper_2002_03000_amd import Server
    srv = Server(pool_bytes, max_seq)
    if slice_us is not None:
        srv.set_slice(slice_us)
    if stream_ids is None:
        stream_ids = list(range(len(specs)))
    ids = [srv.submit(d, n, N, sd, T, cap, tgt, stream_id=sid)
           for sid, (d, n, N, sd, T, cap, tgt) in zip(stream_ids, specs)]
    done, steps, peak_active = set(), 0, 0
    while len(done) < len(ids):
        fin = srv.step()
        done.update(fin)
        q, a, _ = srv.counts()
        # jobs held at once in this step: still active, or retired by it
        peak_active = max(peak_active, a + len(fin))
        steps += 1
        assert steps < 10000
    out = []
    for jid in ids:
        info = srv.info(jid)
        assert info["state"] == "done", info
        lc, hist = srv.result(jid)
        out.append((info, lc, hist))
    q, a, used = srv.counts()
    assert q == 0 and a == 0
    srv.close()
    return out, peak_active


def _same(a, b):
    ia, la, ha = a
    ib, lb, hb = b
    for f in ("epochs", "tours", "steps", "stop"):
        assert ia[f] == ib[f], (f, ia, ib)
    assert (ia["rel_err"] == ib["rel_err"]) or (np.isnan(ia["rel_err"]) and np.isnan(ib["rel_err"]))
    assert np.array_equal(la.view(np.uint64), lb.view(np.uint64))
    assert np.array_equal(ha, hb)


def test_error_estimate_group_sums_match_oracle():
    for (d, n, N, seed) in ((2, 50, 40, 31), (3, 35, 100, 32)):
        g, o = make_pair(d, n, N, seed, group_stats=True)
        o.group_stats = True
        for T in (1, 1, 2, 4, 4):
            g.run_tours(T)
            o.run_tours(T)
            assert_epoch_equal(g, o, label="group epoch")
            g.merge_epoch()
            o.merge_epoch()
            assert_pooled_equal(g, o, "group merge")
            rec = g.records("gsum")
            assert np.array_equal(rec["m"], o.gsum["m"]) and np.array_equal(rec["e"], o.gsum["e"])
            assert np.array_equal(g.view("gtours").cpu().numpy().view(np.uint64), o.gtours)
            rel, _ = g.error_estimate()
            ref = o.error_estimate()
            if np.isinf(ref):
                assert np.isinf(rel)
            else:
                assert abs(rel / ref - 1) < 1e-12


def test_served_jobs_same_alone_and_in_the_mix():
    specs = _jobs()
    # a pool that holds only a few jobs at a time: admission waits for memory
    tight = 128 * 1024 + int(2.5 * max(_job_bytes(sp) for sp in specs))
    mixed, peak = _serve(specs, pool_bytes=tight)
    print(f"peak active jobs under a {tight} byte pool: {peak}", flush=True)
    assert 1 < peak < len(specs)
    roomy, peak2 = _serve(specs)
    assert peak2 == len(specs)
    # a 1 us slice splits every job's epochs over many more steps
    sliced, _ = _serve(specs, slice_us=1)
    for i, spec in enumerate(specs):
        alone, _ = _serve([spec], stream_ids=[i])
        _same(mixed[i], roomy[i])
        _same(mixed[i], alone[0])
        _same(mixed[i], sliced[i])
    stops = [m[0]["stop"] for m in mixed]
    assert 1 in stops and 2 in stops, stops


def test_served_jobs_match_oracle_replay():
    specs = _jobs()
    served, _ = _serve(specs, pool_bytes=64 * MB)
    for i in (0, 1, 4, 7, 9):
        d, n, N, sd, T, cap, tgt = specs[i]
        info, lc, hist = served[i]
        sched = workloads.Problem(d, n, N, T, info["epochs"] + 8, sd, stream=i).schedule()
        o = oracle.Oracle(d, n, N, sd, stream=i, group_stats=True)
        tours, stop_at = 0, None
        for e, t in enumerate(sched):
            o.run_tours(t)
            o.merge_epoch()
            tours += N * t
            rel = o.error_estimate() if tgt > 0 else np.inf
            if tgt > 0 and rel <= tgt:
                stop_at = (e + 1, 1)
                break
            if tours >= cap:
                stop_at = (e + 1, 2)
                break
        assert stop_at == (info["epochs"], info["stop"]), (i, stop_at, info)
        assert tours == info["tours"]
        assert o.walk_steps() == info["steps"]
        assert np.array_equal(hist, o.HG)
        olc = o.log_estimates()
        fin = np.isfinite(olc)
        assert np.array_equal(fin, np.isfinite(lc))
        np.testing.assert_allclose(lc[fin], olc[fin], rtol=1e-12, atol=0)


def test_sliced_chains_with_stop_rules_match_the_oracle():
    # chained epochs in 1 us slices (so almost every call runs few epochs),
    # stop rule on the device, against the oracle's epoch-by-epoch replay
    from paper_2002_03000_amd import ParallelFlatPERM, run_job_sliced
    specs = [(2, 40, 32, 201, 4, 4000, 0.02), (3, 30, 16, 202, 8, 3000, 0.05), (2, 25, 16, 203, 16, 20000, 0.01)]
    probs = [ParallelFlatPERM(d, n, N, sd, stream_id=i, group_stats=True) for i, (d, n, N, sd, T, cap, tgt) in enumerate(specs)]
    scheds = [workloads.Problem(d, n, N, T, 1000, sd).schedule() for (d, n, N, sd, T, cap, tgt) in specs]
    pos = [0] * len(specs)
    stopped = [0] * len(specs)
    calls = 0
    while not all(stopped):
        live = [i for i in range(len(specs)) if not stopped[i]]
        done, stop, rel = run_job_sliced([probs[i] for i in live], [scheds[i][pos[i]:pos[i] + 50] for i in live],
                                         limits=[(specs[i][6], specs[i][5]) for i in live], slice_us=1)
        for k, i in enumerate(live):
            pos[i] += int(done[k])
            stopped[i] = int(stop[k])
        calls += 1
        assert calls < 5000
    for i, (d, n, N, sd, T, cap, tgt) in enumerate(specs):
        o = oracle.Oracle(d, n, N, sd, stream=i, group_stats=True)
        tours, stop_at = 0, None
        for e, t in enumerate(scheds[i]):
            o.run_tours(t)
            o.merge_epoch()
            tours += N * t
            if o.error_estimate() <= tgt:
                stop_at = (e + 1, 1)
                break
            if tours >= cap:
                stop_at = (e + 1, 2)
                break
        assert stop_at == (pos[i], stopped[i]), (i, stop_at, pos[i], stopped[i])
        assert_pooled_equal(probs[i], o, f"sliced problem {i}")
    print(f"{calls} sliced calls", flush=True)
