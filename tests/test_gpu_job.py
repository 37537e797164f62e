"""Device-side epoch chaining (pperm_run_job): every problem's whole epoch
schedule in persistent launches, bit-identical to running its epochs one
call at a time (lock-step batched rounds, themselves identical to each
problem alone) and to the oracle."""
import numpy as np
import pytest

import oracle
import workloads
from parity_util import assert_pooled_equal, assert_stats_equal, gpu_pooled_state

pytestmark = pytest.mark.gpu


def _make(specs):
    from paper_2002_03000_amd import ParallelFlatPERM
    return [ParallelFlatPERM(d, n, N, sd, mode=mode, stream_id=i) for i, (d, n, N, sd, mode) in enumerate(specs)]


def _state(g):
    rec, hg, mg = gpu_pooled_state(g)
    st = g.sequence_stats()
    t = g.view("t").cpu().numpy().view(np.uint64)
    return rec, hg, mg, st, t


def _assert_same(a, b, label):
    ra, ha, ma, sa, ta = a
    rb, hb, mb, sb, tb = b
    for f in ("m", "e"):
        assert np.array_equal(ra[f], rb[f]), f"{label}: G.{f}"
    assert np.array_equal(ha, hb), f"{label}: HG"
    assert np.array_equal(ma, mb), f"{label}: MG"
    assert np.array_equal(ta, tb), f"{label}: t"
    for f in sa.dtype.names:
        assert np.array_equal(sa[f], sb[f]), f"{label}: stats.{f}"


SPECS = [(2, 40, 17, 21, "shared"), (3, 30, 40, 22, "shared"), (2, 200, 100, 23, "shared"),
         (3, 300, 33, 24, "rosenbluth"), (2, 64, 1, 25, "shared"), (3, 1500, 20, 26, "shared"),
         (2, 2000, 9, 27, "shared"), (3, 60, 130, 28, "shared"), (2, 100, 64, 29, "shared")]
SCHEDS = [[1, 1, 2, 4], [1, 1, 2], [1, 1, 2, 4, 8, 3], [2, 2], [1, 1, 2, 4, 8, 16, 32],
          [1, 1], [1, 1, 1], [1, 1, 2, 4, 5], [3, 1, 4, 1, 5]]


def test_job_matches_lockstep_rounds():
    from paper_2002_03000_amd import run_job, run_schedules
    chained = _make(SPECS)
    stepped = _make(SPECS)
    run_job(chained, SCHEDS)
    run_schedules(stepped, SCHEDS)
    for i, (g, h) in enumerate(zip(chained, stepped)):
        _assert_same(_state(g), _state(h), f"problem {i}")
        lc, hist, tours = g.estimates()
        assert tours == SPECS[i][2] * sum(SCHEDS[i])
    # and the open-epoch sums are back to zero, as after a merge
    for g in chained:
        assert not g.records("L")["m"].any() and not g.view("m").cpu().numpy().any()


def test_job_matches_oracle_small_problems():
    from paper_2002_03000_amd import run_job
    specs = [(2, 40, 17, 31, "shared"), (3, 30, 40, 32, "shared"), (2, 12, 3, 33, "shared")]
    scheds = [[1, 1, 2, 4, 8], [2, 1, 3], [1, 1, 2, 4]]
    gs = _make(specs)
    run_job(gs, scheds)
    for i, ((d, n, N, sd, mode), sch) in enumerate(zip(specs, scheds)):
        o = oracle.Oracle(d, n, N, sd, stream=i)
        for T in sch:
            o.run_tours(T)
            o.merge_epoch()
        assert_pooled_equal(gs[i], o, f"job problem {i}")
        assert_stats_equal(gs[i].sequence_stats(), o.stats)


def test_job_then_more_calls_continue_the_same_chain():
    # a chained job followed by ordinary calls equals ordinary calls throughout
    from paper_2002_03000_amd import run_job
    specs = [(2, 80, 50, 41, "shared"), (3, 50, 20, 42, "shared")]
    a = _make(specs)
    b = _make(specs)
    run_job(a, [[1, 1, 2], [1, 2]])
    for g in a:
        g.run_tours(3)
        g.merge_epoch()
    for g, sch in zip(b, [[1, 1, 2, 3], [1, 2, 3]]):
        for T in sch:
            g.run_tours(T)
            g.merge_epoch()
    for i, (g, h) in enumerate(zip(a, b)):
        _assert_same(_state(g), _state(h), f"continued problem {i}")


def test_job_rejects_independent_mode_and_open_epochs():
    from paper_2002_03000_amd import PPermError, run_job
    ind = _make([(2, 20, 4, 51, "independent")])
    with pytest.raises(PPermError, match="EINVAL"):
        run_job(ind, [[1]])
    op = _make([(2, 20, 4, 52, "shared")])
    op[0].run_tours(1)
    with pytest.raises(PPermError, match="ESTATE"):
        run_job(op, [[1]])


def test_job_mix_subset_matches_lockstep():
    # the first 32 problems of the 256-problem mix, first 6 epochs each
    from paper_2002_03000_amd import ParallelFlatPERM, run_job, run_schedules
    mix = workloads.batched_mix()[:32]
    scheds = [p.schedule()[:6] for p in mix]
    mk = lambda: [ParallelFlatPERM(p.dim, p.n_max, p.n_sequences, p.seed, stream_id=p.stream) for p in mix]
    chained, stepped = mk(), mk()
    run_job(chained, scheds)
    print("chained job done", flush=True)
    run_schedules(stepped, scheds)
    for i, (g, h) in enumerate(zip(chained, stepped)):
        _assert_same(_state(g), _state(h), f"mix problem {i}")


def test_step_cap_stops_only_its_problem_and_is_reported():
    # problem 1 hits its step cap in its third epoch: it stops after that
    # epoch and reports EOVERFLOW; the others run their whole schedules, bit
    # for bit as alone; the launch's report counts the failure and nothing else
    from paper_2002_03000_amd import ParallelFlatPERM, PPermError, job_report, run_job
    specs = [(2, 60, 40, 61), (2, 200, 30, 62), (3, 50, 25, 63)]
    scheds = [[1, 1, 2, 4], [1, 1, 2, 4, 8], [1, 2, 3]]
    caps = [0, 2000, 0]
    gs = [ParallelFlatPERM(d, n, N, sd, stream_id=i, step_cap=caps[i]) for i, (d, n, N, sd) in enumerate(specs)]
    ws = run_job(gs, scheds)
    rep = job_report(ws)
    print(f"job report: {rep}", flush=True)
    assert rep["problems_failed"] == 1 and rep["problems_incomplete"] == 0
    assert rep["waves_left_idle"] == 0 and rep["problems_finished"] == 3
    with pytest.raises(PPermError, match="EOVERFLOW"):
        gs[1].estimates()
    st = gs[1].sequence_stats()
    assert st["capped"].any()
    # the capped problem ran no epoch after the one in which the cap hit: its
    # sequences' tour counters stop there (the oracle, capped the same way,
    # names that epoch)
    o = oracle.Oracle(2, 200, 30, 62, stream=1, step_cap=2000)
    ran = 0
    for T in scheds[1]:
        capped = o.run_tours(T)
        o.merge_epoch()
        ran += T
        if capped:
            break
    assert ran < sum(scheds[1])
    assert np.array_equal(gs[1].view("t").cpu().numpy().view(np.uint64), o.t)
    for i in (0, 2):
        alone = ParallelFlatPERM(specs[i][0], specs[i][1], specs[i][2], specs[i][3], stream_id=i)
        for T in scheds[i]:
            alone.run_tours(T)
            alone.merge_epoch()
        _assert_same(_state(gs[i]), _state(alone), f"uncapped problem {i}")
