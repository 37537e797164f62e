"""The seeded input recipes: epoch schedules, the batched mix and the served stream."""
import math

import numpy as np
import pytest

import workloads


@pytest.mark.parametrize("T,epochs", [(1, 5), (2, 3), (3, 4), (54, 6), (64, 38), (100, 2), (1000, 1)])
def test_warmup_schedule_rule(T, epochs):
    p = workloads.Problem(dim=2, n_max=10, n_sequences=4, tours_per_epoch=T, epochs=epochs, seed=1)
    s = p.schedule()
    # the total budget is unchanged by the warm-up split
    assert sum(s) == T * epochs and p.total_tours == 4 * T * epochs
    if T == 1:
        assert s == [1] * epochs
        return
    # warm-up: 1, then each epoch the running total, while twice the total stays within T,
    # then the remainder of the first T tours; after that epochs of T
    head = s[:len(s) - (epochs - 1)]
    assert sum(head) == T and head[0] == 1
    run = 1
    for x in head[1:-1]:
        assert x == run
        run += x
    assert s[len(head):] == [T] * (epochs - 1)
    assert all(x >= 1 for x in s)


def test_warmup_off_and_known_schedules():
    assert workloads.Problem(2, 10, 1, 64, 3, 1, warmup=False).schedule() == [64, 64, 64]
    assert workloads.PARALLEL_2D.schedule()[:8] == [1, 1, 2, 4, 8, 16, 32, 64]
    assert workloads.PARALLEL_2D.total_tours == 9961472
    assert workloads.PARALLEL_3D.total_tours == 8388608
    assert workloads.LONG_2D.total_tours == 98304
    assert workloads.PLAIN_2D.schedule() == [100000]


def test_batched_mix_follows_its_recipe():
    mix = workloads.batched_mix(4)
    assert len(mix) == 256 and mix == workloads.batched_mix(4)
    assert mix != workloads.batched_mix(5)
    assert {p.dim for p in mix} == {2, 3}
    assert all(64 <= p.n_max <= 2048 for p in mix)
    assert {p.n_sequences for p in mix} <= {64, 128, 256, 512, 1024}
    for i, p in enumerate(mix):
        assert p.seed == 1000 + i and p.stream == i
        assert 1 <= p.tours_per_epoch <= 64
        budget = p.n_sequences * p.tours_per_epoch * p.epochs
        # ceil(B / (N T)) epochs of N T tours: within one epoch's tours of a budget in [1e4, 1e6]
        assert 1e4 <= budget < 1e6 + p.n_sequences * p.tours_per_epoch
    assert sum(p.total_tours for p in mix) == 68673984


def test_served_stream_follows_its_recipe():
    jobs = workloads.served_arrivals(5)
    assert jobs == workloads.served_arrivals(5)
    t = np.array([j.arrival_s for j in jobs])
    assert np.all(np.diff(t) > 0) and t[-1] < 60.0
    # Poisson at 50/s for 60 s: 3000 expected arrivals, the count within 5 sigma
    assert abs(len(jobs) - 3000) < 5 * math.sqrt(3000)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 0.02) < 0.002
    assert {j.problem.dim for j in jobs} == {2, 3}
    assert all(50 <= j.problem.n_max <= 2000 for j in jobs)
    assert all(j.problem.n_sequences == 256 and j.problem.tours_per_epoch == 16 for j in jobs)
    assert len({j.problem.seed for j in jobs}) == len(jobs)
    short = workloads.served_arrivals(5, duration_s=20.0)
    assert [j.arrival_s for j in short] == [j.arrival_s for j in jobs if j.arrival_s < 20.0]
