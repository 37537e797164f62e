"""Seeded synthetic workloads for parallel flatPERM.

This module only describes problems (lattice dimension, maximum length, number
of sequences, epoch schedule, seeds) and draws the mixes and arrival streams
from numpy generators.  It contains none of the method's arithmetic; the HIP
path and the CPU oracle both take their inputs from here and from nothing else.

The workload is intrinsically synthetic: walks are grown from parameters, so
no dataset stands behind any of these shapes.
"""
from dataclasses import dataclass, asdict, replace
import math

import numpy as np


@dataclass(frozen=True)
class Problem:
    dim: int                 # 2 (square lattice) or 3 (cubic lattice)
    n_max: int               # maximum walk length
    n_sequences: int         # N interacting flatPERM sequences
    tours_per_epoch: int     # T tours per sequence between merges
    epochs: int              # number of (run, merge) pairs
    seed: int                # Philox key
    mode: str = "shared"     # "shared" (Algorithm 2), "independent" (Algorithm 1), "rosenbluth"
    stream: int = 0          # xored into the key's high word (problem id in a batch)

    warmup: bool = True      # start with short epochs (see schedule())

    @property
    def total_tours(self) -> int:
        return self.n_sequences * sum(self.schedule())

    def schedule(self):
        """Tours per sequence of each epoch (one merge after each).

        With warm-up the first tours_per_epoch tours are split into epochs of
        1, 1, 2, 4, ... tours (doubling while the running total stays within
        tours_per_epoch) and one epoch of the remainder, so that the sequences
        start sharing their running averages after their first tour; the
        remaining epochs have tours_per_epoch tours.  The total is
        epochs * tours_per_epoch either way."""
        T = self.tours_per_epoch
        if not self.warmup or T == 1:
            return [T] * self.epochs
        head = [1]
        while 2 * sum(head) <= T:
            head.append(sum(head))
        if sum(head) < T:
            head.append(T - sum(head))
        return head + [T] * (self.epochs - 1)

    def as_dict(self):
        return asdict(self)

    def scaled(self, **kw):
        return replace(self, **kw)


# Plain flatPERM: one sequence, square lattice, n_max = 20, 10^5 tours, seed 1.
PLAIN_2D = Problem(dim=2, n_max=20, n_sequences=1, tours_per_epoch=100_000, epochs=1, seed=1,
                   warmup=False)

# Parallel flatPERM on Z^2: 4096 sequences sharing W, a merge every 64 tours,
# n_max = 500, 10^7 tours in total -> 38 epochs' worth of 4096 * 64 tours
# (9,961,472), the first 64 tours of each sequence in warm-up epochs.
PARALLEL_2D = Problem(dim=2, n_max=500, n_sequences=4096, tours_per_epoch=64, epochs=38, seed=2)

# Parallel flatPERM on Z^3: 16384 sequences, a merge every 32 tours, n_max = 1000,
# 16 epochs' worth (8,388,608 tours), the first 32 tours in warm-up epochs.
PARALLEL_3D = Problem(dim=3, n_max=1000, n_sequences=16384, tours_per_epoch=32, epochs=16, seed=3)

# Long walks on Z^2: n_max = 10^4 (the length of the paper's Tables 1 and 2),
# 256 sequences, a merge every 64 tours, 6 epochs' worth (98304 tours).
LONG_2D = Problem(dim=2, n_max=10000, n_sequences=256, tours_per_epoch=64, epochs=6, seed=2024)


def batched_mix(seed: int = 4, count: int = 256):
    """Independent problems for one batched launch.

    d uniform in {2, 3}; n_max uniform in [64, 2048]; N = 2^U{6..10} sequences;
    a tour budget B log-uniform in [1e4, 1e6]; T = clamp(floor(B / (16 N)), 1, 64)
    tours per epoch and ceil(B / (N T)) epochs; problem seed 1000 + i.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        d = int(rng.integers(2, 4))
        n_max = int(rng.integers(64, 2049))
        N = 1 << int(rng.integers(6, 11))
        B = float(10.0 ** rng.uniform(4.0, 6.0))
        T = int(min(64, max(1, math.floor(B / (16 * N)))))
        E = int(math.ceil(B / (N * T)))
        out.append(Problem(dim=d, n_max=n_max, n_sequences=N, tours_per_epoch=T,
                           epochs=E, seed=1000 + i, stream=i))
    return out


@dataclass(frozen=True)
class Job:
    arrival_s: float
    problem: Problem
    target_rel_err: float
    tour_cap: int


def served_arrivals(seed: int = 5, rate_per_s: float = 50.0, duration_s: float = 60.0,
                    n_sequences: int = 256, tours_per_epoch: int = 16,
                    target_rel_err: float = 1e-3, tour_cap: int = 1_000_000):
    """A Poisson stream of sampling jobs: d in {2, 3}, n_max uniform in [50, 2000]."""
    rng = np.random.default_rng(seed)
    t, jobs, i = 0.0, [], 0
    while True:
        t += float(rng.exponential(1.0 / rate_per_s))
        if t >= duration_s:
            break
        d = int(rng.integers(2, 4))
        n_max = int(rng.integers(50, 2001))
        p = Problem(dim=d, n_max=n_max, n_sequences=n_sequences, tours_per_epoch=tours_per_epoch,
                    epochs=max(1, tour_cap // (n_sequences * tours_per_epoch)),
                    seed=5_000_000 + i, stream=i)
        jobs.append(Job(arrival_s=t, problem=p, target_rel_err=target_rel_err, tour_cap=tour_cap))
        i += 1
    return jobs
