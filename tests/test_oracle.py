"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them compares the oracle with
itself: the references are exact enumeration, the Rosenbluth counting theorem
(Sec. 1, eqn (3)), exact small-n values, published Philox vectors, rocRAND's
Philox, statistical unbiasedness of the sample average (eqn (4)) and the
flat-histogram property of flatPERM (Sec. 2).
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _saw_golden():
    out = {2: {}, 3: {}}
    with open(os.path.join(GOLDEN, "saw_counts.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            d, n, c = line.split()
            out[int(d)][int(n)] = int(c)
    return out


SAW = _saw_golden()


def _exact(dim, n_max):
    return np.array([SAW[dim][n] for n in range(n_max + 1)], dtype=np.float64)


# --------------------------------------------------------------------------
# Exact counts and the counting theorem (Sec. 1, eqns (1)-(3))
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dim,n_max", [(2, 20), (3, 13)])
def test_brute_force_counts_match_literature(dim, n_max):
    c = oracle.saw_counts(dim, n_max)
    assert [int(x) for x in c] == [SAW[dim][n] for n in range(n_max + 1)]


def test_small_counts_closed_forms():
    # c_1 = 2d, c_2 = 2d(2d-1), c_3 = 2d(2d-1)^2; c_4 subtracts the 2d(2d-2)
    # four-step walks that would close a unit square onto the origin.
    for d in (2, 3):
        c = oracle.saw_counts(d, 4)
        q = 2 * d
        assert int(c[1]) == q
        assert int(c[2]) == q * (q - 1)
        assert int(c[3]) == q * (q - 1) ** 2
        assert int(c[4]) == q * (q - 1) ** 3 - q * (q - 2)


@pytest.mark.parametrize("dim,n_max", [(2, 13), (3, 9)])
def test_forced_choice_drive_counts_every_walk_once(dim, n_max):
    # Every chain the sampler's scan admits is a SAW and every SAW is reached
    # exactly once; W(S) equals prod a_+ exactly (eqn (2)), hence
    # sum_S Pr(S) W(S) = #chains = c_n (eqn (3)).
    cnt, bad, _ = oracle.forced_enumerate(dim, n_max)
    assert bad == 0
    assert [int(x) for x in cnt] == [SAW[dim][n] for n in range(n_max + 1)]


def _xf_exact(m, e):
    from fractions import Fraction
    return Fraction(float(m)) * (Fraction(2) ** int(e))


def _round_xf(x):
    """Correctly rounded extended-range number (m in [0.5, 1), e) of a Fraction."""
    from fractions import Fraction
    if x == 0:
        return 0.0, 0
    k = x.numerator.bit_length() - x.denominator.bit_length()
    while x / (Fraction(2) ** k) >= 1:
        k += 1
    while x / (Fraction(2) ** k) < Fraction(1, 2):
        k -= 1
    m = float(x / (Fraction(2) ** k))     # Fraction -> float rounds to nearest even
    if m == 1.0:
        m, k = 0.5, k + 1
    return m, k


@pytest.mark.parametrize("op", ["add", "mul", "div"])
def test_extended_range_operations_are_correctly_rounded(op):
    # Weights are m * 2^e with an FP64 mantissa; every operation must equal the
    # exact operation on the represented values, rounded to 53 bits.
    rng = np.random.default_rng({"add": 1, "mul": 2, "div": 3}[op])
    n = 3000
    am, ae = oracle.xf_from_float(rng.uniform(0.5, 1.0, n))
    ae = ae + rng.integers(-3000, 3000, n).astype(np.int32)
    bm, be = oracle.xf_from_float(rng.uniform(0.5, 1.0, n))
    # exponent gaps from 0 to beyond the 63-binade cut-off, both signs
    be = ae + rng.integers(-90, 90, n).astype(np.int32)
    be[:50] = ae[:50]
    k = rng.integers(1, 2 ** 32, n).astype(np.float64)
    k[:100] = rng.integers(1, 7, 100)
    om, oe = oracle.xf_apply(op, am, ae, bm, be, k)
    for i in range(n):
        a = _xf_exact(am[i], ae[i])
        if op == "add":
            x = a + _xf_exact(bm[i], be[i])
        elif op == "mul":
            x = a * int(k[i])
        else:
            from fractions import Fraction
            x = a / Fraction(int(k[i]))
        assert (om[i], int(oe[i])) == _round_xf(x), (op, i)


def test_extended_range_zero_and_ratio():
    om, oe = oracle.xf_apply("add", [0.0], [0], [0.75], [12])
    assert (om[0], oe[0]) == (0.75, 12)
    om, oe = oracle.xf_apply("add", [0.75], [12], [0.0], [0])
    assert (om[0], oe[0]) == (0.75, 12)
    # ratio: ordinary double of a / b, exponent gap clamped at +-1000
    assert oracle.xf_ratio(0.75, 10, 0.5, 9) == 3.0
    assert oracle.xf_ratio(0.5, -5000, 0.5, 0) == 0.0
    assert oracle.xf_ratio(0.0, 0, 0.5, 3) == 0.0


# --------------------------------------------------------------------------
# Philox4x32-10 (the counter-based generator of the RNG contract)
# --------------------------------------------------------------------------

def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        got = oracle.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in got] == v[6:10]


_ROCRAND_PROG = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long off = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    unsigned a = e(), b = e(), c = e(), d = e();
    printf("%08x %08x %08x %08x\n", a, b, c, d);
  }
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc to build the rocRAND host check")
def test_philox_matches_rocrand_host_engine():
    # rocRAND's philox4x32_10 engine, executed on the host: seed -> key,
    # subsequence -> counter words 2,3, offset/4 -> counter words 0,1.
    rng = np.random.default_rng(7)
    rows = []
    for _ in range(200):
        c = rng.integers(0, 2 ** 32, size=4, dtype=np.uint64)
        c[1] %= 2 ** 30          # keeps 4 * offset inside 64 bits
        k = rng.integers(0, 2 ** 32, size=2, dtype=np.uint64)
        rows.append((c, k))
    rows.append((np.array([5, 0, 17, 3], dtype=np.uint64), np.array([1, 0], dtype=np.uint64)))
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "rr.cpp")
        exe = os.path.join(td, "rr")
        with open(src, "w") as f:
            f.write(_ROCRAND_PROG)
        subprocess.run(["hipcc", "-O1", src, "-o", exe], check=True, capture_output=True)
        inp = "\n".join(" ".join("%08x" % int(x) for x in list(c) + list(k)) for c, k in rows)
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for (c, k), line in zip(rows, out):
        want = [int(x, 16) for x in line.split()]
        got = oracle.philox4x32_10(c.astype(np.uint32), k.astype(np.uint32))
        assert [int(x) for x in got] == want


# --------------------------------------------------------------------------
# The occupancy set behind a_+
# --------------------------------------------------------------------------

def test_occupancy_set_against_python_set():
    rng = np.random.default_rng(3)
    n = 20000
    ops = rng.integers(0, 3, size=n)
    pts = rng.integers(-6, 7, size=(n, 3))
    got, count = oracle.set_selftest(ops, pts, max_items=2200)
    ref, want = set(), []
    for op, p in zip(ops, map(tuple, pts)):
        if op == 0:
            ref.add(p)
        elif op == 1:
            ref.discard(p)
        else:
            want.append(int(p in ref))
    assert got.tolist() == want
    assert count == len(ref)


# --------------------------------------------------------------------------
# Exact consequences of the construction (Sec. 1, Sec. 2)
# --------------------------------------------------------------------------

def _cn_hat(o):
    return np.exp(oracle.xf_log(o.G) - np.log(float(o.MG[0])))


def _cn_exact_ratio(o, n):
    """G_n / M_G as an exact rational."""
    from fractions import Fraction
    return _xf_exact(o.G["m"][n], o.G["e"][n]) / Fraction(int(o.MG[0]))


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("N,T,epochs,seed", [(1, 500, 1, 1), (7, 20, 3, 5), (16, 3, 4, 11)])
def test_lengths_up_to_three_are_exact(dim, N, T, epochs, seed):
    # For n <= 3 every walk has the same weight 2d(2d-1)^(n-1) (no endpoint can
    # touch an earlier site before n = 4), so r = 1 exactly and c_1..c_3 come out
    # exact for every seed, sequence count and epoch schedule.
    o = oracle.Oracle(dim, 12, N, seed, step_cap=10 ** 6)
    for _ in range(epochs):
        assert o.run_tours(T) is False
        o.merge_epoch()
    q = 2 * dim
    assert _cn_exact_ratio(o, 0) == 1
    assert _cn_exact_ratio(o, 1) == q
    assert _cn_exact_ratio(o, 2) == q * (q - 1)
    assert _cn_exact_ratio(o, 3) == q * (q - 1) ** 2
    assert int(o.MG[0]) == N * T * epochs
    assert int(o.HG[0]) == N * T * epochs


@pytest.mark.parametrize("dim,seed", [(2, 1), (2, 9), (3, 4)])
def test_first_tour_is_a_rosenbluth_walk(dim, seed):
    # In the first tour of a lone sequence every running average is the walk's
    # own weight (eqn (6) with the weight included), so r = 1, no copies and no
    # pruning: the tour is exactly the Rosenbluth walk drawn from the same numbers.
    a = oracle.Oracle(dim, 60, 1, seed, step_cap=10000)
    assert a.run_tours(1) is False
    b = oracle.Oracle(dim, 60, 1, seed, mode=oracle.MODE_ROSENBLUTH)
    b.run_tours(1)
    assert np.array_equal(a.L["m"], b.L["m"]) and np.array_equal(a.L["e"], b.L["e"])
    assert np.array_equal(a.H, b.H)
    assert a.stats["enrich"][0] == 0 and a.stats["prunes"][0] == 0
    assert a.stats["digest"][0] == b.stats["digest"][0]


def _fnv1a32(data):
    # FNV-1a with 32-bit state, from its published definition
    h = 0x811C9DC5
    for b in data:
        h = ((h ^ b) * 0x01000193) & 0xFFFFFFFF
    return h


@pytest.mark.parametrize("dim,seed,tours", [(2, 3, 1), (2, 5, 2), (3, 7, 3)])
def test_trajectory_digest_is_fnv1a_32_of_the_steps(dim, seed, tours):
    # The published test vector pins the constants; with n_max = 1 every tour is
    # one growth from the origin (no decision is due at n = 0), whose byte is
    # dir | a_+ << 3 with a_+ = 2d, so the digest is FNV-1a 32 of one such byte
    # per tour, for some sequence of directions.
    assert _fnv1a32(b"") == 0x811C9DC5 and _fnv1a32(b"a") == 0xE40C292C
    o = oracle.Oracle(dim, 1, 1, seed)
    o.run_tours(tours)
    assert int(o.stats["steps"][0]) == tours
    import itertools
    byte = lambda d: d | ((2 * dim) << 3)
    candidates = {_fnv1a32(bytes(byte(d) for d in dirs))
                  for dirs in itertools.product(range(2 * dim), repeat=tours)}
    assert int(o.stats["digest"][0]) in candidates


@pytest.mark.parametrize("dim,n_max,seed,tours", [(2, 20, 1, 3000), (2, 40, 2, 2000), (3, 30, 3, 2000)])
def test_iterative_matches_recursive_description(dim, n_max, seed, tours):
    o = oracle.Oracle(dim, n_max, 1, seed)
    o.run_tours(tours)
    L, H = oracle.plain_recursive(dim, n_max, seed, tours)
    assert np.array_equal(o.L[0]["m"], L["m"]) and np.array_equal(o.L[0]["e"], L["e"])
    assert np.array_equal(o.H[0], H)


def test_thread_count_does_not_change_results():
    runs = []
    for th in (1, 3, 8):
        o = oracle.Oracle(3, 40, 19, 77, threads=th)
        for _ in range(2):
            o.run_tours(5)
            o.merge_epoch()
        runs.append((o.G["m"].copy(), o.G["e"].copy(), o.HG.copy(), o.stats.copy()))
    for gm, ge, h, s in runs[1:]:
        assert np.array_equal(gm, runs[0][0]) and np.array_equal(ge, runs[0][1])
        assert np.array_equal(h, runs[0][2])
        assert np.array_equal(s, runs[0][3])


def test_merge_is_the_aligned_pairwise_tree():
    # Values chosen so that the summation order is visible in the rounding:
    # 2^53 + 1 + 1 + 1 + 1 summed as the tree over 8 leaves (3 of them +0).
    o = oracle.Oracle(2, 2, 5, 1)
    vals = [2.0 ** 53, 1.0, 1.0, 1.0, 1.0]
    m, e = oracle.xf_from_float(vals)
    o.L["m"][:, 1] = m
    o.L["e"][:, 1] = e
    o.m[:] = 1
    o.merge_epoch()
    big = 2.0 ** 53
    want = ((big + 1.0) + (1.0 + 1.0)) + ((1.0 + 0.0) + (0.0 + 0.0))
    got = math.ldexp(o.G["m"][1], int(o.G["e"][1]))
    assert got == want
    assert got != (((big + 1.0) + 1.0) + 1.0) + 1.0
    assert int(o.MG[0]) == 5
    assert not o.L["m"].any() and not o.H.any() and not o.m.any()


def test_step_cap_stops_a_sequence():
    o = oracle.Oracle(2, 100, 2, 3, step_cap=50)
    assert o.run_tours(100) is True
    assert (o.stats["capped"] == 1).all()
    assert (o.stats["steps"] == 50).all()


# --------------------------------------------------------------------------
# Statistical pins: <W_n>_M is an unbiased estimate of c_n (eqns (3), (4))
# --------------------------------------------------------------------------

def _replicas(dim, n_max, N, T, epochs, seeds, mode=oracle.MODE_SHARED):
    est = []
    for sd in seeds:
        o = oracle.Oracle(dim, n_max, N, sd, mode=mode)
        for _ in range(epochs):
            o.run_tours(T)
            o.merge_epoch()
        est.append(np.exp(o.log_estimates()))
    return np.array(est)


@pytest.mark.parametrize("case", [
    dict(dim=2, n_max=14, N=1, T=2000, epochs=1, mode=oracle.MODE_SHARED),
    dict(dim=3, n_max=10, N=1, T=2000, epochs=1, mode=oracle.MODE_SHARED),
    dict(dim=2, n_max=14, N=8, T=25, epochs=10, mode=oracle.MODE_SHARED),
    dict(dim=3, n_max=10, N=8, T=25, epochs=10, mode=oracle.MODE_SHARED),
    dict(dim=2, n_max=14, N=4, T=50, epochs=10, mode=oracle.MODE_INDEPENDENT),
    dict(dim=2, n_max=14, N=1, T=4000, epochs=1, mode=oracle.MODE_ROSENBLUTH),
])
def test_sample_average_is_unbiased(case):
    seeds = range(1000, 1096)
    est = _replicas(case["dim"], case["n_max"], case["N"], case["T"], case["epochs"], seeds, case["mode"])
    exact = _exact(case["dim"], case["n_max"])
    mean = est.mean(axis=0)
    se = est.std(axis=0, ddof=1) / math.sqrt(len(seeds))
    # lengths whose estimate does not vary between seeds are exact (n <= 3)
    fixed = se < 1e-12 * exact
    assert np.all(np.abs(mean[fixed] / exact[fixed] - 1.0) < 1e-12)
    z = (mean - exact)[~fixed] / se[~fixed]
    assert np.all(np.abs(z) < 4.5), z
    # and the pooled estimate is close in relative terms
    assert np.all(np.abs(mean / exact - 1.0) < 0.02)


def test_plain_flatperm_c1_budget():
    # Plain flatPERM, one sequence, n_max = 20, 10^5 tours, seed 1: every
    # estimate within 1% of the exact count, n <= 3 exact, histogram flat.
    o = oracle.Oracle(2, 20, 1, 1)
    o.run_tours(100000)
    o.merge_epoch()
    c = _cn_hat(o)
    exact = _exact(2, 20)
    assert np.all(np.abs(c / exact - 1.0) < 1e-2)
    for n in range(4):
        assert _cn_exact_ratio(o, n) == int(exact[n])
    flat = o.HG / float(o.MG[0])
    assert flat.min() > 0.9 and flat.max() < 1.1


def test_group_sums_and_error_estimate_pinned():
    # group k folds the weights recorded at n_max by sequences s = k (mod 16):
    # against exact rational sums of the same records, the tour counts against
    # the pooled count, and the estimate against the statistics module
    import statistics
    from fractions import Fraction
    N, n_max = 40, 12
    o = oracle.Oracle(2, n_max, N, 77, group_stats=True)
    exact = [Fraction(0)] * 16
    adds = [0] * 16
    for T in (1, 1, 2, 4, 3):
        o.run_tours(T)
        for s in range(N):
            rec = o.L[s, n_max]
            exact[s % 16] += Fraction(float(rec["m"])) * Fraction(2) ** int(rec["e"])
            adds[s % 16] += 1
        o.merge_epoch()
    assert int(o.gtours.sum()) == int(o.MG[0])
    for k in range(16):
        got = Fraction(float(o.gsum[k]["m"])) * Fraction(2) ** int(o.gsum[k]["e"])
        assert exact[k] > 0
        # one rounding per addition, each at most half an ulp (2^-53 relative)
        assert abs(got / exact[k] - 1) <= (adds[k] + 5) * Fraction(1, 2 ** 53)
    g = [float(exact[k] / int(o.gtours[k])) * 2.0 ** 0 for k in range(16)]
    ref = statistics.stdev(g) / (4 * statistics.mean(g))
    assert abs(o.error_estimate() / ref - 1) < 1e-12
    # an empty group leaves the estimate undefined
    assert oracle.Oracle(2, n_max, 8, 1, group_stats=True).error_estimate() == math.inf


@pytest.mark.parametrize("dim,n_max", [(2, 10), (3, 7)])
def test_r2_of_every_chain_matches_brute_force(dim, n_max):
    # the endpoint coordinates the oracle's walk carries give the same sum of
    # R^2 over all walks as an independent grid enumeration
    cnt, bad, r2 = oracle.forced_enumerate(dim, n_max)
    c, r2_exact = oracle.saw_counts_r2(dim, n_max)
    assert np.array_equal(cnt, c) and bad == 0
    assert np.array_equal(r2, r2_exact)
    # textbook values: <R^2_1> = 1, <R^2_2> = (4 + 2 (2d - 2)) / (2d - 1)
    assert r2_exact[1] == c[1]
    assert r2_exact[2] * (2 * dim - 1) == c[2] * (4 + 2 * (2 * dim - 2))


def test_ratio_estimator_exact_at_one_step_and_unbiased():
    # <R^2_1> = 1 for every sample (all one-step walks have R^2 = 1)
    n_max = 10
    c, r2 = oracle.saw_counts_r2(2, n_max)
    exact = r2.astype(np.float64) / c.astype(np.float64)
    ests = []
    for seed in range(64):
        o = oracle.Oracle(2, n_max, 8, 500 + seed, observables=True)
        for T in (1, 1, 2, 4, 8):
            o.run_tours(T)
            o.merge_epoch()
        v = o.observable_r2()
        assert v[1] == 1.0
        ests.append(v)
    ests = np.array(ests)
    mean = ests.mean(axis=0)
    se = ests.std(axis=0, ddof=1) / np.sqrt(len(ests))
    for n in range(2, n_max + 1):
        assert abs(mean[n] - exact[n]) < 4.5 * se[n] + 1e-9, (n, mean[n], exact[n], se[n])


def test_observables_do_not_change_the_walks():
    a = oracle.Oracle(3, 30, 10, 77, observables=True)
    b = oracle.Oracle(3, 30, 10, 77)
    for o in (a, b):
        for T in (1, 1, 2):
            o.run_tours(T)
            o.merge_epoch()
    assert np.array_equal(a.G["m"], b.G["m"]) and np.array_equal(a.stats["digest"], b.stats["digest"])


def test_algorithm_1_sequences_do_not_interact():
    # Algorithm 1 (no sharing): sequence s of an N-sequence run is the same run
    # whatever N is, and sequence 0 is plain flatPERM with one sequence
    sched = (1, 1, 2, 4, 8)
    runs = {}
    for N in (1, 3, 8):
        o = oracle.Oracle(2, 30, N, 4242, mode=oracle.MODE_INDEPENDENT)
        for T in sched:
            o.run_tours(T)
            o.merge_epoch()
        runs[N] = o
    plain = oracle.Oracle(2, 30, 1, 4242)
    for T in sched:
        plain.run_tours(T)
        plain.merge_epoch()
    for s in range(3):
        for f in ("m", "e"):
            assert np.array_equal(runs[3].G[f][s], runs[8].G[f][s])
        assert np.array_equal(runs[3].HG[s], runs[8].HG[s])
        assert np.array_equal(runs[3].stats["digest"][s], runs[8].stats["digest"][s])
    for f in ("m", "e"):
        assert np.array_equal(runs[8].G[f][0], runs[1].G[f][0])
        assert np.array_equal(runs[1].G[f][0], plain.G[f])
    assert np.array_equal(runs[1].HG[0], plain.HG)
