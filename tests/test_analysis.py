"""The analysis layer (T_M of eqn (9), the eqn-(16) ratio fit and its band
width E, the mean and geometric combinations) against closed forms."""
import math

import numpy as np

import oracle
from paper_2002_03000_amd import analysis


def _model_logc(n_max, log_mu, gamma, c, log_c1=math.log(4.0)):
    # log c_n built so that log(c_{n+1}/c_n) is exactly the eqn-(16) model
    out = np.zeros(n_max + 1)
    out[1] = log_c1
    for n in range(1, n_max):
        out[n + 1] = out[n] + log_mu + (gamma - 1) * math.log1p(1.0 / n) + c / (n * n)
    return out


def test_ratio_fit_recovers_an_exact_model():
    lc = _model_logc(400, 0.97, 43 / 32, 0.05)
    f = analysis.ratio_fit(lc)
    assert abs(f["log_mu"] - 0.97) < 1e-10 and abs(f["gamma"] - 43 / 32) < 1e-8 and abs(f["c"] - 0.05) < 1e-8
    assert f["E"] < 1e-10 and f["points"] == 399
    g = analysis.ratio_fit(lc, log_mu=0.97)
    assert abs(g["gamma"] - 43 / 32) < 1e-10 and abs(g["c"] - 0.05) < 1e-10 and g["mu"] == math.exp(0.97)


def test_band_width_is_the_rms_residual():
    rng = np.random.default_rng(3)
    lc = _model_logc(20001, 1.5441, 1.157, -0.2)
    sigma = 0.01
    noisy = lc.copy()
    noisy[1:] += np.cumsum(rng.normal(0.0, sigma, len(lc) - 1))   # ratios get iid N(0, sigma^2)
    f = analysis.ratio_fit(noisy)
    assert abs(f["E"] / sigma - 1) < 0.03
    assert abs(f["log_mu"] - 1.5441) < 5e-3


def test_ratio_fit_on_exact_counts_is_near_the_growth_constant():
    c = oracle.saw_counts(2, 20).astype(np.float64)
    lc = np.log(np.where(c > 0, c, 1.0))
    f = analysis.ratio_fit(lc, n_min=4)
    assert abs(f["mu"] - 2.638158) < 0.03


def test_total_abs_error():
    a = np.array([0.0, 1.0, 2.0, 3.0, 4.0])
    assert analysis.total_abs_error(a, a) == 0.0
    assert abs(analysis.total_abs_error(a, a + 0.25) - 0.25) < 1e-15
    b = a.copy()
    b[2] += 0.4
    b[4] -= 0.8
    assert abs(analysis.total_abs_error(a, b) - (0.4 + 0.8) / 4) < 1e-15
    assert abs(analysis.total_abs_error(a, b, M=2) - 0.2) < 1e-15


def test_mean_and_geometric_combinations():
    x = np.log(np.array([[2.0, 1e300], [8.0, 1e302]]))
    m = analysis.combine_mean(x)
    assert abs(m[0] - math.log(5.0)) < 1e-14
    assert abs(m[1] - (math.log(1e300) + math.log(50.5))) < 1e-12
    g = analysis.combine_geometric(x)
    assert abs(g[0] - math.log(4.0)) < 1e-14


def _paper_blocks():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_independent_runs.txt")
    blocks, cur = {}, None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("block"):
            _, name, how, printed, dec = line.split()
            cur = blocks[name] = {"how": how, "printed": float(printed), "decimals": int(dec), "x": [], "w": []}
        else:
            x, w = line.split()
            cur["x"].append(float(x))
            cur["w"].append(float(w))
    return blocks


def test_combinations_reproduce_the_papers_printed_values():
    # the paper's own worked examples (Sec. 3.3, eqns (18)-(24)): combining its
    # printed per-run estimates gives its printed combined values
    blocks = _paper_blocks()
    assert set(blocks) == {"eqn18", "eqn21", "eqn23", "eqn24"}
    assert len(blocks["eqn18"]["x"]) == 7 and len(blocks["eqn21"]["x"]) == 31
    for name, b in blocks.items():
        v = analysis.weighted_average(b["x"], b["w"])
        assert round(v, b["decimals"]) == b["printed"], (name, v)
    # eqn (19)'s average is weighted by iterations: the plain mean of the seven
    # estimates does not give it
    b = blocks["eqn18"]
    assert round(float(np.mean(b["x"])), 9) != b["printed"]


def test_weighted_average_rejects_bad_weights():
    import pytest
    for x, w in (([1.0, 2.0], [1.0]), ([1.0], [-1.0]), ([1.0, 2.0], [0.0, 0.0]), ([], [])):
        with pytest.raises(ValueError):
            analysis.weighted_average(x, w)
    assert analysis.weighted_average([2.0, 5.0], [3.0, 1.0]) == (6.0 + 5.0) / 4.0


def test_weighted_geometric_combination():
    x = np.log(np.array([[2.0, 10.0], [8.0, 1e-300]]))
    g = analysis.combine_geometric(x, weights=[3.0, 1.0])
    assert abs(g[0] - (3 * math.log(2.0) + math.log(8.0)) / 4) < 1e-15
    assert abs(g[1] - (3 * math.log(10.0) + math.log(1e-300)) / 4) < 1e-12
    assert np.array_equal(analysis.combine_geometric(x, weights=[1.0, 1.0]), analysis.combine_geometric(x))


def test_extrapolation_in_inverse_powers_of_the_cutoff():
    n = np.array([10.0, 20.0, 40.0, 80.0, 160.0])
    for theta in (1.0, 0.5, 2.0):
        g, se, b = analysis.extrapolate_inverse(n, 1.157 + 0.3 * n ** -theta, theta=theta)
        assert abs(g - 1.157) < 1e-12 and abs(b - 0.3) < 1e-10 and se < 1e-10
    # the wrong variable leaves a bias
    g, _, _ = analysis.extrapolate_inverse(n, 1.157 + 0.3 / np.sqrt(n), theta=1.0)
    assert abs(g - 1.157) > 1e-3


def _model_corrected(n_max, log_mu, gamma, c, d, p):
    out = np.zeros(n_max + 1)
    out[1] = math.log(6.0)
    for n in range(1, n_max):
        out[n + 1] = out[n] + log_mu + (gamma - 1) * math.log1p(1.0 / n) + c / (n * n) + d / n ** p
    return out


def test_gamma_extrapolation_against_the_cutoff():
    # exact eqn-(16) data: every cut-off gives gamma, so does the limit
    lc = _model_logc(5000, 1.544, 1.157, -0.1)
    r = analysis.gamma_nmin_extrapolation(lc, [10, 20, 40, 80])
    assert all(abs(g - 1.157) < 1e-8 for _, g in r["fits"]) and abs(r["gamma"] - 1.157) < 1e-8
    r2 = analysis.gamma_nmin_extrapolation(lc, [10, 20, 40, 80], log_mu=1.544)
    assert abs(r2["gamma"] - 1.157) < 1e-8
    # a correction d / n^1.5 the model leaves out biases each fit by about
    # n_min^-0.5; extrapolating in n_min^-0.5 removes most of it
    lc = _model_corrected(20000, 1.544, 1.157, -0.1, 0.8, 1.5)
    r = analysis.gamma_nmin_extrapolation(lc, [40, 80, 160, 320, 640], theta=0.5)
    best_single = min(abs(g - 1.157) for _, g in r["fits"])
    assert abs(r["gamma"] - 1.157) < best_single / 3
    assert r["theta"] == 0.5 and len(r["fits"]) == 5
