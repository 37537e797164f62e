"""The analysis layer (T_M of eqn (9), the eqn-(15) ratio fit and its band
width E, the mean and geometric combinations) against closed forms."""
import math

import numpy as np

import oracle
from paper_2002_03000_amd import analysis


def _model_logc(n_max, log_mu, gamma, c, log_c1=math.log(4.0)):
    # log c_n built so that log(c_{n+1}/c_n) is exactly the eqn-(15) model
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
