"""Analysis of estimates of log c_n (host-side numpy; Sec. 4 of the paper).

* total_abs_error: T_M of eqn (9), the mean over lengths 1..M of
  |log c_n^best - log c_n^est|.
* ratio_fit: the model of eqn (16),
      log(c_{n+1} / c_n) ~ log mu + (gamma - 1) log(1 + 1/n) + c / n^2,
  fitted by linear least squares (three parameters, or two with mu fixed),
  with E, the root of the mean squared residual of the fit, as the width of
  the band the estimates scatter in.
* combine_mean / combine_geometric: the two ways of combining independent
  estimates of c_n (the arithmetic mean of eqn (7), and the geometric mean the
  paper's Table 1 uses; weighted by each run's iterations where the runs
  differ in length, as for the 2D estimate of eqn (17));
* weighted_average: independent simulations' estimates of one quantity (a
  fitted log mu, say) combined with weights proportional to their iterations,
  the combination behind eqn (19) (its seven inputs are eqn (18));
* gamma_nmin_extrapolation: gamma from the three-parameter (or, with log mu
  fixed, two-parameter) fit of eqn (16) restricted to n >= n_min, for several
  cut-offs, extrapolated against n_min to n_min -> infinity (Sec. 4,
  eqns (26) and (27)).
"""
import numpy as np


def total_abs_error(log_best, log_est, M=None):
    """T_M = (1/M) sum_{n=1}^{M} |log c_n^best - log c_n^est| (eqn (9))."""
    log_best = np.asarray(log_best, dtype=np.float64)
    log_est = np.asarray(log_est, dtype=np.float64)
    if M is None:
        M = min(len(log_best), len(log_est)) - 1
    d = np.abs(log_best[1:M + 1] - log_est[1:M + 1])
    return float(d.sum() / M)


def ratio_fit(log_c, n_min=1, n_max=None, log_mu=None):
    """Least-squares fit of eqn (16) to y_n = log c_{n+1} - log c_n for
    n_min <= n < n_max (n_max defaults to the last length).

    Returns a dict with log_mu, mu, gamma, c (the 1/n^2 coefficient), E (the
    root mean squared residual) and the number of points.  With log_mu given,
    mu is held at that value and only gamma and c are fitted."""
    log_c = np.asarray(log_c, dtype=np.float64)
    if n_max is None:
        n_max = len(log_c) - 1
    n = np.arange(n_min, n_max, dtype=np.float64)
    y = log_c[n_min + 1:n_max + 1] - log_c[n_min:n_max]
    x1 = np.log1p(1.0 / n)
    x2 = 1.0 / (n * n)
    if log_mu is None:
        A = np.stack([np.ones_like(n), x1, x2], axis=1)
        coef, *_ = np.linalg.lstsq(A, y, rcond=None)
        lm, g1, c = coef
    else:
        A = np.stack([x1, x2], axis=1)
        coef, *_ = np.linalg.lstsq(A, y - log_mu, rcond=None)
        lm = log_mu
        g1, c = coef
    resid = y - (lm + g1 * x1 + c * x2)
    return {"log_mu": float(lm), "mu": float(np.exp(lm)), "gamma": float(1.0 + g1), "c": float(c),
            "E": float(np.sqrt(np.mean(resid * resid))), "points": int(len(n))}


def combine_mean(log_estimates):
    """log of the arithmetic mean of independent estimates (eqn (7)), per length."""
    L = np.asarray(log_estimates, dtype=np.float64)
    top = np.max(L, axis=0)
    with np.errstate(invalid="ignore"):
        return top + np.log(np.mean(np.exp(L - top), axis=0))


def combine_geometric(log_estimates, weights=None):
    """log of the geometric mean of independent estimates, per length; with
    weights (one per run, e.g. its iterations) the weighted geometric mean."""
    L = np.asarray(log_estimates, dtype=np.float64)
    if weights is None:
        return np.mean(L, axis=0)
    w = np.asarray(weights, dtype=np.float64)
    return np.tensordot(w, L, axes=1) / w.sum()


def weighted_average(values, weights):
    """sum_l w_l x_l / sum_l w_l: independent simulations' estimates x_l of one
    quantity combined with weights w_l proportional to their iterations (the
    longer a run, the smaller its variance), as for eqn (19)."""
    x = np.asarray(values, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    if x.shape != w.shape or x.ndim != 1 or len(x) == 0 or np.any(w < 0) or w.sum() <= 0:
        raise ValueError("one nonnegative weight per value, not all zero")
    return float(np.dot(w, x) / w.sum())


def extrapolate_inverse(n_mins, values, theta=1.0):
    """Linear least squares of values against n_min^-theta: the intercept (the
    limit n_min -> infinity), its standard error and the slope.  Needs three
    or more cut-offs (the error has len - 2 degrees of freedom)."""
    n = np.asarray(n_mins, dtype=np.float64)
    v = np.asarray(values, dtype=np.float64)
    if len(n) < 3 or len(n) != len(v):
        raise ValueError("three or more (n_min, value) pairs")
    A = np.stack([np.ones_like(n), n ** -float(theta)], axis=1)
    coef, *_ = np.linalg.lstsq(A, v, rcond=None)
    resid = v - A @ coef
    s2 = float(resid @ resid) / (len(n) - 2)
    cov = s2 * np.linalg.inv(A.T @ A)
    return float(coef[0]), float(np.sqrt(cov[0, 0])), float(coef[1])


def gamma_nmin_extrapolation(log_c, n_mins, n_max=None, log_mu=None, theta=1.0):
    """gamma of the eqn-(16) fit over n_min <= n < n_max for each cut-off
    n_min, extrapolated linearly in n_min^-theta to n_min -> infinity (eqns
    (26), (27); the paper does not name the variable: theta = 1 by default).
    A correction d / n^(1 + theta) to the ratios that the model leaves out
    biases the fitted gamma by about n_min^-theta, which this removes.  With
    log_mu given the fits have two parameters (gamma and the 1/n^2 term) and
    mu is held at log_mu.

    Returns {"gamma": limit, "gamma_se": its standard error, "slope": the
    coefficient of n_min^-theta, "theta", "fits": [(n_min, gamma), ...]}."""
    fits = [(int(m), ratio_fit(log_c, n_min=int(m), n_max=n_max, log_mu=log_mu)["gamma"]) for m in n_mins]
    g, se, b = extrapolate_inverse([m for m, _ in fits], [v for _, v in fits], theta=theta)
    return {"gamma": g, "gamma_se": se, "slope": b, "theta": float(theta), "fits": fits}
