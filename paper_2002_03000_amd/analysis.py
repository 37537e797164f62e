"""Analysis of estimates of log c_n (host-side numpy; Sec. 4 of the paper).

* total_abs_error: T_M of eqn (9), the mean over lengths 1..M of
  |log c_n^best - log c_n^est|.
* ratio_fit: the model of eqn (15),
      log(c_{n+1} / c_n) ~ log mu + (gamma - 1) log(1 + 1/n) + c / n^2,
  fitted by linear least squares (three parameters, or two with mu fixed),
  with E, the root of the mean squared residual of the fit, as the width of
  the band the estimates scatter in.
* combine_mean / combine_geometric: the two ways of combining independent
  estimates (the arithmetic mean of eqn (7), and the geometric mean the
  paper's Table 1 uses).
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
    """Least-squares fit of eqn (15) to y_n = log c_{n+1} - log c_n for
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


def combine_geometric(log_estimates):
    """log of the geometric mean of independent estimates, per length."""
    return np.mean(np.asarray(log_estimates, dtype=np.float64), axis=0)
