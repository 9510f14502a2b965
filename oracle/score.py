"""Score-function (likelihood-ratio) gradient of E[f(X_T)] with respect to
log c_k -- plain numpy reference.  TEST INFRASTRUCTURE ONLY.

For a mass-action network a_k = c_k h_k(X) (Eq. 1), so the log-likelihood of
a path on [0, T] is sum_events log a_mu - sum_k int_0^T a_k ds, and its
derivative in log c_k is n_k - T_k(T): the firing count minus the internal
time of Eq. 15.  With a leave-one-out baseline b_r = (sum f - f_r)/(R - 1),
the estimator is g_k = (1/R) sum_r (f_r - b_r)(n_rk - T_rk), and se_k is the
standard error of the per-path terms.
"""
import numpy as np


def score_grad(f, n, T, baseline=True):
    f = np.asarray(f, dtype=np.float64)
    S = np.asarray(n, dtype=np.float64) - np.asarray(T, dtype=np.float64)
    R = f.shape[0]
    if baseline and R > 1:
        b = (f.sum() - f) / (R - 1)
    else:
        b = np.zeros_like(f)
    y = (f - b)[:, None] * S
    g = y.sum(axis=0) / R
    se = y.std(axis=0, ddof=1) / np.sqrt(R) if R > 1 else np.zeros(S.shape[1])
    return g, se
