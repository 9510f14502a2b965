"""Pin the score-function gradient against the analytic birth-death derivative.

Birth-death 0 -> A (k1), A -> 0 (k2 A), x0 = 0: X_T ~ Poisson(m),
m = (k1/k2)(1 - exp(-k2 T)); d m/d log k1 = m, d m/d log k2 = -m + k1 T exp(-k2 T),
and d E[X^2]/d theta = (1 + 2m) d m/d theta.
"""
import math

import numpy as np

import oracle
from oracle.score import score_grad
from paper_2103_00405_amd import workloads as W


def _analytic(k1, k2, T):
    m = k1 / k2 * (1 - math.exp(-k2 * T))
    dm = np.array([m, -m + k1 * T * math.exp(-k2 * T)])
    return m, dm, (1 + 2 * m) * dm


def test_analytic_values():
    m, dm, dm2 = _analytic(50.0, 1.0, 2.0)
    assert abs(m - 43.233236) < 1e-6
    assert np.allclose(dm, [43.233236, -29.699708], atol=1e-6)
    assert np.allclose(dm2, [3781.4586, -2597.7286], atol=1e-3)


def test_score_gradient_birth_death():
    k1, k2, T = 50.0, 1.0, 2.0
    o = oracle.simulate(W.birth_death(k1, k2), np.array([0], np.int32), T, [T], 11, 60000)
    X = o["x_final"][:, 0].astype(float)
    m, dm, dm2 = _analytic(k1, k2, T)
    # 4 comparisons (2 functions x 2 channels) at family level 0.01, Bonferroni
    z = 3.0233
    for f, ref in ((X, dm), (X * X, dm2)):
        g, se = score_grad(f, o["n"], o["T"])
        assert np.all(np.abs(g - ref) < z * se), (g, ref, se)
    # the baseline does not bias the estimate and reduces its spread
    g0, se0 = score_grad(X, o["n"], o["T"], baseline=False)
    g1, se1 = score_grad(X, o["n"], o["T"], baseline=True)
    assert np.all(se1 < se0)


def test_score_gradient_catches_wrong_sign():
    k1, k2, T = 50.0, 1.0, 2.0
    o = oracle.simulate(W.birth_death(k1, k2), np.array([0], np.int32), T, [T], 12, 30000)
    X = o["x_final"][:, 0].astype(float)
    _, dm, _ = _analytic(k1, k2, T)
    g, se = score_grad(X, o["T"], o["n"])          # T - n instead of n - T
    assert np.any(np.abs(g - dm) > 10 * se)
