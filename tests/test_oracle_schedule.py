"""Pins for piecewise-constant rate constants (the time-dependent rates of the
paper's discussion, Eq. 28, solved piece by piece): closed-form laws of
time-inhomogeneous birth and birth-death processes, the random time-change
identities, and exact identities of the schedule's own logic.

Every pin runs in both forms of the method: the eager one (all clocks advanced
at every firing) and the lazy one (clocks kept in internal time and brought up
to date when a propensity changes, a channel fires or a breakpoint is
crossed)."""
import functools
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2103_00405_amd import workloads as W

P_MIN = 1e-4


@pytest.fixture(autouse=True, params=[False, True], ids=["eager", "lazy"])
def lazy(request, monkeypatch):
    monkeypatch.setattr(oracle, "simulate", functools.partial(oracle.simulate,
                                                              lazy=request.param))
    return request.param


def _chisq(samples, support, pmf):
    obs = np.array([np.sum(samples == v) for v in support], dtype=float)
    exp = np.asarray(pmf) * samples.size
    keep = exp >= 5
    o = np.append(obs[keep], samples.size - obs[keep].sum())
    e = np.append(exp[keep], samples.size - exp[keep].sum())
    e *= o.sum() / e.sum()
    return stats.chisquare(o, e).pvalue


def test_pure_birth_piecewise_poisson_and_clock():
    """Rate 10 on [0,1), 0 on [1,2), 30 on [2,3): X(t) ~ Poisson(int_0^t c)
    and the internal time at t_end is that integral."""
    o = oracle.simulate(W.pure_birth(10.0), [0], 3.0, [0.5, 1.5, 2.5, 3.0], 1, 20000,
                        schedule=([1.0, 2.0], [[0.0], [30.0]]))
    sup = np.arange(0, 90)
    for g, m in enumerate((5.0, 10.0, 25.0, 40.0)):
        assert _chisq(o["samples"][:, g, 0], sup, stats.poisson.pmf(sup, m)) > P_MIN
    assert np.allclose(o["T"][:, 0], 40.0, rtol=1e-13, atol=0)
    assert (o["status"] == oracle.STATUS_OK).all()


def test_birth_death_with_a_rate_switch():
    """Birth 50 then 10 from t = 1, death 1 per molecule, x0 = 0: X(t) is
    Poisson with m' = k1(t) - m, m(t) = 50 (1 - e^-t) up to t = 1 and
    10 + (m(1) - 10) e^-(t-1) after."""
    net = W.birth_death(50.0, 1.0)
    grid = [0.5, 1.0, 1.5, 3.0]
    o = oracle.simulate(net, [0], 3.0, grid, 2, 20000, schedule=([1.0], [[10.0, 1.0]]))
    m1 = 50.0 * (1 - math.exp(-1.0))
    sup = np.arange(0, 120)
    for g, t in enumerate(grid):
        m = 50.0 * (1 - math.exp(-t)) if t <= 1.0 else 10.0 + (m1 - 10.0) * math.exp(-(t - 1.0))
        X = o["samples"][:, g, 0]
        assert _chisq(X, sup, stats.poisson.pmf(sup, m)) > P_MIN
        assert abs(X.mean() - m) < 4 * math.sqrt(m / X.size)


def test_random_time_change_martingale_with_schedule():
    """n_k - T_k has mean 0 and variance E[T_k] under time-varying rates too."""
    w = W.lv_small(4000)
    rates = np.array([[2.0, 0.005, 0.5], [0.5, 0.02, 2.0]])
    o = oracle.simulate(w.net, w.x0, 6.0, [6.0], 3, 4000, schedule=([2.0, 4.0], rates))
    S = o["n"].astype(float) - o["T"]
    for k in range(3):
        ET = o["T"][:, k].mean()
        assert abs(S[:, k].mean()) < 4.5 * math.sqrt(ET / S.shape[0])
        assert abs(S[:, k].var() / ET - 1.0) < 0.15


def test_rates_off_then_on_is_not_absorbed():
    o = oracle.simulate(W.pure_birth(0.0), [0], 4.0, [1.0, 4.0], 4, 20000,
                        schedule=([1.0], [[5.0]]))
    assert (o["samples"][:, 0, 0] == 0).all()
    sup = np.arange(0, 40)
    assert _chisq(o["x_final"][:, 0], sup, stats.poisson.pmf(sup, 15.0)) > P_MIN
    assert (o["status"] == oracle.STATUS_OK).all()
    # zero rates in the last piece: absorbed from there on
    o = oracle.simulate(W.pure_birth(3.0), [0], 4.0, [4.0], 5, 200, schedule=([1.0], [[0.0]]))
    assert (o["status"] == oracle.STATUS_ABSORBED).all()
    assert np.allclose(o["T"][:, 0], 3.0, rtol=1e-15)


def test_schedule_identities():
    w = W.lv_small(64)
    base = oracle.simulate(w.net, w.x0, 5.0, [2.0, 5.0], 7, 64)
    # breakpoints at or after t_end are never reached: identical bits
    late = oracle.simulate(w.net, w.x0, 5.0, [2.0, 5.0], 7, 64,
                           schedule=([5.0, 9.0], [[1.0, 1.0, 1.0], [2.0, 2.0, 2.0]]))
    for k in ("samples", "n", "T", "seq_hash", "t_last"):
        assert np.array_equal(base[k], late[k]), k
    # a breakpoint that keeps the rates gives the same law (Eq. 5 exactly)
    same = oracle.simulate(w.net, w.x0, 5.0, [2.0, 5.0], 7, 4000,
                           schedule=([1.25], [list(w.net.c)]))
    ref = oracle.simulate(w.net, w.x0, 5.0, [2.0, 5.0], 8, 4000)
    for j in range(2):
        assert stats.ks_2samp(same["samples"][:, 1, j], ref["samples"][:, 1, j]).pvalue > P_MIN
    # breakpoints must increase
    with pytest.raises(RuntimeError):
        oracle.simulate(w.net, w.x0, 5.0, [5.0], 1, 4, schedule=([2.0, 2.0], np.ones((2, 3))))

