"""Pins for the oracle's lazy form (section 5's dependency-graph updates kept
in internal times: a channel's clock is brought up to date only when its
propensity changes or it fires; the next event is the smallest absolute
next firing time).

It uses the draws of the eager form and samples the same law, so it is tied to
the mathematics the same way: closed-form laws, the chemical master equation,
the random time-change martingale, Eq. 5 and Gillespie's direct method.  Where
the two forms do the same arithmetic (one channel) their bits must agree; on
other networks they differ only in rounding, so their firing sequences agree
on nearly every trajectory and their internal times to rounding level."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2103_00405_amd import workloads as W
from test_oracle_law import P_MIN, _chisq_discrete, _cme_dimer, _nu_dense

KEYS = ("samples", "n", "T", "x_final", "t_last", "status", "seq_hash", "tie_step")


def _lazy(net, x0, t_end, grid, R, seed=1, **kw):
    return oracle.simulate(net, np.asarray(x0, np.int32), t_end, np.asarray(grid, float), seed,
                           R, lazy=True, **kw)


def _eager(net, x0, t_end, grid, R, seed=1, **kw):
    return oracle.simulate(net, np.asarray(x0, np.int32), t_end, np.asarray(grid, float), seed,
                           R, **kw)


@pytest.mark.parametrize("net,x0", [(W.pure_birth(10.0), [0]), (W.pure_death(1.5), [40])])
def test_one_channel_equals_the_eager_form_bit_for_bit(net, x0):
    """With one channel both forms compute gap = (P - T) / a from T = P_prev
    and end with one fma: every output is the same."""
    e = _eager(net, x0, 3.0, [0.5, 1.0, 3.0], 500, seed=4)
    z = _lazy(net, x0, 3.0, [0.5, 1.0, 3.0], 500, seed=4)
    for k in KEYS:
        assert np.array_equal(e[k], z[k]), k


def test_birth_death_law_and_clocks():
    """k1 = 50, k2 = 1, x0 = 0, T = 2: X ~ Poisson(43.233236), E[T_2] =
    56.766764, and the birth channel's clock is 100 on every path."""
    k1, k2, T = 50.0, 1.0, 2.0
    o = _lazy(W.birth_death(k1, k2), [0], T, [0.5, T], 20000, seed=3)
    for g, t in enumerate((0.5, T)):
        m = k1 / k2 * (1 - math.exp(-k2 * t))
        X = o["samples"][:, g, 0]
        sup = np.arange(0, 120)
        assert _chisq_discrete(X, sup, stats.poisson.pmf(sup, m)) > P_MIN
    assert abs(43.233236 - k1 * (1 - math.exp(-T))) < 1e-6
    T2 = o["T"][:, 1]
    assert abs(T2.mean() - 56.766764) < 4.5 * math.sqrt(T2.var() / T2.size)
    assert np.allclose(o["T"][:, 0], k1 * T, rtol=1e-12, atol=0)


def test_pure_death_binomial_and_absorption():
    o = _lazy(W.pure_death(1.0), [50], 40.0, [0.7, 40.0], 20000, seed=4)
    sup = np.arange(0, 51)
    assert _chisq_discrete(o["samples"][:, 0, 0], sup, stats.binom.pmf(sup, 50, math.exp(-0.7))) > P_MIN
    ext = o["status"] == oracle.STATUS_ABSORBED
    assert ext.mean() > 0.99 and (o["n"][ext, 0] == 50).all()


def test_dimerisation_cme():
    """2A <-> B against the master equation (fixes C(A,2) = A(A-1)/2)."""
    o = _lazy(W.dimerisation(0.05, 1.0), [30, 0], 0.8, [0.2, 0.8], 20000, seed=8)
    for g, t in enumerate((0.2, 0.8)):
        p = _cme_dimer(0.05, 1.0, 30, 0, t)
        assert _chisq_discrete(o["samples"][:, g, 1], np.arange(p.size), p) > P_MIN


@pytest.mark.parametrize("which", ["lv", "random"])
def test_martingale_and_eq5(which):
    if which == "lv":
        w = W.lv_small(4000)
        net, x0, t_end = w.net, w.x0, 5.0
    else:
        rng = np.random.default_rng(12)
        net = W.random_network(6, 15, rng)
        x0 = rng.integers(0, 40, size=6).astype(np.int32)
        t_end = 0.3
    o = _lazy(net, x0, t_end, [t_end], 4000, seed=13)
    pred = x0[None, :].astype(np.int64) + o["n"].astype(np.int64) @ _nu_dense(net)
    assert np.array_equal(pred, o["x_final"].astype(np.int64))
    ok = o["status"] <= oracle.STATUS_ABSORBED
    S = o["n"][ok].astype(float) - o["T"][ok]
    R = S.shape[0]
    for k in range(net.M):
        ET = o["T"][ok, k].mean()
        if ET < 1.0:
            continue
        assert abs(S[:, k].mean()) < 4.5 * math.sqrt(ET / R), k
        assert abs(S[:, k].var() - ET) < 6 * ET * math.sqrt(3.0 / R), k


def test_same_law_as_the_direct_method():
    rng = np.random.default_rng(21)
    net = W.random_network(5, 12, rng)
    x0 = rng.integers(5, 50, size=5).astype(np.int32)
    grid = np.array([0.2, 0.4])
    o = _lazy(net, x0, 0.4, grid, 6000, seed=17)
    d = oracle.dm_simulate(net, x0, 0.4, grid, 99, 6000)
    ps = [stats.ks_2samp(o["samples"][:, g, j], d["samples"][:, g, j]).pvalue
          for g in range(2) for j in range(net.N)]
    assert min(ps) * len(ps) > P_MIN


@pytest.mark.parametrize("which", ["lv", "random_small", "random_mid"])
def test_firing_sequences_match_the_eager_form(which):
    """The two forms differ only in rounding: the same channel fires at nearly
    every step of nearly every trajectory, and where the sequences agree the
    internal times agree to rounding level."""
    if which == "lv":
        w = W.lv_small(256)
        net, x0, t_end, grid, R = w.net, w.x0, w.t_end, w.sample_t, 256
    else:
        N, M = (6, 14) if which == "random_small" else (40, 160)
        rng = np.random.default_rng(7 if which == "random_small" else 8)
        net = W.random_network(N, M, rng, logc=(-1.0, 1.0), bimol_scale=0.05)
        x0 = rng.integers(0, 80, size=N).astype(np.int32)
        t_end = float(3000 / W.initial_total_rate(net, x0))
        grid, R = W.uniform_grid(t_end, 11), 128
    e = _eager(net, x0, t_end, grid, R, seed=9)
    z = _lazy(net, x0, t_end, grid, R, seed=9)
    same = e["seq_hash"] == z["seq_hash"]
    assert same.mean() >= 0.95, same.mean()
    assert np.array_equal(e["n"][same], z["n"][same])
    assert np.array_equal(e["x_final"][same], z["x_final"][same])
    rel = np.abs(e["T"][same] - z["T"][same]) / np.maximum(np.abs(e["T"][same]), 1.0)
    assert rel.max() < 1e-9
    assert abs(e["stats"]["firings"] - z["stats"]["firings"]) <= 0.01 * e["stats"]["firings"]


def test_frozen_channel_and_edge_statuses():
    # a channel with an absent, never produced reactant: never fires, clock 0
    net = W.from_reactions(2, [({0: 1}, {0: 2}, 1.0), ({1: 1}, {}, 5.0), ({0: 1}, {}, 1.0)])
    o = _lazy(net, [20, 0], 2.0, [2.0], 50)
    assert (o["n"][:, 1] == 0).all() and (o["T"][:, 1] == 0.0).all()
    # overflow: stops before the jump, remaining samples -1
    net = W.from_reactions(1, [({0: 1}, {0: 2}, 1.0)])
    o = _lazy(net, [2**31 - 10], 100.0, [1e-12, 100.0], 3)
    assert (o["status"] == oracle.STATUS_OVERFLOW).all()
    assert (o["x_final"][:, 0] == 2**31 - 1).all() and (o["n"][:, 0] == 9).all()
    assert (o["samples"][:, 1, 0] == -1).all()
    # firing cap
    w = W.lv_small(4)
    o = _lazy(w.net, w.x0, w.t_end, w.sample_t, 4, max_firings=1000)
    assert (o["status"] == oracle.STATUS_MAX_FIRINGS).all()
    assert (o["n"].sum(axis=1) == 1000).all() and (o["samples"][:, -1, :] == -1).all()
    # absorbing start, t_end = 0
    o = _lazy(W.pure_death(1.0), [0], 5.0, [0.0, 5.0], 4)
    assert (o["status"] == oracle.STATUS_ABSORBED).all() and (o["t_last"] == 0).all()
    o = _lazy(w.net, w.x0, 0.0, [0.0], 4)
    assert (o["n"] == 0).all() and (o["T"] == 0).all()


def test_threads_and_offsets_do_not_change_bits():
    rng = np.random.default_rng(3)
    net = W.random_network(10, 30, rng)
    x0 = rng.integers(0, 60, size=10).astype(np.int32)
    a = _lazy(net, x0, 0.2, [0.1, 0.2], 40, threads=1)
    b = _lazy(net, x0, 0.2, [0.1, 0.2], 40, threads=5)
    c1 = _lazy(net, x0, 0.2, [0.1, 0.2], 25)
    c2 = _lazy(net, x0, 0.2, [0.1, 0.2], 15, traj_offset=25)
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], np.concatenate([c1[k], c2[k]])), k


@pytest.mark.parametrize("which", ["lv", "random"])
def test_with_a_schedule_the_forms_fire_the_same_sequences(which):
    """With a schedule too the two forms differ only in rounding: the same
    channels fire on nearly every trajectory and the internal times agree to
    rounding level where they do."""
    if which == "lv":
        w = W.lv_small(256)
        net, x0, t_end, R = w.net, w.x0, 4.0, 256
        sched = ([1.0, 2.5], np.array([[2.0, 0.005, 0.5], [0.5, 0.02, 2.0]]))
    else:
        rng = np.random.default_rng(40)
        net = W.random_network(30, 90, rng, logc=(-1.0, 1.0), bimol_scale=0.05)
        x0 = rng.integers(0, 80, size=30).astype(np.int32)
        t_end = float(2000 / W.initial_total_rate(net, x0))
        c = np.asarray(net.c)
        rates = c[None, :] * rng.uniform(0.2, 3.0, size=(3, c.size))
        rates[1, rng.random(c.size) < 0.35] = 0.0
        sched, R = (np.array([0.2, 0.45, 0.7]) * t_end, rates), 128
    grid = W.uniform_grid(t_end, 9)
    z = _lazy(net, x0, t_end, grid, R, seed=9, schedule=sched)
    e = _eager(net, x0, t_end, grid, R, seed=9, schedule=sched)
    same = e["seq_hash"] == z["seq_hash"]
    assert same.mean() >= 0.95, same.mean()
    for k in ("n", "x_final", "samples", "status"):
        assert np.array_equal(e[k][same], z[k][same]), k
    rel = np.abs(e["T"][same] - z["T"][same]) / np.maximum(np.abs(e["T"][same]), 1.0)
    assert rel.max() < 1e-9
