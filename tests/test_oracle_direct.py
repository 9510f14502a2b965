"""Pins for the oracle's keyed direct method (Gillespie's direct method, paper
section 3, Eq. 17-22; one Philox block per firing).  It must sample the same
Markov jump law as the random-time algorithm, which these tests tie to closed
forms and exact identities, not to its own code:
  - pure birth: the count at t is Poisson(k t);
  - birth-death: transient law Poisson(k1/k2 (1 - e^{-k2 t}));
  - pure death: Binomial(n, e^{-k t}); A <-> B: Binomial(n, p(t));
  - 2A <-> B against the chemical master equation (matrix exponential);
  - Eq. 5 on every path; a two-sample test against the random-time oracle on
    Lotka-Volterra (same law, different draws);
  - absorption, overflow, the firing cap and schedule independence.
Every test runs both forms: the sums and running-sum search in channel order,
and the fixed sum tree of fan-out 8 (tree = True).  The tree form is pinned
further by 100 independent births (each channel's count is Poisson(c_i t),
so any bias of the tree search shows), bit equality with the channel-order
form on one channel, and firing sequences equal to that form's on nearly
every trajectory (the two differ only in rounding)."""
import math

import numpy as np
import pytest
from scipy import linalg, stats

import oracle
from paper_2103_00405_amd import workloads as W

P_MIN = 1e-4


TREE = False


@pytest.fixture(params=[False, True], ids=["channel_order", "tree"], autouse=True)
def tree(request):
    """Runs every test of this file for both forms of the direct method."""
    global TREE
    TREE = request.param
    yield request.param
    TREE = False


def _dm(net, x0, t_end, grid, R, seed=1, **kw):
    kw.setdefault("tree", TREE)
    return oracle.direct_simulate(net, np.asarray(x0, np.int32), t_end,
                                  np.asarray(grid, float), seed, R, **kw)


def _chisq(samples, support, pmf):
    obs = np.array([np.sum(samples == v) for v in support], dtype=float)
    exp = np.asarray(pmf) * samples.size
    keep = exp >= 5
    o = np.append(obs[keep], samples.size - obs[keep].sum())
    e = np.append(exp[keep], samples.size - exp[keep].sum())
    e *= o.sum() / e.sum()
    return stats.chisquare(o, e).pvalue


def _nu(net):
    nu = np.zeros((net.M, net.N), dtype=np.int64)
    for k in range(net.M):
        for e in range(net.react_ptr[k], net.react_ptr[k + 1]):
            nu[k, net.react_species[e]] -= net.react_sigma[e]
        for e in range(net.prod_ptr[k], net.prod_ptr[k + 1]):
            nu[k, net.prod_species[e]] += net.prod_mult[e]
    return nu


def test_pure_birth_poisson():
    k = 10.0
    o = _dm(W.pure_birth(k), [0], 3.0, [1.0, 3.0], 20000)
    sup = np.arange(0, 80)
    assert _chisq(o["x_final"][:, 0], sup, stats.poisson.pmf(sup, 30.0)) > P_MIN
    assert _chisq(o["samples"][:, 0, 0], sup, stats.poisson.pmf(sup, 10.0)) > P_MIN


@pytest.mark.parametrize("t", [0.5, 2.0])
def test_birth_death_transient(t):
    o = _dm(W.birth_death(50.0, 1.0), [0], 2.0, [0.5, 2.0], 20000, seed=4)
    X = o["samples"][:, [0.5, 2.0].index(t), 0]
    m = 50.0 * (1 - math.exp(-t))
    sup = np.arange(0, 120)
    assert _chisq(X, sup, stats.poisson.pmf(sup, m)) > P_MIN
    se = math.sqrt(m / X.size)
    assert abs(X.mean() - m) < 4 * se


def test_pure_death_and_isomerisation_binomial():
    o = _dm(W.pure_death(1.0), [40], 0.7, [0.7], 20000, seed=5)
    sup = np.arange(0, 41)
    assert _chisq(o["x_final"][:, 0], sup, stats.binom.pmf(sup, 40, math.exp(-0.7))) > P_MIN
    c1, c2, n, t = 1.0, 2.0, 30, 0.4
    o = _dm(W.isomerisation(c1, c2), [n, 0], t, [t], 20000, seed=6)
    p = c2 / (c1 + c2) + (1 - c2 / (c1 + c2)) * math.exp(-(c1 + c2) * t)
    sup = np.arange(0, n + 1)
    assert _chisq(o["x_final"][:, 0], sup, stats.binom.pmf(sup, n, p)) > P_MIN


def test_dimerisation_master_equation():
    """2A <-> B with A0 = 12, B0 = 0: the law of B(t) by expm of the generator."""
    c1, c2, A0, t = 0.3, 1.0, 12, 0.8
    states = [(A0 - 2 * b, b) for b in range(A0 // 2 + 1)]
    Q = np.zeros((len(states), len(states)))
    for i, (a, b) in enumerate(states):
        r1 = c1 * a * (a - 1) / 2
        r2 = c2 * b
        if i + 1 < len(states):
            Q[i, i + 1] = r1
        if i > 0:
            Q[i, i - 1] = r2
        Q[i, i] = -(Q[i].sum())
    pmf = linalg.expm(Q * t)[0]
    o = _dm(W.dimerisation(c1, c2), [A0, 0], t, [t], 20000, seed=7)
    assert _chisq(o["x_final"][:, 1], np.arange(len(states)), pmf) > P_MIN


def test_eq5_and_status_on_random_network():
    rng = np.random.default_rng(8)
    net = W.random_network(6, 8, rng, logc=(-1.0, 1.0), bimol_scale=0.05)
    x0 = rng.integers(0, 60, size=6).astype(np.int32)
    o = _dm(net, x0, 2.0, [1.0, 2.0], 256)
    pred = x0[None, :].astype(np.int64) + o["n"].astype(np.int64) @ _nu(net)
    assert np.array_equal(pred, o["x_final"].astype(np.int64))
    assert o["stats"]["firings"] == int(o["n"].sum())


def test_same_law_as_random_time_on_lotka_volterra():
    w = W.lv_small(4000)
    a = _dm(w.net, w.x0, 5.0, [2.5, 5.0], 4000, seed=9)
    b = oracle.simulate(w.net, w.x0, 5.0, [2.5, 5.0], 10, 4000)
    for g in range(2):
        for j in range(2):
            assert stats.ks_2samp(a["samples"][:, g, j], b["samples"][:, g, j]).pvalue > P_MIN


def test_absorbing_overflow_cap_and_schedule():
    # all propensities zero at the start
    o = _dm(W.pure_death(1.0), [0], 1.0, [0.5, 1.0], 8)
    assert (o["status"] == oracle.STATUS_ABSORBED).all() and o["n"].sum() == 0
    # overflow stops before the jump
    spec = W.from_reactions(1, [({0: 1}, {0: 2}, 1.0)])
    o = _dm(spec, [2**31 - 3], 50.0, [50.0], 4)
    assert (o["status"] == 2).all()
    assert (o["x_final"][:, 0] <= 2**31 - 1).all() and (o["samples"][:, 0, 0] == -1).all()
    # firing cap
    w = W.lv_small(16)
    o = _dm(w.net, w.x0, w.t_end, [w.t_end], 16, max_firings=100)
    assert (o["status"] == 3).all() and (o["n"].sum(axis=1) == 100).all()
    # threads and trajectory offsets do not change any trajectory
    a = _dm(w.net, w.x0, 3.0, [1.0, 3.0], 24, threads=1)
    b1 = _dm(w.net, w.x0, 3.0, [1.0, 3.0], 10, threads=3)
    b2 = _dm(w.net, w.x0, 3.0, [1.0, 3.0], 14, traj_offset=10, threads=2)
    for k in ("n", "samples", "seq_hash", "t_last"):
        assert np.array_equal(a[k], np.concatenate([b1[k], b2[k]])), k
    # the direct method's stream differs from the random-time one
    c = oracle.simulate(w.net, w.x0, 3.0, [1.0, 3.0], 1, 24)
    assert not np.array_equal(a["n"], c["n"])


def test_independent_births_selection_law():
    """100 pure-birth channels of different species and rates: each count is
    Poisson(c_i t) on its own, so the channel search must pick channel i with
    probability c_i / a_0 whatever the tree shape."""
    M, t = 100, 2.0
    c = 0.5 + (np.arange(M) % 13) * 0.37
    spec = W.from_reactions(M, [({}, {i: 1}, float(c[i])) for i in range(M)])
    o = _dm(spec, np.zeros(M, np.int32), t, [t], 3000, seed=21)
    X = o["x_final"].astype(float)
    m = c * t
    z = (X.mean(axis=0) - m) / np.sqrt(m / X.shape[0])
    assert np.abs(z).max() < 4.5, np.abs(z).max()
    assert stats.chi2.sf(float((z ** 2).sum()), M) > P_MIN


def test_tree_form_against_channel_order():
    # one channel: the same arithmetic, the same bits
    for spec, x0 in ((W.pure_birth(3.0), [0]), (W.pure_death(2.0), [30])):
        a = _dm(spec, x0, 2.0, [1.0, 2.0], 300, seed=3, tree=False)
        b = _dm(spec, x0, 2.0, [1.0, 2.0], 300, seed=3, tree=True)
        for k in ("n", "samples", "seq_hash", "t_last", "status"):
            assert np.array_equal(a[k], b[k]), k
    # many channels: the same firing sequence on nearly every trajectory
    rng = np.random.default_rng(11)
    net = W.random_network(20, 60, rng, logc=(-1.0, 1.0), bimol_scale=0.05)
    x0 = rng.integers(0, 80, size=20).astype(np.int32)
    t_end = float(2000 / W.initial_total_rate(net, x0))
    a = _dm(net, x0, t_end, [t_end], 128, seed=5, tree=False)
    b = _dm(net, x0, t_end, [t_end], 128, seed=5, tree=True)
    assert (a["seq_hash"] == b["seq_hash"]).mean() >= 0.95
