"""Pins of the oracle's selection step (Eq. 25) and near-tie rule (Eq. 4).

The selection returns the lowest channel among the smallest gaps and the
second smallest gap counted with multiplicity; the near-tie rule is
RN(d2 - d1) <= RN(1e-12 d1).  Both are fixed by their definitions, so the
cases here are written out by hand or computed with exact rationals
(``fractions.Fraction``, whose conversion to float rounds to nearest) and
brute force, never by calling the oracle's own arithmetic twice.

The thresholds' binary64 neighbours are found with exact arithmetic, so a
plausible slip (a strict comparison, the threshold scaled by d2 instead of
d1, a second minimum that skips values equal to the minimum, the highest
channel winning a tie) fails at least one case; the planted-mistake test in
test_oracle_mutants.py checks exactly that.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2103_00405_amd import workloads as W

from near_tie_cases import (exact_first_gaps, first_h, plant_first_firing_clamp,
                             plant_first_firing_tie)

INF = math.inf
T12 = 1e-12        # the binary64 nearest to 10^-12


def _rn(q):
    """Round an exact rational to the nearest binary64 (ties to even)."""
    return float(q)


def _is_near_tie(d1, d2):
    """The definition: RN(d2 - d1) <= RN(1e-12 d1), each operation rounded once."""
    if d2 == INF:
        return False
    return _rn(Fraction(d2) - Fraction(d1)) <= _rn(Fraction(T12) * Fraction(d1))


def _boundary(d1):
    """(largest d2 that is a near-tie of d1, the next binary64 above it)."""
    thr = _rn(Fraction(T12) * Fraction(d1))
    d2 = _rn(Fraction(d1) + Fraction(thr))
    # walk to the exact edge of the rule
    while not _is_near_tie(d1, d2):
        d2 = math.nextafter(d2, -INF)
    while _is_near_tie(d1, math.nextafter(d2, INF)):
        d2 = math.nextafter(d2, INF)
    return d2, math.nextafter(d2, INF)


# (values, mu, v1, v2) written out from the definition
SELECTION_CASES = [
    ([3.0, 1.0, 1.0, 2.0], 1, 1.0, 1.0),          # exact tie: lowest k, d2 = d1
    ([5.0, 5.0, 5.0], 0, 5.0, 5.0),
    ([1.0, 2.0, 1.0], 0, 1.0, 1.0),               # equal minima not adjacent
    ([2.0, 7.0], 0, 2.0, 7.0),
    ([7.0, 2.0], 1, 2.0, 7.0),
    ([4.5], 0, 4.5, INF),                         # M = 1
    ([], -1, INF, INF),                           # M = 0
    ([INF, INF], -1, INF, INF),                   # nothing can fire
    ([INF, 4.0, INF], 1, 4.0, INF),
    ([INF, 0.0, 0.0], 1, 0.0, 0.0),               # clamped gaps tie at zero
    ([0.0, 5e-324], 0, 0.0, 5e-324),
    ([9.0, 8.0, 7.0, 6.0, 6.0, 7.0], 3, 6.0, 6.0),
    ([1.0, math.nextafter(1.0, INF), 1.0], 0, 1.0, 1.0),
]


@pytest.mark.parametrize("vals,mu,v1,v2", SELECTION_CASES)
def test_selection_hand_cases(vals, mu, v1, v2):
    got = oracle.argmin2(vals)
    assert got == (mu, v1, v2), (vals, got)


def test_selection_brute_force():
    """Random arrays with many repeated values against a sort-based brute force."""
    rng = np.random.default_rng(41)
    for _ in range(3000):
        M = int(rng.integers(1, 40))
        pool = np.concatenate([rng.exponential(size=4), [0.0, INF]])
        v = rng.choice(pool, size=M)
        finite = [x for x in v if x < INF]
        got = oracle.argmin2(v)
        if not finite:
            assert got == (-1, INF, INF)
            continue
        srt = sorted(v.tolist())
        lo = srt[0]
        assert got[0] == min(k for k in range(M) if v[k] == lo)
        assert got[1] == lo
        assert got[2] == (srt[1] if M > 1 else INF)


def test_near_tie_hand_cases():
    assert oracle.near_tie(1.0, 1.0)                      # exact tie
    assert oracle.near_tie(0.0, 0.0)                      # clamped gaps (0 <= 0)
    assert not oracle.near_tie(0.0, 5e-324)               # RN(1e-12 * 0) = 0
    assert not oracle.near_tie(1.0, INF)                  # one channel left
    assert not oracle.near_tie(1.0, 2.0)
    # at d1 = 1 the threshold is 1e-12 = 4503.6 ulps of 1: 4503 ulps is a
    # near-tie, 4504 is not
    ulp1 = 2.0 ** -52
    assert 4503 * ulp1 <= T12 < 4504 * ulp1
    assert oracle.near_tie(1.0, 1.0 + 4503 * ulp1)
    assert not oracle.near_tie(1.0, 1.0 + 4504 * ulp1)


@pytest.mark.parametrize("d1", [1.0, 3.7, 1e-9, 2.5e-300, 123456.789, 0.1, 7.0e5, 1.9999999])
def test_near_tie_boundary_neighbours(d1):
    """d2 at the binary64 neighbours on either side of the 1e-12 edge."""
    inside, outside = _boundary(d1)
    assert inside > d1
    assert oracle.near_tie(d1, inside)
    assert not oracle.near_tie(d1, outside)
    assert oracle.near_tie(d1, d1)


def _edge_by_d2():
    """A d1 whose edge moves if the threshold were RN(1e-12 d2): the
    threshold RN(1e-12 d1) sits just below a multiple of ulp(d1), so the next
    representable d2 beyond it is outside the rule but within 1e-12 d2."""
    ulp = Fraction(2) ** -52
    # k ulps past d1 is the first step outside; pick d1 in [1, 2) with
    # RN(1e-12 d1) < k ulp <= RN(1e-12 (d1 + k ulp))
    k = 6000
    edge = k * ulp
    # largest d1 (on the 2^-52 grid) with RN(1e-12 d1) < edge, by bisection
    lo_i, hi_i = 0, 2 ** 52
    while hi_i - lo_i > 1:
        mid = (lo_i + hi_i) // 2
        d1 = 1 + mid * ulp
        if Fraction(_rn(Fraction(T12) * d1)) < edge:
            lo_i = mid
        else:
            hi_i = mid
    d1 = float(1 + lo_i * ulp)
    d2 = float(Fraction(d1) + edge)
    return d1, d2


def test_near_tie_threshold_scales_with_d1():
    d1, d2 = _edge_by_d2()
    assert _rn(Fraction(d2) - Fraction(d1)) > _rn(Fraction(T12) * Fraction(d1))
    assert _rn(Fraction(d2) - Fraction(d1)) <= _rn(Fraction(T12) * Fraction(d2))
    assert not oracle.near_tie(d1, d2)
    assert oracle.near_tie(d1, math.nextafter(d2, -INF))


def _planted(M, i, j, exact, seed=5, traj=3, net_id=7):
    rng = np.random.default_rng(M * 31 + i)
    spec = W.random_network(max(2, M // 2), M, rng, order_p=(0.3, 0.7, 0.0), logc=(-1.0, 0.5))
    x0 = rng.integers(5, 60, size=spec.N).astype(np.int32)
    spec, gap = plant_first_firing_tie(spec, x0, seed, traj, net_id, i, j, exact=exact)
    return spec, x0, gap


@pytest.mark.parametrize("M,i,j,exact", [(3, 0, 2, True), (8, 1, 6, True), (8, 2, 5, False),
                                         (40, 31, 33, True), (300, 255, 256, True),
                                         (300, 4, 290, False)])
def test_planted_tie_counted_at_first_firing(M, i, j, exact):
    """A path whose first selection has a tie: the oracle reports a near-tie at
    firing 0, fires the lower channel on an exact tie, and its first gaps
    equal the exact-rational computation from the pinned draws."""
    seed, traj, net_id = 5, 3, 7
    spec, x0, gap = _planted(M, i, j, exact, seed, traj, net_id)
    h = first_h(spec, x0)
    P = [oracle.exp1(seed, traj, net_id, k, 0) for k in range(M)]
    g = exact_first_gaps(P, spec.c, h)
    mu = min(range(M), key=lambda k: (g[k], k))
    srt = sorted(g)
    assert mu == i and srt[0] == gap
    assert (srt[1] == srt[0]) == exact and _is_near_tie(srt[0], srt[1])
    for lazy in (False, True):
        # the first firing alone: channel i, counted as one near-tie
        o = oracle.simulate(spec, x0, 1.0, [], seed, 1, net_id=net_id, traj_offset=traj,
                            lazy=lazy, max_firings=1)
        assert o["tie_step"][0] == 0 and o["stats"]["near_ties"] == 1
        assert o["n"][0, i] == 1 and o["n"][0].sum() == 1
        # run on: the tie stays the first one reported
        o = oracle.simulate(spec, x0, gap * 4, [gap, gap * 4], seed, 1, net_id=net_id,
                            traj_offset=traj, lazy=lazy)
        assert o["tie_step"][0] == 0 and o["stats"]["near_ties"] >= 1
        # the neighbours' paths carry no planted tie
        o2 = oracle.simulate(spec, x0, gap * 1.5, [gap * 1.5], seed, 2, net_id=net_id,
                             traj_offset=traj + 1, lazy=lazy)
        assert (o2["tie_step"] == oracle.TIE_NONE).all()


@pytest.mark.parametrize("M,i,j", [(3, 0, 2), (8, 1, 6), (300, 255, 256)])
def test_planted_clamp_counted_at_second_firing(M, i, j):
    """An exact first-firing tie in which the unfired channel j overshoots:
    with exact rationals, RN(a_j gap) > P_j; the oracle fires i, then j with
    a zero gap (its negative raw gap clamped), counts one clamp, and time
    does not advance at the second firing."""
    seed, traj, net_id = 5, 3, 7
    rng = np.random.default_rng(M * 31 + i)
    spec = W.random_network(max(2, M // 2), M, rng, order_p=(0.3, 0.7, 0.0), logc=(-1.0, 0.5))
    x0 = rng.integers(5, 60, size=spec.N).astype(np.int32)
    spec, gap = plant_first_firing_clamp(spec, x0, seed, traj, net_id, i, j)
    h = first_h(spec, x0)
    P = [oracle.exp1(seed, traj, net_id, k, 0) for k in range(M)]
    g = exact_first_gaps(P, spec.c, h)
    assert g[i] == g[j] == gap and min(g) == gap
    a_j = float(Fraction(spec.c[j]) * Fraction(float(h[j])))
    assert float(Fraction(a_j) * Fraction(gap)) > P[j]          # T_j after firing i
    o = oracle.simulate(spec, x0, 1.0, [], seed, 1, net_id=net_id, traj_offset=traj,
                        max_firings=2)
    assert o["n"][0, i] == 1 and o["n"][0, j] == 1 and o["n"][0].sum() == 2
    assert o["stats"]["clamps"] == 1 and o["tie_step"][0] == 0
    assert o["t_last"][0] == gap


def pin_failures(L):
    """Every definition-fixed case above, run against oracle build L; returns
    the names of the failed groups (used by the planted-mistake test)."""
    failed = []
    for vals, mu, v1, v2 in SELECTION_CASES:
        if oracle.argmin2(vals, _lib=L) != (mu, v1, v2):
            failed.append("selection_hand")
            break
    hand = [((1.0, 1.0), True), ((0.0, 0.0), True), ((0.0, 5e-324), False),
            ((1.0, INF), False), ((1.0, 2.0), False),
            ((1.0, 1.0 + 4503 * 2.0 ** -52), True), ((1.0, 1.0 + 4504 * 2.0 ** -52), False)]
    if any(oracle.near_tie(*a, _lib=L) != want for a, want in hand):
        failed.append("near_tie_hand")
    for d1 in (1.0, 3.7, 1e-9, 0.1):
        inside, outside = _boundary(d1)
        if not oracle.near_tie(d1, inside, _lib=L) or oracle.near_tie(d1, outside, _lib=L):
            failed.append("near_tie_boundary")
            break
    d1, d2 = _edge_by_d2()
    if oracle.near_tie(d1, d2, _lib=L) or not oracle.near_tie(d1, math.nextafter(d2, -INF), _lib=L):
        failed.append("near_tie_scale")
    return failed


def test_pin_runner_passes_on_the_real_oracle():
    assert pin_failures(oracle.lib()) == []
