"""Inputs with a planted tie between two channels (test infrastructure).

Eq. 4 gives two channels firing at once probability zero; in binary64 two
gaps can still round to the same value or to values within the near-tie
threshold.  These helpers build such cases on purpose so that the selection
rule (lowest channel wins an exact tie) and the near-tie count are exercised
at a known firing.

``plant_first_firing_tie`` rewrites the rate constants of channels i < j of a
network so that, for one chosen trajectory, the first gaps of i and j are the
two smallest and equal (``exact=True``) or a few ulps apart.  The first gap of
channel k is RN(P_k RN(1 / a_k)) with a_k = RN(c_k RN(h_k(x0))) and
P_k = E(seed, traj, net_id, k, 0); the draws come from the oracle's Exp(1),
which is pinned on its own against mpmath.  Only the inputs are built here;
every expected value still comes from the oracle's run.
"""
import math
from fractions import Fraction

import numpy as np

import oracle
from paper_2103_00405_amd import workloads as W


def first_h(spec, x0):
    """h_k(x0) of Eq. 2 for every channel, exact integers."""
    h = []
    for k in range(int(spec.M)):
        v = 1
        for e in range(int(spec.react_ptr[k]), int(spec.react_ptr[k + 1])):
            x = int(x0[int(spec.react_species[e])])
            s = int(spec.react_sigma[e])
            v *= 1 if s == 0 else (x if s == 1 else x * (x - 1) // 2)
        h.append(v)
    return h


def first_gap(P, c, h):
    """RN(P RN(1 / RN(c RN(h)))): a channel's gap at t = 0 (T = 0)."""
    a = c * float(h)
    return math.inf if a == 0.0 else P * (1.0 / a)


def plant_first_firing_tie(spec, x0, seed, traj, net_id, i, j, exact=True, ulps=3):
    """Copy of spec with c_i, c_j set so that trajectory ``traj`` starts with
    a tie between channels i < j (both need h > 0 at x0).  Returns (spec,
    gap) with the planted gap value of channel i."""
    assert 0 <= i < j < int(spec.M)
    h = first_h(spec, x0)
    assert h[i] > 0 and h[j] > 0, "both channels must be able to fire at x0"
    P = [oracle.exp1(seed, traj, net_id, k, 0) for k in range(int(spec.M))]
    c = np.array(spec.c, dtype=np.float64).copy()
    others = [first_gap(P[k], c[k], h[k]) for k in range(int(spec.M)) if k not in (i, j)]
    finite = [g for g in others if g < math.inf]
    target = (min(finite) if finite else 1.0) / 8.0
    ci0 = P[i] / target / float(h[i])
    best = None
    ci = ci0
    for _ in range(64):                       # neighbours of c_i until j can match
        gi = first_gap(P[i], ci, h[i])
        cand = P[j] / gi / float(h[j])
        last_dir = 0
        for _ in range(400):
            gj = first_gap(P[j], cand, h[j])
            if exact and gj == gi:
                best = cand
                break
            if not exact and gi < gj <= gi + ulps * math.ulp(gi):
                best = cand
                break
            # a smaller rate gives a larger gap: walk the rate toward the goal;
            # a reversal means the goal lies between two neighbouring rates
            d = -1 if (gj < gi or (not exact and gj == gi)) else 1
            if last_dir and d != last_dir:
                break
            last_dir = d
            cand = math.nextafter(cand, 0.0 if d < 0 else math.inf)
        if best is not None:
            break
        ci = math.nextafter(ci, math.inf)
    assert best is not None, "no rate found for the planted tie"
    c[i] = ci
    c[j] = best
    return W.with_rates(spec, c), gi


def exact_first_gaps(P, c, h):
    """The same first gaps computed with exact rationals and one rounding per
    operation (Fraction -> float rounds to nearest), independent of binary64
    hardware arithmetic."""
    out = []
    for Pk, ck, hk in zip(P, c, h):
        a = float(Fraction(ck) * Fraction(float(hk)))
        if a == 0.0:
            out.append(math.inf)
            continue
        inv = float(1 / Fraction(a))
        out.append(float(Fraction(Pk) * Fraction(inv)))
    return out


def plant_first_firing_clamp(spec, x0, seed, traj, net_id, i, j):
    """Copy of spec with c_i, c_j set so that trajectory ``traj`` starts with
    an exact tie between channels i < j (i fires, the lower channel) and the
    unfired channel j's internal time then overshoots its next firing time:
    RN(a_j gap) > P_j, so that its next raw gap is negative and is clamped to
    0 (counted).  Returns (spec, gap)."""
    assert 0 <= i < j < int(spec.M)
    h = first_h(spec, x0)
    assert h[i] > 0 and h[j] > 0, "both channels must be able to fire at x0"
    P = [oracle.exp1(seed, traj, net_id, k, 0) for k in range(int(spec.M))]
    c = np.array(spec.c, dtype=np.float64).copy()
    others = [first_gap(P[k], c[k], h[k]) for k in range(int(spec.M)) if k not in (i, j)]
    finite = [g for g in others if g < math.inf]
    target = (min(finite) if finite else 1.0) / 8.0
    ci = P[i] / target / float(h[i])
    for _ in range(4096):                     # neighbours of c_i
        gi = first_gap(P[i], ci, h[i])
        # a rate of j whose gap equals gi (a larger rate gives a smaller gap)
        cand = P[j] / gi / float(h[j])
        for _ in range(64):
            gj = first_gap(P[j], cand, h[j])
            if gj == gi:
                break
            cand = math.nextafter(cand, math.inf if gj > gi else 0.0)
        if first_gap(P[j], cand, h[j]) == gi:
            # every neighbouring rate with the same gap, on both sides
            lo = cand
            while first_gap(P[j], math.nextafter(lo, 0.0), h[j]) == gi:
                lo = math.nextafter(lo, 0.0)
            cj = lo
            while first_gap(P[j], cj, h[j]) == gi:
                if (cj * float(h[j])) * gi > P[j]:
                    c[i] = ci
                    c[j] = cj
                    return W.with_rates(spec, c), gi
                cj = math.nextafter(cj, math.inf)
        ci = math.nextafter(ci, math.inf)
    raise AssertionError("no rates found for a planted clamp")
