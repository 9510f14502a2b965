"""The oracle's pins are strong enough to catch plausible mistakes.

Each case copies rto.c, plants one mistake (a dropped term, a wrong index, a
wrong sign or scale, a reused random draw, a reversed comparison), builds the
mutant with gcc and checks that at least one pin fails on it.  The mistakes
are planted in a copy of the oracle on the CPU only.
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2103_00405_amd import workloads as W

ORACLE_DIR = os.path.dirname(os.path.abspath(oracle.__file__))

MUTANTS = {
    "homodimer_x_squared": ("return x * (x - 1) / 2;", "return x * x / 2;"),
    "unfired_clock_frozen": ("if (k != mu) T[k] = fma(a[k], d1, T[k]);", "if (k != mu) T[k] = T[k];"),
    "refresh_half_gap": ("P[mu] = P[mu] + E;", "P[mu] = P[mu] + 0.5 * E;"),
    "reused_draw": ("(uint32_t)mu, n[mu]);", "(uint32_t)mu, n[mu] - 1);"),
    "wrong_half_of_block": ("uint64_t word = (n & 1u) ?", "uint64_t word = (n & 0u) ?"),
    "final_clock_not_advanced": ("for (int k = 0; k < M; k++) T[k] = fma(a[k], dt, T[k]);",
                                 "for (int k = 0; k < M; k++) T[k] = T[k];"),
    "rate_of_next_channel": ("changed species */\n        for (int k = 0; k < M; k++) {\n"
                             "            a[k] = propensity_c(net, X, k, crate[k]);",
                             "changed species */\n        for (int k = 0; k < M; k++) {\n"
                             "            a[k] = propensity_c(net, X, k, crate[(k + 1) % M]);"),
    "time_step_halved": ("double t_new = t + d1;", "double t_new = t + 0.5 * d1;"),
    "argmax_instead_of_argmin": ("if (v[k] < d1) { d2 = d1; d1 = v[k]; best = k; }",
                                 "if (d1 == INFINITY || v[k] > d1) { d2 = d1; d1 = v[k]; best = k; }"),
    "jump_sign_flipped": ("T[mu] = P[mu];\n        t = t_new;\n"
                          "        for (int e = jb->nu_ptr[mu]; e < jb->nu_ptr[mu + 1]; e++)\n"
                          "            X[jb->nu_species[e]] += jb->nu_delta[e];",
                          "T[mu] = P[mu];\n        t = t_new;\n"
                          "        for (int e = jb->nu_ptr[mu]; e < jb->nu_ptr[mu + 1]; e++)\n"
                          "            X[jb->nu_species[e]] -= jb->nu_delta[e];"),
    "philox_key_not_bumped": ("if (round > 0) { k0 += W0; k1 += W1; }", "if (round > 0) { k0 += W0; }"),
    "log_of_wrong_argument": ("double u = (double)(m + 1) * 0x1p-53;", "double u = (double)(m + 2) * 0x1p-53;"),
}


# mistakes in the direct method (Eq. 17-22 with keyed draws)
DIRECT_MUTANTS = {
    "dm_waiting_time_not_scaled": ("double tau = E / a0;", "double tau = E;"),
    "dm_search_target_unscaled": ("double target = (double)(m2 + 1) * 0x1p-53 * a0;",
                                  "double target = (double)(m2 + 1) * 0x1p-53;"),
    "dm_one_uniform_for_both": ("uint64_t m2 = ((((uint64_t)w[3] << 32) | w[2]) >> 11);",
                                "uint64_t m2 = m1;"),
    "dm_next_channel_fires": ("if (run >= target) { mu = k; break; }",
                              "if (run >= target) { mu = (k + 1) % M; break; }"),
    "dm_counter_not_advanced": ("uint32_t ctr[4] = { (uint32_t)fired,",
                                "uint32_t ctr[4] = { 0u,"),
}


# mistakes in the piecewise-constant rate schedule (Eq. 28 solved piece by piece)
SCHEDULE_MUTANTS = {
    "sched_clock_not_run_to_breakpoint": ("for (int k = 0; k < M; k++) T[k] = fma(a[k], db, T[k]);",
                                          "for (int k = 0; k < M; k++) T[k] = T[k];"),
    "sched_rates_one_piece_late": ("crate = jb->sched_c + (size_t)piece * M;\n"
                                   "            piece += 1;\n"
                                   "            b_next = piece < jb->B ? jb->sched_t[piece] : INFINITY;\n"
                                   "            for (int k = 0; k < M; k++) {",
                                   "crate = piece ? jb->sched_c + (size_t)(piece - 1) * M : net->c;\n"
                                   "            piece += 1;\n"
                                   "            b_next = piece < jb->B ? jb->sched_t[piece] : INFINITY;\n"
                                   "            for (int k = 0; k < M; k++) {"),
    "sched_time_not_moved": ("T[k] = fma(a[k], db, T[k]);\n            t = b_next;\n",
                             "T[k] = fma(a[k], db, T[k]);\n"),
}

# the same mistakes in the lazy form's breakpoint (checked by the same pins,
# run in the lazy form)
LAZY_SCHEDULE_MUTANTS = {
    "lazy_sched_clock_not_run": ("                T[k] = fma(a[k], b_next - s_up[k], T[k]);\n", ""),
    "lazy_sched_rates_one_piece_late": (
        "crate = jb->sched_c + (size_t)piece * M;\n"
        "            piece += 1;\n"
        "            b_next = piece < jb->B ? jb->sched_t[piece] : INFINITY;\n"
        "            for (int k = 0; k < M; k++) lazy_refresh",
        "crate = piece ? jb->sched_c + (size_t)(piece - 1) * M : net->c;\n"
        "            piece += 1;\n"
        "            b_next = piece < jb->B ? jb->sched_t[piece] : INFINITY;\n"
        "            for (int k = 0; k < M; k++) lazy_refresh"),
    "lazy_sched_time_not_moved": ("                s_up[k] = b_next;\n            }\n            t = b_next;\n",
                                  "                s_up[k] = b_next;\n            }\n"),
}


# mistakes in the lazy form (dependency-graph updates in internal times)
LAZY_MUTANTS = {
    "lazy_dependents_not_advanced": ("T[k] = fma(a[k], t - s_up[k], T[k]);", "T[k] = T[k];"),
    "lazy_clock_not_restamped": ("            T[k] = fma(a[k], t - s_up[k], T[k]);\n"
                                 "            s_up[k] = t;\n",
                                 "            T[k] = fma(a[k], t - s_up[k], T[k]);\n"),
    "lazy_advance_at_new_rate": ("            T[k] = fma(a[k], t - s_up[k], T[k]);\n"
                                 "            s_up[k] = t;\n"
                                 "            lazy_refresh(jb, X, k, t, T, P, a, inv, tau, crate);",
                                 "            lazy_refresh(jb, X, k, t, T, P, a, inv, tau, crate);\n"
                                 "            T[k] = fma(a[k], t - s_up[k], T[k]);\n"
                                 "            s_up[k] = t;"),
    "lazy_fired_not_refreshed": ("        lazy_refresh(jb, X, mu, t, T, P, a, inv, tau, crate);\n", ""),
    "lazy_tau_not_offset": ("tau[k] = t + gap;", "tau[k] = gap;"),
    "lazy_no_final_advance": ("double t_stop = good ? jb->t_end : t;", "double t_stop = t;"),
    "lazy_reused_draw": ("(uint32_t)mu, n_mu);", "(uint32_t)mu, n_mu - 1);"),
}


# mistakes in the direct method on the sum tree
TREE_DM_MUTANTS = {
    "dt_search_no_subtract": ("                rem = rem - v;", "                rem = rem;"),
    "dt_search_takes_last": ("if (v > 0.0 && rem <= v) { take = i; break; }",
                             "if (0) { take = i; break; }"),
    "dt_node_drops_child": ("return ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));",
                            "return ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + v[6]);"),
    "dt_total_from_one_child": ("const double a0 = lev[top][0];",
                                "const double a0 = top > 1 ? lev[top - 1][0] : lev[top][0];"),
}


# mistakes in the selection step (Eq. 25) and the near-tie rule
ARGMIN_MUTANTS = {
    "near_tie_threshold_on_d2": ("return d2 - d1 <= 1e-12 * d1;", "return d2 - d1 <= 1e-12 * d2;"),
    "near_tie_strict": ("return d2 - d1 <= 1e-12 * d1;", "return d2 - d1 < 1e-12 * d1;"),
    "second_min_skips_equal": ("else if (v[k] < d2) { d2 = v[k]; }",
                               "else if (v[k] < d2 && v[k] != d1) { d2 = v[k]; }"),
    "tie_goes_to_last_channel": ("if (v[k] < d1) { d2 = d1; d1 = v[k]; best = k; }",
                                 "if (v[k] <= d1) { d2 = d1; d1 = v[k]; best = k; }"),
}


def _build_mutant(tmp, name):
    old, new = (MUTANTS.get(name) or DIRECT_MUTANTS.get(name) or SCHEDULE_MUTANTS.get(name)
                or LAZY_MUTANTS.get(name) or LAZY_SCHEDULE_MUTANTS.get(name)
                or ARGMIN_MUTANTS.get(name) or TREE_DM_MUTANTS[name])
    src = open(os.path.join(ORACLE_DIR, "rto.c")).read()
    assert src.count(old) == 1, name
    for f in ("rto.h", "dm.c"):
        shutil.copy(os.path.join(ORACLE_DIR, f), tmp)
    with open(os.path.join(tmp, "rto.c"), "w") as f:
        f.write(src.replace(old, new))
    so = os.path.join(tmp, "librto_mut.so")
    subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-o", so,
                    os.path.join(tmp, "rto.c"), os.path.join(tmp, "dm.c"),
                    "-lquadmath", "-lpthread", "-lm"], check=True, capture_output=True)
    return oracle.load_library(so)


def _pin_failures(L):
    """Run a quick subset of the law pins against library L; return failed names."""
    failed = []

    def sim(net, x0, t_end, grid, R, seed=1, **kw):
        try:
            return oracle.simulate(net, np.asarray(x0, np.int32), t_end, np.asarray(grid, float),
                                   seed, R, _lib=L, **kw)
        except RuntimeError:
            return None

    # 1. Exp(1) draws equal the correctly rounded -ln u of the Philox word
    import mpmath
    for (n, k) in [(0, 0), (1, 2), (2, 1), (5, 3)]:
        w = oracle.philox4x32_10([n >> 1, k, 9, 0], [7, 0])
        word = (int(w[3]) << 32 | int(w[2])) if n & 1 else (int(w[1]) << 32 | int(w[0]))
        with mpmath.workdps(50):
            ref = float(-mpmath.log(mpmath.mpf((word >> 11) + 1) / 2**53))
        if L.rto_exp1(7, 9, 0, k, n) != ref:
            failed.append("exp1")
            break

    # 2. birth-death transient law: Poisson(m(t)), mean and variance
    k1, k2, T = 50.0, 1.0, 2.0
    o = sim(W.birth_death(k1, k2), [0], T, [T], 8000, seed=5)
    if o is None:
        failed.append("bd_run")
    else:
        X = o["x_final"][:, 0].astype(float)
        m = k1 / k2 * (1 - math.exp(-k2 * T))
        if abs(X.mean() - m) > 4.5 * math.sqrt(m / X.size) or \
                abs(X.var() - m) > 5 * m * math.sqrt(2.0 / X.size):
            failed.append("bd_law")
        # martingale n_k - T_k
        S = o["n"].astype(float) - o["T"]
        for kk in range(2):
            ET = o["T"][:, kk].mean()
            if abs(S[:, kk].mean()) > 4.5 * math.sqrt(ET / S.shape[0]):
                failed.append("martingale")
                break
        if not np.allclose(o["T"][:, 0], k1 * T, rtol=1e-12):
            failed.append("constant_rate_clock")

    # 3. dimerisation CME (homodimer convention)
    from test_oracle_law import _cme_dimer, _chisq_discrete
    o = sim(W.dimerisation(0.05, 1.0), [30, 0], 0.8, [0.8], 8000, seed=8)
    if o is None or _chisq_discrete(o["x_final"][:, 1], np.arange(16),
                                    _cme_dimer(0.05, 1.0, 30, 0, 0.8)) < 1e-4:
        failed.append("dimer_cme")

    # 4. Eq. 5 state identity on a random network
    rng = np.random.default_rng(5)
    net = W.random_network(6, 14, rng)
    x0 = rng.integers(0, 40, size=6).astype(np.int32)
    o = sim(net, x0, 0.3, [0.3], 200)
    if o is None:
        failed.append("identity_run")
    else:
        from test_oracle_law import _nu_dense
        pred = x0[None, :].astype(np.int64) + o["n"].astype(np.int64) @ _nu_dense(net)
        if not np.array_equal(pred, o["x_final"].astype(np.int64)) or (o["x_final"] < 0).any():
            failed.append("eq5_identity")

    # 5. two-sample law against Gillespie's direct method (random network)
    if o is not None:
        d = oracle.dm_simulate(net, x0, 0.3, [0.3], 99, 3000)
        o3 = sim(net, x0, 0.3, [0.3], 3000, seed=3)
        ps = [stats.ks_2samp(o3["x_final"][:, j], d["samples"][:, 0, j]).pvalue for j in range(6)]
        if min(ps) * 6 < 1e-4:
            failed.append("dm_two_sample")
    return failed


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name):
    with tempfile.TemporaryDirectory() as tmp:
        L = _build_mutant(tmp, name)
        failed = _pin_failures(L)
    assert failed, "mutant %s passed every pin" % name


def test_pins_pass_on_the_real_oracle():
    assert _pin_failures(oracle.lib()) == []


def _direct_pin_failures(L):
    """A quick subset of the direct method's pins (tests/test_oracle_direct.py)
    against library L; returns the names of the failed pins."""
    failed = []

    def dm(net, x0, t_end, grid, R, seed=1, **kw):
        try:
            return oracle.direct_simulate(net, np.asarray(x0, np.int32), t_end,
                                          np.asarray(grid, float), seed, R, _lib=L, **kw)
        except RuntimeError:
            return None

    k1, k2, T = 50.0, 1.0, 2.0
    o = dm(W.birth_death(k1, k2), [0], T, [0.5, T], 8000, seed=5)
    if o is None:
        failed.append("bd_run")
    else:
        for g, t in enumerate((0.5, T)):
            X = o["samples"][:, g, 0].astype(float)
            m = k1 / k2 * (1 - math.exp(-k2 * t))
            if abs(X.mean() - m) > 4.5 * math.sqrt(m / X.size) or \
                    abs(X.var() - m) > 5 * m * math.sqrt(2.0 / X.size):
                failed.append("bd_law")
                break
    c1, c2, n, t = 1.0, 2.0, 30, 0.4
    o = dm(W.isomerisation(c1, c2), [n, 0], t, [t], 8000, seed=6)
    if o is None:
        failed.append("iso_run")
    else:
        p = c2 / (c1 + c2) + (1 - c2 / (c1 + c2)) * math.exp(-(c1 + c2) * t)
        A = o["x_final"][:, 0].astype(float)
        if abs(A.mean() - n * p) > 4.5 * math.sqrt(n * p * (1 - p) / A.size):
            failed.append("iso_binomial")
    rng = np.random.default_rng(5)
    net = W.random_network(6, 14, rng)
    x0 = rng.integers(0, 40, size=6).astype(np.int32)
    o = dm(net, x0, 0.3, [0.3], 3000, seed=3)
    if o is None:
        failed.append("random_run")
    else:
        from test_oracle_law import _nu_dense
        pred = x0[None, :].astype(np.int64) + o["n"].astype(np.int64) @ _nu_dense(net)
        if not np.array_equal(pred, o["x_final"].astype(np.int64)) or (o["x_final"] < 0).any():
            failed.append("eq5_identity")
        r = oracle.simulate(net, x0, 0.3, [0.3], 99, 3000)
        ps = [stats.ks_2samp(o["x_final"][:, j], r["x_final"][:, j]).pvalue for j in range(6)]
        if min(ps) * 6 < 1e-4:
            failed.append("random_time_two_sample")
    return failed


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(DIRECT_MUTANTS))
def test_direct_pins_catch_planted_mistake(name):
    with tempfile.TemporaryDirectory() as tmp:
        L = _build_mutant(tmp, name)
        failed = _direct_pin_failures(L)
    assert failed, "mutant %s passed every pin" % name


def test_direct_pins_pass_on_the_real_oracle():
    assert _direct_pin_failures(oracle.lib()) == []


def _schedule_pin_failures(L, lazy=False):
    """A quick subset of the schedule pins (tests/test_oracle_schedule.py)."""
    failed = []
    try:
        o = oracle.simulate(W.pure_birth(10.0), [0], 3.0, [0.5, 1.5, 2.5, 3.0], 1, 8000,
                            schedule=([1.0, 2.0], [[0.0], [30.0]]), _lib=L, lazy=lazy)
        for g, m in enumerate((5.0, 10.0, 25.0, 40.0)):
            X = o["samples"][:, g, 0].astype(float)
            if abs(X.mean() - m) > 4.5 * math.sqrt(m / X.size):
                failed.append("birth_law")
                break
        if not np.allclose(o["T"][:, 0], 40.0, rtol=1e-13):
            failed.append("birth_clock")
        o = oracle.simulate(W.birth_death(50.0, 1.0), [0], 3.0, [1.5, 3.0], 2, 8000,
                            schedule=([1.0], [[10.0, 1.0]]), _lib=L, lazy=lazy)
        m1 = 50.0 * (1 - math.exp(-1.0))
        for g, t in enumerate((1.5, 3.0)):
            m = 10.0 + (m1 - 10.0) * math.exp(-(t - 1.0))
            X = o["samples"][:, g, 0].astype(float)
            if abs(X.mean() - m) > 4.5 * math.sqrt(m / X.size):
                failed.append("bd_switch_law")
                break
    except RuntimeError:
        failed.append("run")
    return failed


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(SCHEDULE_MUTANTS))
def test_schedule_pins_catch_planted_mistake(name):
    with tempfile.TemporaryDirectory() as tmp:
        L = _build_mutant(tmp, name)
        failed = _schedule_pin_failures(L)
    assert failed, "mutant %s passed every pin" % name


def test_schedule_pins_pass_on_the_real_oracle():
    assert _schedule_pin_failures(oracle.lib()) == []


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(LAZY_SCHEDULE_MUTANTS))
def test_lazy_schedule_pins_catch_planted_mistake(name):
    with tempfile.TemporaryDirectory() as tmp:
        L = _build_mutant(tmp, name)
        failed = _schedule_pin_failures(L, lazy=True)
    assert failed, "mutant %s passed every pin" % name


def test_lazy_schedule_pins_pass_on_the_real_oracle():
    assert _schedule_pin_failures(oracle.lib(), lazy=True) == []


def _lazy_pin_failures(L):
    """A quick subset of the lazy-form pins (tests/test_oracle_lazy.py)."""
    failed = []

    def sim(net, x0, t_end, grid, R, seed=1, lazy=True):
        try:
            return oracle.simulate(net, np.asarray(x0, np.int32), t_end, np.asarray(grid, float),
                                   seed, R, max_firings=5000, lazy=lazy, _lib=L)
        except RuntimeError:
            return None

    k1, k2, T = 50.0, 1.0, 2.0
    o = sim(W.birth_death(k1, k2), [0], T, [T], 8000, seed=5)
    if o is None or (o["status"] > oracle.STATUS_ABSORBED).any():
        failed.append("bd_run")
    else:
        X = o["x_final"][:, 0].astype(float)
        m = k1 / k2 * (1 - math.exp(-k2 * T))
        if abs(X.mean() - m) > 4.5 * math.sqrt(m / X.size) or \
                abs(X.var() - m) > 5 * m * math.sqrt(2.0 / X.size):
            failed.append("bd_law")
        S = o["n"].astype(float) - o["T"]
        for kk in range(2):
            ET = o["T"][:, kk].mean()
            if abs(S[:, kk].mean()) > 4.5 * math.sqrt(ET / S.shape[0]):
                failed.append("martingale")
                break
        if not np.allclose(o["T"][:, 0], k1 * T, rtol=1e-12):
            failed.append("constant_rate_clock")
    from test_oracle_law import _cme_dimer, _chisq_discrete
    o = sim(W.dimerisation(0.05, 1.0), [30, 0], 0.8, [0.8], 8000, seed=8)
    if o is None or _chisq_discrete(o["x_final"][:, 1], np.arange(16),
                                    _cme_dimer(0.05, 1.0, 30, 0, 0.8)) < 1e-4:
        failed.append("dimer_cme")
    w = W.lv_small(64)
    e = sim(w.net, w.x0, 5.0, [5.0], 64, seed=9, lazy=False)
    z = sim(w.net, w.x0, 5.0, [5.0], 64, seed=9)
    if e is None or z is None or (e["seq_hash"] == z["seq_hash"]).mean() < 0.95:
        failed.append("eager_sequences")
    return failed


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(LAZY_MUTANTS))
def test_lazy_pins_catch_planted_mistake(name):
    with tempfile.TemporaryDirectory() as tmp:
        L = _build_mutant(tmp, name)
        failed = _lazy_pin_failures(L)
    assert failed, "mutant %s passed every pin" % name


def test_lazy_pins_pass_on_the_real_oracle():
    assert _lazy_pin_failures(oracle.lib()) == []


def _tree_dm_pin_failures(L):
    """A quick subset of the tree direct method's pins."""
    failed = []

    def dm(net, x0, t_end, grid, R, seed=1):
        try:
            return oracle.direct_simulate(net, np.asarray(x0, np.int32), t_end,
                                          np.asarray(grid, float), seed, R, _lib=L, tree=True,
                                          max_firings=200000)
        except RuntimeError:
            return None

    k1, k2, T = 50.0, 1.0, 2.0
    o = dm(W.birth_death(k1, k2), [0], T, [T], 8000, seed=5)
    m = k1 / k2 * (1 - math.exp(-k2 * T))
    if o is None or abs(o["x_final"][:, 0].mean() - m) > 4.5 * math.sqrt(m / 8000):
        failed.append("bd_law")
    M, t = 100, 2.0
    c = 0.5 + (np.arange(M) % 13) * 0.37
    spec = W.from_reactions(M, [({}, {i: 1}, float(c[i])) for i in range(M)])
    o = dm(spec, np.zeros(M, np.int32), t, [t], 3000, seed=21)
    if o is None:
        failed.append("births_run")
    else:
        z = (o["x_final"].mean(axis=0) - c * t) / np.sqrt(c * t / 3000)
        if np.abs(z).max() >= 4.5 or stats.chi2.sf(float((z ** 2).sum()), M) <= 1e-4:
            failed.append("births_selection")
    return failed


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(TREE_DM_MUTANTS))
def test_tree_dm_pins_catch_planted_mistake(name):
    with tempfile.TemporaryDirectory() as tmp:
        L = _build_mutant(tmp, name)
        failed = _tree_dm_pin_failures(L)
    assert failed, "mutant %s passed every pin" % name


def test_tree_dm_pins_pass_on_the_real_oracle():
    assert _tree_dm_pin_failures(oracle.lib()) == []


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(ARGMIN_MUTANTS))
def test_selection_pins_catch_planted_mistake(name):
    from test_oracle_argmin import pin_failures
    with tempfile.TemporaryDirectory() as tmp:
        L = _build_mutant(tmp, name)
        failed = pin_failures(L)
    assert failed, "mutant %s passed every pin" % name
