"""Near-ties on the GPU: the selection step of every mapping, and paths with a
tie planted at a known firing, against the oracle.

Eq. 25 selects the lowest channel among the smallest gaps; a near-tie
(RN(d2 - d1) <= RN(1e-12 d1), Eq. 4's probability-zero event seen in
binary64) is counted and its first firing index reported.  The selection
hook runs the kernels' own device functions (the thread mapping's loop, the
lane exchanges of 2..64 lanes, the workgroup's LDS stage) on given rows and
is compared element by element with ``oracle.argmin2`` / ``oracle.near_tie``.
The planted paths put an exact (or few-ulp) tie at the first firing of one
trajectory, with the lower channel owned by a later lane or wavefront, and
a t_end that ends most other trajectories of the same wavefront on that
pass, so that a counter bumped on a repeated pass would show.
"""
import ctypes as C
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2103_00405_amd import workloads as W

from near_tie_cases import first_h, plant_first_firing_clamp, plant_first_firing_tie

pytestmark = pytest.mark.gpu

INF = math.inf


def _api():
    from paper_2103_00405_amd import api
    return api


def _np(t):
    return t.cpu().numpy()


# ------------------------------------------------------------ selection hook
def _select(rows, mapping, lanes):
    from paper_2103_00405_amd._lib import check, lib
    rows = np.ascontiguousarray(rows, dtype=np.float64)
    count, M = rows.shape
    v = torch.from_numpy(rows).cuda()
    mu = torch.empty(count, dtype=torch.int32, device="cuda")
    v1 = torch.empty(count, dtype=torch.float64, device="cuda")
    v2 = torch.empty(count, dtype=torch.float64, device="cuda")
    near = torch.empty(count, dtype=torch.uint8, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda t: C.c_void_p(t.data_ptr())
    check(lib().rtssa_debug_select(p(v), M, count, mapping, lanes, p(mu), p(v1), p(v2), p(near),
                                   stream))
    torch.cuda.synchronize()
    return _np(mu), _np(v1), _np(v2), _np(near)


def _rows(M, count, seed):
    """Rows with heavy repetition, +inf entries, zeros, and ties planted so
    that the lower channel of a tied pair sits in a later lane/slot."""
    rng = np.random.default_rng(seed)
    pool = np.concatenate([rng.exponential(size=6), [0.0, INF, 1.0, 1.0 + 2.0 ** -52]])
    rows = rng.choice(pool, size=(count, M))
    for r in range(0, count, 3):
        # an exact tie between two channels
        i, j = sorted(rng.choice(M, size=2, replace=False)) if M > 1 else (0, 0)
        rows[r, i] = rows[r, j] = 1e-3
    for r in range(1, count, 7):
        rows[r, :] = INF
    for r in range(2, count, 5):
        if M > 1:
            # the binary64 neighbours of the near-tie edge at d1 = 0.5
            i, j = sorted(rng.choice(M, size=2, replace=False))
            rows[r, :] = np.maximum(rows[r, :], 0.75)
            rows[r, i] = 0.5
            rows[r, j] = 0.5 + (4503 if r % 2 else 4504) * 2.0 ** -53
    return rows


# mapping 4: the selection of the workgroup kernel with the propensities in
# LDS (second smallest carried only within near-tie reach)
VARIANTS = [(1, 0)] + [(2, w) for w in (2, 4, 8, 16, 32, 64)] + \
           [(3, l) for l in (64, 128, 256, 512, 1024)] + [(4, l) for l in (64, 128, 256, 512, 1024)]


@pytest.mark.parametrize("mapping,lanes", VARIANTS)
def test_selection_hook_matches_oracle(mapping, lanes):
    Ms = [1, 2, 3, 8] if mapping == 1 else [1, 3, lanes - 1, lanes, 3 * lanes + 5, 8 * lanes]
    if mapping == 4:
        Ms.append(16 * lanes)
    for M in Ms:
        rows = _rows(M, 600, seed=M * 7 + lanes)
        mu, v1, v2, near = _select(rows, mapping, lanes)
        for r in range(rows.shape[0]):
            omu, ov1, ov2 = oracle.argmin2(rows[r])
            assert v1[r] == ov1, (M, r)
            if mapping == 4 and not oracle.near_tie(ov1, ov2):
                # out of reach: any value no smaller than the true one
                assert v2[r] >= ov2 and not oracle.near_tie(ov1, v2[r]), (M, r)
            else:
                assert v2[r] == ov2, (M, r)
            if ov1 < INF:
                assert mu[r] == omu, (M, r, mu[r], omu)
            assert bool(near[r]) == oracle.near_tie(ov1, ov2), (M, r)


def test_selection_hook_edge_rows():
    """The near-tie edge at d1 = 0.5 (threshold 5e-13 = 4503.6 ulps of
    2^-53): 4503 ulps inside, 4504 outside."""
    d1 = 0.5
    inside, outside = d1 + 4503 * 2.0 ** -53, d1 + 4504 * 2.0 ** -53
    assert oracle.near_tie(d1, inside) and not oracle.near_tie(d1, outside)
    for mapping, lanes in VARIANTS:
        M = 3 if mapping == 1 else 2 * lanes + 1
        rows = np.full((4, M), 2.0)
        rows[0, [0, M - 1]] = [inside, d1]            # minimum in the last channel
        rows[1, [0, M - 1]] = [d1, outside]
        rows[2, [M - 1, 1]] = [d1, d1]                # exact tie, lower channel second in memory order
        rows[3, [0, 1]] = [0.0, 0.0]
        mu, v1, v2, near = _select(rows, mapping, lanes)
        assert list(mu) == [M - 1, 0, 1, 0], (mapping, lanes)
        assert list(near) == [1, 0, 1, 1], (mapping, lanes)


# ------------------------------------------------------------ planted paths
def _assert_same(g, ref):
    for k in ("samples", "n", "x_final", "status"):
        assert np.array_equal(_np(g[k]).view(ref[k].dtype), ref[k]), k
    assert np.array_equal(_np(g["T"]).view(np.uint64), ref["T"].view(np.uint64))
    assert np.array_equal(_np(g["t_last"]).view(np.uint64), ref["t_last"].view(np.uint64))
    assert np.array_equal(_np(g["seq_hash"]).view(np.uint64), ref["seq_hash"])
    assert np.array_equal(_np(g["tie_step"]).view(np.uint32), ref["tie_step"])
    gs, rs = g["stats"], ref["stats"]
    for k in ("firings", "near_ties", "clamps", "status_count"):
        assert gs[k] == rs[k], (k, gs[k], rs[k])


def _planted_case(M, i, j, exact, seed):
    rng = np.random.default_rng(seed)
    N = max(2, M // 4)
    spec = W.random_network(N, M, rng, order_p=(0.2, 0.6, 0.2), logc=(-1.0, 0.5),
                            bimol_scale=0.02)
    x0 = rng.integers(5, 80, size=N).astype(np.int32)
    h = first_h(spec, x0)
    # move i and j to the nearest channels that can fire at x0
    while h[i] == 0:
        i += 1
    while h[j] == 0 or j <= i:
        j += 1
    assert j < M
    return spec, x0, i, j


def _pick_trajectory(seed, net_id, i, j, R):
    """The trajectory whose first draws of i and j are smallest: the planted
    rates then leave the other trajectories' channels i and j slow enough
    that many of them fire nothing before t_end = 3 gaps."""
    return min(range(R), key=lambda r: max(oracle.exp1(seed, r, net_id, i, 0),
                                           oracle.exp1(seed, r, net_id, j, 0)))


# (M, i, j, mapping, block, method): the lower channel i sits in a later lane
# (or wavefront) than j wherever the layout allows
CASES = [
    (3, 0, 2, 1, 0, 0), (8, 3, 6, 1, 0, 0), (6, 1, 4, 1, 64, 0),
    (20, 3, 4, 2, 4, 0), (100, 15, 16, 2, 16, 0), (400, 63, 64, 2, 64, 0),
    (300, 255, 256, 3, 256, 0), (2000, 511, 512, 3, 512, 0), (4000, 200, 256 * 9 + 3, 3, 256, 0),
    (1500, 1023, 1024, 3, 1024, 0),
    (50, 10, 30, 0, 0, 2), (4000, 1234, 3000, 0, 0, 2),
]


@pytest.mark.parametrize("exact", [True, False])
@pytest.mark.parametrize("M,i,j,mapping,block,method", CASES)
def test_planted_tie_every_mapping(M, i, j, mapping, block, method, exact):
    api = _api()
    seed, net_id, R = 11, 5, 128
    spec, x0, i, j = _planted_case(M, i, j, exact, seed=M + i)
    traj = _pick_trajectory(seed, net_id, i, j, R)
    spec, gap = plant_first_firing_tie(spec, x0, seed, traj, net_id, i, j, exact=exact)
    net = api.Network(spec)
    lazy = method == api.METHOD_LAZY
    for t_end in (3 * gap, 400 * gap):
        grid = np.linspace(0.0, t_end, 7)
        g = api.simulate(net, x0, t_end, grid, R, seed=seed, net_id=net_id, with_hash=True,
                         mapping=mapping, block=block, method=method)
        torch.cuda.synchronize()
        ref = oracle.simulate(spec, x0, t_end, grid, seed, R, net_id=net_id, lazy=lazy)
        assert ref["tie_step"][traj] == 0
        assert ref["n"][traj, i] >= 1
        if t_end == 3 * gap:
            # trajectories next to the planted one end on its first pass
            lo = traj // 64 * 64
            assert (ref["n"][lo:lo + 64].sum(axis=1) == 0).sum() > 0
        _assert_same(g, ref)
        if mapping:
            assert g["stats"]["mapping"] == mapping


@pytest.mark.parametrize("M,i,j,mapping,block,method", [c for c in CASES if c[5] == 0])
def test_planted_clamp_every_mapping(M, i, j, mapping, block, method):
    """An exact first-firing tie whose unfired channel's internal time then
    overshoots its next firing time: its next raw gap is negative, clamped to
    0 and counted (the workgroup kernel with propensities in LDS takes its
    exact fallback pass there)."""
    api = _api()
    seed, net_id, R = 11, 5, 128
    spec, x0, i, j = _planted_case(M, i, j, True, seed=M + i)
    traj = _pick_trajectory(seed, net_id, i, j, R)
    spec, gap = plant_first_firing_clamp(spec, x0, seed, traj, net_id, i, j)
    net = api.Network(spec)
    for t_end in (3 * gap, 400 * gap):
        grid = np.linspace(0.0, t_end, 7)
        g = api.simulate(net, x0, t_end, grid, R, seed=seed, net_id=net_id, with_hash=True,
                         mapping=mapping, block=block)
        torch.cuda.synchronize()
        ref = oracle.simulate(spec, x0, t_end, grid, seed, R, net_id=net_id)
        assert ref["stats"]["clamps"] >= 1 and ref["tie_step"][traj] == 0
        _assert_same(g, ref)


def test_full_ensemble_near_ties():
    """The ensemble workload at full size (2^20 trajectories), launched as
    the benchmark launches it: every trajectory with a reported near-tie is
    recomputed by the oracle and equal in every output, and the count of
    near-ties equals the oracle's count over those trajectories."""
    api = _api()
    w = W.lv_ensemble()
    net = api.Network(w.net)
    g = api.simulate(net, w.x0, w.t_end, w.sample_t, w.R, seed=w.seed, with_hash=True,
                     want=("samples", "n", "T", "x_final", "t_last", "status", "tie_step"))
    torch.cuda.synchronize()
    ties = np.nonzero(_np(g["tie_step"]).view(np.uint32) != oracle.TIE_NONE)[0]
    print("near-tie trajectories:", ties.tolist(), "count", g["stats"]["near_ties"])
    assert g["stats"]["near_ties"] >= len(ties)
    total = 0
    for r in ties.tolist():
        ref = oracle.simulate(w.net, w.x0, w.t_end, w.sample_t, w.seed, 1, traj_offset=r)
        sl = slice(r, r + 1)
        assert np.array_equal(_np(g["samples"][sl]), ref["samples"])
        assert np.array_equal(_np(g["n"][sl]).view(np.uint32), ref["n"])
        assert np.array_equal(_np(g["T"][sl]).view(np.uint64), ref["T"].view(np.uint64))
        assert np.array_equal(_np(g["t_last"][sl]).view(np.uint64), ref["t_last"].view(np.uint64))
        assert np.array_equal(_np(g["seq_hash"][sl]).view(np.uint64), ref["seq_hash"])
        assert np.array_equal(_np(g["tie_step"][sl]).view(np.uint32), ref["tie_step"])
        total += ref["stats"]["near_ties"]
    assert total == g["stats"]["near_ties"]
    assert len(ties) > 0, "the full ensemble is expected to hold at least one near-tie"
