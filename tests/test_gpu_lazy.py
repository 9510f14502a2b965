"""GPU parity of the lazy form (one wavefront per trajectory, dependency-graph
updates, 8-ary minimum tree in LDS).

Every output is compared bit for bit with the oracle's lazy form on random
networks from 1 to 8000 channels (tree depths 1 to 5), on a network where a
firing touches more than 64 channels, on every end state, with piecewise-constant
rate schedules (alone and in a batch), and on the large random network
(N = 1000, M = 4000) at its full ensemble size, where sampled trajectories are
recomputed by the oracle and Eq. 5 is checked on all."""
import numpy as np
import pytest
import torch

import oracle
from paper_2103_00405_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("samples", "n", "T", "x_final", "t_last", "status", "seq_hash", "tie_step")


def _api():
    from paper_2103_00405_amd import api
    return api


def _np(t):
    return t.cpu().numpy()


def _assert_same(g, ref, stats=True, sl=slice(None)):
    assert np.array_equal(_np(g["samples"][sl]), ref["samples"])
    assert np.array_equal(_np(g["n"][sl]).view(np.uint32), ref["n"])
    assert np.array_equal(_np(g["T"][sl]).view(np.uint64), ref["T"].view(np.uint64))
    assert np.array_equal(_np(g["x_final"][sl]), ref["x_final"])
    assert np.array_equal(_np(g["t_last"][sl]).view(np.uint64), ref["t_last"].view(np.uint64))
    assert np.array_equal(_np(g["status"][sl]), ref["status"])
    assert np.array_equal(_np(g["seq_hash"][sl]).view(np.uint64), ref["seq_hash"])
    assert np.array_equal(_np(g["tie_step"][sl]).view(np.uint32), ref["tie_step"])
    if stats:
        for k in ("firings", "near_ties", "clamps", "status_count"):
            assert g["stats"][k] == ref["stats"][k], k


def _net(N, M, seed):
    rng = np.random.default_rng(seed)
    spec = W.random_network(N, M, rng, logc=(-1.0, 1.0), bimol_scale=0.05)
    x0 = rng.integers(0, 80, size=N).astype(np.int32)
    return spec, x0


def _run(api, spec, x0, t_end, grid, R, seed, **kw):
    net = api.Network(spec)
    g = api.simulate(net, x0, t_end, grid, R, seed=seed, net_id=seed, with_hash=True,
                     method=api.METHOD_LAZY, **kw)
    torch.cuda.synchronize()
    return g


@pytest.mark.parametrize("N,M,seed", [
    (1, 1, 1), (2, 3, 2), (3, 8, 3), (4, 9, 4), (6, 14, 5), (10, 64, 6), (12, 65, 7),
    (30, 100, 8), (60, 513, 9), (100, 800, 10), (250, 2000, 11), (1000, 4000, 12),
    (500, 4097, 13), (2000, 8000, 14),
])
def test_random_networks_bit_exact(N, M, seed):
    api = _api()
    spec, x0 = _net(N, M, seed)
    t_end = float(1500 / max(W.initial_total_rate(spec, x0), 1e-9))
    grid = np.sort(np.random.default_rng(seed).uniform(0, t_end, size=9))
    R = 24
    g = _run(api, spec, x0, t_end, grid, R, seed)
    assert g["stats"]["mapping"] == api.MAP_WAVE and g["stats"]["block"] == 64
    ref = oracle.simulate(spec, x0, t_end, grid, seed, R, net_id=seed, lazy=True)
    _assert_same(g, ref)


def test_lotka_volterra_and_birth_death():
    api = _api()
    w = W.lv_small(256)
    g = _run(api, w.net, w.x0, w.t_end, w.sample_t, 256, 1)
    _assert_same(g, oracle.simulate(w.net, w.x0, w.t_end, w.sample_t, 1, 256, net_id=1,
                                    lazy=True))
    # the eager form fires the same channels on (nearly) every trajectory
    e = api.simulate(api.Network(w.net), w.x0, w.t_end, w.sample_t, 256, seed=1, net_id=1,
                     with_hash=True)
    torch.cuda.synchronize()
    assert (_np(e["seq_hash"]) == _np(g["seq_hash"])).mean() >= 0.95
    bd = W.birth_death(50.0, 1.0)
    g = _run(api, bd, [0], 2.0, [0.5, 1.0, 2.0], 4096, 7)
    _assert_same(g, oracle.simulate(bd, [0], 2.0, [0.5, 1.0, 2.0], 7, 4096, net_id=7,
                                    lazy=True))


def test_more_than_64_touched_channels():
    """Species S is read by 100 channels and changed by all of them and by its
    source: every firing touches 100 channels (two rounds of 64 lanes)."""
    api = _api()
    rx = [({}, {0: 1}, 40.0)]
    rx += [({0: 1, i: 1}, {i: 1}, 0.002 * (1 + i % 7)) for i in range(1, 101)]
    rx += [({i: 1}, {}, 0.01) for i in range(1, 101, 9)]
    spec = W.from_reactions(101, rx)
    x0 = np.concatenate([[0], np.random.default_rng(3).integers(5, 60, size=100)]).astype(np.int32)
    g = _run(api, spec, x0, 3.0, W.uniform_grid(3.0, 7), 64, 3)
    ref = oracle.simulate(spec, x0, 3.0, W.uniform_grid(3.0, 7), 3, 64, net_id=3, lazy=True)
    _assert_same(g, ref)
    assert ref["stats"]["firings"] > 64 * 100


def test_end_states_and_layouts():
    api = _api()
    # overflow stops before the jump
    spec = W.from_reactions(2, [({0: 1}, {0: 2}, 1.0), ({1: 1}, {}, 1.0)])
    x0 = np.array([2**31 - 10, 5], np.int32)
    g = _run(api, spec, x0, 100.0, [1e-12, 100.0], 6, 1)
    _assert_same(g, oracle.simulate(spec, x0, 100.0, [1e-12, 100.0], 1, 6, net_id=1, lazy=True))
    # firing cap, absorbing and per-trajectory initial states
    spec2, x02 = _net(12, 30, 31)
    t_end = float(3000 / W.initial_total_rate(spec2, x02))
    x0r = np.tile(x02, (16, 1))
    x0r[3] = 0
    grid = W.uniform_grid(t_end, 5)
    g = _run(api, spec2, x0r, t_end, grid, 16, 2, max_firings=500)
    _assert_same(g, oracle.simulate(spec2, x0r, t_end, grid, 2, 16, net_id=2, max_firings=500,
                                    lazy=True))
    # t_end = 0, empty grid, absorbing at the start
    g = _run(api, spec2, x02, 0.0, [0.0], 8, 4)
    _assert_same(g, oracle.simulate(spec2, x02, 0.0, [0.0], 4, 8, net_id=4, lazy=True))
    g = _run(api, W.pure_death(1.0), [0], 5.0, np.zeros(0), 4, 5)
    _assert_same(g, oracle.simulate(W.pure_death(1.0), [0], 5.0, np.zeros(0), 5, 4, net_id=5,
                                    lazy=True))
    # traj_offset split and a small grid give the same bits
    net2 = api.Network(spec2)
    kw = dict(seed=6, with_hash=True, method=api.METHOD_LAZY)
    a = api.simulate(net2, x02, t_end, [t_end], 40, **kw)
    b1 = api.simulate(net2, x02, t_end, [t_end], 15, traj_offset=0, grid=3, **kw)
    b2 = api.simulate(net2, x02, t_end, [t_end], 25, traj_offset=15, grid=1, **kw)
    torch.cuda.synchronize()
    for k in ("n", "T", "seq_hash", "x_final"):
        assert torch.equal(torch.cat([b1[k], b2[k]]), a[k]), k
    # partial outputs
    p = api.simulate(net2, x02, t_end, [t_end], 40, want=("n",), **kw)
    torch.cuda.synchronize()
    assert torch.equal(p["n"], a["n"])


def test_refuses_what_it_does_not_run():
    api = _api()
    w = W.lv_small(8)
    net = api.Network(w.net)
    with pytest.raises(api._lib.RtssaError):
        api.simulate(net, w.x0, 1.0, [1.0], 8, method=api.METHOD_LAZY, mapping=api.MAP_THREAD)


def _schedule(spec, t_end, seed):
    """Breakpoints at 0.2, 0.45, 0.7 and 1.3 of t_end (the last one never
    reached); each piece scales every rate by a factor in [0.2, 3] and the
    second switches about a third of the channels off."""
    rng = np.random.default_rng(1000 + seed)
    times = np.array([0.2, 0.45, 0.7, 1.3]) * t_end
    c = np.asarray(spec.c, dtype=np.float64)
    rates = c[None, :] * rng.uniform(0.2, 3.0, size=(times.size, c.size))
    rates[1, rng.random(c.size) < 0.35] = 0.0
    return times, rates


def _run_sched(api, spec, sched, x0, t_end, grid, R, seed):
    net = api.Network(spec)
    net.set_schedule(*sched)
    g = api.simulate(net, np.asarray(x0, np.int32), t_end, grid, R, seed=seed, net_id=seed,
                     with_hash=True, method=api.METHOD_LAZY)
    torch.cuda.synchronize()
    ref = oracle.simulate(spec, x0, t_end, grid, seed, R, net_id=seed, lazy=True,
                          schedule=sched)
    _assert_same(g, ref)
    return g


@pytest.mark.parametrize("N,M,seed", [
    (1, 1, 41), (3, 8, 42), (10, 64, 43), (12, 65, 44), (60, 513, 45), (250, 2000, 46),
    (500, 4097, 47),
])
def test_schedule_random_networks_bit_exact(N, M, seed):
    """Every clock runs to each breakpoint and the leaves and the whole tree
    are rebuilt with the new rates: the bits of the oracle's lazy form."""
    api = _api()
    spec, x0 = _net(N, M, seed)
    t_end = float(1200 / max(W.initial_total_rate(spec, x0), 1e-9))
    grid = np.sort(np.random.default_rng(seed).uniform(0, t_end, size=9))
    _run_sched(api, spec, _schedule(spec, t_end, seed), x0, t_end, grid, 24, seed)


def test_schedule_closed_forms_and_wide_touch():
    api = _api()
    # birth at 10, 0 on [1, 2), 30 after: nothing absorbed, T(3) = 40
    grid = np.array([0.5, 1.5, 2.5, 3.0])
    sched = (np.array([1.0, 2.0]), np.array([[0.0], [30.0]]))
    g = _run_sched(api, W.pure_birth(10.0), sched, [0], 3.0, grid, 256, 4)
    assert (_np(g["status"]) == api.TRAJ_OK).all()
    assert np.allclose(_np(g["T"])[:, 0], 40.0, rtol=1e-13, atol=0)
    # an all-zero last piece absorbs at the breakpoint
    sched = (np.array([1.0]), np.array([[0.0]]))
    g = _run_sched(api, W.pure_birth(10.0), sched, [0], 3.0, grid, 64, 5)
    assert (_np(g["status"]) == api.TRAJ_ABSORBED).all() and (_np(g["t_last"]) == 1.0).all()
    # Lotka-Volterra with a piece where predation stops
    w = W.lv_small(64)
    sched = (np.array([0.5, 1.0, 1.5]),
             np.array([[5.0, 0.02, 5.0], [10.0, 0.0, 2.0], [8.0, 0.01, 12.0]]))
    _run_sched(api, w.net, sched, w.x0, 2.0, W.uniform_grid(2.0, 21), 48, 3)
    # a firing that touches 100 channels, rates switched twice
    rx = [({}, {0: 1}, 40.0)]
    rx += [({0: 1, i: 1}, {i: 1}, 0.002 * (1 + i % 7)) for i in range(1, 101)]
    rx += [({i: 1}, {}, 0.01) for i in range(1, 101, 9)]
    spec = W.from_reactions(101, rx)
    x0 = np.concatenate([[0], np.random.default_rng(3).integers(5, 60, size=100)]).astype(np.int32)
    c = np.asarray(spec.c)
    sched = (np.array([1.0, 2.0]), np.stack([c * 2.0, c * 0.5]))
    _run_sched(api, spec, sched, x0, 3.0, W.uniform_grid(3.0, 7), 64, 6)


def test_schedule_in_a_batch():
    """Lazy items with and without schedules share one class (the scheduled
    kernel runs both); each equals its own run and the oracle."""
    api = _api()
    rng = np.random.default_rng(51)
    jobs, specs = [], []
    for i, M in enumerate([70, 300, 900, 130, 2000, 520]):
        N = max(2, M // 4)
        spec = W.random_network(N, M, rng, logc=(-1.0, 1.0), bimol_scale=0.05)
        x0 = rng.integers(0, 80, size=N).astype(np.int32)
        t_end = float(600 / max(W.initial_total_rate(spec, x0), 1e-9))
        net = api.Network(spec)
        sched = None
        if i % 2 == 0:
            sched = _schedule(spec, t_end, 60 + i)
            net.set_schedule(*sched)
        jobs.append(dict(net=net, x0=x0, t_end=t_end, sample_t=W.uniform_grid(t_end, 6), R=12,
                         net_id=i, method=api.METHOD_LAZY))
        specs.append((spec, sched))
    b = api.Batch(jobs, with_hash=True)
    b.run(seed=5)
    torch.cuda.synchronize()
    for j, o, (spec, sched) in zip(jobs, b.outputs, specs):
        solo = api.simulate(j["net"], j["x0"], j["t_end"], j["sample_t"], j["R"], seed=5,
                            net_id=j["net_id"], with_hash=True, method=api.METHOD_LAZY)
        torch.cuda.synchronize()
        for k in KEYS:
            assert torch.equal(o[k], solo[k]), (j["net_id"], k)
        ref = oracle.simulate(spec, j["x0"], j["t_end"], j["sample_t"], 5, j["R"],
                              net_id=j["net_id"], lazy=True, schedule=sched)
        _assert_same(o, ref, stats=False)
    b.close()


def test_large_random_network_full_size():
    """N = 1000, M = 4000, 512 trajectories of about 1e5 firings: Eq. 5 on
    every trajectory, two trajectories recomputed by the oracle."""
    api = _api()
    w = W.large_random()
    g = _run(api, w.net, w.x0, w.t_end, w.sample_t, w.R, w.seed)
    assert g["stats"]["firings"] > 50 * w.R * 1000
    n = _np(g["n"]).astype(np.int64)
    X = np.tile(w.x0.astype(np.int64), (w.R, 1))
    for k in range(w.net.M):
        for e in range(w.net.react_ptr[k], w.net.react_ptr[k + 1]):
            X[:, w.net.react_species[e]] -= w.net.react_sigma[e] * n[:, k]
        for e in range(w.net.prod_ptr[k], w.net.prod_ptr[k + 1]):
            X[:, w.net.prod_species[e]] += w.net.prod_mult[e] * n[:, k]
    assert np.array_equal(X, _np(g["x_final"]).astype(np.int64))
    for off in (0, 300):
        ref = oracle.simulate(w.net, w.x0, w.t_end, w.sample_t, w.seed, 1, net_id=w.seed,
                              traj_offset=off, lazy=True)
        _assert_same(g, ref, stats=False, sl=slice(off, off + 1))
