"""GPU parity of the direct method on a sum tree (one wavefront per
trajectory, the tree of fan-out 8 in LDS).

Every output is compared bit for bit with the oracle's tree form on random
networks from 1 to 8000 channels, a firing that changes 100 propensities,
every end state, and the large random network (N = 1000, M = 4000) at its full
ensemble size, where sampled trajectories are recomputed by the oracle and
Eq. 5 is checked on all."""
import numpy as np
import pytest
import torch

import oracle
from paper_2103_00405_amd import workloads as W

pytestmark = pytest.mark.gpu


def _api():
    from paper_2103_00405_amd import api
    return api


def _np(t):
    return t.cpu().numpy()


def _assert_same(g, ref, stats=True, sl=slice(None)):
    assert np.array_equal(_np(g["samples"][sl]), ref["samples"])
    assert np.array_equal(_np(g["n"][sl]).view(np.uint32), ref["n"])
    assert np.array_equal(_np(g["x_final"][sl]), ref["x_final"])
    assert np.array_equal(_np(g["t_last"][sl]).view(np.uint64), ref["t_last"].view(np.uint64))
    assert np.array_equal(_np(g["status"][sl]), ref["status"])
    assert np.array_equal(_np(g["seq_hash"][sl]).view(np.uint64), ref["seq_hash"])
    if stats:
        for k in ("firings", "status_count"):
            assert g["stats"][k] == ref["stats"][k], k


def _net(N, M, seed):
    rng = np.random.default_rng(seed)
    spec = W.random_network(N, M, rng, logc=(-1.0, 1.0), bimol_scale=0.05)
    x0 = rng.integers(0, 80, size=N).astype(np.int32)
    return spec, x0


def _run(api, spec, x0, t_end, grid, R, seed, **kw):
    net = api.Network(spec)
    g = api.simulate(net, x0, t_end, grid, R, seed=seed, net_id=seed, with_hash=True,
                     method=api.METHOD_DIRECT_TREE, **kw)
    torch.cuda.synchronize()
    return g


def _ref(spec, x0, t_end, grid, R, seed, **kw):
    return oracle.direct_simulate(spec, x0, t_end, grid, seed, R, net_id=seed, tree=True, **kw)


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
    g = _run(api, spec, x0, t_end, grid, 24, seed)
    assert g["stats"]["mapping"] == api.MAP_WAVE and g["stats"]["block"] == 64
    _assert_same(g, _ref(spec, x0, t_end, grid, 24, seed))
    assert "T" not in g and "tie_step" not in g


def test_lotka_volterra_and_many_touched_channels():
    api = _api()
    w = W.lv_small(256)
    g = _run(api, w.net, w.x0, w.t_end, w.sample_t, 256, 1)
    _assert_same(g, _ref(w.net, w.x0, w.t_end, w.sample_t, 256, 1))
    rx = [({}, {0: 1}, 40.0)]
    rx += [({0: 1, i: 1}, {i: 1}, 0.002 * (1 + i % 7)) for i in range(1, 101)]
    rx += [({i: 1}, {}, 0.01) for i in range(1, 101, 9)]
    spec = W.from_reactions(101, rx)
    x0 = np.concatenate([[0], np.random.default_rng(3).integers(5, 60, size=100)]).astype(np.int32)
    g = _run(api, spec, x0, 3.0, W.uniform_grid(3.0, 7), 64, 3)
    ref = _ref(spec, x0, 3.0, W.uniform_grid(3.0, 7), 64, 3)
    _assert_same(g, ref)
    assert ref["stats"]["firings"] > 64 * 100


def test_end_states_and_errors():
    api = _api()
    spec = W.from_reactions(2, [({0: 1}, {0: 2}, 1.0), ({1: 1}, {}, 1.0)])
    x0 = np.array([2**31 - 10, 5], np.int32)
    g = _run(api, spec, x0, 100.0, [1e-12, 100.0], 6, 1)
    _assert_same(g, _ref(spec, x0, 100.0, [1e-12, 100.0], 6, 1))
    spec2, x02 = _net(12, 30, 31)
    t_end = float(3000 / W.initial_total_rate(spec2, x02))
    x0r = np.tile(x02, (16, 1))
    x0r[3] = 0
    grid = W.uniform_grid(t_end, 5)
    g = _run(api, spec2, x0r, t_end, grid, 16, 2, max_firings=500)
    _assert_same(g, _ref(spec2, x0r, t_end, grid, 16, 2, max_firings=500))
    g = _run(api, spec2, x02, 0.0, [0.0], 8, 4)
    _assert_same(g, _ref(spec2, x02, 0.0, [0.0], 8, 4))
    g = _run(api, W.pure_death(1.0), [0], 5.0, np.zeros(0), 4, 5)
    _assert_same(g, _ref(W.pure_death(1.0), [0], 5.0, np.zeros(0), 4, 5))
    # partial outputs and a trajectory offset split give the same bits
    net2 = api.Network(spec2)
    kw = dict(seed=6, with_hash=True, method=api.METHOD_DIRECT_TREE)
    a = api.simulate(net2, x02, t_end, [t_end], 40, **kw)
    b1 = api.simulate(net2, x02, t_end, [t_end], 15, traj_offset=0, grid=3, **kw)
    b2 = api.simulate(net2, x02, t_end, [t_end], 25, traj_offset=15, grid=1, **kw)
    p = api.simulate(net2, x02, t_end, [t_end], 40, want=("n",), **kw)
    torch.cuda.synchronize()
    for k in ("n", "seq_hash", "x_final"):
        assert torch.equal(torch.cat([b1[k], b2[k]]), a[k]), k
    assert torch.equal(p["n"], a["n"])
    # no internal times or near-ties; no rate schedule; one wavefront per trajectory
    assert "T" not in a and "tie_step" not in a
    with pytest.raises(api._lib.RtssaError):
        api.simulate(net2, x02, t_end, [t_end], 4, method=api.METHOD_DIRECT_TREE,
                     mapping=api.MAP_WORKGROUP)
    net2.set_schedule([t_end / 2], [np.asarray(spec2.c)])
    with pytest.raises(api._lib.RtssaError):
        api.simulate(net2, x02, t_end, [t_end], 4, method=api.METHOD_DIRECT_TREE)


def test_large_random_network_full_size():
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
        ref = oracle.direct_simulate(w.net, w.x0, w.t_end, w.sample_t, w.seed, 1, net_id=w.seed,
                                     traj_offset=off, tree=True)
        _assert_same(g, ref, stats=False, sl=slice(off, off + 1))
