"""GPU parity of Gillespie's direct method (the paper's comparison method,
section 3, Eq. 17-22), run by the thread mapping with one Philox block per
firing: every output equal, bit for bit, to the oracle's keyed direct method,
on Lotka-Volterra and on random networks of every padded size, and through
the end states (absorption, overflow, firing cap)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2103_00405_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("samples", "n", "x_final", "t_last", "status", "seq_hash")


def _api():
    from paper_2103_00405_amd import api
    return api


def _check(g, ref):
    assert np.array_equal(g["samples"].cpu().numpy(), ref["samples"])
    assert np.array_equal(g["n"].cpu().numpy().view(np.uint32), ref["n"])
    assert np.array_equal(g["x_final"].cpu().numpy(), ref["x_final"])
    assert np.array_equal(g["t_last"].cpu().numpy().view(np.uint64), ref["t_last"].view(np.uint64))
    assert np.array_equal(g["status"].cpu().numpy(), ref["status"])
    assert np.array_equal(g["seq_hash"].cpu().numpy().view(np.uint64), ref["seq_hash"])
    assert g["stats"]["firings"] == ref["stats"]["firings"]
    assert g["stats"]["status_count"] == ref["stats"]["status_count"]


def _run(api, net, x0, t_end, grid, R, seed=1, **kw):
    g = api.simulate(api.Network(net), x0, t_end, grid, R, seed=seed, with_hash=True,
                     method=api.METHOD_DIRECT, **kw)
    torch.cuda.synchronize()
    return g


def test_lotka_volterra_small_bit_exact():
    api = _api()
    w = W.lv_small(256)
    g = _run(api, w.net, w.x0, w.t_end, w.sample_t, w.R, seed=w.seed)
    assert g["stats"]["mapping"] == api.MAP_THREAD
    ref = oracle.direct_simulate(w.net, w.x0, w.t_end, w.sample_t, w.seed, w.R)
    _check(g, ref)
    assert ref["stats"]["firings"] > 1_000_000


@pytest.mark.parametrize("N,M,seed", [(1, 2, 1), (2, 3, 2), (3, 4, 3), (4, 6, 4), (6, 8, 5),
                                      (8, 8, 6), (2, 7, 7), (8, 2, 8)])
def test_random_networks_bit_exact(N, M, seed):
    api = _api()
    rng = np.random.default_rng(seed)
    spec = W.random_network(N, M, rng, logc=(-1.0, 1.0), bimol_scale=0.05)
    x0 = rng.integers(0, 80, size=N).astype(np.int32)
    t_end = float(800 / max(W.initial_total_rate(spec, x0), 1e-9))
    grid = np.sort(rng.uniform(0, t_end, size=7))
    g = _run(api, spec, x0, t_end, grid, 64, seed=seed, net_id=seed)
    ref = oracle.direct_simulate(spec, x0, t_end, grid, seed, 64, net_id=seed)
    _check(g, ref)


def test_end_states_and_offsets():
    api = _api()
    # overflow stops before the jump
    spec = W.from_reactions(2, [({0: 1}, {0: 2}, 1.0), ({1: 1}, {}, 1.0)])
    x0 = np.array([2**31 - 10, 5], np.int32)
    g = _run(api, spec, x0, 100.0, [1e-12, 100.0], 6)
    _check(g, oracle.direct_simulate(spec, x0, 100.0, [1e-12, 100.0], 1, 6))
    # absorbing start and the firing cap, per-trajectory initial states
    w = W.lv_small(32)
    x0r = np.tile(w.x0, (32, 1))
    x0r[5] = 0
    g = _run(api, w.net, x0r, w.t_end, W.uniform_grid(w.t_end, 9), 32, max_firings=700)
    _check(g, oracle.direct_simulate(w.net, x0r, w.t_end, W.uniform_grid(w.t_end, 9), 1, 32,
                                     max_firings=700))
    # trajectory offsets: a split run equals the whole
    a = _run(api, w.net, w.x0, 4.0, [4.0], 40)
    b1 = _run(api, w.net, w.x0, 4.0, [4.0], 15)
    b2 = _run(api, w.net, w.x0, 4.0, [4.0], 25, traj_offset=15)
    for k in ("n", "seq_hash", "t_last"):
        assert torch.equal(torch.cat([b1[k], b2[k]]), a[k]), k


def test_direct_method_rejections():
    api = _api()
    w = W.lv_small(8)
    net = api.Network(w.net)
    with pytest.raises(RuntimeError):          # internal times are not defined for it
        api.simulate(net, w.x0, 1.0, [1.0], 8, want=("n",), out={
            "T": torch.empty((8, 3), dtype=torch.float64, device="cuda")},
            method=api.METHOD_DIRECT)
    with pytest.raises(RuntimeError):          # thread mapping only
        api.simulate(net, w.x0, 1.0, [1.0], 8, mapping=api.MAP_WAVE, method=api.METHOD_DIRECT)
    big = W.random_network(10, 20, np.random.default_rng(1))
    with pytest.raises(RuntimeError):
        api.simulate(api.Network(big), np.ones(10, np.int32), 1.0, [1.0], 8,
                     method=api.METHOD_DIRECT)
