"""GPU parity of the wavefront- and workgroup-per-trajectory mappings.

Every output is compared bit for bit with the CPU oracle on random networks
that exercise every reaction kind (order 0, 1, homodimer, heterodimer) and
several channel-to-lane layouts; the same network run through different
mappings and group sizes must give identical bits; the large random network
(N = 1000, M = 4000) is checked on full trajectories and, at its full
ensemble size, by Eq. 5 on every trajectory."""
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


def _assert_same(g, ref, stats=True):
    assert np.array_equal(_np(g["samples"]), ref["samples"])
    assert np.array_equal(_np(g["n"]).view(np.uint32), ref["n"])
    assert np.array_equal(_np(g["T"]).view(np.uint64), ref["T"].view(np.uint64))
    assert np.array_equal(_np(g["x_final"]), ref["x_final"])
    assert np.array_equal(_np(g["t_last"]).view(np.uint64), ref["t_last"].view(np.uint64))
    assert np.array_equal(_np(g["status"]), ref["status"])
    assert np.array_equal(_np(g["seq_hash"]).view(np.uint64), ref["seq_hash"])
    assert np.array_equal(_np(g["tie_step"]).view(np.uint32), ref["tie_step"])
    if stats:
        for k in ("firings", "near_ties", "clamps", "status_count"):
            assert g["stats"][k] == ref["stats"][k], k


def _net(N, M, seed, logc=(-1.0, 1.0), bimol=0.05):
    rng = np.random.default_rng(seed)
    spec = W.random_network(N, M, rng, logc=logc, bimol_scale=bimol)
    x0 = rng.integers(0, 80, size=N).astype(np.int32)
    return spec, x0


def _t_end_for(spec, x0, firings):
    return float(firings / max(W.initial_total_rate(spec, x0), 1e-9))


@pytest.mark.parametrize("N,M,mapping,block,seed", [
    (6, 12, 2, 0, 1), (10, 40, 2, 0, 2), (30, 100, 2, 0, 3), (80, 300, 2, 0, 4),
    (64, 513, 3, 256, 5), (40, 200, 3, 256, 6), (200, 900, 3, 256, 7), (300, 1500, 3, 512, 8),
    (500, 2000, 3, 1024, 9), (1000, 4000, 3, 1024, 10), (8, 8, 3, 1024, 11), (5, 65, 2, 0, 12),
    (6, 12, 2, 4, 13), (20, 60, 2, 8, 14), (30, 100, 2, 16, 15), (60, 200, 2, 32, 16),
    (120, 500, 2, 64, 17), (3, 9, 2, 4, 18),
    # every workgroup instantiation the autotuner can choose
    (30, 200, 3, 64, 19), (60, 500, 3, 64, 20), (100, 1000, 3, 64, 21),
    (200, 900, 3, 128, 22), (250, 1900, 3, 128, 23), (400, 2040, 3, 256, 24),
    (800, 3500, 3, 256, 25), (700, 3000, 3, 512, 26), (1200, 5000, 3, 1024, 27),
    # sub-wavefront with 2 and 4 slots per lane
    (4, 7, 2, 4, 28), (10, 30, 2, 8, 29), (20, 60, 2, 16, 30), (40, 120, 2, 32, 31),
    (60, 250, 2, 64, 32),
])
def test_random_networks_bit_exact(N, M, mapping, block, seed):
    api = _api()
    spec, x0 = _net(N, M, seed)
    t_end = _t_end_for(spec, x0, 1500)
    grid = np.sort(np.random.default_rng(seed).uniform(0, t_end, size=9))
    R = 24
    net = api.Network(spec)
    g = api.simulate(net, x0, t_end, grid, R, seed=seed, net_id=seed, mapping=mapping,
                     block=block, with_hash=True)
    torch.cuda.synchronize()
    assert g["stats"]["mapping"] == mapping
    ref = oracle.simulate(spec, x0, t_end, grid, seed, R, net_id=seed)
    _assert_same(g, ref)
    assert ref["stats"]["firings"] > 50 * R


def test_mappings_agree_on_the_same_network():
    """Thread, wavefront and workgroup mappings (and group sizes) give identical bits."""
    api = _api()
    w = W.lv_small(128)
    net = api.Network(w.net)
    runs = []
    for mapping, block in ((1, 0), (2, 0), (3, 256), (3, 1024)):
        o = api.simulate(net, w.x0, 6.0, W.uniform_grid(6.0, 13), 128, mapping=mapping,
                         block=block, with_hash=True)
        assert o["stats"]["mapping"] == mapping
        runs.append(o)
    for o in runs[1:]:
        for k in KEYS:
            assert torch.equal(o[k], runs[0][k]), k
    spec, x0 = _net(20, 60, 21)
    net2 = api.Network(spec)
    t_end = _t_end_for(spec, x0, 800)
    a = api.simulate(net2, x0, t_end, [t_end], 50, mapping=2, with_hash=True)
    for mapping, block in ((3, 256), (3, 512), (2, 8), (2, 16), (2, 32), (2, 64)):
        b = api.simulate(net2, x0, t_end, [t_end], 50, mapping=mapping, block=block,
                         with_hash=True)
        for k in KEYS:
            assert torch.equal(a[k], b[k]), (mapping, block, k)


def test_group_edge_cases():
    api = _api()
    # no channels, in the mappings chosen explicitly: every trajectory is
    # absorbed at t = 0
    spec0 = W.from_reactions(2, [])
    net0 = api.Network(spec0)
    x00 = np.array([3, 4], np.int32)
    for mapping in (2, 3):
        g = api.simulate(net0, x00, 1.0, [0.0, 1.0], 5, mapping=mapping, with_hash=True)
        ref = oracle.simulate(spec0, x00, 1.0, [0.0, 1.0], 1, 5)
        _assert_same(g, ref)
        assert (_np(g["status"]) == 1).all()
    # overflow stops before the jump
    spec = W.from_reactions(2, [({0: 1}, {0: 2}, 1.0), ({1: 1}, {}, 1.0)])
    net = api.Network(spec)
    x0 = np.array([2**31 - 10, 5], np.int32)
    for mapping in (2, 3):
        g = api.simulate(net, x0, 100.0, [1e-12, 100.0], 6, mapping=mapping, with_hash=True)
        ref = oracle.simulate(spec, x0, 100.0, [1e-12, 100.0], 1, 6)
        _assert_same(g, ref)
    # a count that starts clear of the top and climbs to it: the first firings
    # run without the jump's check, the last ones with it
    x0 = np.array([2**31 - 200, 5], np.int32)
    for mapping in (2, 3):
        g = api.simulate(net, x0, 100.0, [1e-12, 100.0], 6, mapping=mapping, with_hash=True)
        ref = oracle.simulate(spec, x0, 100.0, [1e-12, 100.0], 1, 6)
        assert (np.asarray(ref["status"]) == 2).all()          # every trajectory overflows
        _assert_same(g, ref)
    # firing cap and absorbing states, per-trajectory initial states
    spec2, x02 = _net(12, 30, 31)
    net2 = api.Network(spec2)
    t_end = _t_end_for(spec2, x02, 3000)
    x0r = np.tile(x02, (16, 1))
    x0r[3] = 0
    for mapping in (2, 3):
        g = api.simulate(net2, x0r, t_end, W.uniform_grid(t_end, 5), 16, mapping=mapping,
                         max_firings=500, with_hash=True)
        ref = oracle.simulate(spec2, x0r, t_end, W.uniform_grid(t_end, 5), 1, 16, max_firings=500)
        _assert_same(g, ref)
    # traj_offset split and grid size
    a = api.simulate(net2, x02, t_end, [t_end], 40, mapping=2, with_hash=True)
    b1 = api.simulate(net2, x02, t_end, [t_end], 15, mapping=2, traj_offset=0, with_hash=True,
                      grid=3)
    b2 = api.simulate(net2, x02, t_end, [t_end], 25, mapping=2, traj_offset=15, with_hash=True,
                      grid=1)
    for k in ("n", "T", "seq_hash"):
        assert torch.equal(torch.cat([b1[k], b2[k]]), a[k]), k


def test_large_random_network_full_trajectories():
    """N = 1000, M = 4000, t_end for about 1e5 firings: two full trajectories
    bit-exact against the oracle; the full 512-trajectory ensemble satisfies
    Eq. 5 and every status is a regular end state."""
    api = _api()
    w = W.large_random()
    net = api.Network(w.net)
    g = api.simulate(net, w.x0, w.t_end, w.sample_t, w.R, seed=w.seed, with_hash=True)
    torch.cuda.synchronize()
    st = g["stats"]
    assert st["mapping"] == api.MAP_WORKGROUP
    assert st["firings"] > 50 * w.R * 1000
    # Eq. 5 on every trajectory
    n = _np(g["n"]).astype(np.int64)
    X = np.tile(w.x0.astype(np.int64), (w.R, 1))
    for k in range(w.net.M):
        for e in range(w.net.react_ptr[k], w.net.react_ptr[k + 1]):
            X[:, w.net.react_species[e]] -= w.net.react_sigma[e] * n[:, k]
        for e in range(w.net.prod_ptr[k], w.net.prod_ptr[k + 1]):
            X[:, w.net.prod_species[e]] += w.net.prod_mult[e] * n[:, k]
    assert np.array_equal(X, _np(g["x_final"]).astype(np.int64))
    # two full trajectories recomputed by the oracle
    for off in (0, 300):
        ref = oracle.simulate(w.net, w.x0, w.t_end, w.sample_t, w.seed, 1, traj_offset=off)
        sl = slice(off, off + 1)
        assert np.array_equal(_np(g["samples"][sl]), ref["samples"])
        assert np.array_equal(_np(g["n"][sl]).view(np.uint32), ref["n"])
        assert np.array_equal(_np(g["T"][sl]).view(np.uint64), ref["T"].view(np.uint64))
        assert np.array_equal(_np(g["seq_hash"][sl]).view(np.uint64), ref["seq_hash"])


def test_workgroup_mapping_sees_new_rates():
    """The workgroup kernel reads each dependent channel's rate from the
    network's dependency records: after rtssa_network_set_rates a run must
    use the new rates (oracle on the new rates, bit for bit), in a single run
    and in a batch created before the change."""
    api = _api()
    spec, x0 = _net(150, 700, 41)
    net = api.Network(spec)
    t_end = _t_end_for(spec, x0, 800)
    grid = np.linspace(0.0, t_end, 5)
    g0 = api.simulate(net, x0, t_end, grid, 24, seed=3, with_hash=True, mapping=3)
    assert g0["stats"]["mapping"] == 3
    b = api.Batch([dict(net=net, x0=x0, t_end=t_end, sample_t=grid, R=24, net_id=0)],
                  with_hash=True)
    c2 = np.asarray(spec.c) * np.exp(np.random.default_rng(5).uniform(-1.0, 1.0, spec.M))
    net.set_rates(c2)
    spec2 = W.with_rates(spec, c2)
    ref = oracle.simulate(spec2, x0, t_end, grid, 3, 24)
    g1 = api.simulate(net, x0, t_end, grid, 24, seed=3, with_hash=True, mapping=3)
    torch.cuda.synchronize()
    _assert_same(g1, ref)
    b.run(seed=3)
    torch.cuda.synchronize()
    _assert_same(b.outputs[0], ref, stats=False)
    assert not np.array_equal(_np(g0["n"]), _np(g1["n"]))
