"""GPU parity of piecewise-constant rate schedules (the time-dependent rates
of the paper's discussion, Eq. 28, solved piece by piece).

Every output is compared bit for bit with the CPU oracle run with the same
schedule, in each mapping (thread, sub-wavefront, wavefront, workgroup) and in
the batched form; a schedule with a piece of all-zero rates must not absorb
a trajectory while a breakpoint remains; removing a schedule restores the
plain run's bits; the direct method refuses a schedule."""
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


def _schedule(spec, t_end, seed, zero_piece=True):
    """Breakpoints at 0.2, 0.45, 0.7 and 1.3 of t_end (the last one is never
    reached); each piece scales every rate by a factor in [0.2, 3], and one
    piece switches about a third of the channels off."""
    rng = np.random.default_rng(1000 + seed)
    times = np.array([0.2, 0.45, 0.7, 1.3]) * t_end
    c = np.asarray(spec.c, dtype=np.float64)
    rates = c[None, :] * rng.uniform(0.2, 3.0, size=(times.size, c.size))
    if zero_piece:
        rates[1, rng.random(c.size) < 0.35] = 0.0
    return times, rates


def _net(N, M, seed):
    rng = np.random.default_rng(seed)
    spec = W.random_network(N, M, rng, logc=(-1.0, 1.0), bimol_scale=0.05)
    x0 = rng.integers(0, 80, size=N).astype(np.int32)
    return spec, x0


@pytest.mark.parametrize("N,M,mapping,block,seed", [
    (3, 3, 1, 0, 1), (5, 8, 1, 0, 2), (8, 8, 1, 0, 3), (4, 6, 1, 0, 4),
    (6, 12, 2, 4, 5), (10, 40, 2, 8, 6), (20, 60, 2, 16, 7), (40, 120, 2, 32, 8),
    (60, 250, 2, 64, 9), (30, 100, 2, 0, 10),
    (30, 200, 3, 64, 11), (60, 500, 3, 64, 12), (200, 900, 3, 128, 13),
    (250, 1900, 3, 128, 14), (400, 2040, 3, 256, 15), (700, 3000, 3, 512, 16),
    (64, 513, 3, 1024, 17),
])
def test_random_networks_with_schedule_bit_exact(N, M, mapping, block, seed):
    api = _api()
    spec, x0 = _net(N, M, seed)
    t_end = float(1200 / max(W.initial_total_rate(spec, x0), 1e-9))
    grid = np.sort(np.random.default_rng(seed).uniform(0, t_end, size=9))
    times, rates = _schedule(spec, t_end, seed)
    R = 24
    net = api.Network(spec)
    net.set_schedule(times, rates)
    g = api.simulate(net, x0, t_end, grid, R, seed=seed, net_id=seed, mapping=mapping,
                     block=block, with_hash=True)
    torch.cuda.synchronize()
    assert g["stats"]["mapping"] == mapping
    ref = oracle.simulate(spec, x0, t_end, grid, seed, R, net_id=seed,
                          schedule=(times, rates))
    _assert_same(g, ref)


@pytest.mark.parametrize("mapping,block", [(1, 0), (2, 4), (3, 64), (3, 256)])
def test_lotka_volterra_schedule_every_mapping(mapping, block):
    api = _api()
    w = W.lv_small(1000)
    times = np.array([0.5, 1.0, 1.5])
    rates = np.array([[5.0, 0.02, 5.0], [10.0, 0.0, 2.0], [8.0, 0.01, 12.0]])
    grid = W.uniform_grid(2.0, 21)
    net = api.Network(w.net)
    net.set_schedule(times, rates)
    g = api.simulate(net, w.x0, 2.0, grid, 48, seed=3, mapping=mapping, block=block,
                     with_hash=True)
    torch.cuda.synchronize()
    ref = oracle.simulate(w.net, w.x0, 2.0, grid, 3, 48, schedule=(times, rates))
    _assert_same(g, ref)


@pytest.mark.parametrize("mapping,block", [(1, 0), (2, 4), (3, 64)])
def test_zero_piece_does_not_absorb(mapping, block):
    """Birth at 10, then 0 on [1, 2), then 30: no trajectory is absorbed in
    the middle piece, and T(t_end) is the integral of the rate, 40."""
    api = _api()
    spec = W.pure_birth(10.0)
    times, rates = np.array([1.0, 2.0]), np.array([[0.0], [30.0]])
    net = api.Network(spec)
    net.set_schedule(times, rates)
    grid = np.array([0.5, 1.5, 2.5, 3.0])
    g = api.simulate(net, np.array([0], np.int32), 3.0, grid, 256, seed=4, mapping=mapping,
                     block=block, with_hash=True)
    torch.cuda.synchronize()
    ref = oracle.simulate(spec, [0], 3.0, grid, 4, 256, schedule=(times, rates))
    _assert_same(g, ref)
    assert (_np(g["status"]) == api.TRAJ_OK).all()
    assert np.allclose(_np(g["T"])[:, 0], 40.0, rtol=1e-13, atol=0)
    # an all-zero last piece absorbs (no breakpoint remains)
    net.set_schedule([1.0], [[0.0]])
    g = api.simulate(net, np.array([0], np.int32), 3.0, grid, 64, seed=4, mapping=mapping,
                     block=block, with_hash=True)
    torch.cuda.synchronize()
    ref = oracle.simulate(spec, [0], 3.0, grid, 4, 64, schedule=([1.0], [[0.0]]))
    _assert_same(g, ref)
    assert (_np(g["status"]) == api.TRAJ_ABSORBED).all()
    # the last clock run ends on the breakpoint, and nothing fires after it
    assert (_np(g["t_last"]) == 1.0).all()
    assert np.allclose(_np(g["T"])[:, 0], 10.0, rtol=1e-13, atol=0)


def test_removing_the_schedule_restores_the_plain_run():
    api = _api()
    spec, x0 = _net(12, 50, 21)
    t_end = float(800 / W.initial_total_rate(spec, x0))
    grid = W.uniform_grid(t_end, 5)
    net = api.Network(spec)
    plain = api.simulate(net, x0, t_end, grid, 32, seed=5, with_hash=True)
    net.set_schedule(*_schedule(spec, t_end, 21))
    sched = api.simulate(net, x0, t_end, grid, 32, seed=5, with_hash=True)
    net.set_schedule()
    again = api.simulate(net, x0, t_end, grid, 32, seed=5, with_hash=True)
    torch.cuda.synchronize()
    for k in KEYS:
        assert torch.equal(plain[k], again[k]), k
    assert not torch.equal(plain["seq_hash"], sched["seq_hash"])
    # a schedule whose only breakpoint lies past t_end changes nothing
    net.set_schedule([2.0 * t_end], [np.asarray(spec.c) * 7.0])
    late = api.simulate(net, x0, t_end, grid, 32, seed=5, with_hash=True)
    torch.cuda.synchronize()
    for k in KEYS:
        assert torch.equal(plain[k], late[k]), k


def test_schedule_errors():
    api = _api()
    w = W.lv_small(100)
    net = api.Network(w.net)
    with pytest.raises(api._lib.RtssaError):
        net.set_schedule([1.0, 1.0], np.ones((2, 3)))        # not increasing
    with pytest.raises(api._lib.RtssaError):
        net.set_schedule([0.0], np.ones((1, 3)))             # not > 0
    with pytest.raises(api._lib.RtssaError):
        net.set_schedule([1.0], [[1.0, -1.0, 1.0]])           # negative rate
    with pytest.raises(ValueError):
        net.set_schedule([1.0], np.ones((1, 2)))             # wrong shape
    net.set_schedule([1.0], np.ones((1, 3)))
    with pytest.raises(api._lib.RtssaError):
        api.simulate(net, w.x0, 2.0, [1.0], 8, method=api.METHOD_DIRECT)


def test_batch_mixes_scheduled_and_plain_networks():
    api = _api()
    rng = np.random.default_rng(31)
    jobs, specs = [], []
    for i, M in enumerate([3, 6, 8, 20, 60, 150, 400, 900, 5, 120, 1500]):
        N = max(2, M // 4)
        spec = W.random_network(N, M, rng, logc=(-1.0, 1.0), bimol_scale=0.05)
        x0 = rng.integers(0, 80, size=N).astype(np.int32)
        t_end = float(600 / max(W.initial_total_rate(spec, x0), 1e-9))
        net = api.Network(spec)
        sched = None
        if i % 2 == 0:
            sched = _schedule(spec, t_end, 40 + i)
            net.set_schedule(*sched)
        jobs.append(dict(net=net, x0=x0, t_end=t_end, sample_t=W.uniform_grid(t_end, 6),
                         R=10, net_id=i))
        specs.append((spec, sched))
    b = api.Batch(jobs, with_hash=True)
    b.run(seed=9)
    torch.cuda.synchronize()
    for j, o, (spec, sched) in zip(jobs, b.outputs, specs):
        solo = api.simulate(j["net"], j["x0"], j["t_end"], j["sample_t"], j["R"], seed=9,
                            net_id=j["net_id"], with_hash=True)
        torch.cuda.synchronize()
        for k in KEYS:
            assert torch.equal(o[k], solo[k]), (j["net_id"], k)
        ref = oracle.simulate(spec, j["x0"], j["t_end"], j["sample_t"], 9, j["R"],
                              net_id=j["net_id"], schedule=sched)
        assert np.array_equal(_np(o["n"]).view(np.uint32), ref["n"]), j["net_id"]
        assert np.array_equal(_np(o["T"]).view(np.uint64), ref["T"].view(np.uint64))
        assert np.array_equal(_np(o["samples"]), ref["samples"])
    # the batch holds the schedules' device addresses: no change meanwhile
    with pytest.raises(api._lib.RtssaError):
        jobs[0]["net"].set_schedule()
    b.close()
    jobs[0]["net"].set_schedule()
