"""The C boundary as a caller in a capture-only setting uses it.

With a caller workspace (``rtssa_workspace_size`` bytes) and no stats,
``rtssa_simulate`` allocates nothing and does not synchronise, so it can be
captured into the caller's graph: every replay must reproduce the direct
call bit for bit.  The sample grid is checked on the device: a bad grid runs
nothing and marks every trajectory NOT_RUN.
"""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2103_00405_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("samples", "n", "T", "x_final", "t_last", "status", "seq_hash", "tie_step")


def _api():
    from paper_2103_00405_amd import api
    return api


def _capture_and_replay(net, x0, t_end, grid, R, seed, method=0, replays=3):
    api = _api()
    dev = torch.device("cuda")
    x0d = torch.as_tensor(np.asarray(x0), dtype=torch.int32, device=dev)
    sd = torch.as_tensor(np.asarray(grid, np.float64), device=dev)
    want = tuple(k for k in KEYS if k != "seq_hash" and not (method == 3 and k in ("T", "tie_step")))
    ref = api.simulate(net, x0d, t_end, sd, R, seed=seed, with_hash=True, want=want,
                       method=method)
    torch.cuda.synchronize()
    out = {k: torch.empty_like(ref[k]) for k in want + ("seq_hash",)}
    from paper_2103_00405_amd._lib import Options, check, lib
    nbytes = C.c_size_t()
    opt = Options(0, 0, 0, 0, method)
    check(lib().rtssa_workspace_size(net.handle, R, C.byref(opt), C.byref(nbytes)))
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):            # warm-up on the side stream, as torch advises
        api.simulate(net, x0d, t_end, sd, R, seed=seed, with_hash=True, want=want, out=out,
                     stats=False, workspace=ws, method=method)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        api.simulate(net, x0d, t_end, sd, R, seed=seed, with_hash=True, want=want, out=out,
                     stats=False, workspace=ws, method=method)
    torch.cuda.synchronize()
    for rep in range(replays):
        for t in out.values():               # eager work between the replays
            t.fill_(-7 if t.dtype != torch.uint8 else 77)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k in out:
            assert torch.equal(out[k], ref[k]), (rep, k)
    return ref


def test_simulate_captured_in_caller_graph_thread_mapping():
    api = _api()
    w = W.lv_small(512)
    net = api.Network(w.net)
    ref = _capture_and_replay(net, w.x0, 6.0, W.uniform_grid(6.0, 13), 512, seed=3)
    assert int(ref["n"].to(torch.int64).sum()) > 100000


def test_simulate_captured_in_caller_graph_large_mappings():
    api = _api()
    rng = np.random.default_rng(17)
    for M, method in ((40, 0), (700, 0), (300, api.METHOD_LAZY), (300, api.METHOD_DIRECT_TREE)):
        spec = W.random_network(max(2, M // 4), M, rng, logc=(-1.0, 0.5), bimol_scale=0.01)
        x0 = rng.integers(0, 60, size=spec.N).astype(np.int32)
        net = api.Network(spec)
        _capture_and_replay(net, x0, 0.05, W.uniform_grid(0.05, 5), 96, seed=5, method=method,
                            replays=2)


def test_score_grad_with_caller_workspace():
    api = _api()
    from paper_2103_00405_amd._lib import check, lib
    w = W.bd_gradient(R=4096)
    net = api.Network(w.net)
    o = api.simulate(net, w.x0, w.t_end, w.sample_t, w.R, seed=w.seed)
    f = o["x_final"][:, 0].to(torch.float64)
    g0, se0 = api.score_grad(f, o["n"], o["T"])
    nbytes = C.c_size_t()
    check(lib().rtssa_score_grad_workspace_size(w.R, 2, C.byref(nbytes)))
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
    g1 = torch.empty(2, dtype=torch.float64, device="cuda")
    se1 = torch.empty(2, dtype=torch.float64, device="cuda")
    p = lambda t: C.c_void_p(t.data_ptr())
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    check(lib().rtssa_score_grad(p(f), p(o["n"]), p(o["T"]), w.R, 2, 1, p(g1), p(se1), p(ws),
                                 ws.numel(), stream))
    torch.cuda.synchronize()
    assert torch.equal(g0, g1) and torch.equal(se0, se1)
    # too small a workspace is refused before any launch
    assert lib().rtssa_score_grad(p(f), p(o["n"]), p(o["T"]), w.R, 2, 1, p(g1), p(se1), p(ws),
                                  8, stream) == -1


@pytest.mark.parametrize("bad", ["decreasing", "past_t_end", "negative", "nan"])
def test_bad_grid_is_caught_on_the_device(bad):
    api = _api()
    from paper_2103_00405_amd._lib import RtssaError
    w = W.lv_small(100)
    net = api.Network(w.net)
    grid = np.linspace(0.0, 5.0, 600)
    if bad == "decreasing":
        grid[400], grid[401] = grid[401], grid[400]
    elif bad == "past_t_end":
        grid[-1] = 5.5
    elif bad == "negative":
        grid[0] = -1e-300
    else:
        grid[300] = np.nan
    with pytest.raises(RtssaError) as e:
        api.simulate(net, w.x0, 5.0, grid, 100)
    assert e.value.code == -1
    # without stats the call only enqueues: nothing runs, every status is NOT_RUN
    o = api.simulate(net, w.x0, 5.0, grid, 100, stats=False)
    torch.cuda.synchronize()
    assert (o["status"] == 255).all()
    # the same network and a good grid run normally afterwards
    o = api.simulate(net, w.x0, 5.0, np.sort(np.abs(np.nan_to_num(grid)).clip(0, 5.0)), 100)
    assert o["stats"]["bad_input"] == 0 and (o["status"] <= 1).all()
