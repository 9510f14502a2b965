"""rtssa_simulate_noalloc: the allocation-free variant of rtssa_simulate.

Called through the C ABI on the library's fixed scratch array, it must give
the same outputs, bit for bit, as rtssa_simulate on the same inputs, on two
calls in a row (the second smaller, so stale scratch from the first must not
leak into it), in every mapping and in the lazy form (whose resident grid
the array bounds).
"""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2103_00405_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("samples", "n", "T", "x_final", "t_last", "status", "seq_hash", "tie_step")


def _noalloc(net, x0d, t_end, sd, R, seed, like, method=0, stats=True):
    from paper_2103_00405_amd._lib import Options, Stats, check, lib
    out = {k: torch.full_like(like[k], -5 if like[k].dtype != torch.uint8 else 55) for k in like
           if k != "stats"}
    p = lambda t: None if t is None else C.c_void_p(t.data_ptr())
    smp = out.get("samples")
    st_r, st_g, st_n = smp.stride() if smp is not None else (0, 0, 0)
    opt = Options(0, 0, 0, 0, method)
    st = Stats()
    G = int(sd.numel())
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    check(lib().rtssa_simulate_noalloc(net.handle, p(x0d), 1 if x0d.dim() == 2 else 0,
                                       float(t_end), p(sd) if G else None, G, seed, 0, 0, R,
                                       p(smp), st_r, st_g, st_n, p(out.get("n")),
                                       p(out.get("T")), p(out.get("x_final")),
                                       p(out.get("t_last")), p(out.get("status")),
                                       p(out.get("seq_hash")), p(out.get("tie_step")),
                                       C.byref(opt), stream, C.byref(st) if stats else None))
    torch.cuda.synchronize()
    return out, st.as_dict()


def _compare(net, x0, t_end, grid, Rs, seed, method=0):
    from paper_2103_00405_amd import api
    dev = torch.device("cuda")
    x0d = torch.as_tensor(np.asarray(x0), dtype=torch.int32, device=dev)
    sd = torch.as_tensor(np.asarray(grid, np.float64), device=dev)
    want = tuple(k for k in KEYS if k != "seq_hash" and not (method == 3 and k in ("T", "tie_step")))
    for R in Rs:                       # two calls in a row, the second smaller
        xr = x0d if x0d.dim() == 1 else x0d[:R].contiguous()
        ref = api.simulate(net, xr, t_end, sd, R, seed=seed, with_hash=True, want=want,
                           method=method)
        torch.cuda.synchronize()
        got, st = _noalloc(net, xr, t_end, sd, R, seed, ref, method=method)
        for k in got:
            assert torch.equal(got[k], ref[k]), (R, k)
        for q in ("firings", "near_ties", "clamps", "status_count"):
            assert st[q] == ref["stats"][q], (R, q)
        assert st["mapping"] == ref["stats"]["mapping"]
        assert st["kernel_ms"] == 0.0
    return st


def test_noalloc_thread_mapping_two_calls():
    from paper_2103_00405_amd import api
    w = W.lv_small(512)
    net = api.Network(w.net)
    _compare(net, w.x0, 6.0, W.uniform_grid(6.0, 13), (512, 77), seed=3)


@pytest.mark.parametrize("M", [40, 700])
def test_noalloc_subwave_and_workgroup_two_calls(M):
    from paper_2103_00405_amd import api
    rng = np.random.default_rng(23 + M)
    spec = W.random_network(max(2, M // 4), M, rng, logc=(-1.0, 0.5), bimol_scale=0.01)
    x0 = rng.integers(0, 60, size=(200, spec.N)).astype(np.int32)   # per trajectory
    net = api.Network(spec)
    _compare(net, x0, 0.05, W.uniform_grid(0.05, 5), (200, 31), seed=5)


def test_noalloc_lazy_grid_bounded_by_the_array():
    from paper_2103_00405_amd import api
    from paper_2103_00405_amd._lib import Options, check, lib
    rng = np.random.default_rng(29)
    spec = W.random_network(1000, 4000, rng)
    x0 = rng.integers(0, 500, size=spec.N).astype(np.int32)
    net = api.Network(spec)
    nbytes = C.c_size_t()                                   # builds the lazy rows
    check(lib().rtssa_workspace_size(net.handle, 96, C.byref(Options(0, 0, 0, 0, 2)),
                                     C.byref(nbytes)))
    t_end = 2000.0 / W.initial_total_rate(spec, x0)
    st = _compare(net, x0, t_end, W.uniform_grid(t_end, 7), (96, 40), seed=9,
                  method=api.METHOD_LAZY)
    # 44 bytes per channel per resident wavefront: the 4 MiB array holds fewer
    # wavefronts than the 96 trajectories
    assert 1 <= st["grid"] < 96


def test_noalloc_refuses_a_workspace_and_unbuilt_rows():
    from paper_2103_00405_amd import api
    from paper_2103_00405_amd._lib import Options, Stats, lib
    w = W.lv_small(8)
    net = api.Network(w.net)
    x0d = torch.as_tensor(w.x0, dtype=torch.int32, device="cuda")
    ws = torch.empty(4096, dtype=torch.uint8, device="cuda")
    opt = Options(0, 0, 0, 0, 0, ws.data_ptr(), ws.numel())
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    nulls = [None] * 7
    rc = lib().rtssa_simulate_noalloc(net.handle, C.c_void_p(x0d.data_ptr()), 0, 1.0, None, 0, 1,
                                      0, 0, 8, None, 0, 0, 0, *nulls, C.byref(opt), stream,
                                      C.byref(Stats()))
    assert rc == -1 and b"no workspace" in lib().rtssa_last_error()
    rng = np.random.default_rng(31)
    big = api.Network(W.random_network(50, 200, rng))
    x0b = torch.zeros(50, dtype=torch.int32, device="cuda")
    rc = lib().rtssa_simulate_noalloc(big.handle, C.c_void_p(x0b.data_ptr()), 0, 1.0, None, 0, 1,
                                      0, 0, 8, None, 0, 0, 0, *nulls,
                                      C.byref(Options(0, 0, 0, 0, 2)), stream, C.byref(Stats()))
    assert rc == -1 and b"rows built" in lib().rtssa_last_error()
