"""Python face of librtssa: networks, ensemble simulation, score gradients.

Only argument marshalling happens here: every step of a simulation runs in
the HIP kernels behind the C ABI.  PyTorch provides device memory and the
current stream.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
from typing import Callable, Optional

import numpy as np
import torch

from . import _lib
from ._lib import Options, Stats, check, lib

MAP_AUTO, MAP_THREAD, MAP_WAVE, MAP_WORKGROUP = 0, 1, 2, 3
METHOD_RANDOM_TIME, METHOD_DIRECT, METHOD_LAZY, METHOD_DIRECT_TREE = 0, 1, 2, 3
TRAJ_OK, TRAJ_ABSORBED, TRAJ_OVERFLOW, TRAJ_MAX_FIRINGS = 0, 1, 2, 3
TIE_NONE = 0xFFFFFFFF


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _require_gpu(device):
    if not torch.cuda.is_available():
        raise RuntimeError("rtssa needs a ROCm GPU; none is visible")
    return torch.device(device)


class Network:
    """A compiled mass-action network (device tables owned by the library).

    ``spec`` is any object with N, M, react_ptr, react_species, react_sigma,
    prod_ptr, prod_species, prod_mult and c (see ``workloads.NetSpec``)."""

    def __init__(self, spec, device="cuda"):
        self.device = _require_gpu(device)
        self.N, self.M = int(spec.N), int(spec.M)
        arrs = [np.ascontiguousarray(getattr(spec, k), dtype=np.int32) for k in
                ("react_ptr", "react_species", "react_sigma", "prod_ptr", "prod_species",
                 "prod_mult")]
        c = np.ascontiguousarray(spec.c, dtype=np.float64)
        arrs = [a if a.size else np.zeros(1, np.int32) for a in arrs]
        if c.size == 0:
            c = np.zeros(1, np.float64)
        self._keep = arrs + [c]
        self._h = C.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().rtssa_network_create(self.N, self.M, *[a.ctypes.data for a in arrs],
                                             c.ctypes.data, C.byref(self._h)))
        self.c = c[: self.M].copy()
        self.schedule = None

    def set_rates(self, c):
        c = np.ascontiguousarray(c, dtype=np.float64)
        if c.size != self.M:
            raise ValueError("expected %d rates" % self.M)
        with torch.cuda.device(self.device):
            check(lib().rtssa_network_set_rates(self._h, c.ctypes.data))
        self.c = c.copy()

    def set_schedule(self, times=None, rates=None):
        """Piecewise-constant rates (Eq. 28 solved piece by piece): the
        network's c before times[0], rates[i] ([M]) from times[i] on.  Call
        with no arguments (or an empty ``times``) to remove the schedule."""
        t = np.ascontiguousarray([] if times is None else times, dtype=np.float64).ravel()
        B = int(t.size)
        r = np.ascontiguousarray(np.zeros((0, self.M)) if rates is None else rates,
                                 dtype=np.float64)
        if r.shape != (B, self.M):
            raise ValueError("rates must be [%d, %d], got %s" % (B, self.M, r.shape))
        with torch.cuda.device(self.device):
            check(lib().rtssa_network_set_schedule(self._h, B, t.ctypes.data if B else None,
                                                   r.ctypes.data if B else None))
        self.schedule = (t.copy(), r.copy()) if B else None

    def info(self):
        N, M, mp = C.c_int32(), C.c_int32(), C.c_int32()
        dep = C.c_int64()
        check(lib().rtssa_network_info(self._h, C.byref(N), C.byref(M), C.byref(dep), C.byref(mp)))
        return dict(N=N.value, M=M.value, dep_edges=dep.value, auto_mapping=mp.value)

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        try:
            if h and _lib._lib is not None:
                _lib._lib.rtssa_network_destroy(h)
        except Exception:      # interpreter shutdown: module globals may be gone
            pass
        self._h = None


def simulate(net: Network, x0, t_end: float, sample_t, R: int, seed: int = 1, net_id: int = 0,
             traj_offset: int = 0, max_firings: int = 10_000_000, mapping: int = MAP_AUTO,
             block: int = 0, grid: int = 0, want=("samples", "n", "T", "x_final", "t_last",
                                                  "status", "tie_step"),
             with_hash: bool = False, stats: bool = True, out: Optional[dict] = None,
             method: int = METHOD_RANDOM_TIME, workspace: Optional[torch.Tensor] = None):
    """Run R trajectories on the GPU; returns a dict of device tensors (+ 'stats').

    x0 is [N] (shared) or [R, N] (per trajectory), host or device.  sample_t is
    the sorted sample grid within [0, t_end].  ``want`` selects the outputs to
    produce; ``out`` may supply preallocated tensors with the same keys.
    ``method`` = METHOD_DIRECT runs Gillespie's direct method instead (thread
    mapping only; it has no T or tie_step outputs, which are then dropped from
    ``want``); METHOD_LAZY runs the lazy form for large networks (one
    wavefront per trajectory, dependency-graph updates, a minimum tree in
    LDS); METHOD_DIRECT_TREE the direct method on a sum tree in the same
    mapping (no T or tie_step either).  ``workspace`` (uint8 device tensor,
    256-byte aligned) may supply the call's workspace; by default one of
    ``rtssa_workspace_size`` bytes is taken from torch's allocator.  With
    stats=False the call only enqueues work on the current stream."""
    if method in (METHOD_DIRECT, METHOD_DIRECT_TREE):
        want = tuple(k for k in want if k not in ("T", "tie_step"))
    dev = net.device
    N, M, R = net.N, net.M, int(R)
    x0 = torch.as_tensor(np.asarray(x0) if not torch.is_tensor(x0) else x0, dtype=torch.int32)
    if x0.device.type == "cpu" and x0.numel() and int(x0.min()) < 0:
        # host input is checked before upload; device input is the caller's
        # (no device reduction or synchronisation per call)
        raise ValueError("initial counts must be >= 0")
    x0 = x0.to(dev).contiguous()
    per_traj = 1 if x0.dim() == 2 else 0
    if (per_traj and tuple(x0.shape) != (R, N)) or (not per_traj and tuple(x0.shape) != (N,)):
        raise ValueError("x0 must be [N] or [R, N] with N = %d, got %s" % (N, tuple(x0.shape)))
    s = torch.as_tensor(np.asarray(sample_t, dtype=np.float64) if not torch.is_tensor(sample_t)
                        else sample_t, dtype=torch.float64).to(dev).contiguous()
    G = int(s.numel())
    o = {} if out is None else dict(out)
    shapes = dict(samples=((R, G, N), torch.int32), n=((R, M), torch.int32),
                  T=((R, M), torch.float64), x_final=((R, N), torch.int32),
                  t_last=((R,), torch.float64), status=((R,), torch.uint8),
                  tie_step=((R,), torch.int32), seq_hash=((R,), torch.int64))
    keys = set(want) | ({"seq_hash"} if with_hash else set())
    for k in keys:
        if k not in o:
            shape, dt = shapes[k]
            o[k] = torch.empty(shape, dtype=dt, device=dev)
    smp = o.get("samples")
    st_r, st_g, st_n = (smp.stride() if smp is not None else (0, 0, 0))
    opt = Options(int(max_firings), int(mapping), int(block), int(grid), int(method))
    # the call's device workspace comes from torch's allocator (stream-ordered
    # reuse, no allocation inside the library)
    nbytes = C.c_size_t()
    with torch.cuda.device(dev):
        check(lib().rtssa_workspace_size(net.handle, R, C.byref(opt), C.byref(nbytes)))
    ws = workspace
    if ws is None or ws.numel() < nbytes.value:
        ws = torch.empty(max(1, nbytes.value), dtype=torch.uint8, device=dev)
    opt.workspace = ws.data_ptr()
    opt.workspace_bytes = ws.numel()
    st = Stats()
    with torch.cuda.device(dev):
        check(lib().rtssa_simulate(net.handle, _ptr(x0), per_traj, float(t_end),
                                   _ptr(s) if G else None, G, int(seed) & (2**64 - 1),
                                   int(net_id), int(traj_offset), R, _ptr(smp), st_r, st_g, st_n,
                                   _ptr(o.get("n")), _ptr(o.get("T")), _ptr(o.get("x_final")),
                                   _ptr(o.get("t_last")), _ptr(o.get("status")),
                                   _ptr(o.get("seq_hash")), _ptr(o.get("tie_step")),
                                   C.byref(opt), _stream(dev), C.byref(st) if stats else None))
    if stats:
        o["stats"] = st.as_dict()
    # ws returns to torch's pool here: its reuse is ordered after this call's
    # work on the same stream
    return o


def score_grad(f: torch.Tensor, n: torch.Tensor, T: torch.Tensor, baseline: bool = True):
    """Score-function estimate of d E[f] / d log c_k and its standard error."""
    dev = f.device
    R, M = int(n.shape[0]), int(n.shape[1])
    f = f.to(torch.float64).contiguous()
    n = n.contiguous()
    T = T.to(torch.float64).contiguous()
    grad = torch.empty(M, dtype=torch.float64, device=dev)
    se = torch.empty(M, dtype=torch.float64, device=dev)
    nbytes = C.c_size_t()
    check(lib().rtssa_score_grad_workspace_size(R, M, C.byref(nbytes)))
    ws = torch.empty(max(8, nbytes.value), dtype=torch.uint8, device=dev)
    with torch.cuda.device(dev):
        check(lib().rtssa_score_grad(_ptr(f), _ptr(n), _ptr(T), R, M, 1 if baseline else 0,
                                     _ptr(grad), _ptr(se), _ptr(ws), ws.numel(), _stream(dev)))
    return grad, se


class _Expectation(torch.autograd.Function):
    """E[f(X_T)] as a differentiable function of log c (score-function backward)."""

    @staticmethod
    def forward(ctx, log_c, net, f, x0, t_end, R, seed, baseline):
        c = torch.exp(log_c.detach().to(torch.float64)).cpu().numpy()
        net.set_rates(c)
        o = simulate(net, x0, t_end, [t_end], R, seed=seed, want=("x_final", "n", "T", "status"),
                     stats=False)
        # a path stopped by an overflow or the firing cap has neither X(t_end)
        # nor T_k(t_end): E[f] and the score n_k - T_k would be biased
        bad = int((o["status"] > TRAJ_ABSORBED).sum())
        if bad:
            raise RuntimeError("%d of %d trajectories stopped before t_end (overflow or firing "
                               "cap); the expectation and its gradient are undefined" % (bad, R))
        fx = f(o["x_final"]).to(torch.float64)
        ctx.save_for_backward(fx, o["n"], o["T"])
        ctx.baseline = baseline
        ctx.param_device = log_c.device
        ctx.results = o
        return fx.mean()

    @staticmethod
    def backward(ctx, grad_out):
        fx, n, T = ctx.saved_tensors
        g, _ = score_grad(fx, n, T, baseline=ctx.baseline)
        g = g.to(ctx.param_device)
        return (grad_out.to(torch.float64).to(g.device) * g), None, None, None, None, None, None, None


def expectation(log_c: torch.Tensor, net: Network, f: Callable, x0, t_end: float, R: int,
                seed: int = 1, baseline: bool = True) -> torch.Tensor:
    """Monte-Carlo E[f(X(t_end))] over R trajectories; differentiable in log_c
    through the score n_k - T_k(t_end) of each path."""
    return _Expectation.apply(log_c, net, f, x0, t_end, R, seed, baseline)


class Batch:
    """Many independent networks run by one persistent launch per size class
    (captured once into a hipGraph and replayed).  ``jobs`` is a list of dicts
    with keys net (Network), x0, t_end, sample_t, R and optionally net_id,
    traj_offset, method (METHOD_RANDOM_TIME, METHOD_LAZY or
    METHOD_DIRECT_TREE; the last has no T or tie_step) and weight (the job's
    expected work, e.g. its firings in an earlier run: orders each class's
    queue, heaviest first, and changes no result; default M x R); outputs are allocated
    here (per job: samples, n, T, x_final, t_last, status, seq_hash, tie_step)
    and returned by ``run``."""

    def __init__(self, jobs, max_firings=10_000_000, mapping=MAP_AUTO, plan_path=None,
                 want=("samples", "n", "T", "x_final", "t_last", "status", "tie_step"),
                 with_hash=False, device="cuda"):
        from ._lib import BatchItem
        self.device = _require_gpu(device)
        dev = self.device
        self.jobs, self.outputs, self._keep = [], [], []
        items = (BatchItem * len(jobs))()
        for i, j in enumerate(jobs):
            net = j["net"]
            R = int(j["R"])
            x0 = torch.as_tensor(np.asarray(j["x0"]), dtype=torch.int32).to(dev).contiguous()
            if tuple(x0.shape) not in ((net.N,), (R, net.N)):
                raise ValueError("job %d: x0 must be [N] or [R, N] with N = %d, got %s"
                                 % (i, net.N, tuple(x0.shape)))
            s = torch.as_tensor(np.asarray(j["sample_t"], dtype=np.float64),
                                dtype=torch.float64).to(dev).contiguous()
            G = int(s.numel())
            method = int(j.get("method", METHOD_RANDOM_TIME))
            jwant = tuple(k for k in want if method != METHOD_DIRECT_TREE or
                          k not in ("T", "tie_step"))
            o = {}
            shapes = dict(samples=((R, G, net.N), torch.int32), n=((R, net.M), torch.int32),
                          T=((R, net.M), torch.float64), x_final=((R, net.N), torch.int32),
                          t_last=((R,), torch.float64), status=((R,), torch.uint8),
                          tie_step=((R,), torch.int32), seq_hash=((R,), torch.int64))
            for k in set(jwant) | ({"seq_hash"} if with_hash else set()):
                shape, dt = shapes[k]
                o[k] = torch.empty(shape, dtype=dt, device=dev)
            smp = o.get("samples")
            st = smp.stride() if smp is not None else (0, 0, 0)
            it = items[i]
            it.net = net.handle
            it.x0 = x0.data_ptr() if x0.numel() else None
            it.x0_per_traj = 1 if x0.dim() == 2 else 0
            it.G = G
            it.t_end = float(j["t_end"])
            it.sample_t = s.data_ptr() if G else None
            it.net_id = int(j.get("net_id", i))
            it.method = method
            it.traj_offset = int(j.get("traj_offset", 0))
            it.R = R
            it.weight = float(j.get("weight", 0.0))
            it.samples = smp.data_ptr() if smp is not None and smp.numel() else None
            it.s_stride_r, it.s_stride_g, it.s_stride_n = st
            for k, f in (("n", "n_out"), ("T", "T_out"), ("x_final", "x_final"),
                         ("t_last", "t_last"), ("status", "status"), ("seq_hash", "seq_hash"),
                         ("tie_step", "tie_step")):
                t = o.get(k)
                setattr(it, f, t.data_ptr() if t is not None and t.numel() else None)
            self._keep += [x0, s, net]
            self.outputs.append(o)
            self.jobs.append(j)
        self._items = items
        self._h = C.c_void_p()
        opt = Options(int(max_firings), int(mapping), 0, 0, 0)
        with torch.cuda.device(dev):
            check(lib().rtssa_batch_create(items, len(jobs), C.byref(opt),
                                           plan_path.encode() if plan_path else None,
                                           C.byref(self._h)))

    def run(self, seed=1, use_graph=True, stats=True):
        st = Stats()
        with torch.cuda.device(self.device):
            check(lib().rtssa_batch_run(self._h, int(seed) & (2**64 - 1), 1 if use_graph else 0,
                                        _stream(self.device), C.byref(st) if stats else None))
        return st.as_dict() if stats else None

    def classes(self):
        n = C.c_int32()
        check(lib().rtssa_batch_info(self._h, -1, None, None, C.byref(n), None, None))
        out = []
        for c in range(n.value):
            m, l, k, mm = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
            r = C.c_int64()
            check(lib().rtssa_batch_info(self._h, c, C.byref(m), C.byref(l), C.byref(k),
                                         C.byref(r), C.byref(mm)))
            out.append(dict(mapping=m.value, lanes=l.value, items=k.value,
                            trajectories=r.value, max_M=mm.value))
        return out

    def class_items(self, cls):
        """Item indices of class ``cls`` in queue order (heaviest first)."""
        n = C.c_int32()
        check(lib().rtssa_batch_class_items(self._h, int(cls), None, 0, C.byref(n)))
        out = (C.c_int32 * max(1, n.value))()
        check(lib().rtssa_batch_class_items(self._h, int(cls), out, n.value, C.byref(n)))
        return [int(out[i]) for i in range(n.value)]

    def close(self):
        """Release the batch's device descriptors, streams and graph (its
        networks may then take a new rate schedule)."""
        h = getattr(self, "_h", None)
        self._h = None
        if h and _lib._lib is not None:
            _lib._lib.rtssa_batch_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:      # interpreter shutdown: module globals may be gone
            pass


def autotune(batch_jobs_items, plan_path, samples=16):
    """Write a plan file choosing lanes per trajectory / workgroup size per
    size class by timing short runs (see rtssa_autotune)."""
    b = batch_jobs_items
    with torch.cuda.device(b.device):
        n = lib().rtssa_autotune(b._items, len(b.jobs), int(samples), plan_path.encode(),
                                 _stream(b.device))
    if n < 0:
        check(n)
    return n
