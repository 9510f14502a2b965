"""CPU oracle for the next-reaction random-time SSA (arXiv:2103.00405).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It is a ctypes wrapper
around the plain C implementation in rto.c (algorithm of paper section 4,
Table 2, with the readings listed at the top of rto.c) and dm.c (Gillespie's
direct method, an independent sampler of the same law).

A network is any object with attributes N, M, react_ptr, react_species,
react_sigma, prod_ptr, prod_species, prod_mult (int32 arrays, CSR lists) and
c (float64 rate constants).
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

STATUS_OK, STATUS_ABSORBED, STATUS_OVERFLOW, STATUS_MAX_FIRINGS = 0, 1, 2, 3
TIE_NONE = 0xFFFFFFFF

_lib = None


class _Net(C.Structure):
    _fields_ = [("N", C.c_int32), ("M", C.c_int32),
                ("react_ptr", C.c_void_p), ("react_species", C.c_void_p),
                ("react_sigma", C.c_void_p), ("prod_ptr", C.c_void_p),
                ("prod_species", C.c_void_p), ("prod_mult", C.c_void_p),
                ("c", C.c_void_p)]


class _Stats(C.Structure):
    _fields_ = [("firings", C.c_uint64), ("near_ties", C.c_uint64),
                ("clamps", C.c_uint64), ("status_count", C.c_uint64 * 4),
                ("hard_cases", C.c_int32)]


def load_library(path):
    """Load an oracle build from ``path`` with its ctypes signatures."""
    L = C.CDLL(path)
    _configure(L)
    return L


def lib():
    global _lib
    if _lib is None:
        _lib = load_library(_build.build(force=False))
    return _lib


def _configure(L):
    L.rto_exp1.restype = C.c_double
    L.rto_exp1.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
    L.rto_neglog_u53.restype = C.c_double
    L.rto_neglog_u53.argtypes = [C.c_uint64]
    L.rto_philox4x32_10.restype = None
    L.rto_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    L.rto_argmin2.restype = None
    L.rto_argmin2.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int32),
                              C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.rto_near_tie.restype = C.c_int
    L.rto_near_tie.argtypes = [C.c_double, C.c_double]
    L.rto_simulate.restype = C.c_int
    L.rto_simulate.argtypes = [C.POINTER(_Net), C.c_void_p, C.c_int32, C.c_double,
                               C.c_void_p, C.c_int32, C.c_uint64, C.c_uint32,
                               C.c_uint64, C.c_int64, C.c_uint64,
                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_int32, C.POINTER(_Stats)]
    L.rto_simulate_schedule.restype = C.c_int
    L.rto_simulate_schedule.argtypes = [C.POINTER(_Net), C.c_void_p, C.c_int32, C.c_double,
                                        C.c_void_p, C.c_int32, C.c_uint64, C.c_uint32,
                                        C.c_uint64, C.c_int64, C.c_uint64,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_int32, C.POINTER(_Stats),
                                        C.c_int32, C.c_void_p, C.c_void_p]
    L.rto_lazy_simulate.restype = C.c_int
    L.rto_lazy_simulate.argtypes = L.rto_simulate.argtypes
    L.rto_lazy_simulate_schedule.restype = C.c_int
    L.rto_lazy_simulate_schedule.argtypes = L.rto_simulate_schedule.argtypes
    L.rto_direct_simulate.restype = C.c_int
    L.rto_direct_simulate.argtypes = [C.POINTER(_Net), C.c_void_p, C.c_int32, C.c_double,
                                      C.c_void_p, C.c_int32, C.c_uint64, C.c_uint32,
                                      C.c_uint64, C.c_int64, C.c_uint64,
                                      C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_int32, C.POINTER(_Stats)]
    L.rto_direct_tree_simulate.restype = C.c_int
    L.rto_direct_tree_simulate.argtypes = L.rto_direct_simulate.argtypes
    L.rto_dm_simulate.restype = C.c_int
    L.rto_dm_simulate.argtypes = [C.POINTER(_Net), C.c_void_p, C.c_double, C.c_void_p,
                                  C.c_int32, C.c_uint64, C.c_int64, C.c_uint64,
                                  C.c_void_p, C.c_void_p, C.c_int32]


def _ptr(a):
    return a.ctypes.data if a is not None and a.size else None


def _net_struct(net):
    keep = dict(
        react_ptr=np.ascontiguousarray(net.react_ptr, dtype=np.int32),
        react_species=np.ascontiguousarray(net.react_species, dtype=np.int32),
        react_sigma=np.ascontiguousarray(net.react_sigma, dtype=np.int32),
        prod_ptr=np.ascontiguousarray(net.prod_ptr, dtype=np.int32),
        prod_species=np.ascontiguousarray(net.prod_species, dtype=np.int32),
        prod_mult=np.ascontiguousarray(net.prod_mult, dtype=np.int32),
        c=np.ascontiguousarray(net.c, dtype=np.float64),
    )
    # CSR arrays may be empty; give ctypes a valid pointer anyway
    for k in list(keep):
        if keep[k].size == 0:
            keep[k] = np.zeros(1, dtype=keep[k].dtype)
    s = _Net(int(net.N), int(net.M), *(keep[k].ctypes.data for k in
             ("react_ptr", "react_species", "react_sigma", "prod_ptr", "prod_species",
              "prod_mult", "c")))
    return s, keep


def philox4x32_10(ctr, key):
    """Philox4x32-10 block for one 4-word counter and 2-word key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().rto_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def exp1(seed, traj, net_id, k, n):
    """The Exp(1) draw E(seed, traj, net, k, n) of the n-th refresh of channel k."""
    return lib().rto_exp1(int(seed), int(traj), int(net_id), int(k), int(n))


def neglog_u53(m):
    """RN(-ln((m+1) 2^-53)); -1.0 flags an input the quad log cannot certify."""
    return lib().rto_neglog_u53(int(m))


def argmin2(values, _lib=None):
    """The selection step of Eq. 25 over ``values``: (mu, v1, v2) with mu the
    lowest index among the smallest values (-1 when none is finite), v1 that
    value and v2 the second smallest counted with multiplicity."""
    v = np.ascontiguousarray(values, dtype=np.float64)
    if v.size == 0:
        v = np.zeros(1, np.float64)
        M = 0
    else:
        M = int(v.size)
    mu, v1, v2 = C.c_int32(), C.c_double(), C.c_double()
    (_lib or lib()).rto_argmin2(v.ctypes.data, M, C.byref(mu), C.byref(v1), C.byref(v2))
    return int(mu.value), float(v1.value), float(v2.value)


def near_tie(d1, d2, _lib=None):
    """The near-tie rule: RN(d2 - d1) <= RN(1e-12 d1)."""
    return bool((_lib or lib()).rto_near_tie(float(d1), float(d2)))


def simulate(net, x0, t_end, sample_t, seed, R, net_id=0, traj_offset=0,
             max_firings=10_000_000, threads=0, _lib=None, schedule=None, lazy=False):
    """Run R trajectories of the random-time algorithm; returns a dict of arrays.
    schedule = (times [B], rates [B][M]) gives piecewise-constant rates: the
    network's c before times[0], rates[i] from times[i] on.  lazy = True runs
    the lazy form (dependency-graph updates, smallest absolute firing time)."""
    N, M = int(net.N), int(net.M)
    x0 = np.ascontiguousarray(x0, dtype=np.int32)
    per_traj = 1 if x0.ndim == 2 else 0
    s = np.ascontiguousarray(sample_t, dtype=np.float64)
    G = int(s.size)
    R = int(R)
    out = dict(
        samples=np.zeros((R, G, N), dtype=np.int32),
        n=np.zeros((R, M), dtype=np.uint32),
        T=np.zeros((R, M), dtype=np.float64),
        x_final=np.zeros((R, N), dtype=np.int32),
        t_last=np.zeros(R, dtype=np.float64),
        status=np.zeros(R, dtype=np.uint8),
        seq_hash=np.zeros(R, dtype=np.uint64),
        tie_step=np.zeros(R, dtype=np.uint32),
    )
    ns, keep = _net_struct(net)
    st = _Stats()
    L = _lib or lib()
    args = (C.byref(ns), _ptr(x0), per_traj, float(t_end), _ptr(s), G,
            int(seed), int(net_id), int(traj_offset), R, int(max_firings),
            _ptr(out["samples"]), _ptr(out["n"]), _ptr(out["T"]),
            _ptr(out["x_final"]), _ptr(out["t_last"]), _ptr(out["status"]),
            _ptr(out["seq_hash"]), _ptr(out["tie_step"]), int(threads), C.byref(st))
    if schedule is None:
        rc = (L.rto_lazy_simulate if lazy else L.rto_simulate)(*args)
    else:
        times = np.ascontiguousarray(schedule[0], dtype=np.float64)
        rates = np.ascontiguousarray(schedule[1], dtype=np.float64).reshape(times.size, M)
        fn = L.rto_lazy_simulate_schedule if lazy else L.rto_simulate_schedule
        rc = fn(*args, int(times.size), _ptr(times), _ptr(rates))
    if rc not in (0,):
        raise RuntimeError("oracle rto_simulate failed with code %d (hard cases %d)"
                           % (rc, st.hard_cases))
    out["stats"] = dict(firings=st.firings, near_ties=st.near_ties, clamps=st.clamps,
                        status_count=list(st.status_count))
    return out


def direct_simulate(net, x0, t_end, sample_t, seed, R, net_id=0, traj_offset=0,
                    max_firings=10_000_000, threads=0, _lib=None, tree=False):
    """Run R trajectories of Gillespie's direct method with keyed draws (one
    Philox block per firing); returns a dict of arrays like simulate, without
    T and tie_step.  tree = True sums and searches on the fixed sum tree of
    fan-out 8 instead of in channel order."""
    N, M = int(net.N), int(net.M)
    x0 = np.ascontiguousarray(x0, dtype=np.int32)
    per_traj = 1 if x0.ndim == 2 else 0
    s = np.ascontiguousarray(sample_t, dtype=np.float64)
    G = int(s.size)
    R = int(R)
    out = dict(
        samples=np.zeros((R, G, N), dtype=np.int32),
        n=np.zeros((R, M), dtype=np.uint32),
        x_final=np.zeros((R, N), dtype=np.int32),
        t_last=np.zeros(R, dtype=np.float64),
        status=np.zeros(R, dtype=np.uint8),
        seq_hash=np.zeros(R, dtype=np.uint64),
    )
    ns, keep = _net_struct(net)
    st = _Stats()
    L = _lib or lib()
    fn = L.rto_direct_tree_simulate if tree else L.rto_direct_simulate
    rc = fn(C.byref(ns), _ptr(x0), per_traj, float(t_end),
                                             _ptr(s), G,
                                   int(seed), int(net_id), int(traj_offset), R,
                                   int(max_firings), _ptr(out["samples"]), _ptr(out["n"]),
                                   _ptr(out["x_final"]), _ptr(out["t_last"]),
                                   _ptr(out["status"]), _ptr(out["seq_hash"]), int(threads),
                                   C.byref(st))
    if rc not in (0,):
        raise RuntimeError("oracle rto_direct_simulate failed with code %d (hard cases %d)"
                           % (rc, st.hard_cases))
    out["stats"] = dict(firings=st.firings, status_count=list(st.status_count))
    return out


def dm_simulate(net, x0, t_end, sample_t, seed, R, max_firings=10_000_000, threads=0):
    """Gillespie direct method (independent sampler of the same law)."""
    N, M = int(net.N), int(net.M)
    x0 = np.ascontiguousarray(x0, dtype=np.int32)
    s = np.ascontiguousarray(sample_t, dtype=np.float64)
    G = int(s.size)
    samples = np.zeros((int(R), G, N), dtype=np.int32)
    n = np.zeros((int(R), M), dtype=np.uint32)
    ns, keep = _net_struct(net)
    rc = lib().rto_dm_simulate(C.byref(ns), _ptr(x0), float(t_end), _ptr(s), G, int(seed),
                               int(R), int(max_firings), _ptr(samples), _ptr(n), int(threads))
    if rc != 0:
        raise RuntimeError("oracle rto_dm_simulate failed with code %d" % rc)
    return dict(samples=samples, n=n)


def threads_used(threads, R):
    nt = threads if threads > 0 else (os.cpu_count() or 1)
    return max(1, min(nt, int(R)))
