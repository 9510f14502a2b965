"""rtssa: next-reaction random-time stochastic simulation on AMD MI355X.

The GPU library (librtssa.so, HIP kernels for gfx950 behind a C ABI) is
loaded on first use.  ``workloads`` holds the seeded input generators and
imports nothing else from this package.
"""
__all__ = ["Network", "simulate", "score_grad", "expectation", "workloads"]


def __getattr__(name):
    if name in ("Network", "simulate", "score_grad", "expectation", "MAP_AUTO", "MAP_THREAD",
                "MAP_WAVE", "MAP_WORKGROUP"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
