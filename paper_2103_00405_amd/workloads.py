"""Seeded synthetic inputs: reaction networks, initial states, sample grids.

This module only builds input arrays.  It holds none of the simulation's
arithmetic and is the one piece of code that both the GPU path's tests and
the CPU oracle's tests use.

A network is a ``NetSpec``: N species, M reactions, reactant and product
lists in CSR form (reaction k reads entries [ptr[k], ptr[k+1])), and rate
constants c.  Molecularity (sum of reactant coefficients) is at most 2.
"""
from __future__ import annotations

import math
from typing import NamedTuple, Sequence

import numpy as np


class NetSpec(NamedTuple):
    N: int
    M: int
    react_ptr: np.ndarray
    react_species: np.ndarray
    react_sigma: np.ndarray
    prod_ptr: np.ndarray
    prod_species: np.ndarray
    prod_mult: np.ndarray
    c: np.ndarray
    names: tuple = ()


def from_reactions(N: int, reactions: Sequence, names: Sequence[str] = ()) -> NetSpec:
    """Build a NetSpec from ``[(reactants, products, c), ...]`` where reactants
    and products are dicts {species index: coefficient}."""
    rp, rs, rg, pp, ps, pm, cs = [0], [], [], [0], [], [], []
    for reac, prod, c in reactions:
        for j, s in sorted(reac.items()):
            if s > 0:
                rs.append(j)
                rg.append(s)
        for j, m in sorted(prod.items()):
            if m > 0:
                ps.append(j)
                pm.append(m)
        rp.append(len(rs))
        pp.append(len(ps))
        cs.append(float(c))
    i32 = lambda v: np.asarray(v, dtype=np.int32)
    return NetSpec(int(N), len(reactions), i32(rp), i32(rs), i32(rg), i32(pp), i32(ps),
                   i32(pm), np.asarray(cs, dtype=np.float64), tuple(names))


def with_rates(net: NetSpec, c) -> NetSpec:
    return net._replace(c=np.asarray(c, dtype=np.float64).copy())


# ----------------------------------------------------------------- catalog
def lotka_volterra(c=(1.0, 0.01, 1.0)) -> NetSpec:
    """Predator-prey: X1 -> 2 X1, X1 + X2 -> 2 X2, X2 -> 0 (the paper's Table 4
    model, with species A = X1 prey and B = X2 predator)."""
    return from_reactions(2, [({0: 1}, {0: 2}, c[0]),
                              ({0: 1, 1: 1}, {1: 2}, c[1]),
                              ({1: 1}, {}, c[2])], names=("X1", "X2"))


def birth_death(k1=50.0, k2=1.0) -> NetSpec:
    """0 -> A (k1), A -> 0 (k2 A)."""
    return from_reactions(1, [({}, {0: 1}, k1), ({0: 1}, {}, k2)], names=("A",))


def pure_birth(k=10.0) -> NetSpec:
    return from_reactions(1, [({}, {0: 1}, k)], names=("A",))


def pure_death(k=1.0) -> NetSpec:
    return from_reactions(1, [({0: 1}, {}, k)], names=("A",))


def isomerisation(c1=1.0, c2=2.0) -> NetSpec:
    """A -> B (c1), B -> A (c2)."""
    return from_reactions(2, [({0: 1}, {1: 1}, c1), ({1: 1}, {0: 1}, c2)], names=("A", "B"))


def dimerisation(c1=0.05, c2=1.0) -> NetSpec:
    """2A -> B (c1 A(A-1)/2), B -> 2A (c2 B)."""
    return from_reactions(2, [({0: 2}, {1: 1}, c1), ({1: 1}, {0: 2}, c2)], names=("A", "B"))


# ------------------------------------------------------------ random networks
def random_network(N: int, M: int, rng: np.random.Generator,
                   order_p=(0.1, 0.5, 0.4), logc=(-4.0, 1.0), bimol_scale=1e-3) -> NetSpec:
    """Random mass-action network: reactant order 0/1/2 with probabilities
    order_p, reactant and product species uniform with replacement (a species
    drawn twice becomes a coefficient 2), product count uniform on {0,1,2},
    c_k log-uniform on [10^logc0, 10^logc1], order-2 rates scaled by bimol_scale."""
    orders = rng.choice(3, size=M, p=np.asarray(order_p))
    nprod = rng.integers(0, 3, size=M)
    logcs = rng.uniform(logc[0], logc[1], size=M)
    reactions = []
    for k in range(M):
        reac: dict = {}
        for _ in range(orders[k]):
            j = int(rng.integers(0, N))
            reac[j] = reac.get(j, 0) + 1
        prod: dict = {}
        for _ in range(nprod[k]):
            j = int(rng.integers(0, N))
            prod[j] = prod.get(j, 0) + 1
        c = 10.0 ** logcs[k]
        if orders[k] == 2:
            c *= bimol_scale
        reactions.append((reac, prod, c))
    return from_reactions(N, reactions)


def initial_total_rate(net: NetSpec, x0) -> float:
    """Sum of mass-action rates at x0, used only to pick t_end for a target
    number of firings (a workload parameter, evaluated in plain float64)."""
    x = np.asarray(x0, dtype=np.float64)
    tot = 0.0
    for k in range(net.M):
        h = 1.0
        for e in range(net.react_ptr[k], net.react_ptr[k + 1]):
            v = x[net.react_species[e]]
            h *= v if net.react_sigma[e] == 1 else v * (v - 1.0) / 2.0
        tot += net.c[k] * h
    return tot


class Workload(NamedTuple):
    name: str
    net: NetSpec
    x0: np.ndarray
    t_end: float
    sample_t: np.ndarray
    R: int
    seed: int
    net_id: int = 0


def uniform_grid(t_end: float, G: int) -> np.ndarray:
    return np.linspace(0.0, t_end, G).astype(np.float64)


# ------------------------------------------------------------- configurations
def lv_small(R: int = 256) -> Workload:
    """Lotka-Volterra, c = (1, 0.01, 1), x0 = (100, 100), t_end = 20, 201-point
    grid, seed 1: the small parity case."""
    return Workload("lv_small", lotka_volterra((1.0, 0.01, 1.0)), np.array([100, 100], np.int32),
                    20.0, uniform_grid(20.0, 201), R, 1)


def lv_ensemble(R: int = 1 << 20) -> Workload:
    """Lotka-Volterra, c = (10, 0.01, 10), x0 = (1000, 1000), t_end = 5, 101-point
    grid, 2^20 trajectories: the ensemble-throughput case (the paper's Table 4 model)."""
    return Workload("lv_ensemble", lotka_volterra((10.0, 0.01, 10.0)),
                    np.array([1000, 1000], np.int32), 5.0, uniform_grid(5.0, 101), R, 1)


def large_random(R: int = 512, seed: int = 3, N: int = 1000, M: int = 4000,
                 target_firings: float = 1e5) -> Workload:
    """Random network N = 1000, M = 4000, x0 uniform on {0..500}, t_end chosen
    for about target_firings firings per trajectory, 512 trajectories."""
    rng = np.random.default_rng(seed)
    net = random_network(N, M, rng)
    x0 = rng.integers(0, 501, size=N).astype(np.int32)
    a0 = initial_total_rate(net, x0)
    t_end = float(target_firings / a0)
    return Workload("large_random", net, x0, t_end, uniform_grid(t_end, 101), R, 1)


def batch_networks(n_nets: int = 4096, seed: int = 4, target_firings: float = 2e4,
                   m_range=(3, 2048)):
    """Many independent random networks with M log-uniform in m_range and
    N = max(2, M // 4); per-network t_end for about target_firings firings."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_nets):
        M = int(round(math.exp(rng.uniform(math.log(m_range[0]), math.log(m_range[1])))))
        N = max(2, M // 4)
        net = random_network(N, M, rng)
        x0 = rng.integers(0, 501, size=N).astype(np.int32)
        a0 = initial_total_rate(net, x0)
        t_end = float(target_firings / a0) if a0 > 0 else 1.0
        out.append(Workload("batch_%d" % i, net, x0, t_end, uniform_grid(t_end, 101), 64, 1, i))
    return out


def bd_gradient(R: int = 1 << 18) -> Workload:
    """Birth-death k1 = 50, k2 = 1, x0 = 0, T = 2."""
    return Workload("bd_gradient", birth_death(50.0, 1.0), np.array([0], np.int32), 2.0,
                    np.array([2.0]), R, 1)


def lv_gradient(R: int = 1 << 18) -> Workload:
    w = lv_ensemble(R)
    return w._replace(name="lv_gradient", sample_t=np.array([5.0]))
