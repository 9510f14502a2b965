"""Pins for the oracle's random-number pieces: the Philox4x32-10 block
function and the correctly rounded -ln(u) that turns it into Exp(1) draws
(the per-channel internal-time gaps ln(1/r) of Eq. 23 and Eq. 26)."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat())
def test_philox_known_answers(ctr, key, expect):
    assert list(oracle.philox4x32_10(ctr, key)) == expect


def test_philox_matches_rocrand_engine():
    """Cross-check against rocRAND's host-callable Philox engine (run, not copied)."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    rng = np.random.default_rng(7)
    cases = []
    for _ in range(200):
        ctr = [int(x) for x in rng.integers(0, 2**32, size=4, dtype=np.uint64)]
        ctr[1] >>= 2   # the engine's 64-bit skip offset holds 4 * (ctr0 | ctr1 << 32)
        seed = int(rng.integers(0, 2**63, dtype=np.uint64)) * 2 + int(rng.integers(0, 2))
        cases.append((ctr, seed))
    cases.append(([0, 5, 7, 0], 1))
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "rrk")
        subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(HERE, "rocrand_philox_block.cpp")],
                       check=True, cwd=d, capture_output=True)
        inp = "".join("%d %d %d %d %d\n" % (c[0], c[1], c[2], c[3], s) for c, s in cases)
        res = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True)
    lines = res.stdout.strip().splitlines()
    assert len(lines) == len(cases)
    for (ctr, seed), line in zip(cases, lines):
        ref = [int(x) for x in line.split()]
        key = [seed & 0xFFFFFFFF, seed >> 32]
        assert list(oracle.philox4x32_10(ctr, key)) == ref


def test_philox_single_bit_avalanche():
    """Flipping any counter bit changes about half of the 128 output bits."""
    base = oracle.philox4x32_10([1, 2, 3, 4], [5, 6])
    flips = []
    for w in range(4):
        for b in range(0, 32, 7):
            c = [1, 2, 3, 4]
            c[w] ^= 1 << b
            out = oracle.philox4x32_10(c, [5, 6])
            flips.append(sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(base, out)))
    assert 48 < np.mean(flips) < 80


def _cr_neglog(m):
    """-ln((m+1) 2^-53) to 60 digits with mpmath, rounded to binary64 by mpmath."""
    import mpmath
    with mpmath.workdps(60):
        u = mpmath.mpf(m + 1) / mpmath.mpf(2) ** 53
        v = -mpmath.log(u)
        return float(mpmath.mpf(v, prec=53)) if v != 0 else 0.0


def _edge_ms():
    ms = {0, 1, 2, 3, 2**53 - 1, 2**53 - 2, 2**52 - 1, 2**52, 2**51 - 1, 2**40, 12345}
    for e in range(0, 53):
        ms.add((1 << e) - 1)          # u a power of two
        ms.add(min((1 << e), 2**53 - 1))
    return sorted(ms)


def test_neglog_correctly_rounded_edges():
    for m in _edge_ms():
        assert oracle.neglog_u53(m) == _cr_neglog(m), m


def test_neglog_correctly_rounded_random():
    rng = np.random.default_rng(11)
    # log-spread inputs: u from 2^-53 up to 1
    ms = set()
    for e in range(1, 54):
        lo, hi = (1 << (e - 1)) - 1, (1 << e) - 1
        for m in rng.integers(lo, hi, size=60, endpoint=True, dtype=np.uint64):
            ms.add(int(m))
    for m in rng.integers(2**53 - 2**20, 2**53, size=300, dtype=np.uint64):
        ms.add(int(m))
    for m in sorted(ms):
        assert oracle.neglog_u53(m) == _cr_neglog(m), m


def test_neglog_special_values():
    assert oracle.neglog_u53(2**53 - 1) == 0.0            # u = 1
    assert oracle.neglog_u53(2**52 - 1) == float(np.log(2.0))  # u = 1/2
    # u = 2^-53 gives 53 ln 2 correctly rounded
    assert oracle.neglog_u53(0) == _cr_neglog(0)


def test_exp1_keying_and_halves():
    """E(seed, traj, net, k, n) reads the block at counter (n>>1, k, traj, net):
    even n uses words (1:0), odd n words (3:2)."""
    seed, traj, net, k = 0x1234_5678_9ABC_DEF1, 77, 3, 5
    for n in range(6):
        w = oracle.philox4x32_10([n >> 1, k, traj, net], [seed & 0xFFFFFFFF, seed >> 32])
        word = (int(w[3]) << 32 | int(w[2])) if n & 1 else (int(w[1]) << 32 | int(w[0]))
        assert oracle.exp1(seed, traj, net, k, n) == _cr_neglog(word >> 11)


def test_exp1_distribution():
    """The draws are Exp(1): mean 1, variance 1, KS against the exponential law."""
    from scipy import stats
    vals = np.array([oracle.exp1(1, t, 0, k, n) for t in range(40) for k in range(5)
                     for n in range(50)])
    assert abs(vals.mean() - 1.0) < 4 / np.sqrt(vals.size)
    assert abs(vals.var() - 1.0) < 0.1
    assert stats.kstest(vals, "expon").pvalue > 1e-3
