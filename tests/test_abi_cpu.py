"""CPU checks of the GPU library: it loads, exports every declared symbol, its
numeric core (compiled for the host from the same source as the kernels)
matches the oracle bit for bit, and network validation rejects bad input
before touching the GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_2103_00405_amd import _lib
from paper_2103_00405_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rtssa.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rtssa_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    names = _declared()
    assert "rtssa_simulate" in names and "rtssa_score_grad" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)


def test_version_and_error_strings():
    L = _lib.lib()
    assert b"rtssa" in L.rtssa_version()
    assert isinstance(L.rtssa_last_error(), bytes)


def _host_neglog(m, force=0):
    s = C.c_int32(0)
    v = _lib.lib().rtssa_debug_neglog_host(int(m), force, C.byref(s))
    return v, s.value


def _mp_neglog(m):
    import mpmath
    with mpmath.workdps(60):
        v = -mpmath.log(mpmath.mpf(m + 1) / mpmath.mpf(2) ** 53)
        return float(mpmath.mpf(v, prec=53)) if v != 0 else 0.0


def _reference(m):
    v = oracle.neglog_u53(m)
    return _mp_neglog(m) if v < 0 else v   # the oracle flags inputs it cannot certify


def test_neglog_matches_oracle_on_uniform_draws():
    rng = np.random.default_rng(101)
    for m in rng.integers(0, 2**53, size=60000, dtype=np.uint64):
        v, _ = _host_neglog(int(m))
        assert v == _reference(int(m)), int(m)


def test_neglog_matches_oracle_on_edges_and_spread():
    rng = np.random.default_rng(102)
    ms = set(range(0, 2000)) | set(range(2**53 - 2000, 2**53))
    for e in range(1, 54):
        ms |= {(1 << e) - 1, (1 << e) - 2, 1 << (e - 1)}
        ms |= {int(x) for x in rng.integers((1 << (e - 1)) - 1, (1 << e) - 1, size=300,
                                            endpoint=True, dtype=np.uint64)}
    for m in sorted(ms):
        if m >= 2**53:
            continue
        v, _ = _host_neglog(m)
        assert v == _reference(m), m


def test_neglog_accurate_phase_alone_is_correctly_rounded():
    rng = np.random.default_rng(103)
    ms = [int(x) for x in rng.integers(0, 2**53 - 1, size=3000, dtype=np.uint64)]
    ms += [2**53 - 3, 2**53 - 2, 0, 1, 2**52 - 1, 2**52]
    for m in ms:
        v, slow = _host_neglog(m, force=1)
        assert slow == 1
        assert v == _reference(m), m


def test_neglog_hard_case_near_one():
    """u = 1 - 2^-52: the exact value lies 2^-156/3 above a rounding midpoint."""
    v, slow = _host_neglog(2**53 - 3)
    assert slow == 1 and v == float.fromhex("0x1.0000000000001p-52") == _mp_neglog(2**53 - 3)


def test_fast_phase_error_margin():
    """The fast phase must be far more accurate than the 2^-70 its rounding test assumes."""
    import mpmath
    L = _lib.lib()
    rng = np.random.default_rng(104)
    yh, yl = C.c_double(), C.c_double()
    worst = 0.0
    mpmath.mp.prec = 200
    ms = list(rng.integers(0, 2**53 - 1, size=4000, dtype=np.uint64))
    for e in range(1, 54):
        ms += list(rng.integers((1 << (e - 1)) - 1, (1 << e) - 1, size=40, dtype=np.uint64))
    for m in ms:
        m = int(m)
        L.rtssa_debug_neglog_fast_host(m, C.byref(yh), C.byref(yl))
        ex = -mpmath.log(mpmath.mpf(m + 1) / 2**53)
        worst = max(worst, float(abs(mpmath.mpf(yh.value) + mpmath.mpf(yl.value) - ex) / ex))
    assert worst < 2.0**-76, worst


def test_philox_host_matches_oracle():
    L = _lib.lib()
    rng = np.random.default_rng(105)
    out = np.zeros(4, np.uint32)
    for _ in range(500):
        ctr = rng.integers(0, 2**32, size=4, dtype=np.uint64).astype(np.uint32)
        key = rng.integers(0, 2**32, size=2, dtype=np.uint64).astype(np.uint32)
        L.rtssa_debug_philox_host(ctr.ctypes.data, int(key[0]), int(key[1]), out.ctypes.data)
        assert np.array_equal(out, oracle.philox4x32_10(ctr, key))


# ------------------------------------------------------ validation (no GPU needed)
def _create(N, M, rp, rs, rg, pp, ps, pm, c):
    arrs = [np.asarray(a, np.int32) if len(a) else np.zeros(1, np.int32)
            for a in (rp, rs, rg, pp, ps, pm)]
    cc = np.asarray(c if len(c) else [0.0], np.float64)
    h = C.c_void_p()
    rc = _lib.lib().rtssa_network_create(N, M, *[a.ctypes.data for a in arrs], cc.ctypes.data,
                                          C.byref(h))
    if rc == 0:
        _lib.lib().rtssa_network_destroy(h)
    return rc


@pytest.mark.parametrize("case,code", [
    ("trimolecular", -2), ("homotrimer", -2), ("bad_species", -1), ("neg_rate", -1),
    ("nan_rate", -1), ("tiny_rate", -1), ("repeated_reactant", -1), ("bad_offsets", -1),
    ("zero_sigma", -1), ("bad_product", -1),
])
def test_network_validation(case, code):
    base = dict(N=3, M=1, rp=[0, 1], rs=[0], rg=[1], pp=[0, 1], ps=[1], pm=[1], c=[1.0])
    b = dict(base)
    if case == "trimolecular":
        b.update(rp=[0, 3], rs=[0, 1, 2], rg=[1, 1, 1])
    elif case == "homotrimer":
        b.update(rg=[3])
    elif case == "bad_species":
        b.update(rs=[3])
    elif case == "neg_rate":
        b.update(c=[-1.0])
    elif case == "nan_rate":
        b.update(c=[float("nan")])
    elif case == "tiny_rate":
        b.update(c=[1e-300])
    elif case == "repeated_reactant":
        b.update(rp=[0, 2], rs=[0, 0], rg=[1, 1])
    elif case == "bad_offsets":
        b.update(rp=[1, 1])
    elif case == "zero_sigma":
        b.update(rg=[0])
    elif case == "bad_product":
        b.update(ps=[7])
    rc = _create(b["N"], b["M"], b["rp"], b["rs"], b["rg"], b["pp"], b["ps"], b["pm"], b["c"])
    assert rc == code, (case, rc, _lib.lib().rtssa_last_error())


def test_null_arguments_rejected():
    L = _lib.lib()
    assert L.rtssa_network_create(1, 1, None, None, None, None, None, None, None, None) == -1
    assert L.rtssa_simulate(None, None, 0, 1.0, None, 0, 1, 0, 0, 1, None, 0, 0, 0, None, None,
                            None, None, None, None, None, None, None, None) == -1
    assert L.rtssa_score_grad(None, None, None, 0, 0, 1, None, None, None, 0, None) == -1


def test_struct_layouts_match_header(tmp_path):
    """The binding's ctypes structures have the header's field offsets and
    sizes (a C program built against include/rtssa.h prints them)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"rtssa_stats": _lib.Stats, "rtssa_options": _lib.Options,
               "rtssa_batch_item": _lib.BatchItem}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "rtssa.h"',
             'int main(void) {']
    for cname, py in structs.items():
        lines.append('printf("%s sizeof %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));'
                         % (cname, f[0], cname, f[0]))
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for ln in out.split("\n"):
        if ln:
            c, f, v = ln.split()
            got[(c, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "sizeof")] == C.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])
