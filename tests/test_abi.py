"""CPU checks of the library boundary: libhc.so loads without a GPU, exports
every function include/*.h declares, and its host-side decompression (Alg. 6
with Alg. 1 and Alg. 4) recovers sparse vectors exactly."""
import ctypes
import glob
import itertools
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(hc_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    from paper_2408_17063_amd import hc
    names = declared_functions()
    assert len(names) >= 25
    for name in names:
        assert hasattr(hc.lib(), name), name
    assert set(hc.EXPORTED) == set(names)


def test_decompress_all_subsets_tiny():
    from paper_2408_17063_amd import hc
    p, N, s = 17, 8, 4
    for t in range(s + 1):
        for I in itertools.combinations(range(1, N + 1), t):
            vals = [(5 * i + 2) % p for i in I]
            w = [sum(pow(i, j, p) for i in I) % p for j in range(1, s + 1)]
            e = [sum(pow(i, j, p) * v for i, v in zip(I, vals)) % p for j in range(1, s + 1)]
            assert hc.decompress(p, N, s, w, [e]) == (list(I), [vals])


def test_decompress_matches_oracle_large():
    from paper_2408_17063_amd import hc
    from oracle import decompress as D
    p, N, s = 786433, 1 << 19, 256
    r = np.random.default_rng(3)
    I = sorted(int(x) + 1 for x in r.choice(N, size=200, replace=False))
    vals = r.integers(0, 1 << 16, size=(2, len(I)))
    x = np.array(I, dtype=np.int64)
    pw = x % p
    w, es = [], [[], []]
    for _ in range(s):
        w.append(int(pw.sum() % p))
        for c in range(2):
            es[c].append(int((pw * vals[c]).sum() % p))
        pw = pw * x % p
    idx, got = hc.decompress(p, N, s, w, es)
    assert idx == I and got == [list(map(int, vals[0])), list(map(int, vals[1]))]
    oidx, ogot = D.decompress_group(p, N, w, es)
    assert oidx == idx and ogot == got


def test_decompress_reports_overflow_and_bad_input():
    from paper_2408_17063_amd import hc
    p, N, s = 65537, 4096, 8
    r = np.random.default_rng(4)
    fails = 0
    for _ in range(10):
        I = sorted(int(x) + 1 for x in r.choice(N, size=s + 2, replace=False))
        w = [sum(pow(i, j, p) for i in I) % p for j in range(1, s + 1)]
        try:
            idx, _ = hc.decompress(p, N, s, w, [])
            assert idx != I
        except hc.HcError as ex:
            assert ex.status == hc.HC_EDECODE
            fails += 1
    assert fails >= 9
    with pytest.raises(hc.HcError):
        hc.decompress(p, p, s, [0] * s, [])  # N_group must be below p
