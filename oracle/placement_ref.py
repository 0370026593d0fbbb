"""Independent re-implementation of the placement lookup rule (the advisor of
Sec. III-A), used only to check the library's integer lookup bit-exactly.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Rule: n_key = the smallest tabulated n >= n (below the first key: the first
key; the SE(3) ops ignore n); batch_key = the tabulated batch nearest in
|log2| distance, ties to the smaller key.  This version compares exact
rational log-distances with fractions (log2(b/k1) vs log2(k2/b) is decided by
b/k1 vs k2/b), a different route from the library's integer test.
"""
from __future__ import annotations

import math
import re
from fractions import Fraction


def n_key(keys, n):
    for k in keys:
        if k >= n:
            return k
    return keys[-1]


def batch_key(keys, b):
    best, best_d = None, None
    for k in keys:
        ratio = Fraction(b, k) if b >= k else Fraction(k, b)
        d = math.log2(ratio.numerator) - math.log2(ratio.denominator)
        # exact comparison via the ratio itself (log2 is monotone)
        if best is None or ratio < best_d or (ratio == best_d and k < best):
            best, best_d = k, ratio
    return best


def load_table(path):
    text = open(path).read()
    text = re.sub(r"//[^\n]*", "", text)
    nk = [int(v) for v in re.search(r"kTableN\[\d+\]\s*=\s*\{([^}]*)\}", text).group(1).split(",")]
    bk = [int(v) for v in re.search(r"kTableB\[\d+\]\s*=\s*\{([^}]*)\}", text).group(1).split(",")]
    body = text[text.index("kPlace"):]
    body = body[body.index("=") + 1:]
    # expand the stub macros if present
    macros = dict(re.findall(r"#define\s+(\w+)\s+(.*)", body))
    body = re.sub(r"#(define|undef)[^\n]*", "", body)
    for _ in range(4):
        for name, val in macros.items():
            body = re.sub(r"\b%s\b" % name, val, body)
    nums = [int(v) for v in re.findall(r"\d+", body)]
    n_ops = 8
    need = n_ops * len(nk) * len(bk) * 2
    nums = nums[:need]
    assert len(nums) == need, (len(nums), need)
    place = {}
    it = iter(nums)
    for op in range(n_ops):
        for ni in range(len(nk)):
            for bi in range(len(bk)):
                place[(op, ni, bi)] = (next(it), next(it))
    return {"n": nk, "b": bk, "place": place}


def lookup(table, op, n, batch):
    ni = 0 if op in (6, 7) else table["n"].index(n_key(table["n"], n))
    bi = table["b"].index(batch_key(table["b"], batch))
    return table["place"][(op, ni, bi)]
