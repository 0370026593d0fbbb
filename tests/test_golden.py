"""Oracle against the hand-derived fixtures in tests/golden/."""
import os
from fractions import Fraction

import numpy as np

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def read_blocks(name):
    blocks, cur = {}, None
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line[0].isalpha():
            cur = line
            blocks[cur] = []
        else:
            blocks[cur].append([Fraction(t) for t in line.split()])
    return blocks


def test_laplacian4_factor_and_inverse():
    g = read_blocks("laplacian4.txt")
    A = np.array([[float(x) for x in r] for r in g["A"]])
    L, X, info = oracle.posv(A[None], np.eye(4)[None])
    assert info[0] == 0
    Ainv = np.array([[float(x) for x in r] for r in g["Ainv"]])
    assert np.max(np.abs(X[0] - Ainv)) <= 1e-15 * 8
    # squared entries of L (signs: diagonal +, subdiagonal -)
    Lsq = np.array([[float(x) for x in r] for r in g["Lsq"]])
    assert np.max(np.abs(L[0] * np.abs(L[0]) - np.where(np.eye(4) > 0, Lsq, -Lsq))) <= 1e-15 * 8


def test_singular3_info():
    g = read_blocks("singular3.txt")
    A = np.array([[float(x) for x in r] for r in g["A"]])
    _, info = oracle.potrf(A[None])
    assert info[0] == int(g["info"][0][0])
