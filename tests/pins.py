"""Pins for the CPU oracle: checks that come from the mathematics, not from
the oracle's own formula.

Each check takes an implementation `impl(X) -> (n11[n, n], mi[n, n])` for a
binary matrix X (rows = samples, columns = variables) and raises
AssertionError on a mismatch.  The oracle must pass all of them; the mutant
implementations in test_oracle.py (each with one planted mistake) must fail at
least one, which shows the pins are sensitive to the mistakes that matter.

Sources of truth used here:
  * brute-force enumeration of every binary matrix with m <= 4 rows, with MI
    computed a different way, H(X) + H(Y) - H(X,Y), in 40-digit decimal;
  * hand-derived closed forms in tests/golden/closed_forms.json;
  * textbook facts: MI(X;X) = H(X), MI(X; not X) = H(X), symmetry,
    0 <= MI <= min(H(X), H(Y)), MI = 0 exactly for columns that are exact
    products of their marginals, and the small-dependence limit
    MI ~ chi^2 / (2 m ln 2);
  * numpy's float64 X^T X (exact for these sizes) for the 1-1 counts.
"""
from __future__ import annotations

import itertools
import json
import math
import os
from decimal import Decimal, getcontext

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "closed_forms.json")

getcontext().prec = 40
_LN2 = Decimal(2).ln()


def _dlog2(x: int) -> Decimal:
    return Decimal(x).ln() / _LN2


def entropy_bits_decimal(counts, m: int) -> Decimal:
    """H = log2 m - (1/m) sum c log2 c over the nonzero counts (40 digits)."""
    s = Decimal(0)
    for c in counts:
        if c > 0:
            s += Decimal(c) * _dlog2(c)
    return _dlog2(m) - s / Decimal(m)


def mi_by_entropies(x: np.ndarray, y: np.ndarray) -> float:
    """MI(X;Y) = H(X) + H(Y) - H(X,Y) from explicit enumeration of the rows."""
    m = len(x)
    joint = {}
    for a, b in zip(x.tolist(), y.tolist()):
        joint[(a, b)] = joint.get((a, b), 0) + 1
    cx = [sum(1 for a in x.tolist() if a == v) for v in (0, 1)]
    cy = [sum(1 for b in y.tolist() if b == v) for v in (0, 1)]
    h = entropy_bits_decimal(cx, m) + entropy_bits_decimal(cy, m) - entropy_bits_decimal(joint.values(), m)
    return float(h)


def entropy_bits(c: int, m: int) -> float:
    """Binary entropy of a column with c ones out of m, in bits (float64)."""
    p = c / m
    return -sum(v * math.log2(v) for v in (p, 1.0 - p) if v > 0)


def check_brute_force(impl, max_m: int = 4, ns=(2, 3), tol: float = 1e-12) -> int:
    """Every binary matrix with 1 <= m <= max_m rows and n in `ns` columns."""
    checked = 0
    for n in ns:
        for m in range(1, max_m + 1):
            if m * n > 12:
                continue
            for bits in itertools.product((0, 1), repeat=m * n):
                X = np.array(bits, dtype=np.uint8).reshape(m, n)
                n11, mi = impl(X)
                for i in range(n):
                    for j in range(n):
                        want11 = int(np.sum((X[:, i] == 1) & (X[:, j] == 1)))
                        assert int(n11[i, j]) == want11, (X.tolist(), i, j, n11[i, j], want11)
                        want = mi_by_entropies(X[:, i], X[:, j])
                        assert abs(float(mi[i, j]) - want) <= tol, (X.tolist(), i, j, float(mi[i, j]), want)
                checked += 1
    return checked


def check_golden(impl, tol: float = 1e-15) -> None:
    with open(GOLDEN) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        X = np.stack([np.array(case["x"], dtype=np.uint8), np.array(case["y"], dtype=np.uint8)], axis=1)
        n11, mi = impl(X)
        assert int(n11[0, 1]) == case["n11"], case["name"]
        assert abs(float(mi[0, 1]) - case["mi_bits"]) <= tol, (case["name"], float(mi[0, 1]), case["mi_bits"])
        assert abs(float(mi[1, 0]) - case["mi_bits"]) <= tol, (case["name"], float(mi[1, 0]), case["mi_bits"])


def check_cells(pairs_impl) -> None:
    """The four cell counts of a pair list, each on its own (MI is symmetric in
    the two variables, so a swap of n10 and n01 leaves it unchanged and only a
    check of the cells themselves can see it).

    pairs_impl(X, pi, pj) returns a dict with int arrays n11, n10, n01, n00 for
    the pairs (pi[k], pj[k]).  Checked against the hand counts of the golden
    cases in both orders (n10 of (i, j) is n01 of (j, i)), and against the
    definitions counted by enumeration on every 2-column matrix of 1..6 rows:
    n10 = #{X_i = 1, X_j = 0}, n01 = #{X_i = 0, X_j = 1}."""
    with open(GOLDEN) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        X = np.stack([np.array(case["x"], dtype=np.uint8), np.array(case["y"], dtype=np.uint8)], axis=1)
        r = pairs_impl(X, [0, 1], [1, 0])
        got = [(int(r["n11"][k]), int(r["n10"][k]), int(r["n01"][k]), int(r["n00"][k])) for k in (0, 1)]
        want = (case["n11"], case["n10"], case["n01"], case["n00"])
        assert got[0] == want, (case["name"], "(x, y)", got[0], want)
        assert got[1] == (want[0], want[2], want[1], want[3]), (case["name"], "(y, x)", got[1])
    for m in range(1, 7):
        for bits in itertools.product((0, 1), repeat=2 * m):
            X = np.array(bits, dtype=np.uint8).reshape(m, 2)
            r = pairs_impl(X, [0, 1, 0], [1, 0, 0])
            for k, (i, j) in enumerate(((0, 1), (1, 0), (0, 0))):
                xi, xj = X[:, i].tolist(), X[:, j].tolist()
                want = tuple(sum(1 for a, b in zip(xi, xj) if (a, b) == cell) for cell in ((1, 1), (1, 0), (0, 1), (0, 0)))
                got = (int(r["n11"][k]), int(r["n10"][k]), int(r["n01"][k]), int(r["n00"][k]))
                assert got == want, (X.tolist(), i, j, got, want)


def check_identities(impl, X: np.ndarray, tol: float = 1e-12) -> None:
    """Symmetry, diagonal = entropy, bounds, and 1-1 counts equal to X^T X."""
    m, n = X.shape
    n11, mi = impl(X)
    gram = X.astype(np.float64).T @ X.astype(np.float64)          # exact: integers < 2^53
    assert np.array_equal(np.asarray(n11, dtype=np.int64), gram.astype(np.int64)), "n11 != X^T X"
    mi = np.asarray(mi, dtype=np.float64)
    assert np.array_equal(mi, mi.T), "MI not symmetric"
    c = X.sum(axis=0).astype(np.int64)
    H = np.array([entropy_bits(int(v), m) for v in c])
    assert np.allclose(np.diag(mi), H, rtol=0, atol=tol), "diagonal != H(X_i)"
    assert (mi >= -tol).all(), "negative MI"
    bound = np.minimum(H[:, None], H[None, :])
    assert (mi <= bound + tol).all(), "MI above min(H_i, H_j)"


def check_complement(impl, tol: float = 1e-12) -> None:
    """MI(X; not X) = H(X)."""
    rng = np.random.default_rng(7)
    for m in (5, 64, 999):
        x = (rng.random(m) < 0.3).astype(np.uint8)
        X = np.stack([x, 1 - x], axis=1)
        _, mi = impl(X)
        want = entropy_bits(int(x.sum()), m)
        assert abs(float(mi[0, 1]) - want) <= tol, (m, float(mi[0, 1]), want)


def product_columns(r: int, s: int, r1: int, s1: int) -> np.ndarray:
    """m = r*s rows; X_k = [k div s < r1], Y_k = [k mod s < s1]: exact independence."""
    k = np.arange(r * s)
    return np.stack([(k // s < r1), (k % s < s1)], axis=1).astype(np.uint8)


def check_product_zero(impl) -> None:
    """Columns that are exact products of their marginals give MI == 0.0 exactly."""
    for r, s, r1, s1 in ((2, 2, 1, 1), (3, 5, 1, 2), (7, 11, 3, 4), (40, 25, 13, 9), (100, 100, 1, 99)):
        X = product_columns(r, s, r1, s1)
        _, mi = impl(X)
        assert float(mi[0, 1]) == 0.0 and float(mi[1, 0]) == 0.0, (r, s, r1, s1, float(mi[0, 1]))


def check_constant(impl) -> None:
    """A constant column has zero entropy and zero MI with everything."""
    rng = np.random.default_rng(3)
    m = 37
    X = np.stack([np.zeros(m), np.ones(m), rng.random(m) < 0.5], axis=1).astype(np.uint8)
    _, mi = impl(X)
    for i in (0, 1):
        for j in range(3):
            assert float(mi[i, j]) == 0.0, (i, j, float(mi[i, j]))


def check_small_dependence(impl) -> None:
    """For weak dependence MI -> Delta^2 / (2 ln2 c_i (m-c_i) c_j (m-c_j)), Delta = n11 m - c_i c_j
    (the chi-square limit); the relative gap shrinks with the deviation."""
    m, ci, cj = 200_000, 60_000, 90_000
    base = ci * cj // m                     # 27,000: exactly independent n11
    for d in (3, 10, 30):
        n11 = base + d
        x = np.zeros(m, dtype=np.uint8)
        y = np.zeros(m, dtype=np.uint8)
        x[:ci] = 1
        y[:n11] = 1                          # rows 0..n11-1 are 1-1
        y[ci:ci + (cj - n11)] = 1            # the rest of Y's ones where X = 0
        X = np.stack([x, y], axis=1)
        _, mi = impl(X)
        delta = n11 * m - ci * cj
        approx = delta ** 2 / (2 * math.log(2) * ci * (m - ci) * cj * (m - cj))
        rel = abs(float(mi[0, 1]) - approx) / approx
        assert rel < 1e-2, (d, float(mi[0, 1]), approx, rel)


def check_against_entropies(impl, X: np.ndarray, tol: float = 1e-12) -> None:
    """Every pair of a random matrix against H(X) + H(Y) - H(X,Y) in float64 via numpy counts."""
    m, n = X.shape
    _, mi = impl(X)
    Xi = X.astype(np.int64)
    c = Xi.sum(axis=0)
    g = Xi.T @ Xi

    def H(*cnt):
        return -sum((v / m) * math.log2(v / m) for v in cnt if v > 0)

    for i in range(n):
        for j in range(n):
            n11 = int(g[i, j]); n10 = int(c[i] - g[i, j]); n01 = int(c[j] - g[i, j]); n00 = m - n11 - n10 - n01
            want = H(int(c[i]), m - int(c[i])) + H(int(c[j]), m - int(c[j])) - H(n11, n10, n01, n00)
            assert abs(float(mi[i, j]) - want) <= tol, (i, j, float(mi[i, j]), want)


def run_all(impl) -> None:
    rng = np.random.default_rng(11)
    check_golden(impl)
    check_complement(impl)
    check_product_zero(impl)
    check_constant(impl)
    check_small_dependence(impl)
    X = (rng.random((301, 23)) < rng.uniform(0.02, 0.7, size=23)).astype(np.uint8)
    X[:, 5] = X[:, 2] ^ (rng.random(301) < 0.1)
    check_identities(impl, X)
    check_against_entropies(impl, X)
    check_brute_force(impl)
