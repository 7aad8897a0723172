"""Pins for the categorical MI oracle: checks that come from the mathematics,
not from the oracle's own formula.

Each check takes an implementation `impl(X, levels) -> mi[v, v]` (bits) for a
matrix X of codes (rows = samples, column j holding codes 0 .. levels[j]-1)
and raises AssertionError on a mismatch.  The oracle must pass all of them;
the mutants in test_oracle_categorical.py (each with one planted mistake)
must fail at least one.

Sources of truth used here:
  * every matrix with up to 4 rows over small level sets, with MI computed a
    different way, H(X) + H(Y) - H(X,Y) in 40-digit decimal from an explicit
    enumeration of the rows;
  * hand-derived closed forms in tests/golden/categorical_closed_forms.json;
  * textbook facts: symmetry, MI(X;X) = H(X), invariance under a relabelling
    of either variable's codes, MI(X; g(X)) = H(g(X)), the data-processing
    bound MI(X; g(Y)) <= MI(X; Y), 0 <= MI <= min(H(X), H(Y)), MI = 0 exactly
    for a product design, the binary case L = 2 against the binary
    entropies, and the small-dependence limit MI -> chi^2 / (2 m ln 2).
"""
from __future__ import annotations

import itertools
import json
import math
import os

import numpy as np

from tests.pins import entropy_bits_decimal

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "categorical_closed_forms.json")


def mi_by_entropies(x, y) -> float:
    """H(X) + H(Y) - H(X,Y) from explicit counts of the rows (40 digits)."""
    x = list(map(int, x)); y = list(map(int, y))
    m = len(x)
    cx, cy, cxy = {}, {}, {}
    for a, b in zip(x, y):
        cx[a] = cx.get(a, 0) + 1
        cy[b] = cy.get(b, 0) + 1
        cxy[(a, b)] = cxy.get((a, b), 0) + 1
    h = entropy_bits_decimal(cx.values(), m) + entropy_bits_decimal(cy.values(), m) - entropy_bits_decimal(cxy.values(), m)
    return float(h)


def entropy_of(x) -> float:
    m = len(x)
    _, c = np.unique(np.asarray(x), return_counts=True)
    return float(entropy_bits_decimal([int(v) for v in c], m))


def check_brute_force(impl, tol: float = 1e-12) -> int:
    """Every 2-variable matrix with m rows over the listed level pairs."""
    checked = 0
    for (la, lb), ms in (((3, 2), (1, 2, 3, 4)), ((3, 3), (1, 2, 3)), ((2, 4), (2, 3)), ((4, 4), (2,)), ((1, 3), (2, 3))):
        for m in ms:
            cells = list(itertools.product(range(la), range(lb)))
            for rows in itertools.product(cells, repeat=m):
                X = np.array(rows, dtype=np.uint8).reshape(m, 2)
                mi = np.asarray(impl(X, [la, lb]), dtype=np.float64)
                want = mi_by_entropies(X[:, 0], X[:, 1])
                assert abs(mi[0, 1] - want) <= tol, (X.tolist(), (la, lb), mi[0, 1], want)
                assert abs(mi[1, 0] - want) <= tol, (X.tolist(), (la, lb), mi[1, 0], want)
                for d in (0, 1):
                    h = entropy_of(X[:, d])
                    assert abs(mi[d, d] - h) <= tol, (X.tolist(), d, mi[d, d], h)
                checked += 1
    return checked


def check_golden(impl, tol: float = 1e-15) -> None:
    with open(GOLDEN) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        X = np.stack([np.array(case["x"]), np.array(case["y"])], axis=1).astype(np.uint8)
        mi = np.asarray(impl(X, case["levels"]), dtype=np.float64)
        for v in (mi[0, 1], mi[1, 0]):
            assert abs(v - case["mi_bits"]) <= tol, (case["name"], v, case["mi_bits"])


def check_identities(impl, X: np.ndarray, levels, tol: float = 1e-12) -> None:
    """Symmetry, diagonal = entropy, bounds, every pair against the entropies."""
    m, v = X.shape
    mi = np.asarray(impl(X, levels), dtype=np.float64)
    assert mi.shape == (v, v)
    assert np.array_equal(mi, mi.T), "MI not symmetric"
    H = np.array([entropy_of(X[:, j]) for j in range(v)])
    assert np.allclose(np.diag(mi), H, rtol=0, atol=tol), "diagonal != H(X_j)"
    assert (mi >= -tol).all(), "negative MI"
    assert (mi <= np.minimum(H[:, None], H[None, :]) + tol).all(), "MI above min(H_i, H_j)"
    for i in range(v):
        for j in range(i + 1, v):
            want = mi_by_entropies(X[:, i], X[:, j])
            assert abs(mi[i, j] - want) <= tol, (i, j, mi[i, j], want)


def check_relabel_invariance(impl, tol: float = 1e-12) -> None:
    """Permuting the codes of every variable leaves MI unchanged."""
    rng = np.random.default_rng(21)
    levels = [2, 3, 5, 7, 4]
    m = 513
    X = np.stack([rng.integers(0, L, size=m) for L in levels], axis=1).astype(np.uint8)
    X[:, 2] = (X[:, 1] + (rng.random(m) < 0.3) * rng.integers(0, 5, size=m)) % 5
    base = np.asarray(impl(X, levels), dtype=np.float64)
    for _ in range(3):
        Y = X.copy()
        for j, L in enumerate(levels):
            perm = rng.permutation(L)
            Y[:, j] = perm[X[:, j]]
        got = np.asarray(impl(Y, levels), dtype=np.float64)
        assert np.allclose(got, base, rtol=0, atol=tol), np.abs(got - base).max()


def check_functions_of_x(impl, tol: float = 1e-12) -> None:
    """MI(X; f(X)) = H(f(X)); for a bijective f that is H(X)."""
    rng = np.random.default_rng(22)
    m = 777
    x = rng.integers(0, 6, size=m)
    f_bij = np.array([3, 0, 5, 1, 4, 2])[x]
    f_many = np.array([0, 0, 1, 2, 2, 1])[x]
    X = np.stack([x, f_bij, f_many], axis=1).astype(np.uint8)
    mi = np.asarray(impl(X, [6, 6, 3]), dtype=np.float64)
    assert abs(mi[0, 1] - entropy_of(x)) <= tol, (mi[0, 1], entropy_of(x))
    assert abs(mi[0, 2] - entropy_of(f_many)) <= tol, (mi[0, 2], entropy_of(f_many))


def check_data_processing(impl, tol: float = 1e-12) -> None:
    """Merging codes of Y cannot raise MI(X; Y)."""
    rng = np.random.default_rng(23)
    m = 1000
    x = rng.integers(0, 4, size=m)
    y = (x * 2 + rng.integers(0, 3, size=m)) % 8
    g = np.array([0, 0, 1, 1, 2, 2, 3, 3])[y]
    X = np.stack([x, y, g], axis=1).astype(np.uint8)
    mi = np.asarray(impl(X, [4, 8, 4]), dtype=np.float64)
    assert mi[0, 2] <= mi[0, 1] + tol, (mi[0, 2], mi[0, 1])
    assert mi[0, 1] - mi[0, 2] > 1e-3, "the merge should lose information here"


def product_design(wx, wy) -> np.ndarray:
    """Rows (x, y) repeated wx[x] * wy[y] times: n_xy m = r_x s_y exactly."""
    rows = [(a, b) for a, ca in enumerate(wx) for b, cb in enumerate(wy) for _ in range(ca * cb)]
    return np.array(rows, dtype=np.uint8)


def check_product_zero(impl) -> None:
    for wx, wy in (([1, 1], [1, 1, 1]), ([2, 3, 1], [1, 4]), ([5, 1, 2, 3], [2, 1, 3, 1, 1]), ([1, 0, 3], [2, 2])):
        X = product_design(wx, wy)
        mi = np.asarray(impl(X, [len(wx), len(wy)]), dtype=np.float64)
        assert mi[0, 1] == 0.0 and mi[1, 0] == 0.0, (wx, wy, mi[0, 1])


def check_single_level(impl) -> None:
    """A variable with one level has zero entropy and zero MI with everything."""
    rng = np.random.default_rng(24)
    m = 41
    X = np.stack([np.zeros(m), rng.integers(0, 5, size=m), rng.integers(0, 2, size=m)], axis=1).astype(np.uint8)
    mi = np.asarray(impl(X, [1, 5, 2]), dtype=np.float64)
    assert (mi[0, :] == 0.0).all() and (mi[:, 0] == 0.0).all(), mi


def check_binary_case(impl, tol: float = 1e-12) -> None:
    """Levels 2 everywhere: the binary MI from the 2 x 2 cell counts."""
    rng = np.random.default_rng(25)
    m, n = 301, 9
    X = (rng.random((m, n)) < rng.uniform(0.05, 0.9, size=n)).astype(np.uint8)
    mi = np.asarray(impl(X, [2] * n), dtype=np.float64)
    for i in range(n):
        for j in range(n):
            a = int(np.sum((X[:, i] == 1) & (X[:, j] == 1))); b = int(np.sum((X[:, i] == 1) & (X[:, j] == 0)))
            c = int(np.sum((X[:, i] == 0) & (X[:, j] == 1))); d = m - a - b - c
            ci, cj = a + b, a + c

            def h(*cnt):
                return -sum((k / m) * math.log2(k / m) for k in cnt if k > 0)

            want = h(ci, m - ci) + h(cj, m - cj) - h(a, b, c, d)
            assert abs(mi[i, j] - want) <= tol, (i, j, mi[i, j], want)


def rows_from_table(table) -> np.ndarray:
    """Rows (x, y) repeated table[x][y] times."""
    t = np.asarray(table, dtype=np.int64)
    xs, ys = np.nonzero(t >= 0)
    reps = t[xs, ys]
    return np.stack([np.repeat(xs, reps), np.repeat(ys, reps)], axis=1).astype(np.uint8)


def check_small_dependence(impl) -> None:
    """Weak dependence: MI -> chi^2 / (2 m ln 2), chi^2 = sum (n - E)^2 / E over
    the cells, for a table whose deviations from independence sum to zero in
    every row and column; the relative gap shrinks with the deviation."""
    r = np.array([300_000, 200_000, 500_000])          # row marginals (m = 1,000,000)
    c = np.array([250_000, 250_000, 500_000])          # column marginals
    m = int(r.sum())
    E = np.outer(r, c) // m                             # exact: products divisible by m
    pattern = np.array([[1, -1, 0], [-1, 2, -1], [0, -1, 1]])  # zero row and column sums
    for d in (20, 60, 200):
        table = E + d * pattern
        X = rows_from_table(table)
        mi = float(np.asarray(impl(X, [3, 3]), dtype=np.float64)[0, 1])
        chi2 = float(((table - E) ** 2 / E).sum())
        approx = chi2 / (2 * m * math.log(2))
        rel = abs(mi - approx) / approx
        assert rel < 1e-2, (d, mi, approx, rel)


def random_case(seed: int, m: int, levels):
    """Codes with skewed level frequencies and some dependent columns."""
    rng = np.random.default_rng(seed)
    cols = []
    for j, L in enumerate(levels):
        p = rng.dirichlet(np.full(L, 0.7))
        col = rng.choice(L, size=m, p=p)
        if j >= 2 and j % 3 == 2:
            src = cols[j - 1]
            keep = rng.random(m) < 0.6
            col = np.where(keep, src % L, col)
        cols.append(col)
    return np.stack(cols, axis=1).astype(np.uint8)


def run_all(impl) -> None:
    check_golden(impl)
    check_product_zero(impl)
    check_single_level(impl)
    check_functions_of_x(impl)
    check_data_processing(impl)
    check_relabel_invariance(impl)
    check_binary_case(impl)
    check_small_dependence(impl)
    levels = [2, 3, 4, 5, 3, 9, 2, 16, 6]
    check_identities(impl, random_case(26, 257, levels), levels)
    check_brute_force(impl)
