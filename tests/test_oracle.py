"""The CPU oracle against its pins (no GPU).

Also: each of several mutants, an implementation with one planted mistake
(all on the CPU, here in the test), must fail at least one pin.  That shows
the pins catch a dropped term, a wrong orientation, a wrong sign or log base,
or a counting slip.
"""
import math

import numpy as np
import pytest

import oracle
from tests import pins


def oracle_impl(X):
    return oracle.all_pairs(X)


def test_oracle_builds_and_loads():
    oracle.build(force=True)
    assert oracle.threads() >= 1


def test_oracle_golden_closed_forms():
    pins.check_golden(oracle_impl)


def test_oracle_brute_force_exhaustive():
    assert pins.check_brute_force(oracle_impl) > 4000


def test_oracle_complement_and_self():
    pins.check_complement(oracle_impl)


def test_oracle_exact_independence_is_zero():
    pins.check_product_zero(oracle_impl)


def test_oracle_constant_columns():
    pins.check_constant(oracle_impl)


def test_oracle_small_dependence_limit():
    pins.check_small_dependence(oracle_impl)


@pytest.mark.parametrize("seed,m,n", [(1, 1, 5), (2, 17, 9), (3, 301, 23), (4, 1000, 40)])
def test_oracle_identities_random(seed, m, n):
    rng = np.random.default_rng(seed)
    X = (rng.random((m, n)) < rng.uniform(0.0, 1.0, size=n)).astype(np.uint8)
    pins.check_identities(oracle_impl, X)
    pins.check_against_entropies(oracle_impl, X)


def test_oracle_pairs_matches_all_and_cells_sum_to_m():
    rng = np.random.default_rng(5)
    X = (rng.random((257, 31)) < 0.2).astype(np.uint8)
    n11, mi = oracle.all_pairs(X)
    pi, pj = np.triu_indices(31)
    r = oracle.pairs(X, pi, pj)
    assert np.array_equal(r["n11"], n11[pi, pj])
    assert np.array_equal(r["mi"], mi[pi, pj])
    assert np.array_equal(r["n11"] + r["n10"] + r["n01"] + r["n00"], np.full(len(pi), 257))
    c = oracle.colsums(X)
    assert np.array_equal(c, X.sum(axis=0))
    assert np.array_equal(np.diag(n11), c)


def test_oracle_pairs_cells_pinned():
    """n11, n10, n01, n00 of oracle.pairs one by one (golden hand counts, both orders, enumeration)."""
    pins.check_cells(oracle.pairs)


def test_oracle_transposed_layout_pinned():
    """pairs_t / colsums_t (column-major input) against the cell pins and the row-major functions."""
    pins.check_cells(lambda X, pi, pj: oracle.pairs_t(np.ascontiguousarray(X.T), pi, pj))
    rng = np.random.default_rng(12)
    X = (rng.random((1003, 37)) < rng.uniform(0.0, 0.8, size=37)).astype(np.uint8)
    Xt = np.ascontiguousarray(X.T)
    pi, pj = np.meshgrid(np.arange(37), np.arange(37), indexing="ij")
    pi, pj = pi.ravel(), pj.ravel()
    a, b = oracle.pairs(X, pi, pj), oracle.pairs_t(Xt, pi, pj)
    for k in ("n11", "n10", "n01", "n00", "mi"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(oracle.colsums_t(Xt), X.sum(axis=0))
    assert np.array_equal(oracle.colsums_t(Xt, n=20), oracle.colsums(X, n=20))


def test_cell_pin_catches_swapped_off_diagonal_cells():
    """A pair list that returns n10 and n01 swapped has the same MI (it is symmetric) and the
    same n11; the cell pin must still fail on it."""
    def swapped(X, pi, pj):
        r = oracle.pairs(X, pi, pj)
        r["n10"], r["n01"] = r["n01"], r["n10"]
        return r
    with pytest.raises(AssertionError):
        pins.check_cells(swapped)


def test_oracle_pitch_and_column_subset():
    rng = np.random.default_rng(6)
    full = (rng.random((100, 16)) < 0.4).astype(np.uint8)
    n11a, mia = oracle.all_pairs(full[:, :11])
    n11b, mib = oracle.all_pairs(full, n=11)            # pitch 16, first 11 columns
    assert np.array_equal(n11a, n11b) and np.array_equal(mia, mib)


def test_oracle_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.pairs(np.zeros((4, 3), np.uint8), [0], [3])
    with pytest.raises(ValueError):
        oracle.all_pairs(np.zeros((0, 3), np.uint8))


# ---------------------------------------------------------------- mutants --

def _counts(X):
    Xi = X.astype(np.int64)
    m = X.shape[0]
    g = Xi.T @ Xi
    c = Xi.sum(axis=0)
    return m, g, c


def _mi_generic(X, term, pair=lambda ci, cj, m: ((ci, cj), (ci, m - cj), (m - ci, cj), (m - ci, m - cj)),
                cells=None, scale=None):
    m, g, c = _counts(X)
    n = X.shape[1]
    mi = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            n11 = int(g[i, j]); ci = int(c[i]); cj = int(c[j])
            cl = (n11, ci - n11, cj - n11, m - ci - cj + n11) if cells is None else cells(n11, ci, cj, m)
            s = 0.0
            for nxy, (a, b) in zip(cl, pair(ci, cj, m)):
                s += term(nxy, a, b, m)
            mi[i, j] = s / m if scale is None else scale(s, m)
    return g, mi


def _t(nxy, a, b, m):
    return 0.0 if nxy == 0 else nxy * math.log2(nxy * m / (a * b))


MUTANTS = {
    "drops_n00_term": lambda X: _mi_generic(X, _t, cells=lambda n11, ci, cj, m: (n11, ci - n11, cj - n11, 0)),
    "swapped_orientation": lambda X: _mi_generic(
        X, _t, pair=lambda ci, cj, m: ((ci, cj), (m - ci, cj), (ci, m - cj), (m - ci, m - cj))),
    "natural_log": lambda X: _mi_generic(X, lambda nxy, a, b, m: 0.0 if nxy == 0 else nxy * math.log(nxy * m / (a * b))),
    "wrong_sign": lambda X: _mi_generic(X, lambda nxy, a, b, m: 0.0 if nxy == 0 else nxy * math.log2(a * b / (nxy * m))),
    "n00_sign_slip": lambda X: _mi_generic(X, _t, cells=lambda n11, ci, cj, m: (n11, ci - n11, cj - n11, m - ci - cj - n11 if m - ci - cj - n11 > 0 else 0)),
    "epsilon_in_log": lambda X: _mi_generic(X, lambda nxy, a, b, m: nxy * math.log2((nxy + 1e-3) * m / (a * b))),
    "no_division_by_m": lambda X: _mi_generic(X, _t, scale=lambda s, m: s),
    "or_instead_of_and": lambda X: (lambda g, mi: (((X.astype(np.int64)[:, :, None] | X.astype(np.int64)[:, None, :]).sum(0)), mi))(*_mi_generic(X, _t)),
}


def test_reference_python_implementation_passes():
    # The un-mutated Python form of the same arithmetic passes every pin, so a
    # mutant's failure below is due to its planted mistake alone.
    pins.run_all(lambda X: _mi_generic(X, _t))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name):
    with pytest.raises(AssertionError):
        pins.run_all(MUTANTS[name])
