"""The categorical CPU oracle against its pins (no GPU).

Also a Python form of the indicator-Gram derivation (each variable's codes
1 .. L-1 as indicator columns, their Gram product giving the cells with both
codes >= 1, and the cells with a code 0 derived from the marginals and m, the
way Section 3.1 derives n10, n01 and n00 from n11), checked against the same
pins; and mutants of it, each with one planted mistake, that must fail at
least one pin.
"""
import math

import numpy as np
import pytest

import oracle
from tests import pins_cat


def oracle_impl(X, levels):
    return oracle.cat_all_pairs(X, levels)


def test_categorical_oracle_golden():
    pins_cat.check_golden(oracle_impl)


def test_categorical_oracle_brute_force_exhaustive():
    assert pins_cat.check_brute_force(oracle_impl) > 3000


def test_categorical_oracle_product_zero_and_single_level():
    pins_cat.check_product_zero(oracle_impl)
    pins_cat.check_single_level(oracle_impl)


def test_categorical_oracle_functions_relabel_and_processing():
    pins_cat.check_functions_of_x(oracle_impl)
    pins_cat.check_relabel_invariance(oracle_impl)
    pins_cat.check_data_processing(oracle_impl)


def test_categorical_oracle_small_dependence_limit():
    pins_cat.check_small_dependence(oracle_impl)


def test_categorical_oracle_binary_case():
    pins_cat.check_binary_case(oracle_impl)
    rng = np.random.default_rng(27)
    X = (rng.random((211, 13)) < 0.3).astype(np.uint8)
    _, mib = oracle.all_pairs(X)
    assert np.allclose(oracle.cat_all_pairs(X, [2] * 13), mib, rtol=0, atol=1e-14)


@pytest.mark.parametrize("seed,m,levels", [(1, 1, [3, 2]), (2, 97, [2, 3, 4, 5]), (3, 1000, [7, 1, 16, 2, 3, 255, 4])])
def test_categorical_oracle_identities_random(seed, m, levels):
    X = pins_cat.random_case(seed, m, levels)
    pins_cat.check_identities(oracle_impl, X, levels)


def test_categorical_table_counts_rows():
    rng = np.random.default_rng(28)
    levels = [3, 5, 2]
    X = np.stack([rng.integers(0, L, size=300) for L in levels], axis=1).astype(np.uint8)
    for i in range(3):
        for j in range(3):
            t = oracle.cat_table(X, levels, i, j)
            want = np.bincount(X[:, i].astype(np.int64) * levels[j] + X[:, j], minlength=levels[i] * levels[j])
            assert np.array_equal(t.ravel(), want)
            # the matrix holds the i <= j orientation in both triangles
            assert abs(oracle.cat_from_table(t) - oracle.cat_all_pairs(X, levels)[i, j]) <= 1e-15
            if i <= j:
                assert oracle.cat_from_table(t) == oracle.cat_all_pairs(X, levels)[i, j]


def test_categorical_oracle_pitch_and_rejects():
    rng = np.random.default_rng(29)
    full = rng.integers(0, 3, size=(50, 8)).astype(np.uint8)
    a = oracle.cat_all_pairs(full[:, :5], [3] * 5)
    b = oracle.cat_all_pairs(full, [3] * 5, v=5)
    assert np.array_equal(a, b)
    with pytest.raises(ValueError):
        oracle.cat_all_pairs(full, [2] * 8)          # code 2 with 2 levels
    with pytest.raises(ValueError):
        oracle.cat_all_pairs(full, [3] * 7)          # one count per variable
    with pytest.raises(ValueError):
        oracle.cat_all_pairs(full, [3] * 7 + [0])    # a level count below 1


# --------------------------------------------- the indicator-Gram derivation --

def _indicators(X, levels):
    """Indicator columns of codes 1 .. L_j - 1 for each variable, and offsets."""
    cols, off = [], [0]
    for j, L in enumerate(levels):
        for x in range(1, L):
            cols.append((X[:, j] == x).astype(np.int64))
        off.append(off[-1] + L - 1)
    Y = np.stack(cols, axis=1) if cols else np.zeros((X.shape[0], 0), np.int64)
    return Y, off


def _derived_mi(X, levels, cell_fn=None, log=math.log2, zero_row=True, swap=False, n00_sign=1, scale_m=True,
                gram_fn=None):
    m = X.shape[0]
    Y, off = _indicators(X, levels)
    G = Y.T @ Y if gram_fn is None else gram_fn(Y)
    c = Y.sum(axis=0)
    v = len(levels)
    mi = np.zeros((v, v))
    for a in range(v):
        for b in range(a, v):  # a <= b, mirrored below
            La, Lb = levels[a], levels[b]
            blk = G[off[a]:off[a + 1], off[b]:off[b + 1]]
            r = [0] + [int(t) for t in c[off[a]:off[a + 1]]]
            s = [0] + [int(t) for t in c[off[b]:off[b + 1]]]
            r[0] = m - sum(r[1:])
            s[0] = m - sum(s[1:])
            if swap:
                r, s = s[:La] + [0] * max(0, La - len(s)), r[:Lb] + [0] * max(0, Lb - len(r))
            t = np.zeros((La, Lb), dtype=np.int64)
            t[1:, 1:] = blk
            t[1:, 0] = [r[x] - int(blk[x - 1].sum()) for x in range(1, La)]
            t[0, 1:] = [s[y] - int(blk[:, y - 1].sum()) for y in range(1, Lb)]
            t[0, 0] = m - sum(r[1:]) - sum(s[1:]) + n00_sign * int(blk.sum())
            if not zero_row:
                t[0, :] = 0
            acc = 0.0
            for x in range(La):
                for y in range(Lb):
                    n = int(t[x, y])
                    if n > 0 and r[x] > 0 and s[y] > 0:
                        acc += n * log(n * m / (r[x] * s[y])) if cell_fn is None else cell_fn(n, r[x], s[y], m)
            mi[a, b] = mi[b, a] = acc / m if scale_m else acc
    return mi


def test_indicator_gram_derivation_passes_the_pins():
    # The Python form of the derivation the GPU path uses passes every pin, so
    # a mutant's failure below is due to its planted mistake alone.
    pins_cat.run_all(_derived_mi)


MUTANTS = {
    "drops_code0_row": lambda X, L: _derived_mi(X, L, zero_row=False),
    "swapped_marginals": lambda X, L: _derived_mi(X, L, swap=True),
    "natural_log": lambda X, L: _derived_mi(X, L, log=math.log),
    "n00_sign_slip": lambda X, L: _derived_mi(X, L, n00_sign=-1),
    "no_division_by_m": lambda X, L: _derived_mi(X, L, scale_m=False),
    "epsilon_in_log": lambda X, L: _derived_mi(X, L, cell_fn=lambda n, r, s, m: n * math.log2((n + 1e-3) * m / (r * s))),
    "or_gram": lambda X, L: _derived_mi(X, L, gram_fn=lambda Y: (Y[:, :, None] | Y[:, None, :]).sum(0)),
    "last_codes_merged": lambda X, L: _derived_mi(np.minimum(X, np.maximum(np.array(L) - 2, 0)).astype(np.uint8), L),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_categorical_pins_catch_planted_mistake(name):
    with pytest.raises(AssertionError):
        pins_cat.run_all(MUTANTS[name])
