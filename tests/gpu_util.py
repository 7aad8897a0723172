"""Helpers for the GPU parity tests: run the library, compare with the oracle."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
from paper_2411_19702_amd import mi

MI_TOL = 1e-5  # bits, absolute, against the FP64 oracle


def say(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def run_gpu(X: torch.Tensor, n=None, **kw):
    """(out, n11, colsum) as numpy arrays from one mi_all_pairs_ex call."""
    m, cols = X.shape
    n = cols if n is None else n
    out = torch.full((n, n), float("nan"), dtype=torch.float32, device=X.device)
    n11 = torch.full((n, n), -1, dtype=torch.int32, device=X.device)
    cs = torch.full((max(n, 1),), -1, dtype=torch.int32, device=X.device)
    mi.mi_all_pairs_ex(X, out=out, n=n, n11_out=n11, colsum_out=cs, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy(), n11.cpu().numpy(), cs.cpu().numpy()[:n]


def compare_full(Xh: np.ndarray, n: int, out: np.ndarray, n11: np.ndarray, cs: np.ndarray, tol: float = MI_TOL) -> float:
    """Every element against the oracle; returns the max |dMI| in bits."""
    o_n11, o_mi = oracle.all_pairs(Xh, n=n)
    assert np.array_equal(n11.astype(np.int64), o_n11), "n11 differs from the oracle"
    assert np.array_equal(cs.astype(np.int64), np.diag(o_n11)), "column sums differ from the oracle"
    assert np.array_equal(out, out.T), "MI output is not bitwise symmetric"
    assert np.isfinite(out).all(), "non-finite MI"
    err = float(np.max(np.abs(out.astype(np.float64) - o_mi))) if n else 0.0
    assert err <= tol, f"max |dMI| = {err} > {tol}"
    return err


def compare_columns(Xs: np.ndarray, cols, out: np.ndarray, n11: np.ndarray, cs: np.ndarray, tol: float = MI_TOL) -> float:
    """Sampled check: Xs holds only the listed columns (all rows); compare every pair among them."""
    cols = np.asarray(cols)
    o_n11, o_mi = oracle.all_pairs(Xs)
    g_n11 = n11[np.ix_(cols, cols)].astype(np.int64)
    g_mi = out[np.ix_(cols, cols)].astype(np.float64)
    assert np.array_equal(g_n11, o_n11), "sampled n11 differs from the oracle"
    assert np.array_equal(cs[cols].astype(np.int64), np.diag(o_n11)), "sampled column sums differ"
    err = float(np.max(np.abs(g_mi - o_mi)))
    assert err <= tol, f"sampled max |dMI| = {err} > {tol}"
    return err
