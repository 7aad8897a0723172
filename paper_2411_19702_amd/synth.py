"""Seeded synthetic binary datasets shaped like the paper's workloads.

The paper benchmarks on its own synthetic binary matrices (Section 4.1-4.2:
rows 1k-100k, columns 100-10,000, 90% sparsity, and a 50%-99.5% sparsity
sweep) without publishing a generator, so the workloads here are stand-ins
with the same shapes and density ranges plus planted dependent columns.

This module is shared by the GPU path's tests/bench and by the oracle's tests.
It only draws random bits; it contains none of the mutual-information
arithmetic.

Bits come from a counter-based hash so that any column subset can be
regenerated on any device (CPU for the oracle, GPU for the kernels) with
identical results:

    u(seed, row, col) = lowbias32(lowbias32(seed_mix + row) ^ colmix(col))
    X[row, col]       = 1  iff  u < floor(p_col * 2^32)

lowbias32 is Chris Wellons' published 32-bit integer hash (xorshift-multiply,
constants 0x7feb352d and 0x846ca68b).  All arithmetic is done on int64 torch
tensors with the 32x32-bit products split into 16-bit halves, so nothing
overflows and CPU and GPU agree bit for bit.

Per-column parameters (densities, planted pairs, derived columns) are drawn
with numpy's PCG64 from the dataset seed.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

_M32 = 0xFFFFFFFF


def _mul32(x: torch.Tensor, c: int) -> torch.Tensor:
    """(x * c) mod 2^32 for int64 tensors holding values in [0, 2^32)."""
    lo = x & 0xFFFF
    hi = x >> 16
    return (lo * c + (((hi * c) & 0xFFFF) << 16)) & _M32


def _lowbias32(x: torch.Tensor) -> torch.Tensor:
    x = x ^ (x >> 16)
    x = _mul32(x, 0x7FEB352D)
    x = x ^ (x >> 15)
    x = _mul32(x, 0x846CA68B)
    x = x ^ (x >> 16)
    return x


def _row_keys(seed: int, stream: int, rows: torch.Tensor) -> torch.Tensor:
    base = (seed * 0x9E3779B9 + stream * 0x632BE5AB) & _M32
    return _lowbias32((rows + base) & _M32)


def _col_keys(seed: int, stream: int, cols: torch.Tensor) -> torch.Tensor:
    base = (seed * 0x85EBCA77 + stream * 0x27D4EB2F + 0x165667B1) & _M32
    return _lowbias32((_mul32(cols, 0xC2B2AE3D) + base) & _M32)


def uniform_u32(seed: int, stream: int, rows: torch.Tensor, cols: torch.Tensor) -> torch.Tensor:
    """Hash values in [0, 2^32) for the outer product rows x cols (int64)."""
    rk = _row_keys(seed, stream, rows)
    ck = _col_keys(seed, stream, cols)
    return _lowbias32(rk[:, None] ^ ck[None, :])


@dataclasses.dataclass
class DatasetSpec:
    """Everything needed to regenerate one m x n binary matrix."""

    m: int
    n: int
    seed: int
    p: np.ndarray                                  # float64[n], P(X_j = 1) of base columns
    planted: List[Tuple[int, int, float]] = dataclasses.field(default_factory=list)
    # (dst, src, q): column dst := column src XOR Bernoulli(q)
    derived: List[Tuple[int, int, int, str]] = dataclasses.field(default_factory=list)
    # (dst, a, b, op): column dst := a AND b  (op "and") or a XOR b (op "xor")
    ldx: Optional[int] = None                      # row pitch in bytes (>= n); None means n
    name: str = ""

    @property
    def pitch(self) -> int:
        return self.n if self.ldx is None else self.ldx

    def thresholds(self) -> np.ndarray:
        return np.floor(np.clip(self.p, 0.0, 1.0) * 4294967296.0).astype(np.int64)


# Hash streams: 0 = base bits, 1 = flip bits of planted pairs.
_BASE, _FLIP = 0, 1


def _base_columns(spec: DatasetSpec, rows: torch.Tensor, cols: Sequence[int], device) -> torch.Tensor:
    cols_t = torch.as_tensor(list(cols), dtype=torch.int64, device=device)
    thr = torch.as_tensor(spec.thresholds()[list(cols)], dtype=torch.int64, device=device)
    u = uniform_u32(spec.seed, _BASE, rows, cols_t)
    return (u < thr[None, :]).to(torch.uint8)


def _closure(spec: DatasetSpec, cols: Sequence[int]) -> List[int]:
    """Columns whose base bits are needed to build `cols` (derivations may chain)."""
    parents = {}
    for dst, src, _q in spec.planted:
        parents[dst] = [src]
    for dst, a, b, _op in spec.derived:
        parents[dst] = [a, b]
    need, stack = set(), list(cols)
    while stack:
        c = stack.pop()
        if c in need:
            continue
        need.add(c)
        stack.extend(parents.get(c, []))
    return sorted(need)


def _apply_structure(spec: DatasetSpec, block: torch.Tensor, index: dict, rows: torch.Tensor, device) -> None:
    """Overwrite planted and derived columns in `block` (rows x len(index))."""
    for dst, src, q in spec.planted:
        if dst not in index:
            continue
        thr = int(math.floor(q * 4294967296.0))
        u = uniform_u32(spec.seed, _FLIP, rows, torch.tensor([dst], dtype=torch.int64, device=device))[:, 0]
        flip = (u < thr).to(torch.uint8)
        block[:, index[dst]] = block[:, index[src]] ^ flip
    for dst, a, b, op in spec.derived:
        if dst not in index:
            continue
        if op == "and":
            block[:, index[dst]] = block[:, index[a]] & block[:, index[b]]
        elif op == "xor":
            block[:, index[dst]] = block[:, index[a]] ^ block[:, index[b]]
        else:
            raise ValueError(op)


def columns(spec: DatasetSpec, cols: Sequence[int], device="cpu", row_chunk: int = 1 << 18) -> torch.Tensor:
    """Regenerate only the listed columns: returns uint8 (m, len(cols)), C-contiguous."""
    cols = list(cols)
    need = _closure(spec, cols)
    index = {c: k for k, c in enumerate(need)}
    out = torch.empty((spec.m, len(cols)), dtype=torch.uint8, device=device)
    sel = torch.as_tensor([index[c] for c in cols], dtype=torch.int64, device=device)
    for r0 in range(0, spec.m, row_chunk):
        r1 = min(spec.m, r0 + row_chunk)
        rows = torch.arange(r0, r1, dtype=torch.int64, device=device)
        block = _base_columns(spec, rows, need, device)
        _apply_structure(spec, block, index, rows, device)
        out[r0:r1] = block.index_select(1, sel)
    return out


def generate(spec: DatasetSpec, device="cpu", row_chunk: Optional[int] = None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Materialise the whole matrix as uint8 (m, pitch); bytes in columns >= n are zero."""
    m, n, ld = spec.m, spec.n, spec.pitch
    if out is None:
        out = torch.zeros((m, ld), dtype=torch.uint8, device=device)
    else:
        assert out.shape == (m, ld) and out.dtype == torch.uint8
        if ld > n:
            out[:, n:].zero_()
    if row_chunk is None:
        row_chunk = max(1, (1 << 26) // max(1, n))
    all_cols = list(range(n))
    index = {c: c for c in all_cols}
    for r0 in range(0, m, row_chunk):
        r1 = min(m, r0 + row_chunk)
        rows = torch.arange(r0, r1, dtype=torch.int64, device=out.device)
        block = _base_columns(spec, rows, all_cols, out.device)
        _apply_structure(spec, block, index, rows, out.device)
        out[r0:r1, :n] = block
    return out


# ---------------------------------------------------------------------------
# Workload recipes.  Each returns a DatasetSpec (or a list of them); the recipe
# of every workload is written out in the design notes.
# ---------------------------------------------------------------------------

SEED0 = 241119702


def _pick_planted(rng: np.random.Generator, n: int, count: int, qmax: float, taken: set) -> List[Tuple[int, int, float]]:
    """`count` (dst, src, q) pairs with distinct destinations that are not sources."""
    planted = []
    free = [c for c in range(n) if c not in taken]
    rng.shuffle(free)
    count = min(count, len(free) // 2)
    for k in range(count):
        dst, src = int(free[2 * k]), int(free[2 * k + 1])
        planted.append((dst, src, float(rng.uniform(0.0, qmax))))
        taken.add(dst)
        taken.add(src)
    return planted


def spec_small(seed: int = SEED0 + 0, m: int = 1000, n: int = 200) -> DatasetSpec:
    """1,000 x 200; p_j ~ U[0.05, 0.5]; 20 planted copy-with-flip pairs, q ~ U[0, 0.3]."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.05, 0.5, size=n)
    planted = _pick_planted(rng, n, 20, 0.3, set())
    return DatasetSpec(m=m, n=n, seed=seed, p=p, planted=planted, name=f"small_{m}x{n}")


def spec_mid(seed: int = SEED0 + 1, m: int = 100_000, n: int = 1024) -> DatasetSpec:
    """100,000 x 1,024; p_j ~ Beta(0.5, 2) clipped to [0.005, 0.95]; 64 planted pairs
    (q ~ U[0, 0.4]); 32 derived columns (16 AND + 16 XOR of two base columns)."""
    rng = np.random.default_rng(seed)
    p = np.clip(rng.beta(0.5, 2.0, size=n), 0.005, 0.95)
    taken: set = set()
    planted = _pick_planted(rng, n, 64, 0.4, taken)
    derived = []
    free = [c for c in range(n) if c not in taken]
    rng.shuffle(free)
    nder = min(32, len(free) // 3)
    for k in range(nder):
        dst, a, b = (int(v) for v in free[3 * k: 3 * k + 3])
        derived.append((dst, a, b, "and" if k < nder // 2 else "xor"))
    return DatasetSpec(m=m, n=n, seed=seed, p=p, planted=planted, derived=derived, name=f"mid_{m}x{n}")


def spec_large(seed: int = SEED0 + 2, m: int = 1_000_000, n: int = 4096) -> DatasetSpec:
    """1,000,000 x 4,096 fingerprint-like; p_j log-uniform in [0.001, 0.2]; no planted pairs."""
    rng = np.random.default_rng(seed)
    p = np.exp(rng.uniform(math.log(0.001), math.log(0.2), size=n))
    return DatasetSpec(m=m, n=n, seed=seed, p=p, name=f"large_{m}x{n}")


def spec_outbound(seed: int = SEED0 + 5, m: int = 2000, n: int = 8192) -> DatasetSpec:
    """2,000 x 8,192 (few rows, many columns: the n x n FP32 output, 268 MB,
    outweighs the 16 MB input); p_j ~ U[0.01, 0.5]; floor(1% n) planted pairs."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.01, 0.5, size=n)
    planted = _pick_planted(rng, n, n // 100, 0.3, set())
    return DatasetSpec(m=m, n=n, seed=seed, p=p, planted=planted, name=f"outbound_{m}x{n}")


def spec_wide(seed: int = SEED0 + 6, m: int = 20_000, n: int = 32_768) -> DatasetSpec:
    """20,000 x 32,768 (many variables: the dense FP32 output would be 4.3 GB,
    the use case of the sparse threshold output); p_j log-uniform in
    [0.01, 0.3]; floor(0.5% n) planted pairs, q ~ U[0, 0.3]."""
    rng = np.random.default_rng(seed)
    p = np.exp(rng.uniform(math.log(0.01), math.log(0.3), size=n))
    planted = _pick_planted(rng, n, n // 200, 0.3, set())
    return DatasetSpec(m=m, n=n, seed=seed, p=p, planted=planted, name=f"wide_{m}x{n}")


def _log_uniform_int(rng: np.random.Generator, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def specs_batched(seed: int = SEED0 + 3, count: int = 256, m_range=(500, 50_000), n_range=(64, 2048)) -> List[DatasetSpec]:
    """`count` datasets: m log-uniform, n uniform, p_j ~ U[0.01, 0.5], floor(5% n) planted pairs (q ~ U[0, 0.3])."""
    rng = np.random.default_rng(seed)
    specs = []
    for d in range(count):
        m = _log_uniform_int(rng, *m_range)
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        p = rng.uniform(0.01, 0.5, size=n)
        planted = _pick_planted(rng, n, int(math.floor(0.05 * n)), 0.3, set())
        specs.append(DatasetSpec(m=m, n=n, seed=seed * 1000 + d, p=p, planted=planted, name=f"batch{d}_{m}x{n}"))
    return specs


@dataclasses.dataclass
class Request:
    arrival_s: float
    spec: DatasetSpec


def request_trace(seed: int = SEED0 + 4, count: int = 64, qps: float = 100.0,
                  m_range=(1000, 200_000), n_range=(128, 8192)) -> List[Request]:
    """Poisson arrivals at `qps`; m and n log-uniform; p_j ~ U[0.005, 0.5]."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for r in range(count):
        t += float(rng.exponential(1.0 / qps))
        m = _log_uniform_int(rng, *m_range)
        n = _log_uniform_int(rng, *n_range)
        p = rng.uniform(0.005, 0.5, size=n)
        reqs.append(Request(arrival_s=t, spec=DatasetSpec(m=m, n=n, seed=seed * 100000 + r, p=p, name=f"req{r}_{m}x{n}")))
    return reqs


def spec_random(seed: int, m: int, n: int, p_lo: float = 0.0, p_hi: float = 1.0, ldx: Optional[int] = None,
                planted: int = 0) -> DatasetSpec:
    """Generic seeded dataset for tests (edge shapes, ragged tails, padded pitch)."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(p_lo, p_hi, size=n)
    pl = _pick_planted(rng, n, planted, 0.3, set()) if planted else []
    return DatasetSpec(m=m, n=n, seed=seed, p=p, planted=pl, ldx=ldx, name=f"rand_{m}x{n}")


# ---------------------------------------------------------------------------
# Categorical datasets (codes 0 .. L-1 per column).  Codes come from the same
# counter-based hash: code = number of cumulative thresholds of the column
# that u(seed, row, col) reaches, so P(code <= k) = cum[col, k].
# ---------------------------------------------------------------------------

_CODE, _CFLIP = 2, 3


@dataclasses.dataclass
class CatSpec:
    """Everything needed to regenerate one m x v categorical matrix."""

    m: int
    v: int
    seed: int
    levels: np.ndarray                             # int32[v], codes per column (1 .. 256)
    cum: np.ndarray                                # float64[v, Lmax - 1], P(code <= k); 1.0 past L - 2
    planted: List[Tuple[int, int, float]] = dataclasses.field(default_factory=list)
    # (dst, src, q): column dst := (code of src) mod L_dst, except where a Bernoulli(q) draw keeps its own code
    ldx: Optional[int] = None
    name: str = ""

    @property
    def pitch(self) -> int:
        return self.v if self.ldx is None else self.ldx

    def thresholds(self) -> np.ndarray:
        return np.floor(np.clip(self.cum, 0.0, 1.0) * 4294967296.0).astype(np.int64)


def _cat_base(spec: CatSpec, rows: torch.Tensor, cols: Sequence[int], device) -> torch.Tensor:
    cols = list(cols)
    cols_t = torch.as_tensor(cols, dtype=torch.int64, device=device)
    thr = torch.as_tensor(spec.thresholds()[cols], dtype=torch.int64, device=device)   # (k, Lmax - 1)
    u = uniform_u32(spec.seed, _CODE, rows, cols_t)
    code = torch.zeros(u.shape, dtype=torch.int64, device=device)
    for k in range(thr.shape[1]):
        code += (u >= thr[None, :, k]).to(torch.int64)
    return code.to(torch.uint8)


def _cat_block(spec: CatSpec, rows: torch.Tensor, cols: Sequence[int], device) -> torch.Tensor:
    cols = list(cols)
    need = sorted(set(cols) | {src for dst, src, _q in spec.planted if dst in set(cols)})
    index = {c: k for k, c in enumerate(need)}
    block = _cat_base(spec, rows, need, device)
    for dst, src, q in spec.planted:
        if dst not in index:
            continue
        thr = int(math.floor(q * 4294967296.0))
        u = uniform_u32(spec.seed, _CFLIP, rows, torch.tensor([dst], dtype=torch.int64, device=device))[:, 0]
        keep = u < thr
        copied = (block[:, index[src]].to(torch.int64) % int(spec.levels[dst])).to(torch.uint8)
        block[:, index[dst]] = torch.where(keep, block[:, index[dst]], copied)
    sel = torch.as_tensor([index[c] for c in cols], dtype=torch.int64, device=device)
    return block.index_select(1, sel)


def cat_columns(spec: CatSpec, cols: Sequence[int], device="cpu", row_chunk: int = 1 << 18) -> torch.Tensor:
    """Regenerate only the listed columns: uint8 (m, len(cols)), C-contiguous."""
    cols = list(cols)
    out = torch.empty((spec.m, len(cols)), dtype=torch.uint8, device=device)
    for r0 in range(0, spec.m, row_chunk):
        r1 = min(spec.m, r0 + row_chunk)
        rows = torch.arange(r0, r1, dtype=torch.int64, device=device)
        out[r0:r1] = _cat_block(spec, rows, cols, device)
    return out


def cat_generate(spec: CatSpec, device="cpu", row_chunk: Optional[int] = None) -> torch.Tensor:
    """The whole matrix as uint8 (m, pitch); bytes in columns >= v are zero."""
    m, v, ld = spec.m, spec.v, spec.pitch
    out = torch.zeros((m, ld), dtype=torch.uint8, device=device)
    if v == 0:
        return out
    if row_chunk is None:
        row_chunk = max(1, (1 << 25) // max(1, v * max(1, spec.cum.shape[1])))
    for r0 in range(0, m, row_chunk):
        r1 = min(m, r0 + row_chunk)
        rows = torch.arange(r0, r1, dtype=torch.int64, device=out.device)
        out[r0:r1, :v] = _cat_block(spec, rows, range(v), out.device)
    return out


def _cat_spec(seed: int, m: int, probs: List[np.ndarray], planted, ldx, name) -> CatSpec:
    v = len(probs)
    levels = np.array([len(p) for p in probs], dtype=np.int32)
    width = max(1, int(levels.max(initial=1)) - 1)
    cum = np.ones((v, width), dtype=np.float64)
    for j, p in enumerate(probs):
        c = np.cumsum(p)[:-1]
        cum[j, :len(c)] = c
    return CatSpec(m=m, v=v, seed=seed, levels=levels, cum=cum, planted=planted, ldx=ldx, name=name)


def spec_genotypes(seed: int = SEED0 + 7, m: int = 1_000_000, v: int = 2048, ldx: Optional[int] = None) -> CatSpec:
    """Genotype-like data: 3 codes per column with Hardy-Weinberg frequencies
    (1-f)^2, 2f(1-f), f^2 for a minor-allele frequency f ~ U[0.05, 0.5], and
    v // 100 planted pairs copying a column with probability 1 - q, q ~ U[0, 0.3]."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.05, 0.5, size=v)
    probs = [np.array([(1 - a) ** 2, 2 * a * (1 - a), a * a]) for a in f]
    planted = _pick_planted(rng, v, v // 100, 0.3, set())
    return _cat_spec(seed, m, probs, planted, ldx, f"genotypes_{m}x{v}")


def spec_categorical(seed: int, m: int, v: int, lmin: int = 2, lmax: int = 16, ldx: Optional[int] = None,
                     planted: int = 0, alpha: float = 0.7, levels: Optional[Sequence[int]] = None) -> CatSpec:
    """Generic categorical data for tests: level counts uniform in [lmin, lmax]
    (or given), code probabilities Dirichlet(alpha), optional planted pairs."""
    rng = np.random.default_rng(seed)
    lv = rng.integers(lmin, lmax + 1, size=v) if levels is None else np.asarray(levels)
    probs = [rng.dirichlet(np.full(int(L), alpha)) if L > 1 else np.array([1.0]) for L in lv]
    pl = _pick_planted(rng, v, planted, 0.3, set()) if planted else []
    return _cat_spec(seed, m, probs, pl, ldx, f"cat_{m}x{v}")
