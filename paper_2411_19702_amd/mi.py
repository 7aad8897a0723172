"""Python binding of libmi.so (include/mi.h), with the same entry-point names.

Argument marshalling only: tensors are passed by device pointer and the
current torch stream by handle; every step of the computation runs in the HIP
library.  There is no fallback -- if the library is not built, or a tensor is
not on the GPU, the call raises.

X is a 2-D uint8 (or int8/bool) tensor on the GPU of shape (m, n) whose rows
may be padded: X.stride(1) must be 1 and X.stride(0) is the row pitch ldx.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional, Sequence, Tuple

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmi.so")

MI_OK = 0
STATUS_NAMES = {
    0: "MI_OK", 1: "MI_ERR_INVALID_ARG", 2: "MI_ERR_NOT_BINARY", 3: "MI_ERR_OUT_OF_MEMORY", 4: "MI_ERR_BUDGET",
    5: "MI_ERR_QUEUE_FULL", 6: "MI_ERR_NOT_READY", 7: "MI_ERR_DEVICE", 8: "MI_ERR_TIMEOUT", 9: "MI_ERR_UNKNOWN_TICKET",
    10: "MI_ERR_BAD_CODE",
}
MI_EPI_FP32, MI_EPI_FP32_FP64_FALLBACK, MI_EPI_FP64 = 0, 1, 2
MI_ALGO_DENSE, MI_ALGO_SPARSE, MI_ALGO_AUTO = 0, 1, 2
MI_TILE_AUTO, MI_TILE_128, MI_TILE_256 = 0, 1, 2
MI_BATCH_PERSISTENT, MI_BATCH_GRAPH, MI_BATCH_SEQUENTIAL = 0, 1, 2
MI_INPUT_BYTES, MI_INPUT_BITS, MI_INPUT_FP4 = 0, 1, 2
MI_GRAM_AUTO, MI_GRAM_INT8, MI_GRAM_FP4 = 0, 1, 2


class MIError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class mi_problem(ctypes.Structure):
    _fields_ = [
        ("X", ctypes.c_void_p),
        ("m", ctypes.c_int64),
        ("n", ctypes.c_int64),
        ("ldx", ctypes.c_int64),
        ("out", ctypes.c_void_p),
        ("n11_out", ctypes.c_void_p),
        ("colsum_out", ctypes.c_void_p),
        ("epilogue", ctypes.c_int32),
        ("fallback_tau", ctypes.c_float),
        ("validate", ctypes.c_int32),
        ("tile", ctypes.c_int32),
        ("splits", ctypes.c_int32),
        ("pairs", ctypes.c_void_p),
        ("pairs_capacity", ctypes.c_int64),
        ("pairs_count", ctypes.c_void_p),
        ("pairs_threshold", ctypes.c_float),
        ("algo", ctypes.c_int32),
        ("packed", ctypes.c_int32),
        ("gram", ctypes.c_int32),
    ]


class mi_cat_problem(ctypes.Structure):
    _fields_ = [
        ("X", ctypes.c_void_p),
        ("m", ctypes.c_int64),
        ("v", ctypes.c_int64),
        ("ldx", ctypes.c_int64),
        ("levels", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("epilogue", ctypes.c_int32),
        ("fallback_tau", ctypes.c_float),
        ("validate", ctypes.c_int32),
        ("tile", ctypes.c_int32),
        ("splits", ctypes.c_int32),
        ("counts_out", ctypes.c_void_p),
        ("sums_out", ctypes.c_void_p),
        ("pairs", ctypes.c_void_p),
        ("pairs_capacity", ctypes.c_int64),
        ("pairs_count", ctypes.c_void_p),
        ("pairs_threshold", ctypes.c_float),
        ("gram", ctypes.c_int32),
    ]


class mi_server_stats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
        ("batches", ctypes.c_uint64), ("max_in_flight", ctypes.c_uint64),
        ("max_bytes_in_flight", ctypes.c_size_t), ("bytes_in_flight", ctypes.c_size_t),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libmi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, vp, f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_float
    P = ctypes.POINTER
    sig = {
        "mi_problem_init": (None, [P(mi_problem), vp, i64, i64, vp]),
        "mi_all_pairs": (i32, [vp, i64, i64, vp]),
        "mi_all_pairs_async": (i32, [vp, i64, i64, vp, vp]),
        "mi_all_pairs_ex": (i32, [P(mi_problem), vp]),
        "mi_all_pairs_batched": (i32, [P(mi_problem), i64, vp, i32]),
        "mi_all_pairs_noalloc": (i32, [P(mi_problem), vp]),
        "mi_plan": (i32, [i64, i64, i64, P(i32), P(i32)]),
        "mi_tune": (i32, [i64, i64, i64, P(i32), P(i32), P(ctypes.c_double)]),
        "mi_tune_batched": (i32, [P(mi_problem), i64, vp, P(ctypes.c_double), P(ctypes.c_double)]),
        "mi_plan_batched": (i32, [P(mi_problem), i64, vp, vp]),
        "mi_tuner_save": (i32, [ctypes.c_char_p]),
        "mi_tuner_load": (i32, [ctypes.c_char_p]),
        "mi_tuner_clear": (None, []),
        "mi_last_error": (ctypes.c_char_p, []),
        "mi_server_create": (i32, [P(vp), ctypes.c_size_t, i32, i32]),
        "mi_server_submit": (i32, [vp, P(mi_problem), P(ctypes.c_uint64)]),
        "mi_server_poll": (i32, [vp, ctypes.c_uint64]),
        "mi_server_wait": (i32, [vp, ctypes.c_uint64, ctypes.c_double, P(ctypes.c_double)]),
        "mi_server_get_stats": (i32, [vp, P(mi_server_stats)]),
        "mi_server_destroy": (i32, [vp]),
        "mi_version": (ctypes.c_char_p, []),
        "mi_cat_problem_init": (None, [P(mi_cat_problem), vp, i64, i64, vp, vp]),
        "mi_pack_bits": (i32, [vp, i64, i64, i64, vp, i64, vp]),
        "mi_pack_fp4": (i32, [vp, i64, i64, i64, vp, i64, vp]),
        "mi_plan_ex": (i32, [vp, vp, vp, vp]),
        "mi_cat_indicators": (i32, [vp, i64, P(i64)]),
        "mi_all_pairs_categorical": (i32, [P(mi_cat_problem), vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status: int) -> None:
    if status != MI_OK:
        msg = lib().mi_last_error()
        raise MIError(status, msg.decode() if msg else "")


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _layout_code(packed) -> int:
    """packed: False / MI_INPUT_BYTES, True / MI_INPUT_BITS, or MI_INPUT_FP4."""
    code = int(packed)
    if code not in (MI_INPUT_BYTES, MI_INPUT_BITS, MI_INPUT_FP4):
        raise ValueError(f"bad input layout {packed!r}")
    return code


def _x_layout(X: torch.Tensor, n: Optional[int], packed=False) -> Tuple[int, int, int]:
    if not isinstance(X, torch.Tensor) or X.dim() != 2:
        raise ValueError("X must be a 2-D tensor (rows x columns)")
    if not X.is_cuda:
        raise ValueError("X must be on the GPU (the library has no CPU path)")
    if X.dtype not in (torch.uint8, torch.int8, torch.bool):
        raise ValueError("X must hold bytes (uint8/int8/bool) with values 0/1")
    m, cols = X.shape
    if m > 1 and X.stride(1) != 1:
        raise ValueError("X rows must be contiguous (stride(1) == 1)")
    ldx = X.stride(0) if m > 1 else max(cols, 1)
    code = _layout_code(packed)
    if code != MI_INPUT_BYTES:
        per = 8 if code == MI_INPUT_BITS else 2
        if n is None:
            raise ValueError(f"a packed X needs n (its bytes hold {per} columns each)")
        if (n + per - 1) // per > cols:
            raise ValueError(f"n exceeds {per} * X.shape[1]")
        return m, n, ldx
    n = cols if n is None else n
    if n > cols:
        raise ValueError("n exceeds X.shape[1]")
    return m, n, ldx


def make_problem(X: torch.Tensor, out: Optional[torch.Tensor], n: Optional[int] = None,
                 n11_out: Optional[torch.Tensor] = None, colsum_out: Optional[torch.Tensor] = None,
                 epilogue: int = MI_EPI_FP32, fallback_tau: float = 1e-3, validate: bool = False, tile: int = 0,
                 splits: int = 0, pairs: Optional[torch.Tensor] = None, pairs_count: Optional[torch.Tensor] = None,
                 pairs_threshold: float = 0.0, algo: int = 0, packed=False, gram: int = MI_GRAM_AUTO) -> mi_problem:
    """pairs: int32 GPU tensor of shape (capacity, 3) receiving (i, j, MI bits as FP32) rows;
    pairs_count: int64 GPU tensor with one element (the number of qualifying pairs).
    packed: False (bytes), True / MI_INPUT_BITS (mi_pack_bits) or MI_INPUT_FP4 (mi_pack_fp4).
    gram: MI_GRAM_AUTO, MI_GRAM_INT8 or MI_GRAM_FP4 (the Gram's matrix instructions).
    The returned problem keeps references to the tensors it points to."""
    m, n, ldx = _x_layout(X, n, packed)
    for name, t, dt in (("out", out, torch.float32), ("n11_out", n11_out, torch.int32),
                        ("colsum_out", colsum_out, torch.int32), ("pairs", pairs, torch.int32),
                        ("pairs_count", pairs_count, torch.int64)):
        if t is None:
            continue
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dt} GPU tensor")
    if (out is not None and out.numel() < n * n) or (n11_out is not None and n11_out.numel() < n * n) or \
            (colsum_out is not None and colsum_out.numel() < n):
        raise ValueError("output tensor too small")
    if pairs is not None and (pairs.dim() != 2 or pairs.shape[1] != 3 or pairs_count is None or pairs_count.numel() < 1):
        raise ValueError("pairs must be (capacity, 3) int32 with a one-element int64 pairs_count")
    p = mi_problem()
    p.X, p.m, p.n, p.ldx = X.data_ptr(), m, n, ldx
    p.out, p.n11_out, p.colsum_out = _ptr(out), _ptr(n11_out), _ptr(colsum_out)
    p.epilogue, p.fallback_tau, p.validate = int(epilogue), float(fallback_tau), 1 if validate else 0
    p.tile, p.splits = int(tile), int(splits)
    p.pairs, p.pairs_capacity = _ptr(pairs), (pairs.shape[0] if pairs is not None else 0)
    p.pairs_count, p.pairs_threshold = _ptr(pairs_count), float(pairs_threshold)
    p.algo = int(algo)
    p.packed = _layout_code(packed)
    p.gram = int(gram)
    # The struct holds raw pointers: keep the tensors alive as long as the problem.
    p._keep = (X, out, n11_out, colsum_out, pairs, pairs_count)
    return p


def mi_all_pairs_threshold(X: torch.Tensor, threshold: float, capacity: int, dense_out: Optional[torch.Tensor] = None,
                           stream=None, **kw):
    """Sparse output: (pairs, count) where pairs[:min(count, capacity)] holds the (i, j, MI) rows
    with i < j and MI >= threshold (order unspecified); count (GPU int64 tensor) is the total."""
    pairs = torch.empty((max(int(capacity), 0), 3), dtype=torch.int32, device=X.device)
    count = torch.empty((1,), dtype=torch.int64, device=X.device)
    p = make_problem(X, dense_out, pairs=pairs, pairs_count=count, pairs_threshold=threshold, **kw)
    _check(lib().mi_all_pairs_ex(ctypes.byref(p), _stream_handle(stream)))
    return pairs, count


def _new_out(X: torch.Tensor, n: Optional[int]) -> torch.Tensor:
    n = X.shape[1] if n is None else n
    return torch.empty((n, n), dtype=torch.float32, device=X.device)


def mi_all_pairs(X: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Blocking MI matrix of X (contiguous m x n) on the default stream."""
    m, n, ldx = _x_layout(X, None)
    if ldx != n:
        raise ValueError("mi_all_pairs needs a dense X; use mi_all_pairs_ex for a pitched X")
    out = _new_out(X, n) if out is None else out
    _check(lib().mi_all_pairs(X.data_ptr(), m, n, out.data_ptr()))
    return out


def mi_all_pairs_async(X: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    m, n, ldx = _x_layout(X, None)
    if ldx != n:
        raise ValueError("mi_all_pairs_async needs a dense X; use mi_all_pairs_ex for a pitched X")
    out = _new_out(X, n) if out is None else out
    _check(lib().mi_all_pairs_async(X.data_ptr(), m, n, out.data_ptr(), _stream_handle(stream)))
    return out


def mi_all_pairs_ex(X: torch.Tensor, out: Optional[torch.Tensor] = None, n: Optional[int] = None, stream=None,
                    dense: bool = True, **kw) -> Optional[torch.Tensor]:
    """The extended call (make_problem's keywords).  out=None allocates the n x n
    matrix unless dense=False: then no MI matrix is written (counts only with
    n11_out / colsum_out, or the sparse pairs output), and None is returned."""
    if out is None and dense:
        out = _new_out(X, n)
    p = make_problem(X, out, n=n, **kw)
    _check(lib().mi_all_pairs_ex(ctypes.byref(p), _stream_handle(stream)))
    return out


def mi_all_pairs_noalloc(X: torch.Tensor, out: Optional[torch.Tensor] = None, n: Optional[int] = None, stream=None,
                         dense: bool = True, **kw) -> Optional[torch.Tensor]:
    """mi_all_pairs_ex through the entry point that allocates no device memory
    (the library's fixed scratch array; byte input on the int8 Gram).  out=None
    allocates the n x n matrix here, in torch, unless dense=False."""
    if out is None and dense:
        out = _new_out(X, n)
    p = make_problem(X, out, n=n, **kw)
    _check(lib().mi_all_pairs_noalloc(ctypes.byref(p), _stream_handle(stream)))
    return out


def problem_array(problems: Sequence[mi_problem]) -> ctypes.Array:
    """The problems as one C array (what the batched calls take), built once
    for a batch that is run repeatedly; it keeps the problems' tensors alive."""
    arr = (mi_problem * len(problems))(*problems)
    arr._keep = [getattr(p, "_keep", None) for p in problems]
    return arr


def _as_array(problems) -> ctypes.Array:
    return problems if isinstance(problems, ctypes.Array) else problem_array(problems)


def mi_all_pairs_batched(problems, mode: int = MI_BATCH_PERSISTENT, stream=None) -> None:
    """problems: a sequence of make_problem results, or problem_array() of one."""
    arr = _as_array(problems)
    _check(lib().mi_all_pairs_batched(arr, len(arr), _stream_handle(stream), int(mode)))


def mi_plan(m: int, n: int, ldx: int = 0) -> Tuple[int, int]:
    t, s = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().mi_plan(m, n, ldx, ctypes.byref(t), ctypes.byref(s)))
    return t.value, s.value


def mi_plan_ex(X: torch.Tensor, n: Optional[int] = None, **kw) -> Tuple[int, int, int]:
    """(tile, splits, gram) the library would use for this problem (make_problem's keywords;
    no output needed, nothing launched).  gram is MI_GRAM_INT8 or MI_GRAM_FP4."""
    p = make_problem(X, None, n=n, **kw)
    t, s, g = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().mi_plan_ex(ctypes.byref(p), ctypes.byref(t), ctypes.byref(s), ctypes.byref(g)))
    return t.value, s.value, g.value


def mi_tune(m: int, n: int, ldx: int = 0) -> Tuple[int, int, float]:
    t, s, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check(lib().mi_tune(m, n, ldx, ctypes.byref(t), ctypes.byref(s), ctypes.byref(ms)))
    return t.value, s.value, ms.value


def mi_tune_batched(problems, stream=None) -> Tuple[float, float]:
    """Tune the persistent plan of this batch on its own data; returns (chosen ms, heuristic ms)."""
    arr = _as_array(problems)
    best, heur = ctypes.c_double(), ctypes.c_double()
    _check(lib().mi_tune_batched(arr, len(arr), _stream_handle(stream), ctypes.byref(best), ctypes.byref(heur)))
    return best.value, heur.value


def mi_plan_batched(problems) -> Tuple[List[int], List[int]]:
    """(tiles, splits) per dataset of the persistent mode's plan for this batch."""
    arr = _as_array(problems)
    k = len(arr)
    tiles, splits = (ctypes.c_int32 * max(k, 1))(), (ctypes.c_int32 * max(k, 1))()
    _check(lib().mi_plan_batched(arr, k, ctypes.cast(tiles, ctypes.c_void_p), ctypes.cast(splits, ctypes.c_void_p)))
    return list(tiles)[:k], list(splits)[:k]


def mi_tuner_save(path: str) -> None:
    _check(lib().mi_tuner_save(path.encode()))


def mi_tuner_load(path: str) -> None:
    _check(lib().mi_tuner_load(path.encode()))


def mi_tuner_clear() -> None:
    lib().mi_tuner_clear()


def mi_last_error() -> str:
    return (lib().mi_last_error() or b"").decode()


def mi_version() -> str:
    return lib().mi_version().decode()


class Server:
    """Continuous-batching request loop (include/mi_server.h)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 4, max_queue: int = 0):
        h = ctypes.c_void_p()
        _check(lib().mi_server_create(ctypes.byref(h), int(hbm_budget_bytes), int(max_slots), int(max_queue)))
        self._h = h
        self._keep = {}  # ticket -> tensors the request reads or writes (kept alive until collected)

    def submit(self, X: torch.Tensor, out: torch.Tensor, keep=(), **kw) -> int:
        p = make_problem(X, out, **kw)
        t = ctypes.c_uint64()
        _check(lib().mi_server_submit(self._h, ctypes.byref(p), ctypes.byref(t)))
        self._keep[t.value] = (p._keep, tuple(keep))  # every tensor the request reads or writes
        return t.value

    def poll(self, ticket: int) -> bool:
        st = lib().mi_server_poll(self._h, ticket)
        if st == 6:
            return False
        _check(st)
        return True

    def wait(self, ticket: int, timeout_s: float = 0.0) -> float:
        lat = ctypes.c_double()
        st = lib().mi_server_wait(self._h, ticket, float(timeout_s), ctypes.byref(lat))
        if st != 8:  # a timeout leaves the ticket pending
            self._keep.pop(ticket, None)
        _check(st)
        return lat.value

    def stats(self) -> dict:
        s = mi_server_stats()
        _check(lib().mi_server_get_stats(self._h, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in s._fields_}

    def close(self) -> None:
        if self._h:
            _check(lib().mi_server_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ------------------------------------------------------------- categorical --

def _levels_array(levels, v: int):
    lv = (ctypes.c_int32 * max(v, 1))()
    vals = [int(x) for x in levels]
    if len(vals) != v:
        raise ValueError("levels must hold one count per variable")
    for j, x in enumerate(vals):
        lv[j] = x
    return lv


def mi_cat_indicators(levels) -> int:
    """N = sum (levels[j] - 1): the side of the indicator count matrix."""
    v = len(levels)
    lv = _levels_array(levels, v)
    N = ctypes.c_int64()
    _check(lib().mi_cat_indicators(lv, v, ctypes.byref(N)))
    return int(N.value)


def mi_all_pairs_categorical(X: torch.Tensor, levels, out: Optional[torch.Tensor] = None, v: Optional[int] = None,
                             epilogue: int = MI_EPI_FP32, fallback_tau: float = 1e-3, validate: bool = False,
                             tile: int = 0, splits: int = 0, counts_out: Optional[torch.Tensor] = None,
                             sums_out: Optional[torch.Tensor] = None, stream=None,
                             pairs: Optional[torch.Tensor] = None, pairs_count: Optional[torch.Tensor] = None,
                             pairs_threshold: float = 0.0, dense: bool = True, gram: int = MI_GRAM_AUTO):
    """MI matrix (v x v FP32, bits) of categorical X: column j holds codes 0 .. levels[j]-1.
    X is a uint8 GPU tensor (m, cols) with contiguous rows; v defaults to cols.
    pairs / pairs_count / pairs_threshold: the sparse output as in make_problem;
    dense=False writes no matrix (returns None)."""
    if not isinstance(X, torch.Tensor) or X.dim() != 2 or not X.is_cuda or X.dtype not in (torch.uint8, torch.int8):
        raise ValueError("X must be a 2-D uint8 GPU tensor of codes")
    m, cols = X.shape
    if m > 1 and X.stride(1) != 1:
        raise ValueError("X rows must be contiguous (stride(1) == 1)")
    ldx = X.stride(0) if m > 1 else max(cols, 1)
    v = cols if v is None else int(v)
    if v > cols:
        raise ValueError("v exceeds X.shape[1]")
    lv = _levels_array(levels, v)
    if out is None and dense:
        out = torch.empty((v, v), dtype=torch.float32, device=X.device)
    if pairs is not None and (pairs.dim() != 2 or pairs.shape[1] != 3 or pairs_count is None or pairs_count.numel() < 1):
        raise ValueError("pairs must be (capacity, 3) int32 with a one-element int64 pairs_count")
    for name, t, dt in (("out", out, torch.float32), ("counts_out", counts_out, torch.int32),
                        ("sums_out", sums_out, torch.int32), ("pairs", pairs, torch.int32),
                        ("pairs_count", pairs_count, torch.int64)):
        if t is not None and (not t.is_cuda or t.dtype != dt or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {dt} GPU tensor")
    N = sum(int(x) - 1 for x in levels[:v]) if v else 0
    if (out is not None and out.numel() < v * v) or (counts_out is not None and counts_out.numel() < N * N) or \
            (sums_out is not None and sums_out.numel() < N):
        raise ValueError("output tensor too small")
    p = mi_cat_problem()
    lib().mi_cat_problem_init(ctypes.byref(p), X.data_ptr(), m, v, ctypes.cast(lv, ctypes.c_void_p), _ptr(out))
    p.ldx = ldx
    p.epilogue, p.fallback_tau, p.validate = int(epilogue), float(fallback_tau), 1 if validate else 0
    p.tile, p.splits = int(tile), int(splits)
    p.counts_out, p.sums_out = _ptr(counts_out), _ptr(sums_out)
    p.pairs, p.pairs_capacity = _ptr(pairs), (pairs.shape[0] if pairs is not None else 0)
    p.pairs_count, p.pairs_threshold = _ptr(pairs_count), float(pairs_threshold)
    p.gram = int(gram)
    _check(lib().mi_all_pairs_categorical(ctypes.byref(p), _stream_handle(stream)))
    return out


def mi_pack_fp4(X: torch.Tensor, n: Optional[int] = None, out: Optional[torch.Tensor] = None,
                stream=None) -> torch.Tensor:
    """Pack a 0/1 byte matrix (m x n) into (m, ceil(n/2)) bytes of FP4 (E2M1) codes: the low nibble of
    byte c is 0b0010 (1.0) if column 2c is nonzero, else 0; the high nibble likewise for column 2c + 1."""
    m, n, ldx = _x_layout(X, n)
    nb = (n + 1) // 2
    if out is None:
        out = torch.empty((m, max(nb, 1)), dtype=torch.uint8, device=X.device)
    if not out.is_cuda or out.dtype != torch.uint8 or out.dim() != 2 or out.shape[0] != m or out.shape[1] < nb \
            or (m > 1 and out.stride(1) != 1):
        raise ValueError("out must be a uint8 GPU tensor of shape (m, >= ceil(n/2)) with contiguous rows")
    ldq = out.stride(0) if m > 1 else max(out.shape[1], 1)
    _check(lib().mi_pack_fp4(X.data_ptr(), m, n, ldx, out.data_ptr(), ldq, _stream_handle(stream)))
    return out


def mi_pack_bits(X: torch.Tensor, n: Optional[int] = None, out: Optional[torch.Tensor] = None,
                 stream=None) -> torch.Tensor:
    """Bit-pack a 0/1 byte matrix (m x n) into (m, ceil(n/8)) bytes, bit k of byte b = column 8b + k."""
    m, n, ldx = _x_layout(X, n)
    nb = (n + 7) // 8
    if out is None:
        out = torch.empty((m, max(nb, 1)), dtype=torch.uint8, device=X.device)
    if not out.is_cuda or out.dtype != torch.uint8 or out.dim() != 2 or out.shape[0] != m or out.shape[1] < nb \
            or (m > 1 and out.stride(1) != 1):
        raise ValueError("out must be a uint8 GPU tensor of shape (m, >= ceil(n/8)) with contiguous rows")
    ldp = out.stride(0) if m > 1 else max(out.shape[1], 1)
    _check(lib().mi_pack_bits(X.data_ptr(), m, n, ldx, out.data_ptr(), ldp, _stream_handle(stream)))
    return out
