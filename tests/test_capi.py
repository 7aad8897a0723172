"""The C-ABI library on the CPU (no GPU): it builds, loads, exports every
symbol the headers declare, and its host-side argument checks return the
documented status codes without touching a device."""
import ctypes
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2411_19702_amd import build, mi
    if build.is_stale():
        build.build_library()
    return mi.lib()


def declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(mi_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_headers_declare_the_boundary():
    names = declared_functions()
    for required in ("mi_all_pairs", "mi_all_pairs_async", "mi_all_pairs_ex", "mi_all_pairs_batched",
                     "mi_last_error", "mi_tune", "mi_server_create", "mi_server_submit", "mi_server_wait"):
        assert required in names, required


def test_library_exports_every_declared_symbol(L):
    from paper_2411_19702_amd import mi
    out = subprocess.run(["nm", "-D", "--defined-only", mi.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT\s+(\w+)$", out, flags=re.M))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


def test_library_has_gfx950_code_object():
    from paper_2411_19702_amd import mi
    data = open(mi.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def _problem(mi, **kw):
    p = mi.mi_problem()
    mi.lib().mi_problem_init(ctypes.byref(p), None, 10, 4, None)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("field,value", [("m", 0), ("m", -3), ("m", 2 ** 31), ("n", -1), ("ldx", 3), ("epilogue", 3),
                                         ("epilogue", -1), ("tile", 7), ("splits", -2)])
def test_invalid_arguments_rejected_on_host(L, field, value):
    from paper_2411_19702_amd import mi
    p = _problem(mi, X=16, out=16)
    setattr(p, field, value)
    st = L.mi_all_pairs_ex(ctypes.byref(p), None)
    assert st == 1, (field, value, st)
    assert L.mi_last_error()


def test_null_pointers_rejected_and_empty_is_noop(L):
    from paper_2411_19702_amd import mi
    p = _problem(mi)                      # X = out = NULL, n = 4
    assert L.mi_all_pairs_ex(ctypes.byref(p), None) == 1
    assert b"NULL" in L.mi_last_error()
    p.n = 0                               # n == 0 is a no-op even with NULL pointers
    assert L.mi_all_pairs_ex(ctypes.byref(p), None) == 0
    assert L.mi_all_pairs_ex(None, None) == 1
    assert L.mi_all_pairs(None, 0, 5, None) == 1


def test_batched_argument_checks(L):
    from paper_2411_19702_amd import mi
    assert L.mi_all_pairs_batched(None, 0, None, 0) == 0
    assert L.mi_all_pairs_batched(None, -1, None, 0) == 1
    assert L.mi_all_pairs_batched(None, 3, None, 0) == 1
    arr = (mi.mi_problem * 2)(_problem(mi, X=16, out=16), _problem(mi, X=16, out=16))
    assert L.mi_all_pairs_batched(arr, 2, None, 9) == 1       # bad mode
    arr[1].m = 0
    assert L.mi_all_pairs_batched(arr, 2, None, 0) == 1
    assert b"problem 1" in L.mi_last_error()
    arr[1].m = 10
    arr[1].validate = 1
    assert L.mi_all_pairs_batched(arr, 2, None, 0) == 1


def test_plan_and_tuner_argument_checks(L, tmp_path):
    i32 = ctypes.c_int32
    t, s = i32(), i32()
    assert L.mi_plan(0, 10, 0, ctypes.byref(t), ctypes.byref(s)) == 1
    assert L.mi_plan(10, 10, 5, ctypes.byref(t), ctypes.byref(s)) == 1
    assert L.mi_tune(0, 10, 0, None, None, None) == 1
    assert L.mi_tuner_load(str(tmp_path / "missing.jsonl").encode()) == 1
    L.mi_tuner_clear()
    f = tmp_path / "tuned.jsonl"
    assert L.mi_tuner_save(str(f).encode()) == 0
    f.write_text('{"mb": 40, "nb": 16, "aligned": 1, "tile": 128, "splits": 7, "ms": 1.5}\nnot json\n'
                 '{"mb": 41, "nb": 16, "aligned": 1, "tile": 96, "splits": 7, "ms": 1.5}\n'
                 '{"mb": 80, "nb": 64, "aligned": 1, "tile": 256, "splits": 9, "ms": 3.2, "fp4": 1}\n'
                 '{"mb": 81, "nb": 64, "aligned": 1, "tile": 256, "splits": 9, "ms": 3.2, "fp4": 7}\n')
    assert L.mi_tuner_load(str(f).encode()) == 0
    out = tmp_path / "again.jsonl"
    assert L.mi_tuner_save(str(out).encode()) == 0
    text = out.read_text()
    lines = text.strip().split("\n")
    assert len(lines) == 2 and '"tile": 96' not in text and '"fp4": 7' not in text
    assert any('"splits": 7' in ln and '"fp4": 0' in ln for ln in lines)      # an entry without the field: int8
    assert any('"splits": 9' in ln and '"fp4": 1' in ln for ln in lines)
    L.mi_tuner_clear()


def test_version_string(L):
    assert b"gfx950" in L.mi_version()


def test_python_binding_refuses_cpu_tensors(L):
    import torch
    from paper_2411_19702_amd import mi
    with pytest.raises(ValueError):
        mi.mi_all_pairs(torch.zeros((4, 3), dtype=torch.uint8))


def test_server_argument_checks_on_host(L):
    from paper_2411_19702_amd import mi
    h = ctypes.c_void_p()
    assert L.mi_server_create(None, 1 << 30, 4, 0) == 1
    assert L.mi_server_create(ctypes.byref(h), 0, 4, 0) == 1
    assert L.mi_server_create(ctypes.byref(h), 1 << 30, 0, 0) == 1
    assert L.mi_server_create(ctypes.byref(h), 1 << 30, 65, 0) == 1
    assert L.mi_server_create(ctypes.byref(h), 1 << 30, 4, -1) == 1
    t = ctypes.c_uint64()
    p = _problem(mi, X=16, out=16)
    assert L.mi_server_submit(None, ctypes.byref(p), ctypes.byref(t)) == 1
    assert L.mi_server_poll(None, 1) == 1
    assert L.mi_server_wait(None, 1, 0.0, None) == 1
    assert L.mi_server_destroy(None) == 1


def test_sparse_output_argument_checks(L):
    """Sparse (threshold) output: pairs need a counter, capacity >= 0 and a finite
    threshold; out may be NULL only when pairs is given."""
    import math
    from paper_2411_19702_amd import mi
    P = mi.mi_problem
    def prob(**kw):
        p = P()
        p.X, p.m, p.n, p.ldx, p.out = 16, 10, 8, 8, 0
        for k, v in kw.items():
            setattr(p, k, v)
        return p
    assert L.mi_all_pairs_ex(ctypes.byref(prob()), None) == 1                      # neither out nor pairs
    assert L.mi_all_pairs_ex(ctypes.byref(prob(pairs=64, pairs_capacity=4)), None) == 1   # no counter
    assert L.mi_all_pairs_ex(ctypes.byref(prob(pairs=64, pairs_capacity=-1, pairs_count=128)), None) == 1
    assert L.mi_all_pairs_ex(ctypes.byref(prob(pairs=64, pairs_capacity=4, pairs_count=128,
                                                pairs_threshold=math.nan)), None) == 1


def test_categorical_argument_checks(L):
    """Categorical entry points: level counts 1 .. 256, non-NULL buffers, and the
    indicator count N = sum (L_j - 1), all checked on the host."""
    from paper_2411_19702_amd import mi
    lv = (ctypes.c_int32 * 4)(3, 1, 256, 2)
    N = ctypes.c_int64(-1)
    assert L.mi_cat_indicators(lv, 4, ctypes.byref(N)) == 0 and N.value == 2 + 0 + 255 + 1
    assert L.mi_cat_indicators(lv, 0, ctypes.byref(N)) == 0 and N.value == 0
    assert L.mi_cat_indicators(None, 3, ctypes.byref(N)) == 1
    bad = (ctypes.c_int32 * 2)(3, 0)
    assert L.mi_cat_indicators(bad, 2, ctypes.byref(N)) == 1
    big = (ctypes.c_int32 * 2)(257, 2)
    assert L.mi_cat_indicators(big, 2, ctypes.byref(N)) == 1

    def prob(lvs, **kw):
        p = mi.mi_cat_problem()
        L.mi_cat_problem_init(ctypes.byref(p), 16, 10, len(lvs), ctypes.cast(lvs, ctypes.c_void_p), 32)
        for k, v in kw.items():
            setattr(p, k, v)
        return p
    assert L.mi_all_pairs_categorical(None, None) == 1
    assert L.mi_all_pairs_categorical(ctypes.byref(prob(bad)), None) == 1
    assert L.mi_all_pairs_categorical(ctypes.byref(prob(big)), None) == 1
    assert L.mi_all_pairs_categorical(ctypes.byref(prob(lv, out=None)), None) == 1
    assert L.mi_all_pairs_categorical(ctypes.byref(prob(lv, levels=None)), None) == 1
    assert L.mi_all_pairs_categorical(ctypes.byref(prob(lv, m=0)), None) == 1
    assert L.mi_all_pairs_categorical(ctypes.byref(prob(lv, ldx=3)), None) == 1
    assert L.mi_all_pairs_categorical(ctypes.byref(prob(lv, epilogue=3)), None) == 1
    assert L.mi_all_pairs_categorical(ctypes.byref(prob(lv, tile=5)), None) == 1
    assert L.mi_all_pairs_categorical(ctypes.byref(prob(lv, gram=3)), None) == 1
    empty = mi.mi_cat_problem()
    L.mi_cat_problem_init(ctypes.byref(empty), None, 5, 0, None, None)
    assert L.mi_all_pairs_categorical(ctypes.byref(empty), None) == 0        # v == 0: no-op


def test_packed_argument_checks(L):
    """Bit-packed input: the pitch counts bytes of 8 columns; the sparse algorithm
    and batches reject it; the packing utility checks its pitches."""
    from paper_2411_19702_amd import mi
    def prob(**kw):
        p = mi.mi_problem()
        p.X, p.m, p.n, p.out, p.packed = 16, 10, 17, 32, 1
        for k, v in kw.items():
            setattr(p, k, v)
        return p
    assert L.mi_all_pairs_ex(ctypes.byref(prob(ldx=2)), None) == 1               # 17 columns need 3 bytes
    assert L.mi_all_pairs_ex(ctypes.byref(prob(ldx=3, algo=1)), None) == 1       # sparse + packed
    arr = (mi.mi_problem * 1)(prob(ldx=3))
    assert L.mi_all_pairs_batched(arr, 1, None, 0) == 1                          # persistent mode: bytes only
    assert L.mi_pack_bits(16, 10, 17, 16, 32, 3, None) == 1                      # ldx < n
    assert L.mi_pack_bits(16, 10, 17, 17, 32, 2, None) == 1                      # ldp < ceil(n / 8)
    assert L.mi_pack_bits(None, 10, 17, 17, 32, 3, None) == 1
    assert L.mi_pack_bits(16, 0, 17, 17, 32, 3, None) == 0                       # empty: no-op


def test_fp4_argument_checks(L):
    """FP4 input (2 columns per byte) and the Gram choice: pitch in bytes of 2
    columns and at most 2^23, no sparse algorithm, no int8 Gram;
    batches check each problem the same way;
    the packing utility checks its pitches."""
    from paper_2411_19702_amd import mi
    def prob(**kw):
        p = mi.mi_problem()
        p.X, p.m, p.n, p.out, p.packed, p.ldx = 16, 10, 17, 32, mi.MI_INPUT_FP4, 9
        for k, v in kw.items():
            setattr(p, k, v)
        return p
    ex = lambda **kw: L.mi_all_pairs_ex(ctypes.byref(prob(**kw)), None)
    assert ex(ldx=8) == 1                                      # 17 columns need 9 bytes
    assert ex(gram=mi.MI_GRAM_INT8) == 1                       # FP4 input, int8 Gram
    assert ex(algo=mi.MI_ALGO_SPARSE) == 1
    assert ex(ldx=(1 << 23) + 16) == 1                         # 128-row stages, 32-bit offsets
    assert ex(packed=3) == 1 and ex(gram=3) == 1 and ex(gram=-1) == 1
    assert ex(packed=mi.MI_INPUT_BYTES, ldx=17, gram=mi.MI_GRAM_FP4, algo=mi.MI_ALGO_SPARSE) == 1
    for mode in (mi.MI_BATCH_PERSISTENT, mi.MI_BATCH_GRAPH, mi.MI_BATCH_SEQUENTIAL):
        arr = (mi.mi_problem * 1)(prob(gram=mi.MI_GRAM_INT8))
        assert L.mi_all_pairs_batched(arr, 1, None, mode) == 1    # checked per problem in batches too
    assert L.mi_pack_fp4(16, 10, 17, 16, 32, 9, None) == 1     # ldx < n
    assert L.mi_pack_fp4(16, 10, 17, 17, 32, 8, None) == 1     # ldq < ceil(n / 2)
    assert L.mi_pack_fp4(None, 10, 17, 17, 32, 9, None) == 1
    assert L.mi_pack_fp4(16, 0, 17, 17, 32, 9, None) == 0      # empty: no-op


def test_column_limit(L):
    """Tile coordinates are 16-bit fields: more than 32,767 panels of 128 columns
    is rejected before any device work (pairs-only problem, no n x n output)."""
    from paper_2411_19702_amd import mi
    p = mi.mi_problem()
    p.X, p.m, p.n, p.ldx = 16, 10, 32767 * 128 + 1, 32767 * 128 + 1
    p.pairs, p.pairs_capacity, p.pairs_count, p.pairs_threshold = 64, 4, 128, 0.5
    assert L.mi_all_pairs_ex(ctypes.byref(p), None) == 1
    assert b"n must be" in L.mi_last_error()


def test_noalloc_argument_checks(L):
    """The no-allocation entry point: the checks of mi_all_pairs_ex, plus no
    repack (aligned X and pitch only), no FP4 conversion of bytes and the dense
    algorithm only, all before any device work."""
    from paper_2411_19702_amd import mi
    def na(**kw):
        return L.mi_all_pairs_noalloc(ctypes.byref(_problem(mi, **{"X": 16, "out": 16, "ldx": 16, **kw})), None)
    assert L.mi_all_pairs_noalloc(None, None) == 1
    assert na(m=0) == 1 and na(ldx=3) == 1 and na(epilogue=5) == 1
    assert na(X=17) == 1 and b"aligned" in L.mi_last_error()
    assert na(ldx=24) == 1 and b"aligned" in L.mi_last_error()
    assert na(gram=mi.MI_GRAM_FP4) == 1 and b"FP4" in L.mi_last_error()
    assert na(algo=mi.MI_ALGO_SPARSE) == 1 and na(algo=mi.MI_ALGO_AUTO) == 1
    assert na(n=0) == 0                                         # no-op, no device work


def test_problem_array_keeps_its_tensors_and_passes_through():
    """problem_array copies the problems into one C array and keeps every
    problem's tensors referenced; the batched calls take it as it is."""
    import gc
    import weakref

    from paper_2411_19702_amd import mi

    class Held:  # stands in for a tensor a problem points to
        pass

    held = [Held() for _ in range(3)]
    refs = [weakref.ref(h) for h in held]
    probs = []
    for k, h in enumerate(held):
        p = mi.mi_problem()
        p.m, p.n = 10 + k, 4
        p._keep = (h,)
        probs.append(p)
    arr = mi.problem_array(probs)
    del probs, held, p, h
    gc.collect()
    assert all(r() is not None for r in refs)
    assert isinstance(arr, ctypes.Array) and len(arr) == 3 and [a.m for a in arr] == [10, 11, 12]
    assert mi._as_array(arr) is arr
    del arr
    gc.collect()
    assert all(r() is None for r in refs)
