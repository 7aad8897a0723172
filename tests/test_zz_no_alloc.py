"""GPU: mi_all_pairs_noalloc, the entry point that allocates no device memory
(its scratch is the library's fixed device array), against mi_all_pairs_ex.

Both run the same kernels on the same plan, so MI, the counts and the column
sums must be bitwise equal.  Each case makes two calls in a row, the second on
a smaller input, so the second one runs on the array the first one left.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_2411_19702_amd import mi, synth
from tests.gpu_util import compare_full, say

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _pad16(k):
    return (k + 15) // 16 * 16


def _outputs(n):
    return (torch.full((n, n), float("nan"), device=DEV), torch.full((n, n), -1, dtype=torch.int32, device=DEV),
            torch.full((max(n, 1),), -1, dtype=torch.int32, device=DEV))


def _both(X, n, **kw):
    """(noalloc outputs, mi_all_pairs_ex outputs) for the same problem."""
    a = _outputs(n)
    b = _outputs(n)
    mi.mi_all_pairs_noalloc(X, out=a[0], n=n, n11_out=a[1], colsum_out=a[2], **kw)
    mi.mi_all_pairs_ex(X, out=b[0], n=n, n11_out=b[1], colsum_out=b[2], **kw)
    torch.cuda.synchronize()
    return a, b


def _same(a, b, what):
    for x, y, name in zip(a, b, ("MI", "n11", "column sums")):
        assert torch.equal(x, y), f"{what}: no-allocation {name} differ from mi_all_pairs_ex"


def _bytes(seed, m, n):
    spec = synth.spec_random(seed, m, n, 0.0, 0.7, ldx=_pad16(n), planted=max(1, n // 25))
    return synth.generate(spec, device=DEV)


# (m, n, tile, splits) of the first call, then of the second, smaller one.
PAIRS = [
    ((20000, 700, mi.MI_TILE_256, 3), (3000, 300, mi.MI_TILE_256, 2)),
    ((9000, 530, mi.MI_TILE_128, 5), (700, 130, mi.MI_TILE_128, 1)),
    ((50000, 1100, 0, 0), (4097, 257, 0, 0)),
]


@pytest.mark.parametrize("first,second", PAIRS)
def test_noalloc_bytes_two_calls(first, second):
    for k, (m, n, tile, splits) in enumerate((first, second)):
        say(f"[noalloc] bytes {m}x{n} tile={tile} splits={splits} call {k}")
        X = _bytes(7 * m + n, m, n)
        a, b = _both(X[:, :n], n, tile=tile, splits=splits, gram=mi.MI_GRAM_INT8)
        _same(a, b, f"{m}x{n}")
        if m * n <= 3_000_000:
            compare_full(X[:, :n].cpu().numpy(), n, a[0].cpu().numpy(), a[1].cpu().numpy(), a[2].cpu().numpy()[:n])


def test_noalloc_byte_input_defaults_to_int8():
    say("[noalloc] bytes 60000x1600, library's plan")
    m, n = 60000, 1600
    X = _bytes(991, m, n)[:, :n]
    a = _outputs(n)
    mi.mi_all_pairs_noalloc(X, out=a[0], n11_out=a[1], colsum_out=a[2])
    t, s, g = mi.mi_plan_ex(X, gram=mi.MI_GRAM_INT8)
    b = _outputs(n)
    mi.mi_all_pairs_ex(X, out=b[0], n11_out=b[1], colsum_out=b[2], gram=mi.MI_GRAM_INT8, tile=t, splits=s)
    torch.cuda.synchronize()
    _same(a, b, "library's plan")


def test_noalloc_fp4_and_bit_input_two_calls():
    for k, (m, n) in enumerate(((30000, 1500), (5000, 600))):
        say(f"[noalloc] FP4 and bit input {m}x{n} call {k}")
        X = _bytes(13 * m + n, m, n)[:, :n]
        nb4, nb1 = (n + 1) // 2, (n + 7) // 8
        Q = torch.zeros((m, _pad16(nb4)), dtype=torch.uint8, device=DEV)
        mi.mi_pack_fp4(X, n, out=Q[:, :nb4])
        B = torch.zeros((m, _pad16(nb1)), dtype=torch.uint8, device=DEV)
        mi.mi_pack_bits(X, n, out=B[:, :nb1])
        ref = _outputs(n)
        mi.mi_all_pairs_ex(X, out=ref[0], n11_out=ref[1], colsum_out=ref[2], gram=mi.MI_GRAM_INT8)
        for what, src, packed in (("FP4", Q, mi.MI_INPUT_FP4), ("bits", B, mi.MI_INPUT_BITS)):
            a, b = _both(src, n, packed=packed, splits=3)
            _same(a, b, f"{what} {m}x{n}")
            _same(a, ref, f"{what} {m}x{n} against the byte input")


def test_noalloc_threshold_pairs_and_fp64_epilogue():
    for k, (m, n) in enumerate(((12000, 900), (2500, 400))):
        say(f"[noalloc] pairs + epilogues {m}x{n} call {k}")
        X = _bytes(5 * m + n, m, n)[:, :n]
        for epi in (mi.MI_EPI_FP32_FP64_FALLBACK, mi.MI_EPI_FP64):
            a, b = _both(X, n, epilogue=epi, splits=2, gram=mi.MI_GRAM_INT8)
            _same(a, b, f"epilogue {epi}")
        cap = n * n
        got = []
        for fn in (mi.mi_all_pairs_noalloc, mi.mi_all_pairs_ex):
            pairs = torch.full((cap, 3), -1, dtype=torch.int32, device=DEV)
            cnt = torch.full((1,), -1, dtype=torch.int64, device=DEV)
            fn(X, dense=False, pairs=pairs, pairs_count=cnt, pairs_threshold=0.002, splits=2, gram=mi.MI_GRAM_INT8)
            torch.cuda.synchronize()
            c = int(cnt.item())
            rows = pairs[:c].cpu().numpy()
            got.append((c, rows[np.lexsort((rows[:, 1], rows[:, 0]))]))
        assert got[0][0] == got[1][0] and got[0][0] > 0
        assert np.array_equal(got[0][1], got[1][1])


def test_noalloc_workspace_limit():
    # 5,700 columns at 256-wide tiles: 276 tiles, 73 MB of workspace with
    # splits; the library's plan then runs unsplit.
    m, n = 20000, 5700
    say(f"[noalloc] {m}x{n}: workspace above the array")
    X = _bytes(4242, m, n)[:, :n]
    a = _outputs(n)
    mi.mi_all_pairs_noalloc(X, out=a[0], n11_out=a[1], colsum_out=a[2], tile=mi.MI_TILE_256)
    b = _outputs(n)
    mi.mi_all_pairs_ex(X, out=b[0], n11_out=b[1], colsum_out=b[2], tile=mi.MI_TILE_256, splits=1,
                       gram=mi.MI_GRAM_INT8)
    torch.cuda.synchronize()
    _same(a, b, "unsplit fallback")
    with pytest.raises(mi.MIError) as e:  # an explicit split count that does not fit
        mi.mi_all_pairs_noalloc(X, out=a[0], tile=mi.MI_TILE_256, splits=2)
    assert e.value.status == 1 and "workspace" in e.value.message


def test_noalloc_rejections_and_validate():
    say("[noalloc] rejections")
    m, n = 1000, 64
    X = _bytes(77, m, n)[:, :n]
    out = torch.empty((n, n), device=DEV)
    for kw in (dict(gram=mi.MI_GRAM_FP4), dict(algo=mi.MI_ALGO_SPARSE), dict(algo=mi.MI_ALGO_AUTO)):
        with pytest.raises(mi.MIError) as e:
            mi.mi_all_pairs_noalloc(X, out=out, **kw)
        assert e.value.status == 1
    Y = torch.zeros((m, n + 1), dtype=torch.uint8, device=DEV)  # pitch 65: not a multiple of 16
    with pytest.raises(mi.MIError) as e:
        mi.mi_all_pairs_noalloc(Y[:, :n], out=out)
    assert e.value.status == 1 and "aligned" in e.value.message
    Z = X.clone()
    Z[500, 7] = 3
    with pytest.raises(mi.MIError) as e:
        mi.mi_all_pairs_noalloc(Z, out=out, validate=True)
    assert e.value.status == 2
    # and the entry point still works after the errors
    a, b = _both(X, n, gram=mi.MI_GRAM_INT8, validate=True)
    _same(a, b, "after rejections")
    p = mi.make_problem(X, None, n=0)
    assert mi.lib().mi_all_pairs_noalloc(ctypes.byref(p), None) == 0  # n == 0: no-op
