"""GPU: the FP4 Gram (E2M1 operands, FP32 accumulation) against the int8 Gram
and the oracle.

A 0/1 entry is the E2M1 code of 1.0 or 0, so every product is exactly 0 or 1
and the FP32 accumulator holds the exact count while it stays below 2^24 (a
unit covers at most 2^24 rows).  The counts, hence every output, must then be
bitwise identical to the int8 path's; small cases are also checked against the
FP64 oracle.  The FP4 packing utility must equal a numpy nibble packing.
"""
import numpy as np
import pytest
import torch

from paper_2411_19702_amd import mi, synth
from tests.gpu_util import compare_full, say

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _pack_ref(Xh, n):
    nz = (Xh[:, :n] != 0).astype(np.uint8) * 2
    if n % 2:
        nz = np.concatenate([nz, np.zeros((nz.shape[0], 1), np.uint8)], axis=1)
    return (nz[:, 0::2] | (nz[:, 1::2] << 4)).astype(np.uint8)


def _run(X, n, **kw):
    out = torch.full((n, n), float("nan"), device=DEV)
    n11 = torch.full((n, n), -1, dtype=torch.int32, device=DEV)
    cs = torch.full((max(n, 1),), -1, dtype=torch.int32, device=DEV)
    mi.mi_all_pairs_ex(X, out=out, n=n, n11_out=n11, colsum_out=cs, **kw)
    torch.cuda.synchronize()
    return out, n11, cs


def _same(a, b, what=""):
    for x, y, name in zip(a, b, ("MI", "n11", "column sums")):
        assert torch.equal(x, y), f"{what}: FP4 {name} differ from the int8 Gram"


@pytest.mark.parametrize("m,n,pitch", [(5, 1, None), (100, 7, None), (1000, 64, None), (777, 129, 160),
                                       (300, 1000, 1003), (2, 4096, None), (70, 33, None)])
def test_pack_fp4_matches_numpy(m, n, pitch):
    say(f"[fp4 pack] {m}x{n} pitch={pitch}")
    spec = synth.spec_random(61 + n, m, n, 0.0, 1.0, ldx=pitch)
    X = synth.generate(spec, device=DEV)[:, :n]
    Q = mi.mi_pack_fp4(X, n)
    torch.cuda.synchronize()
    nb = (n + 1) // 2
    assert np.array_equal(Q.cpu().numpy()[:, :nb], _pack_ref(X.cpu().numpy(), n))
    # a pitched, unaligned destination; its bytes past ceil(n / 2) stay untouched
    W = torch.full((m, nb + 21), 0xAB, dtype=torch.uint8, device=DEV)
    mi.mi_pack_fp4(X, n, out=W[:, 3:3 + nb])
    torch.cuda.synchronize()
    Wh = W.cpu().numpy()
    assert np.array_equal(Wh[:, 3:3 + nb], _pack_ref(X.cpu().numpy(), n))
    assert (Wh[:, :3] == 0xAB).all() and (Wh[:, 3 + nb:] == 0xAB).all()


CASES = [  # (m, n): one and several 128-row stages, ragged rows and columns, several tiles
    (1, 1), (3, 2), (63, 17), (128, 16), (129, 129), (200, 300), (1000, 257), (4097, 130), (129, 385),
    (1000, 200), (20000, 1000), (515, 513),
]


@pytest.mark.parametrize("m,n", CASES)
@pytest.mark.parametrize("epi", [0, 1, 2])
def test_fp4_gram_equals_int8(m, n, epi):
    say(f"[fp4] {m}x{n} epi={epi}")
    spec = synth.spec_random(11 * m + n, m, n, 0.0, 1.0, planted=max(1, n // 20))
    X = synth.generate(spec, device=DEV)
    b = _run(X, n, epilogue=epi, gram=mi.MI_GRAM_INT8)
    f = _run(X, n, epilogue=epi, gram=mi.MI_GRAM_FP4)
    _same(b, f, "converted bytes")
    Q = mi.mi_pack_fp4(X, n)
    q = _run(Q, n, epilogue=epi, packed=mi.MI_INPUT_FP4)
    _same(b, q, "FP4 input")
    if m * n <= 1_000_000:
        compare_full(X.cpu().numpy(), n, f[0].cpu().numpy(), f[1].cpu().numpy(), f[2].cpu().numpy()[:n])


def test_fp4_sparse_pairs_output():
    """The threshold pair list on the FP4 Gram: the same set of (i, j, MI) as
    on the int8 Gram (append order is unspecified), and the same exact count."""
    say("[fp4] sparse pairs output")
    spec = synth.spec_random(77, 20000, 1700, 0.0, 0.6, planted=40)
    X = synth.generate(spec, device=DEV)
    res = []
    for g in (mi.MI_GRAM_INT8, mi.MI_GRAM_FP4):
        pairs, count = mi.mi_all_pairs_threshold(X, threshold=0.02, capacity=1 << 16, gram=g)
        torch.cuda.synchronize()
        k = int(count.item())
        assert 0 < k <= (1 << 16)
        rows = pairs[:k].cpu().numpy()
        res.append((k, set(map(tuple, rows.tolist()))))
    assert res[0][0] == res[1][0] and res[0][1] == res[1][1]


@pytest.mark.parametrize("tile,splits", [(1, 1), (2, 1), (1, 5), (2, 3), (2, 7)])
def test_fp4_configurations(tile, splits):
    say(f"[fp4] tile={tile} splits={splits}")
    spec = synth.spec_random(71, 30000, 700, 0.0, 0.5, planted=10)
    X = synth.generate(spec, device=DEV)
    b = _run(X, 700, tile=tile, splits=splits, gram=mi.MI_GRAM_INT8)
    f = _run(X, 700, tile=tile, splits=splits, gram=mi.MI_GRAM_FP4)
    _same(b, f, f"tile {tile} splits {splits}")


def test_fp4_unaligned_inputs_and_counts_only():
    say("[fp4] unaligned byte and FP4 inputs, counts-only output")
    spec = synth.spec_random(73, 5000, 333, 0.0, 0.7, planted=5)
    X = synth.generate(spec, device=DEV)
    b = _run(X, 333, gram=mi.MI_GRAM_INT8)
    wide = torch.zeros((5000, 333 + 9), dtype=torch.uint8, device=DEV)
    Xu = wide[:, 1:334]                      # bytes: base off by one, pitch 342
    Xu.copy_(X[:, :333])
    _same(b, _run(Xu, 333, gram=mi.MI_GRAM_FP4), "unaligned bytes")
    nb = (333 + 1) // 2
    Qw = torch.zeros((5000, nb + 7), dtype=torch.uint8, device=DEV)
    Qu = Qw[:, 3:3 + nb]                     # FP4: base off by 3, pitch nb + 7 (repacked)
    mi.mi_pack_fp4(X, 333, out=Qu)
    _same(b, _run(Qu, 333, packed=mi.MI_INPUT_FP4), "unaligned FP4")
    n11 = torch.empty((333, 333), dtype=torch.int32, device=DEV)
    mi.mi_all_pairs_ex(X, out=None, dense=False, n11_out=n11, gram=mi.MI_GRAM_FP4)
    torch.cuda.synchronize()
    assert torch.equal(n11, b[1])


def test_fp4_large_workload_equals_int8():
    """The 1,000,000 x 4,096 workload: the library's choice (FP4 at this shape)
    and both explicit Grams give bitwise the same MI matrix."""
    spec = synth.spec_large()
    say(f"[fp4] {spec.m}x{spec.n}")
    X = synth.generate(spec, device=DEV)
    outs = []
    for g in (mi.MI_GRAM_INT8, mi.MI_GRAM_FP4, mi.MI_GRAM_AUTO):
        o = torch.empty((spec.n, spec.n), device=DEV)
        mi.mi_all_pairs_ex(X, out=o, gram=g)
        outs.append(o)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])


def test_fp4_units_stay_below_2_24_rows():
    """m = 2^24 + 2^22 rows with one split requested: the library splits the
    rows so that no FP32 accumulator exceeds 2^24, and the counts stay exact
    (column sums above 2^24 included)."""
    m, n = (1 << 24) + (1 << 22), 40
    say(f"[fp4] {m}x{n}, splits=1 requested")
    g = torch.Generator(device=DEV)
    g.manual_seed(5)
    p = torch.linspace(0.8, 0.99, n, device=DEV)
    X = (torch.rand((m, n), generator=g, device=DEV) < p).to(torch.uint8)
    b = _run(X, n, splits=1, gram=mi.MI_GRAM_INT8)
    f = _run(X, n, splits=1, gram=mi.MI_GRAM_FP4)
    _same(b, f, "2^24 + 2^22 rows")
    cs = X.sum(dim=0, dtype=torch.int64)
    assert torch.equal(f[2].to(torch.int64), cs)
    assert int(cs.max()) > (1 << 24), "the case must hold counts above 2^24"


@pytest.mark.parametrize("mode", [mi.MI_BATCH_PERSISTENT, mi.MI_BATCH_GRAPH, mi.MI_BATCH_SEQUENTIAL])
def test_fp4_input_in_batches(mode):
    """FP4 and byte problems in one batch (every mode): each equal to its single int8 call."""
    say(f"[fp4] batch mode {mode}")
    specs = [synth.spec_random(950 + k, 2000 + 900 * k, 70 + 53 * k, 0.0, 0.8, planted=3) for k in range(4)]
    Xs = [synth.generate(s, device=DEV) for s in specs]
    outs = [torch.full((s.n, s.n), float("nan"), device=DEV) for s in specs]
    probs, keep = [], []  # problems hold raw pointers: keep the packed tensors alive
    for k, (s, X, o) in enumerate(zip(specs, Xs, outs)):
        if k % 2 == 0:
            keep.append(mi.mi_pack_fp4(X))
            probs.append(mi.make_problem(keep[-1], o, n=s.n, packed=mi.MI_INPUT_FP4))
        else:
            probs.append(mi.make_problem(X, o))
    for _ in range(2):  # the graph mode replays its cached graph the second time
        for o in outs:
            o.fill_(float("nan"))
        mi.mi_all_pairs_batched(probs, mode=mode)
        torch.cuda.synchronize()
        for X, o in zip(Xs, outs):
            want = torch.empty_like(o)
            mi.mi_all_pairs_ex(X, out=want, gram=mi.MI_GRAM_INT8)
            torch.cuda.synchronize()
            assert torch.equal(o, want)


@pytest.mark.parametrize("tile", [mi.MI_TILE_AUTO, mi.MI_TILE_128])
@pytest.mark.parametrize("mode", [mi.MI_BATCH_PERSISTENT, mi.MI_BATCH_GRAPH, mi.MI_BATCH_SEQUENTIAL])
def test_fp4_gram_on_bytes_in_batches(mode, tile):
    """Byte problems converted to FP4 inside a batch (aligned, pitched and
    unaligned, mixed with int8 ones and with the library's choice; the
    persistent mode runs one launch per Gram): each bitwise equal to its
    single int8 call, over two calls (the graph mode replays its graph)."""
    say(f"[fp4] byte problems with the FP4 Gram, batch mode {mode}, tile {tile}")
    shapes = [(3000, 200, None), (20000, 1700, None), (5000, 333, 341), (777, 129, None), (40000, 1600, None),
              (100, 40, 45)]
    Xs, specs = [], []
    for k, (m, n, pitch) in enumerate(shapes):
        spec = synth.spec_random(980 + k, m, n, 0.0, 0.8, planted=2, ldx=pitch)
        X = synth.generate(spec, device=DEV)[:, :n]
        if k == 2:  # base off by one byte: unaligned
            W = torch.zeros((m, n + 9), dtype=torch.uint8, device=DEV)
            W[:, 1:1 + n].copy_(X)
            X = W[:, 1:1 + n]
        Xs.append(X)
        specs.append(spec)
    grams = [mi.MI_GRAM_FP4, mi.MI_GRAM_AUTO, mi.MI_GRAM_FP4, mi.MI_GRAM_INT8, mi.MI_GRAM_FP4, mi.MI_GRAM_FP4]
    outs = [torch.full((s.n, s.n), float("nan"), device=DEV) for s in specs]
    n11s = [torch.full((s.n, s.n), -1, dtype=torch.int32, device=DEV) for s in specs]
    probs = [mi.make_problem(X, o, n11_out=c, gram=g, tile=tile) for X, o, c, g in zip(Xs, outs, n11s, grams)]
    for _ in range(2):
        for o in outs:
            o.fill_(float("nan"))
        mi.mi_all_pairs_batched(probs, mode=mode)
        torch.cuda.synchronize()
        for X, o, c in zip(Xs, outs, n11s):
            want, wc = _run(X, X.shape[1], gram=mi.MI_GRAM_INT8)[:2]
            assert torch.equal(o, want) and torch.equal(c, wc)


def test_fp4_validate_and_plan_ex():
    """validate checks the bytes before the FP4 conversion; mi_plan_ex reports
    the Gram each call runs (FP4 from n >= 1536 and m n^2 >= 6e10, and for
    layouts that need a copy)."""
    X = (torch.rand((3000, 1600), device=DEV) < 0.3).to(torch.uint8)
    out = mi.mi_all_pairs_ex(X, validate=True, gram=mi.MI_GRAM_FP4)
    want = mi.mi_all_pairs_ex(X, gram=mi.MI_GRAM_INT8)
    torch.cuda.synchronize()
    assert torch.equal(out, want)
    X[1234, 777] = 2
    with pytest.raises(mi.MIError) as ei:
        mi.mi_all_pairs_ex(X, validate=True, gram=mi.MI_GRAM_FP4)
    assert ei.value.status == 2                      # MI_ERR_NOT_BINARY
    big = torch.zeros((40000, 2048), dtype=torch.uint8, device=DEV)
    assert mi.mi_plan_ex(big)[2] == mi.MI_GRAM_FP4       # 1.7e11 >= 6e10
    assert mi.mi_plan_ex(big[:5000])[2] == mi.MI_GRAM_INT8  # 2.1e10
    assert mi.mi_plan_ex(big[:, :1024])[2] == mi.MI_GRAM_INT8
    assert mi.mi_plan_ex(big, gram=mi.MI_GRAM_INT8)[2] == mi.MI_GRAM_INT8
    assert mi.mi_plan_ex(big[:5000, 1:1001])[2] == mi.MI_GRAM_FP4   # unaligned: converted, not repacked
    assert mi.mi_plan_ex(big[:5000, :1000])[2] == mi.MI_GRAM_INT8   # pitch 2048, aligned
    assert mi.mi_plan_ex(big[:5000], gram=mi.MI_GRAM_FP4)[2] == mi.MI_GRAM_FP4
    Q = mi.mi_pack_fp4(big[:100])
    assert mi.mi_plan_ex(Q, n=2048, packed=mi.MI_INPUT_FP4)[2] == mi.MI_GRAM_FP4
    tile, splits, _ = mi.mi_plan_ex(big)
    assert tile in (mi.MI_TILE_128, mi.MI_TILE_256) and splits >= 1


def test_fp4_rejected_where_unsupported():
    X = torch.zeros((10, 40), dtype=torch.uint8, device=DEV)
    out = torch.empty((40, 40), device=DEV)
    with pytest.raises(mi.MIError):
        mi.mi_all_pairs_ex(X, out=out, gram=mi.MI_GRAM_FP4, algo=mi.MI_ALGO_SPARSE)
    with mi.Server(hbm_budget_bytes=1 << 30) as srv:
        with pytest.raises(mi.MIError):
            srv.submit(mi.mi_pack_fp4(X), out, n=40, packed=mi.MI_INPUT_FP4)


def test_fp4_input_validate():
    """validate on FP4 input: every code of columns < n must be 0 or 0b0010 (MI_ERR_NOT_BINARY
    otherwise); the unused high nibble of the last byte (odd n) is not checked."""
    say("[fp4] validate FP4 input")
    m, n = 777, 41
    X = synth.generate(synth.spec_random(4242, m, n, 0.0, 0.7, planted=2), device=DEV)
    Q = mi.mi_pack_fp4(X)
    want = mi.mi_all_pairs_ex(X, gram=mi.MI_GRAM_INT8)
    Q[:, -1] |= 0x70                                   # column 41 (past n): ignored
    got = mi.mi_all_pairs_ex(Q, n=n, packed=mi.MI_INPUT_FP4, validate=True)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    for row, byte, code in ((500, 7, 0x04), (0, 0, 0x30), (m - 1, 20, 0x01)):
        Qb = Q.clone()
        Qb[row, byte] = (Qb[row, byte] & 0xF0) | code if code < 0x10 else (Qb[row, byte] & 0x0F) | code
        with pytest.raises(mi.MIError) as ei:
            mi.mi_all_pairs_ex(Qb, n=n, packed=mi.MI_INPUT_FP4, validate=True)
        assert ei.value.status == 2, (row, byte, code)


def test_fp4_in_server():
    """Requests on the FP4 Gram (the library's choice and forced) next to
    int8 ones in the server: each bitwise equal to its single int8 call."""
    say("[fp4] server requests")
    shapes = [(30000, 1700, mi.MI_GRAM_AUTO), (4000, 300, mi.MI_GRAM_FP4), (20000, 2000, mi.MI_GRAM_INT8),
              (9000, 777, mi.MI_GRAM_FP4), (100, 50, mi.MI_GRAM_AUTO)]
    Xs = [synth.generate(synth.spec_random(990 + k, m, n, 0.0, 0.6, planted=2), device=DEV)
          for k, (m, n, _) in enumerate(shapes)]
    outs = [torch.full((n, n), float("nan"), device=DEV) for (_, n, _) in shapes]
    with mi.Server(hbm_budget_bytes=8 << 30, max_slots=3) as srv:
        tickets = [srv.submit(X, o, gram=g) for X, o, (_, _, g) in zip(Xs, outs, shapes)]
        for t in tickets:
            srv.wait(t)
    for X, o in zip(Xs, outs):
        want = torch.empty_like(o)
        mi.mi_all_pairs_ex(X, out=want, gram=mi.MI_GRAM_INT8)
        torch.cuda.synchronize()
        assert torch.equal(o, want)
