"""GPU: bit-packed input (8 columns per byte) against the byte layout and the
oracle.

The packed kernel unpacks each stage on chip into the same LDS layout the
byte kernel stages, so MI, counts and column sums must be bitwise identical
to the byte path's; small cases are also checked against the FP64 oracle.
The packing utility must equal numpy.packbits(..., bitorder="little").
"""
import numpy as np
import pytest
import torch

from paper_2411_19702_amd import mi, synth
from tests.gpu_util import compare_full, say

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _pack_ref(Xh, n):
    return np.packbits(Xh[:, :n] != 0, axis=1, bitorder="little")


def _run(X, n, packed, **kw):
    out = torch.full((n, n), float("nan"), device=DEV)
    n11 = torch.full((n, n), -1, dtype=torch.int32, device=DEV)
    cs = torch.full((max(n, 1),), -1, dtype=torch.int32, device=DEV)
    mi.mi_all_pairs_ex(X, out=out, n=n, n11_out=n11, colsum_out=cs, packed=packed, **kw)
    torch.cuda.synchronize()
    return out, n11, cs


@pytest.mark.parametrize("m,n,pitch", [(5, 1, None), (100, 7, None), (1000, 64, None), (777, 129, 160),
                                       (300, 1000, 1003), (2, 4096, None)])
def test_pack_bits_matches_numpy(m, n, pitch):
    say(f"[pack] {m}x{n} pitch={pitch}")
    spec = synth.spec_random(31 + n, m, n, 0.0, 1.0, ldx=pitch)
    X = synth.generate(spec, device=DEV)[:, :n]
    P = mi.mi_pack_bits(X, n)
    torch.cuda.synchronize()
    assert np.array_equal(P.cpu().numpy()[:, :(n + 7) // 8], _pack_ref(X.cpu().numpy(), n))
    # a pitched, unaligned destination
    Q = torch.zeros((m, (n + 7) // 8 + 5), dtype=torch.uint8, device=DEV)[:, 3:3 + (n + 7) // 8]
    mi.mi_pack_bits(X, n, out=Q)
    torch.cuda.synchronize()
    assert np.array_equal(Q.cpu().numpy(), _pack_ref(X.cpu().numpy(), n))


CASES = [  # (m, n)
    (1, 1), (3, 2), (63, 17), (64, 16), (65, 129), (200, 300), (1000, 257), (4097, 130), (129, 385),
    (1000, 200), (20000, 1000),
]


@pytest.mark.parametrize("m,n", CASES)
@pytest.mark.parametrize("epi", [0, 2])
def test_packed_equals_bytes(m, n, epi):
    say(f"[packed] {m}x{n} epi={epi}")
    spec = synth.spec_random(7 * m + n, m, n, 0.0, 1.0, planted=max(1, n // 20))
    X = synth.generate(spec, device=DEV)
    P = mi.mi_pack_bits(X, n)
    b = _run(X, n, False, epilogue=epi)
    p = _run(P, n, True, epilogue=epi)
    for x, y, name in zip(b, p, ("MI", "n11", "column sums")):
        assert torch.equal(x, y), f"packed {name} differ from the byte layout"
    if m * n <= 1_000_000:
        compare_full(X.cpu().numpy(), n, p[0].cpu().numpy(), p[1].cpu().numpy(), p[2].cpu().numpy()[:n])


@pytest.mark.parametrize("tile,splits", [(1, 1), (2, 1), (1, 5), (2, 3)])
def test_packed_configurations(tile, splits):
    say(f"[packed] tile={tile} splits={splits}")
    spec = synth.spec_random(41, 30000, 700, 0.0, 0.5, planted=10)
    X = synth.generate(spec, device=DEV)
    P = mi.mi_pack_bits(X)
    b = _run(X, 700, False, tile=tile, splits=splits)
    p = _run(P, 700, True, tile=tile, splits=splits)
    for x, y in zip(b, p):
        assert torch.equal(x, y)


def test_packed_unaligned_pitch_and_counts_only():
    say("[packed] unaligned packed pitch (repacked), counts-only output")
    spec = synth.spec_random(43, 5000, 333, 0.0, 0.7, planted=5)
    X = synth.generate(spec, device=DEV)
    nb = (333 + 7) // 8
    wide = torch.zeros((5000, nb + 9), dtype=torch.uint8, device=DEV)
    Pu = wide[:, 1:1 + nb]                         # base off by one byte, pitch nb + 9
    mi.mi_pack_bits(X, out=Pu)
    b = _run(X, 333, False)
    p = _run(Pu, 333, True)
    for x, y in zip(b, p):
        assert torch.equal(x, y)
    n11 = torch.empty((333, 333), dtype=torch.int32, device=DEV)
    mi.mi_all_pairs_ex(Pu, out=None, dense=False, n=333, n11_out=n11, packed=True)
    torch.cuda.synchronize()
    assert torch.equal(n11, b[1])


def test_packed_large_workload_equals_bytes():
    """The 1,000,000 x 4,096 workload, packed: every output bitwise equal to the byte path."""
    spec = synth.spec_large()
    say(f"[packed] {spec.m}x{spec.n}")
    X = synth.generate(spec, device=DEV)
    P = mi.mi_pack_bits(X)
    out_b = torch.empty((spec.n, spec.n), device=DEV)
    out_p = torch.empty((spec.n, spec.n), device=DEV)
    mi.mi_all_pairs_ex(X, out=out_b)
    mi.mi_all_pairs_ex(P, out=out_p, n=spec.n, packed=True)
    torch.cuda.synchronize()
    assert torch.equal(out_b, out_p)


def test_packed_rejected_where_unsupported():
    X = torch.zeros((10, 2), dtype=torch.uint8, device=DEV)
    out = torch.empty((16, 16), device=DEV)
    with pytest.raises(mi.MIError):
        mi.mi_all_pairs_ex(X, out=out, n=16, packed=True, algo=mi.MI_ALGO_SPARSE)
    p = mi.make_problem(X, out, n=16, packed=True)
    with pytest.raises(mi.MIError):
        mi.mi_all_pairs_batched([p], mode=mi.MI_BATCH_PERSISTENT)
    with pytest.raises(ValueError):
        mi.mi_all_pairs_ex(X, out=out, n=17, packed=True)   # needs 3 bytes per row


@pytest.mark.parametrize("mode", [mi.MI_BATCH_GRAPH, mi.MI_BATCH_SEQUENTIAL])
def test_packed_in_batches(mode):
    """Packed and byte problems in one graph / sequential batch: each equal to its single call."""
    say(f"[packed] batch mode {mode}")
    specs = [synth.spec_random(900 + k, 2000 + 900 * k, 70 + 53 * k, 0.0, 0.8, planted=3) for k in range(4)]
    Xs = [synth.generate(s, device=DEV) for s in specs]
    Ps = [mi.mi_pack_bits(X) for X in Xs]
    nb = (specs[3].n + 7) // 8
    Pu = torch.zeros((specs[3].m, nb + 3), dtype=torch.uint8, device=DEV)[:, 1:1 + nb]   # unaligned: repacked
    mi.mi_pack_bits(Xs[3], out=Pu)
    Ps[3] = Pu
    outs = [torch.full((s.n, s.n), float("nan"), device=DEV) for s in specs]
    probs = []
    for k, (s, X, P, o) in enumerate(zip(specs, Xs, Ps, outs)):
        probs.append(mi.make_problem(P, o, n=s.n, packed=True) if k % 2 == 0 or k == 3 else mi.make_problem(X, o))
    for _ in range(2):   # the graph mode replays its cached graph the second time
        for o in outs:
            o.fill_(float("nan"))
        mi.mi_all_pairs_batched(probs, mode=mode)
        torch.cuda.synchronize()
        for s, X, o in zip(specs, Xs, outs):
            want = torch.empty_like(o)
            mi.mi_all_pairs_ex(X, out=want)
            torch.cuda.synchronize()
            assert torch.equal(o, want)


@pytest.mark.parametrize("m,n", CASES)
def test_packed_bits_on_fp4_gram_equal_bytes(m, n):
    """Bits unpacked on chip to FP4 codes (gram = FP4): MI, n11 and column sums
    bitwise equal to the byte layout on the int8 Gram; small cases against the oracle."""
    say(f"[packed fp4] {m}x{n}")
    spec = synth.spec_random(9 * m + n, m, n, 0.0, 1.0, planted=max(1, n // 20))
    X = synth.generate(spec, device=DEV)
    P = mi.mi_pack_bits(X, n)
    b = _run(X, n, False, gram=mi.MI_GRAM_INT8)
    p = _run(P, n, True, gram=mi.MI_GRAM_FP4)
    for x, y, name in zip(b, p, ("MI", "n11", "column sums")):
        assert torch.equal(x, y), f"bits on the FP4 Gram: {name} differ from the byte layout"
    if m * n <= 1_000_000:
        compare_full(X.cpu().numpy(), n, p[0].cpu().numpy(), p[1].cpu().numpy(), p[2].cpu().numpy()[:n])


@pytest.mark.parametrize("tile,splits", [(1, 1), (2, 1), (1, 5), (2, 3)])
def test_packed_bits_on_fp4_gram_configurations(tile, splits):
    spec = synth.spec_random(45, 30000, 700, 0.0, 0.5, planted=10)
    X = synth.generate(spec, device=DEV)
    P = mi.mi_pack_bits(X)
    b = _run(X, 700, False, tile=tile, splits=splits, gram=mi.MI_GRAM_INT8)
    p = _run(P, 700, True, tile=tile, splits=splits, gram=mi.MI_GRAM_FP4)
    for x, y in zip(b, p):
        assert torch.equal(x, y)


def test_packed_bits_on_fp4_gram_large_workload_and_batches():
    """The 1,000,000 x 4,096 workload from bits on the FP4 Gram, bitwise equal
    to the byte path; bits-on-FP4 problems in graph and sequential batches."""
    spec = synth.spec_large()
    say(f"[packed fp4] {spec.m}x{spec.n}")
    X = synth.generate(spec, device=DEV)
    P = mi.mi_pack_bits(X)
    out_b = torch.empty((spec.n, spec.n), device=DEV)
    out_p = torch.empty((spec.n, spec.n), device=DEV)
    mi.mi_all_pairs_ex(X, out=out_b, gram=mi.MI_GRAM_INT8)
    mi.mi_all_pairs_ex(P, out=out_p, n=spec.n, packed=True, gram=mi.MI_GRAM_FP4)
    torch.cuda.synchronize()
    assert torch.equal(out_b, out_p)
    del X, P, out_b, out_p
    specs = [synth.spec_random(960 + k, 3000 + 700 * k, 90 + 41 * k, 0.0, 0.8, planted=3) for k in range(3)]
    Xs = [synth.generate(s, device=DEV) for s in specs]
    Ps = [mi.mi_pack_bits(X) for X in Xs]
    for mode in (mi.MI_BATCH_GRAPH, mi.MI_BATCH_SEQUENTIAL):
        outs = [torch.full((s.n, s.n), float("nan"), device=DEV) for s in specs]
        probs = [mi.make_problem(P, o, n=s.n, packed=True, gram=mi.MI_GRAM_FP4) for P, o, s in zip(Ps, outs, specs)]
        for _ in range(2):
            mi.mi_all_pairs_batched(probs, mode=mode)
            torch.cuda.synchronize()
            for X, o in zip(Xs, outs):
                want = torch.empty_like(o)
                mi.mi_all_pairs_ex(X, out=want, gram=mi.MI_GRAM_INT8)
                torch.cuda.synchronize()
                assert torch.equal(o, want)


def test_graph_batches_alternating_gram_on_the_same_buffers():
    """The graph mode keys its cached graphs by each problem's Gram too: the same bit-packed
    buffers and plan asked for the int8 and the FP4 Gram in turn replay the graph of the Gram
    asked for, and every replay equals the byte layout's single call."""
    say("[packed] graph batches alternating int8 / FP4 Gram")
    spec = synth.spec_random(961, 5000, 333, 0.0, 0.7, planted=4)
    X = synth.generate(spec, device=DEV)
    P = mi.mi_pack_bits(X)
    want = torch.empty((spec.n, spec.n), device=DEV)
    mi.mi_all_pairs_ex(X, out=want, gram=mi.MI_GRAM_INT8)
    out = torch.empty_like(want)
    for gram in (mi.MI_GRAM_INT8, mi.MI_GRAM_FP4, mi.MI_GRAM_INT8, mi.MI_GRAM_FP4):
        out.fill_(float("nan"))
        p = mi.make_problem(P, out, n=spec.n, packed=True, gram=gram, tile=mi.MI_TILE_128, splits=1)
        mi.mi_all_pairs_batched([p], mode=mi.MI_BATCH_GRAPH)
        torch.cuda.synchronize()
        assert torch.equal(out, want), gram
