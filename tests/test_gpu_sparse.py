"""GPU: the sparse (threshold) output, the blockwise form of the result.

Every pair i < j with MI >= threshold is appended to a list in no particular
order.  The list must be exactly the dense output filtered at the threshold
(same values, bitwise), computed in the same call; against the FP64 oracle
it must hold every pair clearly above the threshold and nothing clearly
below it; a too-small capacity keeps the true count and a valid subset.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2411_19702_amd import mi, synth
from tests.gpu_util import MI_TOL, say

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _pairs_to_dict(pairs: torch.Tensor, count: int):
    k = min(count, pairs.shape[0])
    a = pairs[:k].cpu().numpy()
    vals = a[:, 2].copy().view(np.float32)
    d = {}
    for (i, j), v in zip(a[:, :2].tolist(), vals.tolist()):
        assert (i, j) not in d, f"duplicate pair {(i, j)}"
        d[(i, j)] = v
    return d


def _dense_filter(out: np.ndarray, thr: float):
    n = out.shape[0]
    iu, ju = np.triu_indices(n, 1)
    v = out[iu, ju]
    keep = v >= np.float32(thr)
    return {(int(i), int(j)): float(x) for i, j, x in zip(iu[keep], ju[keep], v[keep])}


@pytest.mark.parametrize("shape,thr,tile", [((1000, 200), 0.01, 0), ((1000, 200), 0.0, 0), ((700, 300), 0.002, 1),
                                            ((700, 300), 0.002, 2), ((3000, 513), 0.005, 0)])
def test_sparse_equals_filtered_dense_and_oracle(shape, thr, tile):
    m, n = shape
    spec = synth.spec_random(123 + n, m, n, 0.02, 0.6, planted=max(2, n // 20))
    say(f"[sparse] {m}x{n} thr={thr} tile={tile}")
    X = synth.generate(spec, device=DEV)
    out = torch.full((n, n), float("nan"), device=DEV)
    pairs, count = mi.mi_all_pairs_threshold(X, thr, n * n, dense_out=out, tile=tile)
    torch.cuda.synchronize()
    cnt = int(count.item())
    got = _pairs_to_dict(pairs, cnt)
    assert len(got) == cnt
    dense = out.cpu().numpy()
    assert got == _dense_filter(dense, thr), "sparse output differs from the filtered dense output"
    _, o_mi = oracle.all_pairs(X.cpu().numpy())
    iu, ju = np.triu_indices(n, 1)
    ov = o_mi[iu, ju]
    must = {(int(i), int(j)) for i, j, v in zip(iu, ju, ov) if v >= thr + MI_TOL}
    may = {(int(i), int(j)) for i, j, v in zip(iu, ju, ov) if v >= thr - MI_TOL}
    assert must <= set(got), "a pair clearly above the threshold is missing"
    assert set(got) <= may, "a pair clearly below the threshold was emitted"
    for (i, j), v in got.items():
        assert abs(v - o_mi[i, j]) <= MI_TOL
    say(f"  {cnt} pairs")


def test_sparse_without_dense_and_overflow():
    spec = synth.spec_small()
    X = synth.generate(spec, device=DEV)
    thr = 0.0005
    say("[sparse] no dense output; capacity overflow")
    pairs, count = mi.mi_all_pairs_threshold(X, thr, spec.n * spec.n)
    torch.cuda.synchronize()
    full = _pairs_to_dict(pairs, int(count.item()))
    ref = torch.empty((spec.n, spec.n), device=DEV)
    mi.mi_all_pairs_ex(X, out=ref)
    torch.cuda.synchronize()
    assert full == _dense_filter(ref.cpu().numpy(), thr)
    cap = max(1, len(full) // 3)
    p2, c2 = mi.mi_all_pairs_threshold(X, thr, cap)
    torch.cuda.synchronize()
    assert int(c2.item()) == len(full), "the count must be the total even past capacity"
    part = _pairs_to_dict(p2, int(c2.item()))
    assert len(part) == cap
    for k, v in part.items():
        assert full[k] == v
    p3, c3 = mi.mi_all_pairs_threshold(X, 1e9, 16)        # nothing qualifies
    torch.cuda.synchronize()
    assert int(c3.item()) == 0


def test_sparse_in_all_batch_modes():
    specs = synth.specs_batched(count=12, m_range=(500, 6000), n_range=(64, 700))
    Xs = [synth.generate(s, device=DEV) for s in specs]
    thr = 0.003
    say("[sparse] batched modes")
    results = {}
    for name, mode in (("sequential", mi.MI_BATCH_SEQUENTIAL), ("persistent", mi.MI_BATCH_PERSISTENT),
                       ("graph", mi.MI_BATCH_GRAPH)):
        pl = [torch.empty((s.n * s.n, 3), dtype=torch.int32, device=DEV) for s in specs]
        cl = [torch.full((1,), -1, dtype=torch.int64, device=DEV) for s in specs]
        probs = [mi.make_problem(X, None, pairs=p, pairs_count=c, pairs_threshold=thr) for X, p, c in zip(Xs, pl, cl)]
        for _rep in range(2 if mode == mi.MI_BATCH_GRAPH else 1):   # a graph replay re-zeroes the counters
            mi.mi_all_pairs_batched(probs, mode=mode)
            torch.cuda.synchronize()
        results[name] = [_pairs_to_dict(p, int(c.item())) for p, c in zip(pl, cl)]
    assert results["sequential"] == results["persistent"] == results["graph"]
    for X, s, got in list(zip(Xs, specs, results["persistent"]))[:4]:
        ref = torch.empty((s.n, s.n), device=DEV)
        mi.mi_all_pairs_ex(X, out=ref)
        torch.cuda.synchronize()
        assert got == _dense_filter(ref.cpu().numpy(), thr)
