"""GPU: the sparse-input path (1-1 counts as the sum over rows of the pairs of
ones) against the dense int8 matrix-core path and the oracle.

Both paths evaluate MI with the same per-pair arithmetic from the same exact
counts, so their outputs (MI, counts, column sums, pair lists) must be
bitwise identical; small cases are also checked element by element against
the FP64 oracle.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2411_19702_amd import mi, synth
from tests.gpu_util import MI_TOL, compare_full, say

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _run(X, n, algo, epi=0, **kw):
    out = torch.full((n, n), float("nan"), device=DEV)
    n11 = torch.full((n, n), -1, dtype=torch.int32, device=DEV)
    cs = torch.full((max(n, 1),), -1, dtype=torch.int32, device=DEV)
    mi.mi_all_pairs_ex(X, out=out, n=n, n11_out=n11, colsum_out=cs, epilogue=epi, algo=algo, **kw)
    torch.cuda.synchronize()
    return out, n11, cs


def _sparse_X(seed, m, n, density, pitch=None):
    spec = synth.spec_random(seed, m, n, 0.0, 2.0 * density, ldx=pitch, planted=max(1, n // 50))
    return synth.generate(spec, device=DEV)[:, :n]


CASES = [  # (m, n, density, pitch)
    (1000, 200, 0.01, None),
    (4097, 300, 0.005, None),
    (777, 129, 0.02, 160),       # pitched, aligned
    (5000, 513, 0.003, 515),     # unaligned pitch
    (64, 17, 0.1, None),
]


@pytest.mark.parametrize("m,n,density,pitch", CASES)
@pytest.mark.parametrize("epi", [0, 1, 2])
def test_sparse_input_equals_dense(m, n, density, pitch, epi):
    say(f"[sparse-in] {m}x{n} d={density} pitch={pitch} epi={epi}")
    X = _sparse_X(1000 + n, m, n, density, pitch)
    d = _run(X, n, mi.MI_ALGO_DENSE, epi)
    s = _run(X, n, mi.MI_ALGO_SPARSE, epi)
    for a, b, name in zip(d, s, ("MI", "n11", "column sums")):
        assert torch.equal(a, b), f"sparse-input {name} differ from the dense path"
    if m * n <= 2_000_000:
        compare_full(X.cpu().numpy(), n, s[0].cpu().numpy(), s[1].cpu().numpy(), s[2].cpu().numpy()[:n])


def test_sparse_input_extreme_rows_and_many_columns():
    say("[sparse-in] all-ones and empty rows; 17,000 columns (global column sums)")
    X = _sparse_X(7, 300, 700, 0.01)
    X[5, :] = 1          # a row with every column set: 244,650 pairs in one wave
    X[6, :] = 0
    d = _run(X, 700, mi.MI_ALGO_DENSE)
    s = _run(X, 700, mi.MI_ALGO_SPARSE)
    assert all(torch.equal(a, b) for a, b in zip(d, s))
    compare_full(X.cpu().numpy(), 700, s[0].cpu().numpy(), s[1].cpu().numpy(), s[2].cpu().numpy()[:700])
    W = _sparse_X(8, 200, 17000, 0.002)
    d = _run(W, 17000, mi.MI_ALGO_DENSE)
    s = _run(W, 17000, mi.MI_ALGO_SPARSE)
    assert all(torch.equal(a, b) for a, b in zip(d, s))


def test_auto_and_pairs_output():
    say("[sparse-in] auto choice and the pair list")
    for density in (0.002, 0.3):
        X = _sparse_X(21, 3000, 400, density)
        d = _run(X, 400, mi.MI_ALGO_DENSE)
        a = _run(X, 400, mi.MI_ALGO_AUTO)
        assert all(torch.equal(x, y) for x, y in zip(d, a))
    X = _sparse_X(22, 3000, 400, 0.004)
    lists = []
    for algo in (mi.MI_ALGO_DENSE, mi.MI_ALGO_SPARSE):
        pairs, count = mi.mi_all_pairs_threshold(X, 0.001, 400 * 400, algo=algo)
        torch.cuda.synchronize()
        k = int(count.item())
        rows = pairs[:k].cpu().numpy()
        lists.append(sorted(map(tuple, rows.tolist())))
    assert lists[0] == lists[1] and len(lists[0]) > 0


def test_auto_from_a_row_sample():
    """More rows than twice the 4,096-row sample: the choice starts from the
    sample (dense when it is clearly cheaper, else the full count decides)."""
    say("[sparse-in] auto from a row sample")
    for density in (0.0005, 0.01, 0.3):
        X = _sparse_X(23, 40000, 300, density)
        d = _run(X, 300, mi.MI_ALGO_DENSE)
        a = _run(X, 300, mi.MI_ALGO_AUTO)
        assert all(torch.equal(x, y) for x, y in zip(d, a)), density


def test_row_offset_scan_over_many_chunks():
    """4,300,000 rows: the row-offset scan runs more than 1,024 chunks of
    4,096 rows, so its one-block scan of the chunk sums takes several passes."""
    say("[sparse-in] 4,300,000 x 40: multi-pass scan")
    X = _sparse_X(24, 4_300_000, 40, 0.05)
    d = _run(X, 40, mi.MI_ALGO_DENSE)
    s = _run(X, 40, mi.MI_ALGO_SPARSE)
    for a, b, name in zip(d, s, ("MI", "n11", "column sums")):
        assert torch.equal(a, b), f"sparse-input {name} differ from the dense path"


def test_batches_and_server_reject_sparse_algo():
    X = _sparse_X(23, 100, 64, 0.05)
    out = torch.empty((64, 64), device=DEV)
    p = mi.make_problem(X, out, algo=mi.MI_ALGO_SPARSE)
    with pytest.raises(mi.MIError) as ei:
        mi.mi_all_pairs_batched([p], mode=mi.MI_BATCH_PERSISTENT)
    assert ei.value.status == 1
    with mi.Server(hbm_budget_bytes=1 << 30, max_slots=1) as srv:
        with pytest.raises(mi.MIError) as ei:
            srv.submit(X, out, algo=mi.MI_ALGO_SPARSE)
        assert ei.value.status == 1
