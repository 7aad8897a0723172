"""GPU: many datasets in one call (persistent / hipGraph / sequential modes).

All three modes must give bitwise identical results (the counts are exact and
the epilogue is a pure function of them), and those results must match the
CPU oracle.  The full-size case is the 256-dataset recipe (m log-uniform in
[500, 50000], n uniform in [64, 2048], p_j ~ U[0.01, 0.5], 5% planted pairs).
"""
import numpy as np
import pytest
import torch

from paper_2411_19702_amd import mi, synth
from tests.gpu_util import compare_columns, compare_full, say

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _problems(Xs, outs, n11s, css, **kw):
    return [mi.make_problem(X, o, n11_out=a, colsum_out=c, **kw) for X, o, a, c in zip(Xs, outs, n11s, css)]


def _alloc(specs):
    outs = [torch.full((s.n, s.n), float("nan"), device=DEV) for s in specs]
    n11s = [torch.full((s.n, s.n), -1, dtype=torch.int32, device=DEV) for s in specs]
    css = [torch.full((max(s.n, 1),), -1, dtype=torch.int32, device=DEV) for s in specs]
    return outs, n11s, css


def _run(specs, Xs, mode, **kw):
    outs, n11s, css = _alloc(specs)
    mi.mi_all_pairs_batched(_problems(Xs, outs, n11s, css, **kw), mode=mode)
    torch.cuda.synchronize()
    return outs, n11s, css


def _equal(a, b):
    return all(torch.equal(x, y) for x, y in zip(a, b))


def _oracle_check(specs, Xs, res, idx_full, idx_sampled):
    outs, n11s, css = res
    for d in idx_full:
        s = specs[d]
        compare_full(Xs[d].cpu().numpy(), s.n, outs[d].cpu().numpy(), n11s[d].cpu().numpy(), css[d].cpu().numpy()[:s.n])
    rng = np.random.default_rng(3)
    for d in idx_sampled:
        s = specs[d]
        cols = sorted(set(rng.choice(s.n, size=min(s.n, 24), replace=False).tolist()) | {0, s.n - 1})
        Xs_cols = Xs[d][:, cols].cpu().numpy()
        compare_columns(Xs_cols, cols, outs[d].cpu().numpy(), n11s[d].cpu().numpy(), css[d].cpu().numpy())


def test_batched_modes_agree_and_match_oracle():
    specs = synth.specs_batched(count=40, m_range=(500, 20000), n_range=(64, 700))
    say(f"[batched] {len(specs)} datasets")
    Xs = [synth.generate(s, device=DEV) for s in specs]
    seq = _run(specs, Xs, mi.MI_BATCH_SEQUENTIAL)
    per = _run(specs, Xs, mi.MI_BATCH_PERSISTENT)
    gra = _run(specs, Xs, mi.MI_BATCH_GRAPH)
    for k in range(3):
        assert _equal(seq[k], per[k]), "persistent differs from sequential"
        assert _equal(seq[k], gra[k]), "graph differs from sequential"
    cost = [s.m * s.n * s.n for s in specs]
    order = np.argsort(cost)
    _oracle_check(specs, Xs, per, idx_full=order[:5].tolist(), idx_sampled=order[-3:].tolist())


def test_graph_replay_reuses_cached_graph():
    specs = synth.specs_batched(count=12, m_range=(500, 5000), n_range=(64, 300))
    say("[batched] graph replay")
    Xs = [synth.generate(s, device=DEV) for s in specs]
    outs, n11s, css = _alloc(specs)
    probs = _problems(Xs, outs, n11s, css)
    ref = None
    for rep in range(3):                      # capture once, replay twice, eager work in between
        for o in outs:
            o.fill_(float("nan"))
        mi.mi_all_pairs_batched(probs, mode=mi.MI_BATCH_GRAPH)
        torch.cuda.synchronize()
        _ = torch.ones(1000, device=DEV).sum().item()
        cur = [o.clone() for o in outs]
        if ref is None:
            ref = cur
        else:
            assert _equal(ref, cur)
    seq = _run(specs, Xs, mi.MI_BATCH_SEQUENTIAL)
    assert _equal(seq[0], ref)


def test_batched_mixed_layouts_and_edge_shapes():
    say("[batched] mixed layouts")
    base = synth.generate(synth.spec_random(41, 3000, 600, 0.02, 0.6), device=DEV)
    Xs = [
        base[:, :100],                        # pitched, aligned (ldx 600? 600 % 16 != 0 -> repacked)
        base[:, 3:250],                       # misaligned base pointer
        base[:1, :40],                        # one row
        base[:, :1],                          # one column
        synth.generate(synth.spec_random(42, 777, 512, 0.0, 1.0), device=DEV),   # aligned dense
        torch.zeros((64, 32), dtype=torch.uint8, device=DEV),
    ]
    specs = [type("S", (), {"n": X.shape[1], "m": X.shape[0]})() for X in Xs]
    seq = _run(specs, Xs, mi.MI_BATCH_SEQUENTIAL, splits=0)
    per = _run(specs, Xs, mi.MI_BATCH_PERSISTENT)
    for k in range(3):
        assert _equal(seq[k], per[k])
    for d, X in enumerate(Xs):
        n = X.shape[1]
        compare_full(X.cpu().numpy(), n, per[0][d].cpu().numpy(), per[1][d].cpu().numpy(), per[2][d].cpu().numpy()[:n])


def test_batched_full_recipe_256():
    specs = synth.specs_batched()
    say(f"[batched] full recipe: {len(specs)} datasets, {sum(s.m * s.n for s in specs) / 1e9:.2f} GB of X")
    Xs = [synth.generate(s, device=DEV) for s in specs]
    per = _run(specs, Xs, mi.MI_BATCH_PERSISTENT)
    seq = _run(specs, Xs, mi.MI_BATCH_SEQUENTIAL)
    for k in range(3):
        assert _equal(seq[k], per[k]), "persistent differs from 256 sequential plain calls"
    del seq
    cost = [s.m * s.n * s.n for s in specs]
    order = np.argsort(cost)
    _oracle_check(specs, Xs, per, idx_full=order[:4].tolist(), idx_sampled=order[-2:].tolist())


@pytest.mark.parametrize("mode", [mi.MI_BATCH_PERSISTENT, mi.MI_BATCH_GRAPH, mi.MI_BATCH_SEQUENTIAL])
def test_batched_counts_only_problems(mode):
    """Problems with no MI output (n11 and column sums only) mixed with full ones."""
    say(f"[batched] counts-only problems, mode {mode}")
    specs = [synth.spec_random(600 + k, 3000 + 700 * k, 90 + 37 * k, 0.02, 0.6, planted=3) for k in range(5)]
    Xs = [synth.generate(s, device=DEV) for s in specs]
    outs, n11s, css = _alloc(specs)
    probs = [mi.make_problem(X, None if k % 2 else o, n11_out=a, colsum_out=c)
             for k, (X, o, a, c) in enumerate(zip(Xs, outs, n11s, css))]
    mi.mi_all_pairs_batched(probs, mode=mode)
    torch.cuda.synchronize()
    for k, (s, X) in enumerate(zip(specs, Xs)):
        o, a, c = _run([s], [X], mi.MI_BATCH_SEQUENTIAL)
        assert torch.equal(n11s[k], a[0]) and torch.equal(css[k][:s.n], c[0][:s.n])
        if k % 2 == 0:
            assert torch.equal(outs[k], o[0])
        else:
            assert torch.isnan(outs[k]).all()       # untouched


def test_batched_wide_unaligned_and_aligned_share_one_gram():
    """A persistent batch whose unaligned datasets (converted to FP4, one of
    them with rows of several 64-chunk steps) hold most of the work runs its
    aligned byte datasets on the FP4 Gram too: bitwise the sequential mode's
    outputs (each dataset on its own choice), and the oracle's."""
    say("[batched] wide unaligned rows with aligned datasets")
    base = synth.generate(synth.spec_random(43, 4000, 2600, 0.02, 0.5), device=DEV)
    Xs = [
        base[:, 5:2505],                      # unaligned, 2,500 columns: 79 chunks per converted row
        base[:2000, 1:1201],                  # unaligned, 1,200 columns
        synth.generate(synth.spec_random(44, 900, 256, 0.0, 0.8), device=DEV),    # aligned, small
        synth.generate(synth.spec_random(45, 1200, 64, 0.0, 0.8), device=DEV),    # aligned, narrow
    ]
    specs = [type("S", (), {"n": X.shape[1], "m": X.shape[0]})() for X in Xs]
    seq = _run(specs, Xs, mi.MI_BATCH_SEQUENTIAL)
    per = _run(specs, Xs, mi.MI_BATCH_PERSISTENT)
    for k in range(3):
        assert _equal(seq[k], per[k])
    for d in (2, 3):
        X = Xs[d]
        n = X.shape[1]
        compare_full(X.cpu().numpy(), n, per[0][d].cpu().numpy(), per[1][d].cpu().numpy(), per[2][d].cpu().numpy()[:n])
    cols = [0, 1, 127, 128, 1023, 1024, 2047, 2048, 2499]
    compare_columns(Xs[0][:, cols].cpu().numpy(), cols, per[0][0].cpu().numpy(), per[1][0].cpu().numpy(),
                    per[2][0].cpu().numpy())
