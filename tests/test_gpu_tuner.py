"""GPU: the autotuner.  It times the Gram the library would run for the shape
(int8, or FP4 from n >= 1536 and m n^2 >= 6e10) and the planner then uses the
fastest (tile, splits); outputs do not depend on the plan (counts are exact),
so they stay bitwise the same.  Entries survive a save / clear / load round
trip.  Each test clears the tuner afterwards (entries live for the process).
"""
import pytest
import torch

from paper_2411_19702_amd import mi, synth
from tests.gpu_util import say

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(autouse=True)
def _clear_tuner():
    mi.mi_tuner_clear()
    yield
    mi.mi_tuner_clear()


@pytest.mark.parametrize("m,n,pitch,gram", [(20000, 700, 704, mi.MI_GRAM_INT8), (20000, 700, 700, mi.MI_GRAM_FP4),
                                            (2000, 8192, 8192, mi.MI_GRAM_FP4)])
def test_tuned_plan_is_used_and_results_unchanged(m, n, pitch, gram):
    """int8 for an aligned pitch; FP4 for a large shape and for a pitch that
    is not a multiple of 16 (its conversion replaces the repack)."""
    say(f"[tune] {m}x{n} pitch {pitch}")
    X = synth.generate(synth.spec_random(61, m, n, 0.0, 0.6, ldx=pitch, planted=4), device=DEV)[:, :n]
    before = mi.mi_all_pairs_ex(X)
    torch.cuda.synchronize()
    assert mi.mi_plan_ex(X)[2] == gram
    tile, splits, ms = mi.mi_tune(m, n, X.stride(0))
    assert tile in (mi.MI_TILE_128, mi.MI_TILE_256) and splits >= 1 and 0 < ms < 1e3
    assert mi.mi_plan_ex(X) == (tile, splits, gram)
    after = mi.mi_all_pairs_ex(X)
    torch.cuda.synchronize()
    assert torch.equal(before, after)


def test_tuner_file_round_trip(tmp_path):
    X = synth.generate(synth.spec_random(62, 2000, 8192, 0.0, 0.6), device=DEV)
    tile, splits, _ = mi.mi_tune(2000, 8192, 8192)
    path = str(tmp_path / "tuned.jsonl")
    mi.mi_tuner_save(path)
    text = open(path).read()
    assert '"fp4": 1' in text and f'"splits": {splits}' in text
    mi.mi_tuner_clear()
    mi.mi_tuner_load(path)
    assert mi.mi_plan_ex(X)[:2] == (tile, splits)


def _batch(count, m_range, n_range, seed=33):
    from tests.test_gpu_batched import _alloc, _problems
    specs = synth.specs_batched(seed=seed, count=count, m_range=m_range, n_range=n_range)
    Xs = [synth.generate(s, device=DEV) for s in specs]
    outs, n11s, css = _alloc(specs)
    return specs, Xs, (outs, n11s, css), _problems(Xs, outs, n11s, css)


def test_batch_tuner_entry_changes_the_persistent_plan_not_the_results(tmp_path):
    """A batch entry (loaded from a tuner file) changes the persistent mode's
    tiles and splits; the outputs stay bitwise those of the heuristic plan."""
    specs, Xs, bufs, probs = _batch(24, (500, 20000), (64, 900))
    say(f"[tune batched] {len(specs)} datasets: entry from a file")
    tiles0, splits0 = mi.mi_plan_batched(probs)
    mi.mi_all_pairs_batched(probs, mode=mi.MI_BATCH_PERSISTENT)
    torch.cuda.synchronize()
    ref = [[t.clone() for t in ts] for ts in bufs]
    # Tune, then rewrite the stored entry to a different plan and load it back.
    best, heur = mi.mi_tune_batched(probs)
    assert 0 < best <= heur < 1e4
    path = tmp_path / "tuned.jsonl"
    mi.mi_tuner_save(str(path))
    lines = [ln for ln in path.read_text().splitlines() if '"batch"' in ln]
    assert len(lines) == 1
    forced = tiles0.count(mi.MI_TILE_256) >= tiles0.count(mi.MI_TILE_128)
    tile_code = mi.MI_TILE_128 if forced else mi.MI_TILE_256
    sig = lines[0].split('"batch": "')[1].split('"')[0]
    path.write_text('{"batch": "%s", "tile": %d, "narrow": 512, "fdiv": 16, "ms": 1.0}\n' % (sig, tile_code))
    mi.mi_tuner_clear()
    assert mi.mi_plan_batched(probs) == (tiles0, splits0)       # cleared: the heuristic again
    mi.mi_tuner_load(str(path))
    tiles1, splits1 = mi.mi_plan_batched(probs)
    want = [mi.MI_TILE_128 if forced else mi.MI_TILE_256] * len(specs)
    assert tiles1 == want and tiles1 != tiles0
    assert sum(splits1) >= sum(splits0)                         # a finer split target
    for ts in bufs:
        for t in ts:
            t.fill_(-7)
    mi.mi_all_pairs_batched(probs, mode=mi.MI_BATCH_PERSISTENT)
    torch.cuda.synchronize()
    for k in range(3):
        for a, b in zip(bufs[k], ref[k]):
            assert torch.equal(a, b), "tuned persistent plan changed the outputs"


def test_batch_tuner_on_a_mixed_batch_is_no_slower_than_the_heuristic():
    specs, Xs, bufs, probs = _batch(48, (500, 50000), (64, 2048), seed=34)
    say(f"[tune batched] {len(specs)} datasets: tuned vs heuristic")
    best, heur = mi.mi_tune_batched(probs)
    assert best <= heur
    tiles, splits = mi.mi_plan_batched(probs)
    assert all(t in (mi.MI_TILE_128, mi.MI_TILE_256) for t in tiles) and all(s >= 1 for s in splits)
    mi.mi_all_pairs_batched(probs, mode=mi.MI_BATCH_PERSISTENT)
    torch.cuda.synchronize()
    from tests.test_gpu_batched import _run
    seq = _run(specs, Xs, mi.MI_BATCH_SEQUENTIAL)
    for k in range(3):
        for a, b in zip(bufs[k], seq[k]):
            assert torch.equal(a, b)
