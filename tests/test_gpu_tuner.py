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


@pytest.mark.parametrize("m,n,gram", [(20000, 700, mi.MI_GRAM_INT8), (2000, 8192, mi.MI_GRAM_FP4)])
def test_tuned_plan_is_used_and_results_unchanged(m, n, gram):
    say(f"[tune] {m}x{n}")
    X = synth.generate(synth.spec_random(61, m, n, 0.0, 0.6, planted=4), device=DEV)
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
