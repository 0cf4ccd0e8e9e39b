"""The block-size and launch autotuner on a small problem: it times real passes for each
candidate, writes its choice to the cache, answers from the cache the second time, and the
epoch at the chosen settings (a different b is a different trajectory) matches the oracle."""
import copy
import json

import pytest

import synth
from paper_2110_14044_amd import autotune
from tests.gpu_util import need_gpu, say
from tests.test_gpu_parity import _epoch_check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def test_autotune_choice_is_cached_and_matches_the_oracle(tmp_path):
    p = synth.small_problem(600, 3000, 400, 60_000, 128, 64, zipf_s=0.8, std=0.1)
    cache = tmp_path / "tune.json"
    r = autotune.tune(p, candidates=(32, 64, 128), cache_path=str(cache), log=say, min_gain=0.0)
    say(f"tuned: b={r['block']} deal={r['deal']} seg_len={r['seg_len']} ({r['epoch_ms']:.2f} ms estimated)")
    assert r["block"] in (32, 64, 128) and r["deal"] in ("auto",) + autotune.DEALS
    assert r["seg_len"] in autotune.SEG_LENS and r["gram_split"] in autotune.GRAM_SPLITS
    assert {t["gram_split"] for t in r["trials"]} == set(autotune.GRAM_SPLITS)
    blocks = {t["block"] for t in r["trials"]}
    assert blocks == {32, 64, 128}
    assert r["epoch_ms"] == min(t["epoch_ms"] for t in r["trials"])
    stored = json.loads(cache.read_text())
    assert stored[r["key"]]["block"] == r["block"]
    again = autotune.tune(p, candidates=(32, 64, 128), cache_path=str(cache), min_gain=0.0)
    assert again == stored[r["key"]]
    q = copy.copy(p)
    q.block = r["block"]
    _epoch_check(q, 1, 1e-4, 1e-6, deal=r["deal"], seg_len=r["seg_len"], gram_split=r["gram_split"])
