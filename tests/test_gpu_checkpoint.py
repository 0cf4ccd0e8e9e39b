"""Resume from a checkpoint and per-epoch metrics records, through the C ABI.

A run stopped after two epochs, saved, and resumed in a new context on the same device for two
more must give the W, H and per-epoch losses of four uninterrupted epochs bit for bit (the
kernels are deterministic and the state at an epoch boundary is W, H and the configuration).
"""
import json

import numpy as np
import pytest

import synth
from paper_2110_14044_amd import Trainer, binding
from tests.gpu_util import host, need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


CASES = [
    # name, problem, trainer options
    ("b | d, eager", lambda: synth.small_problem(400, 2000, 300, 40_000, 64, 32, labels=True, zipf_s=0.9), {}),
    ("ragged block, segments, graph",
     lambda: synth.small_problem(401, 2000, 120, 40_000, 48, 32, labels=True, zipf_s=0.8),
     {"graph": True, "seg_len": 256}),
    ("bfloat16", lambda: synth.small_problem(402, 1500, 200, 30_000, 64, 64), {"precision": binding.IALS_PREC_BF16}),
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_resume_repeats_the_uninterrupted_run(tmp_path, name, make, kw):
    p = make()
    a = Trainer(p, **kw)
    rec_a = a.fit(4, metrics_path=str(tmp_path / "a.jsonl"))
    Wa, Ha = host(a.W), host(a.H)
    a.close()

    b = Trainer(p, **kw)
    b.fit(2)
    ck = str(tmp_path / "ck.npz")
    b.save_checkpoint(ck)
    b.close()
    c = Trainer.resume(ck, p, **kw)
    assert c.epochs_done == 2
    rec_c = c.fit(2)
    Wc, Hc = host(c.W), host(c.H)
    c.close()
    say(f"{name}: losses {[r['loss'] for r in rec_a]} resumed {[r['loss'] for r in rec_c]}")
    assert np.array_equal(Wa, Wc) and np.array_equal(Ha, Hc)
    assert [r["loss"] for r in rec_a[2:]] == [r["loss"] for r in rec_c]
    assert [r["epoch"] for r in rec_c] == [3, 4]
    lines = [json.loads(x) for x in open(tmp_path / "a.jsonl")]
    assert [r["epoch"] for r in lines] == [1, 2, 3, 4]
    assert [r["loss"] for r in lines] == [r["loss"] for r in rec_a]


def test_resume_refuses_other_settings(tmp_path):
    p = synth.small_problem(403, 500, 100, 5000, 32, 16)
    a = Trainer(p)
    a.fit(1, with_loss=False)
    ck = str(tmp_path / "ck.npz")
    a.save_checkpoint(ck)
    a.close()
    with pytest.raises(ValueError, match="precision"):
        Trainer.resume(ck, p, precision=binding.IALS_PREC_BF16)


def test_metrics_records(tmp_path):
    p = synth.small_problem(404, 3000, 200, 60_000, 64, 32, zipf_s=0.9)
    tr = Trainer(p, chol_fallback_ratio=1.0)  # every row redone in float64: the count is known
    seen = []
    recs = tr.fit(2, metrics_path=str(tmp_path / "m.jsonl"), profile=True,
                  extra=lambda t, e: seen.append(e) or {"tag": e})
    L_now = tr.loss()[0]
    tr.close()
    say(f"metrics: {json.dumps(recs[-1])[:400]}")
    assert seen == [1, 2] and [r["tag"] for r in recs] == [1, 2]
    assert recs[-1]["loss"] == L_now
    for r in recs:
        assert r["epoch_s"] > 0 and r["nnz_b_per_s"] == pytest.approx(2 * p.nnz * p.dim / r["epoch_s"])
        # tau = 1 sends every row of every pass to the float64 path: (U + I) rows per block
        assert r["fallback_rows"] == (p.num_users + p.num_items) * (p.dim // p.block)
        assert r["kernels"]["rows_user"]["launches"] >= 1 and r["kernels"]["predict"]["launches"] >= 1
    assert len(open(tmp_path / "m.jsonl").read().splitlines()) == 2
