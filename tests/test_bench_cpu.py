"""Host-side pieces of bench.py that its JSON line depends on, checked without a GPU."""
import numpy as np
import pytest

import bench
import synth


def test_traffic_is_reported_only_for_the_profiled_kernel_and_source(tmp_path, monkeypatch):
    # a counter summary in the committed format, for a source file of known content
    src = tmp_path / "paper_2110_14044_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "k.hip").write_text("kernel source\n")
    import hashlib
    h = hashlib.sha256(b"kernel source\n").hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic_rows_user_move_msd_like.txt").write_text(
        "# comment\nkernel=rows_user_move\nworkload=msd_like\nblock=64\nprecision=fp32\nseg_len=512\nsource=k.hip\n"
        f"source_sha256={h}\nfetch_kib=1000\nwrite_kib=100\nfetch_scale=2.0\nwrite_scale=1.0\n\n"
        "kernel=rows_user_move\nworkload=msd_like\nblock=64\nprecision=fp32\nseg_len=2048\nsource=k.hip\n"
        f"source_sha256={h}\nfetch_kib=3000\nwrite_kib=300\nfetch_scale=2.0\nwrite_scale=1.0\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # FETCH_SIZE x 2 + WRITE_SIZE x 1, in KiB
    assert bench.measured_traffic("rows_user_move", "msd_like", 64, "fp32") == (2000 + 100) * 1024
    assert bench.measured_traffic("rows_user", "msd_like", 64, "fp32") is None
    assert bench.measured_traffic("rows_user_move", "msd_like", 32, "fp32") is None
    assert bench.measured_traffic("rows_user_move", "msd_like", 64, "bf16") is None
    assert bench.measured_traffic("rows_user_move", "msd_like", 64, "fp32", 2048) == (6000 + 300) * 1024
    assert bench.measured_traffic("rows_user_move", "msd_like", 64, "fp32", 1024) is None
    assert bench.measured_traffic("rows_user_move", "msd_like", 64, "fp32", 512) == (2000 + 100) * 1024
    (src / "k.hip").write_text("kernel source, changed\n")
    assert bench.measured_traffic("rows_user_move", "msd_like", 64, "fp32") is None


def test_row_work_counts():
    # rows of 3, 0 and 600 observations at b = 16 with segments of 512: the long row's
    # observations belong to the segment kernel, every row is solved
    b = 16
    flops, bytes_ = bench.rows_work(np.array([3, 0, 600]), b, 512)
    per_obs = 2 * b * b + 4 * b       # rank-1 Hessian update, gradient and cache work
    per_row = b ** 3 / 3 + 2 * b * b  # factorisation and the two triangular solves
    assert flops == pytest.approx(3 * per_obs + 3 * per_row, rel=1e-12)
    assert bytes_ == pytest.approx(3 * (4 * b + 12) + 3 * 12 * b, rel=1e-12)


def test_epoch_work_matches_the_per_epoch_totals():
    # MSD-shaped at b = 64: Hessian 2|S|b^2 per pass (2 d/b passes), Gramian + dense term
    # 2 (U + I) d^2 each per epoch, solves (U + I) d b^2 / 3 (+ the triangular solves)
    wl = synth.workload("msd_like")
    p = synth.Problem(wl.num_users, wl.num_items, 2048, 64, 0.1, 0.05, np.zeros(wl.nnz, np.int32),
                      np.zeros(wl.nnz, np.int32), None, None, None, None, "msd_like")
    work = bench.epoch_work(p)
    tot = {}
    for name, fl, by, _ in work:
        k = name.split("_")[0]
        tot[k] = tot.get(k, 0.0) + fl
    S, U, I, d, b = wl.nnz, wl.num_users, wl.num_items, 2048, 64
    assert tot["hessian"] == pytest.approx(2 * (d // b) * S * (2 * b * b + 4 * b))
    assert tot["gram"] + tot["dense"] == pytest.approx(4 * (U + I) * d * d)
    assert tot["solve"] == pytest.approx((U + I) * (d // b) * (b ** 3 / 3 + 2 * b * b))
    assert tot["predict"] == pytest.approx(2 * S * d)
    floor, parts = bench.epoch_floor(p, "fp32")
    # the Hessian alone at the float32 matrix peak: 2|S| d (2b + 4) / 157.3 TFLOP/s, about 113 ms
    assert parts["hessian"] == pytest.approx(2 * (d // b) * S * (2 * b * b + 4 * b) / 157.3e12, rel=1e-9)
    assert 0.2 < floor < 0.3
    # with bfloat16 operands the gathered Hessian is bound by its float32 gathers (b floats, id and
    # cache entry per observation) at 8 TB/s
    floor16, parts16 = bench.epoch_floor(p, "bf16")
    assert parts16["hessian"] == pytest.approx(2 * (d // b) * S * (4 * b + 12) / 8e12, rel=1e-9)
    assert floor16 < floor


def test_segment_rate_against_both_rooflines():
    # 3,000 users x 120 items, 60k observations: most item rows are longer than 512, so the
    # item segments carry most observations.  With a made-up launch time the segment entry
    # must report the gather bytes against HBM and the 2b^2 + 4b FLOP per observation against
    # the matrix peak, and name the matrix cores as the binding roofline at b = 64.
    p = synth.small_problem(5, 3000, 120, 60_000, 128, 64, zipf_s=0.8)
    li = np.bincount(p.item, minlength=p.num_items)
    seg_nnz = int(li[li > 512].sum())
    assert seg_nnz > 30_000
    kern = {name: {"ms_per_epoch": 1.0, "launches": 2, "avg_ms": 0.5}
            for name in ("rows_user", "rows_user_move", "rows_item", "seg_item", "gram_item", "dense_user",
                         "predict")}
    kern["rows_user_move"]["ms_per_epoch"] = 2.0
    kern["seg_item"]["avg_ms"] = 0.002  # large rates, so the rounding to 0.01 does not matter
    roof, rates, eroof = bench.rooflines(p, "fp32", kern, 512, 0.01)
    s = rates["seg_item"]
    t = 0.002e-3
    assert s["achieved"] == pytest.approx(seg_nnz * (4 * 64 + 12) / t / 1e9, rel=1e-3)
    assert s["flop_achieved"] == pytest.approx(seg_nnz * (2 * 64 * 64 + 4 * 64) / t / 1e12, rel=1e-3)
    assert s["flop_frac"] == pytest.approx(s["flop_achieved"] / 157.3, rel=1e-3)
    assert s["bound"] == "mfma"
    # at b = 4 the same observations gather 28 bytes for 48 FLOP: HBM binds
    p4 = synth.small_problem(5, 3000, 120, 60_000, 16, 4, zipf_s=0.8)
    _, rates4, _ = bench.rooflines(p4, "fp32", kern, 512, 0.01)
    assert rates4["seg_item"]["bound"] == "hbm"
