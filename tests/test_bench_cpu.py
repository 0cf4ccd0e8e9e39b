"""Host-side pieces of bench.py that its JSON line depends on, checked without a GPU."""
import numpy as np
import pytest

import bench


def test_traffic_is_reported_only_for_the_profiled_kernel_and_source():
    t = bench.measured_traffic("rows_user_move", "ml20m_like", 64, "fp32")
    # FETCH_SIZE x 2 + WRITE_SIZE x 1 (KiB) of the committed counter summary: about 1.2 GB
    assert t is not None and 1.0e9 < t < 1.5e9
    assert bench.measured_traffic("rows_user", "ml20m_like", 64, "fp32") is None
    assert bench.measured_traffic("rows_user_move", "msd_like", 64, "fp32") is None
    assert bench.measured_traffic("rows_user_move", "ml20m_like", 64, "bf16") is None


@pytest.mark.parametrize("trans", [0.0, 1.0])
def test_row_work_counts(trans):
    # rows of 3, 0 and 600 observations at b = 16 with segments of 512: the long row's
    # observations belong to the segment kernel, every row is solved
    b = 16
    flops, bytes_ = bench.rows_work(np.array([3, 0, 600]), b, trans, 512)
    per_obs = 2 * b * b + 4 * b + trans * 2 * b  # rank-1 update, gradient, prediction (old block)
    per_row = b ** 3 / 3 + 2 * b * b             # LDL^T factorisation and the two triangular solves
    assert flops == pytest.approx(3 * per_obs + 3 * per_row, rel=1e-12)
    per_obs_bytes = 4 * b + 8 + trans * (4 * b + 4)
    per_row_bytes = 12 * b + trans * 4 * b
    assert bytes_ == pytest.approx(3 * per_obs_bytes + 3 * per_row_bytes, rel=1e-12)
