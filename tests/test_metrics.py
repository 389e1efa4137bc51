"""Error metric of the paper (Section IV-F) on hand-checkable cases."""
import numpy as np

from paper_2609_24294_amd import metrics


def test_block_errors_by_hand():
    x = np.ones((4, 4, 8))
    xh = x.copy()
    xh[0, 0, 0] = 2.0          # block 0: one value off by 1 -> sqrt(1 / 64)
    xh[:, :, 4:] *= 1.5        # block 1: every value off by 0.5 -> 0.5
    e = metrics.block_relative_errors(x, xh)
    assert np.allclose(e, [1 / 8, 0.5])


def test_partial_blocks_use_real_values_only():
    x = np.arange(1.0, 1.0 + 5 * 3 * 6).reshape(5, 3, 6)
    xh = x * (1 + 1e-3)
    e = metrics.block_relative_errors(x, xh)
    assert e.shape == (2 * 1 * 2,) and np.allclose(e, 1e-3)


def test_zero_blocks_skipped_and_report():
    x = np.zeros((4, 4, 8))
    x[:, :, 4:] = 3.0
    e = metrics.block_relative_errors(x, x)
    assert e.shape == (1,) and e[0] == 0
    r = metrics.error_report(x, x + (x != 0) * 0.03)
    assert np.isclose(r["block_mean"], 0.01) and np.isclose(r["global"], 0.01)
    assert np.isclose(r["point_max"], 0.01)


def test_bytes_reduction():
    assert metrics.bytes_reduction(56536064, 902720 * 8 * 16) == 4 * 56536064 / (902720 * 128)
    assert abs(metrics.bytes_reduction(56536064, 902720 * 8 * 16) - 1.957) < 1e-3
