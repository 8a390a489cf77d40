"""Host-side logic of the package: recall (Eq. recall@k)."""
import numpy as np
import pytest


def test_recall_definition():
    from paper_2307_10479_amd import metrics
    gt = np.array([[1, 2, 3, 4], [5, 6, 7, 8]])
    got = np.array([[4, 3, 9, 9], [5, 6, 7, 8]])
    assert metrics.recall_at_k(got, gt, 4) == pytest.approx((2 / 4 + 1) / 2)
    assert metrics.recall_at_k(got, gt, 2) == pytest.approx((0 + 1) / 2)


