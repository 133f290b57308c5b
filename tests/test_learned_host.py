"""Host-side logic of the learned-theta part (no GPU needed)."""
import numpy as np
import pytest

LT = pytest.importorskip("paper_1509_07370_amd.learned_theta")


def test_labels_envelope():
    errs = np.array([[1e-5, 1e-5, 2e-3], [2e-4, 5e-3, 3e-3], [9e-4, 1e-4, 4e-3], [2e-3, 1e-4, 5e-3]])
    th = np.array([0.2, 0.4, 0.6, 0.8])
    lab = LT.labels_from_errors(errs, 1e-3, th)
    assert lab.tolist() == pytest.approx([0.6, 0.2, 0.2])


def test_theta_grid():
    assert LT.THETA_GRID[0] == 0.2 and LT.THETA_GRID[-1] == 1.0 and len(LT.THETA_GRID) == 17
