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


def test_estimated_rms_uses_the_next_tabulated_theta():
    th = np.array([0.2, 0.25, 0.3])
    e = np.array([[1e-5, 1e-5], [1e-4, 2e-5], [1e-3, 3e-5]], np.float32)
    assert LT.estimated_rms(e, np.array([0.2, 0.25]), th) == pytest.approx(np.sqrt((1e-10 + 4e-10) / 2), rel=1e-6)
    assert LT.estimated_rms(e, np.array([0.21, 0.3]), th) == pytest.approx(np.sqrt((1e-8 + 9e-10) / 2), rel=1e-6)
