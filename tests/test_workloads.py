"""Synthetic workloads against what the paper prints about them (CPU)."""
import os

import numpy as np
import pytest

from paper_1409_0074_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_sec51_workload_matches_the_paper():
    """The Sec. 5.1 design, response and predictive grid: sizes and the
    mean-only in-sample RMSE printed beside Table 1 (a dropped term or a wrong
    sign in w, or a misplaced grid, moves it off 0.2085)."""
    vals = {}
    with open(os.path.join(GOLDEN, "sec51_values.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v, tol = line.split()
                vals[k] = (float(v), float(tol))
    w = W.paper2d()
    assert w.X.shape == (int(vals["N"][0]), 2) and w.XX.shape == (int(vals["M"][0]), 2)
    rmse = float(np.sqrt(np.mean((w.y - w.y.mean()) ** 2)))
    v, tol = vals["mean_only_rmse"]
    assert abs(rmse - v) <= tol
    # the grid spans [-2, 2]^2 in steps of 0.02; no predictive location is on it
    assert w.X.min() == -2.0 and w.X.max() == pytest.approx(2.0, abs=1e-12)
    steps = (w.XX + 2.0) / 0.02
    assert np.all(np.abs(steps - np.round(steps)) > 0.4)


def test_sec51_w_special_values():
    """w at points where the sine term vanishes reduces to the two Gaussian
    bumps."""
    x = np.array([-0.1, -0.1 + np.pi / 8])
    ref = np.exp(-((x - 1.0) ** 2)) + np.exp(-0.8 * (x + 1.0) ** 2)
    assert W.w_sec51(x) == pytest.approx(ref, abs=1e-15)
    assert W.f_sec51(np.array([[1.0, 1.0]]))[0] == pytest.approx(
        -(1.0 + np.exp(-3.2) - 0.05 * np.sin(8.8)) ** 2, rel=1e-15)
