"""Pins of the oracle's SE(3) exponential (the pose update T <- Exp(xi) T)
against the matrix exponential, a hand-derived screw motion, and group laws."""
import json
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import se3

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _twist(xi):
    X = np.zeros((4, 4))
    X[:3, :3] = se3.hat(xi[:3])
    X[:3, 3] = xi[3:]
    return X


@pytest.mark.parametrize("scale", [0.0, 1e-9, 1e-5, 9.9e-5, 1.01e-4, 1e-2, 0.5, 2.0, 3.0])
def test_exp_matches_expm(scale):
    rng = np.random.default_rng(int(scale * 1e6) % 1000)
    for _ in range(20):
        xi = rng.normal(size=6)
        xi[:3] *= scale / max(np.linalg.norm(xi[:3]), 1e-300)
        T = se3.exp_se3(xi)
        E = scipy.linalg.expm(_twist(xi))
        assert np.abs(T - E).max() < 1e-12


def test_golden_quarter_turn():
    g = json.load(open(os.path.join(GOLD, "exp_quarter_turn.json")))
    T = se3.exp_se3(np.array(g["xi"]))
    assert np.abs(T[:3, :3] - np.array(g["expected_R"])).max() < 1e-15
    assert np.abs(T[:3, 3] - np.array(g["expected_t"])).max() < 1e-15


def test_group_laws():
    rng = np.random.default_rng(0)
    for _ in range(50):
        xi = rng.normal(size=6)
        T = se3.exp_se3(xi)
        Ti = se3.exp_se3(-xi)
        assert np.abs(T @ Ti - np.eye(4)).max() < 1e-12
        R = T[:3, :3]
        assert np.abs(R.T @ R - np.eye(3)).max() < 1e-14
        assert abs(np.linalg.det(R) - 1) < 1e-14
        assert np.abs(se3.inv(T) - Ti).max() < 1e-12


def test_log_inverts_exp():
    rng = np.random.default_rng(1)
    for ang in [1e-9, 1e-4, 0.3, 2.0, np.pi - 1e-3]:
        w = rng.normal(size=3)
        w *= ang / np.linalg.norm(w)
        R = se3.exp_se3(np.concatenate([w, np.zeros(3)]))[:3, :3]
        assert np.abs(se3.log_so3(R) - w).max() < 1e-9


def test_pose_error():
    T = se3.exp_se3(np.array([0, 0, 0.01, 0.003, 0, 0.004]))
    dr, dt = se3.pose_error(np.eye(4), T)
    assert abs(dr - 0.01) < 1e-15
    assert abs(dt - np.linalg.norm(T[:3, 3])) < 1e-15
