"""Pins of the oracle's rigid revolving-plate kinematics (Sec. 4.2.2, Eq. (revolving_angle))."""

import numpy as np
import pytest

from oracle import kinematics as kin
import synth


@pytest.mark.parametrize("law", [kin.LAW_RAMP, kin.LAW_EXP])
def test_angle_is_integral_of_rate(law):
    om, tr = 2 * np.pi, 0.4
    ts = np.linspace(0.0, 1.0, 20001)
    rates = np.array([kin.angle_and_rate(t, om, tr, law)[1] for t in ts])
    integral = np.concatenate([[0.0], np.cumsum(0.5 * (rates[1:] + rates[:-1]) * np.diff(ts))])
    phis = np.array([kin.angle_and_rate(t, om, tr, law)[0] for t in ts])
    assert np.max(np.abs(phis - integral)) < 1e-7
    assert phis[0] == pytest.approx(0.0, abs=1e-15)


def test_ramp_sweeps_a_fifth_of_a_revolution():
    phi, rate = kin.angle_and_rate(0.4, 2 * np.pi, 0.4)
    assert phi == pytest.approx(0.2 * 2 * np.pi, rel=1e-15)
    assert rate == 2 * np.pi


def test_pose_is_rigid_and_velocity_is_time_derivative():
    cfg = synth.revolving_plate()
    s, c = cfg["span_coord"], cfg["chord_coord"]
    args = (cfg["alpha"], cfg["omega"], cfg["t_ramp"], cfg["axis_point"])
    for t in (0.05, 0.3, 0.7):
        x, v = kin.plate_pose(s, c, t, *args)
        e = 1e-6
        xp, _ = kin.plate_pose(s, c, t + e, *args)
        xm, _ = kin.plate_pose(s, c, t - e, *args)
        assert np.max(np.abs((xp - xm) / (2 * e) - v)) < 1e-6
        rel = x - np.asarray(cfg["axis_point"])
        assert np.allclose(np.hypot(rel[:, 0], rel[:, 1]), np.hypot(s, c * np.cos(cfg["alpha"])))
        assert np.allclose(rel[:, 2], c * np.sin(cfg["alpha"]))
    x0, v0 = kin.plate_pose(s, c, 0.0, *args)
    assert np.all(v0 == 0.0)


def test_plate_frame_maps_local_coordinates_to_the_pose():
    rng = np.random.default_rng(3)
    s, c = rng.random(10) * 3.0, rng.random(10) - 0.5
    axis = np.array([6.0, 6.0, 6.0])
    for t in (0.0, 0.13, 0.9):
        F = kin.plate_frame(t, 0.6, 2 * np.pi, 0.4)
        x, _ = kin.plate_pose(s, c, t, 0.6, 2 * np.pi, 0.4, axis)
        assert np.allclose(x, axis + np.stack([s, c, 0 * s], 1) @ F.T, atol=1e-14)
        assert np.allclose(F.T @ F, np.eye(3), atol=1e-15) and np.linalg.det(F) > 0
