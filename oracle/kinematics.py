"""Rigid revolving-plate kinematics (oracle; test infrastructure only).

Sec. 4.2.2 revolves a rigid wing at a fixed angle of attack alpha about a
vertical axis, with the rotation angle following Eq. (revolving_angle).  The
solid velocity of a point of a rigid wing is the frame velocity of
Eq. (relative_velocities) with no deformation velocity: u_s = Omega e_z x r.

Readings (listed in the design notes):
* the plate spans the radial axis from the rotation axis (root) to R, the
  chord is pitched about the mid-chord line with the leading edge up: in the
  wing frame at phi = 0 a point at span s and chord offset c sits at
  (s, c cos alpha, c sin alpha) from the axis point, and the plate moves +y;
* "ramp" law: Omega(t) = Omega (1 - cos(pi t / T_r)) / 2 for t < T_r, Omega
  after, phi its integral;  "exp" law: phi(t) = Omega (tau e^{-t/tau} + t - tau),
  Eq. (revolving_angle) scaled by Omega.

Pins (tests/test_oracle_kinematics.py): phi is the integral of Omega (checked by
quadrature), |x - axis| is preserved, v = Omega e_z x (x - axis) by finite
differences of x in time.
"""

import numpy as np

LAW_RAMP = 0
LAW_EXP = 1


def angle_and_rate(t, omega, t_ramp, law=LAW_RAMP):
    """Return (phi(t), dphi/dt(t))."""
    if law == LAW_RAMP:
        if t_ramp <= 0.0 or t >= t_ramp:
            phi0 = 0.5 * omega * max(t_ramp, 0.0)
            return phi0 + omega * (t - max(t_ramp, 0.0)), omega
        rate = 0.5 * omega * (1.0 - np.cos(np.pi * t / t_ramp))
        phi = 0.5 * omega * (t - (t_ramp / np.pi) * np.sin(np.pi * t / t_ramp))
        return phi, rate
    tau = t_ramp
    phi = omega * (tau * np.exp(-t / tau) + t - tau)
    rate = omega * (1.0 - np.exp(-t / tau))
    return phi, rate


def plate_pose(s, c, t, alpha, omega, t_ramp, axis_point, law=LAW_RAMP):
    """Vertex positions and velocities (nv, 3) of the rigid revolving plate at time t.

    ``s``, ``c``: span and chord coordinates of each vertex (chord measured from
    the mid-chord line); ``axis_point``: a point on the vertical rotation axis at
    the plate's mid-height.
    """
    s = np.asarray(s, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    phi, rate = angle_and_rate(t, omega, t_ramp, law)
    local = np.stack([s, c * np.cos(alpha), c * np.sin(alpha)], axis=1)
    cp, sp = np.cos(phi), np.sin(phi)
    rot = np.array([[cp, -sp, 0.0], [sp, cp, 0.0], [0.0, 0.0, 1.0]])
    rel = local @ rot.T
    x = np.asarray(axis_point, dtype=np.float64)[None, :] + rel
    v = np.stack([-rate * rel[:, 1], rate * rel[:, 0], np.zeros(len(s))], axis=1)
    return x, v


def plate_frame(t, alpha, omega, t_ramp, law=LAW_RAMP):
    """Wing frame of the revolving plate at time t: columns span, chord and
    normal directions, Rz(phi) applied to (1, 0, 0), (0, cos a, sin a) and
    (0, -sin a, cos a) (the pitched plate of plate_pose)."""
    phi, _ = angle_and_rate(t, omega, t_ramp, law)
    cp, sp = np.cos(phi), np.sin(phi)
    rot = np.array([[cp, -sp, 0.0], [sp, cp, 0.0], [0.0, 0.0, 1.0]])
    pitch = np.array([[1.0, 0.0, 0.0], [0.0, np.cos(alpha), -np.sin(alpha)], [0.0, np.sin(alpha), np.cos(alpha)]])
    return rot @ pitch


def motion_direction(phi):
    """Unit vector of the plate's motion at angle phi: e_z x e_span."""
    return np.array([-np.sin(phi), np.cos(phi), 0.0])
