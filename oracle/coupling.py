"""Staggered fluid-structure coupling (oracle; test infrastructure only).

Sec. 4.1 (staggered scheme paragraph) with the wing model of Sec. 2.  One
coupled step n: the fluid advances with the mask and solid velocity of the
wing at t^n (giving F^n and p^n); the wing advances to t^{n+1} by the BDF2
step of oracle.structure with the pressure loads of p^n (reading: lagged
pressure), root vertices clamped to the rigid kinematics at t^{n+1}, bending
angles in the wing frame at t^{n+1}.  Masses are lumped from the triangle
areas; the wing rests in its initial configuration (frame at t = 0).
"""

import numpy as np

from . import kinematics, pressure, structure
from .ns import OracleNS


class CoupledOracle:
    def __init__(self, n, L, nu, eta, tw, h, profile, wing, bend_ijk, bend_kb, bend_axis, kin, tol=1e-12):
        self.fluid = OracleNS(n, L, nu, eta, tw, h, profile)
        self.L = L
        self.d = tw + h
        self.w = wing
        self.kin = kin
        self.tol = tol
        self.tri = np.asarray(wing["tri"])
        self.clamped = np.asarray(wing["clamped"])
        x0, v0 = self._root_pose(0.0, None)
        mass = structure.lumped_masses(x0, self.tri, wing["density"])
        self.net = structure.rest_network(mass, x0, wing["ext_ij"], wing["ext_k"], bend_ijk, bend_kb, bend_axis,
                                          self.clamped, self._frame(0.0))
        self.q = np.stack([x0, v0])
        self.q_prev = None
        self.dt_prev = None
        self.t = 0.0

    def _root_pose(self, t, idx):
        k = self.kin
        s = np.asarray(self.w["span_coord"])
        c = np.asarray(self.w["chord_coord"])
        if idx is not None:
            s, c = s[idx], c[idx]
        return kinematics.plate_pose(s, c, t, k["alpha"], k["omega"], k["t_ramp"], k["axis_point"], k.get("law", 0))

    def _frame(self, t):
        k = self.kin
        return kinematics.plate_frame(t, k["alpha"], k["omega"], k["t_ramp"], k.get("law", 0))

    def step(self, dt):
        x, v = self.q
        self.fluid.set_wing(x, v, self.tri)
        F = self.fluid.step(dt=dt)["F"]
        loads, _ = pressure.wing_loads(self.fluid.p_last, self.L, x, self.tri, self.d)
        t1 = self.t + dt
        xc, vc = self._root_pose(t1, self.clamped)
        q_new, _ = structure.bdf2_step(self.net, self.q, self.q_prev, dt, self.dt_prev, self._frame(t1), loads,
                                       clamp_x=xc, clamp_v=vc, tol=self.tol)
        self.q_prev, self.q, self.dt_prev, self.t = self.q, q_new, dt, t1
        return F
