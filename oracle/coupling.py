"""Staggered fluid-structure coupling (oracle; test infrastructure only).

Sec. 4.1 (staggered scheme paragraph) with the wing model of Sec. 2.  One
coupled step n (fluid at t^n, wing q^n = [x^n, v^n]):
 1. the fluid advances u^n -> u^{n+1} with the mask and solid velocity of the
    wing at t^n (giving the force F^n);
 2. the pressure that loads the wing is
    - order "lagged" (default reading): p^n, the pressure of the nonlinear
      term of that fluid step (u^n, chi^n): no second nonlinear evaluation;
    - order "paper": p^{n+1}, computed from u^{n+1} (with the mask of the
      wing still at t^n, the only one known then), as the paragraph states;
 3. the wing advances to t^{n+1} by the BDF2 step of oracle.structure with
    the loads of that pressure on the wing at x^n, root vertices clamped to
    the rigid kinematics at t^{n+1}, bending angles in the wing frame at
    t^{n+1}.
Masses are lumped from the triangle areas with a uniform areal density, or
given per vertex (the functional wing of Sec. 2.2: vein masses spread over the
vein's vertices, the membrane mass law elsewhere); the wing rests in its
initial configuration (frame at t = 0).

Pins (tests/test_oracle_coupling.py): with a prescribed pressure field linear
in space and in time, a free vertex without springs follows the closed-form
ballistic BDF2 recurrence with the load of p^n (lagged) or p^{n+1} (paper),
clamped vertices sit at the pose of t^{n+1} and the fluid sees the wing of
t^n; the implicit-Euler residual of a bending-spring wing vanishes only with
the frame of t^{n+1}; a wing clamped at every vertex reproduces the rigid
revolving-plate fluid run bit for bit.
"""

import numpy as np

from . import kinematics, pressure, structure
from .ns import OracleNS

ORDERS = ("lagged", "paper")


class CoupledOracle:
    def __init__(self, n, L, nu, eta, tw, h, profile, wing, bend_ijk, bend_kb, bend_axis, kin, tol=1e-12,
                 order="lagged"):
        if order not in ORDERS:
            raise ValueError("order must be one of %s" % (ORDERS,))
        self.fluid = OracleNS(n, L, nu, eta, tw, h, profile)
        self.L = L
        self.d = tw + h
        self.w = wing
        self.kin = kin
        self.tol = tol
        self.order = order
        self.tri = np.asarray(wing["tri"])
        self.clamped = np.asarray(wing["clamped"])
        x0, v0 = self._root_pose(0.0, None)
        # masses: given per vertex (functional wing model), else lumped from the
        # triangle areas with a uniform areal density
        mass = (np.asarray(wing["mass"], dtype=np.float64) if wing.get("mass") is not None
                else structure.lumped_masses(x0, self.tri, wing["density"]))
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

    def step(self, dt=None, cfl=None, c_eta=None, dt_max=None):
        """One coupled step of size dt, or (dt None) of the fluid's adaptive dt
        (CFL and penalization rule at t^n), which the structure step then uses."""
        x, v = self.q
        self.fluid.set_wing(x, v, self.tri)
        # diagnostics of the fluid step
        self.last = (self.fluid.step(dt=dt) if dt is not None
                     else self.fluid.step(cfl=cfl, c_eta=c_eta, dt_max=dt_max))
        if dt is None:
            dt = self.last["dt"]
        F = self.last["F"]
        if self.order == "paper":
            # p^{n+1} from u^{n+1}; the wing (and so the mask) is still at t^n
            self.fluid.nonlinear(*self.fluid.combined_mask())
        loads, _ = pressure.wing_loads(self.fluid.p_last, self.L, x, self.tri, self.d)
        t1 = self.t + dt
        xc, vc = self._root_pose(t1, self.clamped)
        q_new, _ = structure.bdf2_step(self.net, self.q, self.q_prev, dt, self.dt_prev, self._frame(t1), loads,
                                       clamp_x=xc, clamp_v=vc, tol=self.tol)
        self.q_prev, self.q, self.dt_prev, self.t = self.q, q_new, dt, t1
        return F
