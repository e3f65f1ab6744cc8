"""Staggered fluid-structure coupling of a mass-spring wing revolving about the
vertical axis (Sec. 4.1, staggered scheme paragraph; wing model of Sec. 2).

One coupled step n (state: fluid at t^n, wing q^n = [x^n, v^n]):
 1. the fluid step uses the mask and solid velocity of the wing at t^n
    (fsi_set_wing, fsi_step) and yields the force F^n;
 2. the pressure of that step gives the vertex loads (fsi_get_pressure_loads;
    reading: the structure is advanced with p^n, so no second nonlinear
    evaluation is needed per step);
 3. the wing advances to t^{n+1} by the BDF2/Newton step of the native
    mass-spring solver (fsi_ms_step) with those loads, its root vertices
    clamped to the rigid kinematics at t^{n+1} and the bending angles measured
    in the wing frame at t^{n+1} (fsi_plate_frame).
The structure is solved in the inertial frame: positions and velocities are
those of the fluid's frame, so u_s needs no frame transformation.

This module only sequences library calls; every computation runs in libfsi.
"""

import numpy as np

from . import fsi


class FlexibleWingFSI:
    """A wing (synth-style dict: span_coord, chord_coord, tri, ext_ij, ext_k,
    clamped, density) with bending springs bend_ijk / bend_kb / bend_axis,
    driven at its root by the revolving-plate kinematics ``kin`` (alpha, omega,
    t_ramp, axis_point, law)."""

    def __init__(self, solver, wing, bend_ijk, bend_kb, bend_axis, kin, tol=1e-10, max_iter=30):
        self.s = solver
        self.w = wing
        self.kin = kin
        self.tol = tol
        self.max_iter = max_iter
        self.tri = np.asarray(wing["tri"], dtype=np.int32)
        self.clamped = np.asarray(wing["clamped"], dtype=np.int32)
        x0, v0 = self._root_pose(0.0, None)
        mass = fsi.lumped_masses(x0, self.tri, wing["density"])
        ms = fsi.MassSpring(mass)
        ext = np.asarray(wing["ext_ij"])
        ms.add_extension(ext, wing["ext_k"], np.ones(len(ext)))
        ms.add_bending(bend_ijk, bend_kb, None, bend_axis)
        ms.set_clamped(self.clamped)
        ms.set_state(x0, v0)
        ms.set_rest(self._frame(0.0))
        self.ms = ms
        self.t = 0.0
        self.iters = []

    def _root_pose(self, t, idx):
        k = self.kin
        s = np.asarray(self.w["span_coord"])
        c = np.asarray(self.w["chord_coord"])
        if idx is not None:
            s, c = s[idx], c[idx]
        x, v, _ = fsi.plate_pose(s, c, t, k["alpha"], k["omega"], k["t_ramp"], k["axis_point"], k.get("law", 0))
        return x, v

    def _frame(self, t):
        k = self.kin
        return fsi.plate_frame(t, k["alpha"], k["omega"], k["t_ramp"], k.get("law", 0))

    def step(self, dt):
        """One coupled step of size dt; returns the fluid force F^n."""
        x, v = self.ms.state()
        self.s.set_wing(x, v, self.tri)
        self.s.step(dt)
        F = self.s.info()["F"]
        loads, _ = self.s.pressure_loads()
        t1 = self.t + dt
        xc, vc = self._root_pose(t1, self.clamped)
        self.iters.append(self.ms.step(dt, self._frame(t1), loads, xc, vc, self.tol, self.max_iter))
        self.t = t1
        return F

    def state(self):
        return self.ms.state()
