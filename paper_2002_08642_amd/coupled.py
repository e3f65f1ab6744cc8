"""Staggered fluid-structure coupling of a mass-spring wing revolving about the
vertical axis (Sec. 4.1, staggered scheme paragraph; wing model of Sec. 2).

One coupled step n (state: fluid at t^n, wing q^n = [x^n, v^n]):
 1. the fluid step uses the mask and solid velocity of the wing at t^n
    (fsi_set_wing, fsi_step) and yields the force F^n;
 2. the pressure gives the vertex loads (fsi_get_pressure_loads): order
    "lagged" (default reading) uses p^n of that step, so no second nonlinear
    evaluation is needed per step; order "paper" first replaces it by
    p^{n+1} of the new velocity (fsi_eval_pressure, the wing still at t^n),
    as the staggered-scheme paragraph orders it;
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

    def __init__(self, solver, wing, bend_ijk, bend_kb, bend_axis, kin, tol=1e-10, max_iter=30, order="lagged"):
        if order not in ("lagged", "paper"):
            raise ValueError("order must be 'lagged' or 'paper'")
        self.order = order
        self.s = solver
        self.w = wing
        self.kin = kin
        self.tol = tol
        self.max_iter = max_iter
        self.tri = np.asarray(wing["tri"], dtype=np.int32)
        self.clamped = np.asarray(wing["clamped"], dtype=np.int32)
        x0, v0 = self._root_pose(0.0, None)
        # per-vertex masses of the functional wing model, else lumped from the areas
        mass = (np.asarray(wing["mass"], dtype=np.float64) if wing.get("mass") is not None
                else fsi.lumped_masses(x0, self.tri, wing["density"]))
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
        return self._step(dt, None)

    def step_adaptive(self, cfl, c_eta, dt_max):
        """One coupled step whose dt the fluid step chooses on the device (CFL
        and penalization rule at t^n); the structure step uses the same dt.
        Returns the fluid force F^n (the dt is in self.s.info())."""
        return self._step(None, (cfl, c_eta, dt_max))

    def _step(self, dt, rule):
        x, v = self.ms.state()
        self.s.set_wing(x, v, self.tri)
        if rule is None:
            self.s.step(dt)
        else:
            self.s.step_adaptive(*rule)
        info = self.s.info()
        dt = info["dt"] if rule is not None else dt
        F = info["F"]
        if self.order == "paper":
            self.s.eval_pressure()
        loads, _ = self.s.pressure_loads()
        t1 = self.t + dt
        xc, vc = self._root_pose(t1, self.clamped)
        self.iters.append(self.ms.step(dt, self._frame(t1), loads, xc, vc, self.tol, self.max_iter))
        self.t = t1
        return F

    def state(self):
        return self.ms.state()


class HingeRollout:
    """Mean lift of a hinged plate revolving with pitch alpha, and its gradient
    with respect to theta = (alpha, k_h1, .., k_h4) by the hand-written adjoint.

    ``plate`` is a hinge-plate dict (synth.hinge_plate: bend_group g >= 0 marks
    the spanwise springs of hinge g, whose stiffness is k_hg * plate['scale'];
    all other springs keep their stiffness), ``kin`` the root kinematics
    (omega, t_ramp, axis_point, law), ``dts`` a fixed dt sequence (dt is not
    differentiated).  J = sum_n dt_n F_z^n / sum_n dt_n.

    Forward: coupled steps (FlexibleWingFSI order), fluid checkpoint and wing
    state saved every K steps.  Reverse, per segment: reload, recompute the K
    steps keeping the fluid tape, the wing states and the pressure boxes, then
    for n = last..first: the transposed wing step (fsi_ms_step_adjoint, with
    the pitch entering through the wing frame and the clamped root), the
    transposed loads (fsi_loads_adjoint) giving the mesh cotangent and the
    pressure seed, and the transposed fluid step (fsi_step_adjoint with that
    seed and dJ/dF^n), whose mesh cotangents close the loop.  The initial wing
    state is the pose at t = 0, which depends on alpha.
    """

    def __init__(self, solver, plate, kin, dts, K=10, tol=1e-12, max_iter=30):
        self.s = solver
        self.p = plate
        self.kin = kin
        self.dts = [float(d) for d in dts]
        self.K = int(K)
        self.tol, self.max_iter = tol, max_iter
        self.times = np.concatenate([[0.0], np.cumsum(self.dts)])[:-1]
        self.w = np.array(self.dts) / float(np.sum(self.dts))
        self.nseg = (len(self.dts) + self.K - 1) // self.K
        if self.nseg + self.K > 64:
            raise ValueError("checkpoints + tape exceed the 64 state slots")
        self.tri = np.asarray(plate["tri"], dtype=np.int32)
        self.clamped = np.asarray(plate["clamped"], dtype=np.int32)
        self.s_coord = np.asarray(plate["span_coord"])
        self.c_coord = np.asarray(plate["chord_coord"])
        self.group = np.asarray(plate["bend_group"])
        nx, ny, nz = solver.n
        self.dxs = np.array(solver.L) / np.array([nx, ny, nz])
        self.d = solver.tw + solver.h
        x0, _ = self._pose(0.0, np.pi / 4, None)
        ms = fsi.MassSpring(fsi.lumped_masses(x0, self.tri, plate["density"]))
        ext = np.asarray(plate["ext_ij"])
        ms.add_extension(ext, plate["ext_k"], np.ones(len(ext)))
        ms.add_bending(plate["bend_ijk"], plate["bend_kb"], None, plate["bend_axis"])
        ms.set_clamped(self.clamped)
        self.ms = ms

    def _pose(self, t, alpha, idx):
        k = self.kin
        s, c = (self.s_coord, self.c_coord) if idx is None else (self.s_coord[idx], self.c_coord[idx])
        x, v, _ = fsi.plate_pose(s, c, t, alpha, k["omega"], k["t_ramp"], k["axis_point"], k.get("law", 0))
        return x, v

    def _frame(self, t, alpha):
        k = self.kin
        return fsi.plate_frame(t, alpha, k["omega"], k["t_ramp"], k.get("law", 0))

    def _kb(self, kh):
        kb = np.array(self.p["bend_kb"], dtype=np.float64)
        for g in range(len(kh)):
            kb[self.group == g] = kh[g] * self.p["scale"]
        return kb

    def _reset(self, alpha, kh):
        nx, ny, nz = self.s.n
        self.s.set_velocity(np.zeros((3, nz, ny, nx)))
        self.ms.set_bending_k(self._kb(kh))
        x0, v0 = self._pose(0.0, alpha, None)
        self.ms.set_state(x0, v0)
        self.ms.set_rest(self._frame(0.0, alpha))
        self.ms.set_history(None)

    def _step(self, n, alpha, record, tape=None):
        x, v = self.ms.state()
        self.s.set_wing(x, v, self.tri)
        if tape is None:
            self.s.step(self.dts[n])
        else:  # keep u_hat^n in tape slot `tape` for the reverse step
            self.s.step_record(self.dts[n], tape)
        F = self.s.info()["F"]
        loads, _ = self.s.pressure_loads()
        rec = None
        if record:
            box0, pbox = self.s.pressure_box()
            rec = dict(x=x, v=v, box0=box0, pbox=pbox)
        t1 = self.times[n] + self.dts[n]
        xc, vc = self._pose(t1, alpha, self.clamped)
        self.ms.step(self.dts[n], self._frame(t1, alpha), loads, xc, vc, self.tol, self.max_iter)
        if record:
            rec["x1"] = self.ms.state()[0]
        return F, rec

    def forward(self, theta):
        alpha, kh = float(theta[0]), np.asarray(theta[1:], dtype=np.float64)
        self._reset(alpha, kh)
        self.ckpt = []
        F = []
        prev = None
        for n in range(len(self.dts)):
            if n % self.K == 0:
                self.s.save(n // self.K)
                x, v = self.ms.state()
                self.ckpt.append((x, v, prev))
            x, v = self.ms.state()
            f, _ = self._step(n, alpha, False)
            prev = (x, v, self.dts[n])
            F.append(f)
        self.forces = np.array(F)
        return float(np.dot(self.w, self.forces[:, 2]))

    def backward(self, theta):
        """dJ/dtheta after forward(theta) filled the checkpoints."""
        alpha = float(theta[0])
        N, nv = len(self.dts), self.ms.nv
        lam_x = np.zeros((N + 1, nv, 3))
        lam_v = np.zeros((N + 1, nv, 3))
        g_alpha, g_k = 0.0, np.zeros(len(theta) - 1)
        tape0 = self.nseg
        self.s.adjoint_set(None, None)
        for seg in reversed(range(self.nseg)):
            n0, n1 = seg * self.K, min(seg * self.K + self.K, N)
            self.s.load(seg)
            x, v, prev = self.ckpt[seg]
            self.ms.set_state(x, v)
            if prev is None:
                self.ms.set_history(None)
            else:
                self.ms.set_history(*prev)
            recs = []
            for n in range(n0, n1):
                recs.append(self._step(n, alpha, True, tape=tape0 + n - n0)[1])
            for n in reversed(range(n0, n1)):
                rec = recs[n - n0]
                t1 = self.times[n] + self.dts[n]
                dtp = self.dts[n - 1] if n > 0 else None
                k = self.kin
                g = self.ms.step_adjoint(self.dts[n], dtp, self._frame(t1, alpha), rec["x1"], lam_x[n + 1],
                                         lam_v[n + 1],
                                         dframe=fsi.plate_frame_dalpha(t1, alpha, k["omega"], k["t_ramp"],
                                                                       k.get("law", 0)))
                lam_x[n] += g["xn"]
                lam_v[n] += g["vn"]
                if n > 0:
                    lam_x[n - 1] += g["xp"]
                    lam_v[n - 1] += g["vp"]
                for gi in range(len(g_k)):
                    g_k[gi] += self.p["scale"] * float(np.sum(g["kb"][self.group == gi]))
                dxa, dva = fsi.plate_pose_dalpha(self.s_coord[self.clamped], self.c_coord[self.clamped], t1, alpha,
                                                 k["omega"], k["t_ramp"], k.get("law", 0))
                g_alpha += g["dframe"] + float(np.sum(g["clamp_x"] * dxa) + np.sum(g["clamp_v"] * dva))
                lx, lp = fsi.loads_adjoint(rec["x"], self.tri, self.d, self.dxs, rec["box0"], rec["pbox"], g["load"])
                lam_x[n] += lx
                self.s.set_wing(rec["x"], rec["v"], self.tri)
                self.s.adjoint_set_pressure_seed(rec["box0"], lp)
                dx, dv = self.s.step_adjoint(tape0 + n - n0, self.dts[n], self.dts[n - 1] if n > 0 else self.dts[n],
                                             1 if n == 0 else 0, (0.0, 0.0, self.w[n]))
                lam_x[n] += dx
                lam_v[n] += dv
        k = self.kin
        dxa, dva = fsi.plate_pose_dalpha(self.s_coord, self.c_coord, 0.0, alpha, k["omega"], k["t_ramp"],
                                         k.get("law", 0))
        g_alpha += float(np.sum(lam_x[0] * dxa) + np.sum(lam_v[0] * dva))
        return np.concatenate([[g_alpha], g_k])

    def value_and_grad(self, theta):
        J = self.forward(theta)
        return J, self.backward(theta)


try:
    import torch

    class HingeLift(torch.autograd.Function):
        """J(theta), theta = (alpha, k_h1..k_h4), as a torch autograd node."""

        @staticmethod
        def forward(ctx, theta, rollout):
            th = theta.detach().cpu().double().numpy()
            J = rollout.forward(th)
            ctx.rollout = rollout
            ctx.theta = th
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gJ):
            g = ctx.rollout.backward(ctx.theta)
            return gJ * torch.tensor(g, dtype=torch.float64), None

except ImportError:  # pragma: no cover
    HingeLift = None
