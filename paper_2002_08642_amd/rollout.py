"""Differentiable rollouts of the penalized step: mean lift of a revolving plate.

The objective is the time-averaged lift J = sum_n dt_n F_z^n / sum_n dt_n over
a fixed dt sequence, F^n the penalization force of step n (Sec. 4.2.2 defines
lift as the vertical force).  Its gradient with respect to the plate pitch
alpha is obtained with the library's hand-written adjoint step
(fsi_step_adjoint), reverse through the steps with checkpointed recomputation:
the forward run saves the state every K steps; the reverse sweep reloads each
checkpoint, recomputes the K steps of its segment saving every step's state as
a tape, and reverses them, chaining the vertex cotangents through the host
derivative of the plate pose (fsi_plate_pose_dalpha).

``PlateLift`` wraps this as a torch.autograd.Function (torch only carries the
scalar; all arithmetic runs in the library).
"""

import numpy as np

from . import fsi


class PlateRollout:
    """Rigid revolving plate driven through a fixed dt sequence."""

    def __init__(self, solver, cfg, dts, K=10, law=0, u0=None, uh0=None):
        self.s = solver
        self.cfg = cfg
        self.dts = [float(d) for d in dts]
        self.K = int(K)
        self.law = law
        self.u0 = u0
        self.uh0 = uh0
        self.times = np.concatenate([[0.0], np.cumsum(self.dts)])[:-1]
        self.w = np.array(self.dts) / float(np.sum(self.dts))
        self.nseg = (len(self.dts) + self.K - 1) // self.K
        if self.nseg + self.K > 64:
            raise ValueError("checkpoints + tape exceed the 64 state slots")
        self.forces = None

    def _pose(self, t, alpha):
        c = self.cfg
        x, v, _ = fsi.plate_pose(c["span_coord"], c["chord_coord"], t, alpha, c["omega"], c["t_ramp"],
                                 c["axis_point"], self.law)
        return x, v

    def _reset(self):
        if self.uh0 is not None:
            self.s.set_spectrum(self.uh0)
            return
        nx, ny, nz = self.s.n
        u0 = self.u0 if self.u0 is not None else np.zeros((3, nz, ny, nx))
        self.s.set_velocity(u0)

    def _step(self, n, alpha, tape=None):
        x, v = self._pose(self.times[n], alpha)
        self.s.set_wing(x, v, self.cfg["tri"])
        if tape is None:
            self.s.step(self.dts[n])
        else:  # keep u_hat^n in tape slot `tape` for the reverse step
            self.s.step_record(self.dts[n], tape)
        return self.s.info()["F"]

    def forward(self, alpha):
        """Run all steps, saving a checkpoint every K steps; returns J."""
        self._reset()
        forces = []
        for n in range(len(self.dts)):
            if n % self.K == 0:
                self.s.save(n // self.K)
            forces.append(self._step(n, alpha))
        self.forces = np.array(forces)
        return float(np.dot(self.w, self.forces[:, 2]))

    def backward(self, alpha):
        """dJ/dalpha by the adjoint, after ``forward(alpha)`` filled the checkpoints."""
        self.s.adjoint_set(None, None)
        grad = 0.0
        for seg in reversed(range(self.nseg)):
            grad = self.reverse_segment(seg, alpha, grad)
        return grad

    def reverse_segment(self, seg, alpha, grad=0.0):
        """Reload checkpoint ``seg``, recompute its steps into tape slots and
        reverse them, adding each step's share of dJ/dalpha to ``grad`` (one
        running sum over all steps, so the segment length does not change the
        result); returns the sum."""
        cfg = self.cfg
        tape0 = self.nseg
        N = len(self.dts)
        n0, n1 = seg * self.K, min(seg * self.K + self.K, N)
        self.s.load(seg)
        for n in range(n0, n1):
            self._step(n, alpha, tape=tape0 + n - n0)
        for n in reversed(range(n0, n1)):
            x, v = self._pose(self.times[n], alpha)
            self.s.set_wing(x, v, cfg["tri"])
            first = 1 if n == 0 else 0
            dtp = self.dts[n - 1] if n > 0 else self.dts[n]
            dx, dv = self.s.step_adjoint(tape0 + n - n0, self.dts[n], dtp, first, (0.0, 0.0, self.w[n]))
            dxa, dva = fsi.plate_pose_dalpha(cfg["span_coord"], cfg["chord_coord"], self.times[n], alpha,
                                             cfg["omega"], cfg["t_ramp"], self.law)
            grad += float(np.sum(dx * dxa) + np.sum(dv * dva))
        return grad

    def value_and_grad(self, alpha):
        J = self.forward(alpha)
        return J, self.backward(alpha)


try:
    import torch

    class PlateLift(torch.autograd.Function):
        """J(alpha) as a torch autograd node; backward runs the checkpointed adjoint."""

        @staticmethod
        def forward(ctx, alpha, rollout):
            a = float(alpha.detach().cpu().item())
            J = rollout.forward(a)
            ctx.rollout = rollout
            ctx.alpha = a
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gJ):
            g = ctx.rollout.backward(ctx.alpha)
            return gJ * torch.tensor(g, dtype=torch.float64), None

except ImportError:  # pragma: no cover - torch is optional for the rollout itself
    PlateLift = None
