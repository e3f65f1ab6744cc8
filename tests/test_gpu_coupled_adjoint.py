"""Gradient of the mean lift of a hinged revolving plate through the coupled
fluid-structure rollout (checkpointed hand-written adjoint).

At the differentiation workload's own size (128^3, 50 FP32 steps, checkpoints
every 10) the FP32 adjoint gradient is checked against central differences of
the GPU FP64 rollout with the same bar.

theta = (pitch alpha, hinge stiffnesses k_h1..k_h4) of a 4-segment plate
(synth.hinge_plate, areal density 1) in a 32^3 box of side 12, 8 coupled
steps of dt = 1.5e-3, checkpoints every 4 steps.  The adjoint gradient is
checked per component against central differences of the GPU FP64 rollout
(h = 1e-5 for alpha, 1e-4 relative for k_h) and, for alpha and k_h1,
against central differences of the FP64 oracle rollout
(oracle.coupling); bar |g - g_FD| <= 1e-3 max(|g_FD|, 1e-3 |g_FD|_inf).
"""

import numpy as np
import pytest

from oracle.coupling import CoupledOracle
from paper_2002_08642_amd import fsi
from paper_2002_08642_amd.coupled import HingeRollout, HingeLift
import synth

pytestmark = pytest.mark.gpu

THETA0 = np.array([np.pi / 4, 1e-2, 1e-2, 1e-2, 1e-2])
STEPS, DT = 8, 1.5e-3


# A rotation axis on a grid line puts grid points exactly above chordwise
# edges of the plate at t = 0 (grid spacing 0.375 = 5 span spacings): the
# distance is a min over tied triangles there and J is only one-sidedly
# differentiable in alpha (central differences then miss the adjoint by 2 %).
# The axis is moved off the grid.
AXIS = (6.0137, 5.9871, 6.0213)


def case():
    cfg = synth.revolving_plate(n=32, fixed_eta=2.5e-3, t_ramp=0.02)
    plate = synth.hinge_plate(density=1.0)
    kin = dict(omega=cfg["omega"], t_ramp=cfg["t_ramp"], axis_point=AXIS)
    return cfg, plate, kin


def rollout(prec, K=4):
    cfg, plate, kin = case()
    s = fsi.Solver(cfg["n"], cfg["L"], cfg["nu"], cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"], prec,
                   pressure=True)
    return HingeRollout(s, plate, kin, [DT] * STEPS, K=K), cfg, plate, kin


def steps_for(theta):
    h = np.zeros_like(theta)
    h[0] = 1e-5
    h[1:] = 1e-4 * np.abs(theta[1:])
    return h


def close(g, fd, scale):
    return abs(g - fd) <= 1e-3 * max(abs(fd), 1e-3 * scale)


def test_hinge_gradient_matches_gpu_finite_differences():
    ro, _, _, _ = rollout(fsi.PREC_FP64)
    J, g = ro.value_and_grad(THETA0)
    h = steps_for(THETA0)
    fd = np.zeros(5)
    for i in range(5):
        e = np.zeros(5)
        e[i] = h[i]
        fd[i] = (ro.forward(THETA0 + e) - ro.forward(THETA0 - e)) / (2 * h[i])
    print("J %.10e\nadjoint %s\nFD      %s" % (J, g, fd), flush=True)
    scale = np.max(np.abs(fd))
    for i in range(5):
        assert close(g[i], fd[i], scale), (i, g[i], fd[i])


def oracle_J(theta, cfg, plate, kin):
    k = dict(kin, alpha=float(theta[0]))
    kb = np.array(plate["bend_kb"], dtype=np.float64)
    for gi in range(4):
        kb[plate["bend_group"] == gi] = theta[1 + gi] * plate["scale"]
    o = CoupledOracle(cfg["n"], cfg["L"], cfg["nu"], cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"], plate,
                      plate["bend_ijk"], kb, plate["bend_axis"], k)
    o.fluid.set_velocity(np.zeros((3,) + cfg["n"]))
    F = [o.step(DT) for _ in range(STEPS)]
    return float(np.mean(np.array(F)[:, 2]))


def test_hinge_gradient_matches_oracle_finite_differences():
    ro, cfg, plate, kin = rollout(fsi.PREC_FP64)
    J, g = ro.value_and_grad(THETA0)
    Jo = oracle_J(THETA0, cfg, plate, kin)
    h = steps_for(THETA0)
    for i in (0, 1):
        e = np.zeros(5)
        e[i] = h[i]
        fdo = (oracle_J(THETA0 + e, cfg, plate, kin) - oracle_J(THETA0 - e, cfg, plate, kin)) / (2 * h[i])
        print("param %d: adjoint %.8e oracle FD %.8e (J %.10e oracle %.10e)" % (i, g[i], fdo, J, Jo), flush=True)
        assert close(g[i], fdo, abs(fdo))
    assert abs(J - Jo) <= 1e-9 * abs(Jo)


def test_fp32_hinge_adjoint():
    ro64, _, _, _ = rollout(fsi.PREC_FP64)
    ro32, _, _, _ = rollout(fsi.PREC_FP32)
    _, g64 = ro64.value_and_grad(THETA0)
    _, g32 = ro32.value_and_grad(THETA0)
    print("FP32 adjoint %s\nFP64 adjoint %s" % (g32, g64), flush=True)
    scale = np.max(np.abs(g64))
    for i in range(5):
        assert close(g32[i], g64[i], scale)


def test_segment_length_does_not_change_the_gradient():
    ro_a, _, _, _ = rollout(fsi.PREC_FP64, K=8)
    ro_b, _, _, _ = rollout(fsi.PREC_FP64, K=3)
    _, ga = ro_a.value_and_grad(THETA0)
    _, gb = ro_b.value_and_grad(THETA0)
    assert np.array_equal(ga, gb)


def test_hinge_lift_autograd():
    import torch
    ro, _, _, _ = rollout(fsi.PREC_FP64)
    th = torch.tensor(THETA0, dtype=torch.float64, requires_grad=True)
    J = HingeLift.apply(th, ro)
    J.backward()
    _, g = ro.value_and_grad(THETA0)
    assert np.allclose(th.grad.numpy(), g, rtol=1e-12, atol=0)


def test_hinge_gradient_at_workload_size():
    """128^3 box of side 12, 50 coupled steps of dt = 1.5e-3 (inside the 0.2
    revolution ramp), checkpoints every 10 steps; FP32 adjoint against central
    differences of the FP64 rollout."""
    cfg = synth.revolving_plate(n=128, t_ramp=0.2)
    plate = synth.hinge_plate(density=1.0)
    kin = dict(omega=cfg["omega"], t_ramp=cfg["t_ramp"], axis_point=AXIS)
    steps = [DT] * 50

    def make(prec, K):
        s = fsi.Solver(cfg["n"], cfg["L"], cfg["nu"], cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"], prec,
                       pressure=True)
        return HingeRollout(s, plate, kin, steps, K=K)

    ro32 = make(fsi.PREC_FP32, 10)
    J32, g32 = ro32.value_and_grad(THETA0)
    del ro32
    ro64 = make(fsi.PREC_FP64, 10)
    h = steps_for(THETA0)
    fd = np.zeros(5)
    for i in range(5):
        e = np.zeros(5)
        e[i] = h[i]
        fd[i] = (ro64.forward(THETA0 + e) - ro64.forward(THETA0 - e)) / (2 * h[i])
    print("128^3 J %.8e\nFP32 adjoint %s\nFP64 FD      %s" % (J32, g32, fd), flush=True)
    scale = np.max(np.abs(fd))
    for i in range(5):
        assert close(g32[i], fd[i], scale), (i, g32[i], fd[i])
