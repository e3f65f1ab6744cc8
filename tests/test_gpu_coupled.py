"""GPU parity of the staggered fluid-structure coupling against the oracle.

A small flexible wing (11 x 6 membrane, 3 veins of 9 nodes, EI and membrane
stiffness drawn as in the flexible-wing recipe, areal density 1) revolving in a
48^3 box of side 12: fluid step on the GPU (FSI mode), pressure loads, native
BDF2/Newton structure step - against oracle.coupling (numpy fluid, FD-Jacobian
Newton structure).  Tolerances relative to the largest value: FP64 1e-9
(positions, velocities, forces); FP32 fluid 1e-4 (forces and deflections carry
the FP32 rounding of the loads through the structure).
"""

import numpy as np
import pytest

from oracle import structure as st
from oracle.coupling import CoupledOracle
from paper_2002_08642_amd import fsi
from paper_2002_08642_amd.coupled import FlexibleWingFSI
import synth

pytestmark = pytest.mark.gpu

TOL = {fsi.PREC_FP64: 1e-9, fsi.PREC_FP32: 1e-4}


def small_case(n=48, density=1.0):
    cfg = synth.revolving_plate(n=n, t_ramp=0.05)
    w = synth.flexible_wing(ns=11, nc=6, n_veins=3, vein_nodes=9, density=density)
    ijk, owner = synth.vein_bending(w)
    kin = dict(alpha=cfg["alpha"], omega=cfg["omega"], t_ramp=cfg["t_ramp"], axis_point=cfg["axis_point"])
    return cfg, w, ijk, owner, kin


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("order", ["lagged", "paper"])
@pytest.mark.parametrize("prec", [fsi.PREC_FP64, fsi.PREC_FP32])
def test_coupled_flexible_wing_matches_oracle(prec, order):
    """Both pressure orders of the staggered step: p^n of the fluid step
    (lagged), or p^{n+1} of the new velocity (the paper's order, one more
    nonlinear evaluation per step: fsi_eval_pressure)."""
    cfg, w, ijk, owner, kin = small_case()
    kb_o = np.array([st.bending_stiffness(w["vein_EI"][v], w["vein_length"], len(w["veins"][v]) - 2) for v in owner])
    kb_g = np.array([fsi.bending_stiffness(w["vein_EI"][v], w["vein_length"], len(w["veins"][v]) - 2) for v in owner])
    axis = np.zeros(len(ijk), dtype=np.int32)
    o = CoupledOracle(cfg["n"], cfg["L"], cfg["nu"], cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"], w, ijk, kb_o,
                      axis, kin, order=order)
    s = fsi.Solver(cfg["n"], cfg["L"], cfg["nu"], cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"], prec,
                   pressure=True)
    s.set_velocity(np.zeros((3,) + cfg["n"]))
    g = FlexibleWingFSI(s, w, ijk, kb_g, axis, kin, tol=1e-12, order=order)
    fo, fg = [], []
    for k in range(10):
        fo.append(o.step(2e-3))
        fg.append(g.step(2e-3))
    x, v = g.state()
    xr, _ = o._root_pose(o.t, None)
    ex, ev, ef = rel(x - xr, o.q[0] - xr), rel(v, o.q[1]), rel(fg, fo)
    print("coupled %s prec %d: deflection %.3e velocity %.3e force %.3e (max deflection %.3e, Newton its %s)"
          % (order, prec, ex, ev, ef, np.max(np.abs(o.q[0] - xr)), g.iters), flush=True)
    assert ex < TOL[prec] and ev < TOL[prec] and ef < TOL[prec]
    assert max(g.iters) <= 8


# 96^3, and the flexible-wing workload's own 256^3 (eta scales as dx^2 there:
# dt / eta = 0.64)
@pytest.mark.parametrize("n,dt,nsteps", [(96, 1e-3, 12), (256, 4e-4, 20)], ids=["96", "256"])
def test_full_flexible_wing_fp32_follows_fp64(n, dt, nsteps):
    """The config-2 wing (31 x 16 membrane, 8 veins of 25 nodes): the FP32 fluid
    with the FP64 structure follows the FP64 run."""
    cfg = synth.revolving_plate(n=n, t_ramp=0.05)
    w = synth.flexible_wing(density=1.0)
    ijk, owner = synth.vein_bending(w)
    kb = np.array([fsi.bending_stiffness(w["vein_EI"][v], w["vein_length"], len(w["veins"][v]) - 2) for v in owner])
    kin = dict(alpha=cfg["alpha"], omega=cfg["omega"], t_ramp=cfg["t_ramp"], axis_point=cfg["axis_point"])
    runs = {}
    for prec in (fsi.PREC_FP64, fsi.PREC_FP32):
        s = fsi.Solver(cfg["n"], cfg["L"], cfg["nu"], cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"], prec,
                       pressure=True)
        s.set_velocity(np.zeros((3,) + cfg["n"]))
        g = FlexibleWingFSI(s, w, ijk, kb, np.zeros(len(ijk), np.int32), kin, tol=1e-10)
        F = [g.step(dt) for _ in range(nsteps)]
        runs[prec] = (g.state()[0], np.array(F), g)
    x64, F64, g64 = runs[fsi.PREC_FP64]
    x32, F32, _ = runs[fsi.PREC_FP32]
    xr, _ = g64._root_pose(g64.t, None)
    ed, ef = rel(x32 - xr, x64 - xr), rel(F32, F64)
    print("config-2 wing %d^3: FP32 vs FP64 deflection %.3e force %.3e (max deflection %.3e)"
          % (n, ed, ef, np.max(np.abs(x64 - xr))), flush=True)
    assert ed < 1e-4 and ef < 1e-4


@pytest.mark.parametrize("prec", [fsi.PREC_FP64, fsi.PREC_FP32])
def test_functional_wing_coupled_96(prec):
    """The functional bumblebee forewing (31 x 16 vertices, the 21 veins of
    the table with their masses, the membrane mass law elsewhere, vein EI of the
    flexible wing through Eq. EI_k_relation) revolving in the 96^3 box: GPU
    fluid + native structure against oracle.coupling, 10 steps of dt = 1e-3."""
    cfg = synth.revolving_plate(n=96, t_ramp=0.05)
    w = synth.functional_wing()
    kb_o = np.array([st.bending_stiffness(e, l, n) for e, l, n in zip(w["bend_EI"], w["bend_lb"], w["bend_nb"])])
    kb_g = np.array([fsi.bending_stiffness(e, l, n) for e, l, n in zip(w["bend_EI"], w["bend_lb"], w["bend_nb"])])
    kin = dict(alpha=cfg["alpha"], omega=cfg["omega"], t_ramp=cfg["t_ramp"], axis_point=cfg["axis_point"])
    print("functional wing 96^3 prec %d" % prec, flush=True)
    o = CoupledOracle(cfg["n"], cfg["L"], cfg["nu"], cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"], w,
                      w["bend_ijk"], kb_o, w["bend_axis"], kin, tol=1e-12)
    o.fluid.set_velocity(np.zeros((3,) + cfg["n"]))
    s = fsi.Solver(cfg["n"], cfg["L"], cfg["nu"], cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"], prec,
                   pressure=True)
    s.set_velocity(np.zeros((3,) + cfg["n"]))
    g = FlexibleWingFSI(s, w, w["bend_ijk"], kb_g, w["bend_axis"], kin, tol=1e-12)
    fo, fg = [], []
    for _ in range(10):
        fo.append(o.step(1e-3))
        fg.append(g.step(1e-3))
    x, v = g.state()
    xr, _ = o._root_pose(o.t, None)
    ex, ev, ef = rel(x - xr, o.q[0] - xr), rel(v, o.q[1]), rel(fg, fo)
    print("functional wing 96^3 prec %d: deflection %.3e velocity %.3e force %.3e (max deflection %.3e, "
          "Newton its %s)" % (prec, ex, ev, ef, np.max(np.abs(o.q[0] - xr)), g.iters), flush=True)
    assert np.max(np.abs(o.q[0] - xr)) > 1e-5
    assert ex < TOL[prec] and ev < TOL[prec] and ef < TOL[prec]
    assert max(g.iters) <= 10
