"""GPU parity of the channel workload (Sec. 4.2.1: channel walls, a cylinder
and a Poiseuille inflow as a static z-independent penalization, a flexible
mass-spring flag behind the cylinder) against the oracle.

* the penalized channel alone, from rest: velocity after the steps and the
  weighted force on the cylinder at every step;
* the static plane on the 512-point register x pass (its own kernel
  instantiation) with a plate crossing it (max rule of the two masks);
* the flag coupled to the channel flow (static root inside the cylinder,
  lagged pressure order) against oracle.coupling with the same static plane;
* the reverse step refuses the static plane (FSI_ESTATE).
Tolerances as the other parity tests: FP64 1e-11 (velocity) / 1e-10 (forces),
FP32 1e-5 / 1e-4; the coupled flag as tests/test_gpu_coupled.py.
"""

import numpy as np
import pytest

from oracle import ns as ons, structure as st
from oracle.coupling import CoupledOracle
from paper_2002_08642_amd import fsi
from paper_2002_08642_amd.coupled import FlexibleWingFSI
from tests.helpers import rel_max
import synth

pytestmark = pytest.mark.gpu

VTOL = {fsi.PREC_FP64: 1e-11, fsi.PREC_FP32: 1e-5}
FTOL = {fsi.PREC_FP64: 1e-10, fsi.PREC_FP32: 1e-4}
NU = 1e-3
ETA = 2e-3


@pytest.mark.parametrize("prec", [fsi.PREC_FP64, fsi.PREC_FP32])
def test_channel_static_mask_parity(prec):
    ch = synth.turek_channel(96, 24, 8)
    nx, ny, nz = ch["n"]
    print("channel static mask", prec, flush=True)
    o = ons.OracleNS(ch["n"], ch["L"], NU, ETA)
    s = fsi.Solver(ch["n"], ch["L"], NU, ETA, 0.0, ch["h"], fsi.PROFILE_COS, prec)
    o.set_static_mask(*ch["static"])
    s.set_static_mask(*ch["static"])
    o.set_velocity(np.zeros((3, nz, ny, nx)))
    s.set_velocity(np.zeros((3, nz, ny, nx)))
    fo, fg = [], []
    for k in range(12):
        dt = 2.0 / 3.0 * ETA if k != 5 else 0.5 * ETA
        d = o.step(dt=dt)
        s.step(dt)
        fo.append(d["F_static"])
        fg.append(s.static_force())
        assert not np.any(s.info()["F"])  # no wing
    ev = rel_max(s.velocity(), o.velocity())
    ef = rel_max(np.array(fg), np.array(fo))
    print("channel prec %d: velocity %.3e cylinder force %.3e (max |F| %.3e)"
          % (prec, ev, ef, np.max(np.abs(fo))), flush=True)
    assert np.max(np.abs(np.array(fo))) > 1e-2
    assert ev < VTOL[prec] and ef < FTOL[prec]


@pytest.mark.parametrize("prec", [fsi.PREC_FP64, fsi.PREC_FP32])
def test_static_plane_on_the_512_point_x_pass(prec):
    n, L = (512, 16, 12), (8.0, 1.0, 0.75)
    nx, ny, nz = n
    nu, eta, tw, h = 0.01, 0.05, 0.05, 0.03
    rng = np.random.default_rng(31)
    x = np.arange(nx) * (L[0] / nx)
    y = np.arange(ny) * (L[1] / ny)
    # a static solid with chi = 1 from x = 4.0 (sharp: across the plate at
    # x = 4.0, whose support it halves: the static solid wins there on the tie
    # chi = 1 and where the plate's chi is smaller), a smooth edge over
    # x in [4.6, 4.9] and a y-dependent smooth layer elsewhere.  No point has
    # both chi strictly between 0 and 1: where they cross, FP32 and FP64 may
    # pick different solids (the max rule is discontinuous there).
    ramp = np.clip((4.9 - x) / 0.3, 0.0, 1.0)
    slab = np.where(x >= 4.0, 0.5 * (1 - np.cos(np.pi * ramp)), 0.0)
    layer = np.where((x > 5.5) & (x < 7.5), 0.5 * (1 - np.cos(2 * np.pi * (x - 5.5) / 2.0)), 0.0)
    chi = np.maximum(slab[None, :], layer[None, :] * (0.5 + 0.5 * np.cos(2 * np.pi * y / L[1]))[:, None])
    us = np.zeros((3, ny, nx))
    us[0] = 0.3 * np.cos(2 * np.pi * y / L[1])[:, None]
    us[2] = 0.1
    w = (rng.uniform(0, 1, (ny, nx)) > 0.3).astype(float)
    o = ons.OracleNS(n, L, nu, eta, tw, h, 0)
    s = fsi.Solver(n, L, nu, eta, tw, h, 0, prec)
    u0 = synth.random_solenoidal(n, L, seed=21)
    o.set_velocity(u0)
    s.set_velocity(u0)
    xp, tri = synth.flat_rectangle((4.0, 0.5, 0.4), (0, 1, 0), (0, 0, 1), 0.2, 0.15, 5, 4)
    v = np.tile(np.array([0.3, 0.0, 0.1]), (len(xp), 1))
    for side in (o, s):
        side.set_wing(xp, v, tri)
        side.set_static_mask(chi, us, w)
    fo, fg, so, sg = [], [], [], []
    for _ in range(5):
        d = o.step(dt=0.02)
        s.step(0.02)
        fo.append(d["F"])
        so.append(d["F_static"])
        fg.append(s.info()["F"])
        sg.append(s.static_force())
    ev = rel_max(s.velocity(), o.velocity())
    ef, es = rel_max(np.array(fg), np.array(fo)), rel_max(np.array(sg), np.array(so))
    print("512 x pass, static plane, prec %d: velocity %.3e wing force %.3e static force %.3e"
          % (prec, ev, ef, es), flush=True)
    assert np.max(np.abs(np.array(fo))) > 1e-3 and np.max(np.abs(np.array(so))) > 1e-3
    assert ev < VTOL[prec] and ef < FTOL[prec] and es < FTOL[prec]


@pytest.mark.parametrize("prec", [fsi.PREC_FP64, fsi.PREC_FP32])
def test_channel_flag_coupled_parity(prec):
    ch = synth.turek_channel(128, 32, 16)
    nx, ny, nz = ch["n"]
    wing, ijk, bend, axis, kin, tw = synth.turek_flag(ch)
    # k^b of Eq. EI_k_relation on each side
    kb_o = bend["factor"] * np.array([st.bending_stiffness(e, l, n) for e, l, n in zip(bend["EI"], bend["lb"], bend["nb"])])
    kb_g = bend["factor"] * np.array([fsi.bending_stiffness(e, l, n) for e, l, n in zip(bend["EI"], bend["lb"], bend["nb"])])
    print("channel flag", prec, flush=True)
    o = CoupledOracle(ch["n"], ch["L"], NU, ETA, tw, ch["h"], fsi.PROFILE_COS, wing, ijk, kb_o, axis, kin, tol=1e-12)
    # from the developed channel flow: the flag is loaded from the first step
    u0 = synth.turek_inflow_field(ch)
    o.fluid.set_static_mask(*ch["static"])
    o.fluid.set_velocity(u0)
    s = fsi.Solver(ch["n"], ch["L"], NU, ETA, tw, ch["h"], fsi.PROFILE_COS, prec, pressure=True)
    s.set_static_mask(*ch["static"])
    s.set_velocity(u0)
    g = FlexibleWingFSI(s, wing, ijk, kb_g, axis, kin, tol=1e-12)
    fo, fg, so, sg = [], [], [], []
    dt = 2.0 / 3.0 * ETA
    for _ in range(10):
        fo.append(o.step(dt))
        so.append(o.last["F_static"])
        fg.append(g.step(dt))
        sg.append(s.static_force())
    x, v = g.state()
    xr, _ = o._root_pose(o.t, None)
    ex = rel_max(x - xr, o.q[0] - xr)
    ev = rel_max(v, o.q[1])
    ef = rel_max(np.array(fg), np.array(fo))
    es = rel_max(np.array(sg), np.array(so))
    eu = rel_max(s.velocity(), o.fluid.velocity())
    print("channel flag prec %d: deflection %.3e velocity %.3e flag force %.3e cylinder force %.3e flow %.3e "
          "(max deflection %.3e)" % (prec, ex, ev, ef, es, eu, np.max(np.abs(o.q[0] - xr))), flush=True)
    tol = {fsi.PREC_FP64: 1e-9, fsi.PREC_FP32: 1e-4}[prec]
    assert np.max(np.abs(o.q[0] - xr)) > 1e-6
    assert ex < tol and ev < tol and ef < tol and es < tol and eu < tol


def test_reverse_step_refuses_the_static_plane():
    ch = synth.turek_channel(96, 24, 8)
    s = fsi.Solver(ch["n"], ch["L"], NU, ETA, 0.0, ch["h"], fsi.PROFILE_COS, fsi.PREC_FP64)
    s.set_static_mask(*ch["static"])
    s.step_record(ETA / 2, 0)
    with pytest.raises(fsi.FsiError) as e:
        s.step_adjoint(0, ETA / 2, ETA / 2, 1, (0.0, 0.0, 0.0))
    assert e.value.code == -5
    s.set_static_mask(None, None)
    chi = np.full((24, 96), 1.5)
    with pytest.raises(fsi.FsiError) as e:
        s.set_static_mask(chi, np.zeros((3, 24, 96)))
    assert e.value.code == -1
