"""GPU parity of the vorticity sponge term (Sec. 4.1, sponge term of the
penalized equations; sign and mask readings in oracle/sponge.py) against the
FP64 oracle, and the adjoint of the step with the sponge on.

The sponge layers are cosine tapers at the x faces and at the top z face, a
tilted plate sits in the middle, and the field is the random k^-5/3 field.
Tolerances as for the plain step (velocity 1e-5 / 1e-11 relative, forces
1e-4 / 1e-10 for FP32 / FP64).  A z length of 512 selects the compile-time
512-point column kernels (the sponge's z pass among them).
"""

import numpy as np
import pytest

from oracle import ns as ons
from paper_2002_08642_amd import fsi
from tests.helpers import rel_max
from tests.test_gpu_adjoint import run_two_steps
import synth

pytestmark = pytest.mark.gpu

VTOL = {fsi.PREC_FP64: 1e-11, fsi.PREC_FP32: 1e-5}
FTOL = {fsi.PREC_FP64: 1e-10, fsi.PREC_FP32: 1e-4}


def face_taper(m, width):
    """1 at the two faces of an axis of m points, cosine taper to 0 over `width` points."""
    i = np.arange(m)
    d = np.minimum(i, m - i) / float(width)
    return np.where(d < 1.0, 0.5 * (1.0 + np.cos(np.pi * d)), 0.0)


def top_taper(m, width):
    i = np.arange(m)
    d = (m - 1 - i) / float(width)
    return np.where(d < 1.0, 0.5 * (1.0 + np.cos(np.pi * d)), 0.0)


# (512, 16, 12): the register-resident sponge x pass; (16, 12, 512): the
# compile-time 512-point column kernels
CASES = [((32, 24, 20), (2.0, 1.5, 1.25)), ((16, 12, 512), (1.0, 0.75, 32.0)), ((512, 16, 12), (8.0, 0.25, 0.1875))]
# wing thickness, smoothing and plate sides per case (the thin box needs a small plate)
GEOM = {(32, 24, 20): (0.05, 0.03, 0.3, 0.2), (16, 12, 512): (0.05, 0.03, 0.3, 0.2),
        (512, 16, 12): (0.03, 0.016, 0.3, 0.025)}


@pytest.mark.parametrize("prec", [fsi.PREC_FP64, fsi.PREC_FP32])
@pytest.mark.parametrize("n,L", CASES)
def test_sponge_parity(n, L, prec):
    tw, h, pa, pb = GEOM[n]
    nu, eta, c_sp = 0.01, 0.05, 0.08
    print("sponge", n, prec, flush=True)
    o = ons.OracleNS(n, L, nu, eta, tw, h, 0)
    s = fsi.Solver(n, L, nu, eta, tw, h, 0, prec)
    u0 = synth.random_solenoidal(n, L, seed=31)
    o.set_velocity(u0)
    s.set_velocity(u0)
    gx, gz = face_taper(n[0], n[0] // 5), top_taper(n[2], max(3, n[2] // 6))
    o.set_sponge(c_sp, gx=gx, gz=gz)
    s.set_sponge(c_sp, gx=gx, gz=gz)
    centre = (0.5 * L[0] + 0.013, 0.5 * L[1] + 0.021, 0.5 * L[2] - 0.007)
    ua = np.array([1.0, 0.05, 0.02]) / np.linalg.norm([1.0, 0.05, 0.02])
    va = np.array([0.0, 0.3, 1.0]) / np.linalg.norm([0.0, 0.3, 1.0])
    x, tri = synth.flat_rectangle(centre, ua, va, pa, pb, 6, 4)
    v = np.tile(np.array([0.2, -0.1, 0.05]), (len(x), 1))
    o.set_wing(x, v, tri)
    s.set_wing(x, v, tri)
    fo, fg = [], []
    for _ in range(5):
        d = o.step(dt=2e-3)
        s.step(2e-3)
        i = s.info()
        fo.append(d["F"])
        fg.append(i["F"])
        assert i["umax"] == pytest.approx(d["umax"], rel=VTOL[prec] * 10)
    ev = rel_max(s.velocity(), o.velocity())
    ef = rel_max(np.array(fg), np.array(fo))
    print("sponge %s velocity %.3e force %.3e" % (n, ev, ef), flush=True)
    assert ev < VTOL[prec]
    assert ef < FTOL[prec]


def test_sponge_changes_the_flow():
    """The parity test above would pass with a sponge that does nothing: the
    sponge must change the velocity by far more than the tolerance."""
    n, L = CASES[0]
    runs = []
    for on in (False, True):
        s = fsi.Solver(n, L, 0.01, 0.05, precision=fsi.PREC_FP64)
        s.set_velocity(synth.random_solenoidal(n, L, seed=31))
        if on:
            s.set_sponge(0.08, gx=face_taper(n[0], n[0] // 5))
        for _ in range(5):
            s.step(2e-3)
        runs.append(s.velocity())
    assert rel_max(runs[1], runs[0]) > 1e-3


@pytest.mark.parametrize("prec", [fsi.PREC_FP64, fsi.PREC_FP32])
def test_uniform_sponge_recurrence(prec):
    """chi_sp = 1 on the 2-D Taylor-Green field: the scalar IF-AB2 recurrence of a
    linear damping 1/C_sp (closed form, as pinned for the oracle)."""
    n, L = (32, 32, 16), (2 * np.pi,) * 3
    nu, c_sp = 0.02, 0.3
    s = fsi.Solver(n, L, nu, 1.0, precision=prec)
    u0 = synth.taylor_green_2d(n, L)
    s.set_velocity(u0)
    s.set_sponge(c_sp, gx=np.ones(n[0]))
    a_prev, a, dt_prev = None, 1.0, None
    for dt in np.random.default_rng(4).uniform(0.005, 0.03, 10):
        s.step(dt)
        en = np.exp(-2 * nu * dt)
        if a_prev is None:
            a_new = en * (1 - dt / c_sp) * a
        else:
            xi = dt / dt_prev
            ep = np.exp(-2 * nu * dt_prev)
            a_new = en * (1 - dt * (1 + xi / 2) / c_sp) * a + dt * (xi / 2) / c_sp * en * ep * a_prev
        a_prev, a, dt_prev = a, a_new, dt
    assert rel_max(s.velocity(), a * u0) < (1e-12 if prec == fsi.PREC_FP64 else 2e-6)


def test_sponge_switches_off():
    n, L = CASES[0]
    a = fsi.Solver(n, L, 0.01, 0.05, precision=fsi.PREC_FP64)
    b = fsi.Solver(n, L, 0.01, 0.05, precision=fsi.PREC_FP64)
    for s in (a, b):
        s.set_velocity(synth.random_solenoidal(n, L, seed=3))
    a.set_sponge(0.1, gy=np.ones(n[1]))
    a.set_sponge(0.0)
    for s in (a, b):
        s.step(2e-3)
    assert np.array_equal(a.spectrum(), b.spectrum())
    with pytest.raises(fsi.FsiError):
        a.set_sponge(0.1, gx=-np.ones(n[0]))


# Adjoint of the step with the sponge on: dot-product test (two steps, an
# integrating-factor Euler step then an AB2 step) against central differences
# of the GPU forward map, for perturbations of the initial spectrum, of the
# mesh vertex positions and of their velocities, with force seeds and random
# cotangents of the final state.  (32, 24, 20): the LDS x passes; (512, 16, 12):
# the register-resident adjoint x pass next to the sponge's LDS x transforms.
ADJ_CASES = [((32, 24, 20), (2.0, 1.5, 1.25), (0.05, 0.03, 0.3, 0.2)),
             ((512, 16, 12), (8.0, 0.25, 0.1875), (0.03, 0.016, 0.3, 0.025))]


def sponge_adjoint_case(n, L, geom, prec, c_sp=0.08, part="all"):
    tw, h, pa, pb = geom
    s = fsi.Solver(n, L, 0.02, 0.05, tw, h, fsi.PROFILE_COS, prec)
    s.set_sponge(c_sp, gx=face_taper(n[0], n[0] // 5), gz=top_taper(n[2], max(3, n[2] // 6)))
    rng = np.random.default_rng(23)
    u0 = synth.random_solenoidal_compact(n, L, seed=8)
    du = synth.random_solenoidal_compact(n, L, seed=9) if part in ("u", "all") else 0 * u0
    centre = (0.5 * L[0] + 0.013, 0.5 * L[1] + 0.021, 0.5 * L[2] - 0.007)
    ua = np.array([1.0, 0.05, 0.02]) / np.linalg.norm([1.0, 0.05, 0.02])
    va = np.array([0.0, 0.3, 1.0]) / np.linalg.norm([0.0, 0.3, 1.0])
    x0, tri = synth.flat_rectangle(centre, ua, va, pa, pb, 6, 4)
    x0 = x0 + 0.002 * rng.standard_normal(x0.shape)
    v0 = rng.standard_normal(x0.shape)
    dx = 0.005 * rng.standard_normal(x0.shape) if part in ("x", "all") else 0 * x0
    dv = rng.standard_normal(x0.shape) if part in ("v", "all") else 0 * x0
    g = [rng.standard_normal(3), rng.standard_normal(3)]
    lam_u = rng.standard_normal(u0.shape) + 1j * rng.standard_normal(u0.shape)
    lam_n = rng.standard_normal(u0.shape) + 1j * rng.standard_normal(u0.shape)
    return run_two_steps(s, u0, x0, v0, tri, (0.01, 0.013), g, lam_u, lam_n, du, dx, dv)


@pytest.mark.parametrize("part", ["u", "all"])
@pytest.mark.parametrize("n,L,geom", ADJ_CASES, ids=["32x24x20", "512x16x12"])
def test_sponge_adjoint_dot_product(n, L, geom, part):
    print("sponge adjoint", n, part, flush=True)
    adj, fd, _ = sponge_adjoint_case(n, L, geom, fsi.PREC_FP64, part=part)
    print("sponge adjoint %s %s: adjoint %.12e fd %.12e" % (n, part, adj, fd), flush=True)
    assert abs(adj - fd) <= 1e-7 * max(abs(fd), 1e-8)


def test_sponge_adjoint_changes_the_gradient():
    """The dot-product test would pass with the sponge left out of both the
    forward and the adjoint: the sponge must change the initial-state cotangent
    by far more than the tolerance."""
    n, L, geom = ADJ_CASES[0]
    _, _, (lu_on, _, _, _) = sponge_adjoint_case(n, L, geom, fsi.PREC_FP64, part="u")
    _, _, (lu_off, _, _, _) = sponge_adjoint_case(n, L, geom, fsi.PREC_FP64, c_sp=0.0, part="u")
    assert rel_max(lu_on, lu_off) > 1e-3


def test_sponge_adjoint_fp32_matches_fp64():
    n, L, geom = ADJ_CASES[1]
    _, _, (lu64, ln64, gx64, gv64) = sponge_adjoint_case(n, L, geom, fsi.PREC_FP64, part="u")
    _, _, (lu32, ln32, gx32, gv32) = sponge_adjoint_case(n, L, geom, fsi.PREC_FP32, part="u")
    e = [rel_max(lu32, lu64), rel_max(ln32, ln64), rel_max(gx32, gx64), rel_max(gv32, gv64)]
    print("sponge adjoint FP32 vs FP64: %s" % e, flush=True)
    assert max(e) < 1e-3
