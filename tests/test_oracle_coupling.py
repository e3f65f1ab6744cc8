"""Pins of the staggered coupling order of oracle.coupling (Sec. 4.1, staggered
scheme paragraph; Sec. 2.1 Eq. discretized_ODEs).

The order inside one coupled step is checked against things that do not share
its sequence:

* a prescribed pressure p(x, t) = g(t) a.x (linear in space: the 4-point
  kernel interpolates it exactly, so every vertex load has a closed form) acts
  on a two-triangle wing whose tip vertices carry no springs: they move
  ballistically, and their positions must follow the BDF2 recurrence with the
  load of p^n (lagged order) or of p^{n+1} (paper's order), evaluated on the
  wing of t^n; the root sits at the pose of t^{n+1}; the fluid is handed the
  wing of t^n;
* a wing with bending springs, one step from rest with no load: the
  implicit-Euler residual vanishes with the wing frame of t^{n+1} and not with
  that of t^n;
* a wing clamped at every vertex is the rigid revolving plate: the coupled
  fluid run equals the rigid-plate run of oracle.ns bit for bit;
* evidence for the areal-density reading: with mass ratio 1e-3 the lagged
  explicit coupling diverges within a few steps (added-mass instability),
  with density 1 it stays bounded.
"""

import math

import numpy as np
import pytest

from oracle import kinematics, structure
from oracle.coupling import CoupledOracle
from oracle.ns import OracleNS
import synth

N, BOX = (24, 24, 24), (12.0, 12.0, 12.0)
DX = BOX[0] / N[0]
TW, H = 2 * DX, DX


class StubFluid:
    """Stands in for the fluid of CoupledOracle: records the wing it is handed
    and leaves p(x, t) = g(t) a.x on the grid, with t = t^n after step() (the
    pressure of the step's nonlinear term) and t = t^{n+1} after nonlinear()
    (the pressure of the new velocity)."""

    def __init__(self, g, a):
        nx, ny, nz = N
        z, y, x = np.meshgrid(np.arange(nz) * DX, np.arange(ny) * DX, np.arange(nx) * DX, indexing="ij")
        self.X = (x, y, z)
        self.g, self.a = g, np.asarray(a, dtype=np.float64)
        self.t = 0.0
        self.seen = []
        self.p_last = None

    def _p(self, t):
        return self.g(t) * (self.a[0] * self.X[0] + self.a[1] * self.X[1] + self.a[2] * self.X[2])

    def set_wing(self, x, v, tri):
        self.seen.append((self.t, np.array(x), np.array(v)))

    def step(self, dt):
        self.p_last = self._p(self.t)
        self.t += dt
        return {"F": np.zeros(3)}

    def combined_mask(self):
        return None, None, None, None

    def nonlinear(self, chi, us, fw=None, sw=None):
        self.p_last = self._p(self.t)


def kin(t_ramp=0.4):
    return dict(alpha=math.pi / 4, omega=2 * math.pi, t_ramp=t_ramp, axis_point=(6.0, 6.0, 6.0))


def two_triangle_wing(density):
    s, c = synth.plate_span_chord(2, 2, 3.0, 1.0)
    return dict(span_coord=s, chord_coord=c, tri=synth.grid_triangles(2, 2), clamped=np.array([0, 2]),
                ext_ij=np.array([[0, 1], [2, 3], [0, 2], [1, 3], [0, 3]]), ext_k=np.zeros(5), density=density)


def tri_area_normal(p0, p1, p2):
    """A_T n_T of a triangle from its vertex order."""
    return 0.5 * np.cross(p1 - p0, p2 - p0)


@pytest.mark.parametrize("order", ["lagged", "paper"])
def test_loads_time_level_and_clamp_closed_form(order):
    g = lambda t: 1.0 + 40.0 * t  # noqa: E731
    a = np.array([0.3, -0.5, 0.8])
    d = TW + H
    dens = 0.7
    w = two_triangle_wing(dens)
    K = kin()
    co = CoupledOracle(N, BOX, 0.01, 1.0, TW, H, 0, w, np.zeros((0, 3), int), np.zeros(0), np.zeros(0, int), K,
                       order=order)
    co.fluid = StubFluid(g, a)
    tri = w["tri"]
    # masses lumped at rest: tip vertex 1 in one triangle, vertex 3 in two (each of area 1.5)
    x0 = co.q[0]
    A0 = np.linalg.norm(tri_area_normal(x0[0], x0[1], x0[3]))
    A1 = np.linalg.norm(tri_area_normal(x0[0], x0[3], x0[2]))
    assert A0 == pytest.approx(1.5) and A1 == pytest.approx(1.5)
    mass = {1: dens * A0 / 3, 3: dens * (A0 + A1) / 3}
    free = [1, 3]
    dts = [0.004, 0.006, 0.005, 0.0045]
    hist = [co.q.copy()]
    t = 0.0
    for n, dt in enumerate(dts):
        xn = co.q[0].copy()
        co.step(dt)
        # the fluid was handed the wing of t^n
        assert co.fluid.seen[n][0] == pytest.approx(t, abs=1e-15)
        assert np.array_equal(co.fluid.seen[n][1], xn)
        t1 = t + dt
        # root at the pose of t^{n+1}
        xr, vr = kinematics.plate_pose(w["span_coord"][[0, 2]], w["chord_coord"][[0, 2]], t1, K["alpha"],
                                       K["omega"], K["t_ramp"], K["axis_point"])
        assert np.max(np.abs(co.q[0][[0, 2]] - xr)) < 1e-14
        assert np.max(np.abs(co.q[1][[0, 2]] - vr)) < 1e-12
        # closed-form load on the wing of t^n: c_v = (1/3) sum A_T n_T,
        # dp_v = g (a . (2 d n_v)), load = -dp_v c_v
        an0 = tri_area_normal(xn[0], xn[1], xn[3])
        an1 = tri_area_normal(xn[0], xn[3], xn[2])
        c = {1: an0 / 3, 3: (an0 + an1) / 3}
        t_p = t if order == "lagged" else t1
        load = {v: -g(t_p) * float(a @ (2 * d * c[v] / np.linalg.norm(c[v]))) * c[v] for v in free}
        # ballistic BDF2 (implicit Euler on the first step) of the free tips
        al, be, ga = structure.bdf2_coefficients(dt, None if n == 0 else dts[n - 1])
        qp = hist[-2] if n > 0 else hist[-1]
        for v in free:
            v1 = al * hist[-1][1][v] - be * qp[1][v] + ga * dt * load[v] / mass[v]
            x1 = al * hist[-1][0][v] - be * qp[0][v] + ga * dt * v1
            assert np.max(np.abs(co.q[1][v] - v1)) < 1e-11 * np.max(np.abs(v1))
            assert np.max(np.abs(co.q[0][v] - x1)) < 1e-12 * np.max(np.abs(x1))
            # the test tells the time levels apart: the other level's load moves the tip by far more
            t_o = t1 if order == "lagged" else t
            lo = -g(t_o) * float(a @ (2 * d * c[v] / np.linalg.norm(c[v]))) * c[v]
            assert np.max(np.abs(ga * dt * (lo - load[v]) / mass[v])) > 1e-6
        hist.append(co.q.copy())
        t = t1


def test_bending_frame_at_new_time_level():
    """One step from rest at full rotation speed, no load: the implicit-Euler
    residual of the free vertices vanishes with the frame of t^{n+1} only.
    The tip column is swept forward so that the springs have nonzero rest
    angles (a straight spring's projected angles do not depend on the frame)."""
    s, c = synth.plate_span_chord(3, 2, 3.0, 1.0)
    c = c + np.array([0.0, 0.0, 0.3, 0.0, 0.0, 0.3])
    w = dict(span_coord=s, chord_coord=c, tri=synth.grid_triangles(3, 2), clamped=np.array([0, 1, 3, 4]),
             ext_ij=np.array([[0, 1], [1, 2], [3, 4], [4, 5], [0, 3], [1, 4], [2, 5], [0, 4], [1, 5]]),
             ext_k=np.full(9, 20.0), density=1.0)
    K = kin(t_ramp=0.0)
    co = CoupledOracle(N, BOX, 0.01, 1.0, TW, H, 0, w, np.array([[0, 1, 2], [3, 4, 5]]), np.array([50.0, 50.0]),
                       np.array([0, 0]), K)
    co.fluid = StubFluid(lambda t: 0.0, (0.0, 0.0, 0.0))
    x0, v0 = co.q[0].copy(), co.q[1].copy()
    dt = 0.01
    co.step(dt)
    x1, v1 = co.q
    free = [2, 5]
    m = co.net.mass[free][:, None]

    def residual(frame):
        f = structure.internal_forces(co.net, x1, frame)[free]
        return np.max(np.abs(m * (x1[free] - x0[free] - dt * v0[free]) / dt ** 2 - f))

    scale = np.max(np.abs(structure.internal_forces(co.net, x1, kinematics.plate_frame(dt, K["alpha"], K["omega"],
                                                                                         0.0))[free]))
    r_new = residual(kinematics.plate_frame(dt, K["alpha"], K["omega"], 0.0))
    r_old = residual(kinematics.plate_frame(0.0, K["alpha"], K["omega"], 0.0))
    assert np.max(np.abs(v1[free] - (x1[free] - x0[free]) / dt)) < 1e-10 * np.max(np.abs(v1[free]))
    assert r_new < 1e-8 * scale
    assert r_old > 1e-3 * scale


def test_all_clamped_wing_is_the_rigid_plate():
    cfg = synth.revolving_plate(n=24, t_ramp=0.05)
    s, c = synth.plate_span_chord(9, 4, 3.0, 1.0)
    tri = synth.grid_triangles(9, 4)
    w = dict(span_coord=s, chord_coord=c, tri=tri, clamped=np.arange(36), ext_ij=np.array([[0, 1]]),
             ext_k=np.ones(1), density=1.0)
    K = dict(alpha=cfg["alpha"], omega=cfg["omega"], t_ramp=cfg["t_ramp"], axis_point=cfg["axis_point"])
    co = CoupledOracle(cfg["n"], cfg["L"], cfg["nu"], cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"], w,
                       np.zeros((0, 3), int), np.zeros(0), np.zeros(0, int), K)
    o = OracleNS(cfg["n"], cfg["L"], cfg["nu"], cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"])
    co.fluid.set_velocity(np.zeros((3,) + cfg["n"]))
    o.set_velocity(np.zeros((3,) + cfg["n"]))
    t = 0.0
    for dt in (1.5e-3, 1.5e-3, 1.2e-3, 1.4e-3):
        x, v = kinematics.plate_pose(s, c, t, K["alpha"], K["omega"], K["t_ramp"], K["axis_point"])
        o.set_wing(x, v, tri)
        F = o.step(dt=dt)["F"]
        Fc = co.step(dt)
        assert np.array_equal(F, Fc)
        t += dt
    assert np.max(np.abs(F)) > 1e-3
    assert np.array_equal(o.uh, co.fluid.uh)


def _growth(density, steps, order):
    cfg = synth.revolving_plate(n=48, t_ramp=0.05)
    w = synth.flexible_wing(ns=11, nc=6, n_veins=3, vein_nodes=9, density=density)
    ijk, owner = synth.vein_bending(w)
    kb = np.array([structure.bending_stiffness(w["vein_EI"][v], w["vein_length"], len(w["veins"][v]) - 2)
                   for v in owner])
    K = dict(alpha=cfg["alpha"], omega=cfg["omega"], t_ramp=cfg["t_ramp"], axis_point=cfg["axis_point"])
    co = CoupledOracle(cfg["n"], cfg["L"], cfg["nu"], cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"], w, ijk, kb,
                       np.zeros(len(ijk), int), K, tol=1e-10, order=order)
    co.fluid.set_velocity(np.zeros((3,) + cfg["n"]))
    defl, force = [], []
    for _ in range(steps):
        try:
            F = co.step(2e-3)
        except RuntimeError:  # Newton failed: the structure blew up
            defl.append(np.inf)
            force.append(np.inf)
            break
        xr, _ = co._root_pose(co.t, None)
        defl.append(float(np.max(np.abs(co.q[0] - xr))))
        force.append(float(np.linalg.norm(F)))
    return np.array(defl), np.array(force)


@pytest.mark.parametrize("order", ["lagged", "paper"])
def test_explicit_coupling_diverges_for_a_light_wing(order):
    """Reading of the areal density (48^3, the small flexible wing of the GPU
    parity case): with density 1e-3 the explicit staggered coupling is unstable
    in either pressure order (added-mass instability: the force grows about
    30-fold per step and Newton fails within six steps), with density 1 the same
    run stays smooth."""
    light_d, light_f = _growth(1e-3, 6, order)
    heavy_d, heavy_f = _growth(1.0, 6, order)
    print(order, "density 1e-3: deflection", light_d, "force", light_f)
    print(order, "density 1:    deflection", heavy_d, "force", heavy_f)
    assert np.all(np.isfinite(heavy_d)) and heavy_d[-1] < 0.02 and np.max(heavy_f) < 10.0
    assert not np.isfinite(light_d[-1])
    f = light_f[2:][np.isfinite(light_f[2:])]
    assert len(f) >= 2 and np.all(f[1:] / f[:-1] > 10.0)
