"""Pins of the mass-spring oracle (Sec. 2) against values the mathematics and
the paper fix.

* Forces are the exact negative gradient of the energy (central differences),
  internal forces sum to zero, and the extension force is the printed one.
* Projected bending angles of a planar polyline are its turning angles; a
  spring along another wing axis measures its angles in the permuted planes.
* Small-deflection cantilever: with k^b from the EI relation the tip deflection
  is F l^3 / (3 EI) (Euler-Bernoulli), the identity the relation is built on.
* Large deflection: the printed table (tests/golden) - the network's tip
  position agrees with the paper's mass-spring columns and, within the printed
  1 % error, with the nonlinear beam; the beam column itself is reproduced by
  an independent elastica shooting solution.
* BDF2 with variable steps converges at second order on a linear oscillator;
  the first step is implicit Euler; total momentum of a free network is conserved.
"""

import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.optimize import brentq

from oracle import structure as st

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cantilever_large_deflection.txt")


def random_network(seed, n=7):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 3))
    ext = [(i, i + 1, 1.0 + rng.random(), 0.8 + 0.4 * rng.random()) for i in range(n - 1)] + [(0, 3, 2.0, 1.0)]
    bend = [(i - 1, i, i + 1, 0.5 + rng.random(), 0.1 * rng.standard_normal(), 0.1 * rng.standard_normal(),
             i % 3) for i in range(1, n - 1)]  # springs along each wing axis
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    return st.Network(1.0 + rng.random(n), ext, bend), x, q


def test_forces_are_minus_energy_gradient():
    net, x, frame = random_network(0)
    f = st.internal_forces(net, x, frame)
    h = 1e-6
    g = np.zeros_like(x)
    for p in range(x.shape[0]):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[p, c] += h
            xm[p, c] -= h
            g[p, c] = (st.energy(net, xp, frame) - st.energy(net, xm, frame)) / (2 * h)
    assert np.max(np.abs(f + g)) < 1e-7 * max(1.0, np.max(np.abs(g)))


def test_internal_forces_sum_to_zero():
    net, x, frame = random_network(1)
    assert np.max(np.abs(st.internal_forces(net, x, frame).sum(axis=0))) < 1e-12


def test_extension_force_is_the_printed_law():
    # two points: F_i = k (|x_ij| - l0) e_ij, F_j = -F_i
    net = st.Network([1.0, 1.0], ext=[(0, 1, 3.0, 0.5)])
    x = np.array([[0.1, 0.2, 0.3], [1.1, -0.4, 0.7]])
    d = x[1] - x[0]
    L = np.linalg.norm(d)
    f = st.internal_forces(net, x, np.eye(3))
    assert np.allclose(f[0], 3.0 * (L - 0.5) * d / L, atol=1e-15)
    assert np.allclose(f[1], -f[0], atol=1e-15)


def test_axis_of_a_bending_spring_permutes_the_projection_planes():
    # a polyline along wing y, bent in the (y, z) plane, measured as an axis-1 spring
    x = np.array([[0.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 2.0, 0.3]])
    th = st.bending_angles(x, [(0, 1, 2)], np.eye(3), axis=[1])
    assert th[0, 0] == pytest.approx(np.arctan2(0.3, 1.0), abs=1e-15)  # plane (y, z)
    assert th[0, 1] == pytest.approx(0.0, abs=1e-15)                    # plane (y, x)


def test_projected_angles_of_planar_polyline_are_turning_angles():
    phis = np.array([0.2, 0.9, -0.4, 1.3])  # forward-going, as along a vein
    pts = np.concatenate([[[0.0, 0.0]], np.cumsum(np.stack([np.cos(phis), np.sin(phis)], 1), axis=0)])
    x = np.zeros((len(pts), 3))
    x[:, :2] = pts
    th = st.bending_angles(x, [(0, 1, 2), (1, 2, 3), (2, 3, 4)], np.eye(3))
    turn = np.angle(np.exp(1j * np.diff(phis)))
    assert np.allclose(th[:, 0], turn, atol=1e-14)
    assert np.allclose(th[:, 1], 0.0, atol=1e-14)


@pytest.mark.parametrize("n", [1, 4, 16])
def test_small_deflection_cantilever_matches_euler_bernoulli(n):
    L, EI, F = 0.3, 0.24, 1e-6
    net, x0 = st.cantilever(n, L, EI, ke=1e9)
    fe = np.zeros_like(x0)
    fe[-1, 1] = -F
    x = st.static_equilibrium(net, x0, np.eye(3), fe, clamp_x=x0[net.clamped], load_steps=1)
    assert x[-1, 1] == pytest.approx(-F * L ** 3 / (3 * EI), rel=1e-8)


def golden_rows():
    return np.loadtxt(GOLDEN, comments="#")


def elastica_tip(F, L, EI):
    """Inextensible cantilever with a downward tip load F: the bending moment
    EI theta' = -F (x_tip - x(s)) gives EI theta'' = F cos theta, with
    theta(0) = 0 and theta'(L) = 0 (shooting on theta'(0)); returns the tip
    position (x, y)."""

    def shoot(k0):
        sol = solve_ivp(lambda s, y: [y[1], F / EI * np.cos(y[0]), np.cos(y[0]), np.sin(y[0])],
                        (0, L), [0.0, k0, 0.0, 0.0], rtol=1e-12, atol=1e-14)
        return sol.y[:, -1]

    k0 = brentq(lambda k: shoot(k)[1], -F * L / EI * 1.5, 0.0)
    end = shoot(k0)
    return end[2], end[3]


def test_golden_beam_column_is_the_elastica():
    for F, xr, yr, *_ in golden_rows():
        x, y = elastica_tip(F, 0.3, 0.24)
        # printed to 0.01; the printed beam values come from elliptic integrals
        # and agree with this shooting solution to 0.02 (0.2 %)
        assert abs(100 * x - xr) <= 0.02 and abs(100 * y - yr) <= 0.02


@pytest.mark.slow
def test_large_deflection_table():
    rows = golden_rows()
    net, x0 = st.cantilever(64, 0.3, 0.24, ke=1e9)
    for F, xr, yr, xm, ym, ex, ey in rows:
        fe = np.zeros_like(x0)
        fe[-1, 1] = -F
        x = st.static_equilibrium(net, x0, np.eye(3), fe, clamp_x=x0[net.clamped], load_steps=5, tol=1e-10)
        dx, dy = 100 * (x[-1, 0] - x[0, 0]), 100 * x[-1, 1]
        print("F %.2f: network (%.3f, %.3f), paper network (%.2f, %.2f), beam (%.2f, %.2f)" % (F, dx, dy, xm, ym, xr, yr))
        # the paper's own network, to its print precision plus 0.2 %
        assert abs(dx - xm) <= 0.005 + 2e-3 * abs(xm) and abs(dy - ym) <= 0.005 + 2e-3 * abs(ym)
        # the continuum beam, within the printed error bound (<= 1 %)
        assert abs(dx - xr) <= 0.01 * abs(xr) and abs(dy - yr) <= 0.01 * abs(yr)


def oscillator_error(h, T=2.0):
    # point 1 on a spring of stiffness k from the clamped point 0: x = l0 + A cos(w t)
    k, m, l0, A = 4.0, 1.0, 1.0, 0.1
    net = st.Network([1.0, m], ext=[(0, 1, k, l0)], clamped=[0])
    q = np.zeros((2, 2, 3))
    q[0, 1, 0] = l0 + A
    q_prev = None
    t, dt_prev, n = 0.0, None, 0
    while t < T - 1e-12:
        dt = min(h * (1.0 + 0.3 * np.sin(1.7 * n)), T - t)
        q_new, _ = st.bdf2_step(net, q, q_prev, dt, dt_prev, np.eye(3), np.zeros((2, 3)),
                                clamp_x=np.zeros((1, 3)), clamp_v=np.zeros((1, 3)))
        q_prev, q, dt_prev, t, n = q, q_new, dt, t + dt, n + 1
    w = np.sqrt(k / m)
    return abs(q[0, 1, 0] - (l0 + A * np.cos(w * T)))


def test_bdf2_variable_steps_converge_at_second_order():
    e1, e2, e3 = oscillator_error(0.02), oscillator_error(0.01), oscillator_error(0.005)
    assert 3.4 < e1 / e2 < 4.6 and 3.4 < e2 / e3 < 4.6


def test_first_step_is_implicit_euler():
    # linear spring, one step: x1 = x0 + dt v1, m v1 = m v0 + dt F(x1)
    k, m, dt = 3.0, 2.0, 0.1
    net = st.Network([1.0, m], ext=[(0, 1, k, 1.0)], clamped=[0])
    q = np.zeros((2, 2, 3))
    q[0, 1, 0] = 1.2
    q[1, 1, 0] = 0.5
    q1, _ = st.bdf2_step(net, q, None, dt, None, np.eye(3), np.zeros((2, 3)), clamp_x=np.zeros((1, 3)),
                         clamp_v=np.zeros((1, 3)))
    # eliminate v1: (1 + dt^2 k / m) x1 = x0 + dt v0 + dt^2 k l0 / m
    x1 = (1.2 + dt * 0.5 + dt * dt * k * 1.0 / m) / (1 + dt * dt * k / m)
    assert q1[0, 1, 0] == pytest.approx(x1, rel=1e-13)
    assert q1[1, 1, 0] == pytest.approx((x1 - 1.2) / dt, rel=1e-11)


def test_free_network_conserves_momentum():
    net, x, frame = random_network(2)
    rng = np.random.default_rng(5)
    q = np.stack([x, rng.standard_normal(x.shape)])
    p0 = (net.mass[:, None] * q[1]).sum(axis=0)
    q_prev, dtp = None, None
    for dt in (0.01, 0.013, 0.008):
        qn, _ = st.bdf2_step(net, q, q_prev, dt, dtp, frame, np.zeros_like(x))
        q_prev, q, dtp = q, qn, dt
    assert np.allclose((net.mass[:, None] * q[1]).sum(axis=0), p0, atol=1e-11)
