"""Native FP64 mass-spring solver (include/fsi_ms.h) against the oracle.

Host code only (no GPU).  Forces, energy and projected angles agree with the
oracle to rounding; BDF2 steps with clamped points, external loads, a rotating
wing frame and variable dt agree with the oracle's Newton on the full phase
vector; the static cantilever reproduces the paper's printed table; Newton
converges quadratically (3-5 iterations) with the analytic Hessian.
"""

import os

import numpy as np
import pytest

from oracle import structure as st
from paper_2002_08642_amd import fsi

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cantilever_large_deflection.txt")


def rot(axis, ang):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K


def plate_network(ns=7, nc=4, seed=0, span=1.0, chord=0.4, chordwise=False):
    """A small plate: membrane extension springs on a grid with diagonals,
    spanwise bending springs on every chordwise row (and, if chordwise, springs
    along wing y on every spanwise column), root column clamped."""
    rng = np.random.default_rng(seed)
    s = np.linspace(0, span, ns)
    c = np.linspace(-chord / 2, chord / 2, nc)
    x = np.array([[si, ci, 0.0] for ci in c for si in s])
    x += 0.01 * rng.standard_normal(x.shape)
    idx = lambda i, j: j * ns + i
    ext = []
    for j in range(nc):
        for i in range(ns):
            for di, dj in ((1, 0), (0, 1), (1, 1)):
                if i + di < ns and j + dj < nc:
                    a, b = idx(i, j), idx(i + di, j + dj)
                    ext.append((a, b, 50.0 * (1 + rng.random()), np.linalg.norm(x[b] - x[a])))
    trip = [(idx(i - 1, j), idx(i, j), idx(i + 1, j)) for j in range(nc) for i in range(1, ns - 1)]
    th0 = st.bending_angles(x, trip, np.eye(3))
    bend = [(a, b, cc, 0.05 * (1 + rng.random()), t[0], t[1]) for (a, b, cc), t in zip(trip, th0)]
    if chordwise:
        ctrip = [(idx(i, j - 1), idx(i, j), idx(i, j + 1)) for i in range(ns) for j in range(1, nc - 1)]
        cth0 = st.bending_angles(x, ctrip, np.eye(3), axis=np.ones(len(ctrip), int))
        bend += [(a, b, cc, 0.08 * (1 + rng.random()), t[0], t[1], 1) for (a, b, cc), t in zip(ctrip, cth0)]
    mass = 0.01 * (1 + rng.random(ns * nc))
    clamped = [idx(0, j) for j in range(nc)]
    return mass, ext, bend, clamped, x


def native(mass, ext, bend, clamped):
    ms = fsi.MassSpring(mass)
    e = np.array(ext)
    ms.add_extension(e[:, :2], e[:, 2], e[:, 3])
    b = np.array([tuple(r) + (0,) * (7 - len(r)) for r in bend], dtype=float)
    ms.add_bending(b[:, :3], b[:, 3], b[:, 4:6], b[:, 6])
    ms.set_clamped(sorted(clamped))
    return ms


@pytest.mark.parametrize("chordwise", [False, True])
def test_forces_energy_and_angles_match_oracle(chordwise):
    mass, ext, bend, clamped, x0 = plate_network(seed=1, chordwise=chordwise)
    rng = np.random.default_rng(3)
    net = st.Network(mass, ext, bend, clamped)
    ms = native(mass, ext, bend, clamped)
    for trial in range(5):
        x = x0 + 0.05 * rng.standard_normal(x0.shape)
        F = rot(rng.standard_normal(3), rng.random())
        f, e = ms.forces(x, F)
        fo = st.internal_forces(net, x, F)
        assert np.max(np.abs(f - fo)) <= 1e-12 * np.max(np.abs(fo))
        assert e == pytest.approx(st.energy(net, x, F), rel=1e-13)
        assert np.allclose(ms.bending_angles(x, F), st.bending_angles(x, net.bend_ijk, F, net.bend_axis), atol=1e-14)


@pytest.mark.parametrize("chordwise", [False, True])
def test_bdf2_steps_match_oracle(chordwise):
    mass, ext, bend, clamped, x0 = plate_network(seed=2, chordwise=chordwise)
    clamped = sorted(clamped)
    net = st.Network(mass, ext, bend, clamped)
    ms = native(mass, ext, bend, clamped)
    rng = np.random.default_rng(4)
    v0 = 0.1 * rng.standard_normal(x0.shape)
    v0[clamped] = 0.0
    ms.set_state(x0, v0)
    q, q_prev, dtp = np.stack([x0, v0]), None, None
    omega = 2.0
    t = 0.0
    for n, dt in enumerate([0.01, 0.012, 0.009, 0.011, 0.01, 0.013]):
        t1 = t + dt
        F = rot([0, 0, 1], omega * t1)
        fext = np.zeros_like(x0)
        fext[:, 2] = 0.02 * np.sin(3 * t1 + np.arange(len(mass)))
        xc = x0[clamped] @ F.T
        vc = np.cross([0, 0, omega], xc)
        it = ms.step(dt, F, fext, xc, vc, tol=1e-13, max_iter=20)
        assert it <= 6
        q_new, _ = st.bdf2_step(net, q, q_prev, dt, dtp, F, fext, clamp_x=xc, clamp_v=vc, tol=1e-13)
        q_prev, q, dtp, t = q, q_new, dt, t1
        x, v = ms.state()
        assert np.max(np.abs(x - q[0])) <= 1e-10 * np.max(np.abs(q[0]))
        assert np.max(np.abs(v - q[1])) <= 1e-9 * np.max(np.abs(q[1]))


def test_static_cantilever_reproduces_the_printed_table():
    rows = np.loadtxt(GOLDEN, comments="#")
    net, x0 = st.cantilever(64, 0.3, 0.24, ke=1e9)
    ext = np.column_stack([net.ext_ij, net.ext_k, net.ext_l0])
    bend = np.column_stack([net.bend_ijk, net.bend_kb, net.bend_th0])
    for F, xr, yr, xm, ym, *_ in rows:
        ms = native(net.mass, ext, bend, net.clamped)
        ms.set_state(x0)
        fe = np.zeros_like(x0)
        fe[-1, 1] = -F
        ms.static(fe, load_steps=5, tol=1e-12)
        x, _ = ms.state()
        dx, dy = 100 * (x[-1, 0] - x[0, 0]), 100 * x[-1, 1]
        assert abs(dx - xm) <= 0.005 + 2e-3 * abs(xm) and abs(dy - ym) <= 0.005 + 2e-3 * abs(ym)
        assert abs(dx - xr) <= 0.01 * abs(xr) and abs(dy - yr) <= 0.01 * abs(yr)
    # and the same equilibrium as the oracle's (FD-Jacobian Newton) at the largest load
    fe = np.zeros_like(x0)
    fe[-1, 1] = -rows[-1, 0]
    xo = st.static_equilibrium(net, x0, np.eye(3), fe, clamp_x=x0[net.clamped], load_steps=5, tol=1e-12)
    assert np.max(np.abs(x - xo)) <= 1e-9


def test_small_deflection_tip_is_euler_bernoulli():
    for n in (1, 8, 64):
        net, x0 = st.cantilever(n, 0.3, 0.24, ke=1e9)
        ms = native(net.mass, np.column_stack([net.ext_ij, net.ext_k, net.ext_l0]),
                    np.column_stack([net.bend_ijk, net.bend_kb, net.bend_th0]), net.clamped)
        ms.set_state(x0)
        fe = np.zeros_like(x0)
        fe[-1, 1] = -1e-6
        ms.static(fe, load_steps=1, tol=1e-14)
        x, _ = ms.state()
        assert x[-1, 1] == pytest.approx(-1e-6 * 0.3 ** 3 / (3 * 0.24), rel=1e-7)


def test_error_paths():
    with pytest.raises(fsi.FsiError):
        fsi.MassSpring([1.0, 0.0])
    ms = fsi.MassSpring([1.0, 1.0, 1.0])
    with pytest.raises(fsi.FsiError):
        ms.add_extension([[0, 3]], [1.0], [1.0])
    with pytest.raises(fsi.FsiError):
        ms.add_extension([[0, 1]], [1.0], [0.0])
    with pytest.raises(fsi.FsiError):
        ms.add_bending([[0, 0, 1]], [1.0], [[0.0, 0.0]])
    with pytest.raises(fsi.FsiError):
        ms.set_clamped([0, 0])
    ms.add_extension([[0, 1], [1, 2]], [1e3, 1e3], [1.0, 1.0])
    ms.set_state(np.array([[0, 0, 0], [1.5, 0, 0], [2.0, 0.3, 0]], float))
    with pytest.raises(fsi.FsiError):
        ms.step(0.0)
    x_before, _ = ms.state()
    with pytest.raises(fsi.FsiError) as e:
        ms.step(0.1, tol=1e-15, max_iter=1)  # cannot converge in one iteration
    assert e.value.code == -5
    assert np.array_equal(ms.state()[0], x_before)  # unchanged on failure


def test_rest_state_stiffness_masses_and_frame_helpers():
    mass, ext, bend, clamped, x0 = plate_network(seed=5, chordwise=True)
    rng = np.random.default_rng(6)
    F = rot(rng.standard_normal(3), 0.7)
    x = x0 @ F.T + 0.01 * rng.standard_normal(x0.shape)
    e = np.array(ext)
    b = np.array([tuple(r) + (0,) * (7 - len(r)) for r in bend], dtype=float)
    ms = fsi.MassSpring(mass)
    ms.add_extension(e[:, :2], e[:, 2], np.ones(len(e)))
    ms.add_bending(b[:, :3], b[:, 3], None, b[:, 6])
    ms.set_state(x)
    ms.set_rest(F)
    net = st.rest_network(mass, x, e[:, :2].astype(int), e[:, 2], b[:, :3].astype(int), b[:, 3],
                          b[:, 6].astype(int), [], F)
    f, en = ms.forces(x, F)
    assert en < 1e-24 and np.max(np.abs(f)) < 1e-10  # at rest in its own configuration
    xp = x + 0.02 * rng.standard_normal(x.shape)
    assert np.allclose(ms.forces(xp, F)[0], st.internal_forces(net, xp, F), rtol=0, atol=1e-12)
    assert fsi.bending_stiffness(0.24, 0.3, 64) == pytest.approx(st.bending_stiffness(0.24, 0.3, 64), rel=1e-15)
    tri = np.array([[0, 1, 8], [1, 9, 8], [5, 6, 12]])
    assert np.allclose(fsi.lumped_masses(x, tri, 1e-3), st.lumped_masses(x, tri, 1e-3), rtol=1e-14, atol=0)
    from oracle import kinematics
    for t in (0.0, 0.1, 0.5):
        assert np.allclose(fsi.plate_frame(t, 0.7, 2 * np.pi, 0.4), kinematics.plate_frame(t, 0.7, 2 * np.pi, 0.4),
                           atol=1e-15)


def step_map(ms, x_n, v_n, hist, dt, F, fext, xc, vc, kext, kb):
    """q^{n+1} of one native step from a given state, history and parameters."""
    ms.set_extension_k(kext)
    ms.set_bending_k(kb)
    ms.set_state(x_n, v_n)
    if hist is not None:
        ms.set_history(*hist)
    ms.step(dt, F, fext, xc, vc, tol=1e-14, max_iter=40)
    return ms.state()


@pytest.mark.parametrize("first", [True, False])
@pytest.mark.parametrize("part", ["state", "prev", "load", "stiffness", "clamp", "frame"])
def test_structure_step_adjoint_dot_product(part, first):
    mass, ext, bend, clamped, x0 = plate_network(seed=7, chordwise=True)
    clamped = sorted(clamped)
    ms = native(mass, ext, bend, clamped)
    rng = np.random.default_rng(11)
    nv = len(mass)
    alpha = 0.4
    Fr = lambda a: rot([0, 0, 1], 0.3) @ rot([1, 0, 0], a)
    dFr = (Fr(alpha + 1e-7) - Fr(alpha - 1e-7)) / 2e-7
    x_n = x0 @ Fr(alpha).T + 0.02 * rng.standard_normal(x0.shape)
    v_n = 0.2 * rng.standard_normal(x0.shape)
    hist = None if first else (x_n - 0.01 * v_n + 0.001 * rng.standard_normal(x0.shape), v_n.copy(), 0.012)
    dt = 0.01
    fext = 0.05 * rng.standard_normal(x0.shape)
    xc = x_n[clamped] + 0.003
    vc = 0.1 * rng.standard_normal((len(clamped), 3))
    e = np.array(ext)
    b = np.array([tuple(r) + (0,) * (7 - len(r)) for r in bend], dtype=float)
    kext, kb = e[:, 2].copy(), b[:, 3].copy()
    lam_x, lam_v = rng.standard_normal((nv, 3)), rng.standard_normal((nv, 3))
    # perturbation direction
    d = dict(xn=0 * x_n, vn=0 * v_n, xp=0 * x_n, vp=0 * v_n, load=0 * fext, kext=0 * kext, kb=0 * kb,
             cx=0 * xc, cv=0 * vc, a=0.0)
    if part == "state":
        d["xn"], d["vn"] = rng.standard_normal(x_n.shape), rng.standard_normal(v_n.shape)
    elif part == "prev":
        if first:
            pytest.skip("no history on the implicit-Euler step")
        d["xp"], d["vp"] = rng.standard_normal(x_n.shape), rng.standard_normal(v_n.shape)
    elif part == "load":
        d["load"] = rng.standard_normal(fext.shape)
    elif part == "stiffness":
        d["kext"], d["kb"] = kext * rng.standard_normal(len(kext)), kb * rng.standard_normal(len(kb))
    elif part == "clamp":
        d["cx"], d["cv"] = rng.standard_normal(xc.shape), rng.standard_normal(vc.shape)
    else:
        d["a"] = 1.0

    def J(eps):
        h = None if hist is None else (hist[0] + eps * d["xp"], hist[1] + eps * d["vp"], hist[2])
        x1, v1 = step_map(ms, x_n + eps * d["xn"], v_n + eps * d["vn"], h, dt, Fr(alpha + eps * d["a"]),
                          fext + eps * d["load"], xc + eps * d["cx"], vc + eps * d["cv"],
                          kext + eps * d["kext"], kb + eps * d["kb"])
        return float(np.sum(lam_x * x1) + np.sum(lam_v * v1))

    # O(eps^2) truncation vs Newton tolerance (1e-14) / eps: random state moves are
    # strongly curved, the frame's effect is small
    eps = 3e-5 if part == "frame" else 1e-6
    fd = (J(eps) - J(-eps)) / (2 * eps)
    x1, _ = step_map(ms, x_n, v_n, hist, dt, Fr(alpha), fext, xc, vc, kext, kb)
    g = ms.step_adjoint(dt, None if first else hist[2], Fr(alpha), x1, lam_x, lam_v, dframe=dFr)
    adj = (np.sum(g["xn"] * d["xn"]) + np.sum(g["vn"] * d["vn"]) + np.sum(g["xp"] * d["xp"]) +
           np.sum(g["vp"] * d["vp"]) + np.sum(g["load"] * d["load"]) + np.sum(g["kext"] * d["kext"]) +
           np.sum(g["kb"] * d["kb"]) + np.sum(g["clamp_x"] * d["cx"]) + np.sum(g["clamp_v"] * d["cv"]) +
           g["dframe"] * d["a"])
    assert abs(adj - fd) <= 1e-6 * max(abs(fd), 1e-6), (adj, fd)


def test_plate_frame_dalpha_is_the_derivative():
    for t in (0.0, 0.21):
        h = 1e-6
        fd = (fsi.plate_frame(t, 0.7 + h, 2 * np.pi, 0.4) - fsi.plate_frame(t, 0.7 - h, 2 * np.pi, 0.4)) / (2 * h)
        assert np.allclose(fsi.plate_frame_dalpha(t, 0.7, 2 * np.pi, 0.4), fd, atol=1e-9)
