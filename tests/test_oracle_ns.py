"""Pins of the oracle's time step (Sec. 4.1, penalized NS + Adams-Bashforth with adaptive dt).

Closed forms (Taylor-Green decay), energy identities of the nonlinear and
penalization terms, the scalar recurrence of a uniform mask, the force of a
uniform flow, the adaptive-dt rule and the rigid-mask limit trend.
"""

import numpy as np
import pytest

from oracle import ns, mask, dft
import synth


def test_taylor_green_2d_exact_decay_any_dt_sequence(rng):
    n = (16, 16, 8)
    L = (2 * np.pi,) * 3
    nu = 0.05
    o = ns.OracleNS(n, L, nu, eta=1.0)
    u0 = synth.taylor_green_2d(n, L)
    o.set_velocity(u0)
    t = 0.0
    for dt in rng.uniform(1e-3, 2e-2, 12):
        o.step(dt=dt)
        t += dt
        err = np.max(np.abs(o.velocity() - np.exp(-2 * nu * t) * u0))
        assert err < 1e-13


def test_taylor_green_3d_energy_decay():
    cfg = synth.config0(False)
    o = ns.OracleNS(cfg["n"], cfg["L"], cfg["nu"], cfg["eta"])
    o.set_velocity(synth.taylor_green_3d(cfg["n"], cfg["L"]))
    e0 = None
    t = 0.0
    for _ in range(cfg["steps"]):
        d = o.step(dt=cfg["dt"])
        if e0 is None:
            e0 = d["E"]
            assert e0 == pytest.approx((2 * np.pi) ** 3 / 8, rel=1e-14)
        else:
            assert d["E"] / e0 == pytest.approx(np.exp(-6 * cfg["nu"] * t), abs=1e-6)
        t += d["dt"]


def _sum_conj(a, b):
    return float(np.real(np.sum(np.conj(a) * b)))


def test_nonlinear_term_does_no_work(rng):
    n = (16, 12, 10)
    L = (2.0, 1.5, 1.2)
    o = ns.OracleNS(n, L, nu=0.0, eta=1.0)
    o.set_velocity(synth.random_solenoidal(n, L, seed=4))
    nx, ny, nz = n
    nh, _ = o.nonlinear(np.zeros((nz, ny, nx)), np.zeros((3, nz, ny, nx)))
    scale = np.sqrt(_sum_conj(o.uh, o.uh) * _sum_conj(nh, nh))
    assert abs(_sum_conj(o.uh, nh)) < 1e-13 * scale


def test_penalization_energy_identity(rng):
    n = (16, 12, 10)
    L = (2.0, 1.5, 1.2)
    eta = 0.3
    o = ns.OracleNS(n, L, nu=0.0, eta=eta)
    o.set_velocity(synth.random_solenoidal(n, L, seed=5))
    nx, ny, nz = n
    chi = rng.uniform(0, 1, (nz, ny, nx))
    us = rng.standard_normal((3, nz, ny, nx))
    nh, _ = o.nonlinear(chi, us)
    u = o.velocity()
    expect = -np.sum(chi * np.sum(u * (u - us), axis=0)) / (eta * nx * ny * nz)
    assert _sum_conj(o.uh, nh) == pytest.approx(expect, rel=1e-12)


def test_uniform_mask_scalar_recurrence(rng):
    n = (16, 16, 8)
    L = (2 * np.pi,) * 3
    nu, eta, c = 0.02, 0.05, 0.7
    o = ns.OracleNS(n, L, nu, eta)
    u0 = synth.taylor_green_2d(n, L)
    o.set_velocity(u0)
    nx, ny, nz = n
    chi = np.full((nz, ny, nx), c)
    us = np.zeros((3, nz, ny, nx))
    a_prev, a = None, 1.0
    dt_prev = None
    for dt in rng.uniform(0.005, 0.03, 10):
        o.step(dt=dt, mask_override=(chi, us))
        en = np.exp(-2 * nu * dt)
        if a_prev is None:
            a_new = en * (1 - dt * c / eta) * a
        else:
            xi = dt / dt_prev
            ep = np.exp(-2 * nu * dt_prev)
            a_new = en * (1 - dt * (1 + xi / 2) * c / eta) * a + dt * (xi / 2) * (c / eta) * en * ep * a_prev
        a_prev, a, dt_prev = a, a_new, dt
        assert np.max(np.abs(o.velocity() - a * u0)) < 1e-13


def test_force_of_uniform_flow_through_static_mask():
    cfg = synth.config0(True)
    n, L = cfg["n"], cfg["L"]
    o = ns.OracleNS(n, L, 0.0, cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"])
    U = np.array([0.3, -0.2, 0.1])
    nx, ny, nz = n
    o.set_velocity(np.broadcast_to(U[:, None, None, None], (3, nz, ny, nx)).copy())
    x, v, tri = cfg["wing"]
    o.set_wing(x, v, tri)
    chi, _ = o.mask()
    d = o.step(dt=1e-4)
    dV = np.prod(np.array(L) / np.array(n))
    assert np.allclose(d["F"], dV / cfg["eta"] * U * np.sum(chi), rtol=1e-12, atol=0)


def test_adaptive_dt_closed_form():
    n = (16, 16, 16)
    L = (2 * np.pi, 4.0, 3.0)
    o = ns.OracleNS(n, L, 0.01, 1e-2)
    o.set_velocity(synth.taylor_green_3d(n, L))
    umax = float(np.max(np.sqrt(np.sum(o.velocity() ** 2, axis=0))))
    d = o.step(cfl=0.1, c_eta=10.0, dt_max=1.0)
    assert d["umax"] == pytest.approx(umax, rel=1e-14)
    assert d["dt"] == pytest.approx(0.1 * (3.0 / 16) / umax, rel=1e-14)
    d = o.step(cfl=0.1, c_eta=2.0 / 3.0, dt_max=1.0)
    assert d["dt"] == 2.0 / 3.0 * 1e-2
    o2 = ns.OracleNS(n, L, 0.01, 1e-2)
    d = o2.step(cfl=0.1, c_eta=1e9, dt_max=0.25)
    assert d["umax"] == 0.0 and d["dt"] == 0.25


def test_rigid_mask_limit_trend():
    # Tangential uniform flow past a thick smooth slab (well resolved, so the
    # residual is set by the penalization and not by spectral truncation): at a
    # fixed time the velocity left inside the solid shrinks as eta -> 0
    # (Darcy-type convergence of volume penalization).
    n = (64, 4, 4)
    L = (2 * np.pi,) * 3
    x = np.arange(64) * L[0] / 64
    chi1 = 0.5 * (1 - np.tanh((np.abs(x - np.pi) - 1.0) / 0.2))
    chi = np.broadcast_to(chi1[None, None, :], (4, 4, 64)).copy()
    us = np.zeros((3, 4, 4, 64))
    res = []
    for eta in (1e-2, 1e-3, 1e-4):
        o = ns.OracleNS(n, L, 0.05, eta)
        u0 = np.zeros((3, 4, 4, 64))
        u0[1] = 1.0
        o.set_velocity(u0)
        dt = min(2.0 / 3.0 * eta, 1e-2)
        for _ in range(int(round(0.2 / dt))):
            o.step(dt=dt, mask_override=(chi, us))
        u = o.velocity()
        res.append(np.max(np.sqrt(np.sum(u * u, axis=0))[chi > 0.999]))
    assert res[0] > res[1] > res[2]
    assert res[2] < 1e-4


def test_config0_plate_run_stays_bounded():
    cfg = synth.config0(True)
    o = ns.OracleNS(cfg["n"], cfg["L"], cfg["nu"], cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"])
    o.set_velocity(synth.taylor_green_3d(cfg["n"], cfg["L"]))
    x, v, tri = cfg["wing"]
    o.set_wing(x, v, tri)
    es = [o.step(dt=cfg["dt"])["E"] for _ in range(cfg["steps"])]
    assert all(np.isfinite(es))
    assert es[-1] < es[0]


def test_save_load_roundtrip():
    n = (8, 8, 8)
    L = (2 * np.pi,) * 3
    o = ns.OracleNS(n, L, 0.01, 1.0)
    o.set_velocity(synth.taylor_green_3d(n, L))
    o.step(dt=0.01)
    s = o.save()
    o.step(dt=0.02)
    a = o.velocity()
    o.load(s)
    o.step(dt=0.02)
    assert np.array_equal(a, o.velocity())
    assert np.max(np.abs(dft.forward(a).imag)) < 1.0


def _compact_to_full(uh_c, n):
    """Hermitian extension of the compact half-band layout (test helper)."""
    nx, ny, nz = n
    Kx, Ky, Kz = (nx - 1) // 3, (ny - 1) // 3, (nz - 1) // 3
    full = np.zeros((3, nz, ny, nx), dtype=np.complex128)
    mz = np.concatenate([np.arange(Kz + 1), np.arange(-Kz, 0)])
    my = np.concatenate([np.arange(Ky + 1), np.arange(-Ky, 0)])
    for a, zz in enumerate(mz):
        for b, yy in enumerate(my):
            full[:, zz % nz, yy % ny, :Kx + 1] = uh_c[:, a, b, :]
            full[:, (-zz) % nz, (-yy) % ny, (nx - np.arange(1, Kx + 1)) % nx] = np.conj(uh_c[:, a, b, 1:])
    return full


@pytest.mark.parametrize("L", [(2 * np.pi,) * 3, (3.0, 3.0, 3.0)])
def test_beltrami_exact_decay_any_dt_sequence(L, rng):
    """Helical modes of one |k| (on every axis, z included): curl u = |k| u, so
    u x omega = 0 pointwise and the step leaves only exp(-nu |k|^2 t)."""
    from oracle import spectral
    n = (24, 24, 24)
    nu = 0.03
    modes = synth.beltrami_modes(n, L, 6, seed=1)  # |m|^2 = 6: (1,1,2) and permutations
    assert {abs(m[0][2]) for m in modes} == {1, 2}
    full = _compact_to_full(synth.modes_to_compact(n, modes), n)
    kmag = 2 * np.pi / L[0] * np.sqrt(6.0)
    # the generator's field is real and a curl eigenfunction
    u0 = dft.inverse_real(full)
    assert np.max(np.abs(dft.forward(u0) - full)) < 1e-14 * np.max(np.abs(full))
    w0 = dft.inverse_real(spectral.curl(full, n, L))
    assert np.max(np.abs(w0 - kmag * u0)) < 1e-12 * kmag * np.max(np.abs(u0))
    o = ns.OracleNS(n, L, nu, eta=1.0)
    o.set_velocity(u0)
    t = 0.0
    for dt in rng.uniform(1e-3, 2e-2, 6):
        o.step(dt=dt)
        t += dt
    assert np.max(np.abs(o.velocity() - np.exp(-nu * kmag ** 2 * t) * u0)) < 1e-13 * np.max(np.abs(u0))
