"""Parity at the full 512^3 size in the launch configuration bench.py times.

At this size the FP64 oracle cannot run a whole step inside a test, so the
checks are outputs it computes one by one, closed forms, and identities of the
discrete method that hold at any size:

* 2-D Taylor-Green at 512^3: the step (all passes, the compile-time 512-point
  kernels, the fused update/z-inverse pass) reproduces the exact decay
  exp(-2 nu t) for a random dt sequence (closed form, FP32 and FP64); the same
  at 800^3 (FP32), the largest configuration;
* the bench workload (k^-5/3 field, revolving plate at full speed, adaptive dt),
  first step in FP32:
  - mask chi and u_s at sampled grid points against the oracle's distance to
    the triangles (brute force over all triangles, point by point);
  - the velocity at sampled points against the direct sum over the stored
    spectrum (point by point, FP64);
  - E, u_max, the force and dt against their definitions on the device's own
    velocity and mask (the reductions and the CFL rule at full size);
  - the nonlinear term is solenoidal and does exactly the penalization work
    Re sum w conj(u_hat).N_hat = -(1/(eta N^3)) sum chi u.(u - u_s) (u x omega
    does none);
  - the update is the first (Euler) integrating-factor step of that term;
  - the nonlinear term at every stored mode against u x omega - (chi/eta)(u - u_s),
    truncated and projected, computed in FP64 from the same spectrum and mask
    with scipy's FFTs;
* the adjoint of two steps of the bench workload (the kernels the adjoint leg of
  bench.py times), without and with the sponge layers of the sponge leg: FP64
  against central differences of the FP64 forward map (dot-product test), FP32
  cotangents against the FP64 ones;
* the uniform sponge on 2-D Taylor-Green: the closed-form damped recurrence.
"""

import numpy as np
import pytest

from oracle import mask as omask
from paper_2002_08642_amd import fsi
from tests.helpers import rel_max
from tests.test_gpu_adjoint import run_two_steps
import bench
import synth

pytestmark = pytest.mark.gpu

N = 512


def compact_wavenumbers(s, L):
    """kx, ky, kz broadcastable to the compact shape (iz, iy, ix), band order."""
    nz_b, ny_b, nx_b = s.compact_shape
    Kz, Ky = (nz_b - 1) // 2, (ny_b - 1) // 2
    mz = np.concatenate([np.arange(Kz + 1), np.arange(-Kz, 0)])
    my = np.concatenate([np.arange(Ky + 1), np.arange(-Ky, 0)])
    mx = np.arange(nx_b)
    return (2 * np.pi * mx / L[0])[None, None, :], (2 * np.pi * my / L[1])[None, :, None], \
        (2 * np.pi * mz / L[2])[:, None, None]


# 800^3 (= 2^5 5^2, the largest configuration: run-time mixed-radix plans) in FP32
@pytest.mark.parametrize("m,prec", [(N, fsi.PREC_FP32), (N, fsi.PREC_FP64), (800, fsi.PREC_FP32)])
def test_fullsize_taylor_green_exact_decay(m, prec):
    n, L, nu = (m, m, m), (2 * np.pi,) * 3, 0.05
    print("%d^3 Taylor-Green" % m, prec, flush=True)
    s = fsi.Solver(n, L, nu, 1.0, precision=prec)
    u0 = synth.taylor_green_2d(n, L)
    s.set_velocity(u0)
    t = 0.0
    for dt in np.random.default_rng(9).uniform(1e-3, 2e-2, 4):
        s.step(dt)
        t += dt
    err = rel_max(s.velocity(), np.exp(-2 * nu * t) * u0)
    print("%d^3 Taylor-Green prec %d: %.3e" % (m, prec, err), flush=True)
    assert err < (1e-12 if prec == fsi.PREC_FP64 else 2e-6)


def test_fullsize_bench_first_step():
    cfg = bench.workload(N)
    n, L = cfg["n"], cfg["L"]
    print("512^3 bench workload, first step", flush=True)
    s = fsi.Solver(n, L, cfg["nu"], cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"], fsi.PREC_FP32)
    uh0 = synth.random_solenoidal_compact(n, L, seed=0)
    s.set_spectrum(uh0)
    x, v, _ = fsi.plate_pose(cfg["span_coord"], cfg["chord_coord"], 0.0, cfg["alpha"], cfg["omega"], 0.0,
                             cfg["axis_point"])
    tri = np.asarray(cfg["tri"])
    s.set_wing(x, v, tri)
    uh0 = s.spectrum()  # the stored (FP32-rounded) initial spectrum
    u0 = s.velocity()
    chi, us = s.mask()
    dx = L[0] / N
    rng = np.random.default_rng(17)

    # mask at sampled points: oracle distance to every triangle, lowest index wins ties
    inside = np.argwhere(chi > 0)
    pick = inside[rng.choice(len(inside), 300, replace=False)]
    lo = np.floor((x.min(0) - cfg["tw"] - cfg["h"]) / dx).astype(int)
    hi = np.ceil((x.max(0) + cfg["tw"] + cfg["h"]) / dx).astype(int)
    extra = np.stack([rng.integers(lo[2], hi[2], 100), rng.integers(lo[1], hi[1], 100),
                      rng.integers(lo[0], hi[0], 100)], axis=1)
    idx = np.concatenate([pick, extra])  # (z, y, x)
    pts = idx[:, ::-1] * dx
    best = np.full(len(pts), np.inf)
    wb = np.zeros((len(pts), 3))
    tb = np.zeros(len(pts), dtype=np.int64)
    for t in range(len(tri)):
        d, w = omask.point_triangle(pts, x[tri[t, 0]], x[tri[t, 1]], x[tri[t, 2]])
        upd = d < best
        best[upd], wb[upd], tb[upd] = d[upd], w[upd], t
    r = omask.support_radius(cfg["tw"], cfg["h"], cfg["profile"])
    ins = best < r
    chi_o = np.where(ins, omask.chi_profile(np.where(ins, best, 0.0), cfg["tw"], cfg["h"], cfg["profile"]), 0.0)
    us_o = np.where(ins[:, None], np.einsum("pk,pkc->pc", wb, v[tri[tb]]), 0.0)
    chi_g = chi[idx[:, 0], idx[:, 1], idx[:, 2]]
    us_g = us[:, idx[:, 0], idx[:, 1], idx[:, 2]].T
    e_chi = np.max(np.abs(chi_g - chi_o))
    e_us = np.max(np.abs(us_g - us_o)) / np.max(np.abs(v))
    print("mask at %d points: chi %.3e u_s %.3e" % (len(pts), e_chi, e_us), flush=True)
    assert e_chi < 1e-6 and e_us < 1e-5

    # velocity at sampled points: direct FP64 sum over the stored band
    kx, ky, kz = compact_wavenumbers(s, L)
    wgt = np.where(kx == 0, 1.0, 2.0)
    umax_abs = np.max(np.abs(u0))
    for p in rng.integers(0, N, (3, 3)):
        ph = np.exp(1j * (kx * (p[0] * dx) + ky * (p[1] * dx) + kz * (p[2] * dx))) * wgt
        uo = np.array([np.sum(uh0[c] * ph).real for c in range(3)])
        eu = np.max(np.abs(u0[:, p[2], p[1], p[0]] - uo)) / umax_abs
        assert eu < 1e-5, (p, eu)

    s.step_adaptive(cfg["cfl"], cfg["c_eta"], cfg["dt_max"])
    info = s.info()
    nh0 = s.nonlinear()
    uh1 = s.spectrum()

    # reductions and the CFL rule on the device's own fields
    dV = dx ** 3
    speed2 = np.sum(u0 * u0, axis=0)
    E = 0.5 * dV * np.sum(speed2)
    umax = np.sqrt(np.max(speed2))
    slip = u0 - us
    F = (dV / cfg["eta"]) * np.array([np.sum(chi * slip[c]) for c in range(3)])
    dt = min(cfg["cfl"] * dx / info["umax"], cfg["c_eta"] * cfg["eta"], cfg["dt_max"])
    print("E %.3e umax %.3e F %.3e dt %.3e" % (abs(info["E"] / E - 1), abs(info["umax"] / umax - 1),
                                               rel_max(np.asarray(info["F"]), F), abs(info["dt"] / dt - 1)),
          flush=True)
    assert info["E"] == pytest.approx(E, rel=1e-6)
    assert info["umax"] == pytest.approx(umax, rel=1e-6)
    assert rel_max(np.asarray(info["F"]), F) < 1e-5
    assert info["dt"] == pytest.approx(dt, rel=1e-12)

    # the nonlinear term: solenoidal, and the work it does is the penalization's
    k2 = kx * kx + ky * ky + kz * kz
    div = np.abs(kx * nh0[0] + ky * nh0[1] + kz * nh0[2])
    assert np.max(div) <= 1e-5 * np.max(np.sqrt(k2) * np.max(np.abs(nh0), axis=0))
    work = float(np.sum(wgt * np.real(np.conj(uh0) * nh0)))
    pen = -float(np.sum(chi * np.sum(u0 * slip, axis=0))) / (cfg["eta"] * N ** 3)
    scale = float(np.sum(wgt * np.abs(uh0) * np.abs(nh0)))
    print("work %.6e penalization %.6e (scale %.3e)" % (work, pen, scale), flush=True)
    assert abs(work - pen) < 1e-5 * scale

    # first step: integrating-factor Euler
    expect = np.exp(-cfg["nu"] * k2 * info["dt"]) * (uh0 + info["dt"] * nh0)
    eup = rel_max(uh1, expect)
    print("update %.3e" % eup, flush=True)
    assert eup < 1e-6


def _band_to_half(c, n):
    """Compact band (2Kz+1, 2Ky+1, Kx+1) -> half spectrum (nz, ny, nx//2+1), zero elsewhere."""
    nx, ny, nz = n
    Kz, Ky = (c.shape[0] - 1) // 2, (c.shape[1] - 1) // 2
    iz = np.concatenate([np.arange(Kz + 1), np.arange(nz - Kz, nz)])
    iy = np.concatenate([np.arange(Ky + 1), np.arange(ny - Ky, ny)])
    h = np.zeros((nz, ny, nx // 2 + 1), dtype=np.complex128)
    h[np.ix_(iz, iy, np.arange(c.shape[2]))] = c
    return h, iz, iy


@pytest.mark.parametrize("N", [512, 800])
def test_fullsize_nonlinear_elementwise(N):
    """The nonlinear term of the bench workload's first step at 512^3 and at
    800^3 (FP32), every stored mode: against u x omega - (chi/eta)(u - u_s),
    2/3-truncated and projected, computed in FP64 from the same stored spectrum
    and the device's mask with scipy's FFTs (an independent transform library)."""
    import scipy.fft as sfft
    cfg = bench.workload(N)
    n, L = cfg["n"], cfg["L"]
    print("%d^3 nonlinear term, element by element" % N, flush=True)
    s = fsi.Solver(n, L, cfg["nu"], cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"], fsi.PREC_FP32)
    s.set_spectrum(synth.random_solenoidal_compact(n, L, seed=0))
    x, v, _ = fsi.plate_pose(cfg["span_coord"], cfg["chord_coord"], 0.0, cfg["alpha"], cfg["omega"], 0.0,
                             cfg["axis_point"])
    s.set_wing(x, v, np.asarray(cfg["tri"]))
    uh0 = s.spectrum()
    chi, us = s.mask()
    s.step_adaptive(cfg["cfl"], cfg["c_eta"], cfg["dt_max"])
    nh0 = s.nonlinear()
    del s
    kx, ky, kz = compact_wavenumbers(_Shape(uh0.shape[1:]), L)
    N3 = float(N) ** 3
    W = 16

    def to_grid(c):
        h, _, _ = _band_to_half(c, n)
        return sfft.irfftn(h, s=(N, N, N), workers=W) * N3

    u = [to_grid(uh0[q]) for q in range(3)]
    # omega_hat = i k x u_hat on the band
    w = [to_grid(1j * (ky * uh0[2] - kz * uh0[1])), to_grid(1j * (kz * uh0[0] - kx * uh0[2])),
         to_grid(1j * (kx * uh0[1] - ky * uh0[0]))]
    ce = chi / cfg["eta"]
    g = [u[1] * w[2] - u[2] * w[1] - ce * (u[0] - us[0]),
         u[2] * w[0] - u[0] * w[2] - ce * (u[1] - us[1]),
         u[0] * w[1] - u[1] * w[0] - ce * (u[2] - us[2])]
    del u, w
    _, iz, iy = _band_to_half(uh0[0], n)
    gh = []
    for q in range(3):
        full = sfft.rfftn(g[q], workers=W) / N3
        gh.append(full[np.ix_(iz, iy, np.arange(uh0.shape[3]))])
        g[q] = None
    gh = np.array(gh)
    k2 = kx * kx + ky * ky + kz * kz
    kdot = (kx * gh[0] + ky * gh[1] + kz * gh[2]) / np.where(k2 > 0, k2, 1.0)
    ref = np.array([gh[0] - kx * kdot, gh[1] - ky * kdot, gh[2] - kz * kdot])
    err = rel_max(nh0, ref)
    print("nonlinear term, %d modes: max relative difference %.3e" % (ref.size, err), flush=True)
    assert np.max(np.abs(ref)) > 1.0
    assert err < 1e-5  # the FP32 velocity bar


class _Shape:
    """Stand-in with the compact shape, for compact_wavenumbers."""

    def __init__(self, shape):
        self.compact_shape = tuple(shape)


@pytest.mark.parametrize("prec", [fsi.PREC_FP32, fsi.PREC_FP64])
def test_fullsize_uniform_sponge_recurrence(prec):
    """chi_sp = 1 on the 2-D Taylor-Green field at 512^3: the scalar IF-AB2
    recurrence of a linear damping 1/C_sp (closed form; the sponge kernels of the
    bench's sponge leg at full size)."""
    n, L, nu, c_sp = (N, N, N), (2 * np.pi,) * 3, 0.02, 0.3
    s = fsi.Solver(n, L, nu, 1.0, precision=prec)
    u0 = synth.taylor_green_2d(n, L)
    s.set_velocity(u0)
    s.set_sponge(c_sp, gx=np.ones(N))
    a_prev, a, dt_prev = None, 1.0, None
    for dt in np.random.default_rng(4).uniform(0.005, 0.03, 4):
        s.step(dt)
        en = np.exp(-2 * nu * dt)
        if a_prev is None:
            a_new = en * (1 - dt / c_sp) * a
        else:
            xi = dt / dt_prev
            ep = np.exp(-2 * nu * dt_prev)
            a_new = en * (1 - dt * (1 + xi / 2) / c_sp) * a + dt * (xi / 2) / c_sp * en * ep * a_prev
        a_prev, a, dt_prev = a, a_new, dt
    err = rel_max(s.velocity(), a * u0)
    print("512^3 uniform sponge prec %d: %.3e" % (prec, err), flush=True)
    assert err < (1e-12 if prec == fsi.PREC_FP64 else 2e-6)


@pytest.mark.parametrize("sponge", [False, True], ids=["plain", "sponge"])
def test_fullsize_adjoint_two_steps(sponge):
    cfg = bench.workload(N)
    n, L = cfg["n"], cfg["L"]
    x, v, _ = fsi.plate_pose(cfg["span_coord"], cfg["chord_coord"], 0.0, cfg["alpha"], cfg["omega"], 0.0,
                             cfg["axis_point"])
    tri = np.asarray(cfg["tri"])
    rng = np.random.default_rng(29)
    # jittered off the flat plate, so that no grid point is equidistant from two
    # triangles (where the distance to the mesh has a kink)
    x = x + 2e-3 * rng.standard_normal(x.shape)
    u0 = synth.random_solenoidal_compact(n, L, seed=0)
    du = synth.random_solenoidal_compact(n, L, seed=1)
    dx = 1e-3 * rng.standard_normal(x.shape)
    dv = rng.standard_normal(x.shape)
    g = [rng.standard_normal(3), rng.standard_normal(3)]
    lam_u = rng.standard_normal(u0.shape) + 1j * rng.standard_normal(u0.shape)
    lam_n = rng.standard_normal(u0.shape) + 1j * rng.standard_normal(u0.shape)
    dts = (1.0e-4, 1.2e-4)
    out = {}
    for prec in (fsi.PREC_FP64, fsi.PREC_FP32):
        print("512^3 adjoint, precision", prec, flush=True)
        s = fsi.Solver(n, L, cfg["nu"], cfg["eta"], cfg["tw"], cfg["h"], cfg["profile"], prec)
        if sponge:  # the layers of the bench's sponge leg
            gx, gz = bench.sponge_layers(N)
            s.set_sponge(bench.SPONGE_C, gx=gx, gz=gz)
        out[prec] = run_two_steps(s, u0, x, v, tri, dts, g, lam_u, lam_n, du, dx, dv)
        del s
    adj, fd, r64 = out[fsi.PREC_FP64]
    print("512^3 dot product FP64: adjoint %.12e fd %.12e" % (adj, fd), flush=True)
    assert abs(adj - fd) <= 1e-6 * max(abs(fd), 1e-8)
    r32 = out[fsi.PREC_FP32][2]
    for name, a32, a64 in zip(("lambda_u", "lambda_N", "dJ/dx", "dJ/dv"), r32, r64):
        ref = np.max(np.abs(a64))
        if name == "lambda_N":  # reversing the first (Euler) step leaves no N^{-1} cotangent
            assert ref == 0.0 and np.max(np.abs(a32)) == 0.0
            continue
        err = np.max(np.abs(a32 - a64)) / ref
        print("512^3 FP32 vs FP64 adjoint %s: %.3e" % (name, err), flush=True)
        assert err < 1e-4
