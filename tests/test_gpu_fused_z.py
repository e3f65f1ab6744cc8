"""The first pass of a step (z inverse of u and of omega_x, omega_y) is fused into
the last pass of the previous step when nothing has replaced u_hat since.  These
tests check that the fused and the stand-alone pass give the same bits, and that
every call that replaces u_hat or reuses the work buffers drops the fused result.

A z length of 512 selects the compile-time 512-point column kernels, a z length
of 48 the run-time plan.
"""

import numpy as np
import pytest

from paper_2002_08642_amd import fsi
import synth

pytestmark = pytest.mark.gpu

CASES = [((32, 24, 512), (2.0, 1.5, 8.0)), ((40, 36, 48), (2.0, 1.8, 2.4))]


def solver(n, L, prec, pressure=False):
    s = fsi.Solver(n, L, 0.02, 0.05, 0.05, 0.03, fsi.PROFILE_COS, prec, pressure=pressure)
    rng = np.random.default_rng(3)
    centre = (0.5 * L[0] + 0.013, 0.5 * L[1] + 0.021, 0.5 * L[2] - 0.007)
    x, tri = synth.flat_rectangle(centre, np.array([1.0, 0.05, 0.02]) / np.linalg.norm([1.0, 0.05, 0.02]),
                                  np.array([0.0, 0.3, 1.0]) / np.linalg.norm([0.0, 0.3, 1.0]), 0.6, 0.3, 7, 4)
    v = rng.standard_normal(x.shape)
    s.set_spectrum(synth.random_solenoidal_compact(n, L, seed=7))
    s.set_wing(x, v, tri)
    return s


@pytest.mark.parametrize("prec", [fsi.PREC_FP32, fsi.PREC_FP64])
@pytest.mark.parametrize("n,L", CASES)
def test_fused_and_standalone_z_inverse_agree_bitwise(n, L, prec):
    a, b = solver(n, L, prec), solver(n, L, prec)
    for k in range(5):
        a.step(2e-3)
        b.step(2e-3)
        # save + load puts the same u_hat back: b's next step runs the stand-alone pass
        b.save(1)
        b.load(1)
    ua, ub = a.spectrum(), b.spectrum()
    print("n %s prec %d: max |u_a - u_b| = %.3e" % (n, prec, np.max(np.abs(ua - ub))), flush=True)
    assert np.array_equal(ua, ub)
    ia, ib = a.info(), b.info()
    assert np.array_equal(np.asarray(ia["F"]), np.asarray(ib["F"])) and ia["umax"] == ib["umax"]


@pytest.mark.parametrize("n,L", CASES)
def test_new_velocity_drops_the_fused_pass(n, L):
    """After two steps, a new spectrum must not be stepped with the old fused
    z inverse: the result equals that of a fresh solver given the same spectrum."""
    a = solver(n, L, fsi.PREC_FP64)
    a.step(2e-3)
    a.step(2e-3)
    u1 = synth.random_solenoidal_compact(n, L, seed=11)
    a.set_spectrum(u1)
    a.step(2e-3)
    b = solver(n, L, fsi.PREC_FP64)
    b.set_spectrum(u1)
    b.step(2e-3)
    assert np.array_equal(a.spectrum(), b.spectrum())


def test_pressure_transform_between_steps_keeps_the_fused_pass():
    """Sampling the pressure between steps runs single-field transforms on the
    work buffers; the following step is the same as without the sampling."""
    n, L = CASES[0]
    a = solver(n, L, fsi.PREC_FP64, pressure=True)
    b = solver(n, L, fsi.PREC_FP64, pressure=True)
    pts = np.array([[0.5 * L[0] + 0.1, 0.5 * L[1], 0.5 * L[2] + 0.2]])
    for k in range(3):
        a.step(2e-3)
        b.step(2e-3)
        a.sample_pressure(pts)
        a.velocity()  # three-field transform: drops the fused pass
    assert np.array_equal(a.spectrum(), b.spectrum())
