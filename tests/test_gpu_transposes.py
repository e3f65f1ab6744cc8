"""The transposition rules the hand-written adjoint is built on, checked on the
library's transforms through the C ABI (inner products: real sum on physical
arrays, Re sum conj(a) b on the stored half spectrum):

    <mu, R2C f> = <f, N^-3 C2R(mu / m_k)>,   m_k = 1 on the k_x = 0 plane, 2 elsewhere,

for a random real f and a random complex mu on the stored band (not Hermitian on
the k_x = 0 plane): R2C^T = N^-3 C2R(. / m_k), equivalently C2R^T = N^3 m_k R2C.
Shapes with 512- and 800-point axes and generic lengths, both precisions.
"""

import numpy as np
import pytest

from paper_2002_08642_amd import fsi
import synth

pytestmark = pytest.mark.gpu

SHAPES = [(64, 48, 40), (512, 12, 10), (12, 512, 10), (10, 12, 512), (800, 12, 10), (36, 30, 50)]
TOL = {fsi.PREC_FP64: 1e-13, fsi.PREC_FP32: 2e-6}


@pytest.mark.parametrize("prec", [fsi.PREC_FP64, fsi.PREC_FP32])
@pytest.mark.parametrize("shape", SHAPES)
def test_r2c_transpose_is_scaled_c2r(shape, prec):
    nx, ny, nz = shape
    s = fsi.Solver(shape, (1.0, 1.3, 0.7), 0.0, 1.0, precision=prec)
    rng = np.random.default_rng(nx + 7 * ny + 13 * nz)
    f = synth.random_field((nz, ny, nx), seed=nx * 3 + ny)
    fh = s.fft_r2c(f)
    mu = rng.standard_normal(fh.shape) + 1j * rng.standard_normal(fh.shape)
    m = np.full(fh.shape[-1], 2.0)
    m[0] = 1.0
    g = s.fft_c2r(mu / m) / float(nx * ny * nz)
    lhs = float(np.sum((np.conj(mu) * fh).real))
    rhs = float(np.sum(f * g))
    scale = float(np.sqrt(np.sum(np.abs(mu) ** 2) * np.sum(np.abs(fh) ** 2)))
    print("transpose %s prec %d: <mu, R2C f> %.6e  <f, R2C^T mu> %.6e  rel %.2e"
          % (shape, prec, lhs, rhs, abs(lhs - rhs) / scale), flush=True)
    assert abs(lhs - rhs) <= TOL[prec] * scale
