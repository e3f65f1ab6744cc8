"""Host wing loads from a pressure box and their transpose (include/fsi_ms.h).

The host loads equal the oracle's (oracle.pressure.wing_loads) on the same
grid pressure; fsi_loads_adjoint passes dot-product tests against central
differences with respect to the vertex positions and the box values.
"""

import numpy as np
import pytest

from oracle import pressure
from paper_2002_08642_amd import fsi
import synth


def setup(seed=0):
    n, L = 32, 4.0
    dx = L / n
    xs = np.arange(n) * dx
    Z, Y, X = np.meshgrid(xs, xs, xs, indexing="ij")
    p = np.sin(1.3 * X + 0.4) * np.cos(0.9 * Y - 0.2) + 0.3 * np.cos(1.7 * Z) + 0.1 * X * Y
    u_ax = np.array([1.0, 0.2, 0.1]) / np.linalg.norm([1.0, 0.2, 0.1])
    v_ax = np.cross([0.1, -0.3, 1.0], u_ax)
    v_ax /= np.linalg.norm(v_ax)
    x, tri = synth.flat_rectangle((2.03, 1.97, 2.01), u_ax, v_ax, 0.7, 0.4, 6, 4)
    rng = np.random.default_rng(seed)
    x = x + 0.02 * rng.standard_normal(x.shape)
    box0 = (4, 4, 4)
    pbox = p[4:28, 4:28, 4:28].copy()
    return p, (L, L, L), x, tri, np.full(3, dx), box0, pbox


def test_host_loads_match_oracle():
    p, L, x, tri, dx, box0, pbox = setup()
    d = 0.3
    lg, dpg = fsi.loads_from_box(x, tri, d, dx, box0, pbox)
    lo, dpo = pressure.wing_loads(p, L, x, tri, d)
    assert np.allclose(lg, lo, atol=1e-14, rtol=0) and np.allclose(dpg, dpo, atol=1e-14, rtol=0)


@pytest.mark.parametrize("part", ["x", "p"])
def test_loads_adjoint_dot_product(part):
    p, L, x, tri, dx, box0, pbox = setup(1)
    d = 0.3
    rng = np.random.default_rng(2)
    lam = rng.standard_normal(x.shape)
    dxv = rng.standard_normal(x.shape) if part == "x" else 0 * x
    dpb = rng.standard_normal(pbox.shape) if part == "p" else 0 * pbox

    def J(eps):
        loads, _ = fsi.loads_from_box(x + eps * dxv, tri, d, dx, box0, pbox + eps * dpb)
        return float(np.sum(lam * loads))

    eps = 1e-6
    fd = (J(eps) - J(-eps)) / (2 * eps)
    lx, lp = fsi.loads_adjoint(x, tri, d, dx, box0, pbox, lam)
    adj = float(np.sum(lx * dxv) + np.sum(lp * dpb))
    assert abs(adj - fd) <= 1e-7 * max(abs(fd), 1e-8), (adj, fd)
