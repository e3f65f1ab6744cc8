"""Pressure and wing loads of the FSI coupling (oracle; test infrastructure only).

Sec. 4.1 (pressure interpolation and staggered scheme paragraphs): the total
pressure Pi = p + |u|^2/2 of the penalized equations is the part of the
nonlinear term removed by the projection, so with N' = u x omega -
(chi/eta)(u - u_s) (before projection) grad Pi is the gradient part of N':
Pi_hat = -i k.N'_hat / |k|^2 for k != 0 and 0 at k = 0.  The pressure
p = Pi - |u|^2/2 is interpolated onto the mass points with a delta kernel and
each triangle loads its three vertices along its normal with pressure x area/3.

Readings (no formula given in the paper): the delta kernel is the 4-point
kernel of Peskin (a stand-in for the smoothed kernel the paper cites); the
load uses the pressure jump across the wing, dp_v = p(x_v + d n_v) -
p(x_v - d n_v) with d = t_w + h and n_v the normalized sum of A_T n_T over the
triangles of v, and load_v = -dp_v (1/3) sum_T A_T n_T.
Pins: tests/test_oracle_pressure.py.
"""

import numpy as np

from . import dft, spectral


def total_pressure_hat(nh_unprojected, n, L):
    """Pi_hat = -i k.N'_hat / |k|^2 (0 at k = 0)."""
    kx, ky, kz = spectral.wavenumbers(n, L)
    k2 = kx * kx + ky * ky + kz * kz
    kdotn = kx * nh_unprojected[0] + ky * nh_unprojected[1] + kz * nh_unprojected[2]
    inv = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
    return -1j * kdotn * inv


def pressure_field(pi_hat, u):
    """p = Pi - |u|^2 / 2 on the grid, u (3, nz, ny, nx) physical."""
    return dft.inverse_real(pi_hat) - 0.5 * np.sum(u * u, axis=0)


def delta4(r):
    """Peskin's 4-point kernel phi(r) (grid units)."""
    r = np.abs(np.asarray(r, dtype=np.float64))
    inner = (3.0 - 2.0 * r + np.sqrt(np.clip(1.0 + 4.0 * r - 4.0 * r * r, 0.0, None))) / 8.0
    outer = (5.0 - 2.0 * r - np.sqrt(np.clip(-7.0 + 12.0 * r - 4.0 * r * r, 0.0, None))) / 8.0
    return np.where(r < 1.0, inner, np.where(r < 2.0, outer, 0.0))


def sample(p, L, pts):
    """Interpolate the grid field p (nz, ny, nx) at points (m, 3) with the
    tensor-product 4-point kernel; grid point (i, j, k) sits at (i, j, k) * dx."""
    nz, ny, nx = p.shape
    dx = np.array([L[0] / nx, L[1] / ny, L[2] / nz])
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(len(pts))
    for s, X in enumerate(pts):
        g = X / dx
        base = np.floor(g).astype(int) - 1
        idx = [base[q] + np.arange(4) for q in range(3)]
        w = [delta4(g[q] - idx[q]) for q in range(3)]
        block = p[np.ix_(idx[2] % nz, idx[1] % ny, idx[0] % nx)]
        out[s] = np.einsum("k,j,i,kji->", w[2], w[1], w[0], block)
    return out


def vertex_load_vectors(x, tri):
    """c_v = (1/3) sum over the triangles T of v of A_T n_T (n_T from the vertex order)."""
    x = np.asarray(x, dtype=np.float64)
    c = np.zeros_like(x)
    for t in np.asarray(tri):
        an = 0.5 * np.cross(x[t[1]] - x[t[0]], x[t[2]] - x[t[0]])  # A_T n_T
        for v in t:
            c[v] += an / 3.0
    return c


def wing_loads(p, L, x, tri, d):
    """Vertex loads -dp_v c_v and the jumps dp_v from the grid pressure p."""
    c = vertex_load_vectors(x, tri)
    nrm = np.linalg.norm(c, axis=1)
    nv = np.where(nrm[:, None] > 0, c / np.where(nrm > 0, nrm, 1.0)[:, None], 0.0)
    plus = sample(p, L, x + d * nv)
    minus = sample(p, L, x - d * nv)
    dp = plus - minus
    return -dp[:, None] * c, dp
