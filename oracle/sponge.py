"""Vorticity sponge term (oracle; test infrastructure only).

Sec. 4.1, Eq. of the penalized equations: besides the penalization the
momentum equation carries a sponge term built from the vorticity masked by a
sponge mask chi_sp, divided by C_sp, under a curl and an inverse Laplacian;
the text calls it a vorticity damping that relieves the periodicity of the
Fourier discretization.  Two points the paper leaves open, and their readings:

* Sign (reading).  Taken literally with 1/lap as the inverse Laplacian the
  term becomes +u/C_sp for chi_sp = 1 (lap^-1 curl omega = -u for a
  solenoidal u), i.e. it would amplify the flow.  Damping fixes the sign: the
  term added to du/dt is
      T = -(1/C_sp) curl( (-lap)^-1 (chi_sp omega) ),
      T_hat = -(1/C_sp) i k x S_hat / |k|^2,  S = chi_sp omega,  T_hat(0) = 0,
  so that chi_sp = 1 gives T = -u/C_sp and curl T = -(1/C_sp) P(chi_sp omega).
* Sponge mask (reading).  Not given.  Here chi_sp(x, y, z) =
  max(g_x(x), g_y(y), g_z(z)) from three 1-D profiles on the grid points
  (e.g. layers at the box faces); a uniform chi_sp is g_x = const.

T is divergence-free, so the projection and the total pressure are
unchanged; it enters the nonlinear term before the 2/3 truncation and the
projection (oracle.ns).

Pins (tests/test_oracle_sponge.py): chi_sp = 1 gives T_hat = -u_hat/C_sp for
a band-limited solenoidal field; with chi_sp = 1 the 2-D Taylor-Green field
follows the scalar two-term recurrence of the IF-AB2 step exactly; k.T_hat = 0
for any chi_sp; the mask places g_x along x, g_y along y, g_z along z.
"""

import numpy as np

from . import dft, spectral


def sponge_mask(n, gx=None, gy=None, gz=None):
    """chi_sp[z, y, x] = max(gx[x], gy[y], gz[z]); a missing profile counts as 0."""
    nx, ny, nz = n
    px = np.zeros(nx) if gx is None else np.asarray(gx, dtype=np.float64)
    py = np.zeros(ny) if gy is None else np.asarray(gy, dtype=np.float64)
    pz = np.zeros(nz) if gz is None else np.asarray(gz, dtype=np.float64)
    return np.maximum(np.maximum(px[None, None, :], py[None, :, None]), pz[:, None, None])


def sponge_term_hat(uh, chi_sp, c_sp, n, L):
    """T_hat = -(1/C_sp) i k x DFT(chi_sp omega) / |k|^2 (zero at k = 0), full spectrum."""
    w = dft.inverse_real(spectral.curl(uh, n, L))
    sh = dft.forward(chi_sp[None] * w)
    kx, ky, kz = spectral.wavenumbers(n, L)
    k2 = kx * kx + ky * ky + kz * kz
    inv = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
    c = 1j * np.stack([ky * sh[2] - kz * sh[1], kz * sh[0] - kx * sh[2], kx * sh[1] - ky * sh[0]])
    return -(1.0 / c_sp) * c * inv
