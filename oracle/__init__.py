"""FP64 CPU oracle for the penalized pseudo-spectral Navier-Stokes step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP library (no kernels, headers, tables or helpers) and the HIP library
never imports it.

What it computes is the Fourier pseudo-spectral, volume-penalized
incompressible Navier-Stokes step of Sec. 4.1 (penalized NS equations, the
mask function Eq. (mask_function), the distance function to the triangulated
wing mid-surface, the barycentric solid velocity), written plainly in numpy
FP64 with its own naive matrix-product DFT:

* ``dft``        - naive DFT along each axis (no FFT library).
* ``spectral``   - wavenumbers, the 2/3 band, curl, Leray projection.
* ``mask``       - point/triangle distance, smoothed mask profiles, the mask
                   and solid-velocity fields.
* ``ns``         - one time step (rotational nonlinear term, penalization,
                   reductions, adaptive dt, projection, integrating-factor AB2).
* ``kinematics`` - rigid revolving-plate pose (Sec. 4.2.2).

Parity status of every function is listed in each module header.
"""

from . import dft, spectral, mask, ns, kinematics  # noqa: F401
