"""Seeded synthetic inputs shared by the oracle tests and the HIP-path tests.

This module holds no arithmetic of the method (no transforms of the solver,
no projection, no mask, no time stepping): only initial velocity fields with
known closed forms, seeded random fields, wing triangulations in their own
frame, and the numeric parameters of each workload.  The paper's measured
wing geometry and flow data are not used; these inputs stand in with the
shapes of its revolving-wing runs (Sec. 4.2.2, Sec. 5).
"""

import json
import math
import os

import numpy as np

# ---------------------------------------------------------------------------
# velocity fields
# ---------------------------------------------------------------------------


def _coords(n, L):
    nx, ny, nz = n
    lx, ly, lz = L
    x = np.arange(nx) * (2.0 * np.pi / nx)   # phase 2 pi x / L
    y = np.arange(ny) * (2.0 * np.pi / ny)
    z = np.arange(nz) * (2.0 * np.pi / nz)
    return x[None, None, :], y[None, :, None], z[:, None, None]


def taylor_green_3d(n, L=(2 * np.pi,) * 3):
    """u = (sin x cos y cos z, -cos x sin y cos z, 0) in phase coordinates 2 pi x_j / L_j."""
    x, y, z = _coords(n, L)
    nx, ny, nz = n
    u = np.zeros((3, nz, ny, nx))
    u[0] = np.sin(x) * np.cos(y) * np.cos(z)
    u[1] = -np.cos(x) * np.sin(y) * np.cos(z)
    return u


def taylor_green_2d(n, L=(2 * np.pi,) * 3):
    """u = (sin x cos y, -cos x sin y, 0), independent of z."""
    x, y, z = _coords(n, L)
    nx, ny, nz = n
    u = np.zeros((3, nz, ny, nx))
    u[0] = np.sin(x) * np.cos(y) + 0.0 * z
    u[1] = -np.cos(x) * np.sin(y) + 0.0 * z
    return u


def random_field(shape, seed):
    """Gaussian white noise (FP64) of any shape."""
    return np.random.default_rng(seed).standard_normal(shape)


def random_solenoidal(n, L, seed=0, energy=1.0, slope=-11.0 / 6.0):
    """Random divergence-free, band-limited field with a k^(-5/3) energy spectrum.

    Construction (Rogallo's method, not the solver's projection): every mode
    with 1 <= |m| and 3|m_j| < N_j gets amplitude |m|^slope along two unit
    vectors orthogonal to its wave vector (a fixed-axis Craya-Herring frame),
    with complex Gaussian coefficients from ``default_rng(seed)``.  The real
    part of the inverse numpy FFT keeps the field divergence-free (each mode
    and its conjugate partner stay orthogonal to their wave vectors); it is then
    scaled so that E = <|u|^2>/2 = ``energy``.
    """
    nx, ny, nz = n
    lx, ly, lz = L
    rng = np.random.default_rng(seed)

    def modes(m):
        j = np.arange(m)
        return np.where(j <= m // 2, j, j - m)

    mx = modes(nx)[None, None, :].astype(np.float64)
    my = modes(ny)[None, :, None].astype(np.float64)
    mz = modes(nz)[:, None, None].astype(np.float64)
    kx = np.broadcast_to(2 * np.pi * mx / lx, (nz, ny, nx))
    ky = np.broadcast_to(2 * np.pi * my / ly, (nz, ny, nx))
    kz = np.broadcast_to(2 * np.pi * mz / lz, (nz, ny, nx))
    kvec = np.stack([kx, ky, kz], axis=-1)
    kmag = np.sqrt(np.sum(kvec * kvec, axis=-1))
    mmag = np.sqrt(mx * mx + my * my + mz * mz)
    keep = ((3 * np.abs(mx) < nx) & (3 * np.abs(my) < ny) & (3 * np.abs(mz) < nz) & (mmag >= 1.0))

    # Craya-Herring frame: e1 = k x a / |k x a|, e2 = khat x e1, with a = e_z
    # unless k is parallel to e_z (then a = e_x).
    a = np.zeros_like(kvec)
    par = (np.abs(kx) + np.abs(ky)) == 0.0
    a[..., 2] = np.where(par, 0.0, 1.0)
    a[..., 0] = np.where(par, 1.0, 0.0)
    e1 = np.cross(kvec, a)
    e1 /= np.maximum(np.linalg.norm(e1, axis=-1, keepdims=True), 1e-300)
    khat = kvec / np.maximum(kmag[..., None], 1e-300)
    e2 = np.cross(khat, e1)

    c1 = rng.standard_normal((nz, ny, nx)) + 1j * rng.standard_normal((nz, ny, nx))
    c2 = rng.standard_normal((nz, ny, nx)) + 1j * rng.standard_normal((nz, ny, nx))
    amp = np.where(keep, np.power(np.maximum(mmag, 1.0), slope), 0.0)
    spec = amp[..., None] * (c1[..., None] * e1 + c2[..., None] * e2)
    u = np.stack([np.fft.ifftn(spec[..., c]).real for c in range(3)])
    e = 0.5 * np.mean(np.sum(u * u, axis=0))
    return u * math.sqrt(energy / e)


def _band_modes(K):
    return np.concatenate([np.arange(K + 1), np.arange(-K, 0)])


def random_solenoidal_compact(n, L, seed=0, energy=1.0, slope=-11.0 / 6.0):
    """Compact-band spectrum (3, 2Kz+1, 2Ky+1, Kx+1) of a random solenoidal field.

    Same construction as ``random_solenoidal`` (Craya-Herring frame, amplitude
    |m|^slope, complex Gaussian coefficients), written directly in the compact
    layout of the library (iz, iy in natural band order, ix = m_x >= 0,
    K_j = max{m : 3m < n_j}); the kx = 0 plane is made Hermitian and the field is
    scaled so that E = <|u|^2>/2 = ``energy`` (Parseval on the half spectrum).
    """
    nx, ny, nz = n
    lx, ly, lz = L
    Kx, Ky, Kz = (nx - 1) // 3, (ny - 1) // 3, (nz - 1) // 3
    rng = np.random.default_rng(seed)
    mz = _band_modes(Kz).astype(np.float64)[:, None, None]
    my = _band_modes(Ky).astype(np.float64)[None, :, None]
    mx = np.arange(Kx + 1, dtype=np.float64)[None, None, :]
    shape = (2 * Kz + 1, 2 * Ky + 1, Kx + 1)
    kx = np.broadcast_to(2 * np.pi * mx / lx, shape)
    ky = np.broadcast_to(2 * np.pi * my / ly, shape)
    kz = np.broadcast_to(2 * np.pi * mz / lz, shape)
    mmag = np.sqrt(mx * mx + my * my + mz * mz)
    kmag = np.sqrt(kx * kx + ky * ky + kz * kz)
    par = (kx == 0.0) & (ky == 0.0)
    # e1 = k x a / |k x a| with a = e_z (e_x when k is parallel to e_z)
    e1x = np.where(par, 0.0, ky)
    e1y = np.where(par, kz, -kx)
    e1z = np.zeros(shape)
    nrm = np.maximum(np.sqrt(e1x * e1x + e1y * e1y), 1e-300)
    e1x, e1y = e1x / nrm, e1y / nrm
    inv = 1.0 / np.maximum(kmag, 1e-300)
    hx, hy, hz = kx * inv, ky * inv, kz * inv
    e2x = hy * e1z - hz * e1y
    e2y = hz * e1x - hx * e1z
    e2z = hx * e1y - hy * e1x
    amp = np.where(mmag >= 1.0, np.power(np.maximum(mmag, 1.0), slope), 0.0)
    c1 = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    c2 = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    uh = np.stack([amp * (c1 * e1x + c2 * e2x), amp * (c1 * e1y + c2 * e2y), amp * (c1 * e1z + c2 * e2z)])
    # Hermitian kx = 0 plane: u(0, -my, -mz) = conj u(0, my, mz)
    iz = (-np.arange(2 * Kz + 1)) % (2 * Kz + 1)
    iy = (-np.arange(2 * Ky + 1)) % (2 * Ky + 1)
    p0 = uh[:, :, :, 0]
    uh[:, :, :, 0] = 0.5 * (p0 + np.conj(p0[:, iz][:, :, iy]))
    w = np.ones(Kx + 1)
    w[1:] = 2.0
    e = 0.5 * float(np.sum(w * np.sum(np.abs(uh) ** 2, axis=(0, 1, 2))))
    return uh * np.sqrt(energy / e)


def beltrami_modes(n, L, m2, seed=0):
    """A Beltrami (ABC-type) field: a sum of helical Fourier modes that all have
    the same |k|, so that curl u = |k| u, u x omega = 0 and the field decays as
    exp(-nu |k|^2 t) under the Navier-Stokes equations with no mask.

    The modes are every integer vector m with |k(m)|^2 = (2 pi)^2 m2 / L_x^2
    (k_j = 2 pi m_j / L_j) on the half space m_x > 0, or m_x = 0 and (m_y, m_z)
    positive lexicographically; each carries a seeded complex amplitude times
    the positive-helicity vector h = (e1 + i e2)/sqrt(2) (e1, e2, k/|k| a
    right-handed orthonormal frame; i k x h = |k| h).  Returns a list of
    (m, u_hat) pairs; the partner at -m is the conjugate (real field).  Every
    m must lie in the 2/3 band of n.
    """
    nx, ny, nz = n
    lx, ly, lz = L
    target = (2 * np.pi) ** 2 * m2 / lx ** 2
    rng = np.random.default_rng(seed)
    r = int(math.isqrt(int(m2))) + 1
    scale = [lx / lx, lx / ly, lx / lz]
    out = []
    for mx_ in range(0, int(r / scale[0]) + 2):
        for my_ in range(-int(r / scale[1]) - 2, int(r / scale[1]) + 3):
            for mz_ in range(-int(r / scale[2]) - 2, int(r / scale[2]) + 3):
                if mx_ == 0 and (my_ < 0 or (my_ == 0 and mz_ <= 0)):
                    continue
                k = np.array([2 * np.pi * mx_ / lx, 2 * np.pi * my_ / ly, 2 * np.pi * mz_ / lz])
                if abs(float(k @ k) - target) > 1e-12 * target:
                    continue
                if not (3 * abs(mx_) < nx and 3 * abs(my_) < ny and 3 * abs(mz_) < nz):
                    raise ValueError("Beltrami mode outside the 2/3 band")
                kh = k / np.linalg.norm(k)
                a = np.array([0.0, 0.0, 1.0]) if abs(kh[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
                e1 = np.cross(kh, a)
                e1 /= np.linalg.norm(e1)
                e2 = np.cross(kh, e1)
                c = rng.standard_normal() + 1j * rng.standard_normal()
                out.append(((mx_, my_, mz_), c * (e1 + 1j * e2) / math.sqrt(2.0)))
    if not out:
        raise ValueError("no integer mode with that |k|")
    return out


def modes_to_compact(n, modes):
    """Compact-band spectrum (3, 2Kz+1, 2Ky+1, Kx+1) holding the given half-space
    modes (and, on the kx = 0 plane, their conjugate partners)."""
    nx, ny, nz = n
    Kx, Ky, Kz = (nx - 1) // 3, (ny - 1) // 3, (nz - 1) // 3
    uh = np.zeros((3, 2 * Kz + 1, 2 * Ky + 1, Kx + 1), dtype=np.complex128)
    for (mx_, my_, mz_), c in modes:
        uh[:, mz_ % (2 * Kz + 1), my_ % (2 * Ky + 1), mx_] = c
        if mx_ == 0:
            uh[:, (-mz_) % (2 * Kz + 1), (-my_) % (2 * Ky + 1), 0] = np.conj(c)
    return uh


# ---------------------------------------------------------------------------
# wing triangulations (wing frame; no pose)
# ---------------------------------------------------------------------------


def grid_triangles(ns, nc):
    """Triangles of an ns x nc vertex grid (vertex id = j * ns + i, i along span).

    Each quad (i, j)-(i+1, j+1) is split along the diagonal (i, j) -> (i+1, j+1)."""
    tri = []
    for j in range(nc - 1):
        for i in range(ns - 1):
            v00 = j * ns + i
            v10 = v00 + 1
            v01 = v00 + ns
            v11 = v01 + 1
            tri.append((v00, v10, v11))
            tri.append((v00, v11, v01))
    return np.array(tri, dtype=np.int32)


def plate_span_chord(ns, nc, span, chord):
    """Span coordinate s in [0, span] and chord coordinate c in [-chord/2, chord/2] per vertex."""
    i = np.arange(ns)
    j = np.arange(nc)
    s = np.tile(i * (span / (ns - 1)), nc)
    c = np.repeat(-0.5 * chord + j * (chord / (nc - 1)), ns)
    return s, c


def flat_rectangle(center, u_axis, v_axis, a, b, ns=2, nc=2):
    """Vertices (ns*nc, 3) of a flat rectangle of half-sides a (along u_axis) and b (along v_axis)."""
    center = np.asarray(center, dtype=np.float64)
    u_axis = np.asarray(u_axis, dtype=np.float64)
    v_axis = np.asarray(v_axis, dtype=np.float64)
    s = np.linspace(-a, a, ns)
    t = np.linspace(-b, b, nc)
    pts = [center + s[i] * u_axis + t[j] * v_axis for j in range(nc) for i in range(ns)]
    return np.array(pts), grid_triangles(ns, nc)


def random_triangles(nt, lo, hi, size, seed):
    """A soup of nt random triangles with vertices in a box, for distance tests."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    centers = lo + (hi - lo) * rng.random((nt, 3))
    x = (centers[:, None, :] + size * (rng.random((nt, 3, 3)) - 0.5)).reshape(-1, 3)
    tri = np.arange(3 * nt, dtype=np.int32).reshape(nt, 3)
    return x, tri


# ---------------------------------------------------------------------------
# workload parameters (readings of the paper's setups)
# ---------------------------------------------------------------------------

PROFILE_COS = 0
PROFILE_TANH = 1


def config0(with_plate):
    """32^3 Taylor-Green box [0, 2 pi)^3, nu = 0.01, dt = 1e-3, 20 steps; optional static plate."""
    n = (32, 32, 32)
    L = (2 * np.pi,) * 3
    dx = L[0] / n[0]
    cfg = dict(n=n, L=L, nu=0.01, eta=1e-3, tw=2 * dx, h=dx, profile=PROFILE_TANH,
               dt=1e-3, steps=20)
    if with_plate:
        # 1.0 x 0.3 rectangle, normal e_x, 1.0 along y, 0.3 along z, centred where the
        # Taylor-Green flow is (1, 0, 0): head-on.
        x, tri = flat_rectangle((np.pi / 2, np.pi, np.pi), (0, 1, 0), (0, 0, 1), 0.5, 0.15)
        cfg["wing"] = (x, np.zeros_like(x), tri)
    return cfg


def revolving_plate(n=128, box=12.0, fixed_eta=None, t_ramp=0.4):
    """Rigid revolving plate (span R = 3, chord 1, alpha = 45 deg) in a cubic box of side 4R.

    Time unit = one revolution: Omega = 2 pi, tip speed 6 pi, Re = Omega R c / nu = 1800
    gives nu = pi / 300.  eta keeps K_eta = sqrt(nu eta)/dx constant (2.5e-3 at 128^3).
    """
    dx = box / n
    eta = fixed_eta if fixed_eta is not None else 2.5e-3 * (128.0 / n) ** 2
    ns, nc = 41, 13
    s, c = plate_span_chord(ns, nc, 3.0, 1.0)
    return dict(n=(n, n, n), L=(box, box, box), nu=math.pi / 300.0, eta=eta,
                tw=2 * dx, h=dx, profile=PROFILE_COS,
                alpha=math.pi / 4, omega=2 * math.pi, t_ramp=t_ramp,
                axis_point=(box / 2, box / 2, box / 2),
                span_coord=s, chord_coord=c, tri=grid_triangles(ns, nc),
                cfl=0.1, c_eta=2.0 / 3.0, dt_max=1e-2)


# ---------------------------------------------------------------------------
# flexible wings (mass-spring networks): geometry, topology and seeded draws
# ---------------------------------------------------------------------------

def _grid_edges(ns, nc):
    """Vertex pairs of the triangle edges of grid_triangles: spanwise, chordwise
    and the (i, j)-(i+1, j+1) diagonals."""
    e = []
    for j in range(nc):
        for i in range(ns):
            v = j * ns + i
            if i + 1 < ns:
                e.append((v, v + 1))
            if j + 1 < nc:
                e.append((v, v + ns))
            if i + 1 < ns and j + 1 < nc:
                e.append((v, v + ns + 1))
    return np.array(e, dtype=np.int32)


def structure_units(omega=2 * math.pi, span=3.0):
    """Factor converting structure stiffnesses given in units with unit tip speed
    into the fluid units used here (one revolution per time unit): forces scale
    with the square of the tip speed, so stiffness x (omega span)^2."""
    return (omega * span) ** 2


def flexible_wing(ns=31, nc=16, n_veins=8, vein_nodes=25, span=3.0, chord=1.0, seed=0,
                  EI_range=(1e-3, 1e-1), k_membrane_range=(1e-4, 1e-2), k_vein=1.0, density=1e-3):
    """Membrane of ns x nc vertices over span x chord with veins on every other
    chordwise row (rows 0, 2, ..., 2 (n_veins - 1)), each vein the first
    vein_nodes spanwise vertices of its row.  Draws (numpy default_rng(seed)):
    one EI per vein, log-uniform in EI_range, and one stiffness per membrane
    spring, log-uniform in k_membrane_range; vein edges have stiffness k_vein.
    Stiffnesses are returned in fluid units (structure_units()).  The first two
    spanwise columns are clamped to the root motion."""
    rng = np.random.default_rng(seed)
    s, c = plate_span_chord(ns, nc, span, chord)
    tri = grid_triangles(ns, nc)
    edges = _grid_edges(ns, nc)
    scale = structure_units(span=span)
    lo, hi = np.log(EI_range[0]), np.log(EI_range[1])
    EI = np.exp(lo + (hi - lo) * rng.random(n_veins)) * scale
    klo, khi = np.log(k_membrane_range[0]), np.log(k_membrane_range[1])
    k = np.exp(klo + (khi - klo) * rng.random(len(edges))) * scale
    rows = [2 * v for v in range(n_veins)]
    vein_edge = set()
    for r in rows:
        for i in range(vein_nodes - 1):
            vein_edge.add((r * ns + i, r * ns + i + 1))
    for e, (a, b) in enumerate(edges):
        if (int(a), int(b)) in vein_edge:
            k[e] = k_vein * scale
    veins = [np.array([r * ns + i for i in range(vein_nodes)], dtype=np.int32) for r in rows]
    clamped = np.array([j * ns + i for j in range(nc) for i in (0, 1)], dtype=np.int32)
    return dict(span_coord=s, chord_coord=c, tri=tri, ext_ij=edges, ext_k=k, veins=veins, vein_EI=EI,
                vein_length=span / (ns - 1) * (vein_nodes - 1), clamped=clamped, density=density)


def vein_bending(wing):
    """Bending triples (axis 0) of the veins and the vein each belongs to: every
    interior vein node carries one spring (n = vein_nodes - 2 per vein)."""
    ijk, owner = [], []
    for v, nodes in enumerate(wing["veins"]):
        for m in range(1, len(nodes) - 1):
            ijk.append((nodes[m - 1], nodes[m], nodes[m + 1]))
            owner.append(v)
    return np.array(ijk, dtype=np.int32), np.array(owner, dtype=np.int32)


HINGE_COLUMNS = (2, 10, 20, 30)


def hinge_plate(ns=41, nc=13, span=3.0, chord=1.0, k_hinge=(1e-2, 1e-2, 1e-2, 1e-2), k_ext=1e2, density=1e-3,
                hinge_columns=HINGE_COLUMNS):
    """Plate of four spanwise segments joined by hinges: extension springs on
    all triangle edges (k_ext), spanwise bending springs (axis 0) at every
    interior column of every chordwise row and chordwise bending springs
    (axis 1) at every interior row of every spanwise column.  Spanwise springs
    at hinge column hinge_columns[g] have stiffness k_hinge[g] (group g); all
    other bending springs are rigid, 1e3 max(k_hinge) (group -1).  Columns 0 and
    1 are clamped.  Stiffnesses in fluid units (structure_units())."""
    scale = structure_units(span=span)
    s, c = plate_span_chord(ns, nc, span, chord)
    tri = grid_triangles(ns, nc)
    edges = _grid_edges(ns, nc)
    k_rigid = 1e3 * max(k_hinge)
    ijk, axis, group, kb = [], [], [], []
    for j in range(nc):
        for i in range(1, ns - 1):
            v = j * ns + i
            ijk.append((v - 1, v, v + 1))
            axis.append(0)
            g = hinge_columns.index(i) if i in hinge_columns else -1
            group.append(g)
            kb.append((k_hinge[g] if g >= 0 else k_rigid) * scale)
    for i in range(ns):
        for j in range(1, nc - 1):
            v = j * ns + i
            ijk.append((v - ns, v, v + ns))
            axis.append(1)
            group.append(-1)
            kb.append(k_rigid * scale)
    clamped = np.array([j * ns + i for j in range(nc) for i in (0, 1)], dtype=np.int32)
    return dict(span_coord=s, chord_coord=c, tri=tri, ext_ij=edges, ext_k=np.full(len(edges), k_ext * scale),
                bend_ijk=np.array(ijk, dtype=np.int32), bend_axis=np.array(axis, dtype=np.int32),
                bend_group=np.array(group, dtype=np.int32), bend_kb=np.array(kb), clamped=clamped,
                density=density, scale=scale)


# ---------------------------------------------------------------------------
# channel with a cylinder and a flexible flag (the FSI3-style workload of
# Sec. 4.2.1): static penalization plane and flag network
# ---------------------------------------------------------------------------

TUREK_H = 0.41      # channel height
TUREK_LEN = 2.5     # channel length
TUREK_R = 0.05      # cylinder radius
TUREK_C = (0.2, 0.2)  # cylinder centre from the inlet and the lower wall
TUREK_FLAG = (0.35, 0.02)  # flag length and thickness
TUREK_UMEAN = 2.0   # mean inflow velocity


def _smooth_step(sigma, h):
    """Solid indicator from a signed distance sigma (> 0 inside the solid),
    smoothed over |sigma| < h with the cosine shape of the wing mask: 0 at
    sigma = -h, 1/2 on the surface, 1 at sigma = h."""
    sig = np.clip(np.asarray(sigma, dtype=np.float64), -h, h)
    return 0.5 * (1.0 + np.sin(0.5 * np.pi * sig / h))


def turek_channel(nx, ny, nz, wall=0.05, inflow=0.2, h_cells=1.0, depth_cells=None):
    """Quasi-2-D channel of height 0.41 and length 2.5 between penalized walls of
    thickness `wall`, a penalized inflow layer of width `inflow` upstream of the
    inlet imposing the Poiseuille profile of mean 2 (periodic box: the outflow
    re-enters through it), and a cylinder of radius 0.05 centred 0.2 behind
    the inlet and 0.2 above the lower wall.  Box (2.5 + inflow, 0.41 + 2 wall,
    nz dx); smoothing half-width h = h_cells dx.  Returns the workload dict with
    the static plane (chi, u_s [3], weight: 1 on the cylinder) and the flag
    plate (span along x behind the cylinder, chord along z, normal along y)."""
    Lx = TUREK_LEN + inflow
    Ly = TUREK_H + 2 * wall
    dx = Lx / nx
    Lz = nz * dx if depth_cells is None else depth_cells * dx
    h = h_cells * dx
    x = (np.arange(nx) * dx)[None, :]
    y = (np.arange(ny) * (Ly / ny))[:, None]
    # walls: below y = wall and above y = wall + H (periodic in y: one slab)
    s_wall = np.maximum(wall - y, y - (wall + TUREK_H)) + 0.0 * x
    chi_wall = _smooth_step(s_wall, h)
    # inflow layer x in [0, inflow] (distance to its faces, periodic in x)
    s_in = np.where(x <= inflow, np.minimum(x, inflow - x), -np.minimum(x - inflow, Lx - x)) + 0.0 * y
    chi_in = _smooth_step(s_in, h)
    xc, yc = inflow + TUREK_C[0], wall + TUREK_C[1]
    s_cyl = TUREK_R - np.sqrt((x - xc) ** 2 + (y - yc) ** 2)
    chi_cyl = _smooth_step(s_cyl, h)
    chi = np.maximum(np.maximum(chi_wall, chi_in), chi_cyl)
    us = np.zeros((3, ny, nx))
    eta_y = np.clip((y - wall) / TUREK_H, 0.0, 1.0)
    poiseuille = 6.0 * TUREK_UMEAN * eta_y * (1.0 - eta_y)  # mean 2, maximum 3
    inflow_wins = (chi_in >= chi_wall) & (chi_in >= chi_cyl)
    us[0] = np.where(inflow_wins, poiseuille + 0.0 * x, 0.0)
    weight = ((chi_cyl > chi_wall) & (chi_cyl > chi_in)).astype(np.float64)
    return dict(n=(nx, ny, nz), L=(Lx, Ly, Lz), dx=dx, h=h, static=(chi, us, weight),
                cylinder=(xc, yc, TUREK_R), wall=wall, inflow=inflow)


def turek_inflow_field(ch):
    """u = (U(y), 0, 0) with the Poiseuille profile of the inflow layer between
    the walls (mean 2, zero outside the channel): a developed channel flow to
    start from."""
    nx, ny, nz = ch["n"]
    y = np.arange(ny) * (ch["L"][1] / ny)
    eta_y = np.clip((y - ch["wall"]) / TUREK_H, 0.0, 1.0)
    u = np.zeros((3, nz, ny, nx))
    u[0] = (6.0 * TUREK_UMEAN * eta_y * (1.0 - eta_y))[None, :, None]
    return u


def turek_flag(ch, ns=15, nc=4, tw=None, density=0.02, E=5.6e6 / 1000.0, k_ext_scale=1.0):
    """Mass-spring flag of the channel workload: a plate of length 0.35 behind
    the cylinder (root inside it), chord along z over the box depth minus the
    mask support and the pressure stencil at both ends.  Material in units of the fluid density
    (rho_s = rho_f, E / rho_f): areal density rho_s h / rho_f = 0.02, bending
    rigidity per unit depth E h^3 / 12, extension E h.  Bending springs along
    the span on every chordwise row (k^b of Eq. EI_k_relation for that row's
    share of the depth) and stiff chordwise bending (the flag stays plane in z);
    the first two span columns (inside the cylinder) are clamped.  Each bending
    spring carries (EI, l_b, n_b, factor): a solver takes k^b = factor x k^b(EI,
    l_b, n_b) by Eq. EI_k_relation (factor 1e3 on the chordwise springs)."""
    xc, yc, R = ch["cylinder"]
    thick = TUREK_FLAG[1]
    tw = 0.5 * thick if tw is None else tw
    rsup = tw + ch["h"]
    # the pressure box (the 4-point stencils of points within t_w + h of the
    # mesh) must stay inside the box depth: a margin of t_w + h + 3 dx each side
    depth = ch["L"][2] - 2.0 * (rsup + 3.0 * ch["dx"])
    if depth <= 0:
        raise ValueError("box too shallow for the flag: increase nz")
    x_root = xc + np.sqrt(R * R - (0.5 * thick) ** 2) - 0.02  # clamped nodes inside the cylinder
    span = xc + R + TUREK_FLAG[0] - x_root
    s, c = plate_span_chord(ns, nc, span, depth)
    tri = grid_triangles(ns, nc)
    edges = _grid_edges(ns, nc)
    lens = np.where(np.abs(edges[:, 1] - edges[:, 0]) == 1, span / (ns - 1),
                    np.where(np.abs(edges[:, 1] - edges[:, 0]) == ns, depth / (nc - 1),
                             np.hypot(span / (ns - 1), depth / (nc - 1))))
    k_ext = k_ext_scale * E * thick * depth / lens / nc  # axial stiffness of the strip a spring stands for
    EI_row = E * thick ** 3 / 12.0 * depth / nc
    n_b = ns - 2
    ijk, axis, factor = [], [], []
    for j in range(nc):
        for i in range(1, ns - 1):
            v = j * ns + i
            ijk.append((v - 1, v, v + 1))
            axis.append(0)
            factor.append(1.0)
    for i in range(ns):
        for j in range(1, nc - 1):
            v = j * ns + i
            ijk.append((v - ns, v, v + ns))
            axis.append(1)
            factor.append(1e3)
    m = len(ijk)
    bend = dict(EI=np.full(m, EI_row), lb=np.full(m, span), nb=np.full(m, n_b, dtype=np.int32),
                factor=np.array(factor))
    clamped = np.array([j * ns + i for j in range(nc) for i in (0, 1)], dtype=np.int32)
    kin = dict(alpha=0.5 * np.pi, omega=0.0, t_ramp=0.0, axis_point=(x_root, yc, 0.5 * ch["L"][2]))
    wing = dict(span_coord=s, chord_coord=c, tri=tri, ext_ij=edges, ext_k=k_ext, clamped=clamped,
                density=density)
    return wing, np.array(ijk, dtype=np.int32), bend, np.array(axis, dtype=np.int32), kin, tw


# ---------------------------------------------------------------------------
# functional bumblebee forewing (Sec. 3): printed vein diameters and masses,
# membrane mass law, vein stiffness from a Young modulus, on a synthetic
# planform and vein layout (the measured venation is not available)
# ---------------------------------------------------------------------------

# Table vein_mass, forewing: (nominal diameter, nominal mass), normalized by the
# wing length L and by rho_air L^3
FOREWING_VEINS = [
    (0.0070, 0.0209), (0.0074, 0.0237), (0.0055, 0.0076), (0.0070, 0.0063), (0.0040, 0.0031),
    (0.0048, 0.0094), (0.0040, 0.0019), (0.0038, 0.0009), (0.0041, 0.0023), (0.0048, 0.0064),
    (0.0045, 0.0017), (0.0038, 0.0018), (0.0042, 0.0010), (0.0038, 0.0020), (0.0034, 0.0008),
    (0.0032, 0.0005), (0.0032, 0.0004), (0.0044, 0.0009), (0.0015, 0.0001), (0.0018, 0.0001),
    (0.0020, 0.0009),
]
RHO_CUTICLE = 1300.0 / 1.2248   # cuticle density over air density (the mass scale 2.817 mg over (13.2 mm)^3)
E_FLEXIBLE = 1.25e8           # Young modulus of the flexible wing (35 kPa) in the wing's units, Sec. 4.3
E_HIGHLY_FLEXIBLE = 1.25e7    # highly flexible wing (3.5 kPa)


def membrane_mass(x, y):
    """Mass of a membrane mass point at (x, y) (wing lengths; x spanwise from the
    root, y chordwise increasing towards the leading edge), Sec. 3.2 bi-linear law."""
    return 1.75e-4 - 2.83e-4 * np.asarray(x) + 4.91e-4 * np.asarray(y)


def functional_wing(ns=31, nc=16, span=3.0, omega=2 * math.pi, E=E_FLEXIBLE, seed=0,
                    k_membrane_range=(10.0, 100.0), y_le=0.32, root_chord=0.30, tip_chord=0.08):
    """Forewing of the functional model (Sec. 2.3 vein and membrane models,
    Sec. 3.2 masses, Sec. 3.3 stiffness) on a synthetic layout.

    Planform (wing lengths): straight leading edge at y = y_le, chord tapering
    linearly from root_chord to tip_chord; an ns x nc mapped grid, triangulated
    as grid_triangles.  The 21 veins of the table keep their nominal diameter d
    and mass m; each vein's length follows from them (a cuticle rod:
    l = 4 m / (rho_c pi d^2)).  Veins of length >= 0.25 run spanwise from the
    root along the rows j = nc-1, nc-3, ... (leading edge first); the others
    are chordwise cross veins from the leading edge down the columns 2, 4, ...
    (2, 3, ... on a grid too short for that);
    a vein covers round(l / grid spacing) segments (at least two).  Vein mass is
    spread evenly over its nodes; every other node takes the membrane mass law.
    Vein flexural rigidity EI = E pi d^4 / 64 (E dimensionless as printed in
    Sec. 4.3); each bending spring carries its vein's EI, length l_b and
    spring count n_b, from which a solver takes k^b by Eq. EI_k_relation.  The
    vein extension springs only keep the vein's length: their stiffness is an
    artificial choice, here the rod's axial stiffness E pi d^2 / 4 / (edge
    length); membrane edges get a seeded stiffness log-uniform in
    k_membrane_range (no membrane data in the paper).  Units: the wing's
    (length L, tip speed 1, rho_air) converted to the fluid's (span `span`,
    angular speed `omega`, density 1): mass x span^3, EI x omega^2 span^6,
    axial stiffness x omega^2 span^3, lengths x span.  Root columns 0, 1 are
    clamped."""
    rng = np.random.default_rng(seed)
    i = np.arange(ns)
    j = np.arange(nc)
    xw = i / (ns - 1.0)
    chord = root_chord + (tip_chord - root_chord) * xw
    yw = (y_le - chord)[None, :] + (j / (nc - 1.0))[:, None] * chord[None, :]  # [j][i]
    X = np.tile(xw, nc)
    Y = yw.reshape(-1)
    y_mid = y_le - 0.5 * root_chord
    s_coord = X * span
    c_coord = (Y - y_mid) * span
    tri = grid_triangles(ns, nc)
    edges = _grid_edges(ns, nc)
    lengths = [4.0 * m / (RHO_CUTICLE * math.pi * d * d) for d, m in FOREWING_VEINS]
    order = sorted(range(len(FOREWING_VEINS)), key=lambda v: -lengths[v])
    veins = [None] * len(FOREWING_VEINS)
    row, col = nc - 1, 2
    n_cross = len(FOREWING_VEINS) - min(sum(l >= 0.25 for l in lengths), (nc + 1) // 2)
    col_step = 2 if 2 + 2 * (n_cross - 1) < ns else 1
    for v in order:
        if lengths[v] >= 0.25 and row >= 0:
            nseg = max(2, min(ns - 1, int(round(lengths[v] * (ns - 1)))))
            veins[v] = np.array([row * ns + a for a in range(nseg + 1)], dtype=np.int32)
            row -= 2
        else:
            if col >= ns:
                raise ValueError("grid too small for the cross veins")
            dy = chord[col] / (nc - 1.0)
            nseg = max(2, min(nc - 1, int(round(lengths[v] / dy))))
            veins[v] = np.array([(nc - 1 - b) * ns + col for b in range(nseg + 1)], dtype=np.int32)
            col += col_step
    nv = ns * nc
    mass = np.zeros(nv)
    in_vein = np.zeros(nv, dtype=bool)
    for v, nodes in enumerate(veins):
        mass[nodes] += FOREWING_VEINS[v][1] / len(nodes)
        in_vein[nodes] = True
    mem = ~in_vein
    mass[mem] = membrane_mass(X[mem], Y[mem])
    if np.any(mass <= 0):
        raise ValueError("membrane mass law gives a non-positive mass on this planform")
    mscale, kscale, eiscale = span ** 3, omega ** 2 * span ** 3, omega ** 2 * span ** 6
    # axial stiffness: vein edges from the vein's cross-section, membrane edges drawn
    vein_edge = {}
    for v, nodes in enumerate(veins):
        for a, b in zip(nodes[:-1], nodes[1:]):
            vein_edge[(min(a, b), max(a, b))] = v
    P = np.stack([X, Y], axis=1)
    klo, khi = np.log(k_membrane_range[0]), np.log(k_membrane_range[1])
    ext_k = np.exp(klo + (khi - klo) * rng.random(len(edges)))
    for e, (a, b) in enumerate(edges):
        v = vein_edge.get((min(int(a), int(b)), max(int(a), int(b))))
        if v is not None:
            d = FOREWING_VEINS[v][0]
            ext_k[e] = E * math.pi * d * d / 4.0 / float(np.linalg.norm(P[a] - P[b]))
    ext_k = ext_k * kscale
    # bending springs along each vein with the vein's EI, l_b and n_b
    ijk, EI, lb, nb, axis, owner = [], [], [], [], [], []
    for v, nodes in enumerate(veins):
        d = FOREWING_VEINS[v][0]
        l_b = float(np.sum(np.linalg.norm(np.diff(P[nodes], axis=0), axis=1))) * span
        ax = 0 if abs(int(nodes[1]) - int(nodes[0])) == 1 else 1
        for m in range(1, len(nodes) - 1):
            ijk.append((nodes[m - 1], nodes[m], nodes[m + 1]))
            EI.append(E * math.pi * d ** 4 / 64.0 * eiscale)
            lb.append(l_b)
            nb.append(len(nodes) - 2)
            axis.append(ax)
            owner.append(v)
    clamped = np.array([jj * ns + ii for jj in range(nc) for ii in (0, 1)], dtype=np.int32)
    return dict(span_coord=s_coord, chord_coord=c_coord, tri=tri, ext_ij=edges, ext_k=ext_k, clamped=clamped,
                mass=mass * mscale, density=None, veins=veins, vein_length=[lengths[v] * span for v in range(len(veins))],
                bend_ijk=np.array(ijk, dtype=np.int32), bend_EI=np.array(EI), bend_lb=np.array(lb),
                bend_nb=np.array(nb, dtype=np.int32), bend_axis=np.array(axis, dtype=np.int32),
                bend_owner=np.array(owner, dtype=np.int32), E=E, xw=X, yw=Y, ns=ns, nc=nc, span=span)


# ---------------------------------------------------------------------------
# workload files (configs/*.json): parameters and readings of each workload
# ---------------------------------------------------------------------------

CONFIG_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "configs")


def load_config(name):
    """The workload file configs/<name>.json (or a path) as a dict, with the
    inputs its kind needs built from it: ``case`` holds the revolving-plate
    parameters (revolving_plate) for the plate and wing kinds, ``wing`` the
    flexible wing for flexible_wing, ``plate`` the hinge plate for hinge_plate,
    ``case`` the config0 dict for taylor_green."""
    path = name if os.path.exists(name) else os.path.join(CONFIG_DIR, name + ".json")
    with open(path) as f:
        c = json.load(f)
    kind = c["kind"]
    if kind == "taylor_green":
        c["case"] = config0(True)
    elif kind in ("revolving_plate", "flexible_wing", "hinge_plate"):
        c["case"] = revolving_plate(n=int(c["n"]), box=float(c["box"]), t_ramp=float(c["t_ramp"]))
        if kind == "flexible_wing":
            w = c["wing"]
            c["wing_net"] = flexible_wing(ns=w["ns"], nc=w["nc"], n_veins=w["n_veins"], vein_nodes=w["vein_nodes"],
                                          seed=w["seed"], EI_range=tuple(w["EI_range"]),
                                          k_membrane_range=tuple(w["k_membrane_range"]), k_vein=w["k_vein"],
                                          density=w["density"])
        if kind == "hinge_plate":
            p = c["plate"]
            c["plate_net"] = hinge_plate(ns=p["ns"], nc=p["nc"], k_hinge=tuple(c["theta"][1:]), k_ext=p["k_ext"],
                                         density=p["density"], hinge_columns=tuple(p["hinge_columns"]))
    elif kind != "throughput":
        raise ValueError("unknown workload kind %r" % kind)
    return c

