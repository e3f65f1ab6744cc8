"""Mask function and solid velocity from a triangulated wing (oracle; test infrastructure only).

Sec. 4.1 encodes the wing in a smoothed mask chi(delta), Eq. (mask_function),
where delta is the distance from a grid node to the wing mid-surface, the
minimum over the mesh triangles of the point/triangle distance (Eberly's
distance between a point and a triangle in 3-D), restricted to triangles whose
bounding box (enlarged by the mask support) contains the node.  The solid
velocity u_s at a node is the barycentric interpolation of the vertex
velocities of the closest triangle at the node's closest point.

Readings (listed in the design notes):
* closest point = projection onto the triangle's plane when that projection
  falls inside the triangle, otherwise the nearest point of the three edges;
  u_s uses the barycentric weights of that (clamped) closest point;
* ties between triangles go to the lowest triangle index;
* cosine profile exactly as Eq. (mask_function), support radius t_w + h;
  the tanh profile chi = (1 - tanh((delta - t_w)/h))/2 is cut to zero at
  delta >= t_w + 6h (support radius t_w + 6h);
* u_s = 0 wherever chi = 0 (delta >= support radius);
* the enlarged bounding box of the whole mesh must lie in [0, L] on every
  axis (no periodic wrap of the mask), else ValueError.

Pins (tests/test_oracle_mask.py): distance to a flat rectangle against its
closed form for 2-triangle and 40x12 triangulations, culled = brute-force
minimum over all triangles, profile values at t_w - h, t_w, t_w + h, rigid
rotation u_s = Omega e_z x closest point.
"""

import numpy as np

PROFILE_COS = 0
PROFILE_TANH = 1
TANH_CUTOFF_WIDTHS = 6.0


def support_radius(tw, h, profile):
    if profile == PROFILE_COS:
        return tw + h
    if profile == PROFILE_TANH:
        return tw + TANH_CUTOFF_WIDTHS * h
    raise ValueError("unknown profile")


def chi_profile(delta, tw, h, profile):
    """chi(delta): Eq. (mask_function) for the cosine profile, the tanh variant otherwise."""
    delta = np.asarray(delta, dtype=np.float64)
    r = support_radius(tw, h, profile)
    if profile == PROFILE_COS:
        ramp = 0.5 * (1.0 + np.cos(np.pi * (delta - tw + h) / (2.0 * h)))
        out = np.where(delta <= tw - h, 1.0, np.where(delta >= tw + h, 0.0, ramp))
    else:
        out = 0.5 * (1.0 - np.tanh((delta - tw) / h))
    return np.where(delta >= r, 0.0, out)


def _segment_closest(p, a, b):
    """Closest point on segment [a, b] to points p (M, 3): returns (dist^2, t)."""
    d = b - a
    dd = float(d @ d)
    if dd > 0.0:
        t = np.clip(((p - a) @ d) / dd, 0.0, 1.0)
    else:
        t = np.zeros(p.shape[0])
    q = a[None, :] + t[:, None] * d[None, :]
    r = p - q
    return np.einsum("ij,ij->i", r, r), t


def point_triangle(p, a, b, c):
    """Distance from points p (M, 3) to the closed triangle (a, b, c).

    Returns (dist (M,), weights (M, 3)) where ``weights`` are the barycentric
    coordinates of the closest point with respect to (a, b, c).  Plain textbook
    form: project onto the plane; if the projection is inside the triangle it is
    the closest point, otherwise the closest point lies on one of the edges.
    """
    p = np.asarray(p, dtype=np.float64)
    m = p.shape[0]
    e0 = b - a
    e1 = c - a
    nrm = np.cross(e0, e1)
    area2 = float(np.sqrt(nrm @ nrm))

    # edges (a,b), (b,c), (c,a); first edge wins an exact tie
    d_ab, t_ab = _segment_closest(p, a, b)
    d_bc, t_bc = _segment_closest(p, b, c)
    d_ca, t_ca = _segment_closest(p, c, a)
    best = d_ab.copy()
    w = np.stack([1.0 - t_ab, t_ab, np.zeros(m)], axis=1)
    sel = d_bc < best
    best = np.where(sel, d_bc, best)
    w[sel] = np.stack([np.zeros(sel.sum()), 1.0 - t_bc[sel], t_bc[sel]], axis=1)
    sel = d_ca < best
    best = np.where(sel, d_ca, best)
    w[sel] = np.stack([t_ca[sel], np.zeros(sel.sum()), 1.0 - t_ca[sel]], axis=1)

    if area2 > 0.0:
        nhat = nrm / area2
        ap = p - a[None, :]
        h = ap @ nhat
        q = ap - h[:, None] * nhat[None, :]            # projection, relative to a
        d00 = e0 @ e0
        d01 = e0 @ e1
        d11 = e1 @ e1
        d20 = q @ e0
        d21 = q @ e1
        den = d00 * d11 - d01 * d01
        beta = (d11 * d20 - d01 * d21) / den
        gamma = (d00 * d21 - d01 * d20) / den
        alpha = 1.0 - beta - gamma
        inside = (alpha >= 0.0) & (beta >= 0.0) & (gamma >= 0.0)
        best = np.where(inside, h * h, best)
        w[inside] = np.stack([alpha[inside], beta[inside], gamma[inside]], axis=1)
    return np.sqrt(best), w


def grid_coords(n, L):
    nx, ny, nz = n
    lx, ly, lz = L
    return (np.arange(nx) * (lx / nx), np.arange(ny) * (ly / ny), np.arange(nz) * (lz / nz))


def check_bounds(x, n, L, r):
    lo = x.min(axis=0) - r
    hi = x.max(axis=0) + r
    if np.any(lo < 0.0) or np.any(hi > np.asarray(L, dtype=np.float64)):
        raise ValueError("enlarged wing bounding box leaves the periodic box")


def build_mask(n, L, x, v, tri, tw, h, profile, cull=True):
    """Mask chi (nz, ny, nx) and solid velocity u_s (3, nz, ny, nx) for a triangulated wing.

    ``x``, ``v``: vertex positions and velocities (nv, 3); ``tri``: (nt, 3) vertex indices.
    With ``cull`` each triangle is only tested against the nodes inside its
    bounding box enlarged by the support radius (Sec. 4.1); without it, every
    node is tested against every triangle (brute force).
    """
    x = np.asarray(x, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64)
    nx, ny, nz = n
    r = support_radius(tw, h, profile)
    chi = np.zeros((nz, ny, nx))
    us = np.zeros((3, nz, ny, nx))
    if tri.shape[0] == 0:
        return chi, us
    check_bounds(x, n, L, r)
    gx, gy, gz = grid_coords(n, L)
    dx = np.array([L[0] / nx, L[1] / ny, L[2] / nz])

    best = np.full((nz, ny, nx), np.inf)
    wbest = np.zeros((nz, ny, nx, 3))
    tbest = np.full((nz, ny, nx), -1, dtype=np.int64)

    if cull:
        for t in range(tri.shape[0]):
            a, b, c = x[tri[t, 0]], x[tri[t, 1]], x[tri[t, 2]]
            lo = np.minimum(np.minimum(a, b), c) - r
            hi = np.maximum(np.maximum(a, b), c) + r
            i0 = np.maximum(np.ceil(lo / dx).astype(int), 0)
            i1 = np.minimum(np.floor(hi / dx).astype(int), np.array([nx, ny, nz]) - 1)
            if np.any(i1 < i0):
                continue
            zz, yy, xx = np.meshgrid(np.arange(i0[2], i1[2] + 1), np.arange(i0[1], i1[1] + 1),
                                     np.arange(i0[0], i1[0] + 1), indexing="ij")
            pts = np.stack([gx[xx.ravel()], gy[yy.ravel()], gz[zz.ravel()]], axis=1)
            d, w = point_triangle(pts, a, b, c)
            cur = best[zz.ravel(), yy.ravel(), xx.ravel()]
            upd = d < cur
            if not np.any(upd):
                continue
            iz, iy, ix = zz.ravel()[upd], yy.ravel()[upd], xx.ravel()[upd]
            best[iz, iy, ix] = d[upd]
            wbest[iz, iy, ix] = w[upd]
            tbest[iz, iy, ix] = t
    else:
        zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        pts = np.stack([gx[xx.ravel()], gy[yy.ravel()], gz[zz.ravel()]], axis=1)
        flat_best = best.ravel()
        flat_w = wbest.reshape(-1, 3)
        flat_t = tbest.ravel()
        for t in range(tri.shape[0]):
            a, b, c = x[tri[t, 0]], x[tri[t, 1]], x[tri[t, 2]]
            d, w = point_triangle(pts, a, b, c)
            upd = d < flat_best
            flat_best[upd] = d[upd]
            flat_w[upd] = w[upd]
            flat_t[upd] = t

    inside = best < r
    chi = np.where(inside, chi_profile(np.where(inside, best, 0.0), tw, h, profile), 0.0)
    tb = np.where(inside, tbest, 0)
    for comp in range(3):
        vv = (wbest[..., 0] * v[tri[tb, 0], comp] + wbest[..., 1] * v[tri[tb, 1], comp]
              + wbest[..., 2] * v[tri[tb, 2], comp])
        us[comp] = np.where(inside, vv, 0.0)
    return chi, us


def distance_field(n, L, x, tri, rmax):
    """Brute-force min distance (capped at rmax) from every node to the mesh, for tests."""
    nx, ny, nz = n
    gx, gy, gz = grid_coords(n, L)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pts = np.stack([gx[xx.ravel()], gy[yy.ravel()], gz[zz.ravel()]], axis=1)
    best = np.full(pts.shape[0], np.inf)
    for t in range(len(tri)):
        d, _ = point_triangle(pts, x[tri[t, 0]], x[tri[t, 1]], x[tri[t, 2]])
        best = np.minimum(best, d)
    return np.minimum(best, rmax).reshape(nz, ny, nx)
