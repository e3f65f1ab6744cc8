"""Pins of the oracle's mask function and solid velocity (Sec. 4.1, Eq. (mask_function)).

Closed-form distance to a flat rectangle, brute force versus bounding-box
culling, dense sampling of triangles, the profile's fixed values, and the
rigid-rotation solid velocity.
"""

import numpy as np
import pytest

from oracle import mask
import synth


def rect_distance(p, center, a, b):
    # rectangle in the plane x = xc, half sides a (y) and b (z)
    dy = np.maximum(np.abs(p[:, 1] - center[1]) - a, 0.0)
    dz = np.maximum(np.abs(p[:, 2] - center[2]) - b, 0.0)
    dxn = p[:, 0] - center[0]
    return np.sqrt(dxn * dxn + dy * dy + dz * dz)


@pytest.mark.parametrize("ns,nc", [(2, 2), (41, 13)])
def test_flat_rectangle_distance_closed_form(ns, nc, rng):
    center = np.array([1.1, 2.0, 1.7])
    a, b = 0.5, 0.15
    x, tri = synth.flat_rectangle(center, (0, 1, 0), (0, 0, 1), a, b, ns, nc)
    p = center + rng.uniform(-0.8, 0.8, (400, 3))
    best = np.full(len(p), np.inf)
    for t in range(len(tri)):
        d, w = mask.point_triangle(p, x[tri[t, 0]], x[tri[t, 1]], x[tri[t, 2]])
        assert np.all(w >= -1e-12) and np.allclose(w.sum(axis=1), 1.0)
        best = np.minimum(best, d)
    assert np.max(np.abs(best - rect_distance(p, center, a, b))) < 1e-12


def test_point_triangle_against_dense_sampling(rng):
    x, tri = synth.random_triangles(20, (0, 0, 0), (1, 1, 1), 0.6, seed=3)
    p = rng.uniform(-0.3, 1.3, (50, 3))
    m = 300
    uu, vv = np.meshgrid(np.linspace(0, 1, m), np.linspace(0, 1, m))
    keep = uu + vv <= 1.0
    uu, vv = uu[keep], vv[keep]
    for t in range(len(tri)):
        a, b, c = x[tri[t, 0]], x[tri[t, 1]], x[tri[t, 2]]
        d, w = mask.point_triangle(p, a, b, c)
        cp = w @ np.stack([a, b, c])
        # the reported closest point reproduces the distance
        assert np.max(np.abs(np.linalg.norm(p - cp, axis=1) - d)) < 1e-12
        samples = a + uu[:, None] * (b - a) + vv[:, None] * (c - a)
        dd = np.sqrt(((p[:, None, :] - samples[None]) ** 2).sum(-1)).min(axis=1)
        spacing = max(np.linalg.norm(b - a), np.linalg.norm(c - a)) / (m - 1)
        assert np.all(d <= dd + 1e-12)
        assert np.all(d >= dd - 2 * spacing)


def test_profile_fixed_values():
    tw, h = 0.2, 0.1
    c = mask.chi_profile([tw - h - 1e-3, tw - h, tw, tw + h, tw + h + 1e-3], tw, h, mask.PROFILE_COS)
    assert list(c) == [1.0, 1.0, pytest.approx(0.5, abs=1e-15), 0.0, 0.0]
    t = mask.chi_profile([tw, tw + 6 * h - 1e-9, tw + 6 * h], tw, h, mask.PROFILE_TANH)
    assert t[0] == 0.5
    assert t[1] == pytest.approx(0.5 * (1 - np.tanh(6.0)), rel=1e-6)
    assert t[2] == 0.0
    # C1 continuity of the cosine ramp at both ends
    e = 1e-6
    d1 = (mask.chi_profile(tw - h + e, tw, h, 0) - 1.0) / e
    d2 = (mask.chi_profile(tw + h - e, tw, h, 0)) / e
    assert abs(d1) < 1e-4 and abs(d2) < 1e-4


def test_culled_equals_brute_force(rng):
    n = (20, 16, 18)
    L = (2.0, 1.6, 1.8)
    x, tri = synth.random_triangles(12, (0.6, 0.55, 0.6), (1.4, 1.05, 1.2), 0.4, seed=7)
    v = rng.standard_normal(x.shape)
    for prof in (mask.PROFILE_COS, mask.PROFILE_TANH):
        c1, u1 = mask.build_mask(n, L, x, v, tri, 0.1, 0.03, prof, cull=True)
        c2, u2 = mask.build_mask(n, L, x, v, tri, 0.1, 0.03, prof, cull=False)
        assert np.array_equal(c1, c2)
        assert np.array_equal(u1, u2)
        assert np.count_nonzero(c1) > 100


def test_mask_of_flat_plate_matches_closed_form():
    n = (32, 32, 32)
    L = (2 * np.pi,) * 3
    dx = L[0] / 32
    center = np.array([np.pi / 2, np.pi, np.pi])
    x, tri = synth.flat_rectangle(center, (0, 1, 0), (0, 0, 1), 0.5, 0.15, 41, 13)
    chi, us = mask.build_mask(n, L, x, np.zeros_like(x), tri, 2 * dx, dx, mask.PROFILE_COS)
    g = np.arange(32) * dx
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    p = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    d = rect_distance(p, center, 0.5, 0.15).reshape(32, 32, 32)
    expect = mask.chi_profile(d, 2 * dx, dx, mask.PROFILE_COS)
    assert np.max(np.abs(chi - expect)) < 1e-12
    assert np.all(us == 0.0)


def test_rigid_rotation_solid_velocity():
    # plate in the plane z = zc rotating rigidly about the vertical axis through (xa, ya)
    n = (24, 24, 16)
    L = (3.0, 3.0, 2.0)
    dx = L[0] / 24
    center = np.array([1.7, 1.4, 1.0])
    x, tri = synth.flat_rectangle(center, (1, 0, 0), (0, 1, 0), 0.6, 0.3, 7, 4)
    axis = np.array([1.0, 1.5, 0.0])
    om = 2.5
    v = np.stack([-om * (x[:, 1] - axis[1]), om * (x[:, 0] - axis[0]), np.zeros(len(x))], axis=1)
    chi, us = mask.build_mask(n, L, x, v, tri, 2 * dx, dx, mask.PROFILE_COS)
    gx = np.arange(24) * dx
    gy = np.arange(24) * dx
    gz = np.arange(16) * (L[2] / 16)
    zz, yy, xx = np.meshgrid(gz, gy, gx, indexing="ij")
    cx = np.clip(xx, center[0] - 0.6, center[0] + 0.6)
    cy = np.clip(yy, center[1] - 0.3, center[1] + 0.3)
    ex = -om * (cy - axis[1])
    ey = om * (cx - axis[0])
    on = chi > 0
    assert np.count_nonzero(on) > 50
    assert np.max(np.abs(us[0][on] - ex[on])) < 1e-12
    assert np.max(np.abs(us[1][on] - ey[on])) < 1e-12
    assert np.all(us[2] == 0.0)
    assert np.all(us[:, ~on] == 0.0)


def test_bounds_error():
    n = (16, 16, 16)
    L = (1.0, 1.0, 1.0)
    x, tri = synth.flat_rectangle((0.05, 0.5, 0.5), (0, 1, 0), (0, 0, 1), 0.2, 0.2)
    with pytest.raises(ValueError):
        mask.build_mask(n, L, x, np.zeros_like(x), tri, 0.1, 0.05, mask.PROFILE_COS)
