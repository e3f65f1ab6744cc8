"""Mass-spring wing model (Sec. 2, "Flexible wing") - FP64 oracle.

Test infrastructure only: a plain, slow and obviously correct statement of the
structure model that the library's native solver is checked against.

* Newton's second law for mass points, written as a first-order system
  dq/dt = f(q) with the phase vector q = [x, v] (Sec. 2.1, Eqs. Newton_law,
  Newton_law_first_order, first_order_ODEs).
* Variable-step second-order backward differentiation in time (Sec. 2.1,
  Eq. discretized_ODEs), solved for q^{n+1} by Newton-Raphson from the guess
  q^n.  Reading: the first step has no q^{n-1} and uses xi = 0 (implicit
  Euler); Newton stops when ||dq|| <= tol max(1, ||q||).
* Linear extension springs (Sec. 2.2, Eq. extension_spring): energy
  k/2 (|x_j - x_i| - l0)^2, whose gradient gives the printed force.
* Bending springs (Sec. 2.2, Eqs. bending_spring_moment, two_bending_angles):
  two projected angles theta^y (Oxy plane) and theta^z (Oxz plane) between the
  segments i->j and j->k, measured in the wing frame.  Reading: the printed
  angles suit springs along the wing x axis; a spring along wing axis a uses
  the planes (a, a+1) and (a, a+2) (cyclic), a = 0 being the printed case.
  Reading: the printed
  force formula omits the 1/length factors of the angle's gradient, so the
  force is taken as the exact negative gradient of the energy
  k^b/2 [(theta^y - theta^y_0)^2 + (theta^z - theta^z_0)^2]; its moment is the
  printed -k^b (theta - theta_0).
* Bending stiffness from flexural rigidity (Sec. 2.3.1, Eq. EI_k_relation).

The Newton Jacobian here is a central finite difference of the residual (the
root is fixed by the residual alone, so the Jacobian only affects the path);
columns whose rows do not overlap (vertices more than two springs apart) are
differenced together, and the sparse system is solved by scipy.
Pins: tests/test_oracle_structure.py.
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


# ---------------------------------------------------------------------------
# spring network description
# ---------------------------------------------------------------------------

class Network:
    """Mass points with extension and bending springs.

    mass: (n,) ; ext: rows (i, j, k, l0) ; bend: rows (i, j, k, kb, th0y, th0z)
    or (i, j, k, kb, th0_1, th0_2, axis) for a spring along wing axis ``axis``;
    clamped: indices of points whose motion is prescribed.
    """

    def __init__(self, mass, ext=(), bend=(), clamped=()):
        self.mass = np.asarray(mass, dtype=np.float64)
        ext = np.asarray(ext, dtype=np.float64).reshape(-1, 4)
        bend = [tuple(b) + (0,) * (7 - len(b)) for b in bend]
        bend = np.asarray(bend, dtype=np.float64).reshape(-1, 7)
        self.ext_ij = ext[:, :2].astype(np.int64)
        self.ext_k, self.ext_l0 = ext[:, 2].copy(), ext[:, 3].copy()
        self.bend_ijk = bend[:, :3].astype(np.int64)
        self.bend_kb, self.bend_th0 = bend[:, 3].copy(), bend[:, 4:6].copy()
        self.bend_axis = bend[:, 6].astype(np.int64)
        self.clamped = np.array(sorted(set(int(c) for c in clamped)), dtype=np.int64)

    @property
    def n(self):
        return len(self.mass)


def bending_stiffness(EI, l_b, n):
    """k^b of a vein of length l_b carrying n bending springs (Eq. EI_k_relation)."""
    return EI / l_b * n * (2 * n + 1) / (2.0 * (n + 1))


def projected_angle(a, b):
    """Signed angle from segment a to segment b of 2-D polylines (Eq. theta_2D),
    with its gradients with respect to a and b; a, b: (..., 2)."""
    c = a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]
    d = a[..., 0] * b[..., 0] + a[..., 1] * b[..., 1]
    th = np.arctan2(c, d)
    s = c * c + d * d
    # d theta = (d dc - c dd) / (c^2 + d^2)
    ga = np.stack([d * b[..., 1] - c * b[..., 0], -d * b[..., 0] - c * b[..., 1]], axis=-1) / s[..., None]
    gb = np.stack([-d * a[..., 1] - c * a[..., 0], d * a[..., 0] - c * a[..., 1]], axis=-1) / s[..., None]
    return th, ga, gb


def _segments(x, ijk, frame, axis):
    """Segments i->j and j->k of every bending spring in wing coordinates,
    cyclically permuted so that component 0 is the spring's own wing axis."""
    a = (x[ijk[:, 1]] - x[ijk[:, 0]]) @ frame
    b = (x[ijk[:, 2]] - x[ijk[:, 1]]) @ frame
    perm = (np.asarray(axis)[:, None] + np.arange(3)[None, :]) % 3
    rows = np.arange(len(a))[:, None]
    return a[rows, perm], b[rows, perm], perm


def bending_angles(x, ijk, frame, axis=None):
    """(theta^y, theta^z) of Eq. two_bending_angles, (m, 2), for points x given
    in the inertial frame; ``frame`` (3x3) has the wing axes as columns."""
    ijk = np.asarray(ijk).reshape(-1, 3)
    axis = np.zeros(len(ijk), dtype=np.int64) if axis is None else np.asarray(axis)
    a, b, _ = _segments(x, ijk, frame, axis)
    ty, _, _ = projected_angle(a[:, [0, 1]], b[:, [0, 1]])
    tz, _, _ = projected_angle(a[:, [0, 2]], b[:, [0, 2]])
    return np.stack([ty, tz], axis=-1)


def energy(net, x, frame):
    """Elastic energy of the network at positions x (n, 3)."""
    L = np.linalg.norm(x[net.ext_ij[:, 1]] - x[net.ext_ij[:, 0]], axis=1)
    e = 0.5 * np.sum(net.ext_k * (L - net.ext_l0) ** 2)
    if len(net.bend_kb):
        th = bending_angles(x, net.bend_ijk, frame, net.bend_axis)
        e += 0.5 * np.sum(net.bend_kb[:, None] * (th - net.bend_th0) ** 2)
    return e


def internal_forces(net, x, frame):
    """-grad energy (n, 3)."""
    f = np.zeros_like(x)
    i, j = net.ext_ij[:, 0], net.ext_ij[:, 1]
    d = x[j] - x[i]
    L = np.linalg.norm(d, axis=1)
    fi = (net.ext_k * (L - net.ext_l0) / L)[:, None] * d  # Eq. extension_spring
    np.add.at(f, i, fi)
    np.add.at(f, j, -fi)
    if len(net.bend_kb):
        ijk = net.bend_ijk
        a, b, perm = _segments(x, ijk, frame, net.bend_axis)
        ga3 = np.zeros_like(a)
        gb3 = np.zeros_like(b)
        for col, (p, q) in enumerate(((0, 1), (0, 2))):
            th, ga, gb = projected_angle(a[:, [p, q]], b[:, [p, q]])
            m = net.bend_kb * (th - net.bend_th0[:, col])  # dE/dtheta
            ga3[:, [p, q]] += m[:, None] * ga
            gb3[:, [p, q]] += m[:, None] * gb
        # undo the permutation, back to the inertial frame; a = x_j - x_i, b = x_k - x_j
        rows = np.arange(len(a))[:, None]
        gaw = np.zeros_like(ga3)
        gbw = np.zeros_like(gb3)
        gaw[rows, perm] = ga3
        gbw[rows, perm] = gb3
        ga3 = gaw @ frame.T
        gb3 = gbw @ frame.T
        np.add.at(f, ijk[:, 0], ga3)
        np.add.at(f, ijk[:, 1], gb3 - ga3)
        np.add.at(f, ijk[:, 2], -gb3)
    return f


# ---------------------------------------------------------------------------
# time stepping
# ---------------------------------------------------------------------------

def bdf2_coefficients(dt, dt_prev):
    """(alpha, beta, gamma) with q^{n+1} - alpha q^n + beta q^{n-1} = gamma dt f(q^{n+1})
    (Eq. discretized_ODEs); dt_prev = None gives implicit Euler (xi = 0)."""
    xi = 0.0 if dt_prev is None else dt / dt_prev
    return (1 + xi) ** 2 / (1 + 2 * xi), xi ** 2 / (1 + 2 * xi), (1 + xi) / (1 + 2 * xi)


def rhs(net, q, frame, f_ext):
    """f(q) = [v, (F_int + F_ext) / m] (Eq. first_order_ODEs), q = (2, n, 3)."""
    x, v = q
    a = (internal_forces(net, x, frame) + f_ext) / net.mass[:, None]
    return np.stack([v, a])


def neighbourhoods(net):
    """N[v]: v and every point sharing a spring with it."""
    nb = [{v} for v in range(net.n)]
    for i, j in net.ext_ij:
        nb[i].add(j)
        nb[j].add(i)
    for t in net.bend_ijk:
        for a in t:
            nb[a].update(int(b) for b in t)
    return [np.array(sorted(x)) for x in nb]


def colours(nbhd):
    """Greedy colouring with N[a] and N[b] disjoint within a colour."""
    n = len(nbhd)
    col = -np.ones(n, dtype=np.int64)
    for v in range(n):
        near = set()
        for w in nbhd[v]:
            for u in nbhd[w]:
                if col[u] >= 0:
                    near.add(int(col[u]))
        c = 0
        while c in near:
            c += 1
        col[v] = c
    return col


def fd_jacobian(residual, z, groups, m, fd_h):
    """Central-difference Jacobian (m x len(z), sparse): groups is a list of
    lists of (column, rows) whose row sets are disjoint within a group."""
    rows_all, cols_all, vals_all = [], [], []
    for grp in groups:
        h = np.zeros_like(z)
        for c, _ in grp:
            h[c] = fd_h * max(1.0, abs(z[c]))
        d = residual(z + h) - residual(z - h)
        for c, rows in grp:
            rows_all.append(rows)
            cols_all.append(np.full(len(rows), c))
            vals_all.append(d[rows] / (2 * h[c]))
    return sp.csr_matrix((np.concatenate(vals_all), (np.concatenate(rows_all), np.concatenate(cols_all))),
                         shape=(m, len(z)))


def bdf2_step(net, q, q_prev, dt, dt_prev, frame, f_ext, clamp_x=None, clamp_v=None, tol=1e-12, max_iter=50,
              fd_h=1e-7):
    """One structure step: returns (q^{n+1}, Newton iterations).

    q, q_prev: (2, n, 3) phase vectors at t^n and t^{n-1} (q_prev ignored when
    dt_prev is None); clamped points take clamp_x, clamp_v at t^{n+1}."""
    alpha, beta, gamma = bdf2_coefficients(dt, dt_prev)
    base = alpha * q - (beta * q_prev if dt_prev is not None else 0.0)
    n = net.n
    free = np.ones(n, dtype=bool)
    free[net.clamped] = False

    def residual(qn):
        r = qn - base - gamma * dt * rhs(net, qn, frame, f_ext)
        if len(net.clamped):
            r[0, net.clamped] = qn[0, net.clamped] - clamp_x
            r[1, net.clamped] = qn[1, net.clamped] - clamp_v
        return r.reshape(-1)

    qn = q.copy()
    if len(net.clamped):
        qn[0, net.clamped] = clamp_x
        qn[1, net.clamped] = clamp_v
    m = qn.size
    # column groups: x of vertex v touches its x row and the v rows of N[v]; v of
    # a vertex touches only its own rows
    nbhd = neighbourhoods(net)
    col = colours(nbhd)
    groups = []
    for c in range(3):
        for k in range(int(col.max()) + 1):
            grp = []
            for v in np.flatnonzero(col == k):
                vrows = (n * 3 + nbhd[v][:, None] * 3 + np.arange(3)[None, :]).ravel()
                grp.append((v * 3 + c, np.concatenate([[v * 3 + c], vrows])))
            groups.append(grp)
        groups.append([(n * 3 + v * 3 + c, np.array([v * 3 + c, n * 3 + v * 3 + c])) for v in range(n)])
    for it in range(1, max_iter + 1):
        r = residual(qn)
        J = fd_jacobian(lambda z: residual(z.reshape(qn.shape)), qn.reshape(-1), groups, m, fd_h)
        dq = spla.spsolve(J.tocsc(), -r)
        qn = qn + dq.reshape(qn.shape)
        if np.linalg.norm(dq) <= tol * max(1.0, np.linalg.norm(qn)):
            return qn, it
    raise RuntimeError("Newton did not converge")


def static_equilibrium(net, x0, frame, f_ext, clamp_x=None, load_steps=20, tol=1e-12, max_iter=50, fd_h=1e-7):
    """Positions with F_int(x) + F_ext = 0 (clamped points fixed), by Newton with
    the load applied in ``load_steps`` equal increments."""
    x = x0.copy()
    free = np.ones(net.n, dtype=bool)
    free[net.clamped] = False
    if len(net.clamped):
        x[net.clamped] = clamp_x
    idx = np.flatnonzero(np.repeat(free, 3))
    for s in range(1, load_steps + 1):
        fe = f_ext * (s / load_steps)

        def res(xf):
            xx = x.copy().reshape(-1)
            xx[idx] = xf
            return (internal_forces(net, xx.reshape(x.shape), frame) + fe).reshape(-1)[idx]

        xf = x.reshape(-1)[idx].copy()
        for _ in range(max_iter):
            r = res(xf)
            J = np.empty((len(idx), len(idx)))
            for c in range(len(idx)):
                h = fd_h * max(1.0, abs(xf[c]))
                hp = xf.copy()
                hm = xf.copy()
                hp[c] += h
                hm[c] -= h
                J[:, c] = (res(hp) - res(hm)) / (2 * h)
            d = np.linalg.solve(J, -r)
            xf = xf + d
            if np.linalg.norm(d) <= tol * max(1.0, np.linalg.norm(xf)):
                break
        else:
            raise RuntimeError("static Newton did not converge")
        xx = x.reshape(-1).copy()
        xx[idx] = xf
        x = xx.reshape(x.shape)
    return x


# ---------------------------------------------------------------------------
# networks of the paper's tests
# ---------------------------------------------------------------------------

def cantilever(n, l_b, EI, ke, mass=1.0):
    """Vein along the wing x axis: n + 2 points spaced l_b / (n + 1) from the
    root (point 0) to the tip (point n + 1), the first two clamped, extension
    springs between neighbours (stiffness ke) and n bending springs of
    stiffness k^b(EI) at points 1..n (Sec. 2.3.1: the beam of length l_b whose
    energy the network matches)."""
    npts = n + 2
    ds = l_b / (n + 1)
    x = np.zeros((npts, 3))
    x[:, 0] = ds * np.arange(npts)  # root point 0 at the origin, tip at l_b
    kb = bending_stiffness(EI, l_b, n)
    ext = [(i, i + 1, ke, ds) for i in range(npts - 1)]
    bend = [(i - 1, i, i + 1, kb, 0.0, 0.0) for i in range(1, npts - 1)]
    return Network(np.full(npts, mass), ext, bend, clamped=(0, 1)), x


def lumped_masses(x, tri, density):
    """Mass of each point: areal density x one third of the area of its triangles
    (reading of the wing's mass distribution for a uniform membrane)."""
    x = np.asarray(x, dtype=np.float64)
    m = np.zeros(len(x))
    for t in np.asarray(tri):
        area = 0.5 * np.linalg.norm(np.cross(x[t[1]] - x[t[0]], x[t[2]] - x[t[0]]))
        m[t] += density * area / 3.0
    return m


def rest_network(mass, x, ext_ij, ext_k, bend_ijk, bend_kb, bend_axis, clamped, frame):
    """Network at rest in configuration x: rest lengths and rest angles from x."""
    x = np.asarray(x, dtype=np.float64)
    ext_ij = np.asarray(ext_ij).reshape(-1, 2)
    l0 = np.linalg.norm(x[ext_ij[:, 1]] - x[ext_ij[:, 0]], axis=1)
    bend_ijk = np.asarray(bend_ijk).reshape(-1, 3)
    th0 = bending_angles(x, bend_ijk, frame, bend_axis)
    ext = [(i, j, k, l) for (i, j), k, l in zip(ext_ij, ext_k, l0)]
    bend = [(i, j, k, kb, t[0], t[1], a) for (i, j, k), kb, t, a in zip(bend_ijk, bend_kb, th0, bend_axis)]
    return Network(mass, ext, bend, clamped)
