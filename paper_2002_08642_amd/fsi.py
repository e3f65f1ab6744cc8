"""Thin ctypes binding of libfsi.so (include/fsi.h, include/fsi_ms.h).

Argument marshalling only: every step of the method runs in the HIP library.
The library must be built (``python -m paper_2002_08642_amd.build`` or
``__graft_entry__.build()``); loading fails loudly if it is missing.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfsi.so")

FSI_OK = 0
STATUS = {
    0: "FSI_OK", -1: "FSI_EINVAL", -2: "FSI_ENOMEM", -3: "FSI_EDEVICE", -4: "FSI_EBOUNDS",
    -5: "FSI_ESTATE", -6: "FSI_ENAN", -7: "FSI_ESTABILITY",
}
PROFILE_COS = 0
PROFILE_TANH = 1
PREC_FP32 = 0
PREC_FP64 = 1
NPASS = 7
TIME_PASSES = 0x100  # FSI_TIME_PASSES
PASS_NAMES = ["mask", "z_inverse_curl", "y_inverse", "x_fused", "reduce_dt", "y_forward", "z_forward_update"]

# every symbol declared in include/*.h
EXPORTS = [
    "fsi_ms_create", "fsi_ms_destroy", "fsi_ms_last_error", "fsi_ms_add_extension", "fsi_ms_add_bending",
    "fsi_ms_set_extension_k", "fsi_ms_set_bending_k", "fsi_ms_set_clamped", "fsi_ms_bending_angles",
    "fsi_ms_forces", "fsi_ms_set_state", "fsi_ms_get_state", "fsi_ms_step", "fsi_ms_static",
    "fsi_ms_set_rest", "fsi_ms_bending_stiffness", "fsi_ms_lumped_masses", "fsi_plate_frame",
    "fsi_ms_set_history", "fsi_ms_step_adjoint", "fsi_plate_frame_dalpha", "fsi_loads_from_box",
    "fsi_loads_adjoint",
    "fsi_version", "fsi_create", "fsi_destroy", "fsi_last_error", "fsi_create_error", "fsi_band",
    "fsi_set_velocity", "fsi_set_velocity_device", "fsi_set_spectrum", "fsi_get_velocity", "fsi_get_spectrum",
    "fsi_set_wing", "fsi_set_sponge", "fsi_get_mask", "fsi_step", "fsi_step_record", "fsi_adjoint_reset",
    "fsi_step_adaptive", "fsi_get_step_info",
    "fsi_fft_r2c", "fsi_fft_c2r", "fsi_save_state", "fsi_load_state", "fsi_synchronize",
    "fsi_set_timing", "fsi_get_pass_times", "fsi_plate_pose", "fsi_get_nonlinear",
    "fsi_adjoint_set", "fsi_adjoint_get", "fsi_step_adjoint", "fsi_plate_pose_dalpha",
    "fsi_sample_pressure", "fsi_get_pressure_loads", "fsi_get_pressure_box", "fsi_adjoint_set_pressure_seed",
    "fsi_get_mask_noalloc", "fsi_eval_pressure", "fsi_set_static_mask", "fsi_get_static_force",
    "fsi_debug_poison_padding",
]
NOALLOC_MASK_CELLS = 1 << 20  # FSI_NOALLOC_MASK_CELLS


class FsiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
        ("nu", ctypes.c_double), ("eta", ctypes.c_double),
        ("tw", ctypes.c_double), ("h", ctypes.c_double),
        ("mask_profile", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("fsi_pressure", ctypes.c_int32), ("stream", ctypes.c_void_p),
    ]


_lib = None


def load_library():
    """Load libfsi.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("HIP library %s is not built; run paper_2002_08642_amd.build.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    D = ctypes.POINTER(ctypes.c_double)
    I32 = ctypes.c_int32
    lib.fsi_version.restype = I32
    lib.fsi_create.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(P)]
    lib.fsi_destroy.argtypes = [P]
    lib.fsi_last_error.argtypes = [P]
    lib.fsi_last_error.restype = ctypes.c_char_p
    lib.fsi_create_error.restype = ctypes.c_char_p
    lib.fsi_band.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(ctypes.c_int64)]
    lib.fsi_set_velocity.argtypes = [P, D]
    lib.fsi_set_velocity_device.argtypes = [P, P, I32]
    lib.fsi_set_spectrum.argtypes = [P, D]
    lib.fsi_get_velocity.argtypes = [P, D]
    lib.fsi_get_spectrum.argtypes = [P, D]
    lib.fsi_set_wing.argtypes = [P, I32, D, D, I32, ctypes.POINTER(I32)]
    lib.fsi_set_sponge.argtypes = [P, ctypes.c_double, D, D, D]
    lib.fsi_step_record.argtypes = [P, ctypes.c_double, I32]
    lib.fsi_adjoint_reset.argtypes = [P]
    lib.fsi_get_mask.argtypes = [P, D, D]
    lib.fsi_get_mask_noalloc.argtypes = [P, P, P]
    lib.fsi_step.argtypes = [P, ctypes.c_double]
    lib.fsi_step_adaptive.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.fsi_get_step_info.argtypes = [P, D, D, D, D, D, ctypes.POINTER(ctypes.c_int64)]
    lib.fsi_fft_r2c.argtypes = [P, D, D]
    lib.fsi_fft_c2r.argtypes = [P, D, D]
    lib.fsi_save_state.argtypes = [P, I32]
    lib.fsi_load_state.argtypes = [P, I32]
    lib.fsi_synchronize.argtypes = [P]
    lib.fsi_set_timing.argtypes = [P, I32]
    lib.fsi_get_pass_times.argtypes = [P, D, ctypes.POINTER(I32)]
    lib.fsi_debug_poison_padding.argtypes = [P, ctypes.c_double]
    lib.fsi_plate_pose.argtypes = [I32, D, D, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, I32, D, D, D, D]
    lib.fsi_get_nonlinear.argtypes = [P, D]
    lib.fsi_adjoint_set.argtypes = [P, D, D]
    lib.fsi_adjoint_get.argtypes = [P, D, D]
    lib.fsi_step_adjoint.argtypes = [P, I32, ctypes.c_double, ctypes.c_double, I32, D, D, D]
    lib.fsi_plate_pose_dalpha.argtypes = [I32, D, D, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, I32, D, D]
    lib.fsi_sample_pressure.argtypes = [P, I32, D, D]
    lib.fsi_get_pressure_loads.argtypes = [P, D, D]
    lib.fsi_eval_pressure.argtypes = [P]
    lib.fsi_set_static_mask.argtypes = [P, D, D, D]
    lib.fsi_get_static_force.argtypes = [P, D]
    lib.fsi_get_pressure_box.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I32), D]
    lib.fsi_adjoint_set_pressure_seed.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I32), D]
    lib.fsi_ms_create.argtypes = [I32, D, ctypes.POINTER(P)]
    lib.fsi_ms_destroy.argtypes = [P]
    lib.fsi_ms_last_error.argtypes = [P]
    lib.fsi_ms_last_error.restype = ctypes.c_char_p
    lib.fsi_ms_add_extension.argtypes = [P, I32, ctypes.POINTER(I32), D, D, ctypes.POINTER(I32)]
    lib.fsi_ms_add_bending.argtypes = [P, I32, ctypes.POINTER(I32), D, D, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    lib.fsi_ms_set_rest.argtypes = [P, D]
    lib.fsi_ms_bending_stiffness.argtypes = [ctypes.c_double, ctypes.c_double, I32, D]
    lib.fsi_ms_lumped_masses.argtypes = [I32, D, I32, ctypes.POINTER(I32), ctypes.c_double, D]
    lib.fsi_plate_frame.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, I32, D, D]
    lib.fsi_plate_frame_dalpha.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, I32, D]
    lib.fsi_ms_set_history.argtypes = [P, D, D, ctypes.c_double]
    lib.fsi_loads_from_box.argtypes = [I32, D, I32, ctypes.POINTER(I32), ctypes.c_double, D, ctypes.POINTER(I32),
                                       ctypes.POINTER(I32), D, D, D]
    lib.fsi_loads_adjoint.argtypes = [I32, D, I32, ctypes.POINTER(I32), ctypes.c_double, D, ctypes.POINTER(I32),
                                      ctypes.POINTER(I32), D, D, D, D]
    lib.fsi_ms_step_adjoint.argtypes = [P, ctypes.c_double, ctypes.c_double, D, D, D, D, D] + [D] * 10
    lib.fsi_ms_set_extension_k.argtypes = [P, D]
    lib.fsi_ms_set_bending_k.argtypes = [P, D]
    lib.fsi_ms_set_clamped.argtypes = [P, I32, ctypes.POINTER(I32)]
    lib.fsi_ms_bending_angles.argtypes = [P, D, D, D]
    lib.fsi_ms_forces.argtypes = [P, D, D, D, D]
    lib.fsi_ms_set_state.argtypes = [P, D, D]
    lib.fsi_ms_get_state.argtypes = [P, D, D]
    lib.fsi_ms_step.argtypes = [P, ctypes.c_double, D, D, D, D, ctypes.c_double, I32, ctypes.POINTER(I32)]
    lib.fsi_ms_static.argtypes = [P, D, D, I32, ctypes.c_double, I32]
    for name in EXPORTS:
        getattr(lib, name).restype = getattr(lib, name).restype if name in (
            "fsi_last_error", "fsi_create_error", "fsi_version", "fsi_ms_last_error") else ctypes.c_int32
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != tuple(shape):
        a = a.reshape(shape)
    return a


def plate_pose(s, c, t, alpha, omega, t_ramp, axis, law=0):
    """Rigid revolving-plate vertex positions and velocities (fsi_plate_pose)."""
    lib = load_library()
    s = _f64(s)
    c = _f64(c)
    nv = s.shape[0]
    x = np.zeros((nv, 3))
    v = np.zeros((nv, 3))
    ph = np.zeros(2)
    ax = _f64(axis)
    rc = lib.fsi_plate_pose(nv, _dptr(s), _dptr(c), t, alpha, omega, t_ramp, law, _dptr(ax),
                            _dptr(x), _dptr(v), _dptr(ph))
    if rc != FSI_OK:
        raise FsiError(rc, "fsi_plate_pose")
    return x, v, ph


def plate_pose_dalpha(s, c, t, alpha, omega, t_ramp, law=0):
    """Derivatives of the rigid plate pose with respect to the pitch (fsi_plate_pose_dalpha)."""
    lib = load_library()
    s = _f64(s)
    c = _f64(c)
    nv = s.shape[0]
    dx = np.zeros((nv, 3))
    dv = np.zeros((nv, 3))
    rc = lib.fsi_plate_pose_dalpha(nv, _dptr(s), _dptr(c), t, alpha, omega, t_ramp, law, _dptr(dx), _dptr(dv))
    if rc != FSI_OK:
        raise FsiError(rc, "fsi_plate_pose_dalpha")
    return dx, dv


class Solver:
    """One context of the penalized pseudo-spectral step (see include/fsi.h)."""

    def __init__(self, n, L, nu, eta, tw=0.0, h=1.0, profile=PROFILE_COS, precision=PREC_FP32, stream=None,
                 pressure=False):
        self.lib = load_library()
        self.n = tuple(int(a) for a in n)
        self.L = tuple(float(a) for a in L)
        self.tw, self.h = float(tw), float(h)
        nx, ny, nz = self.n
        d = Desc(nx, ny, nz, float(L[0]), float(L[1]), float(L[2]), float(nu), float(eta), float(tw),
                 float(h), int(profile), int(precision), 1 if pressure else 0, stream)
        ctx = ctypes.c_void_p()
        rc = self.lib.fsi_create(ctypes.byref(d), ctypes.byref(ctx))
        if rc != FSI_OK:
            raise FsiError(rc, self.lib.fsi_create_error().decode())
        self.ctx = ctx
        K = (ctypes.c_int32 * 3)()
        cl = ctypes.c_int64()
        self._check(self.lib.fsi_band(self.ctx, K, ctypes.byref(cl)))
        self.K = (K[0], K[1], K[2])
        self.compact_len = cl.value

    def _check(self, rc):
        if rc != FSI_OK:
            raise FsiError(rc, self.lib.fsi_last_error(self.ctx).decode())

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.fsi_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape3(self):
        nx, ny, nz = self.n
        return (nz, ny, nx)

    @property
    def compact_shape(self):
        Kx, Ky, Kz = self.K
        return (2 * Kz + 1, 2 * Ky + 1, Kx + 1)

    def set_velocity(self, u):
        u = _f64(u, (3,) + self.shape3)
        self._check(self.lib.fsi_set_velocity(self.ctx, _dptr(u)))

    def set_velocity_device(self, ptr, dtype):
        self._check(self.lib.fsi_set_velocity_device(self.ctx, ctypes.c_void_p(ptr), int(dtype)))

    def set_spectrum(self, uh):
        uh = np.asarray(uh, dtype=np.complex128).reshape((3,) + self.compact_shape)
        buf = np.ascontiguousarray(np.stack([uh.real, uh.imag], axis=-1))
        self._check(self.lib.fsi_set_spectrum(self.ctx, _dptr(buf)))

    def velocity(self):
        u = np.zeros((3,) + self.shape3)
        self._check(self.lib.fsi_get_velocity(self.ctx, _dptr(u)))
        return u

    def spectrum(self):
        out = np.zeros((3,) + self.compact_shape + (2,))
        self._check(self.lib.fsi_get_spectrum(self.ctx, _dptr(out)))
        return out[..., 0] + 1j * out[..., 1]

    def nonlinear(self):
        out = np.zeros((3,) + self.compact_shape + (2,))
        self._check(self.lib.fsi_get_nonlinear(self.ctx, _dptr(out)))
        return out[..., 0] + 1j * out[..., 1]

    def _cbuf(self, a):
        if a is None:
            return None
        a = np.asarray(a, dtype=np.complex128).reshape((3,) + self.compact_shape)
        return np.ascontiguousarray(np.stack([a.real, a.imag], axis=-1))

    def adjoint_reset(self):
        self._check(self.lib.fsi_adjoint_reset(self.ctx))

    def step_record(self, dt, slot):
        """fsi_step_record: save the state in tape slot `slot`, then step."""
        self._check(self.lib.fsi_step_record(self.ctx, float(dt), int(slot)))

    def adjoint_set(self, lam_u=None, lam_n=None):
        bu, bn = self._cbuf(lam_u), self._cbuf(lam_n)
        self._check(self.lib.fsi_adjoint_set(self.ctx, None if bu is None else _dptr(bu),
                                             None if bn is None else _dptr(bn)))

    def adjoint_get(self):
        bu = np.zeros((3,) + self.compact_shape + (2,))
        bn = np.zeros((3,) + self.compact_shape + (2,))
        self._check(self.lib.fsi_adjoint_get(self.ctx, _dptr(bu), _dptr(bn)))
        return bu[..., 0] + 1j * bu[..., 1], bn[..., 0] + 1j * bn[..., 1]

    def step_adjoint(self, slot, dt, dt_prev, first, dJdF):
        """Reverse one step (fsi_step_adjoint); returns dJ/dx, dJ/dv of the current wing's vertices."""
        g = _f64(dJdF, (3,))
        nv = getattr(self, "_nv", 0)
        dx = np.zeros((max(nv, 1), 3))
        dv = np.zeros((max(nv, 1), 3))
        self._check(self.lib.fsi_step_adjoint(self.ctx, int(slot), float(dt), float(dt_prev), int(first), _dptr(g),
                                              _dptr(dx), _dptr(dv)))
        return dx[:nv], dv[:nv]

    def set_wing(self, x, v, tri):
        x = _f64(x)
        v = _f64(v)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        nv = x.shape[0] if x.ndim == 2 else 0
        nt = tri.shape[0] if tri.ndim == 2 else 0
        self._check(self.lib.fsi_set_wing(self.ctx, nv, _dptr(x), _dptr(v), nt,
                                          tri.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        self._nv = nv if nt > 0 else 0

    def set_sponge(self, c_sp, gx=None, gy=None, gz=None):
        """Vorticity sponge: chi_sp = max(gx[x], gy[y], gz[z]) (None = 0); c_sp <= 0 switches it off."""
        prof = [None if g is None else _f64(g).ravel() for g in (gx, gy, gz)]
        for g, m in zip(prof, self.n):
            if g is not None and g.size != m:
                raise ValueError("sponge profile length must match the grid")
        self._check(self.lib.fsi_set_sponge(self.ctx, float(c_sp),
                                            *[None if g is None else _dptr(g) for g in prof]))
        self._sponge_keep = prof

    def set_static_mask(self, chi, us, weight=None):
        """Static z-independent penalization chi (ny, nx), u_s (3, ny, nx), force
        weight (ny, nx) or None; chi = None removes it (fsi_set_static_mask)."""
        nx, ny, _ = self.n
        if chi is None:
            self._check(self.lib.fsi_set_static_mask(self.ctx, None, None, None))
            return
        c = _f64(chi, (ny, nx))
        u = _f64(us, (3, ny, nx))
        w = None if weight is None else _f64(weight, (ny, nx))
        self._check(self.lib.fsi_set_static_mask(self.ctx, _dptr(c), _dptr(u), _optd(w)))

    def static_force(self):
        """Weighted force of the static penalization at t^n of the last step."""
        F = np.zeros(3)
        self._check(self.lib.fsi_get_static_force(self.ctx, _dptr(F)))
        return F

    def clear_wing(self):
        self._check(self.lib.fsi_set_wing(self.ctx, 0, None, None, 0, None))
        self._nv = 0

    def sample_pressure(self, pts):
        """p = Pi - |u|^2/2 of the last step at points (n, 3) (fsi_sample_pressure)."""
        pts = _f64(pts).reshape(-1, 3)
        out = np.zeros(pts.shape[0])
        self._check(self.lib.fsi_sample_pressure(self.ctx, pts.shape[0], _dptr(pts), _dptr(out)))
        return out

    def pressure_loads(self):
        """Vertex loads (nv, 3) and pressure jumps (nv,) of the current mesh (fsi_get_pressure_loads)."""
        loads = np.zeros((self._nv, 3))
        dp = np.zeros(self._nv)
        self._check(self.lib.fsi_get_pressure_loads(self.ctx, _dptr(loads), _dptr(dp)))
        return loads, dp

    def eval_pressure(self):
        """fsi_eval_pressure: the pressure of the current velocity (paper's coupling order)."""
        self._check(self.lib.fsi_eval_pressure(self.ctx))

    def pressure_box(self, values=True):
        """(box0, p) of the current pressure box; p (nz, ny, nx of the box) of the
        last step if values (fsi_get_pressure_box)."""
        b0 = np.zeros(3, dtype=np.int32)
        bn = np.zeros(3, dtype=np.int32)
        self._check(self.lib.fsi_get_pressure_box(self.ctx, _iptr(b0), _iptr(bn), None))
        if not values:
            return b0, None
        p = np.zeros((bn[2], bn[1], bn[0]))
        self._check(self.lib.fsi_get_pressure_box(self.ctx, _iptr(b0), _iptr(bn), _dptr(p)))
        return b0, p

    def adjoint_set_pressure_seed(self, box0, lam_p):
        """Seed the next step_adjoint with the cotangent of p on the pressure box."""
        b0 = _i32(box0, (3,))
        if lam_p is None:
            bn = np.zeros(3, dtype=np.int32)
            self._check(self.lib.fsi_get_pressure_box(self.ctx, _iptr(b0), _iptr(bn), None))
            self._check(self.lib.fsi_adjoint_set_pressure_seed(self.ctx, _iptr(b0), _iptr(bn), None))
            return
        lam_p = _f64(lam_p)
        bn = _i32([lam_p.shape[2], lam_p.shape[1], lam_p.shape[0]])
        self._check(self.lib.fsi_adjoint_set_pressure_seed(self.ctx, _iptr(b0), _iptr(bn), _dptr(lam_p)))

    def mask(self):
        chi = np.zeros(self.shape3)
        us = np.zeros((3,) + self.shape3)
        self._check(self.lib.fsi_get_mask(self.ctx, _dptr(chi), _dptr(us)))
        return chi, us

    def mask_noalloc(self, chi_ptr, us_ptr):
        """fsi_get_mask_noalloc into caller-owned device arrays (addresses as ints,
        the context's precision, [nz][ny][nx] and [3][nz][ny][nx]); no sync."""
        self._check(self.lib.fsi_get_mask_noalloc(self.ctx, ctypes.c_void_p(chi_ptr), ctypes.c_void_p(us_ptr)))

    def step(self, dt):
        self._check(self.lib.fsi_step(self.ctx, float(dt)))

    def step_adaptive(self, cfl, c_eta, dt_max):
        self._check(self.lib.fsi_step_adaptive(self.ctx, float(cfl), float(c_eta), float(dt_max)))

    def info(self):
        F = np.zeros(3)
        v = np.zeros(4)
        ns = ctypes.c_int64()
        rc = self.lib.fsi_get_step_info(self.ctx, _dptr(F), _dptr(v[0:1]), _dptr(v[1:2]), _dptr(v[2:3]),
                                        _dptr(v[3:4]), ctypes.byref(ns))
        self._check(rc)
        return {"F": F, "dt": float(v[0]), "E": float(v[1]), "umax": float(v[2]), "t": float(v[3]),
                "nstep": int(ns.value)}

    def fft_r2c(self, f):
        f = _f64(f, self.shape3)
        out = np.zeros(self.compact_shape + (2,))
        self._check(self.lib.fsi_fft_r2c(self.ctx, _dptr(f), _dptr(out)))
        return out[..., 0] + 1j * out[..., 1]

    def fft_c2r(self, fh):
        fh = np.asarray(fh, dtype=np.complex128).reshape(self.compact_shape)
        buf = np.ascontiguousarray(np.stack([fh.real, fh.imag], axis=-1))
        f = np.zeros(self.shape3)
        self._check(self.lib.fsi_fft_c2r(self.ctx, _dptr(buf), _dptr(f)))
        return f

    def save(self, slot):
        self._check(self.lib.fsi_save_state(self.ctx, int(slot)))

    def load(self, slot):
        self._check(self.lib.fsi_load_state(self.ctx, int(slot)))

    def synchronize(self):
        self._check(self.lib.fsi_synchronize(self.ctx))

    def set_timing(self, on, passes=None):
        """Per-pass HIP-event timing: on/off for every pass, or only the passes
        named in ``passes`` (names of PASS_NAMES)."""
        if on and passes is not None:
            mask = 0
            for p in passes:
                mask |= 1 << PASS_NAMES.index(p)
            self._check(self.lib.fsi_set_timing(self.ctx, TIME_PASSES | mask))
        else:
            self._check(self.lib.fsi_set_timing(self.ctx, 1 if on else 0))

    def poison_padding(self, value):
        """Write (value, value) into the padding columns of every spectral
        buffer (fsi_debug_poison_padding; a layout check for tests)."""
        self._check(self.lib.fsi_debug_poison_padding(self.ctx, float(value)))

    def pass_times(self):
        ms = np.zeros(NPASS)
        n = ctypes.c_int32()
        self._check(self.lib.fsi_get_pass_times(self.ctx, _dptr(ms), ctypes.byref(n)))
        return dict(zip(PASS_NAMES, ms)), int(n.value)


def _i32(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.int32)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _optd(a):
    return None if a is None else _dptr(a)


class MassSpring:
    """Native FP64 mass-spring wing solver (include/fsi_ms.h)."""

    def __init__(self, mass):
        self.lib = load_library()
        mass = _f64(mass)
        self.nv = int(mass.shape[0])
        self.ptr = ctypes.c_void_p()
        rc = self.lib.fsi_ms_create(self.nv, _dptr(mass), ctypes.byref(self.ptr))
        if rc != FSI_OK:
            self.ptr = None
            raise FsiError(rc, "fsi_ms_create")
        self.n_ext = 0
        self.n_bend = 0
        self.clamped = np.zeros(0, dtype=np.int32)

    def _check(self, rc, what):
        if rc != FSI_OK:
            raise FsiError(rc, "%s: %s" % (what, self.lib.fsi_ms_last_error(self.ptr).decode()))

    def close(self):
        if getattr(self, "ptr", None):
            self.lib.fsi_ms_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_extension(self, ij, k, l0):
        ij = _i32(ij, (-1, 2))
        n = ij.shape[0]
        first = ctypes.c_int32()
        self._check(self.lib.fsi_ms_add_extension(self.ptr, n, _iptr(ij), _dptr(_f64(k, (n,))), _dptr(_f64(l0, (n,))),
                                                  ctypes.byref(first)), "fsi_ms_add_extension")
        self.n_ext += n
        return first.value

    def add_bending(self, ijk, kb, theta0=None, axis=None):
        ijk = _i32(ijk, (-1, 3))
        n = ijk.shape[0]
        first = ctypes.c_int32()
        th = np.zeros((n, 2)) if theta0 is None else _f64(theta0, (n, 2))
        ax = None if axis is None else _i32(axis, (n,))
        self._check(self.lib.fsi_ms_add_bending(self.ptr, n, _iptr(ijk), _dptr(_f64(kb, (n,))), _dptr(th),
                                                None if ax is None else _iptr(ax), ctypes.byref(first)),
                    "fsi_ms_add_bending")
        self.n_bend += n
        return first.value

    def set_extension_k(self, k):
        self._check(self.lib.fsi_ms_set_extension_k(self.ptr, _dptr(_f64(k, (self.n_ext,)))), "fsi_ms_set_extension_k")

    def set_bending_k(self, kb):
        self._check(self.lib.fsi_ms_set_bending_k(self.ptr, _dptr(_f64(kb, (self.n_bend,)))), "fsi_ms_set_bending_k")

    def set_rest(self, frame=None):
        fr = None if frame is None else _f64(frame, (3, 3))
        self._check(self.lib.fsi_ms_set_rest(self.ptr, _optd(fr)), "fsi_ms_set_rest")

    def set_clamped(self, idx):
        idx = _i32(idx, (-1,))
        self._check(self.lib.fsi_ms_set_clamped(self.ptr, idx.shape[0], _iptr(idx)), "fsi_ms_set_clamped")
        self.clamped = idx.copy()

    def bending_angles(self, x, frame=None):
        th = np.zeros((self.n_bend, 2))
        fr = None if frame is None else _f64(frame, (3, 3))
        self._check(self.lib.fsi_ms_bending_angles(self.ptr, _dptr(_f64(x, (self.nv, 3))), _optd(fr), _dptr(th)),
                    "fsi_ms_bending_angles")
        return th

    def forces(self, x, frame=None):
        f = np.zeros((self.nv, 3))
        e = ctypes.c_double()
        fr = None if frame is None else _f64(frame, (3, 3))
        self._check(self.lib.fsi_ms_forces(self.ptr, _dptr(_f64(x, (self.nv, 3))), _optd(fr), _dptr(f),
                                           ctypes.byref(e)), "fsi_ms_forces")
        return f, e.value

    def set_state(self, x, v=None):
        vv = None if v is None else _f64(v, (self.nv, 3))
        self._check(self.lib.fsi_ms_set_state(self.ptr, _dptr(_f64(x, (self.nv, 3))), _optd(vv)), "fsi_ms_set_state")

    def state(self):
        x = np.zeros((self.nv, 3))
        v = np.zeros((self.nv, 3))
        self._check(self.lib.fsi_ms_get_state(self.ptr, _dptr(x), _dptr(v)), "fsi_ms_get_state")
        return x, v

    def step(self, dt, frame=None, f_ext=None, x_clamp=None, v_clamp=None, tol=1e-6, max_iter=30):
        nc = len(self.clamped)
        fr = None if frame is None else _f64(frame, (3, 3))
        fe = None if f_ext is None else _f64(f_ext, (self.nv, 3))
        xc = None if x_clamp is None else _f64(x_clamp, (nc, 3))
        vc = None if v_clamp is None else _f64(v_clamp, (nc, 3))
        it = ctypes.c_int32()
        self._check(self.lib.fsi_ms_step(self.ptr, float(dt), _optd(fr), _optd(fe), _optd(xc), _optd(vc), float(tol),
                                         int(max_iter), ctypes.byref(it)), "fsi_ms_step")
        return it.value

    def set_history(self, x_prev=None, v_prev=None, dt_prev=0.0):
        xp = None if x_prev is None else _f64(x_prev, (self.nv, 3))
        vp = None if v_prev is None else _f64(v_prev, (self.nv, 3))
        self._check(self.lib.fsi_ms_set_history(self.ptr, _optd(xp), _optd(vp), float(dt_prev)), "fsi_ms_set_history")

    def step_adjoint(self, dt, dt_prev, frame, x_new, lam_x, lam_v, dframe=None):
        """Transpose of one step (fsi_ms_step_adjoint); returns a dict of cotangents."""
        nv, nc = self.nv, len(self.clamped)
        out = dict(xn=np.zeros((nv, 3)), vn=np.zeros((nv, 3)), xp=np.zeros((nv, 3)), vp=np.zeros((nv, 3)),
                   load=np.zeros((nv, 3)), kext=np.zeros(self.n_ext), kb=np.zeros(self.n_bend),
                   clamp_x=np.zeros((nc, 3)), clamp_v=np.zeros((nc, 3)), dframe=np.zeros(1))
        fr = None if frame is None else _f64(frame, (3, 3))
        dfr = None if dframe is None else _f64(dframe, (3, 3))
        self._check(self.lib.fsi_ms_step_adjoint(
            self.ptr, float(dt), float(dt_prev if dt_prev is not None else 0.0), _optd(fr), _optd(dfr),
            _dptr(_f64(x_new, (nv, 3))), _dptr(_f64(lam_x, (nv, 3))), _dptr(_f64(lam_v, (nv, 3))),
            _dptr(out["xn"]), _dptr(out["vn"]), _dptr(out["xp"]), _dptr(out["vp"]), _dptr(out["load"]),
            _dptr(out["kext"]), _dptr(out["kb"]), _dptr(out["clamp_x"]), _dptr(out["clamp_v"]),
            _dptr(out["dframe"])), "fsi_ms_step_adjoint")
        out["dframe"] = float(out["dframe"][0])
        return out

    def static(self, f_ext, frame=None, load_steps=10, tol=1e-10, max_iter=50):
        fr = None if frame is None else _f64(frame, (3, 3))
        self._check(self.lib.fsi_ms_static(self.ptr, _optd(fr), _dptr(_f64(f_ext, (self.nv, 3))), int(load_steps),
                                           float(tol), int(max_iter)), "fsi_ms_static")


def bending_stiffness(EI, l_b, n):
    """k^b from the flexural rigidity (fsi_ms_bending_stiffness)."""
    kb = ctypes.c_double()
    rc = load_library().fsi_ms_bending_stiffness(float(EI), float(l_b), int(n), ctypes.byref(kb))
    if rc != FSI_OK:
        raise FsiError(rc, "fsi_ms_bending_stiffness")
    return kb.value


def lumped_masses(x, tri, density):
    """Per-vertex masses from triangle areas (fsi_ms_lumped_masses)."""
    x = _f64(x).reshape(-1, 3)
    tri = _i32(tri, (-1, 3))
    m = np.zeros(x.shape[0])
    rc = load_library().fsi_ms_lumped_masses(x.shape[0], _dptr(x), tri.shape[0], _iptr(tri), float(density), _dptr(m))
    if rc != FSI_OK:
        raise FsiError(rc, "fsi_ms_lumped_masses")
    return m


def plate_frame(t, alpha, omega, t_ramp, law=0):
    """Wing frame (3x3, columns span/chord/normal) of the revolving plate (fsi_plate_frame)."""
    fr = np.zeros((3, 3))
    ph = np.zeros(2)
    rc = load_library().fsi_plate_frame(float(t), float(alpha), float(omega), float(t_ramp), int(law), _dptr(fr),
                                        _dptr(ph))
    if rc != FSI_OK:
        raise FsiError(rc, "fsi_plate_frame")
    return fr


def plate_frame_dalpha(t, alpha, omega, t_ramp, law=0):
    """d frame / d alpha of the revolving plate (fsi_plate_frame_dalpha)."""
    fr = np.zeros((3, 3))
    rc = load_library().fsi_plate_frame_dalpha(float(t), float(alpha), float(omega), float(t_ramp), int(law),
                                               _dptr(fr))
    if rc != FSI_OK:
        raise FsiError(rc, "fsi_plate_frame_dalpha")
    return fr


def loads_from_box(x, tri, d, dx, box0, pbox):
    """Wing loads and pressure jumps from a host pressure box (fsi_loads_from_box);
    pbox has shape (nz, ny, nx) of the box."""
    x = _f64(x).reshape(-1, 3)
    tri = _i32(tri, (-1, 3))
    pbox = _f64(pbox)
    boxn = _i32([pbox.shape[2], pbox.shape[1], pbox.shape[0]])
    b0 = _i32(box0, (3,))
    loads = np.zeros_like(x)
    dp = np.zeros(x.shape[0])
    rc = load_library().fsi_loads_from_box(x.shape[0], _dptr(x), tri.shape[0], _iptr(tri), float(d),
                                           _dptr(_f64(dx, (3,))), _iptr(b0), _iptr(boxn), _dptr(pbox),
                                           _dptr(loads), _dptr(dp))
    if rc != FSI_OK:
        raise FsiError(rc, "fsi_loads_from_box")
    return loads, dp


def loads_adjoint(x, tri, d, dx, box0, pbox, lam_load):
    """Cotangents (of x, of pbox) of the loads map (fsi_loads_adjoint)."""
    x = _f64(x).reshape(-1, 3)
    tri = _i32(tri, (-1, 3))
    pbox = _f64(pbox)
    boxn = _i32([pbox.shape[2], pbox.shape[1], pbox.shape[0]])
    b0 = _i32(box0, (3,))
    lx = np.zeros_like(x)
    lp = np.zeros_like(pbox)
    rc = load_library().fsi_loads_adjoint(x.shape[0], _dptr(x), tri.shape[0], _iptr(tri), float(d),
                                          _dptr(_f64(dx, (3,))), _iptr(b0), _iptr(boxn), _dptr(pbox),
                                          _dptr(_f64(lam_load, x.shape)), _dptr(lx), _dptr(lp))
    if rc != FSI_OK:
        raise FsiError(rc, "fsi_loads_adjoint")
    return lx, lp
