"""One penalized pseudo-spectral Navier-Stokes step (oracle; test infrastructure only).

Sec. 4.1 (penalized NS equations): the code advances
    du/dt = u x omega - grad(Pi) + nu lap(u) - (chi/C_eta)(u - u_s),  div u = 0,
with Pi = p + |u|^2/2, a Fourier pseudo-spectral discretization, adaptive
time stepping and an Adams-Bashforth scheme (Sec. 4.1, last paragraph).  The
vorticity sponge term of the same equation is optional (set_sponge; off by
default, as in the paper's workloads): oracle.sponge.

Algorithm of one step n (state: u_hat^n, N_hat^{n-1}, dt_{n-1}, t^n):
 1. u = IDFT(u_hat), omega = IDFT(i k x u_hat);
 2. chi, u_s from the wing mesh (oracle.mask) or an explicit override;
 3. G = u x omega - (chi/eta)(u - u_s);
 4. diagnostics: F = (dV/eta) sum chi (u - u_s) (force on the body),
    u_max = max |u|_2, E = dV/2 sum |u|^2;
 5. dt_n given, or adaptive: min(CFL dx_min / u_max, C_eta eta, dt_max),
    the CFL term being +inf when u_max = 0;
 6. N_hat' = D (DFT(G) + T_hat) (2/3 band; T_hat the sponge term, if set),
    N_hat = P N_hat' (Leray projection);
 6b. the total pressure of the step, Pi_hat = -i k.N_hat' / |k|^2, and
    p = Pi - |u|^2/2 are kept for the wing loads (oracle.pressure);
 7. integrating-factor AB2 with variable step (IF-Euler at n = 0):
    u_hat^{n+1} = E_n [u_hat^n + dt_n (1 + xi/2) N_hat^n]
                  - dt_n (xi/2) E_n E_{n-1} N_hat^{n-1},
    E_j = exp(-nu |k|^2 dt_j), xi = dt_n / dt_{n-1};
    the coefficients come from integrating the linear interpolant of
    exp(nu |k|^2 t) N_hat(t) over [t_n, t_{n+1}].

Static penalization (set_static_mask; off by default): a second solid given on
the grid instead of a mesh, independent of z (channel walls, fixed obstacles,
an inflow layer imposing a velocity profile: the channel workload of
Sec. 4.2.1), chi_st(x, y), u_st(x, y).  Reading: the two masks form one mask
function chi = max(chi_wing, chi_st), with the solid velocity of the solid
whose chi is larger (the static one on ties).  The force F is the wing's
(points where the wing's chi is the larger); F_st = (dV/eta) sum w chi
(u - u_st) over the points where the static solid wins, with a caller's
weight w(x, y) (1 on the obstacle whose force is wanted, 0 on walls and the
inflow layer).

Pins (tests/test_oracle_ns.py): 2-D Taylor-Green decays exactly as
exp(-2 nu t) for any dt sequence; 3-D Taylor-Green energy follows
exp(-6 nu t) within the nonlinear-transfer bound; with nu = 0 and chi = 0 the
nonlinear term does no work (Re sum conj(u_hat).N_hat = 0); with a mask it does
exactly -(1/(eta N^3)) sum chi u.(u - u_s); a uniform mask chi = c reduces the
step to a scalar two-term recurrence; the force of a uniform flow through a
static mask equals (dV/eta) U sum chi; adaptive dt matches its closed form.
"""

import numpy as np

from . import dft, spectral, pressure, mask as mask_mod, sponge as sponge_mod


class OracleNS:
    def __init__(self, n, L, nu, eta, tw=0.0, h=0.0, profile=mask_mod.PROFILE_COS):
        self.n = tuple(int(a) for a in n)
        self.L = tuple(float(a) for a in L)
        self.nu = float(nu)
        self.eta = float(eta)
        self.tw = float(tw)
        self.h = float(h)
        self.profile = int(profile)
        nx, ny, nz = self.n
        self.dV = (self.L[0] / nx) * (self.L[1] / ny) * (self.L[2] / nz)
        self.dx_min = min(self.L[0] / nx, self.L[1] / ny, self.L[2] / nz)
        self.k2 = spectral.k_squared(self.n, self.L)
        self.uh = np.zeros((3, nz, ny, nx), dtype=np.complex128)
        self.nh_prev = None
        self.dt_prev = None
        self.t = 0.0
        self.nstep = 0
        self.wing = None
        self.p_last = None  # p = Pi - |u|^2/2 of the last step (oracle.pressure)
        self.sponge = None  # (chi_sp, C_sp)
        self.static = None  # (chi_st [ny][nx], u_st [3][ny][nx], w [ny][nx])

    def set_static_mask(self, chi, us, weight=None):
        """z-independent static penalization chi_st (ny, nx), u_st (3, ny, nx) and
        the weight of its force (ny, nx; None = 0); chi = None removes it."""
        if chi is None:
            self.static = None
            return
        nx, ny, nz = self.n
        chi = np.asarray(chi, dtype=np.float64).reshape(ny, nx)
        us = np.asarray(us, dtype=np.float64).reshape(3, ny, nx)
        w = np.zeros((ny, nx)) if weight is None else np.asarray(weight, dtype=np.float64).reshape(ny, nx)
        self.static = (chi, us, w)

    def combined_mask(self):
        """(chi, u_s, wing force weight, static force weight) on the grid."""
        chi_w, us_w = self.mask()
        if self.static is None:
            return chi_w, us_w, np.ones_like(chi_w), np.zeros_like(chi_w)
        nz = self.n[2]
        chi_s = np.broadcast_to(self.static[0][None], chi_w.shape)
        us_s = np.broadcast_to(self.static[1][:, None], us_w.shape)
        w_s = np.broadcast_to(self.static[2][None], chi_w.shape)
        wing = chi_w > chi_s
        chi = np.where(wing, chi_w, chi_s)
        us = np.where(wing[None], us_w, us_s)
        return chi, us, wing.astype(np.float64), np.where(wing, 0.0, w_s)

    def set_sponge(self, c_sp, gx=None, gy=None, gz=None):
        """Vorticity sponge with chi_sp = max(gx[x], gy[y], gz[z]); c_sp <= 0 removes it."""
        self.sponge = None if c_sp <= 0 else (sponge_mod.sponge_mask(self.n, gx, gy, gz), float(c_sp))

    # -- state ---------------------------------------------------------------
    def set_velocity(self, u):
        """Dealias and project a physical field (3, nz, ny, nx); resets the AB history."""
        uh = dft.forward(np.asarray(u, dtype=np.float64))
        self.uh = spectral.project(spectral.dealias(uh, self.n), self.n, self.L)
        self.nh_prev = None
        self.dt_prev = None
        self.nstep = 0

    def velocity(self):
        return dft.inverse_real(self.uh)

    def set_wing(self, x, v, tri):
        self.wing = (np.asarray(x, dtype=np.float64), np.asarray(v, dtype=np.float64),
                     np.asarray(tri, dtype=np.int64))

    def clear_wing(self):
        self.wing = None

    def mask(self):
        nx, ny, nz = self.n
        if self.wing is None:
            return np.zeros((nz, ny, nx)), np.zeros((3, nz, ny, nx))
        x, v, tri = self.wing
        return mask_mod.build_mask(self.n, self.L, x, v, tri, self.tw, self.h, self.profile)

    def save(self):
        return (self.uh.copy(), None if self.nh_prev is None else self.nh_prev.copy(),
                self.dt_prev, self.t, self.nstep)

    def load(self, s):
        self.uh = s[0].copy()
        self.nh_prev = None if s[1] is None else s[1].copy()
        self.dt_prev, self.t, self.nstep = s[2], s[3], s[4]

    # -- one step ------------------------------------------------------------
    def nonlinear(self, chi, us, fw=None, sw=None):
        """Return (N_hat (projected, dealiased), diagnostics dict) at the current
        state; fw, sw: weights of the wing force and of the static-mask force
        (None: every point for the wing, none for the static mask)."""
        u = dft.inverse_real(self.uh)
        w = dft.inverse_real(spectral.curl(self.uh, self.n, self.L))
        slip = u - us
        g = spectral.cross(u, w) - (chi / self.eta)[None] * slip
        cw = chi if fw is None else chi * fw
        force = (self.dV / self.eta) * np.array([np.sum(cw * slip[c]) for c in range(3)])
        cs = np.zeros_like(chi) if sw is None else chi * sw
        force_st = (self.dV / self.eta) * np.array([np.sum(cs * slip[c]) for c in range(3)])
        speed2 = np.sum(u * u, axis=0)
        diag = {
            "F": force,
            "F_static": force_st,
            "E": 0.5 * self.dV * float(np.sum(speed2)),
            "umax": float(np.sqrt(np.max(speed2))),
        }
        gh = dft.forward(g)
        if self.sponge is not None:
            gh = gh + sponge_mod.sponge_term_hat(self.uh, self.sponge[0], self.sponge[1], self.n, self.L)
        nh = spectral.dealias(gh, self.n)
        # pressure of this step (FSI coupling): Pi from the unprojected term
        self.p_last = pressure.pressure_field(pressure.total_pressure_hat(nh, self.n, self.L), u)
        nh = spectral.project(nh, self.n, self.L)
        return nh, diag

    def adaptive_dt(self, umax, cfl, c_eta, dt_max):
        cfl_term = np.inf if umax == 0.0 else cfl * self.dx_min / umax
        return float(min(cfl_term, c_eta * self.eta, dt_max))

    def step(self, dt=None, cfl=None, c_eta=None, dt_max=None, mask_override=None):
        """Advance one step; returns the diagnostics at t^n plus the dt used."""
        if mask_override is not None:
            chi, us = mask_override
            fw = sw = None
        else:
            chi, us, fw, sw = self.combined_mask()
        nh, diag = self.nonlinear(chi, us, fw, sw)
        if dt is None:
            dt = self.adaptive_dt(diag["umax"], cfl, c_eta, dt_max)
        dt = float(dt)
        en = np.exp(-self.nu * self.k2 * dt)
        if self.nh_prev is None:
            self.uh = en * (self.uh + dt * nh)
        else:
            xi = dt / self.dt_prev
            ep = np.exp(-self.nu * self.k2 * self.dt_prev)
            self.uh = en * (self.uh + dt * (1.0 + 0.5 * xi) * nh) - dt * 0.5 * xi * en * ep * self.nh_prev
        self.nh_prev = nh
        self.dt_prev = dt
        self.t += dt
        self.nstep += 1
        diag["dt"] = dt
        return diag
