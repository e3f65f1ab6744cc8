/*
 * fsi.h - C ABI of the MI355X (gfx950) penalized pseudo-spectral Navier-Stokes step.
 *
 * The library advances the incompressible, volume-penalized Navier-Stokes
 * equations of Sec. 4.1 (penalized NS equations in rotational form,
 * Pi = p + |u|^2/2) on a periodic box with a Fourier pseudo-spectral method:
 *
 *   du/dt = u x omega - grad Pi + nu lap u - (chi/eta)(u - u_s),   div u = 0,
 *
 * with the mask chi rebuilt every step from a triangulated wing mid-surface
 * (Sec. 4.1, Eq. (mask_function) and the distance function that follows it),
 * the solid velocity u_s interpolated barycentrically from the mesh vertex
 * velocities, the Leray projection, an integrating factor for viscosity, a
 * variable-step Adams-Bashforth scheme (Sec. 4.1, staggered scheme paragraph)
 * with adaptive dt, and the penalization force integral used for the lift and
 * drag of Sec. 4.2.2.
 *
 * Conventions
 *  - Every function returns fsi_status (0 = FSI_OK, < 0 = error). Nothing
 *    throws or longjmps across the ABI. After an error, fsi_last_error()
 *    returns a message owned by the context (valid until the next call).
 *  - Argument checks run on the host before any GPU work; a call that fails
 *    them leaves the context state unchanged.
 *  - Grid: nx, ny, nz even, each of the form 2^a 3^b 5^c, 8 <= n <= 2048.
 *    Grid point (i, j, k) sits at (i lx/nx, j ly/ny, k lz/nz).
 *  - Physical host arrays are C-ordered doubles [comp][nz][ny][nx] (x fastest).
 *  - Spectral host arrays use the compact dealiased layout: modes with
 *    3|m_j| < n_j on every axis (2/3 rule), stored [iz][iy][ix] as interleaved
 *    (re, im) doubles, ix = m_x in [0, Kx], iy/iz in natural order
 *    (i <= K -> m = i, i > K -> m = i - (2K + 1)), K_j = max{m : 3m < n_j}.
 *    Coefficients are normalized: f(x) = sum_k fhat_k exp(i k.x) with the
 *    Hermitian partner modes (m_x < 0) implied.
 *  - The caller owns every host array it passes; the library copies in and
 *    out and never keeps a host pointer. The context owns all device memory.
 *  - Work is queued on the stream given in the descriptor (NULL = default
 *    stream). Calls documented as "synchronizes" wait for that stream.
 *  - One context per host thread; calls on one context must not overlap.
 */
#ifndef FSI_H
#define FSI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fsi_ctx fsi_ctx;

typedef enum {
  FSI_OK = 0,
  FSI_EINVAL = -1,      /* invalid argument or descriptor */
  FSI_ENOMEM = -2,      /* device or host allocation failed */
  FSI_EDEVICE = -3,     /* HIP runtime error (no device, launch failure, ...) */
  FSI_EBOUNDS = -4,     /* wing mesh (enlarged by the mask support) leaves the box */
  FSI_ESTATE = -5,      /* call not valid in the current state */
  FSI_ENAN = -6,        /* non-finite value detected on the device */
  FSI_ESTABILITY = -7   /* dt * max(chi) / eta > 1: explicit penalization unstable */
} fsi_status;

/* Mask profiles: 0 = cosine ramp of Eq. (mask_function), support t_w + h;
 * 1 = tanh ramp (1 - tanh((delta - t_w)/h))/2, cut to zero at delta >= t_w + 6h. */
enum { FSI_PROFILE_COS = 0, FSI_PROFILE_TANH = 1 };
/* Arithmetic of the bulk fields: 0 = FP32 fields and transforms with FP64
 * reductions and FP64 dt; 1 = FP64 throughout. */
enum { FSI_PREC_FP32 = 0, FSI_PREC_FP64 = 1 };

typedef struct {
  int32_t nx, ny, nz;   /* grid (see conventions) */
  double lx, ly, lz;    /* periodic box [0, l)^3, > 0 */
  double nu;            /* kinematic viscosity, >= 0 */
  double eta;           /* penalization parameter C_eta of Sec. 4.1, > 0 */
  double tw;            /* wing half-thickness t_w of Eq. (mask_function), >= 0 */
  double h;             /* smoothing half-width h of Eq. (mask_function), > 0 */
  int32_t mask_profile; /* FSI_PROFILE_* */
  int32_t precision;    /* FSI_PREC_* */
  int32_t fsi_pressure; /* 1 = FSI mode: every step keeps its total pressure Pi and the
                           velocity near the wing for fsi_sample_pressure and
                           fsi_get_pressure_loads; 0 = off */
  void* stream;         /* hipStream_t to queue work on; NULL = default stream */
} fsi_desc;

/* Library version as an integer (major * 10000 + minor * 100 + patch). */
int32_t fsi_version(void);

/* Create a context: plans the transforms and allocates every device buffer.
 * On success *out owns the context; on error *out is NULL. */
fsi_status fsi_create(const fsi_desc* desc, fsi_ctx** out);

/* Destroy a context (synchronizes its stream first). NULL is accepted. */
fsi_status fsi_destroy(fsi_ctx* ctx);

/* Message describing the last error on this context ("" if none). Owned by ctx. */
const char* fsi_last_error(const fsi_ctx* ctx);

/* Message of the last fsi_create failure (thread-local, static storage). */
const char* fsi_create_error(void);

/* Band sizes: K[0..2] = (Kx, Ky, Kz); compact spectral component length in complex values. */
fsi_status fsi_band(const fsi_ctx* ctx, int32_t K[3], int64_t* compact_len);

/* Set the velocity from a physical host field u[3][nz][ny][nx]: the field is
 * transformed, truncated to the 2/3 band and Leray-projected (Sec. 4.1,
 * div u = 0). Resets the Adams-Bashforth history and the step counter; the
 * next step is an integrating-factor Euler step. Synchronizes. */
fsi_status fsi_set_velocity(fsi_ctx* ctx, const double* u_host);

/* Same from a device array u[3][nz][ny][nx] of dtype 0 = float, 1 = double
 * (borrowed for the duration of the call only). */
fsi_status fsi_set_velocity_device(fsi_ctx* ctx, const void* u_dev, int32_t dtype);

/* Set the velocity from its compact spectrum uhat[3][compact_len] (interleaved
 * re, im; layout of the conventions above). The field is taken through the
 * physical grid (imaginary parts that a real field cannot carry on the kx = 0
 * plane are dropped) and Leray-projected; resets the Adams-Bashforth history
 * like fsi_set_velocity. Synchronizes. */
fsi_status fsi_set_spectrum(fsi_ctx* ctx, const double* uhat_host);

/* Vorticity sponge (Sec. 4.1, the sponge term of the penalized equations: a
 * vorticity damping against the periodicity of the Fourier discretization).
 * Readings: the term added to du/dt is T = -(1/C_sp) curl((-lap)^-1 (chi_sp
 * omega)), i.e. T_hat = -(1/C_sp) i k x S_hat / |k|^2 with S = chi_sp omega and
 * T_hat(0) = 0 (the sign that damps: chi_sp = 1 gives T = -u/C_sp); the sponge
 * mask is chi_sp(x, y, z) = max(gx[ix], gy[iy], gz[iz]) from per-axis profiles
 * on the grid points (gx: nx values, gy: ny, gz: nz, each >= 0; NULL = 0).
 * T enters the nonlinear term before the 2/3 truncation and the projection.
 * c_sp <= 0 (or all profiles NULL) switches the sponge off (the default).
 * Copied; FSI_EINVAL for a non-finite c_sp or a negative or non-finite
 * profile value.  fsi_step_adjoint reverses the term with the sponge as set
 * when it is called (the sponge of the taped steps must not have changed). */
fsi_status fsi_set_sponge(fsi_ctx* ctx, double c_sp, const double* gx, const double* gy,
                          const double* gz);

/* Physical velocity u[3][nz][ny][nx] of the current state. Synchronizes. */
fsi_status fsi_get_velocity(fsi_ctx* ctx, double* u_host);

/* Compact spectral velocity uhat[3][compact_len] (interleaved re, im). Synchronizes. */
fsi_status fsi_get_spectrum(fsi_ctx* ctx, double* uhat_host);

/* Wing mid-surface mesh (Sec. 4.1): nv vertices x[nv][3], their velocities
 * v[nv][3] in the box frame (Eq. (relative_velocities) already applied), nt
 * triangles tri[nt][3] of 0-based vertex ids. Copied. The mesh enlarged by the
 * mask support radius must lie in [0, l] on every axis (no periodic wrap),
 * else FSI_EBOUNDS. nt = 0 clears the wing. */
fsi_status fsi_set_wing(fsi_ctx* ctx, int32_t nv, const double* x, const double* v,
                        int32_t nt, const int32_t* tri);

/* Static penalization (Sec. 4.1 penalized equations; the channel walls,
 * cylinder and inflow layer of the Sec. 4.2.1 workload): a second solid given
 * on the grid, independent of z: chi[ny][nx] in [0, 1], u_s us[3][ny][nx]
 * (component stride ny*nx), weight[ny][nx] of its force (NULL = 0, e.g. 1 on
 * an obstacle, 0 on walls and inflow layers).  It combines with the wing's mask
 * into one mask function chi = max(chi_wing, chi_static), with the solid
 * velocity of the solid whose chi is larger (the static one on ties).  The
 * step's force F (fsi_get_step_info) is the wing's (points where the wing's chi
 * is larger); fsi_get_static_force returns (dV/eta) sum weight chi (u - u_s)
 * over the points where the static solid wins, at t^n of the last step.
 * chi = NULL removes it.  Arrays are copied; FSI_EINVAL on values out of
 * range.  The reverse step (fsi_step_adjoint) does not include it and returns
 * FSI_ESTATE while it is set. */
fsi_status fsi_set_static_mask(fsi_ctx* ctx, const double* chi, const double* us, const double* weight);
fsi_status fsi_get_static_force(fsi_ctx* ctx, double F[3]);

/* Mask chi[nz][ny][nx] and solid velocity us[3][nz][ny][nx] built from the
 * current wing (zero everywhere without a wing; the static penalization is
 * not included). Synchronizes. */
fsi_status fsi_get_mask(fsi_ctx* ctx, double* chi, double* us);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the mask of
 * fsi_get_mask written into caller-owned device arrays, with no allocation of
 * any kind.  chi: device array [nz][ny][nx], us: device array [3][nz][ny][nx],
 * both of the context's precision (float for FSI_PREC_FP32, double for
 * FSI_PREC_FP64), overwritten everywhere (zero outside the wing's support).
 * The argmin keys of the mask kernels live in a fixed scratch array compiled
 * into the library, one per device, of FSI_NOALLOC_MASK_CELLS sub-box cells
 * (the grid points within the mask support of the wing's bounding box):
 * FSI_EINVAL (state unchanged) if the current wing needs more.  Queued on the
 * context's stream, no host synchronization; the outputs are ready after
 * fsi_synchronize or any synchronizing call.  Every call on a device uses that
 * device's one scratch array: calls that overlap on one device (several
 * contexts or streams of one process) race and must be serialized by the
 * caller.  No memset is queued (fills are kernels), so the call can be
 * captured in a HIP graph. */
#define FSI_NOALLOC_MASK_CELLS (1 << 20)
fsi_status fsi_get_mask_noalloc(fsi_ctx* ctx, void* chi, void* us);

/* One step with a given dt > 0 (queued on the stream, no host sync).
 * FSI_ESTABILITY if a wing is set and dt > eta. */
fsi_status fsi_step(fsi_ctx* ctx, double dt);

/* One step with dt computed on the device from the current state:
 * dt = min(cfl * dx_min / u_max, c_eta * eta, dt_max), the first term taken as
 * +inf when u_max = 0. Requires cfl > 0, 0 < c_eta <= 1, dt_max > 0. */
fsi_status fsi_step_adaptive(fsi_ctx* ctx, double cfl, double c_eta, double dt_max);

/* Diagnostics of the last step, evaluated at the start of that step (t^n):
 * F = force on the body (1/eta) * integral of chi (u - u_s) dV, dt used,
 * E = kinetic energy (1/2) integral |u|^2 dV, umax = max |u|_2 over the grid
 * points, t = time after the step, nstep = steps since fsi_set_velocity.
 * Any pointer may be NULL. Waits until these values of the last step are on the
 * host (after a step, the step's last passes may still run on the stream; every
 * call that reads or replaces device state orders itself after them);
 * FSI_ENAN if a non-finite value was met. */
fsi_status fsi_get_step_info(fsi_ctx* ctx, double F[3], double* dt_used, double* E,
                             double* umax, double* t, int64_t* nstep);

/* ---- pressure loads on the wing (FSI mode, fsi_pressure = 1) ---------------
 * Sec. 4.1, pressure interpolation and staggered coupling paragraphs: the
 * wing is loaded by the fluid pressure p = Pi - |u|^2/2 interpolated onto the
 * mass points with a delta kernel, each triangle giving its three vertices a
 * force along its normal of magnitude pressure x area / 3.
 * Readings: Pi of step n is the pressure of that step's nonlinear term,
 * Pi_hat = -i k.N'_hat / |k|^2 (N' = u x omega - (chi/eta)(u - u_s) before the
 * projection; Pi_hat = 0 at k = 0), so p^n pairs with u^n and the mesh of step
 * n (the structure step n -> n+1 uses p^n).  The delta kernel is the 4-point
 * kernel phi(r) = (3 - 2|r| + sqrt(1 + 4|r| - 4r^2))/8 for |r| < 1,
 * (5 - 2|r| - sqrt(-7 + 12|r| - 4r^2))/8 for 1 <= |r| < 2, per axis in grid
 * units.  A mid-surface carries no net load from a single pressure, so the
 * load uses the jump across the wing: with c_v = (1/3) sum over the triangles
 * T of v of A_T n_T (n_T from the vertex order), n_v = c_v / |c_v| and
 * d = t_w + h, dp_v = p(x_v + d n_v) - p(x_v - d n_v) and load_v = -dp_v c_v.
 * The pressure box holds the 4-point stencils of every point within d of the
 * mesh bounding box (per axis, grid indices floor((lo - d)/dx) - 1 ..
 * floor((hi + d)/dx) + 2); in FSI mode fsi_set_wing returns FSI_EBOUNDS if it
 * leaves the grid (no periodic wrap). */

/* p^n of the last step at n points pts[n][3]; FSI_EBOUNDS if a point's
 * 4 x 4 x 4 stencil leaves the pressure box, FSI_ESTATE if FSI mode is off or
 * no step ran since fsi_set_wing / fsi_load_state.  Synchronizes. */
fsi_status fsi_sample_pressure(fsi_ctx* ctx, int32_t n, const double* pts, double* p_out);
/* Vertex loads load[nv][3] of the current mesh from p^n of the last step (see
 * above) and, if dp is not NULL, the pressure jumps dp[nv].  Same errors as
 * fsi_sample_pressure.  Synchronizes. */
fsi_status fsi_get_pressure_loads(fsi_ctx* ctx, double* loads, double* dp);

/* Sec. 4.1, staggered-scheme paragraph, in the paper's order: after the fluid
 * step u^n -> u^{n+1}, the pressure p^{n+1} of the new velocity (with the mask
 * of the current wing, i.e. still the wing of t^n) replaces the step's p^n, so
 * that fsi_sample_pressure, fsi_get_pressure_loads and fsi_get_pressure_box
 * return it.  One more evaluation of the nonlinear term (mask, inverse
 * transforms, fused x pass, forward transforms, Pi_hat = -i k.N'/|k|^2 with
 * N' = u x omega - (chi/eta)(u - u_s)); u_hat, the Adams-Bashforth history,
 * dt and the step diagnostics are unchanged.  Queued on the stream.
 * FSI_ESTATE if FSI mode is off or no wing is set. */
fsi_status fsi_eval_pressure(fsi_ctx* ctx);

/* The pressure box of the current mesh (box0[3]: grid index of its first
 * cell, boxn[3]: cells per axis) and, if p is not NULL, p = Pi - |u|^2/2 of
 * the last step at its cells, p[boxn[2]][boxn[1]][boxn[0]] (the data the host
 * needs to transpose the loads, fsi_loads_adjoint).  FSI_ESTATE without FSI
 * mode or wing, or (p != NULL) without a step since fsi_set_wing.
 * Synchronizes. */
fsi_status fsi_get_pressure_box(fsi_ctx* ctx, int32_t* box0, int32_t* boxn, double* p);

/* Stand-alone transforms on the context's grid, for testing the FFT passes.
 * r2c: physical f[nz][ny][nx] -> normalized compact band fhat (interleaved).
 * c2r: compact band fhat -> physical f (real part of the inverse transform,
 * Hermitian partners implied). Both synchronize. They use internal buffers and
 * must not be interleaved with a step. */
fsi_status fsi_fft_r2c(fsi_ctx* ctx, const double* f, double* fhat);
fsi_status fsi_fft_c2r(fsi_ctx* ctx, const double* fhat, double* f);

/* Save / restore the time-stepping state (velocity, previous nonlinear term,
 * previous dt, time, step counter) in one of 64 slots held in device memory.
 * Loading an empty slot is FSI_ESTATE. */
fsi_status fsi_save_state(fsi_ctx* ctx, int32_t slot);
fsi_status fsi_load_state(fsi_ctx* ctx, int32_t slot);

/* Compact spectrum of the previous nonlinear term N_hat^{n-1}[3][compact_len]
 * (the Adams-Bashforth history; zero right after fsi_set_velocity). Synchronizes. */
fsi_status fsi_get_nonlinear(fsi_ctx* ctx, double* nhat_host);

/* ---- adjoint of the step (dt held fixed) --------------------------------
 * The step maps (u_hat^n, N_hat^{n-1}) to (u_hat^{n+1}, N_hat^n) and yields the
 * force F^n; its transpose under the inner product Re sum conj(a).b over the
 * stored compact spectrum is applied by fsi_step_adjoint to the context's
 * cotangent state (lambda_u, lambda_N), both [3][compact_len] complex.
 * Transposes used: C2R^T = N^3 m_k R2C (m_k = 1 at kx = 0, else 2),
 * R2C^T = N^-3 C2R(./m_k), (i k x)^T = i k x, (u x omega)^T, the projection
 * and integrating factors (real symmetric per mode). */

/* Set the cotangent state (either pointer may be NULL = zero). Synchronizes. */
fsi_status fsi_adjoint_set(fsi_ctx* ctx, const double* lam_uhat, const double* lam_nprev);
/* Read the cotangent state (either pointer may be NULL). Synchronizes. */
fsi_status fsi_adjoint_get(fsi_ctx* ctx, double* lam_uhat, double* lam_nprev);
/* Zero the cotangent state (the start of a reverse sweep). Synchronizes. */
fsi_status fsi_adjoint_reset(fsi_ctx* ctx);

/* Forward step with its tape: saves the velocity spectrum u_hat^n at the start
 * of the step in tape_slot (all that fsi_step_adjoint needs: it re-derives u and
 * omega from it) and takes the step (as fsi_step), so that
 * fsi_step_adjoint(tape_slot, ...) can reverse it later.  A tape slot is not a
 * full state: fsi_load_state refuses it (FSI_ESTATE) until fsi_save_state
 * overwrites it.  Errors as fsi_save_state and fsi_step. */
fsi_status fsi_step_record(fsi_ctx* ctx, double dt, int32_t tape_slot);

/* Reverse one step. tape_slot holds the state saved (fsi_step_record or
 * fsi_save_state) at the start of the step; the wing of that step must be set (fsi_set_wing); dt is
 * the step's dt, dt_prev the one before (ignored when first = 1, i.e. the step
 * was an integrating-factor Euler step). dJdF[3] is the derivative of the
 * objective with respect to the force F of that step. On return the cotangent
 * state is (dJ/du_hat^n, dJ/dN_hat^{n-1}) and, if non-NULL, dJdx[nv][3] and
 * dJdv[nv][3] hold dJ/d(vertex positions, velocities) of that step's mesh
 * through the mask and the solid velocity.  With the vorticity sponge on
 * (fsi_set_sponge) its term is reversed too. Synchronizes. */
fsi_status fsi_step_adjoint(fsi_ctx* ctx, int32_t tape_slot, double dt, double dt_prev, int32_t first,
                            const double dJdF[3], double* dJdx, double* dJdv);

/* Pressure seed of the next fsi_step_adjoint (FSI coupling): the cotangent
 * lam_p of p = Pi - |u|^2/2 of that step at the cells of the current pressure
 * box (box0/boxn must be those of fsi_get_pressure_box for the current mesh,
 * else FSI_EINVAL; lam_p = NULL clears it).  The reverse step then also
 * carries lam_p back to u_hat^n and to the mesh through Pi_hat =
 * -i k.N'_hat/|k|^2 and through -|u|^2/2.  A new fsi_set_wing clears it.
 * Synchronizes. */
fsi_status fsi_adjoint_set_pressure_seed(fsi_ctx* ctx, const int32_t* box0, const int32_t* boxn,
                                         const double* lam_p);

/* Derivatives of fsi_plate_pose's x and v with respect to the pitch alpha
 * (host, FP64): dxda[nv][3], dvda[nv][3]. */
fsi_status fsi_plate_pose_dalpha(int32_t nv, const double* s, const double* c, double t, double alpha,
                                 double omega, double t_ramp, int32_t law, double* dxda, double* dvda);

/* Wing frame of the revolving plate of fsi_plate_pose at time t (host, FP64):
 * frame[3][3] row-major with the span, chord and normal directions as columns,
 * Rz(phi(t)) applied to (1, 0, 0), (0, cos alpha, sin alpha) and
 * (0, -sin alpha, cos alpha); phi_out[2] (may be NULL) = (phi, dphi/dt).  The
 * frame in which the mass-spring wing measures its bending angles. */
fsi_status fsi_plate_frame(double t, double alpha, double omega, double t_ramp, int32_t law, double* frame,
                           double* phi_out);

/* d frame / d alpha of fsi_plate_frame (host, FP64): Rz(phi(t)) applied to
 * (0, 0, 0), (0, -sin alpha, cos alpha), (0, -cos alpha, -sin alpha). */
fsi_status fsi_plate_frame_dalpha(double t, double alpha, double omega, double t_ramp, int32_t law, double* dframe);

/* Wait for all queued work of the context. */
fsi_status fsi_synchronize(fsi_ctx* ctx);

/* Per-pass timing with HIP events on the streams of the step (off by default).
 * on = 0: off; on = 1 (any value without FSI_TIME_PASSES): every pass;
 * on = FSI_TIME_PASSES | mask: only the passes whose bit (1 << pass index) is
 * set (each recorded event orders its stream, so timing fewer passes
 * disturbs the step less).  fsi_get_pass_times synchronizes, writes the summed
 * milliseconds of each of the FSI_NPASS passes recorded since timing was
 * enabled or last read (0 for passes not timed), and the number of steps they
 * cover, then resets the sums. Pass order: mask, z-inverse+curl, y-inverse,
 * x-fused, reduce, y-forward, z-forward+update.  FSI_EINVAL if on < 0. */
enum { FSI_NPASS = 7 };
#define FSI_TIME_PASSES 0x100
fsi_status fsi_set_timing(fsi_ctx* ctx, int32_t on);
fsi_status fsi_get_pass_times(fsi_ctx* ctx, double ms[FSI_NPASS], int32_t* nsteps);

/* Testing aid for the memory layout, not part of the method: writes
 * (value, value) into the padding columns of every row of the context's
 * spectral buffers (the columns k_x > Kx up to the 128-byte row pitch, in the
 * state, its nonlinear term, the work fields, the pressure and sponge
 * spectra), then synchronizes.  No result of a later call may depend on these
 * columns: a NaN written there must leave every step bit for bit unchanged.
 * FSI_EINVAL for a bad context. */
fsi_status fsi_debug_poison_padding(fsi_ctx* ctx, double value);

/* Rigid revolving-plate pose (Sec. 4.2.2, Eq. (revolving_angle) and
 * Eq. (relative_velocities) without deformation). Host-only, FP64.
 * Inputs: nv vertices with span coordinate s[i] (from the rotation axis) and
 * chord coordinate c[i] (from the mid-chord line), pitch alpha, rotation rate
 * omega, ramp time t_ramp, law (0 = Omega(t) = omega (1 - cos(pi t/t_ramp))/2
 * until t_ramp then omega; 1 = phi(t) = omega (tau e^{-t/tau} + t - tau), tau =
 * t_ramp), axis point axis[3]. At phi = 0 a vertex sits at axis + (s, c cos
 * alpha, c sin alpha). Outputs x[nv][3], v[nv][3] (v = dphi/dt e_z x (x - axis))
 * and phi_out[0..1] = (phi, dphi/dt) if non-NULL. */
fsi_status fsi_plate_pose(int32_t nv, const double* s, const double* c, double t, double alpha,
                          double omega, double t_ramp, int32_t law, const double axis[3],
                          double* x, double* v, double* phi_out);

#ifdef __cplusplus
}
#endif

#endif /* FSI_H */
