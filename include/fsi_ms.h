/* fsi_ms.h - native FP64 mass-spring wing solver (host code, part of libfsi).
 *
 * The wing model of Sec. 2 ("Flexible wing"): mass points obeying Newton's
 * second law as a first-order system in the phase vector q = [x, v]
 * (Sec. 2.1), linear extension springs (Sec. 2.2, Eq. extension_spring) and
 * bending springs on the two projected bending angles of
 * Eq. two_bending_angles, measured in the wing frame, with the restoring moment
 * -k^b (theta - theta_0) of Eq. bending_spring_moment.  The force of a bending
 * spring is the exact negative gradient of its energy
 * k^b/2 [(theta^y - theta^y_0)^2 + (theta^z - theta^z_0)^2].  Time stepping is
 * the variable-step second-order BDF of Eq. discretized_ODEs, solved for
 * q^{n+1} by Newton-Raphson from q^n (Sec. 2.1); the first step after
 * fsi_ms_set_state has no q^{n-1} and is implicit Euler (xi = 0).
 *
 * Conventions
 *  - Vertices are indexed 0..nv-1; position and velocity arrays are
 *    [nv][3] doubles, row-major.  "frame" is a 3x3 row-major rotation whose
 *    COLUMNS are the wing axes (x = span, y, z) in the inertial frame.
 *  - The caller owns every array; the solver copies what it keeps.
 *  - Every function returns an fsi_status; on error the solver state is
 *    unchanged and fsi_ms_last_error() describes the failure.
 *  - A solver object is not thread safe; use one per thread.
 */
#ifndef FSI_MS_H
#define FSI_MS_H

#include "fsi.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fsi_ms fsi_ms;

/* New network of nv mass points with masses mass[nv] (> 0), at rest at the
 * origin.  FSI_EINVAL for nv < 1 or a non-positive mass. */
fsi_status fsi_ms_create(int32_t nv, const double* mass, fsi_ms** out);
fsi_status fsi_ms_destroy(fsi_ms* ms);
/* Description of the last failure of this object (owned by it). */
const char* fsi_ms_last_error(const fsi_ms* ms);

/* Append n extension springs: ij[n][2] vertex pairs, stiffness k[n] >= 0 and
 * rest length l0[n] > 0 (Eq. extension_spring).  Returns the index of the first
 * appended spring in *first (may be NULL). */
fsi_status fsi_ms_add_extension(fsi_ms* ms, int32_t n, const int32_t* ij, const double* k, const double* l0,
                                int32_t* first);
/* Append n bending springs on vertex triples ijk[n][3] (segments i->j and
 * j->k), stiffness kb[n] >= 0 and rest angles theta0[n][2].  axis[n] (NULL =
 * all 0) is the wing axis the spring lies along: Eq. two_bending_angles
 * projects on the wing planes (x, y) and (x, z), which suits springs along x
 * (axis 0); a spring along wing axis a uses the planes (a, a+1) and (a, a+2),
 * cyclically (a reading: the paper's veins all run spanwise).  *first as above. */
fsi_status fsi_ms_add_bending(fsi_ms* ms, int32_t n, const int32_t* ijk, const double* kb, const double* theta0,
                              const int32_t* axis, int32_t* first);
/* Replace the stiffness of all extension springs (k[n_ext]) or bending springs
 * (kb[n_bend]); the topology is unchanged. */
fsi_status fsi_ms_set_extension_k(fsi_ms* ms, const double* k);
fsi_status fsi_ms_set_bending_k(fsi_ms* ms, const double* kb);
/* Mark n vertices idx[n] as clamped: their motion is prescribed at every step. */
fsi_status fsi_ms_set_clamped(fsi_ms* ms, int32_t n, const int32_t* idx);

/* Rest lengths of all extension springs and rest angles of all bending springs
 * (in `frame`, NULL = identity) taken from the current positions. */
fsi_status fsi_ms_set_rest(fsi_ms* ms, const double* frame);
/* k^b of Eq. EI_k_relation for a vein of length l_b (> 0) carrying n (>= 1)
 * bending springs, from its flexural rigidity EI (>= 0). */
fsi_status fsi_ms_bending_stiffness(double EI, double l_b, int32_t n, double* kb);
/* Lumped masses mass[nv]: areal density (> 0) times one third of the area of
 * each triangle tri[nt][3] of positions x[nv][3], summed per vertex. */
fsi_status fsi_ms_lumped_masses(int32_t nv, const double* x, int32_t nt, const int32_t* tri, double density,
                                double* mass);

/* Projected bending angles theta[n_bend][2] of positions x[nv][3] in the given
 * frame (Eq. two_bending_angles). */
fsi_status fsi_ms_bending_angles(const fsi_ms* ms, const double* x, const double* frame, double* theta);
/* Internal (spring) forces f[nv][3] = -grad E at positions x, and the elastic
 * energy in *energy (may be NULL). */
fsi_status fsi_ms_forces(const fsi_ms* ms, const double* x, const double* frame, double* f, double* energy);

/* Set positions and velocities (x, v [nv][3]); clears the step history so the
 * next step is implicit Euler. */
fsi_status fsi_ms_set_state(fsi_ms* ms, const double* x, const double* v);
fsi_status fsi_ms_get_state(const fsi_ms* ms, double* x, double* v);

/* Advance by dt (> 0): BDF2 with xi = dt / dt_prev (implicit Euler on the
 * first step), external forces f_ext[nv][3] held over the step (NULL = none),
 * bending angles in `frame` at t^{n+1}, clamped vertices set to
 * x_clamp/v_clamp[n_clamped][3] (in the order given to fsi_ms_set_clamped;
 * NULL = keep their current position with zero velocity).  Newton stops when
 * ||dq|| <= tol max(1, ||q||) (tol <= 0 selects 1e-6, Sec. 2.1) and returns
 * FSI_ESTATE, leaving the state unchanged, if max_iter iterations do not
 * converge or the Newton matrix is singular.  *iters (may be NULL) receives the
 * iteration count. */
fsi_status fsi_ms_step(fsi_ms* ms, double dt, const double* frame, const double* f_ext, const double* x_clamp,
                       const double* v_clamp, double tol, int32_t max_iter, int32_t* iters);

/* Restore the BDF2 history (positions and velocities at t^{n-1} and the
 * previous dt) for recomputing a step from a stored state; x_prev = NULL
 * clears it (the next step is implicit Euler). */
fsi_status fsi_ms_set_history(fsi_ms* ms, const double* x_prev, const double* v_prev, double dt_prev);

/* Transpose of one fsi_ms_step (the map (q^n, q^{n-1}, f_ext, stiffnesses,
 * clamp values, frame) -> q^{n+1}, at its converged solution).  Given the
 * cotangents lam_x, lam_v [nv][3] of x^{n+1}, v^{n+1} (those of clamped
 * vertices included), it solves the transposed Newton system, whose matrix
 * M + (gamma dt)^2 H(x^{n+1}) is the symmetric Newton matrix of the step, and
 * ADDS the cotangents of: x^n, v^n (lam_xn, lam_vn), x^{n-1}, v^{n-1} (lam_xp,
 * lam_vp; nothing is added when dt_prev <= 0, the implicit-Euler step),
 * f_ext (lam_load [nv][3]), each extension and bending stiffness
 * (lam_kext[n_ext], lam_kb[n_bend]), the prescribed clamp positions and
 * velocities (lam_clamp_x/v [n_clamped][3]), and a frame moving along dframe
 * (3x3, d frame / d parameter; lam_dframe scalar).  Any output may be NULL.
 * x_new = x^{n+1}; dt, dt_prev and frame as in the forward step.  The solver's
 * state is not used or changed (only its masses, springs and clamps). */
fsi_status fsi_ms_step_adjoint(fsi_ms* ms, double dt, double dt_prev, const double* frame, const double* dframe,
                               const double* x_new, const double* lam_x, const double* lam_v, double* lam_xn,
                               double* lam_vn, double* lam_xp, double* lam_vp, double* lam_load, double* lam_kext,
                               double* lam_kb, double* lam_clamp_x, double* lam_clamp_v, double* lam_dframe);

/* ---- wing pressure loads on the host (FSI coupling, Sec. 4.1) -------------
 * The loads of fsi_get_pressure_loads computed from a pressure box held on
 * the host: box0[3] (grid index of its first cell), boxn[3] (cells per axis,
 * >= 4), pbox[boxn[2]][boxn[1]][boxn[0]] = p = Pi - |u|^2/2 at the cells (as
 * returned by fsi_get_pressure_box), grid spacing dx[3]; d = t_w + h.  Mesh as
 * in fsi_set_wing.  FSI_EBOUNDS if a sample stencil leaves the box.  */
fsi_status fsi_loads_from_box(int32_t nv, const double* x, int32_t nt, const int32_t* tri, double d, const double* dx,
                              const int32_t* box0, const int32_t* boxn, const double* pbox, double* loads,
                              double* dp);
/* Transpose of fsi_loads_from_box at (x, pbox): given the load cotangents
 * lam_load[nv][3], ADDS the cotangents of the vertex positions (lam_x[nv][3],
 * through the sample points, normals and areas) and of the box values
 * (lam_pbox, box-shaped).  Either output may be NULL. */
fsi_status fsi_loads_adjoint(int32_t nv, const double* x, int32_t nt, const int32_t* tri, double d, const double* dx,
                             const int32_t* box0, const int32_t* boxn, const double* pbox, const double* lam_load,
                             double* lam_x, double* lam_pbox);

/* Static equilibrium F_int(x) + f_ext = 0 from the current positions, clamped
 * vertices fixed, the load applied in load_steps equal increments with Newton
 * at each; the velocities are set to zero and the history cleared. */
fsi_status fsi_ms_static(fsi_ms* ms, const double* frame, const double* f_ext, int32_t load_steps, double tol,
                         int32_t max_iter);

#ifdef __cplusplus
}
#endif

#endif /* FSI_MS_H */
