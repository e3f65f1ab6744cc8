// api.cpp - the extern "C" boundary declared in include/fsi.h.
#include <math.h>
#include <string.h>

#include <cmath>
#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/fsi.h"
#include "engine.h"

#include <mutex>

struct fsi_ctx {
  fsi::EngineBase* eng = nullptr;
  int device = 0;  // the device current at fsi_create
};

namespace {
thread_local std::string g_create_error;

fsi_status guard(fsi_ctx* c) { return (c && c->eng) ? FSI_OK : FSI_EINVAL; }

// Fixed key scratch of fsi_get_mask_noalloc: two u64 keys per mask sub-box cell,
// FSI_NOALLOC_MASK_CELLS cells (16 MiB per device, held until the process ends).
// Every call on a device shares that device's copy.
static __device__ __align__(256) unsigned long long scratch[2 * FSI_NOALLOC_MASK_CELLS];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (the host-side name is only a stand-in);
// resolved once per device at fsi_create, with that device current.
fsi_status resolve_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return FSI_EDEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return FSI_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FSI_EDEVICE;
  g_scratch_ptr[dev] = static_cast<unsigned long long*>(p);
  return FSI_OK;
}

unsigned long long* scratch_of(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[dev];
}
}  // namespace

extern "C" {

int32_t fsi_version(void) { return 100; }

const char* fsi_create_error(void) { return g_create_error.c_str(); }

fsi_status fsi_create(const fsi_desc* desc, fsi_ctx** out) {
  if (!out) return FSI_EINVAL;
  *out = nullptr;
  if (!desc) {
    g_create_error = "descriptor is NULL";
    return FSI_EINVAL;
  }
  const std::string bad = fsi::check_desc(*desc);
  if (!bad.empty()) {
    g_create_error = bad;
    return FSI_EINVAL;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    g_create_error = "no HIP device available";
    return FSI_EDEVICE;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || resolve_scratch(dev) != FSI_OK) {
    g_create_error = "cannot resolve the device address of the fixed mask scratch";
    return FSI_EDEVICE;
  }
  fsi_ctx* c = new (std::nothrow) fsi_ctx();
  if (!c) return FSI_ENOMEM;
  c->device = dev;
  c->eng = desc->precision == FSI_PREC_FP64 ? fsi::make_engine_f64() : fsi::make_engine_f32();
  const fsi_status st = c->eng->init(*desc);
  if (st != FSI_OK) {
    g_create_error = c->eng->err;
    delete c->eng;
    delete c;
    return st;
  }
  g_create_error.clear();
  *out = c;
  return FSI_OK;
}

fsi_status fsi_destroy(fsi_ctx* ctx) {
  if (!ctx) return FSI_OK;
  delete ctx->eng;
  delete ctx;
  return FSI_OK;
}

const char* fsi_last_error(const fsi_ctx* ctx) {
  if (!ctx || !ctx->eng) return "invalid context";
  return ctx->eng->err.c_str();
}

fsi_status fsi_band(const fsi_ctx* ctx, int32_t K[3], int64_t* compact_len) {
  if (!ctx || !ctx->eng || !K || !compact_len) return FSI_EINVAL;
  int k[3];
  long long cl;
  ctx->eng->band(k, &cl);
  K[0] = k[0];
  K[1] = k[1];
  K[2] = k[2];
  *compact_len = cl;
  return FSI_OK;
}

fsi_status fsi_set_velocity(fsi_ctx* ctx, const double* u_host) {
  if (guard(ctx) != FSI_OK || !u_host) return FSI_EINVAL;
  return ctx->eng->set_velocity_host(u_host);
}

fsi_status fsi_set_velocity_device(fsi_ctx* ctx, const void* u_dev, int32_t dtype) {
  if (guard(ctx) != FSI_OK || !u_dev) return FSI_EINVAL;
  return ctx->eng->set_velocity_device(u_dev, dtype);
}

fsi_status fsi_set_spectrum(fsi_ctx* ctx, const double* uhat_host) {
  if (guard(ctx) != FSI_OK || !uhat_host) return FSI_EINVAL;
  return ctx->eng->set_spectrum(uhat_host);
}

fsi_status fsi_get_velocity(fsi_ctx* ctx, double* u_host) {
  if (guard(ctx) != FSI_OK || !u_host) return FSI_EINVAL;
  return ctx->eng->get_velocity(u_host);
}

fsi_status fsi_get_spectrum(fsi_ctx* ctx, double* uhat_host) {
  if (guard(ctx) != FSI_OK || !uhat_host) return FSI_EINVAL;
  return ctx->eng->get_spectrum(uhat_host);
}

fsi_status fsi_get_nonlinear(fsi_ctx* ctx, double* nhat_host) {
  if (guard(ctx) != FSI_OK || !nhat_host) return FSI_EINVAL;
  return ctx->eng->get_nonlinear(nhat_host);
}

fsi_status fsi_set_wing(fsi_ctx* ctx, int32_t nv, const double* x, const double* v, int32_t nt,
                        const int32_t* tri) {
  if (guard(ctx) != FSI_OK) return FSI_EINVAL;
  return ctx->eng->set_wing(nv, x, v, nt, tri);
}

fsi_status fsi_set_sponge(fsi_ctx* ctx, double c_sp, const double* gx, const double* gy, const double* gz) {
  if (guard(ctx) != FSI_OK) return FSI_EINVAL;
  return ctx->eng->set_sponge(c_sp, gx, gy, gz);
}

fsi_status fsi_set_static_mask(fsi_ctx* ctx, const double* chi, const double* us, const double* weight) {
  if (guard(ctx) != FSI_OK) return FSI_EINVAL;
  return ctx->eng->set_static_mask(chi, us, weight);
}

fsi_status fsi_get_static_force(fsi_ctx* ctx, double F[3]) {
  if (guard(ctx) != FSI_OK || !F) return FSI_EINVAL;
  return ctx->eng->static_force(F);
}

fsi_status fsi_get_mask(fsi_ctx* ctx, double* chi, double* us) {
  if (guard(ctx) != FSI_OK || !chi || !us) return FSI_EINVAL;
  return ctx->eng->get_mask(chi, us);
}

fsi_status fsi_get_mask_noalloc(fsi_ctx* ctx, void* chi, void* us) {
  if (guard(ctx) != FSI_OK || !chi || !us) return FSI_EINVAL;
  unsigned long long* p = scratch_of(ctx->device);
  if (!p) {
    ctx->eng->err = "fixed mask scratch not resolved for this device";
    return FSI_EDEVICE;
  }
  return ctx->eng->get_mask_grid(chi, us, p, FSI_NOALLOC_MASK_CELLS);
}

fsi_status fsi_step(fsi_ctx* ctx, double dt) {
  if (guard(ctx) != FSI_OK) return FSI_EINVAL;
  return ctx->eng->step(false, dt, 0.0, 0.0, 0.0);
}

fsi_status fsi_step_adaptive(fsi_ctx* ctx, double cfl, double c_eta, double dt_max) {
  if (guard(ctx) != FSI_OK) return FSI_EINVAL;
  return ctx->eng->step(true, 0.0, cfl, c_eta, dt_max);
}

fsi_status fsi_get_step_info(fsi_ctx* ctx, double F[3], double* dt_used, double* E, double* umax, double* t,
                             int64_t* nstep) {
  if (guard(ctx) != FSI_OK) return FSI_EINVAL;
  long long ns = 0;
  const fsi_status st = ctx->eng->step_info(F, dt_used, E, umax, t, &ns);
  if (nstep) *nstep = ns;
  return st;
}

fsi_status fsi_sample_pressure(fsi_ctx* ctx, int32_t n, const double* pts, double* p_out) {
  if (guard(ctx) != FSI_OK) return FSI_EINVAL;
  return ctx->eng->sample_pressure(n, pts, p_out);
}

fsi_status fsi_get_pressure_loads(fsi_ctx* ctx, double* loads, double* dp) {
  if (guard(ctx) != FSI_OK) return FSI_EINVAL;
  return ctx->eng->pressure_loads(loads, dp);
}

fsi_status fsi_eval_pressure(fsi_ctx* ctx) {
  if (guard(ctx) != FSI_OK) return FSI_EINVAL;
  return ctx->eng->eval_pressure();
}

fsi_status fsi_get_pressure_box(fsi_ctx* ctx, int32_t* box0, int32_t* boxn, double* p) {
  if (guard(ctx) != FSI_OK || !box0 || !boxn) return FSI_EINVAL;
  int b0[3], bn[3];
  const fsi_status st = ctx->eng->pressure_box(b0, bn, p);
  for (int q = 0; q < 3; ++q) {
    box0[q] = b0[q];
    boxn[q] = bn[q];
  }
  return st;
}

fsi_status fsi_adjoint_set_pressure_seed(fsi_ctx* ctx, const int32_t* box0, const int32_t* boxn, const double* lam_p) {
  if (guard(ctx) != FSI_OK || !box0 || !boxn) return FSI_EINVAL;
  const int b0[3] = {box0[0], box0[1], box0[2]}, bn[3] = {boxn[0], boxn[1], boxn[2]};
  return ctx->eng->set_pressure_seed(b0, bn, lam_p);
}

fsi_status fsi_fft_r2c(fsi_ctx* ctx, const double* f, double* fhat) {
  if (guard(ctx) != FSI_OK || !f || !fhat) return FSI_EINVAL;
  return ctx->eng->fft_r2c(f, fhat);
}

fsi_status fsi_fft_c2r(fsi_ctx* ctx, const double* fhat, double* f) {
  if (guard(ctx) != FSI_OK || !f || !fhat) return FSI_EINVAL;
  return ctx->eng->fft_c2r(fhat, f);
}

fsi_status fsi_save_state(fsi_ctx* ctx, int32_t slot) {
  if (guard(ctx) != FSI_OK) return FSI_EINVAL;
  return ctx->eng->save_state(slot);
}

fsi_status fsi_load_state(fsi_ctx* ctx, int32_t slot) {
  if (guard(ctx) != FSI_OK) return FSI_EINVAL;
  return ctx->eng->load_state(slot);
}

fsi_status fsi_adjoint_set(fsi_ctx* ctx, const double* lam_uhat, const double* lam_nprev) {
  if (guard(ctx) != FSI_OK) return FSI_EINVAL;
  return ctx->eng->adjoint_set(lam_uhat, lam_nprev);
}

fsi_status fsi_adjoint_reset(fsi_ctx* ctx) {
  if (guard(ctx) != FSI_OK) return FSI_EINVAL;
  return ctx->eng->adjoint_set(nullptr, nullptr);
}

fsi_status fsi_step_record(fsi_ctx* ctx, double dt, int32_t tape_slot) {
  if (guard(ctx) != FSI_OK) return FSI_EINVAL;
  return ctx->eng->step_record(dt, tape_slot);
}

fsi_status fsi_adjoint_get(fsi_ctx* ctx, double* lam_uhat, double* lam_nprev) {
  if (guard(ctx) != FSI_OK) return FSI_EINVAL;
  return ctx->eng->adjoint_get(lam_uhat, lam_nprev);
}

fsi_status fsi_step_adjoint(fsi_ctx* ctx, int32_t tape_slot, double dt, double dt_prev, int32_t first,
                            const double dJdF[3], double* dJdx, double* dJdv) {
  if (guard(ctx) != FSI_OK || !dJdF) return FSI_EINVAL;
  return ctx->eng->step_adjoint(tape_slot, dt, dt_prev, first, dJdF, dJdx, dJdv);
}

fsi_status fsi_synchronize(fsi_ctx* ctx) {
  if (guard(ctx) != FSI_OK) return FSI_EINVAL;
  return ctx->eng->synchronize();
}

fsi_status fsi_set_timing(fsi_ctx* ctx, int32_t on) {
  if (guard(ctx) != FSI_OK) return FSI_EINVAL;
  if (on < 0) return FSI_EINVAL;
  const unsigned all = (1u << FSI_NPASS) - 1;
  const unsigned u = (unsigned)on;
  return ctx->eng->set_timing(u == 0 ? 0u : (u & FSI_TIME_PASSES) ? (u & all) : all);
}

fsi_status fsi_debug_poison_padding(fsi_ctx* ctx, double value) {
  if (guard(ctx) != FSI_OK) return FSI_EINVAL;
  return ctx->eng->poison_padding(value);
}

fsi_status fsi_get_pass_times(fsi_ctx* ctx, double ms[FSI_NPASS], int32_t* nsteps) {
  if (guard(ctx) != FSI_OK || !ms) return FSI_EINVAL;
  int n = 0;
  const fsi_status st = ctx->eng->pass_times(ms, &n);
  if (nsteps) *nsteps = n;
  return st;
}

// Rigid revolving plate (Sec. 4.2.2): rotation angle from the ramp law or
// Eq. (revolving_angle); frame velocity Omega e_z x r (Eq. (relative_velocities)
// with a rigid wing).
fsi_status fsi_plate_pose(int32_t nv, const double* s, const double* c, double t, double alpha, double omega,
                          double t_ramp, int32_t law, const double axis[3], double* x, double* v,
                          double* phi_out) {
  if (nv < 0 || (nv > 0 && (!s || !c || !x || !v)) || !axis) return FSI_EINVAL;
  if (!std::isfinite(t) || !std::isfinite(alpha) || !std::isfinite(omega) || !std::isfinite(t_ramp))
    return FSI_EINVAL;
  if (law != 0 && law != 1) return FSI_EINVAL;
  if (law == 1 && !(t_ramp > 0)) return FSI_EINVAL;
  double phi, rate;
  if (law == 0) {
    const double tr = t_ramp > 0 ? t_ramp : 0.0;
    if (tr == 0.0 || t >= tr) {
      phi = 0.5 * omega * tr + omega * (t - tr);
      rate = omega;
    } else {
      const double a = M_PI * t / tr;
      rate = 0.5 * omega * (1.0 - cos(a));
      phi = 0.5 * omega * (t - (tr / M_PI) * sin(a));
    }
  } else {
    const double e = exp(-t / t_ramp);
    phi = omega * (t_ramp * e + t - t_ramp);
    rate = omega * (1.0 - e);
  }
  const double cp = cos(phi), sp = sin(phi), ca = cos(alpha), sa = sin(alpha);
  for (int32_t i = 0; i < nv; ++i) {
    const double lx = s[i], ly = c[i] * ca, lz = c[i] * sa;
    const double rx = cp * lx - sp * ly, ry = sp * lx + cp * ly;
    x[3 * i] = axis[0] + rx;
    x[3 * i + 1] = axis[1] + ry;
    x[3 * i + 2] = axis[2] + lz;
    v[3 * i] = -rate * ry;
    v[3 * i + 1] = rate * rx;
    v[3 * i + 2] = 0.0;
  }
  if (phi_out) {
    phi_out[0] = phi;
    phi_out[1] = rate;
  }
  return FSI_OK;
}

fsi_status fsi_plate_frame(double t, double alpha, double omega, double t_ramp, int32_t law, double* frame,
                           double* phi_out) {
  if (!frame) return FSI_EINVAL;
  // the pose of a vertex at span 1, chord 0 gives phi and its rate
  const double one = 1.0, zero = 0.0, axis0[3] = {0.0, 0.0, 0.0};
  double xs[3], vs[3], ph[2];
  const fsi_status st = fsi_plate_pose(1, &one, &zero, t, alpha, omega, t_ramp, law, axis0, xs, vs, ph);
  if (st != FSI_OK) return st;
  const double cp = cos(ph[0]), sp = sin(ph[0]), ca = cos(alpha), sa = sin(alpha);
  const double cols[3][3] = {{cp, sp, 0.0}, {-sp * ca, cp * ca, sa}, {sp * sa, -cp * sa, ca}};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) frame[3 * r + c] = cols[c][r];
  if (phi_out) {
    phi_out[0] = ph[0];
    phi_out[1] = ph[1];
  }
  return FSI_OK;
}

fsi_status fsi_plate_frame_dalpha(double t, double alpha, double omega, double t_ramp, int32_t law, double* dframe) {
  if (!dframe) return FSI_EINVAL;
  double fr[9], ph[2];
  const fsi_status st = fsi_plate_frame(t, alpha, omega, t_ramp, law, fr, ph);
  if (st != FSI_OK) return st;
  const double cp = cos(ph[0]), sp = sin(ph[0]), ca = cos(alpha), sa = sin(alpha);
  const double cols[3][3] = {{0.0, 0.0, 0.0}, {sp * sa, -cp * sa, ca}, {sp * ca, -cp * ca, -sa}};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) dframe[3 * r + c] = cols[c][r];
  return FSI_OK;
}

// Derivative of the rigid plate pose with respect to the pitch alpha: the pose
// x = axis + Rz(phi) (s, c cos alpha, c sin alpha) gives dx/dalpha = Rz(phi)
// (0, -c sin alpha, c cos alpha) and v = dphi/dt e_z x (x - axis) gives
// dv/dalpha = dphi/dt e_z x dx/dalpha.
fsi_status fsi_plate_pose_dalpha(int32_t nv, const double* s, const double* c, double t, double alpha, double omega,
                                 double t_ramp, int32_t law, double* dxda, double* dvda) {
  if (nv < 0 || (nv > 0 && (!s || !c || !dxda || !dvda))) return FSI_EINVAL;
  double ph[2];
  const double axis0[3] = {0.0, 0.0, 0.0};
  std::vector<double> xs(3 * (size_t)std::max(nv, 1)), vs(3 * (size_t)std::max(nv, 1));
  const fsi_status st = fsi_plate_pose(nv, s, c, t, alpha, omega, t_ramp, law, axis0, xs.data(), vs.data(), ph);
  if (st != FSI_OK) return st;
  const double cp = cos(ph[0]), sp = sin(ph[0]), ca = cos(alpha), sa = sin(alpha);
  for (int32_t i = 0; i < nv; ++i) {
    const double ly = -c[i] * sa, lz = c[i] * ca;
    const double rx = -sp * ly, ry = cp * ly;
    dxda[3 * i] = rx;
    dxda[3 * i + 1] = ry;
    dxda[3 * i + 2] = lz;
    dvda[3 * i] = -ph[1] * ry;
    dvda[3 * i + 1] = ph[1] * rx;
    dvda[3 * i + 2] = 0.0;
  }
  return FSI_OK;
}

}  // extern "C"
