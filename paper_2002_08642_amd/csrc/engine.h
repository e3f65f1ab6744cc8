// engine.h - the step engine behind the C ABI (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/fsi.h"

namespace fsi {

class EngineBase {
 public:
  virtual ~EngineBase() {}
  virtual fsi_status init(const fsi_desc& d) = 0;
  virtual void band(int K[3], long long* clen) const = 0;
  virtual fsi_status set_velocity_host(const double* u) = 0;
  virtual fsi_status set_velocity_device(const void* u, int dtype) = 0;
  virtual fsi_status set_spectrum(const double* uh) = 0;
  virtual fsi_status get_velocity(double* u) = 0;
  virtual fsi_status get_spectrum(double* uh) = 0;
  virtual fsi_status get_nonlinear(double* nh) = 0;
  virtual fsi_status set_wing(int nv, const double* x, const double* v, int nt, const int* tri) = 0;
  virtual fsi_status set_sponge(double c_sp, const double* gx, const double* gy, const double* gz) = 0;
  virtual fsi_status set_static_mask(const double* chi, const double* us, const double* w) = 0;
  virtual fsi_status static_force(double F[3]) = 0;
  virtual fsi_status get_mask(double* chi, double* us) = 0;
  // get_mask into device grids with caller-provided key scratch (2 * max_cells
  // u64); queued on the stream, allocates nothing
  virtual fsi_status get_mask_grid(void* chi, void* us, unsigned long long* scratch, long long max_cells) = 0;
  virtual fsi_status step(bool adaptive, double dt, double cfl, double c_eta, double dt_max) = 0;
  virtual fsi_status step_info(double F[3], double* dt, double* E, double* umax, double* t, long long* nstep) = 0;
  virtual fsi_status fft_r2c(const double* f, double* fh) = 0;
  virtual fsi_status fft_c2r(const double* fh, double* f) = 0;
  virtual fsi_status save_state(int slot) = 0;
  virtual fsi_status save_tape(int slot) = 0;
  virtual fsi_status step_record(double dt, int slot) = 0;
  virtual fsi_status load_state(int slot) = 0;
  virtual fsi_status synchronize() = 0;
  virtual fsi_status adjoint_set(const double* lu, const double* lnp) = 0;
  virtual fsi_status adjoint_get(double* lu, double* lnp) = 0;
  virtual fsi_status step_adjoint(int slot, double dt, double dtp, int first, const double dJdF[3], double* dJdx,
                                  double* dJdv) = 0;
  virtual fsi_status sample_pressure(int n, const double* pts, double* p) = 0;
  virtual fsi_status pressure_loads(double* loads, double* dp) = 0;
  virtual fsi_status eval_pressure() = 0;
  virtual fsi_status pressure_box(int box0[3], int boxn[3], double* p) = 0;
  virtual fsi_status set_pressure_seed(const int box0[3], const int boxn[3], const double* lam) = 0;
  virtual fsi_status set_timing(unsigned pass_mask) = 0;
  virtual fsi_status poison_padding(double v) = 0;
  virtual fsi_status pass_times(double ms[FSI_NPASS], int* nsteps) = 0;
  std::string err;
};

EngineBase* make_engine_f32();
EngineBase* make_engine_f64();

// Validates a descriptor; returns an empty string if it is acceptable.
std::string check_desc(const fsi_desc& d);

}  // namespace fsi
