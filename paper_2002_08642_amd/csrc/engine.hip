// engine.hip - host orchestration of the penalized pseudo-spectral step.
//
// Owns the device buffers, the transform plans and the time-stepping state,
// and queues the passes of one step on the context stream (Sec. 4.1: the
// fluid is advanced with the mask and solid velocity of the current wing
// position, then the Adams-Bashforth update is applied).
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <string>
#include <vector>

#include "engine.h"
#include "launch.h"

namespace fsi {

#define FSI_HIP(expr)                                                          \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      err = std::string(#expr) + ": " + hipGetErrorString(e_);                 \
      return FSI_EDEVICE;                                                      \
    }                                                                          \
  } while (0)

#define FSI_TRY(expr)              \
  do {                             \
    fsi_status s_ = (expr);        \
    if (s_ != FSI_OK) return s_;   \
  } while (0)

static bool factor_ok(int n) {
  if (n < 8 || n > 2048 || (n & 1)) return false;
  int m = n;
  for (int p : {2, 3, 5})
    while (m % p == 0) m /= p;
  return m == 1;
}

static bool make_plan(int n, FftPlan& p) {
  p.n = n;
  p.nst = 0;
  int m = n;
  for (int r : {8, 4, 2, 5, 3}) {
    while (m % r == 0) {
      if (p.nst >= kMaxStages) return false;
      p.radix[p.nst++] = r;
      m /= r;
    }
  }
  return m == 1;
}

static int band_k(int n) { return (n - 1) / 3; }  // largest m with 3m < n

std::string check_desc(const fsi_desc& d) {
  if (!factor_ok(d.nx) || !factor_ok(d.ny) || !factor_ok(d.nz))
    return "grid sizes must be even, 8..2048 and of the form 2^a 3^b 5^c";
  if (!(d.lx > 0) || !(d.ly > 0) || !(d.lz > 0) || !std::isfinite(d.lx) || !std::isfinite(d.ly) || !std::isfinite(d.lz))
    return "box lengths must be positive and finite";
  if (!(d.nu >= 0) || !std::isfinite(d.nu)) return "nu must be >= 0";
  if (!(d.eta > 0) || !std::isfinite(d.eta)) return "eta must be > 0";
  if (!(d.tw >= 0) || !std::isfinite(d.tw)) return "tw must be >= 0";
  if (!(d.h > 0) || !std::isfinite(d.h)) return "h must be > 0";
  if (d.mask_profile != FSI_PROFILE_COS && d.mask_profile != FSI_PROFILE_TANH) return "unknown mask profile";
  if (d.precision != FSI_PREC_FP32 && d.precision != FSI_PREC_FP64) return "unknown precision";
  if (d.fsi_pressure != 0 && d.fsi_pressure != 1) return "fsi_pressure must be 0 or 1";
  return "";
}

template <typename T>
class Engine : public EngineBase {
 public:
  ~Engine() override { release(); }

  fsi_status init(const fsi_desc& dd) override {
    d = dd;
    s = (hipStream_t)d.stream;
    nx = d.nx;
    ny = d.ny;
    nz = d.nz;
    Kx = band_k(nx);
    Ky = band_k(ny);
    Kz = band_k(nz);
    kx1 = Kx + 1;
    {
      const int line = 128 / (int)sizeof(cpx<T>);  // complex values per 128-byte line
      kxp = (kx1 + line - 1) / line * line;
    }
    nby = 2 * Ky + 1;
    nbz = 2 * Kz + 1;
    C1 = (long long)nby * kxp;
    clen = (long long)nbz * C1;
    clen_ext = (long long)nbz * nby * kx1;
    Alen = (long long)nz * C1;
    Blen = (long long)nz * ny * kxp;
    npts = (long long)nx * ny * nz;
    dxs[0] = d.lx / nx;
    dxs[1] = d.ly / ny;
    dxs[2] = d.lz / nz;
    dV = dxs[0] * dxs[1] * dxs[2];
    dx_min = std::min(dxs[0], std::min(dxs[1], dxs[2]));
    rsup = d.tw + (d.mask_profile == FSI_PROFILE_COS ? 1.0 : 6.0) * d.h;
    if (!make_plan(nx, px) || !make_plan(ny, py) || !make_plan(nz, pz)) {
      err = "cannot factor grid";
      return FSI_EINVAL;
    }
    for (int n : {ny, nz}) {
      if (col_width<T>(n) == 0) {
        err = "grid too long for the column passes in this precision";
        return FSI_EINVAL;
      }
    }
    const int L = xpass_lines<T>(nx);
    if (L == 0 || ((long long)ny * nz) % L != 0) {
      err = "nx too long for the x pass in this precision";
      return FSI_EINVAL;
    }
    ngroups = (int)(((long long)ny * nz) / L);
    npart = std::min(ngroups, 4096);
    nfused = xfused_grid(nx, (long long)ny * nz, L);

    FSI_TRY(alloc(&uh, 3 * clen));
    FSI_TRY(alloc(&nh, 3 * clen));
    FSI_TRY(alloc(&A, 6 * Alen));
    FSI_TRY(alloc(&B, 6 * Blen));
    FSI_TRY(alloc(&partials, (long long)std::max(npart, nfused) * 8));
    FSI_TRY(alloc(&sc, 1));
    FSI_HIP(hipHostMalloc((void**)&sc_host, sizeof(DevScalars), hipHostMallocDefault));
    FSI_TRY(make_twiddles(nx, &twx));
    FSI_TRY(make_twiddles(ny, &twy));
    FSI_TRY(make_twiddles(nz, &twz));
    FSI_HIP(hipMemsetAsync(uh, 0, sizeof(cpx<T>) * 3 * clen, s));
    FSI_HIP(hipMemsetAsync(nh, 0, sizeof(cpx<T>) * 3 * clen, s));
    if (d.fsi_pressure) {
      FSI_TRY(alloc(&pi_, clen));
      FSI_HIP(hipMemsetAsync(pi_, 0, sizeof(cpx<T>) * clen, s));
    }
    FSI_TRY(reset_scalars());
    FSI_HIP(hipStreamSynchronize(s));
    slots.resize(64);
    return FSI_OK;
  }

  void band(int K[3], long long* cl) const override {
    K[0] = Kx;
    K[1] = Ky;
    K[2] = Kz;
    *cl = clen_ext;
  }

  // -- velocity in / out -----------------------------------------------------
  fsi_status set_velocity_host(const double* u) override {
    for (long long i = 0; i < 3 * npts; ++i)
      if (!std::isfinite(u[i])) {
        err = "non-finite value in the velocity";
        return FSI_EINVAL;
      }
    FSI_TRY(ensure_phys());
    FSI_TRY(upload_real(u, phys, 3 * npts));
    return finish_set_velocity();
  }

  fsi_status set_velocity_device(const void* u, int dtype) override {
    if (dtype != 0 && dtype != 1) {
      err = "dtype must be 0 (float) or 1 (double)";
      return FSI_EINVAL;
    }
    FSI_TRY(ensure_phys());
    if ((dtype == 1) == (sizeof(T) == 8)) {
      FSI_HIP(hipMemcpyAsync(phys, u, sizeof(T) * 3 * npts, hipMemcpyDeviceToDevice, s));
    } else {
      std::vector<double> h(3 * npts);
      if (dtype == 1) {
        FSI_HIP(hipMemcpyAsync(h.data(), u, sizeof(double) * 3 * npts, hipMemcpyDeviceToHost, s));
        FSI_HIP(hipStreamSynchronize(s));
      } else {
        std::vector<float> f(3 * npts);
        FSI_HIP(hipMemcpyAsync(f.data(), u, sizeof(float) * 3 * npts, hipMemcpyDeviceToHost, s));
        FSI_HIP(hipStreamSynchronize(s));
        for (long long i = 0; i < 3 * npts; ++i) h[i] = f[i];
      }
      FSI_TRY(upload_real(h.data(), phys, 3 * npts));
    }
    return finish_set_velocity();
  }

  fsi_status set_spectrum(const double* in) override {
    for (long long i = 0; i < 6 * clen_ext; ++i)
      if (!std::isfinite(in[i])) {
        err = "non-finite value in the spectrum";
        return FSI_EINVAL;
      }
    FSI_TRY(ensure_phys());
    std::vector<cpx<T>> h(3 * clen);
    memset(h.data(), 0, sizeof(cpx<T>) * 3 * clen);
    for (int q = 0; q < 3; ++q) pad(in + 2 * q * clen_ext, h.data() + q * clen);
    FSI_HIP(hipMemcpyAsync(uh, h.data(), sizeof(cpx<T>) * 3 * clen, hipMemcpyHostToDevice, s));
    zs_valid = false;
    FSI_TRY(run_inverse(uh, clen, 3, phys));
    return finish_set_velocity();
  }

  fsi_status get_velocity(double* u) override {
    FSI_TRY(ensure_phys());
    FSI_TRY(run_inverse(uh, clen, 3, phys));
    FSI_TRY(download_real(phys, u, 3 * npts));
    return nan_status();
  }

  fsi_status get_spectrum(double* out) override {
    std::vector<cpx<T>> h(3 * clen);
    FSI_HIP(hipMemcpyAsync(h.data(), uh, sizeof(cpx<T>) * 3 * clen, hipMemcpyDeviceToHost, s));
    FSI_HIP(hipStreamSynchronize(s));
    for (int q = 0; q < 3; ++q) unpad(h.data() + q * clen, out + 2 * q * clen_ext);
    return nan_status();
  }

  fsi_status get_nonlinear(double* out) override {
    std::vector<cpx<T>> h(3 * clen);
    FSI_HIP(hipMemcpyAsync(h.data(), nh, sizeof(cpx<T>) * 3 * clen, hipMemcpyDeviceToHost, s));
    FSI_HIP(hipStreamSynchronize(s));
    for (int q = 0; q < 3; ++q) unpad(h.data() + q * clen, out + 2 * q * clen_ext);
    return nan_status();
  }

  // -- wing --------------------------------------------------------------------
  fsi_status set_wing(int nv, const double* x, const double* v, int nt, const int* tri) override {
    if (nt < 0 || nv < 0 || (nt > 0 && (nv < 3 || !x || !v || !tri))) {
      err = "invalid mesh sizes or pointers";
      return FSI_EINVAL;
    }
    if (nt == 0) {
      wing_nt = 0;
      bnx = bny = bnz = 0;
      pnx = pny = pnz = 0;
      p_ready = false;
      return FSI_OK;
    }
    for (long long i = 0; i < 3LL * nt; ++i)
      if (tri[i] < 0 || tri[i] >= nv) {
        err = "triangle vertex id out of range";
        return FSI_EINVAL;
      }
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (long long i = 0; i < nv; ++i)
      for (int q = 0; q < 3; ++q) {
        const double a = x[3 * i + q];
        if (!std::isfinite(a) || !std::isfinite(v[3 * i + q])) {
          err = "non-finite vertex position or velocity";
          return FSI_EINVAL;
        }
        lo[q] = std::min(lo[q], a);
        hi[q] = std::max(hi[q], a);
      }
    const double Ls[3] = {d.lx, d.ly, d.lz};
    const int Ns[3] = {nx, ny, nz};
    int i0[3], cnt[3];
    for (int q = 0; q < 3; ++q) {
      const double a = lo[q] - rsup, b = hi[q] + rsup;
      if (a < 0.0 || b > Ls[q]) {
        err = "wing bounding box enlarged by the mask support leaves the box";
        return FSI_EBOUNDS;
      }
      i0[q] = std::max(0, (int)std::floor(a / dxs[q]));
      const int i1 = std::min(Ns[q] - 1, (int)std::ceil(b / dxs[q]));
      cnt[q] = std::max(0, i1 - i0[q] + 1);
    }
    const long long cells = (long long)cnt[0] * cnt[1] * cnt[2];
    // FSI mode: pressure box (every 4-point stencil of a point within d = t_w + h
    // of the mesh bounding box), vertex load vectors and sample points
    int q0[3] = {0, 0, 0}, qn[3] = {0, 0, 0};
    std::vector<double> cv, samp;
    if (d.fsi_pressure) {
      const double dd = d.tw + d.h;
      for (int q = 0; q < 3; ++q) {
        const int a = (int)std::floor((lo[q] - dd) / dxs[q]) - 1;
        const int b = (int)std::floor((hi[q] + dd) / dxs[q]) + 2;
        if (a < 0 || b > Ns[q] - 1) {
          err = "pressure box (mesh bounding box enlarged by t_w + h and the delta-kernel stencil) leaves the box";
          return FSI_EBOUNDS;
        }
        q0[q] = a;
        qn[q] = b - a + 1;
      }
      cv.assign(3 * (size_t)nv, 0.0);
      for (long long t = 0; t < nt; ++t) {
        const int* v3 = tri + 3 * t;
        double e1[3], e2[3];
        for (int q = 0; q < 3; ++q) {
          e1[q] = x[3 * v3[1] + q] - x[3 * v3[0] + q];
          e2[q] = x[3 * v3[2] + q] - x[3 * v3[0] + q];
        }
        // A_T n_T / 3 = (e1 x e2) / 6
        const double c[3] = {(e1[1] * e2[2] - e1[2] * e2[1]) / 6.0, (e1[2] * e2[0] - e1[0] * e2[2]) / 6.0,
                             (e1[0] * e2[1] - e1[1] * e2[0]) / 6.0};
        for (int k = 0; k < 3; ++k)
          for (int q = 0; q < 3; ++q) cv[3 * (size_t)v3[k] + q] += c[q];
      }
      samp.assign(6 * (size_t)nv, 0.0);
      for (long long i = 0; i < nv; ++i) {
        const double* c = &cv[3 * i];
        const double nrm = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        for (int q = 0; q < 3; ++q) {
          const double off = nrm > 0.0 ? dd * c[q] / nrm : 0.0;
          samp[6 * i + q] = x[3 * i + q] + off;
          samp[6 * i + 3 + q] = x[3 * i + q] - off;
        }
      }
    }
    // stage the mesh through pinned memory; it is uploaded in one copy on the
    // side stream (the mask that needs it runs there; work on the context
    // stream that reads it waits for the upload's event)
    FSI_TRY(ensure_side());
    const size_t need = sizeof(double) * 6 * (size_t)nv + sizeof(int) * 3 * (size_t)nt;
    if (need > stage_cap) {
      FSI_TRY(sync_both());
      if (stage) FSI_HIP(hipHostFree(stage));
      stage = nullptr;
      FSI_HIP(hipHostMalloc(&stage, need * 2, hipHostMallocDefault));
      stage_cap = need * 2;
    }
    if (stage_pending) FSI_HIP(hipEventSynchronize(stage_ev));
    double* sx = (double*)stage;
    double* sv = sx + 3 * (size_t)nv;
    int* st = (int*)(sv + 3 * (size_t)nv);
    memcpy(sx, x, sizeof(double) * 3 * (size_t)nv);
    memcpy(sv, v, sizeof(double) * 3 * (size_t)nv);
    memcpy(st, tri, sizeof(int) * 3 * (size_t)nt);
    tri_host.assign(tri, tri + 3 * (size_t)nt);
    if ((long long)need > mesh_cap) {
      FSI_TRY(sync_both());
      free_dev(dmesh_);
      mesh_cap = 2 * (long long)need;
      FSI_TRY(alloc(&dmesh_, mesh_cap));
    }
    if (d.fsi_pressure) {
      const long long pc = (long long)qn[0] * qn[1] * qn[2];
      if (pc > pbox_cap) {
        FSI_HIP(hipStreamSynchronize(s));
        free_dev(up_);
        pbox_cap = pc + pc / 4 + 64;
        FSI_TRY(alloc(&up_, 3 * pbox_cap));
      }
      if (2LL * nv > psamp_cap) {
        FSI_HIP(hipStreamSynchronize(s));
        free_dev(dsamp_);
        free_dev(dpout_);
        psamp_cap = 4LL * nv;
        FSI_TRY(alloc(&dsamp_, 3 * psamp_cap));
        FSI_TRY(alloc(&dpout_, psamp_cap));
      }
    }
    if (cells > box_cap) {
      FSI_TRY(sync_both());
      free_dev(key1);
      free_dev(key2);
      free_dev(chi);
      free_dev(us);
      box_cap = cells + cells / 4 + 64;
      FSI_TRY(alloc(&key1, box_cap));
      FSI_TRY(alloc(&key2, box_cap));
      FSI_TRY(alloc(&chi, box_cap));
      FSI_TRY(alloc(&us, 3 * box_cap));
    }
    // device views with the staging layout: x [nv][3], v [nv][3], tri [nt][3]
    dx_ = reinterpret_cast<double*>(dmesh_);
    dv_ = dx_ + 3 * (size_t)nv;
    dtri_ = reinterpret_cast<int*>(dv_ + 3 * (size_t)nv);
    FSI_HIP(hipMemcpyAsync(dmesh_, stage, need, hipMemcpyHostToDevice, s2));
    if (!stage_ev) FSI_HIP(hipEventCreateWithFlags(&stage_ev, hipEventDisableTiming));
    FSI_HIP(hipEventRecord(stage_ev, s2));
    stage_pending = true;
    FSI_HIP(hipEventRecord(e_up, s2));
    mesh_pending = true;
    wing_nt = nt;
    wing_nv = nv;
    bx0 = i0[0];
    by0 = i0[1];
    bz0 = i0[2];
    bnx = cnt[0];
    bny = cnt[1];
    bnz = cnt[2];
    bcells = cells;
    if (d.fsi_pressure) {
      px0 = q0[0];
      py0 = q0[1];
      pz0 = q0[2];
      pnx = qn[0];
      pny = qn[1];
      pnz = qn[2];
      pcells = (long long)pnx * pny * pnz;
      load_cv.swap(cv);
      samp_host.swap(samp);
    }
    p_ready = false;
    seed_pending = false;
    return FSI_OK;
  }

  // -- pressure samples and wing loads (FSI mode) ----------------------------------
  fsi_status pressure_ready() {
    if (!d.fsi_pressure) {
      err = "FSI mode (fsi_pressure) is off";
      return FSI_ESTATE;
    }
    if (!p_ready || wing_nt == 0 || pcells == 0) {
      err = "no step since the wing was set or the state was loaded";
      return FSI_ESTATE;
    }
    return FSI_OK;
  }

  // p = Pi - |u|^2/2 at n points (host FP64 [n][3]) into out[n]
  fsi_status run_psample(int n, const double* pts_host, double* out) {
    for (int i = 0; i < n; ++i)
      for (int q = 0; q < 3; ++q) {
        const int pq0 = q == 0 ? px0 : (q == 1 ? py0 : pz0), pqn = q == 0 ? pnx : (q == 1 ? pny : pnz);
        const double g = pts_host[3 * i + q] / dxs[q];
        if (!std::isfinite(g)) {
          err = "non-finite sample point";
          return FSI_EINVAL;
        }
        const int a = (int)std::floor(g) - 1;
        if (a < pq0 || a + 3 > pq0 + pqn - 1) {
          err = "sample stencil leaves the pressure box";
          return FSI_EBOUNDS;
        }
      }
    if (n == 0) return FSI_OK;
    if (!phys) FSI_TRY(alloc(&phys, 3 * npts));
    if (n > psamp_cap) {
      FSI_HIP(hipStreamSynchronize(s));
      free_dev(dsamp_);
      free_dev(dpout_);
      psamp_cap = 2LL * n;
      FSI_TRY(alloc(&dsamp_, 3 * psamp_cap));
      FSI_TRY(alloc(&dpout_, psamp_cap));
    }
    FSI_TRY(run_inverse(pi_, clen, 1, phys));  // Pi on the grid
    FSI_HIP(hipMemcpyAsync(dsamp_, pts_host, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s));
    PressArgs<T> a;
    a.pi = phys;
    a.up = up_;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.px0 = px0;
    a.py0 = py0;
    a.pz0 = pz0;
    a.pnx = pnx;
    a.pny = pny;
    a.pnz = pnz;
    a.pcells = pcells;
    a.pts = dsamp_;
    a.ns = n;
    a.dx = dxs[0];
    a.dy = dxs[1];
    a.dz = dxs[2];
    a.out = dpout_;
    FSI_HIP(launch_psample<T>(a, s));
    FSI_HIP(hipMemcpyAsync(out, dpout_, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    FSI_HIP(hipStreamSynchronize(s));
    return FSI_OK;
  }

  fsi_status sample_pressure(int n, const double* pts, double* p) override {
    if (n < 0 || (n > 0 && (!pts || !p))) {
      err = "invalid sample arrays";
      return FSI_EINVAL;
    }
    FSI_TRY(pressure_ready());
    return run_psample(n, pts, p);
  }

  fsi_status pressure_box(int box0[3], int boxn[3], double* p) override {
    if (!d.fsi_pressure || wing_nt == 0 || pcells == 0) {
      err = "no pressure box: FSI mode off or no wing";
      return FSI_ESTATE;
    }
    box0[0] = px0;
    box0[1] = py0;
    box0[2] = pz0;
    boxn[0] = pnx;
    boxn[1] = pny;
    boxn[2] = pnz;
    if (!p) return FSI_OK;
    FSI_TRY(pressure_ready());
    if (!phys) FSI_TRY(alloc(&phys, 3 * npts));
    if (pcells > dpbox_cap) {
      FSI_HIP(hipStreamSynchronize(s));
      free_dev(dpbox_);
      dpbox_cap = pcells + pcells / 4;
      FSI_TRY(alloc(&dpbox_, dpbox_cap));
    }
    FSI_TRY(run_inverse(pi_, clen, 1, phys));
    BoxArgs<T> a = box_args();
    a.pi = phys;
    a.out = dpbox_;
    FSI_HIP(launch_pbox<T>(0, a, s));
    FSI_HIP(hipMemcpyAsync(p, dpbox_, sizeof(double) * pcells, hipMemcpyDeviceToHost, s));
    FSI_HIP(hipStreamSynchronize(s));
    return FSI_OK;
  }

  fsi_status set_pressure_seed(const int box0[3], const int boxn[3], const double* lam) override {
    if (!d.fsi_pressure || wing_nt == 0 || pcells == 0) {
      err = "no pressure box: FSI mode off or no wing";
      return FSI_ESTATE;
    }
    if (box0[0] != px0 || box0[1] != py0 || box0[2] != pz0 || boxn[0] != pnx || boxn[1] != pny || boxn[2] != pnz) {
      err = "pressure seed box differs from the box of the current mesh";
      return FSI_EINVAL;
    }
    if (!lam) {
      seed_pending = false;
      return FSI_OK;
    }
    if (pcells > lp_cap) {
      FSI_HIP(hipStreamSynchronize(s));
      free_dev(lp_);
      lp_cap = pcells + pcells / 4;
      FSI_TRY(alloc(&lp_, lp_cap));
    }
    std::vector<T> h(pcells);
    for (long long c = 0; c < pcells; ++c) h[c] = (T)lam[c];
    FSI_HIP(hipMemcpyAsync(lp_, h.data(), sizeof(T) * pcells, hipMemcpyHostToDevice, s));
    FSI_HIP(hipStreamSynchronize(s));
    seed_pending = true;
    return FSI_OK;
  }

  BoxArgs<T> box_args() {
    BoxArgs<T> a;
    memset(&a, 0, sizeof(a));
    a.up = up_;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.px0 = px0;
    a.py0 = py0;
    a.pz0 = pz0;
    a.pnx = pnx;
    a.pny = pny;
    a.pnz = pnz;
    a.pcells = pcells;
    return a;
  }

  fsi_status pressure_loads(double* loads, double* dp) override {
    if (!loads) {
      err = "loads is NULL";
      return FSI_EINVAL;
    }
    FSI_TRY(pressure_ready());
    std::vector<double> p(2 * (size_t)wing_nv);
    FSI_TRY(run_psample(2 * wing_nv, samp_host.data(), p.data()));
    for (int i = 0; i < wing_nv; ++i) {
      const double jump = p[2 * i] - p[2 * i + 1];
      if (dp) dp[i] = jump;
      for (int q = 0; q < 3; ++q) loads[3 * i + q] = -jump * load_cv[3 * (size_t)i + q];
    }
    return FSI_OK;
  }

  fsi_status get_mask(double* chi_h, double* us_h) override {
    memset(chi_h, 0, sizeof(double) * npts);
    memset(us_h, 0, sizeof(double) * 3 * npts);
    if (wing_nt == 0 || bcells == 0) return FSI_OK;
    FSI_TRY(run_mask(s));
    std::vector<T> c(bcells), u(3 * bcells);
    FSI_HIP(hipMemcpyAsync(c.data(), chi, sizeof(T) * bcells, hipMemcpyDeviceToHost, s));
    FSI_HIP(hipMemcpyAsync(u.data(), us, sizeof(T) * 3 * bcells, hipMemcpyDeviceToHost, s));
    FSI_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < bnz; ++k)
      for (int j = 0; j < bny; ++j)
        for (int i = 0; i < bnx; ++i) {
          const long long cell = ((long long)k * bny + j) * bnx + i;
          const long long g = ((long long)(k + bz0) * ny + (j + by0)) * nx + (i + bx0);
          chi_h[g] = (double)c[cell];
          for (int q = 0; q < 3; ++q) us_h[q * npts + g] = (double)u[q * bcells + cell];
        }
    return FSI_OK;
  }

  fsi_status get_mask_grid(void* chi_out, void* us_out, unsigned long long* scratch, long long max_cells) override {
    if (!chi_out || !us_out) {
      err = "chi and us must be device pointers";
      return FSI_EINVAL;
    }
    const bool wing = wing_nt > 0 && bcells > 0;
    if (wing && bcells > max_cells) {
      err = "mask sub-box of " + std::to_string(bcells) + " cells exceeds the " + std::to_string(max_cells) +
            " cells of the fixed scratch";
      return FSI_EINVAL;
    }
    FSI_TRY(mesh_wait(s));
    MaskArgs<T> m;
    memset(&m, 0, sizeof(m));
    m.x = dx_;
    m.v = dv_;
    m.tri = dtri_;
    m.nt = wing ? wing_nt : 0;
    m.key1 = scratch;
    m.key2 = scratch + max_cells;
    m.chi = (T*)chi_out;
    m.us = (T*)us_out;
    m.bx0 = bx0;
    m.by0 = by0;
    m.bz0 = bz0;
    m.bnx = bnx;
    m.bny = bny;
    m.bnz = bnz;
    m.bcells = wing ? bcells : 0;
    m.dx = dxs[0];
    m.dy = dxs[1];
    m.dz = dxs[2];
    m.rsup = rsup;
    m.tw = d.tw;
    m.h = d.h;
    m.profile = d.mask_profile;
    m.gnx = nx;
    m.gny = ny;
    m.gcells = npts;
    FSI_HIP(launch_mask_grid<T>(m, s));
    return FSI_OK;
  }

  // static z-independent penalization (walls, fixed obstacles, inflow layers)
  fsi_status set_static_mask(const double* chi_h, const double* us_h, const double* w_h) override {
    if (!chi_h) {
      static_on = false;
      return FSI_OK;
    }
    if (!us_h) {
      err = "u_s of the static mask is NULL";
      return FSI_EINVAL;
    }
    const long long np2 = (long long)nx * ny;
    for (long long i = 0; i < np2; ++i) {
      if (!(chi_h[i] >= 0.0 && chi_h[i] <= 1.0)) {
        err = "static chi must lie in [0, 1]";
        return FSI_EINVAL;
      }
      if (w_h && !std::isfinite(w_h[i])) {
        err = "non-finite static force weight";
        return FSI_EINVAL;
      }
    }
    for (long long i = 0; i < 3 * np2; ++i)
      if (!std::isfinite(us_h[i])) {
        err = "non-finite static u_s";
        return FSI_EINVAL;
      }
    if (!st_chi_) {
      FSI_TRY(alloc(&st_chi_, np2));
      FSI_TRY(alloc(&st_us_, 3 * np2));
      FSI_TRY(alloc(&st_w_, np2));
    }
    std::vector<T> h(5 * (size_t)np2);
    for (long long i = 0; i < np2; ++i) {
      h[i] = (T)chi_h[i];
      h[4 * np2 + i] = w_h ? (T)w_h[i] : (T)0;
    }
    for (long long i = 0; i < 3 * np2; ++i) h[np2 + i] = (T)us_h[i];
    FSI_TRY(sync_both());
    FSI_HIP(hipMemcpy(st_chi_, h.data(), sizeof(T) * np2, hipMemcpyHostToDevice));
    FSI_HIP(hipMemcpy(st_us_, h.data() + np2, sizeof(T) * 3 * np2, hipMemcpyHostToDevice));
    FSI_HIP(hipMemcpy(st_w_, h.data() + 4 * np2, sizeof(T) * np2, hipMemcpyHostToDevice));
    static_on = true;
    return FSI_OK;
  }

  fsi_status static_force(double F[3]) override {
    if (info_pending) FSI_HIP(hipEventSynchronize(info_ev));
    else FSI_HIP(hipStreamSynchronize(s));
    for (int q = 0; q < 3; ++q) F[q] = sc_host->fst[q];
    return nan_status();
  }

  // -- one step ------------------------------------------------------------------
  // vorticity sponge: chi_sp = max(gx[x], gy[y], gz[z]) (NULL profile = 0), c_sp <= 0: off
  fsi_status set_sponge(double c_sp, const double* gx, const double* gy, const double* gz) override {
    if (!std::isfinite(c_sp)) {
      err = "c_sp must be finite";
      return FSI_EINVAL;
    }
    if (c_sp <= 0.0 || (!gx && !gy && !gz)) {
      sponge_on = false;
      return FSI_OK;
    }
    std::vector<T> g((size_t)nx + ny + nz, (T)0);
    const double* src[3] = {gx, gy, gz};
    const int len[3] = {nx, ny, nz};
    size_t o = 0;
    for (int q = 0; q < 3; ++q) {
      for (int i = 0; i < len[q]; ++i) {
        const double v = src[q] ? src[q][i] : 0.0;
        if (!(v >= 0.0) || !std::isfinite(v)) {
          err = "sponge profiles must be finite and >= 0";
          return FSI_EINVAL;
        }
        g[o + i] = (T)v;
      }
      o += len[q];
    }
    FSI_TRY(ensure_phys());
    if (!spg_) FSI_TRY(alloc(&spg_, (long long)nx + ny + nz));
    if (!tsp_) FSI_TRY(alloc(&tsp_, 3 * clen));
    FSI_HIP(hipMemcpyAsync(spg_, g.data(), sizeof(T) * g.size(), hipMemcpyHostToDevice, s));
    FSI_HIP(hipStreamSynchronize(s));
    csp = c_sp;
    sponge_on = true;
    return FSI_OK;
  }

  fsi_status step(bool adaptive, double dt, double cfl, double c_eta, double dt_max) override {
    if (adaptive) {
      if (!(cfl > 0) || !(c_eta > 0) || !(dt_max > 0) || !std::isfinite(cfl) || !std::isfinite(dt_max)) {
        err = "adaptive step needs cfl > 0, c_eta > 0, dt_max > 0";
        return FSI_EINVAL;
      }
      if (c_eta > 1.0) {
        err = "c_eta > 1 makes the explicit penalization unstable";
        return FSI_ESTABILITY;
      }
    } else {
      if (!(dt > 0) || !std::isfinite(dt)) {
        err = "dt must be positive and finite";
        return FSI_EINVAL;
      }
      if ((wing_nt > 0 || static_on) && dt / d.eta > 1.0) {
        err = "dt * max(chi) / eta > 1: explicit penalization unstable";
        return FSI_ESTABILITY;
      }
    }
    const int cur = (int)(nstep & 1);
    hipEvent_t* ev = timing ? next_events() : nullptr;
    // The mask depends only on the wing: it runs on the side stream while P1/P2
    // transform the velocity, and P3 waits for it.  It starts after everything
    // queued so far on the context stream (the mesh upload, and the previous
    // step's P3, which read the mask buffers).
    const bool wing = wing_nt > 0 && bcells > 0;
    FSI_TRY(ensure_side());
    if (wing) {
      FSI_HIP(hipEventRecord(e_ready, s));
      FSI_HIP(hipStreamWaitEvent(s2, e_ready, 0));
      if (ev && ev_need[EV_MASK0]) FSI_HIP(hipEventRecord(ev[EV_MASK0], s2));
      FSI_TRY(run_mask(s2));
      if (ev && ev_need[EV_MASK1]) FSI_HIP(hipEventRecord(ev[EV_MASK1], s2));
      FSI_HIP(hipEventRecord(e_mask, s2));
    } else if (ev && ev_need[EV_MASK0]) {
      FSI_HIP(hipEventRecord(ev[EV_MASK0], s));
      FSI_HIP(hipEventRecord(ev[EV_MASK1], s));
    }
    if (ev && ev_need[EV_P1_0]) FSI_HIP(hipEventRecord(ev[EV_P1_0], s));
    // P1: z inverse of u and of omega_x, omega_y (omega = i k x u); the
    // previous step's last pass has already produced it unless u_hat has been
    // replaced or A used since
    if (!zs_valid) {
      ColArgs<T> a = col_base(pz, twz, nz, Kz, C1, C1);
      a.in = uh;
      a.in_fs = clen;
      a.out = A;
      a.out_fs = Alen;
      FSI_HIP(launch_col<T>(COL_INV_CURL5, a, 1, s));  // u, omega_x, omega_y
    }
    zs_valid = false;
    if (ev && ev_need[EV_P2_0]) FSI_HIP(hipEventRecord(ev[EV_P2_0], s));
    // P2: y inverse of the five fields, omega_z = i (kx uy - ky ux) formed on the way
    // (into the step's tape when recording: the reverse step reads u, omega there)
    {
      ColArgs<T> a = col_base(py, twy, ny, Ky, kx1, kxp);
      a.in = A;
      a.in_fs = Alen;
      a.in_bs = C1;
      a.out = rec_bt ? rec_bt : B;
      a.out_fs = Blen;
      a.out_bs = (long long)ny * kxp;
      FSI_HIP(launch_col<T>(COL_INV_WZ, a, nz, s));
    }
    if (ev && ev_need[EV_P2_1]) FSI_HIP(hipEventRecord(ev[EV_P2_1], s));
    if (wing) FSI_HIP(hipStreamWaitEvent(s, e_mask, 0));
    if (ev && ev_need[EV_P3_0]) FSI_HIP(hipEventRecord(ev[EV_P3_0], s));
    // P3: x C2R, nonlinear + penalization term, diagnostics, x R2C
    FSI_HIP(launch_xfused<T>(p3_args(), nfused, s));
    // the reductions need only P3's partials: they run on the side stream
    // alongside the rest of the step, and P5 (which reads dt_n) waits for them
    FSI_HIP(hipEventRecord(e_x, s));
    FSI_HIP(hipStreamWaitEvent(s2, e_x, 0));
    // sponge: S = chi_sp omega from the x-spectral omega left in fields 3-5 of B
    // (x inverse, mask, x forward, back into the same fields)
    if (sponge_on && nx == 512) {  // register transforms, in place
      XArgs<T> a = x_base();
      a.spec = B;
      a.sfs = Blen;
      FSI_HIP(launch_xsponge<T>(a, spg_, nfused, s));
    } else if (sponge_on) {
      XArgs<T> a = x_base();
      a.spec = B + 3 * Blen;
      a.sfs = Blen;
      a.phys = phys;
      a.pfs = npts;
      FSI_HIP(launch_xplain<T>(X_C2R, 3, a, npart, s));
      SpongeArgs<T> m;
      m.phys = phys;
      m.npts = npts;
      m.nx = nx;
      m.ny = ny;
      m.nz = nz;
      m.g = spg_;
      FSI_HIP(launch_sponge_mask<T>(m, s));
      FSI_HIP(launch_xplain<T>(X_R2C, 3, a, npart, s));
    }
    if (ev && ev_need[EV_P3_1]) FSI_HIP(hipEventRecord(ev[EV_P3_1], s));
    // diagnostics and dt_n (side stream)
    {
      if (ev && ev_need[EV_RED0]) FSI_HIP(hipEventRecord(ev[EV_RED0], s2));
      FinalArgs f;
      f.partials = partials;
      f.np = nfused;
      f.sc = sc;
      f.cur = cur;
      f.adaptive = adaptive ? 1 : 0;
      f.dt_fixed = dt;
      f.cfl_dx = adaptive ? cfl * dx_min : 0.0;
      f.cap = adaptive ? std::min(c_eta * d.eta, dt_max) : 0.0;
      f.dV = dV;
      f.inv_eta = 1.0 / d.eta;
      FSI_HIP(launch_finalize(f, s2));
      // the diagnostics and dt_n are final here: the read-back does not wait for
      // the last two passes, so the caller can prepare the next step meanwhile
      FSI_HIP(hipMemcpyAsync(sc_host, sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s2));
      if (!info_ev) FSI_HIP(hipEventCreateWithFlags(&info_ev, hipEventDisableTiming));
      FSI_HIP(hipEventRecord(info_ev, s2));
      info_pending = true;
      if (ev && ev_need[EV_RED1]) FSI_HIP(hipEventRecord(ev[EV_RED1], s2));
      FSI_HIP(hipEventRecord(e_fin, s2));
    }
    // P4: y forward of G, truncated to the y band
    {
      ColArgs<T> a = col_base(py, twy, ny, Ky, kx1, kxp);
      a.in = B;
      a.in_fs = Blen;
      a.in_bs = (long long)ny * kxp;
      a.out = A;
      a.out_fs = Alen;
      a.out_bs = C1;
      a.nf = sponge_on ? 6 : 3;  // G, and S with the sponge
      a.scale = (T)1;
      FSI_HIP(launch_col<T>(COL_FWD_PLAIN, a, nz, s));
    }
    if (sponge_on) {  // z forward of S and the sponge term T_hat = -(1/C_sp) i k x S_hat / |k|^2
      ColArgs<T> a = col_base(pz, twz, nz, Kz, C1, C1);
      a.in = A + 3 * Alen;
      a.in_fs = Alen;
      a.out = tsp_;
      a.cfs = clen;
      a.scale = (T)(1.0 / (double)npts);
      a.csp_inv = (T)(1.0 / csp);
      FSI_HIP(launch_col<T>(COL_FWD_SPONGE, a, 1, s));
    }
    if (ev && ev_need[EV_P4_1]) FSI_HIP(hipEventRecord(ev[EV_P4_1], s));
    FSI_HIP(hipStreamWaitEvent(s, e_fin, 0));
    if (ev && ev_need[EV_P5_0]) FSI_HIP(hipEventRecord(ev[EV_P5_0], s));
    // P5: z forward, dealias, Leray projection, integrating-factor AB2
    {
      ColArgs<T> a = col_base(pz, twz, nz, Kz, C1, C1);
      a.in = A;
      a.in_fs = Alen;
      a.uh = uh;
      a.nh = nh;
      a.cfs = clen;
      a.sc = sc;
      a.cur = cur;
      a.first = have_prev ? 0 : 1;
      a.nu = (T)d.nu;
      a.scale = (T)(1.0 / (double)npts);
      a.pi = d.fsi_pressure ? pi_ : nullptr;
      a.tsp = sponge_on ? tsp_ : nullptr;
      // and P1 of the next step on the same columns (in place: each workgroup
      // has read all rows of its columns of A before it writes them)
      a.zout = A;
      a.zout_fs = Alen;
      FSI_HIP(launch_col<T>(COL_FWD_UPDATE_Z, a, 1, s));
      zs_valid = true;
    }
    if (ev && ev_need[EV_P5_1]) FSI_HIP(hipEventRecord(ev[EV_P5_1], s));
    ++nstep;
    have_prev = true;
    p_ready = d.fsi_pressure && wing_nt > 0 && bcells > 0;
    return FSI_OK;
  }

  // Arguments of the fused x pass: mask sub-box, and the pressure box in FSI mode
  XArgs<T> p3_args() {
    XArgs<T> a = x_base();
    a.spec = rec_bt ? rec_bt : B;  // u, omega (the step's tape when recording)
    a.gout = B;                    // G
    a.sfs = Blen;
    a.partials = partials;
    if (wing_nt > 0 && bcells > 0) {
      a.chi = chi;
      a.us = us;
      a.bx0 = bx0;
      a.by0 = by0;
      a.bz0 = bz0;
      a.bnx = bnx;
      a.bny = bny;
      a.bnz = bnz;
      a.bcells = bcells;
      if (d.fsi_pressure) {
        a.up = up_;
        a.px0 = px0;
        a.py0 = py0;
        a.pz0 = pz0;
        a.pnx = pnx;
        a.pny = pny;
        a.pnz = pnz;
        a.pcells = pcells;
      }
    }
    if (static_on) {
      a.st_chi = st_chi_;
      a.st_us = st_us_;
      a.st_w = st_w_;
    }
    a.inv_eta = (T)(1.0 / d.eta);
    return a;
  }

  // Total pressure of the current velocity with the current wing's mask,
  // without a step: the nonlinear term's passes (mask, z/y inverse, fused x
  // pass, y forward) and a z forward that keeps only Pi_hat = -i k.N'/|k|^2.
  // The state (u_hat, N_hat history, dt, diagnostics) is unchanged.
  fsi_status eval_pressure() override {
    if (!d.fsi_pressure) {
      err = "FSI mode (fsi_pressure) is off";
      return FSI_ESTATE;
    }
    if (wing_nt == 0 || bcells == 0) {
      err = "no wing";
      return FSI_ESTATE;
    }
    FSI_TRY(run_mask(s));
    if (!zs_valid) {
      ColArgs<T> a = col_base(pz, twz, nz, Kz, C1, C1);
      a.in = uh;
      a.in_fs = clen;
      a.out = A;
      a.out_fs = Alen;
      FSI_HIP(launch_col<T>(COL_INV_CURL5, a, 1, s));
    }
    zs_valid = false;  // P4 below overwrites fields 0-2 of A
    {
      ColArgs<T> a = col_base(py, twy, ny, Ky, kx1, kxp);
      a.in = A;
      a.in_fs = Alen;
      a.in_bs = C1;
      a.out = B;
      a.out_fs = Blen;
      a.out_bs = (long long)ny * kxp;
      FSI_HIP(launch_col<T>(COL_INV_WZ, a, nz, s));
    }
    FSI_HIP(launch_xfused<T>(p3_args(), nfused, s));  // partials written, not reduced
    {
      ColArgs<T> a = col_base(py, twy, ny, Ky, kx1, kxp);
      a.in = B;
      a.in_fs = Blen;
      a.in_bs = (long long)ny * kxp;
      a.out = A;
      a.out_fs = Alen;
      a.out_bs = C1;
      a.nf = 3;
      a.scale = (T)1;
      FSI_HIP(launch_col<T>(COL_FWD_PLAIN, a, nz, s));
    }
    {
      ColArgs<T> a = col_base(pz, twz, nz, Kz, C1, C1);
      a.in = A;
      a.in_fs = Alen;
      a.out = nullptr;  // projection computed, only Pi_hat stored
      a.cfs = clen;
      a.nf = 3;
      a.scale = (T)(1.0 / (double)npts);
      a.pi = pi_;
      FSI_HIP(launch_col<T>(COL_FWD_PROJECT, a, 1, s));
    }
    p_ready = true;
    return FSI_OK;
  }

  fsi_status step_info(double F[3], double* dt, double* E, double* umax, double* t, long long* ns) override {
    if (info_pending) FSI_HIP(hipEventSynchronize(info_ev));
    else FSI_HIP(hipStreamSynchronize(s));
    if (F) {
      F[0] = sc_host->info[0];
      F[1] = sc_host->info[1];
      F[2] = sc_host->info[2];
    }
    if (E) *E = sc_host->info[3];
    if (umax) *umax = sc_host->info[4];
    if (dt) *dt = sc_host->info[5];
    if (t) *t = sc_host->t;
    if (ns) *ns = nstep;
    if (sc_host->info[6] != 0.0) {
      err = "non-finite value met during a step";
      return FSI_ENAN;
    }
    return FSI_OK;
  }

  // -- stand-alone transforms ---------------------------------------------------
  fsi_status fft_r2c(const double* f, double* fh) override {
    FSI_TRY(ensure_phys());
    FSI_TRY(ensure_cwork());
    FSI_TRY(upload_real(f, phys, npts));
    FSI_TRY(run_forward(phys, 1, cwork, COL_FWD_PLAIN));
    std::vector<cpx<T>> h(clen);
    FSI_HIP(hipMemcpyAsync(h.data(), cwork, sizeof(cpx<T>) * clen, hipMemcpyDeviceToHost, s));
    FSI_HIP(hipStreamSynchronize(s));
    unpad(h.data(), fh);
    return FSI_OK;
  }

  fsi_status fft_c2r(const double* fh, double* f) override {
    FSI_TRY(ensure_phys());
    FSI_TRY(ensure_cwork());
    std::vector<cpx<T>> h(clen);
    memset(h.data(), 0, sizeof(cpx<T>) * clen);
    pad(fh, h.data());
    FSI_HIP(hipMemcpyAsync(cwork, h.data(), sizeof(cpx<T>) * clen, hipMemcpyHostToDevice, s));
    FSI_TRY(run_inverse(cwork, clen, 1, phys));
    return download_real(phys, f, npts);
  }

  // -- state slots ---------------------------------------------------------------
  fsi_status save_state(int slot) override {
    if (slot < 0 || slot >= (int)slots.size()) {
      err = "slot out of range";
      return FSI_EINVAL;
    }
    Slot& sl = slots[slot];
    if (!sl.uh) {
      FSI_TRY(alloc(&sl.uh, 3 * clen));
      FSI_TRY(alloc(&sl.nh, 3 * clen));
      FSI_TRY(alloc(&sl.sc, 1));
    }
    FSI_HIP(hipMemcpyAsync(sl.uh, uh, sizeof(cpx<T>) * 3 * clen, hipMemcpyDeviceToDevice, s));
    FSI_HIP(hipMemcpyAsync(sl.nh, nh, sizeof(cpx<T>) * 3 * clen, hipMemcpyDeviceToDevice, s));
    FSI_HIP(hipMemcpyAsync(sl.sc, sc, sizeof(DevScalars), hipMemcpyDeviceToDevice, s));
    sl.nstep = nstep;
    sl.have_prev = have_prev;
    sl.used = true;
    sl.tape_only = false;
    sl.bt_valid = false;
    return FSI_OK;
  }

  // A tape entry for the reverse step: only u_hat (the reverse step re-derives
  // u and omega from it; the Adams-Bashforth history is not needed there)
  fsi_status save_tape(int slot) override {
    if (slot < 0 || slot >= (int)slots.size()) {
      err = "slot out of range";
      return FSI_EINVAL;
    }
    Slot& sl = slots[slot];
    if (!sl.uh) {
      FSI_TRY(alloc(&sl.uh, 3 * clen));
      FSI_TRY(alloc(&sl.nh, 3 * clen));
      FSI_TRY(alloc(&sl.sc, 1));
    }
    FSI_HIP(hipMemcpyAsync(sl.uh, uh, sizeof(cpx<T>) * 3 * clen, hipMemcpyDeviceToDevice, s));
    sl.nstep = nstep;
    sl.have_prev = have_prev;
    sl.used = true;
    sl.tape_only = true;
    sl.bt_valid = false;
    return FSI_OK;
  }

  // Forward step with its tape.  Without the sponge the step's y-inverse pass
  // writes u and omega (x spectral, y and z physical: 6 fields of the B layout)
  // straight into the slot and the fused x pass reads them there, so the tape
  // costs no copy and the reverse step skips re-deriving u and omega (one
  // z-inverse and six y-inverse transforms).  With the sponge (its x pass
  // works in place on omega), or if the slot's 6 fields cannot be allocated,
  // the tape is u_hat (save_tape).
  fsi_status step_record(double dt, int slot) override {
    if (slot < 0 || slot >= (int)slots.size()) {
      err = "slot out of range";
      return FSI_EINVAL;
    }
    Slot& sl = slots[slot];
    if (!sponge_on && !sl.bt) {
      void* q = nullptr;
      if (hipMalloc(&q, sizeof(cpx<T>) * 6 * (size_t)Blen) == hipSuccess) sl.bt = (cpx<T>*)q;
      else (void)hipGetLastError();
    }
    if (sponge_on || !sl.bt) {
      FSI_TRY(save_tape(slot));
      return step(false, dt, 0.0, 0.0, 0.0);
    }
    sl.used = false;  // until the step has written it
    rec_bt = sl.bt;
    const fsi_status st = step(false, dt, 0.0, 0.0, 0.0);
    rec_bt = nullptr;
    if (st != FSI_OK) return st;
    sl.used = true;
    sl.tape_only = true;
    sl.bt_valid = true;
    sl.nstep = nstep - 1;
    return FSI_OK;
  }

  fsi_status load_state(int slot) override {
    if (slot < 0 || slot >= (int)slots.size()) {
      err = "slot out of range";
      return FSI_EINVAL;
    }
    Slot& sl = slots[slot];
    if (!sl.used) {
      err = "slot is empty";
      return FSI_ESTATE;
    }
    if (sl.tape_only) {
      err = "slot holds a tape entry of fsi_step_record (velocity only), not a full state";
      return FSI_ESTATE;
    }
    FSI_HIP(hipMemcpyAsync(uh, sl.uh, sizeof(cpx<T>) * 3 * clen, hipMemcpyDeviceToDevice, s));
    zs_valid = false;
    FSI_HIP(hipMemcpyAsync(nh, sl.nh, sizeof(cpx<T>) * 3 * clen, hipMemcpyDeviceToDevice, s));
    FSI_HIP(hipMemcpyAsync(sc, sl.sc, sizeof(DevScalars), hipMemcpyDeviceToDevice, s));
    FSI_HIP(hipMemcpyAsync(sc_host, sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
    info_pending = false;
    nstep = sl.nstep;
    have_prev = sl.have_prev;
    p_ready = false;
    return FSI_OK;
  }

  // -- adjoint of one step (dt held fixed) -----------------------------------------
  fsi_status ensure_adjoint() {
    if (!lu_) {
      FSI_TRY(alloc(&lu_, 3 * clen));
      FSI_TRY(alloc(&lnp_, 3 * clen));
      FSI_TRY(alloc(&A9, 9 * Alen));
      FSI_TRY(alloc(&B9, 9 * Blen));
      FSI_HIP(hipMemsetAsync(lu_, 0, sizeof(cpx<T>) * 3 * clen, s));
      FSI_HIP(hipMemsetAsync(lnp_, 0, sizeof(cpx<T>) * 3 * clen, s));
    }
    return FSI_OK;
  }

  fsi_status adjoint_set(const double* lu, const double* lnp) override {
    FSI_TRY(ensure_adjoint());
    std::vector<cpx<T>> h;
    for (int which = 0; which < 2; ++which) {
      const double* src = which == 0 ? lu : lnp;
      cpx<T>* dst = which == 0 ? lu_ : lnp_;
      if (!src) {  // a null cotangent is zero: clear on the device
        FSI_HIP(hipMemsetAsync(dst, 0, sizeof(cpx<T>) * 3 * clen, s));
        continue;
      }
      h.assign(3 * clen, cpx<T>{});
      for (int q = 0; q < 3; ++q) pad(src + 2 * q * clen_ext, h.data() + q * clen);
      FSI_HIP(hipMemcpyAsync(dst, h.data(), sizeof(cpx<T>) * 3 * clen, hipMemcpyHostToDevice, s));
      FSI_HIP(hipStreamSynchronize(s));
    }
    FSI_HIP(hipStreamSynchronize(s));
    return FSI_OK;
  }

  fsi_status adjoint_get(double* lu, double* lnp) override {
    FSI_TRY(ensure_adjoint());
    std::vector<cpx<T>> h(3 * clen);
    for (int which = 0; which < 2; ++which) {
      double* dst = which == 0 ? lu : lnp;
      if (!dst) continue;
      FSI_HIP(hipMemcpyAsync(h.data(), which == 0 ? lu_ : lnp_, sizeof(cpx<T>) * 3 * clen, hipMemcpyDeviceToHost, s));
      FSI_HIP(hipStreamSynchronize(s));
      for (int q = 0; q < 3; ++q) unpad(h.data() + q * clen, dst + 2 * q * clen_ext);
    }
    return FSI_OK;
  }

  // Sponge share of the reverse step: S = chi_sp omega, so lambda_omega gains
  // chi_sp C2R(nu) (nu from COL_ADJ_MU), which reaches lambda_u through the
  // transposed curl as the nonlinear term's lambda_omega does: z and y
  // inverse of nu, x C2R, mask, x R2C, y forward, z forward accumulating
  // m_k i k x (.) into lambda_u.  A9, B9 and phys are free at this point.
  fsi_status sponge_adjoint() {
    {
      ColArgs<T> a = col_base(pz, twz, nz, Kz, C1, C1);
      a.in = spadj_;
      a.in_fs = clen;
      a.out = A9;
      a.out_fs = Alen;
      a.nf = 3;
      FSI_HIP(launch_col<T>(COL_INV_PLAIN, a, 1, s));
    }
    {
      ColArgs<T> a = col_base(py, twy, ny, Ky, kx1, kxp);
      a.in = A9;
      a.in_fs = Alen;
      a.in_bs = C1;
      a.out = B9;
      a.out_fs = Blen;
      a.out_bs = (long long)ny * kxp;
      a.nf = 3;
      FSI_HIP(launch_col<T>(COL_INV_PLAIN, a, nz, s));
    }
    {
      XArgs<T> a = x_base();
      a.spec = B9;
      a.sfs = Blen;
      a.phys = phys;
      a.pfs = npts;
      FSI_HIP(launch_xplain<T>(X_C2R, 3, a, npart, s));
      SpongeArgs<T> m;
      m.phys = phys;
      m.npts = npts;
      m.nx = nx;
      m.ny = ny;
      m.nz = nz;
      m.g = spg_;
      FSI_HIP(launch_sponge_mask<T>(m, s));
      FSI_HIP(launch_xplain<T>(X_R2C, 3, a, npart, s));
    }
    {
      ColArgs<T> a = col_base(py, twy, ny, Ky, kx1, kxp);
      a.in = B9;
      a.in_fs = Blen;
      a.in_bs = (long long)ny * kxp;
      a.out = A9;
      a.out_fs = Alen;
      a.out_bs = C1;
      a.nf = 3;
      a.scale = (T)1;
      FSI_HIP(launch_col<T>(COL_FWD_PLAIN, a, nz, s));
    }
    {
      ColArgs<T> a = col_base(pz, twz, nz, Kz, C1, C1);
      a.in = A9;
      a.in_fs = Alen;
      a.out = lu_;
      a.cfs = clen;
      a.scale = (T)1;
      FSI_HIP(launch_col<T>(COL_FWD_ACC_CURL, a, 1, s));
    }
    return FSI_OK;
  }

  fsi_status step_adjoint(int slot, double dt, double dtp, int first, const double dJdF[3], double* dJdx,
                          double* dJdv) override {
    if (slot < 0 || slot >= (int)slots.size() || !slots[slot].used) {
      err = "tape slot is empty";
      return FSI_ESTATE;
    }
    if (!(dt > 0) || (!first && !(dtp > 0))) {
      err = "dt and (unless first) dt_prev must be positive";
      return FSI_EINVAL;
    }
    if (!xadj_supported<T>(nx)) {
      err = "nx too long for the adjoint x pass in this precision";
      return FSI_EINVAL;
    }
    if (static_on) {
      err = "the reverse step does not include the static penalization (fsi_set_static_mask)";
      return FSI_ESTATE;
    }
    FSI_TRY(ensure_adjoint());
    const bool wing = wing_nt > 0 && bcells > 0;
    if (wing) {
      if (adj_box_cap < box_cap) {
        FSI_HIP(hipStreamSynchronize(s));
        free_dev(lchi_);
        free_dev(lus_);
        adj_box_cap = box_cap;
        FSI_TRY(alloc(&lchi_, adj_box_cap));
        FSI_TRY(alloc(&lus_, 3 * adj_box_cap));
      }
      if (tgrad_cap < wing_nt) {
        FSI_HIP(hipStreamSynchronize(s));
        free_dev(tgrad_);
        tgrad_cap = wing_nt;
        FSI_TRY(alloc(&tgrad_, 18LL * tgrad_cap));
      }
      FSI_TRY(run_mask(s));
    }
    // pressure seed: lambda_Pi on the grid (zero outside the box), its normalized R2C
    const bool seed = seed_pending && d.fsi_pressure && wing && pcells > 0;
    if (seed) {
      if (!phys) FSI_TRY(alloc(&phys, 3 * npts));
      if (!piadj_) FSI_TRY(alloc(&piadj_, clen));
      FSI_HIP(hipMemsetAsync(phys, 0, sizeof(T) * npts, s));
      BoxArgs<T> b = box_args();
      b.in = lp_;
      b.grid = phys;
      FSI_HIP(launch_pbox<T>(1, b, s));
      FSI_TRY(run_forward(phys, 1, piadj_, COL_FWD_PLAIN));
    }
    seed_pending = false;
    // inverse transforms: u, omega of the taped state, and the update and
    // projection transposes with mu = P(lambda_N)/(m_k N^3) followed by
    // lambda_G = C2R(mu) in one pass (z inverse of mu from registers)
    const bool taped = slots[slot].bt_valid;  // u, omega recorded by the forward step
    {
      if (!taped) {
        ColArgs<T> a = col_base(pz, twz, nz, Kz, C1, C1);
        a.in = slots[slot].uh;
        a.in_fs = clen;
        a.out = A9;
        a.out_fs = Alen;
        FSI_HIP(launch_col<T>(COL_INV_CURL, a, 1, s));
      }
      ColArgs<T> m = col_base(pz, twz, nz, Kz, C1, C1);
      m.uh = lu_;
      m.nh = lnp_;
      m.cfs = clen;
      m.nu = (T)d.nu;
      m.adt = dt;
      m.adtp = first ? dt : dtp;
      m.first = first ? 1 : 0;
      m.invN3 = 1.0 / (double)npts;
      m.lpi = seed ? piadj_ : nullptr;
      if (sponge_on) {
        // every band row of a valid column is written (padding columns are
        // zeroed by the inverse pass that reads nu)
        if (!spadj_) FSI_TRY(alloc(&spadj_, 3 * clen));
        m.spadj = spadj_;
        m.csp_inv = (T)(1.0 / csp);
      }
      m.out = A9 + 6 * Alen;
      m.out_fs = Alen;
      FSI_HIP(launch_col<T>(COL_ADJ_MU, m, 1, s));
    }
    {
      // y inverse of u, omega and lambda_G (9 fields), or of lambda_G alone
      // when u, omega come from the tape
      ColArgs<T> a = col_base(py, twy, ny, Ky, kx1, kxp);
      a.in = taped ? A9 + 6 * Alen : A9;
      a.in_fs = Alen;
      a.in_bs = C1;
      a.out = taped ? B9 + 6 * Blen : B9;
      a.out_fs = Blen;
      a.out_bs = (long long)ny * kxp;
      a.nf = taped ? 3 : 9;
      FSI_HIP(launch_col<T>(COL_INV_PLAIN, a, nz, s));
    }
    {
      XAdjArgs<T> a;
      memset(&a, 0, sizeof(a));
      a.spec = B9;
      a.utape = taped ? slots[slot].bt : nullptr;
      a.sfs = Blen;
      a.ld = kxp;
      a.nlines = ny * nz;
      a.ny = ny;
      a.n = nx;
      a.kx1 = kx1;
      a.plan = px;
      a.tw = twx;
      if (wing) {
        a.chi = chi;
        a.us = us;
        a.lchi = lchi_;
        a.lus = lus_;
        a.bx0 = bx0;
        a.by0 = by0;
        a.bz0 = bz0;
        a.bnx = bnx;
        a.bny = bny;
        a.bnz = bnz;
        a.bcells = bcells;
      }
      if (seed) {
        a.lp = lp_;
        a.px0 = px0;
        a.py0 = py0;
        a.pz0 = pz0;
        a.pnx = pnx;
        a.pny = pny;
        a.pnz = pnz;
        a.pcells = pcells;
      }
      a.inv_eta = (T)(1.0 / d.eta);
      a.g0 = (T)(dV * dJdF[0]);
      a.g1 = (T)(dV * dJdF[1]);
      a.g2 = (T)(dV * dJdF[2]);
      const int grid = (int)std::max(1LL, std::min(((long long)ny * nz) / 2, 4096LL));
      FSI_HIP(launch_xadj<T>(a, grid, s));
    }
    {
      ColArgs<T> a = col_base(py, twy, ny, Ky, kx1, kxp);
      a.in = B9;
      a.in_fs = Blen;
      a.in_bs = (long long)ny * kxp;
      a.out = A9;
      a.out_fs = Alen;
      a.out_bs = C1;
      a.nf = 6;
      a.scale = (T)1;
      FSI_HIP(launch_col<T>(COL_FWD_PLAIN, a, nz, s));
    }
    {
      // C2R^T = N^3 m_k R2C_normalized = m_k R2C_unnormalized
      ColArgs<T> a = col_base(pz, twz, nz, Kz, C1, C1);
      a.in = A9;
      a.in_fs = Alen;
      a.out = lu_;
      a.cfs = clen;
      a.nf = 3;
      a.scale = (T)1;
      FSI_HIP(launch_col<T>(COL_FWD_ACC, a, 1, s));
      a.in = A9 + 3 * Alen;
      FSI_HIP(launch_col<T>(COL_FWD_ACC_CURL, a, 1, s));
    }
    if (sponge_on) FSI_TRY(sponge_adjoint());
    if (dJdx) memset(dJdx, 0, sizeof(double) * 3 * wing_nv);
    if (dJdv) memset(dJdv, 0, sizeof(double) * 3 * wing_nv);
    if (wing) {
      MaskAdjArgs<T> m;
      memset(&m, 0, sizeof(m));
      m.x = dx_;
      m.v = dv_;
      m.tri = dtri_;
      m.nt = wing_nt;
      m.key2 = key2;
      m.chi = chi;
      m.lchi = lchi_;
      m.lus = lus_;
      m.bx0 = bx0;
      m.by0 = by0;
      m.bz0 = bz0;
      m.bnx = bnx;
      m.bny = bny;
      m.bnz = bnz;
      m.bcells = bcells;
      m.dx = dxs[0];
      m.dy = dxs[1];
      m.dz = dxs[2];
      m.rsup = rsup;
      m.tw = d.tw;
      m.h = d.h;
      m.profile = d.mask_profile;
      m.tgrad = tgrad_;
      FSI_HIP(launch_mask_adj<T>(m, s));
      std::vector<double> tg(18LL * wing_nt);
      FSI_HIP(hipMemcpyAsync(tg.data(), tgrad_, sizeof(double) * 18 * wing_nt, hipMemcpyDeviceToHost, s));
      FSI_HIP(hipStreamSynchronize(s));
      for (int t = 0; t < wing_nt; ++t)
        for (int j = 0; j < 3; ++j) {
          const int vtx = tri_host[3 * t + j];
          for (int c = 0; c < 3; ++c) {
            if (dJdx) dJdx[3 * vtx + c] += tg[18LL * t + 3 * j + c];
            if (dJdv) dJdv[3 * vtx + c] += tg[18LL * t + 9 + 3 * j + c];
          }
        }
    } else {
      FSI_HIP(hipStreamSynchronize(s));
    }
    return FSI_OK;
  }

  fsi_status synchronize() override {
    FSI_HIP(hipStreamSynchronize(s));
    return FSI_OK;
  }

  fsi_status set_timing(unsigned mask) override {
    FSI_TRY(sync_both());
    tmask = mask & ((1u << FSI_NPASS) - 1);
    timing = tmask != 0;
    for (int e = 0; e < EV_COUNT; ++e) ev_need[e] = false;
    for (int p = 0; p < FSI_NPASS; ++p)
      if (tmask & (1u << p)) ev_need[kSpan[p][0]] = ev_need[kSpan[p][1]] = true;
    ev_used = 0;
    const bool on = timing;
    // the events of the next kEvPool steps are created here, not inside the
    // steps being timed
    while (on && (int)events.size() < kEvPool) {
      std::array<hipEvent_t, EV_COUNT> e;
      for (auto& h : e) FSI_HIP(hipEventCreate(&h));
      events.push_back(e);
    }
    return FSI_OK;
  }

  // every buffer whose rows have the padded pitch kxp: spectral state and
  // its nonlinear term, the z- and y-slab work fields, the helper transform
  // field, the pressure and sponge spectra, the tapes of the state slots
  fsi_status poison_padding(double v) override {
    FSI_TRY(sync_both());
    const T t = (T)v;
    FSI_HIP(launch_fill_pad<T>(uh, 3 * clen / kxp, kx1, kxp, t, s));
    FSI_HIP(launch_fill_pad<T>(nh, 3 * clen / kxp, kx1, kxp, t, s));
    FSI_HIP(launch_fill_pad<T>(A, 6 * Alen / kxp, kx1, kxp, t, s));
    FSI_HIP(launch_fill_pad<T>(B, 6 * Blen / kxp, kx1, kxp, t, s));
    FSI_HIP(launch_fill_pad<T>(cwork, clen / kxp, kx1, kxp, t, s));
    FSI_HIP(launch_fill_pad<T>(pi_, clen / kxp, kx1, kxp, t, s));
    FSI_HIP(launch_fill_pad<T>(tsp_, 3 * clen / kxp, kx1, kxp, t, s));
    FSI_HIP(launch_fill_pad<T>(spadj_, 3 * clen / kxp, kx1, kxp, t, s));
    FSI_HIP(hipStreamSynchronize(s));
    return FSI_OK;
  }

  fsi_status pass_times(double ms[FSI_NPASS], int* nsteps) override {
    FSI_HIP(hipStreamSynchronize(s));
    if (s2) FSI_HIP(hipStreamSynchronize(s2));
    for (int p = 0; p < FSI_NPASS; ++p) ms[p] = 0.0;
    for (int k = 0; k < ev_used; ++k) {
      for (int p = 0; p < FSI_NPASS; ++p) {
        if (!(tmask & (1u << p))) continue;
        float e = 0.f;
        FSI_HIP(hipEventElapsedTime(&e, events[k][kSpan[p][0]], events[k][kSpan[p][1]]));
        ms[p] += e;
      }
    }
    if (nsteps) *nsteps = ev_used;
    ev_used = 0;
    return FSI_OK;
  }

 private:
  struct Slot {
    cpx<T>* uh = nullptr;
    cpx<T>* nh = nullptr;
    DevScalars* sc = nullptr;
    long long nstep = 0;
    bool have_prev = false;
    bool used = false;
    bool tape_only = false;  // u_hat only (fsi_step_record)
    cpx<T>* bt = nullptr;    // u, omega of a recorded step, 6 fields of the B layout
    bool bt_valid = false;   // bt holds the tape (else uh does)
  };

  template <typename P>
  fsi_status alloc(P** p, long long count) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, sizeof(P) * (size_t)std::max(count, 1LL));
    if (e != hipSuccess) {
      err = std::string("device allocation failed: ") + hipGetErrorString(e);
      return FSI_ENOMEM;
    }
    *p = (P*)q;
    return FSI_OK;
  }

  template <typename P>
  void free_dev(P*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
  }

  void release() {
    if (s || uh) (void)hipStreamSynchronize(s);
    if (s2) {
      (void)hipStreamSynchronize(s2);
      (void)hipStreamDestroy(s2);
      s2 = nullptr;
    }
    for (hipEvent_t* e : {&e_ready, &e_mask, &e_x, &e_fin, &e_up}) {
      if (*e) (void)hipEventDestroy(*e);
      *e = nullptr;
    }
    free_dev(uh);
    free_dev(nh);
    free_dev(A);
    free_dev(B);
    free_dev(partials);
    free_dev(sc);
    free_dev(twx);
    free_dev(twy);
    free_dev(twz);
    free_dev(phys);
    free_dev(cwork);
    free_dev(spg_);
    free_dev(tsp_);
    free_dev(spadj_);
    free_dev(dmesh_);
    free_dev(st_chi_);
    free_dev(st_us_);
    free_dev(st_w_);
    dx_ = dv_ = nullptr;
    dtri_ = nullptr;
    free_dev(key1);
    free_dev(key2);
    free_dev(lu_);
    free_dev(lnp_);
    free_dev(A9);
    free_dev(B9);
    free_dev(lchi_);
    free_dev(lus_);
    free_dev(tgrad_);
    free_dev(chi);
    free_dev(us);
    free_dev(pi_);
    free_dev(up_);
    free_dev(dsamp_);
    free_dev(dpout_);
    free_dev(dpbox_);
    free_dev(lp_);
    free_dev(piadj_);
    for (Slot& sl : slots) {
      free_dev(sl.uh);
      free_dev(sl.nh);
      free_dev(sl.sc);
      free_dev(sl.bt);
    }
    if (sc_host) (void)hipHostFree(sc_host);
    sc_host = nullptr;
    if (stage) (void)hipHostFree(stage);
    stage = nullptr;
    if (stage_ev) (void)hipEventDestroy(stage_ev);
    stage_ev = nullptr;
    if (info_ev) (void)hipEventDestroy(info_ev);
    info_ev = nullptr;
    for (auto& e : events)
      for (hipEvent_t h : e) (void)hipEventDestroy(h);
    events.clear();
  }

  fsi_status make_twiddles(int n, cpx<T>** out) {
    std::vector<cpx<T>> h(n);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int k = 0; k < n; ++k) {
      const long double ang = -2.0L * pi * (long double)k / (long double)n;
      h[k].re = (T)cosl(ang);
      h[k].im = (T)sinl(ang);
    }
    FSI_TRY(alloc(out, n));
    FSI_HIP(hipMemcpy(*out, h.data(), sizeof(cpx<T>) * n, hipMemcpyHostToDevice));
    return FSI_OK;
  }

  fsi_status reset_scalars() {
    // a step's read-back into sc_host may still be in flight
    FSI_HIP(hipStreamSynchronize(s));
    info_pending = false;
    DevScalars z;
    memset(&z, 0, sizeof(z));
    *sc_host = z;
    FSI_HIP(hipMemcpyAsync(sc, sc_host, sizeof(DevScalars), hipMemcpyHostToDevice, s));
    FSI_HIP(hipStreamSynchronize(s));
    return FSI_OK;
  }

  // packed [iz][iy][kx1] interleaved doubles -> padded [iz][iy][kxp]
  void pad(const double* in, cpx<T>* h) const {
    for (long long r = 0; r < (long long)nbz * nby; ++r)
      for (int ix = 0; ix < kx1; ++ix) {
        const long long e = r * kx1 + ix;
        h[r * kxp + ix].re = (T)in[2 * e];
        h[r * kxp + ix].im = (T)in[2 * e + 1];
      }
  }

  // padded [iz][iy][kxp] -> packed [iz][iy][kx1] interleaved doubles
  void unpad(const cpx<T>* h, double* out) const {
    for (long long r = 0; r < (long long)nbz * nby; ++r)
      for (int ix = 0; ix < kx1; ++ix) {
        const long long e = r * kx1 + ix;
        out[2 * e] = (double)h[r * kxp + ix].re;
        out[2 * e + 1] = (double)h[r * kxp + ix].im;
      }
  }

  fsi_status ensure_phys() {
    if (!phys) FSI_TRY(alloc(&phys, 3 * npts));
    return FSI_OK;
  }
  fsi_status ensure_cwork() {
    if (!cwork) FSI_TRY(alloc(&cwork, clen));
    return FSI_OK;
  }

  fsi_status upload_real(const double* h, T* dptr, long long count) {
    if (sizeof(T) == sizeof(double)) {
      FSI_HIP(hipMemcpyAsync(dptr, h, sizeof(double) * count, hipMemcpyHostToDevice, s));
      FSI_HIP(hipStreamSynchronize(s));
      return FSI_OK;
    }
    std::vector<T> tmp(count);
    for (long long i = 0; i < count; ++i) tmp[i] = (T)h[i];
    FSI_HIP(hipMemcpyAsync(dptr, tmp.data(), sizeof(T) * count, hipMemcpyHostToDevice, s));
    FSI_HIP(hipStreamSynchronize(s));
    return FSI_OK;
  }

  fsi_status download_real(const T* dptr, double* h, long long count) {
    if (sizeof(T) == sizeof(double)) {
      FSI_HIP(hipMemcpyAsync(h, dptr, sizeof(double) * count, hipMemcpyDeviceToHost, s));
      FSI_HIP(hipStreamSynchronize(s));
      return FSI_OK;
    }
    std::vector<T> tmp(count);
    FSI_HIP(hipMemcpyAsync(tmp.data(), dptr, sizeof(T) * count, hipMemcpyDeviceToHost, s));
    FSI_HIP(hipStreamSynchronize(s));
    for (long long i = 0; i < count; ++i) h[i] = (double)tmp[i];
    return FSI_OK;
  }

  // C: columns to transform; ld: row pitch (both in complex elements)
  ColArgs<T> col_base(const FftPlan& p, const cpx<T>* tw, int n, int K, long long C, long long ld) {
    ColArgs<T> a;
    memset(&a, 0, sizeof(a));
    a.C = (int)C;
    a.ld = (int)ld;
    a.kxp = kxp;
    a.n = n;
    a.K = K;
    a.nf = 1;
    a.plan = p;
    a.tw = tw;
    a.kx1 = kx1;
    a.Ky = Ky;
    a.kfx = (T)(2.0 * M_PI / d.lx);
    a.kfy = (T)(2.0 * M_PI / d.ly);
    a.kfz = (T)(2.0 * M_PI / d.lz);
    a.scale = (T)1;
    return a;
  }

  XArgs<T> x_base() {
    XArgs<T> a;
    memset(&a, 0, sizeof(a));
    a.nlines = ny * nz;
    a.ny = ny;
    a.n = nx;
    a.kx1 = kx1;
    a.ld = kxp;
    a.plan = px;
    a.tw = twx;
    return a;
  }

  // z-slab work fields of the helper transforms: a single field uses the sixth
  // field of A, which leaves the z inverse kept for the next step (fields 0-4) intact
  cpx<T>* zwork(int nf) {
    if (nf == 1) return A + 5 * Alen;
    zs_valid = false;
    return A;
  }

  // compact (nf fields, stride cstride) -> physical (nf fields)
  fsi_status run_inverse(const cpx<T>* comp, long long cstride, int nf, T* out) {
    cpx<T>* Aw = zwork(nf);
    {
      ColArgs<T> a = col_base(pz, twz, nz, Kz, C1, C1);
      a.in = comp;
      a.in_fs = cstride;
      a.out = Aw;
      a.out_fs = Alen;
      a.nf = nf;
      FSI_HIP(launch_col<T>(COL_INV_PLAIN, a, 1, s));
    }
    {
      ColArgs<T> a = col_base(py, twy, ny, Ky, kx1, kxp);
      a.in = Aw;
      a.in_fs = Alen;
      a.in_bs = C1;
      a.out = B;
      a.out_fs = Blen;
      a.out_bs = (long long)ny * kxp;
      a.nf = nf;
      FSI_HIP(launch_col<T>(COL_INV_PLAIN, a, nz, s));
    }
    {
      XArgs<T> a = x_base();
      a.spec = B;
      a.sfs = Blen;
      a.phys = out;
      a.pfs = npts;
      FSI_HIP(launch_xplain<T>(X_C2R, nf, a, npart, s));
    }
    return FSI_OK;
  }

  // physical (nf fields) -> compact; mode COL_FWD_PLAIN (nf = 1, into cout) or
  // COL_FWD_PROJECT (nf = 3, into cout = uh)
  fsi_status run_forward(T* in, int nf, cpx<T>* cout, int zmode) {
    cpx<T>* Aw = zwork(nf);
    {
      XArgs<T> a = x_base();
      a.spec = B;
      a.sfs = Blen;
      a.phys = in;
      a.pfs = npts;
      FSI_HIP(launch_xplain<T>(X_R2C, nf, a, npart, s));
    }
    {
      ColArgs<T> a = col_base(py, twy, ny, Ky, kx1, kxp);
      a.in = B;
      a.in_fs = Blen;
      a.in_bs = (long long)ny * kxp;
      a.out = Aw;
      a.out_fs = Alen;
      a.out_bs = C1;
      a.nf = nf;
      FSI_HIP(launch_col<T>(COL_FWD_PLAIN, a, nz, s));
    }
    {
      ColArgs<T> a = col_base(pz, twz, nz, Kz, C1, C1);
      a.in = Aw;
      a.in_fs = Alen;
      a.out = cout;
      a.out_fs = clen;
      a.cfs = clen;
      a.nf = nf;
      a.scale = (T)(1.0 / (double)npts);
      FSI_HIP(launch_col<T>(zmode, a, 1, s));
    }
    return FSI_OK;
  }

  fsi_status finish_set_velocity() {
    FSI_TRY(run_forward(phys, 3, uh, COL_FWD_PROJECT));
    FSI_HIP(hipMemsetAsync(nh, 0, sizeof(cpx<T>) * 3 * clen, s));
    nstep = 0;
    have_prev = false;
    FSI_TRY(reset_scalars());
    return FSI_OK;
  }

  // work on the context stream that reads the mesh waits for its upload
  fsi_status mesh_wait(hipStream_t st) {
    if (mesh_pending && st != s2) FSI_HIP(hipStreamWaitEvent(st, e_up, 0));
    return FSI_OK;
  }

  fsi_status sync_both() {
    FSI_HIP(hipStreamSynchronize(s));
    if (s2) FSI_HIP(hipStreamSynchronize(s2));
    return FSI_OK;
  }

  fsi_status run_mask(hipStream_t st) {
    FSI_TRY(mesh_wait(st));
    MaskArgs<T> m;
    memset(&m, 0, sizeof(m));
    m.x = dx_;
    m.v = dv_;
    m.tri = dtri_;
    m.nt = wing_nt;
    m.key1 = key1;
    m.key2 = key2;
    m.chi = chi;
    m.us = us;
    m.bx0 = bx0;
    m.by0 = by0;
    m.bz0 = bz0;
    m.bnx = bnx;
    m.bny = bny;
    m.bnz = bnz;
    m.bcells = bcells;
    m.dx = dxs[0];
    m.dy = dxs[1];
    m.dz = dxs[2];
    m.rsup = rsup;
    m.tw = d.tw;
    m.h = d.h;
    m.profile = d.mask_profile;
    FSI_HIP(launch_mask<T>(m, st));
    return FSI_OK;
  }

  // Side stream of the step (non-blocking, default priority) and the events
  // that order it against the context stream.
  fsi_status ensure_side() {
    if (s2) return FSI_OK;
    FSI_HIP(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
    for (hipEvent_t* e : {&e_ready, &e_mask, &e_x, &e_fin, &e_up})
      FSI_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
    return FSI_OK;
  }

  fsi_status nan_status() {
    if (sc_host && sc_host->info[6] != 0.0) {
      err = "non-finite value met during a step";
      return FSI_ENAN;
    }
    return FSI_OK;
  }

  static constexpr int kEvPool = 64;
  hipEvent_t* next_events() {
    if (ev_used >= 4096) return nullptr;
    if (ev_used == (int)events.size()) {
      std::array<hipEvent_t, EV_COUNT> e;
      for (auto& h : e)
        if (hipEventCreate(&h) != hipSuccess) return nullptr;
      events.push_back(e);
    }
    return events[ev_used++].data();
  }

  fsi_desc d;
  hipStream_t s = nullptr;
  int nx = 0, ny = 0, nz = 0, Kx = 0, Ky = 0, Kz = 0, kx1 = 0, kxp = 0, nby = 0, nbz = 0;
  long long C1 = 0, clen = 0, clen_ext = 0, Alen = 0, Blen = 0, npts = 0;
  double dxs[3] = {0, 0, 0}, dV = 0, dx_min = 0, rsup = 0;
  FftPlan px, py, pz;
  int ngroups = 0, npart = 0, nfused = 0;
  cpx<T>*twx = nullptr, *twy = nullptr, *twz = nullptr;
  cpx<T>*uh = nullptr, *nh = nullptr, *A = nullptr, *B = nullptr, *cwork = nullptr;
  bool zs_valid = false;  // A[0..4] holds the z inverse (P1) of the current u_hat
  bool sponge_on = false;
  double csp = 0.0;
  T* spg_ = nullptr;        // sponge profiles gx, gy, gz
  cpx<T>* tsp_ = nullptr;   // [3][clen] sponge term of the step
  cpx<T>* spadj_ = nullptr; // [3][clen] sponge cotangent nu of the reverse step
  T* phys = nullptr;
  double* partials = nullptr;
  DevScalars* sc = nullptr;
  DevScalars* sc_host = nullptr;
  // wing and mask sub-box
  int wing_nt = 0, wing_nv = 0;
  long long mesh_cap = 0;           // bytes of dmesh_
  unsigned char* dmesh_ = nullptr;  // x, v, tri of the current mesh (views below)
  double *dx_ = nullptr, *dv_ = nullptr;
  int* dtri_ = nullptr;
  void* stage = nullptr;
  size_t stage_cap = 0;
  hipEvent_t stage_ev = nullptr;
  hipEvent_t info_ev = nullptr;  // recorded after the step's read-back of the device scalars
  hipStream_t s2 = nullptr;      // side stream of the step (mask, reductions)
  hipEvent_t e_ready = nullptr, e_mask = nullptr, e_x = nullptr, e_fin = nullptr;
  hipEvent_t e_up = nullptr;  // mesh upload done (side stream)
  cpx<T>* rec_bt = nullptr;   // tape of the step being recorded (u, omega after P2)
  bool static_on = false;     // static penalization plane set
  T *st_chi_ = nullptr, *st_us_ = nullptr, *st_w_ = nullptr;
  bool mesh_pending = false;
  // timing events of one step
  enum { EV_MASK0, EV_MASK1, EV_P1_0, EV_P2_0, EV_P2_1, EV_P3_0, EV_P3_1, EV_RED0, EV_RED1, EV_P4_1, EV_P5_0,
         EV_P5_1, EV_COUNT };
  // (start, end) event of each pass: mask (side stream), P1, P2, P3 (+ sponge
  // x pass), reductions and dt (side stream), P4 (+ sponge z pass), P5
  static constexpr int kSpan[FSI_NPASS][2] = {{EV_MASK0, EV_MASK1}, {EV_P1_0, EV_P2_0}, {EV_P2_0, EV_P2_1},
                                              {EV_P3_0, EV_P3_1},   {EV_RED0, EV_RED1}, {EV_P3_1, EV_P4_1},
                                              {EV_P5_0, EV_P5_1}};
  unsigned tmask = 0;          // passes being timed
  bool ev_need[EV_COUNT] = {};  // events those passes need (each recorded event orders its stream)
  bool info_pending = false;
  bool stage_pending = false;
  int bx0 = 0, by0 = 0, bz0 = 0, bnx = 0, bny = 0, bnz = 0;
  long long bcells = 0, box_cap = 0;
  unsigned long long *key1 = nullptr, *key2 = nullptr;
  std::vector<int> tri_host;
  // adjoint state and work buffers (allocated on first use)
  cpx<T>*lu_ = nullptr, *lnp_ = nullptr, *A9 = nullptr, *B9 = nullptr;
  T *lchi_ = nullptr, *lus_ = nullptr;
  long long adj_box_cap = 0;
  double* tgrad_ = nullptr;
  int tgrad_cap = 0;
  T *chi = nullptr, *us = nullptr;
  // FSI mode: Pi_hat of the last step, u on the pressure box, sample points
  cpx<T>* pi_ = nullptr;
  T* up_ = nullptr;
  double *dsamp_ = nullptr, *dpout_ = nullptr;
  long long pbox_cap = 0, psamp_cap = 0, pcells = 0;
  int px0 = 0, py0 = 0, pz0 = 0, pnx = 0, pny = 0, pnz = 0;
  std::vector<double> load_cv, samp_host;
  bool p_ready = false;
  double* dpbox_ = nullptr;
  long long dpbox_cap = 0, lp_cap = 0;
  T* lp_ = nullptr;          // pressure seed on the box (adjoint)
  cpx<T>* piadj_ = nullptr;  // its normalized R2C (compact)
  bool seed_pending = false;
  // stepping
  long long nstep = 0;
  bool have_prev = false;
  std::vector<Slot> slots;
  // timing
  bool timing = false;
  int ev_used = 0;
  std::vector<std::array<hipEvent_t, EV_COUNT>> events;
};

EngineBase* make_engine_f32() { return new Engine<float>(); }
EngineBase* make_engine_f64() { return new Engine<double>(); }

}  // namespace fsi
