// loads.cpp - wing pressure loads from a pressure box and their transpose (host, FP64).
//
// Sec. 4.1 (pressure interpolation paragraph): the pressure is interpolated
// onto the mass points with a delta kernel and each triangle loads its three
// vertices along its normal with pressure x area / 3.  As in the device path
// (fsi_get_pressure_loads): c_v = (1/3) sum_{T of v} A_T n_T = (1/6) sum
// (x1 - x0) x (x2 - x0), n_v = c_v / |c_v|, dp_v = p(x_v + d n_v) -
// p(x_v - d n_v) with the 4-point kernel on the grid values of a pressure box,
// load_v = -dp_v c_v.  fsi_loads_adjoint applies the transpose of this map
// with respect to the vertex positions and the box values, for the adjoint of
// coupled rollouts.
#include <math.h>
#include <string.h>

#include <cmath>
#include <vector>

#include "../../include/fsi_ms.h"

namespace {

double phi4(double r) {
  r = fabs(r);
  if (r < 1.0) return 0.125 * (3.0 - 2.0 * r + sqrt(1.0 + 4.0 * r - 4.0 * r * r));
  if (r < 2.0) return 0.125 * (5.0 - 2.0 * r - sqrt(-7.0 + 12.0 * r - 4.0 * r * r));
  return 0.0;
}

// d phi / d r
double dphi4(double r) {
  const double s = r < 0.0 ? -1.0 : 1.0;
  r = fabs(r);
  if (r < 1.0) return s * 0.125 * (-2.0 + (2.0 - 4.0 * r) / sqrt(1.0 + 4.0 * r - 4.0 * r * r));
  if (r < 2.0) return s * 0.125 * (-2.0 - (6.0 - 4.0 * r) / sqrt(-7.0 + 12.0 * r - 4.0 * r * r));
  return 0.0;
}

struct Box {
  double dx[3];
  int o[3], n[3];
  const double* p;
  // stencil of point X: base indices (box-relative) and per-axis weights and derivatives
  bool stencil(const double X[3], int b[3], double w[3][4], double dw[3][4]) const {
    for (int q = 0; q < 3; ++q) {
      const double g = X[q] / dx[q];
      if (!std::isfinite(g)) return false;
      const int i0 = (int)floor(g) - 1;
      b[q] = i0 - o[q];
      if (b[q] < 0 || b[q] + 3 > n[q] - 1) return false;
      for (int m = 0; m < 4; ++m) {
        w[q][m] = phi4(g - (double)(i0 + m));
        dw[q][m] = dphi4(g - (double)(i0 + m)) / dx[q];
      }
    }
    return true;
  }
  long long cell(const int b[3], int a, int bb, int c) const {
    return ((long long)(b[2] + c) * n[1] + (b[1] + bb)) * n[0] + (b[0] + a);
  }
  // value and gradient of the interpolated pressure at X
  bool sample(const double X[3], double* val, double grad[3]) const {
    int b[3];
    double w[3][4], dw[3][4];
    if (!stencil(X, b, w, dw)) return false;
    double v = 0.0, g[3] = {0, 0, 0};
    for (int c = 0; c < 4; ++c)
      for (int bb = 0; bb < 4; ++bb)
        for (int a = 0; a < 4; ++a) {
          const double pc = p[cell(b, a, bb, c)];
          v += w[0][a] * w[1][bb] * w[2][c] * pc;
          g[0] += dw[0][a] * w[1][bb] * w[2][c] * pc;
          g[1] += w[0][a] * dw[1][bb] * w[2][c] * pc;
          g[2] += w[0][a] * w[1][bb] * dw[2][c] * pc;
        }
    *val = v;
    if (grad)
      for (int q = 0; q < 3; ++q) grad[q] = g[q];
    return true;
  }
  // lam_box += lam * weights of the stencil of X
  void scatter(const double X[3], double lam, double* lam_box) const {
    int b[3];
    double w[3][4], dw[3][4];
    if (!stencil(X, b, w, dw)) return;
    for (int c = 0; c < 4; ++c)
      for (int bb = 0; bb < 4; ++bb)
        for (int a = 0; a < 4; ++a) lam_box[cell(b, a, bb, c)] += lam * w[0][a] * w[1][bb] * w[2][c];
  }
};

void load_vectors(int nv, const double* x, int nt, const int* tri, std::vector<double>& c) {
  c.assign(3 * (size_t)nv, 0.0);
  for (int t = 0; t < nt; ++t) {
    const int* v = tri + 3 * t;
    double e1[3], e2[3];
    for (int q = 0; q < 3; ++q) {
      e1[q] = x[3 * v[1] + q] - x[3 * v[0] + q];
      e2[q] = x[3 * v[2] + q] - x[3 * v[0] + q];
    }
    const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    for (int k = 0; k < 3; ++k)
      for (int q = 0; q < 3; ++q) c[3 * (size_t)v[k] + q] += cr[q] / 6.0;
  }
}

fsi_status check(int nv, const double* x, int nt, const int* tri, const double* dx, const int* box0, const int* boxn,
                 const double* pbox) {
  if (nv < 1 || nt < 0 || !x || (nt > 0 && !tri) || !dx || !box0 || !boxn || !pbox) return FSI_EINVAL;
  for (int q = 0; q < 3; ++q)
    if (!(dx[q] > 0.0) || boxn[q] < 4) return FSI_EINVAL;
  for (int t = 0; t < 3 * nt; ++t)
    if (tri[t] < 0 || tri[t] >= nv) return FSI_EINVAL;
  return FSI_OK;
}

}  // namespace

extern "C" {

fsi_status fsi_loads_from_box(int32_t nv, const double* x, int32_t nt, const int32_t* tri, double d, const double* dx,
                              const int32_t* box0, const int32_t* boxn, const double* pbox, double* loads,
                              double* dp) {
  if (check(nv, x, nt, tri, dx, box0, boxn, pbox) != FSI_OK || !loads) return FSI_EINVAL;
  const Box B{{dx[0], dx[1], dx[2]}, {box0[0], box0[1], box0[2]}, {boxn[0], boxn[1], boxn[2]}, pbox};
  std::vector<double> c;
  load_vectors(nv, x, nt, tri, c);
  for (int v = 0; v < nv; ++v) {
    const double* cv = &c[3 * (size_t)v];
    const double nrm = sqrt(cv[0] * cv[0] + cv[1] * cv[1] + cv[2] * cv[2]);
    double Xp[3], Xm[3];
    for (int q = 0; q < 3; ++q) {
      const double off = nrm > 0.0 ? d * cv[q] / nrm : 0.0;
      Xp[q] = x[3 * v + q] + off;
      Xm[q] = x[3 * v + q] - off;
    }
    double pp, pm;
    if (!B.sample(Xp, &pp, nullptr) || !B.sample(Xm, &pm, nullptr)) return FSI_EBOUNDS;
    if (dp) dp[v] = pp - pm;
    for (int q = 0; q < 3; ++q) loads[3 * v + q] = -(pp - pm) * cv[q];
  }
  return FSI_OK;
}

fsi_status fsi_loads_adjoint(int32_t nv, const double* x, int32_t nt, const int32_t* tri, double d, const double* dx,
                             const int32_t* box0, const int32_t* boxn, const double* pbox, const double* lam_load,
                             double* lam_x, double* lam_pbox) {
  if (check(nv, x, nt, tri, dx, box0, boxn, pbox) != FSI_OK || !lam_load) return FSI_EINVAL;
  const Box B{{dx[0], dx[1], dx[2]}, {box0[0], box0[1], box0[2]}, {boxn[0], boxn[1], boxn[2]}, pbox};
  std::vector<double> c;
  load_vectors(nv, x, nt, tri, c);
  std::vector<double> lam_c(3 * (size_t)nv, 0.0);
  for (int v = 0; v < nv; ++v) {
    const double* cv = &c[3 * (size_t)v];
    const double* lL = lam_load + 3 * v;
    const double nrm = sqrt(cv[0] * cv[0] + cv[1] * cv[1] + cv[2] * cv[2]);
    double n[3], Xp[3], Xm[3];
    for (int q = 0; q < 3; ++q) {
      n[q] = nrm > 0.0 ? cv[q] / nrm : 0.0;
      Xp[q] = x[3 * v + q] + d * n[q];
      Xm[q] = x[3 * v + q] - d * n[q];
    }
    double pp, pm, gp[3], gm[3];
    if (!B.sample(Xp, &pp, gp) || !B.sample(Xm, &pm, gm)) return FSI_EBOUNDS;
    // load = -dp c
    const double lam_dp = -(cv[0] * lL[0] + cv[1] * lL[1] + cv[2] * lL[2]);
    for (int q = 0; q < 3; ++q) lam_c[3 * (size_t)v + q] += -(pp - pm) * lL[q];
    // dp = p(X+) - p(X-), X+- = x +- d n
    double lam_n[3];
    for (int q = 0; q < 3; ++q) {
      if (lam_x) lam_x[3 * v + q] += lam_dp * (gp[q] - gm[q]);
      lam_n[q] = d * lam_dp * (gp[q] + gm[q]);
    }
    if (lam_pbox) {
      B.scatter(Xp, lam_dp, lam_pbox);
      B.scatter(Xm, -lam_dp, lam_pbox);
    }
    // n = c / |c|:  dn = (I - n n^T) dc / |c|
    if (nrm > 0.0) {
      const double nl = n[0] * lam_n[0] + n[1] * lam_n[1] + n[2] * lam_n[2];
      for (int q = 0; q < 3; ++q) lam_c[3 * (size_t)v + q] += (lam_n[q] - n[q] * nl) / nrm;
    }
  }
  // c_v = (1/6) sum_T e1 x e2:  d(e1 x e2) = de1 x e2 + e1 x de2
  if (lam_x)
    for (int t = 0; t < nt; ++t) {
      const int* v = tri + 3 * t;
      double e1[3], e2[3], L[3] = {0, 0, 0};
      for (int q = 0; q < 3; ++q) {
        e1[q] = x[3 * v[1] + q] - x[3 * v[0] + q];
        e2[q] = x[3 * v[2] + q] - x[3 * v[0] + q];
        for (int k = 0; k < 3; ++k) L[q] += lam_c[3 * (size_t)v[k] + q] / 6.0;
      }
      const double l1[3] = {e2[1] * L[2] - e2[2] * L[1], e2[2] * L[0] - e2[0] * L[2], e2[0] * L[1] - e2[1] * L[0]};
      const double l2[3] = {L[1] * e1[2] - L[2] * e1[1], L[2] * e1[0] - L[0] * e1[2], L[0] * e1[1] - L[1] * e1[0]};
      for (int q = 0; q < 3; ++q) {
        lam_x[3 * v[1] + q] += l1[q];
        lam_x[3 * v[2] + q] += l2[q];
        lam_x[3 * v[0] + q] -= l1[q] + l2[q];
      }
    }
  return FSI_OK;
}

}  // extern "C"
