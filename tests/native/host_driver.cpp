// Exercises the host-only C ABI (include/fsi_ms.h: the FP64 mass-spring solver
// and the wing-load transpose) for an AddressSanitizer / UndefinedBehavior-
// Sanitizer build: a plate network with extension and bending springs along
// both wing axes, clamped root, BDF2 steps under loads in a rotating frame,
// the transposed step, a static solve, loads from a pressure box and their
// transpose, and the error paths.  Exit status 0 when every call behaves as
// documented; the sanitizers abort on any invalid access.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "fsi_ms.h"

#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      return 1;                                                    \
    }                                                              \
  } while (0)

static void rot_z(double a, double* F) {
  const double c = cos(a), s = sin(a);
  const double R[9] = {c, -s, 0, s, c, 0, 0, 0, 1};
  for (int i = 0; i < 9; ++i) F[i] = R[i];
}

int main() {
  const int ns = 9, nc = 5, nv = ns * nc;
  std::vector<double> x(3 * nv), v(3 * nv, 0.0), mass(nv);
  for (int j = 0; j < nc; ++j)
    for (int i = 0; i < ns; ++i) {
      const int p = j * ns + i;
      x[3 * p] = 0.3 * i;
      x[3 * p + 1] = 0.25 * j + 0.01 * sin(1.0 + p);
      x[3 * p + 2] = 0.005 * cos(2.0 * p);
      mass[p] = 0.01 * (1.0 + 0.1 * (p % 3));
    }
  fsi_ms* ms = nullptr;
  CHECK(fsi_ms_create(nv, mass.data(), &ms) == FSI_OK);
  std::vector<int> ij, ijk, axis, tri;
  std::vector<double> k, l0, kb;
  for (int j = 0; j < nc; ++j)
    for (int i = 0; i < ns; ++i) {
      const int p = j * ns + i;
      if (i + 1 < ns) { ij.push_back(p); ij.push_back(p + 1); }
      if (j + 1 < nc) { ij.push_back(p); ij.push_back(p + ns); }
      if (i + 1 < ns && j + 1 < nc) {
        ij.push_back(p); ij.push_back(p + ns + 1);
        tri.insert(tri.end(), {p, p + 1, p + ns + 1, p, p + ns + 1, p + ns});
      }
      if (i > 0 && i + 1 < ns) { ijk.insert(ijk.end(), {p - 1, p, p + 1}); axis.push_back(0); }
      if (j > 0 && j + 1 < nc) { ijk.insert(ijk.end(), {p - ns, p, p + ns}); axis.push_back(1); }
    }
  const int ne = (int)ij.size() / 2, nb = (int)ijk.size() / 3, nt = (int)tri.size() / 3;
  for (int e = 0; e < ne; ++e) {
    const int a = ij[2 * e], b = ij[2 * e + 1];
    double d2 = 0;
    for (int c = 0; c < 3; ++c) d2 += (x[3 * b + c] - x[3 * a + c]) * (x[3 * b + c] - x[3 * a + c]);
    k.push_back(50.0 + e % 7);
    l0.push_back(sqrt(d2));
  }
  for (int b = 0; b < nb; ++b) kb.push_back(0.05 + 0.01 * (b % 5));
  CHECK(fsi_ms_add_extension(ms, ne, ij.data(), k.data(), l0.data(), nullptr) == FSI_OK);
  std::vector<double> th0(2 * nb, 0.0);  // rest angles replaced by fsi_ms_set_rest below
  CHECK(fsi_ms_add_bending(ms, nb, ijk.data(), kb.data(), th0.data(), axis.data(), nullptr) == FSI_OK);
  std::vector<int> cl;
  for (int j = 0; j < nc; ++j) cl.push_back(j * ns);
  CHECK(fsi_ms_set_clamped(ms, (int)cl.size(), cl.data()) == FSI_OK);
  CHECK(fsi_ms_set_state(ms, x.data(), v.data()) == FSI_OK);
  double F[9];
  rot_z(0.0, F);
  CHECK(fsi_ms_set_rest(ms, F) == FSI_OK);
  std::vector<double> th(2 * nb), f(3 * nv), fe(3 * nv);
  double en = -1;
  CHECK(fsi_ms_bending_angles(ms, x.data(), F, th.data()) == FSI_OK);
  CHECK(fsi_ms_forces(ms, x.data(), F, f.data(), &en) == FSI_OK && en >= 0 && en < 1e-20);
  // BDF2 steps in a rotating frame with loads and a moving clamp
  double t = 0.0;
  std::vector<double> xc(3 * cl.size()), vc(3 * cl.size()), xs(3 * nv), vs(3 * nv);
  for (int n = 0; n < 6; ++n) {
    const double dt = 0.01 + 0.002 * (n % 3), t1 = t + dt, om = 2.0;
    rot_z(om * t1, F);
    for (int p = 0; p < nv; ++p) fe[3 * p + 2] = 0.02 * sin(3 * t1 + p);
    for (size_t q = 0; q < cl.size(); ++q) {
      const int p = cl[q];
      for (int r = 0; r < 3; ++r) xc[3 * q + r] = F[3 * r] * x[3 * p] + F[3 * r + 1] * x[3 * p + 1] + F[3 * r + 2] * x[3 * p + 2];
      vc[3 * q] = -om * xc[3 * q + 1];
      vc[3 * q + 1] = om * xc[3 * q];
      vc[3 * q + 2] = 0;
    }
    int it = 0;
    CHECK(fsi_ms_step(ms, dt, F, fe.data(), xc.data(), vc.data(), 1e-12, 30, &it) == FSI_OK && it >= 1);
    t = t1;
  }
  CHECK(fsi_ms_get_state(ms, xs.data(), vs.data()) == FSI_OK);
  for (double a : xs) CHECK(std::isfinite(a));
  // the transposed step with every output requested
  std::vector<double> lx(3 * nv, 0.1), lv(3 * nv, -0.05), lxn(3 * nv), lvn(3 * nv), lxp(3 * nv), lvp(3 * nv),
      lld(3 * nv), lke(ne), lkb(nb), lcx(3 * cl.size()), lcv(3 * cl.size());
  double dF[9] = {0, -1, 0, 1, 0, 0, 0, 0, 0}, ldf = 0;
  CHECK(fsi_ms_step_adjoint(ms, 0.012, 0.01, F, dF, xs.data(), lx.data(), lv.data(), lxn.data(), lvn.data(),
                            lxp.data(), lvp.data(), lld.data(), lke.data(), lkb.data(), lcx.data(), lcv.data(),
                            &ldf) == FSI_OK);
  CHECK(fsi_ms_step_adjoint(ms, 0.012, 0.0, F, nullptr, xs.data(), lx.data(), lv.data(), nullptr, nullptr, nullptr,
                            nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == FSI_OK);
  // static solve from the deformed state
  CHECK(fsi_ms_static(ms, F, fe.data(), 3, 1e-12, 40) == FSI_OK);
  // masses from areas, stiffness from EI
  std::vector<double> lm(nv);
  CHECK(fsi_ms_lumped_masses(nv, x.data(), nt, tri.data(), 1e-3, lm.data()) == FSI_OK);
  double kbv = 0;
  CHECK(fsi_ms_bending_stiffness(0.24, 0.3, 64, &kbv) == FSI_OK && kbv > 0);
  // loads from a pressure box around the wing and their transpose
  const double dx[3] = {0.1, 0.1, 0.1}, d = 0.15;
  int box0[3] = {-5, -5, -5}, boxn[3] = {40, 24, 12};
  std::vector<double> pbox((size_t)boxn[0] * boxn[1] * boxn[2]);
  for (size_t i = 0; i < pbox.size(); ++i) pbox[i] = sin(0.01 * i);
  std::vector<double> loads(3 * nv), dp(nt), lpx(3 * nv, 0.0), lpb(pbox.size(), 0.0), lam(3 * nv, 1.0);
  CHECK(fsi_loads_from_box(nv, x.data(), nt, tri.data(), d, dx, box0, boxn, pbox.data(), loads.data(), dp.data()) ==
        FSI_OK);
  CHECK(fsi_loads_adjoint(nv, x.data(), nt, tri.data(), d, dx, box0, boxn, pbox.data(), lam.data(), lpx.data(),
                          lpb.data()) == FSI_OK);
  // a box too small for the stencils is refused, not read out of bounds
  int small0[3] = {0, 0, 0}, smalln[3] = {4, 4, 4};
  CHECK(fsi_loads_from_box(nv, x.data(), nt, tri.data(), d, dx, small0, smalln, pbox.data(), loads.data(), nullptr) ==
        FSI_EBOUNDS);
  // error paths
  int bad[2] = {0, nv};
  double one = 1.0;
  CHECK(fsi_ms_add_extension(ms, 1, bad, &one, &one, nullptr) == FSI_EINVAL);
  int dup[2] = {3, 3};
  CHECK(fsi_ms_set_clamped(ms, 2, dup) == FSI_EINVAL);
  CHECK(fsi_ms_step(ms, 0.0, F, nullptr, nullptr, nullptr, 1e-12, 30, nullptr) == FSI_EINVAL);
  CHECK(fsi_ms_step(ms, 0.5, F, fe.data(), nullptr, nullptr, 1e-16, 1, nullptr) == FSI_ESTATE);
  fsi_ms* none = nullptr;
  double zero = 0.0;
  CHECK(fsi_ms_create(1, &zero, &none) == FSI_EINVAL && none == nullptr);
  CHECK(fsi_ms_destroy(ms) == FSI_OK);
  printf("host driver: ok (%d vertices, %d extension, %d bending springs, %d triangles)\n", nv, ne, nb, nt);
  return 0;
}
