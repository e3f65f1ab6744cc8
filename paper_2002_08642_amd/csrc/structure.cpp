// structure.cpp - FP64 mass-spring wing solver (host), the C ABI of include/fsi_ms.h.
//
// Sec. 2.1: the phase vector q = [x, v] obeys dq/dt = [v, (F_int + F_ext)/m];
// the variable-step BDF2 of Eq. discretized_ODEs,
//   q^{n+1} - alpha q^n + beta q^{n-1} = gamma dt f(q^{n+1}),
//   alpha = (1+xi)^2/(1+2xi), beta = xi^2/(1+2xi), gamma = (1+xi)/(1+2xi),
// is solved by Newton-Raphson from q^n.  The velocity rows are linear in
// v^{n+1}, so v^{n+1} = (x^{n+1} - b_x) / (gamma dt) (b_x = alpha x^n - beta
// x^{n-1}) is eliminated exactly and Newton runs on the positions alone:
//   r(x) = M (x - b_x) - gamma dt M b_v - (gamma dt)^2 (F_int(x) + F_ext) = 0,
//   A = M + (gamma dt)^2 H(x),   H = Hessian of the elastic energy,
// the same iterates' root as Newton on the full 6n system.  A is assembled in
// band form over the free vertices in reverse Cuthill-McKee order and solved by
// banded LU with partial pivoting.
//
// Springs (Sec. 2.2): extension E = k/2 (|x_j - x_i| - l0)^2; bending
// E = k^b/2 sum_{p in {y,z}} (theta^p - theta^p_0)^2 with theta^p the angle
// from segment a = x_j - x_i to b = x_k - x_j projected on the wing-frame
// plane (x, p) (Eq. two_bending_angles); a spring lying along wing axis
// `axis` uses the planes (axis, axis+1) and (axis, axis+2), cyclically.  The
// angle is the difference of the polar angles of the projections,
// theta = phi(b) - phi(a), which gives the gradient and Hessian in closed form.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <deque>
#include <new>
#include <string>
#include <vector>

#include "../../include/fsi_ms.h"

namespace {

struct V3 {
  double x, y, z;
};

// Band matrix (general, with room for the fill-in of partial pivoting):
// row i stores columns i - kl .. i + kl + ku.
struct Band {
  int n = 0, kl = 0, ku = 0, w = 0;
  std::vector<double> a;
  void init(int n_, int kl_, int ku_) {
    n = n_;
    kl = kl_;
    ku = ku_;
    w = 2 * kl + ku + 1;
    a.assign((size_t)n * w, 0.0);
  }
  double& operator()(int i, int j) { return a[(size_t)i * w + (j - i + kl)]; }
  // Symmetric positive definite case (kl = ku): Cholesky A = L L^T on the lower
  // band, then A x = b in place; false (matrix partly overwritten) if a pivot
  // is not positive.
  bool solve_spd(std::vector<double>& b) {
    const int bw = kl;
    // row r of the band as a pointer indexed by column: at(r)[c] = A(r, c)
    auto at = [&](int r) { return a.data() + (size_t)r * w + kl - r; };
    for (int j = 0; j < n; ++j) {
      const int k0 = std::max(0, j - bw);
      double* rj = at(j);
      double d = rj[j];
      for (int k = k0; k < j; ++k) d -= rj[k] * rj[k];
      if (!(d > 0.0) || !std::isfinite(d)) return false;
      d = sqrt(d);
      rj[j] = d;
      const int iend = std::min(n - 1, j + bw);
      for (int i = j + 1; i <= iend; ++i) {
        double* ri = at(i);
        double sum = ri[j];
        for (int k = std::max(k0, i - bw); k < j; ++k) sum -= ri[k] * rj[k];
        ri[j] = sum / d;
      }
    }
    for (int i = 0; i < n; ++i) {  // L y = b
      const double* ri = at(i);
      double sum = b[i];
      for (int k = std::max(0, i - bw); k < i; ++k) sum -= ri[k] * b[k];
      b[i] = sum / ri[i];
    }
    for (int i = n - 1; i >= 0; --i) {  // L^T x = y
      double sum = b[i];
      for (int k = i + 1; k <= std::min(n - 1, i + bw); ++k) sum -= at(k)[i] * b[k];
      b[i] = sum / at(i)[i];
    }
    return true;
  }

  // LU with partial pivoting, solving A x = b in place; false if singular.
  bool solve(std::vector<double>& b) {
    const int ue = kl + ku;  // upper bandwidth after pivoting
    for (int k = 0; k < n; ++k) {
      const int last = std::min(n - 1, k + kl);
      int p = k;
      double pv = fabs((*this)(k, k));
      for (int i = k + 1; i <= last; ++i)
        if (fabs((*this)(i, k)) > pv) {
          pv = fabs((*this)(i, k));
          p = i;
        }
      if (!(pv > 0.0) || !std::isfinite(pv)) return false;
      const int jend = std::min(n - 1, k + ue);
      if (p != k) {
        for (int j = k; j <= jend; ++j) std::swap((*this)(k, j), (*this)(p, j));
        std::swap(b[k], b[p]);
      }
      const double d = (*this)(k, k);
      for (int i = k + 1; i <= last; ++i) {
        const double l = (*this)(i, k) / d;
        if (l == 0.0) continue;
        for (int j = k + 1; j <= jend; ++j) (*this)(i, j) -= l * (*this)(k, j);
        b[i] -= l * b[k];
      }
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = b[i];
      const int jend = std::min(n - 1, i + ue);
      for (int j = i + 1; j <= jend; ++j) s -= (*this)(i, j) * b[j];
      b[i] = s / (*this)(i, i);
    }
    return true;
  }
};

}  // namespace

struct fsi_ms {
  int nv = 0;
  std::vector<double> mass;
  std::vector<int> ei, ej;
  std::vector<double> ek, el0;
  std::vector<int> bi, bj, bk, bax;
  std::vector<double> bkb, bt0;  // bt0: [nb][2]
  std::vector<int> clamped;      // in the order given
  std::vector<int> is_clamped;
  std::vector<double> x, v, xp, vp;
  double dt_prev = 0.0;
  bool have_prev = false;
  // free-vertex ordering for the band solver
  bool order_valid = false;
  std::vector<int> slot;  // vertex -> position among free vertices (RCM), -1 if clamped
  int nfree = 0, vbw = 0;
  std::string err;
};

namespace {

fsi_status fail(fsi_ms* ms, fsi_status s, const char* msg) {
  if (ms) ms->err = msg;
  return s;
}

// wing-frame components of an inertial vector: a_w = F^T a (F columns = wing axes)
inline V3 to_wing(const double* F, V3 a) {
  return {F[0] * a.x + F[3] * a.y + F[6] * a.z, F[1] * a.x + F[4] * a.y + F[7] * a.z,
          F[2] * a.x + F[5] * a.y + F[8] * a.z};
}
// inertial components of a wing-frame vector: F a_w
inline V3 to_inertial(const double* F, const double* w) {
  return {F[0] * w[0] + F[1] * w[1] + F[2] * w[2], F[3] * w[0] + F[4] * w[1] + F[5] * w[2],
          F[6] * w[0] + F[7] * w[1] + F[8] * w[2]};
}

const double kIdentity[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};

// Elastic energy, forces (-grad) and, optionally, the Hessian blocks of every
// spring handed to `sink(u, w, block[3][3])` (block = d2E / dx_u dx_w).  With
// dF (and hess), df receives the derivative of the forces at fixed x when the
// frame moves along dF (only bending springs depend on the frame).
template <typename Sink>
double springs(const fsi_ms& ms, const double* x, const double* F, double* f, bool hess, Sink&& sink,
               const double* dF = nullptr, double* df = nullptr) {
  double E = 0.0;
  if (f) memset(f, 0, sizeof(double) * 3 * ms.nv);
  if (df) memset(df, 0, sizeof(double) * 3 * ms.nv);
  // extension springs
  for (size_t s = 0; s < ms.ek.size(); ++s) {
    const int i = ms.ei[s], j = ms.ej[s];
    const double d[3] = {x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1], x[3 * j + 2] - x[3 * i + 2]};
    const double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double k = ms.ek[s], ext = L - ms.el0[s];
    E += 0.5 * k * ext * ext;
    const double e[3] = {d[0] / L, d[1] / L, d[2] / L};
    if (f)
      for (int c = 0; c < 3; ++c) {
        const double fi = k * ext * e[c];
        f[3 * i + c] += fi;
        f[3 * j + c] -= fi;
      }
    if (hess) {
      // d2E/dd2 = k [e e^T + (1 - l0/L)(I - e e^T)]
      double K[3][3];
      const double t = 1.0 - ms.el0[s] / L;
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) K[r][c] = k * ((1.0 - t) * e[r] * e[c] + (r == c ? t : 0.0));
      double N[3][3];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) N[r][c] = -K[r][c];
      sink(i, i, K);
      sink(j, j, K);
      sink(i, j, N);
      sink(j, i, N);
    }
  }
  // bending springs
  for (size_t s = 0; s < ms.bkb.size(); ++s) {
    const int vi = ms.bi[s], vj = ms.bj[s], vk = ms.bk[s];
    const V3 a = to_wing(F, {x[3 * vj] - x[3 * vi], x[3 * vj + 1] - x[3 * vi + 1], x[3 * vj + 2] - x[3 * vi + 2]});
    const V3 b = to_wing(F, {x[3 * vk] - x[3 * vj], x[3 * vk + 1] - x[3 * vj + 1], x[3 * vk + 2] - x[3 * vj + 2]});
    const double kb = ms.bkb[s];
    const int ax = ms.bax[s];
    double ga[3] = {0, 0, 0}, gb[3] = {0, 0, 0};  // dE/da, dE/db (permuted wing frame)
    double Hab[6][6];                             // d2E/d(a,b)^2 (permuted wing frame)
    memset(Hab, 0, sizeof(Hab));
    const double aw[3] = {a.x, a.y, a.z}, bw[3] = {b.x, b.y, b.z};
    // component c of the permuted frame is wing component (ax + c) mod 3
    const double av[3] = {aw[ax], aw[(ax + 1) % 3], aw[(ax + 2) % 3]};
    const double bv[3] = {bw[ax], bw[(ax + 1) % 3], bw[(ax + 2) % 3]};
    for (int p = 0; p < 2; ++p) {
      const int q = p + 1;  // projection on the wing plane (x, q): q = y, then z
      const double ra = av[0] * av[0] + av[q] * av[q], rb = bv[0] * bv[0] + bv[q] * bv[q];
      const double th = atan2(bv[q], bv[0]) - atan2(av[q], av[0]);
      // wrap to (-pi, pi], the range of Eq. two_bending_angles
      double t = th;
      if (t > M_PI) t -= 2 * M_PI;
      if (t <= -M_PI) t += 2 * M_PI;
      const double dth = t - ms.bt0[2 * s + p];
      E += 0.5 * kb * dth * dth;
      // grad theta: -grad phi(a), +grad phi(b); grad phi(v) = (-v_q, v_p) / r^2
      double g[6] = {0, 0, 0, 0, 0, 0};
      g[0] = av[q] / ra;
      g[q] = -av[0] / ra;
      g[3] = -bv[q] / rb;
      g[3 + q] = bv[0] / rb;
      for (int c = 0; c < 3; ++c) {
        ga[c] += kb * dth * g[c];
        gb[c] += kb * dth * g[3 + c];
      }
      if (hess) {
        for (int r = 0; r < 6; ++r)
          for (int c = 0; c < 6; ++c) Hab[r][c] += kb * g[r] * g[c];
        // (theta - theta0) * hess theta: -hess phi(a), +hess phi(b);
        // hess phi(v) = [[2 v_p v_q, v_q^2 - v_p^2], [., -2 v_p v_q]] / r^4
        const double fa = -kb * dth / (ra * ra), fb = kb * dth / (rb * rb);
        const int ia[2] = {0, q}, ib[2] = {3, 3 + q};
        const double ha[2][2] = {{2 * av[0] * av[q], av[q] * av[q] - av[0] * av[0]},
                                 {av[q] * av[q] - av[0] * av[0], -2 * av[0] * av[q]}};
        const double hb[2][2] = {{2 * bv[0] * bv[q], bv[q] * bv[q] - bv[0] * bv[0]},
                                 {bv[q] * bv[q] - bv[0] * bv[0], -2 * bv[0] * bv[q]}};
        for (int r = 0; r < 2; ++r)
          for (int c = 0; c < 2; ++c) {
            Hab[ia[r]][ia[c]] += fa * ha[r][c];
            Hab[ib[r]][ib[c]] += fb * hb[r][c];
          }
      }
    }
    // back to wing components
    double gaw[3], gbw[3];
    for (int c = 0; c < 3; ++c) {
      gaw[(ax + c) % 3] = ga[c];
      gbw[(ax + c) % 3] = gb[c];
    }
    if (f) {
      const V3 Ga = to_inertial(F, gaw), Gb = to_inertial(F, gbw);
      // a = x_j - x_i, b = x_k - x_j:  f_i = F ga, f_j = F (gb - ga), f_k = -F gb
      const double A[3] = {Ga.x, Ga.y, Ga.z}, B[3] = {Gb.x, Gb.y, Gb.z};
      for (int c = 0; c < 3; ++c) {
        f[3 * vi + c] += A[c];
        f[3 * vj + c] += B[c] - A[c];
        f[3 * vk + c] -= B[c];
      }
    }
    if (hess) {
      // undo the permutation, then rotate to the inertial frame:
      // G = diag(F, F) Hw diag(F^T, F^T)
      double Hw[6][6];
      for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c)
          Hw[(r / 3) * 3 + (ax + r % 3) % 3][(c / 3) * 3 + (ax + c % 3) % 3] = Hab[r][c];
      double G[6][6];
      for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
          const int rb0 = (r / 3) * 3, cb0 = (c / 3) * 3, rr = r % 3, cc = c % 3;
          double sum = 0.0;
          for (int m = 0; m < 3; ++m)
            for (int n = 0; n < 3; ++n) sum += F[3 * rr + m] * Hw[rb0 + m][cb0 + n] * F[3 * cc + n];
          G[r][c] = sum;
        }
      // x_i -> (-I, 0), x_j -> (I, -I), x_k -> (0, I)
      const int vtx[3] = {vi, vj, vk};
      const double S[3][2] = {{-1, 0}, {1, -1}, {0, 1}};
      for (int u = 0; u < 3; ++u)
        for (int w = 0; w < 3; ++w) {
          double blk[3][3];
          for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
              blk[r][c] = S[u][0] * S[w][0] * G[r][c] + S[u][0] * S[w][1] * G[r][3 + c] +
                          S[u][1] * S[w][0] * G[3 + r][c] + S[u][1] * S[w][1] * G[3 + r][3 + c];
          sink(vtx[u], vtx[w], blk);
        }
      if (dF && df) {
        // d(ga, gb)/d(frame) along dF: Hw (dF^T a, dF^T b); f_i = F ga etc.
        const double ai[3] = {x[3 * vj] - x[3 * vi], x[3 * vj + 1] - x[3 * vi + 1], x[3 * vj + 2] - x[3 * vi + 2]};
        const double bi[3] = {x[3 * vk] - x[3 * vj], x[3 * vk + 1] - x[3 * vj + 1], x[3 * vk + 2] - x[3 * vj + 2]};
        double v6[6];
        for (int c = 0; c < 3; ++c) {
          v6[c] = dF[c] * ai[0] + dF[3 + c] * ai[1] + dF[6 + c] * ai[2];
          v6[3 + c] = dF[c] * bi[0] + dF[3 + c] * bi[1] + dF[6 + c] * bi[2];
        }
        double dg[6];
        for (int r = 0; r < 6; ++r) {
          double sum = 0.0;
          for (int c = 0; c < 6; ++c) sum += Hw[r][c] * v6[c];
          dg[r] = sum;
        }
        const V3 dA1 = to_inertial(dF, gaw), dB1 = to_inertial(dF, gbw);
        const V3 dA2 = to_inertial(F, dg), dB2 = to_inertial(F, dg + 3);
        const double dA[3] = {dA1.x + dA2.x, dA1.y + dA2.y, dA1.z + dA2.z};
        const double dB[3] = {dB1.x + dB2.x, dB1.y + dB2.y, dB1.z + dB2.z};
        for (int c = 0; c < 3; ++c) {
          df[3 * vi + c] += dA[c];
          df[3 * vj + c] += dB[c] - dA[c];
          df[3 * vk + c] -= dB[c];
        }
      }
    }
  }
  return E;
}

// -grad of the unit-stiffness energy (1/2) sum_p (theta^p - theta^p_0)^2 of
// bending spring s, for its vertices (i, j, k): the derivative of the forces
// with respect to k^b_s.
void bend_unit_forces(const fsi_ms& ms, size_t s, const double* x, const double* F, double out[3][3]) {
  const int vi = ms.bi[s], vj = ms.bj[s], vk = ms.bk[s], ax = ms.bax[s];
  const V3 a = to_wing(F, {x[3 * vj] - x[3 * vi], x[3 * vj + 1] - x[3 * vi + 1], x[3 * vj + 2] - x[3 * vi + 2]});
  const V3 b = to_wing(F, {x[3 * vk] - x[3 * vj], x[3 * vk + 1] - x[3 * vj + 1], x[3 * vk + 2] - x[3 * vj + 2]});
  const double aw[3] = {a.x, a.y, a.z}, bw[3] = {b.x, b.y, b.z};
  const double av[3] = {aw[ax], aw[(ax + 1) % 3], aw[(ax + 2) % 3]};
  const double bv[3] = {bw[ax], bw[(ax + 1) % 3], bw[(ax + 2) % 3]};
  double ga[3] = {0, 0, 0}, gb[3] = {0, 0, 0};
  for (int p = 0; p < 2; ++p) {
    const int q = p + 1;
    const double ra = av[0] * av[0] + av[q] * av[q], rb = bv[0] * bv[0] + bv[q] * bv[q];
    double t = atan2(bv[q], bv[0]) - atan2(av[q], av[0]);
    if (t > M_PI) t -= 2 * M_PI;
    if (t <= -M_PI) t += 2 * M_PI;
    const double dth = t - ms.bt0[2 * s + p];
    ga[0] += dth * av[q] / ra;
    ga[q] += -dth * av[0] / ra;
    gb[0] += -dth * bv[q] / rb;
    gb[q] += dth * bv[0] / rb;
  }
  double gaw[3], gbw[3];
  for (int c = 0; c < 3; ++c) {
    gaw[(ax + c) % 3] = ga[c];
    gbw[(ax + c) % 3] = gb[c];
  }
  const V3 A = to_inertial(F, gaw), B = to_inertial(F, gbw);
  const double Av[3] = {A.x, A.y, A.z}, Bv[3] = {B.x, B.y, B.z};
  for (int c = 0; c < 3; ++c) {
    out[0][c] = Av[c];
    out[1][c] = Bv[c] - Av[c];
    out[2][c] = -Bv[c];
  }
}

struct NoSink {
  void operator()(int, int, const double (&)[3][3]) const {}
};

// Order of the free vertices for the band solver: the narrowest band among
// reverse Cuthill-McKee over the spring graph, the index order, and the order
// along the principal axis of the current positions (structured wing meshes).
void build_order(fsi_ms& ms) {
  std::vector<std::vector<int>> adj(ms.nv);
  auto link = [&](int a, int b) {
    if (a == b || ms.is_clamped[a] || ms.is_clamped[b]) return;
    adj[a].push_back(b);
    adj[b].push_back(a);
  };
  for (size_t s = 0; s < ms.ek.size(); ++s) link(ms.ei[s], ms.ej[s]);
  for (size_t s = 0; s < ms.bkb.size(); ++s) {
    link(ms.bi[s], ms.bj[s]);
    link(ms.bj[s], ms.bk[s]);
    link(ms.bi[s], ms.bk[s]);
  }
  for (auto& l : adj) {
    std::sort(l.begin(), l.end());
    l.erase(std::unique(l.begin(), l.end()), l.end());
  }
  auto bandwidth = [&](const std::vector<int>& order) {
    std::vector<int> slot(ms.nv, -1);
    for (size_t k = 0; k < order.size(); ++k) slot[order[k]] = (int)k;
    int bw = 0;
    for (int u = 0; u < ms.nv; ++u)
      for (int w : adj[u]) bw = std::max(bw, std::abs(slot[u] - slot[w]));
    return bw;
  };
  std::vector<std::vector<int>> cand;
  {  // reverse Cuthill-McKee from a minimum-degree vertex of each component
    std::vector<int> order;
    std::vector<char> seen(ms.nv, 0);
    for (;;) {
      int start = -1;
      for (int i = 0; i < ms.nv; ++i)
        if (!ms.is_clamped[i] && !seen[i] && (start < 0 || adj[i].size() < adj[start].size())) start = i;
      if (start < 0) break;
      std::deque<int> qu{start};
      seen[start] = 1;
      while (!qu.empty()) {
        const int u = qu.front();
        qu.pop_front();
        order.push_back(u);
        std::vector<int> nb;
        for (int w : adj[u])
          if (!seen[w]) {
            seen[w] = 1;
            nb.push_back(w);
          }
        std::sort(nb.begin(), nb.end(), [&](int p, int q) { return adj[p].size() < adj[q].size(); });
        for (int w : nb) qu.push_back(w);
      }
    }
    std::reverse(order.begin(), order.end());
    cand.push_back(order);
  }
  {  // index order
    std::vector<int> order;
    for (int i = 0; i < ms.nv; ++i)
      if (!ms.is_clamped[i]) order.push_back(i);
    cand.push_back(order);
  }
  {  // principal axis of the positions (power iteration on the covariance)
    std::vector<int> order;
    double mean[3] = {0, 0, 0};
    for (int i = 0; i < ms.nv; ++i)
      for (int q = 0; q < 3; ++q) mean[q] += ms.x[3 * i + q] / ms.nv;
    double C[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int i = 0; i < ms.nv; ++i)
      for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) C[p][q] += (ms.x[3 * i + p] - mean[p]) * (ms.x[3 * i + q] - mean[q]);
    double e[3] = {1.0, 0.7, 0.3};
    for (int it = 0; it < 100; ++it) {
      double y[3];
      for (int p = 0; p < 3; ++p) y[p] = C[p][0] * e[0] + C[p][1] * e[1] + C[p][2] * e[2];
      const double nrm = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
      if (!(nrm > 0.0)) break;
      for (int p = 0; p < 3; ++p) e[p] = y[p] / nrm;
    }
    std::vector<std::pair<double, int>> key;
    for (int i = 0; i < ms.nv; ++i)
      if (!ms.is_clamped[i]) key.push_back({e[0] * ms.x[3 * i] + e[1] * ms.x[3 * i + 1] + e[2] * ms.x[3 * i + 2], i});
    std::stable_sort(key.begin(), key.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
      return a.first < b.first - 1e-12 * (1.0 + fabs(a.first));
    });
    for (auto& k : key) order.push_back(k.second);
    cand.push_back(order);
  }
  size_t best = 0;
  int best_bw = bandwidth(cand[0]);
  for (size_t c = 1; c < cand.size(); ++c) {
    const int b = bandwidth(cand[c]);
    if (b < best_bw) {
      best_bw = b;
      best = c;
    }
  }
  const std::vector<int>& order = cand[best];
  ms.slot.assign(ms.nv, -1);
  for (size_t k = 0; k < order.size(); ++k) ms.slot[order[k]] = (int)k;
  ms.nfree = (int)order.size();
  ms.vbw = best_bw;
  ms.order_valid = true;
}

// Newton matrix diag(mass) * mscale + hscale * H over the free vertices, and
// the elastic forces at x.
void assemble(fsi_ms& ms, const double* x, const double* F, double mscale, double hscale, Band& A,
              std::vector<double>& f) {
  if (!ms.order_valid) build_order(ms);
  const int bw = 3 * ms.vbw + 2;
  A.init(3 * ms.nfree, bw, bw);
  f.assign(3 * ms.nv, 0.0);
  springs(ms, x, F, f.data(), true, [&](int u, int w, const double (&blk)[3][3]) {
    const int su = ms.slot[u], sw = ms.slot[w];
    if (su < 0 || sw < 0) return;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) A(3 * su + r, 3 * sw + c) += hscale * blk[r][c];
  });
  if (mscale != 0.0)
    for (int u = 0; u < ms.nv; ++u)
      if (ms.slot[u] >= 0)
        for (int c = 0; c < 3; ++c) A(3 * ms.slot[u] + c, 3 * ms.slot[u] + c) += mscale * ms.mass[u];
}

}  // namespace

extern "C" {

fsi_status fsi_ms_create(int32_t nv, const double* mass, fsi_ms** out) {
  if (!out) return FSI_EINVAL;
  *out = nullptr;
  if (nv < 1 || !mass) return FSI_EINVAL;
  for (int i = 0; i < nv; ++i)
    if (!(mass[i] > 0.0) || !std::isfinite(mass[i])) return FSI_EINVAL;
  fsi_ms* ms = new (std::nothrow) fsi_ms;
  if (!ms) return FSI_ENOMEM;
  ms->nv = nv;
  ms->mass.assign(mass, mass + nv);
  ms->is_clamped.assign(nv, 0);
  ms->x.assign(3 * nv, 0.0);
  ms->v.assign(3 * nv, 0.0);
  *out = ms;
  return FSI_OK;
}

fsi_status fsi_ms_destroy(fsi_ms* ms) {
  delete ms;
  return FSI_OK;
}

const char* fsi_ms_last_error(const fsi_ms* ms) { return ms ? ms->err.c_str() : "null solver"; }

fsi_status fsi_ms_add_extension(fsi_ms* ms, int32_t n, const int32_t* ij, const double* k, const double* l0,
                                int32_t* first) {
  if (!ms) return FSI_EINVAL;
  if (n < 0 || (n > 0 && (!ij || !k || !l0))) return fail(ms, FSI_EINVAL, "bad extension spring arrays");
  for (int s = 0; s < n; ++s) {
    if (ij[2 * s] < 0 || ij[2 * s] >= ms->nv || ij[2 * s + 1] < 0 || ij[2 * s + 1] >= ms->nv ||
        ij[2 * s] == ij[2 * s + 1])
      return fail(ms, FSI_EINVAL, "extension spring vertex out of range or repeated");
    if (!(k[s] >= 0.0) || !(l0[s] > 0.0)) return fail(ms, FSI_EINVAL, "extension spring needs k >= 0, l0 > 0");
  }
  if (first) *first = (int32_t)ms->ek.size();
  for (int s = 0; s < n; ++s) {
    ms->ei.push_back(ij[2 * s]);
    ms->ej.push_back(ij[2 * s + 1]);
    ms->ek.push_back(k[s]);
    ms->el0.push_back(l0[s]);
  }
  ms->order_valid = false;
  return FSI_OK;
}

fsi_status fsi_ms_add_bending(fsi_ms* ms, int32_t n, const int32_t* ijk, const double* kb, const double* theta0,
                              const int32_t* axis, int32_t* first) {
  if (!ms) return FSI_EINVAL;
  if (n < 0 || (n > 0 && (!ijk || !kb || !theta0))) return fail(ms, FSI_EINVAL, "bad bending spring arrays");
  for (int s = 0; s < n; ++s) {
    for (int c = 0; c < 3; ++c)
      if (ijk[3 * s + c] < 0 || ijk[3 * s + c] >= ms->nv) return fail(ms, FSI_EINVAL, "bending vertex out of range");
    if (ijk[3 * s] == ijk[3 * s + 1] || ijk[3 * s + 1] == ijk[3 * s + 2])
      return fail(ms, FSI_EINVAL, "bending spring segments must have distinct ends");
    if (!(kb[s] >= 0.0)) return fail(ms, FSI_EINVAL, "bending stiffness must be >= 0");
    if (axis && (axis[s] < 0 || axis[s] > 2)) return fail(ms, FSI_EINVAL, "bending axis must be 0, 1 or 2");
  }
  if (first) *first = (int32_t)ms->bkb.size();
  for (int s = 0; s < n; ++s) {
    ms->bi.push_back(ijk[3 * s]);
    ms->bj.push_back(ijk[3 * s + 1]);
    ms->bk.push_back(ijk[3 * s + 2]);
    ms->bkb.push_back(kb[s]);
    ms->bax.push_back(axis ? axis[s] : 0);
    ms->bt0.push_back(theta0[2 * s]);
    ms->bt0.push_back(theta0[2 * s + 1]);
  }
  ms->order_valid = false;
  return FSI_OK;
}

fsi_status fsi_ms_set_extension_k(fsi_ms* ms, const double* k) {
  if (!ms) return FSI_EINVAL;
  if (!k && !ms->ek.empty()) return fail(ms, FSI_EINVAL, "k is NULL");
  for (size_t s = 0; s < ms->ek.size(); ++s)
    if (!(k[s] >= 0.0)) return fail(ms, FSI_EINVAL, "extension stiffness must be >= 0");
  for (size_t s = 0; s < ms->ek.size(); ++s) ms->ek[s] = k[s];
  return FSI_OK;
}

fsi_status fsi_ms_set_bending_k(fsi_ms* ms, const double* kb) {
  if (!ms) return FSI_EINVAL;
  if (!kb && !ms->bkb.empty()) return fail(ms, FSI_EINVAL, "kb is NULL");
  for (size_t s = 0; s < ms->bkb.size(); ++s)
    if (!(kb[s] >= 0.0)) return fail(ms, FSI_EINVAL, "bending stiffness must be >= 0");
  for (size_t s = 0; s < ms->bkb.size(); ++s) ms->bkb[s] = kb[s];
  return FSI_OK;
}

fsi_status fsi_ms_set_clamped(fsi_ms* ms, int32_t n, const int32_t* idx) {
  if (!ms) return FSI_EINVAL;
  if (n < 0 || (n > 0 && !idx)) return fail(ms, FSI_EINVAL, "bad clamped list");
  std::vector<int> flag(ms->nv, 0);
  for (int c = 0; c < n; ++c) {
    if (idx[c] < 0 || idx[c] >= ms->nv) return fail(ms, FSI_EINVAL, "clamped vertex out of range");
    if (flag[idx[c]]) return fail(ms, FSI_EINVAL, "clamped vertex listed twice");
    flag[idx[c]] = 1;
  }
  ms->clamped.assign(idx, idx + n);
  ms->is_clamped = flag;
  ms->order_valid = false;
  return FSI_OK;
}

fsi_status fsi_ms_bending_angles(const fsi_ms* ms, const double* x, const double* frame, double* theta) {
  if (!ms || !x || !theta) return FSI_EINVAL;
  const double* F = frame ? frame : kIdentity;
  for (size_t s = 0; s < ms->bkb.size(); ++s) {
    const int vi = ms->bi[s], vj = ms->bj[s], vk = ms->bk[s];
    const V3 a = to_wing(F, {x[3 * vj] - x[3 * vi], x[3 * vj + 1] - x[3 * vi + 1], x[3 * vj + 2] - x[3 * vi + 2]});
    const V3 b = to_wing(F, {x[3 * vk] - x[3 * vj], x[3 * vk + 1] - x[3 * vj + 1], x[3 * vk + 2] - x[3 * vj + 2]});
    const double aw[3] = {a.x, a.y, a.z}, bw[3] = {b.x, b.y, b.z};
    const int ax = ms->bax[s];
    const double av[3] = {aw[ax], aw[(ax + 1) % 3], aw[(ax + 2) % 3]};
    const double bv[3] = {bw[ax], bw[(ax + 1) % 3], bw[(ax + 2) % 3]};
    for (int p = 0; p < 2; ++p) {
      const int q = p + 1;
      // Eq. two_bending_angles: atan2 of the cross and dot products of the projections
      theta[2 * s + p] = atan2(av[0] * bv[q] - bv[0] * av[q], av[0] * bv[0] + av[q] * bv[q]);
    }
  }
  return FSI_OK;
}

fsi_status fsi_ms_set_rest(fsi_ms* ms, const double* frame) {
  if (!ms) return FSI_EINVAL;
  const double* x = ms->x.data();
  for (size_t s = 0; s < ms->ek.size(); ++s) {
    const int i = ms->ei[s], j = ms->ej[s];
    const double d[3] = {x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1], x[3 * j + 2] - x[3 * i + 2]};
    const double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (!(L > 0.0)) return fail(ms, FSI_EINVAL, "extension spring of zero length in the rest state");
  }
  std::vector<double> th(2 * ms->bkb.size());
  const fsi_status st = fsi_ms_bending_angles(ms, x, frame, th.data());
  if (st != FSI_OK) return st;
  for (size_t s = 0; s < ms->ek.size(); ++s) {
    const int i = ms->ei[s], j = ms->ej[s];
    const double d[3] = {x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1], x[3 * j + 2] - x[3 * i + 2]};
    ms->el0[s] = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  }
  ms->bt0 = th;
  return FSI_OK;
}

fsi_status fsi_ms_bending_stiffness(double EI, double l_b, int32_t n, double* kb) {
  if (!kb || !(EI >= 0.0) || !(l_b > 0.0) || n < 1) return FSI_EINVAL;
  // Eq. EI_k_relation: equal bending energy of a cantilever of length l_b and of
  // n + 2 mass points (the first two clamped) under a tip force
  *kb = EI / l_b * (double)n * (2.0 * n + 1.0) / (2.0 * (n + 1.0));
  return FSI_OK;
}

fsi_status fsi_ms_lumped_masses(int32_t nv, const double* x, int32_t nt, const int32_t* tri, double density,
                                double* mass) {
  if (nv < 1 || nt < 0 || !x || !mass || (nt > 0 && !tri) || !(density > 0.0)) return FSI_EINVAL;
  for (int t = 0; t < 3 * nt; ++t)
    if (tri[t] < 0 || tri[t] >= nv) return FSI_EINVAL;
  memset(mass, 0, sizeof(double) * nv);
  for (int t = 0; t < nt; ++t) {
    const int* v = tri + 3 * t;
    double e1[3], e2[3];
    for (int q = 0; q < 3; ++q) {
      e1[q] = x[3 * v[1] + q] - x[3 * v[0] + q];
      e2[q] = x[3 * v[2] + q] - x[3 * v[0] + q];
    }
    const double c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double area = 0.5 * sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    for (int k = 0; k < 3; ++k) mass[v[k]] += density * area / 3.0;
  }
  return FSI_OK;
}

fsi_status fsi_ms_forces(const fsi_ms* ms, const double* x, const double* frame, double* f, double* energy) {
  if (!ms || !x || !f) return FSI_EINVAL;
  const double E = springs(*ms, x, frame ? frame : kIdentity, f, false, NoSink{});
  if (energy) *energy = E;
  return FSI_OK;
}

fsi_status fsi_ms_set_state(fsi_ms* ms, const double* x, const double* v) {
  if (!ms || !x) return FSI_EINVAL;
  for (int i = 0; i < 3 * ms->nv; ++i)
    if (!std::isfinite(x[i]) || (v && !std::isfinite(v[i]))) return fail(ms, FSI_EINVAL, "non-finite state");
  ms->x.assign(x, x + 3 * ms->nv);
  if (v)
    ms->v.assign(v, v + 3 * ms->nv);
  else
    ms->v.assign(3 * ms->nv, 0.0);
  ms->have_prev = false;
  return FSI_OK;
}

fsi_status fsi_ms_get_state(const fsi_ms* ms, double* x, double* v) {
  if (!ms) return FSI_EINVAL;
  if (x) memcpy(x, ms->x.data(), sizeof(double) * 3 * ms->nv);
  if (v) memcpy(v, ms->v.data(), sizeof(double) * 3 * ms->nv);
  return FSI_OK;
}

fsi_status fsi_ms_step(fsi_ms* ms, double dt, const double* frame, const double* f_ext, const double* x_clamp,
                       const double* v_clamp, double tol, int32_t max_iter, int32_t* iters) {
  if (!ms) return FSI_EINVAL;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ms, FSI_EINVAL, "dt must be positive");
  if (max_iter < 1) return fail(ms, FSI_EINVAL, "max_iter must be >= 1");
  if (tol <= 0.0) tol = 1e-6;
  const double* F = frame ? frame : kIdentity;
  const int nv = ms->nv;
  const double xi = ms->have_prev ? dt / ms->dt_prev : 0.0;
  const double alpha = (1 + xi) * (1 + xi) / (1 + 2 * xi), beta = xi * xi / (1 + 2 * xi);
  const double gdt = (1 + xi) / (1 + 2 * xi) * dt;
  std::vector<double> bx(3 * nv), bv(3 * nv);
  for (int i = 0; i < 3 * nv; ++i) {
    bx[i] = alpha * ms->x[i] - (ms->have_prev ? beta * ms->xp[i] : 0.0);
    bv[i] = alpha * ms->v[i] - (ms->have_prev ? beta * ms->vp[i] : 0.0);
  }
  std::vector<double> x = ms->x, v(3 * nv);
  for (size_t c = 0; c < ms->clamped.size(); ++c) {
    const int u = ms->clamped[c];
    for (int d = 0; d < 3; ++d) {
      x[3 * u + d] = x_clamp ? x_clamp[3 * c + d] : ms->x[3 * u + d];
      v[3 * u + d] = v_clamp ? v_clamp[3 * c + d] : 0.0;
    }
  }
  Band A;
  std::vector<double> f, r;
  int it = 0;
  bool ok = false;
  for (it = 1; it <= max_iter; ++it) {
    // r = M (x - b_x) - gdt M b_v - gdt^2 (F_int + F_ext);  A = M + gdt^2 H
    assemble(*ms, x.data(), F, 1.0, gdt * gdt, A, f);
    r.assign(3 * ms->nfree, 0.0);
    for (int u = 0; u < nv; ++u) {
      const int su = ms->slot[u];
      if (su < 0) continue;
      for (int d = 0; d < 3; ++d) {
        const double fe = f_ext ? f_ext[3 * u + d] : 0.0;
        r[3 * su + d] = -(ms->mass[u] * (x[3 * u + d] - bx[3 * u + d]) - gdt * ms->mass[u] * bv[3 * u + d] -
                          gdt * gdt * (f[3 * u + d] + fe));
      }
    }
    {
      // A is symmetric; Cholesky, else pivoted LU on a fresh assembly
      const std::vector<double> r0 = r;
      if (!A.solve_spd(r)) {
        assemble(*ms, x.data(), F, 1.0, gdt * gdt, A, f);
        r = r0;
        if (!A.solve(r)) return fail(ms, FSI_ESTATE, "singular Newton matrix");
      }
    }
    double dn = 0.0, qn = 0.0;
    for (int u = 0; u < nv; ++u) {
      const int su = ms->slot[u];
      if (su < 0) continue;
      for (int d = 0; d < 3; ++d) {
        const double dx = r[3 * su + d];
        x[3 * u + d] += dx;
        dn += dx * dx * (1.0 + 1.0 / (gdt * gdt));  // the update of (x, v)
      }
    }
    for (int u = 0; u < nv; ++u)
      if (ms->slot[u] >= 0)
        for (int d = 0; d < 3; ++d) v[3 * u + d] = (x[3 * u + d] - bx[3 * u + d]) / gdt;
    for (int i = 0; i < 3 * nv; ++i) qn += x[i] * x[i] + v[i] * v[i];
    if (!std::isfinite(dn)) return fail(ms, FSI_ESTATE, "Newton produced a non-finite update");
    if (sqrt(dn) <= tol * std::max(1.0, sqrt(qn))) {
      ok = true;
      break;
    }
  }
  if (!ok) return fail(ms, FSI_ESTATE, "Newton did not converge");
  ms->xp.swap(ms->x);
  ms->vp.swap(ms->v);
  ms->x = x;
  ms->v = v;
  ms->dt_prev = dt;
  ms->have_prev = true;
  if (iters) *iters = it;
  return FSI_OK;
}

fsi_status fsi_ms_set_history(fsi_ms* ms, const double* x_prev, const double* v_prev, double dt_prev) {
  if (!ms) return FSI_EINVAL;
  if (!x_prev) {
    ms->have_prev = false;
    return FSI_OK;
  }
  if (!v_prev || !(dt_prev > 0.0)) return fail(ms, FSI_EINVAL, "history needs x_prev, v_prev and dt_prev > 0");
  ms->xp.assign(x_prev, x_prev + 3 * ms->nv);
  ms->vp.assign(v_prev, v_prev + 3 * ms->nv);
  ms->dt_prev = dt_prev;
  ms->have_prev = true;
  return FSI_OK;
}

fsi_status fsi_ms_step_adjoint(fsi_ms* ms, double dt, double dt_prev, const double* frame, const double* dframe,
                               const double* x_new, const double* lam_x, const double* lam_v, double* lam_xn,
                               double* lam_vn, double* lam_xp, double* lam_vp, double* lam_load, double* lam_kext,
                               double* lam_kb, double* lam_clamp_x, double* lam_clamp_v, double* lam_dframe) {
  if (!ms || !x_new || !lam_x || !lam_v) return FSI_EINVAL;
  if (!(dt > 0.0)) return fail(ms, FSI_EINVAL, "dt must be positive");
  const double* F = frame ? frame : kIdentity;
  const int nv = ms->nv;
  const bool first = !(dt_prev > 0.0);
  const double xi = first ? 0.0 : dt / dt_prev;
  const double alpha = (1 + xi) * (1 + xi) / (1 + 2 * xi), beta = xi * xi / (1 + 2 * xi);
  const double gdt = (1 + xi) / (1 + 2 * xi) * dt;
  // A w = gdt lam_x + lam_v over the free vertices, A = M + gdt^2 H(x_new)
  Band A;
  std::vector<double> f;
  assemble(*ms, x_new, F, 1.0, gdt * gdt, A, f);
  std::vector<double> w3(3 * ms->nfree);
  for (int u = 0; u < nv; ++u) {
    const int su = ms->slot[u];
    if (su < 0) continue;
    for (int d = 0; d < 3; ++d) w3[3 * su + d] = gdt * lam_x[3 * u + d] + lam_v[3 * u + d];
  }
  {
    const std::vector<double> w30 = w3;
    if (!A.solve_spd(w3)) {
      assemble(*ms, x_new, F, 1.0, gdt * gdt, A, f);
      w3 = w30;
      if (!A.solve(w3)) return fail(ms, FSI_ESTATE, "singular Newton matrix in the adjoint step");
    }
  }
  std::vector<double> w(3 * nv, 0.0);  // M^-1 mu_v on the free vertices, 0 on clamped ones
  for (int u = 0; u < nv; ++u)
    if (ms->slot[u] >= 0)
      for (int d = 0; d < 3; ++d) w[3 * u + d] = w3[3 * ms->slot[u] + d];
  for (int u = 0; u < nv; ++u) {
    if (ms->slot[u] < 0) continue;
    for (int d = 0; d < 3; ++d) {
      const int i = 3 * u + d;
      const double mv = ms->mass[u] * w[i];        // mu_v
      const double mx = (mv - lam_v[i]) / gdt;      // mu_x
      if (lam_xn) lam_xn[i] += alpha * mx;
      if (lam_vn) lam_vn[i] += alpha * mv;
      if (!first) {
        if (lam_xp) lam_xp[i] -= beta * mx;
        if (lam_vp) lam_vp[i] -= beta * mv;
      }
      if (lam_load) lam_load[i] += gdt * w[i];
    }
  }
  // stiffness parameters
  if (lam_kext)
    for (size_t s = 0; s < ms->ek.size(); ++s) {
      const int i = ms->ei[s], j = ms->ej[s];
      const double d[3] = {x_new[3 * j] - x_new[3 * i], x_new[3 * j + 1] - x_new[3 * i + 1],
                           x_new[3 * j + 2] - x_new[3 * i + 2]};
      const double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      double dot = 0.0;
      for (int c = 0; c < 3; ++c) dot += (L - ms->el0[s]) * d[c] / L * (w[3 * i + c] - w[3 * j + c]);
      lam_kext[s] += gdt * dot;
    }
  if (lam_kb)
    for (size_t s = 0; s < ms->bkb.size(); ++s) {
      double g[3][3];
      bend_unit_forces(*ms, s, x_new, F, g);
      const int vt[3] = {ms->bi[s], ms->bj[s], ms->bk[s]};
      double dot = 0.0;
      for (int m = 0; m < 3; ++m)
        for (int c = 0; c < 3; ++c) dot += g[m][c] * w[3 * vt[m] + c];
      lam_kb[s] += gdt * dot;
    }
  // clamped rows: mu_cx = lam_cx - gdt (H w)_c, mu_cv = lam_cv; they are the
  // cotangents of the prescribed positions and velocities
  if (lam_clamp_x || lam_clamp_v) {
    std::vector<double> Hw(3 * nv, 0.0);
    springs(*ms, x_new, F, nullptr, true, [&](int u, int v2, const double (&blk)[3][3]) {
      if (!ms->is_clamped[u] || ms->is_clamped[v2]) return;
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Hw[3 * u + r] += blk[r][c] * w[3 * v2 + c];
    });
    for (size_t c = 0; c < ms->clamped.size(); ++c) {
      const int u = ms->clamped[c];
      for (int d = 0; d < 3; ++d) {
        if (lam_clamp_x) lam_clamp_x[3 * c + d] += lam_x[3 * u + d] - gdt * Hw[3 * u + d];
        if (lam_clamp_v) lam_clamp_v[3 * c + d] += lam_v[3 * u + d];
      }
    }
  }
  // frame moving along dframe: the forces change by df at fixed x
  if (dframe && lam_dframe) {
    std::vector<double> df(3 * nv);
    springs(*ms, x_new, F, nullptr, true, NoSink{}, dframe, df.data());
    double dot = 0.0;
    for (int i = 0; i < 3 * nv; ++i) dot += df[i] * w[i];
    *lam_dframe += gdt * dot;
  }
  return FSI_OK;
}

fsi_status fsi_ms_static(fsi_ms* ms, const double* frame, const double* f_ext, int32_t load_steps, double tol,
                         int32_t max_iter) {
  if (!ms) return FSI_EINVAL;
  if (load_steps < 1 || max_iter < 1) return fail(ms, FSI_EINVAL, "load_steps and max_iter must be >= 1");
  if (tol <= 0.0) tol = 1e-10;
  const double* F = frame ? frame : kIdentity;
  const int nv = ms->nv;
  std::vector<double> x = ms->x, f, r;
  Band A;
  for (int ls = 1; ls <= load_steps; ++ls) {
    const double lam = (double)ls / load_steps;
    bool ok = false;
    for (int it = 0; it < max_iter; ++it) {
      assemble(*ms, x.data(), F, 0.0, 1.0, A, f);
      r.assign(3 * ms->nfree, 0.0);
      for (int u = 0; u < nv; ++u) {
        const int su = ms->slot[u];
        if (su < 0) continue;
        // H dx = F_int + lam F_ext (Newton on F_int(x) + lam F_ext = 0, with dF_int/dx = -H)
        for (int d = 0; d < 3; ++d) r[3 * su + d] = f[3 * u + d] + lam * (f_ext ? f_ext[3 * u + d] : 0.0);
      }
      {
        const std::vector<double> r0 = r;
        if (!A.solve_spd(r)) {
          assemble(*ms, x.data(), F, 0.0, 1.0, A, f);
          r = r0;
          if (!A.solve(r)) return fail(ms, FSI_ESTATE, "singular stiffness matrix");
        }
      }
      double dn = 0.0, xn = 0.0;
      for (int u = 0; u < nv; ++u) {
        const int su = ms->slot[u];
        if (su < 0) continue;
        for (int d = 0; d < 3; ++d) {
          x[3 * u + d] += r[3 * su + d];
          dn += r[3 * su + d] * r[3 * su + d];
        }
      }
      for (double c : x) xn += c * c;
      if (!std::isfinite(dn)) return fail(ms, FSI_ESTATE, "static Newton produced a non-finite update");
      if (sqrt(dn) <= tol * std::max(1.0, sqrt(xn))) {
        ok = true;
        break;
      }
    }
    if (!ok) return fail(ms, FSI_ESTATE, "static Newton did not converge");
  }
  ms->x = x;
  ms->v.assign(3 * nv, 0.0);
  ms->have_prev = false;
  return FSI_OK;
}

}  // extern "C"
