// adjoint.hip - reverse (transposed) passes of the penalized pseudo-spectral step.
//
// With dt held fixed, one step maps (u_hat^n, N_hat^{n-1}) to
// (u_hat^{n+1}, N_hat^n) and produces the force F^n (Sec. 4.1 penalized
// equations, force of Sec. 4.2.2).  Its transpose, under the real inner
// product on physical arrays and Re sum conj(a) b over the stored half
// spectrum, is assembled from the same transforms:
//   C2R^T(lambda) = N^3 m_k R2C_normalized(lambda),
//   R2C^T(mu)     = N^-3 C2R(mu / m_k),          m_k = 1 at kx = 0, else 2,
//   (i k x)^T = i k x,  (u x omega)^T: lambda_u = omega x lambda, lambda_omega = lambda x u,
// and the Leray projection, the 2/3 band and the integrating factors are real
// symmetric per mode.  The spectral part (update and projection transposes) is
// the column pass COL_ADJ_MU (kernels.hip), fused with the z inverse of its output.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "device_util.h"
#include "kernels.h"
#include "launch.h"
#include "wave512.h"

namespace fsi {

// ---------------------------------------------------------------------------
// fused x pass of the reverse step (two lines per workgroup, LDS transforms)
// ---------------------------------------------------------------------------

// Real signals of the inverse transforms, packed two per complex transform:
// line 0 fields 0..8, then line 1 with its lambda_Gz first.  lambda_G is about
// N^-1.5 of u and omega in size, and a complex transform of two real signals
// rounds each at the scale of the larger one, so the lambda_G components only
// share transforms with each other: (gx, gy), (gz, gz'), (gx', gy').
__device__ __forceinline__ int adj_sig(int l, int q) { return l == 0 ? q : 9 + (q == 8 ? 0 : q + 1); }
__device__ __forceinline__ int adj_sig_line(int r) { return r < 9 ? 0 : 1; }
__device__ __forceinline__ int adj_sig_field(int r) { return r < 9 ? r : (r == 9 ? 8 : r - 10); }

// Input field f: u, omega (f < 6) from the step's tape when there is one
template <typename T>
__device__ __forceinline__ const cpx<T>* adj_in(const XAdjArgs<T>& a, int f) {
  return (f < 6 && a.utape) ? a.utape + (long long)f * a.sfs : a.spec + (long long)f * a.sfs;
}

template <typename T, int NT, int MAXE>
__global__ __launch_bounds__(NT) void xpass_adj(XAdjArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  constexpr int L = 2;
  constexpr int SI = 9;  // 18 real signals (9 fields x 2 lines) packed in pairs
  constexpr int SF = 6;  // 12 real signals (6 fields x 2 lines)
  constexpr int RI = PadStride<SI>::value;
  constexpr int RF = PadStride<SF>::value;
  constexpr int PMAX = (2 * MAXE + 8) / 9 + 1;
  const int n = a.n, K = a.kx1 - 1;
  const int ngroups = a.nlines / L;
  cpx<T>* tws = buf + n * RI;
  for (int i = threadIdx.x; i < n; i += NT) tws[i] = a.tw[i];
  T* bufr = reinterpret_cast<T*>(buf);

  for (int g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const int tid = opaque((int)threadIdx.x);
    const int line0 = g * L;
    // 1) C2R of the 9 fields of both lines: real signals in adj_sig order, pairs (2j, 2j + 1)
    for (int it = tid; it < SI * n; it += NT) {
      const int x = it % n, j = it / n;
      const int ra = 2 * j, rb = 2 * j + 1;
      if (x <= K) {
        const cpx<T> A = adj_in(a, adj_sig_field(ra))[(long long)(line0 + adj_sig_line(ra)) * a.ld + x];
        const cpx<T> B = adj_in(a, adj_sig_field(rb))[(long long)(line0 + adj_sig_line(rb)) * a.ld + x];
        if (x == 0) buf[j] = mk<T>(A.re, B.re);
        else {
          buf[x * RI + j] = mk<T>(A.re - B.im, A.im + B.re);
          buf[(n - x) * RI + j] = mk<T>(A.re + B.im, B.re - A.im);
        }
      } else if (x < n - K) {
        buf[x * RI + j] = mk<T>(0, 0);
      }
    }
    __syncthreads();
    fft_lds<T, SI, RI, NT, MAXE, true>(buf, a.plan, tws);

    // 2) pointwise transpose of G = u x omega - (chi/eta)(u - u_s) and of the force
    T out[PMAX][6];
    const int tid2 = opaque((int)threadIdx.x);
#pragma unroll
    for (int k = 0; k < PMAX; ++k) {
      const int it = tid2 + k * NT;
      if (it < n * L) {
        const int x = it % n, l = it / n;
        T f[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          const int r = adj_sig(l, q);
          f[q] = bufr[2 * (x * RI + (r >> 1)) + (r & 1)];
        }
        const T ux = f[0], uy = f[1], uz = f[2], wx = f[3], wy = f[4], wz = f[5];
        const T gx = f[6], gy = f[7], gz = f[8];
        T lux = wy * gz - wz * gy;  // omega x lambda_G
        T luy = wz * gx - wx * gz;
        T luz = wx * gy - wy * gx;
        const int line = line0 + l;
        const int z = line / a.ny, y = line - z * a.ny;
        if (a.pnx > 0) {
          const int qx = x - a.px0, qy = y - a.py0, qz = z - a.pz0;
          if (qx >= 0 && qx < a.pnx && qy >= 0 && qy < a.pny && qz >= 0 && qz < a.pnz) {
            // p = Pi - |u|^2 / 2: lambda_u -= u lambda_p
            const T lpv = a.lp[((long long)qz * a.pny + qy) * a.pnx + qx];
            lux -= ux * lpv;
            luy -= uy * lpv;
            luz -= uz * lpv;
          }
        }
        const int bx = x - a.bx0, by = y - a.by0, bz = z - a.bz0;
        if (a.bnx > 0 && bx >= 0 && bx < a.bnx && by >= 0 && by < a.bny && bz >= 0 && bz < a.bnz) {
          const long long cell = ((long long)bz * a.bny + by) * a.bnx + bx;
          const T ch = a.chi[cell];
          const T sx = ux - a.us[cell], sy = uy - a.us[a.bcells + cell], sz = uz - a.us[2 * a.bcells + cell];
          // lambda_G and the force seed act on (u - u_s) through chi / eta
          const T hx = (a.g0 - gx) * a.inv_eta, hy = (a.g1 - gy) * a.inv_eta, hz = (a.g2 - gz) * a.inv_eta;
          lux += ch * hx;
          luy += ch * hy;
          luz += ch * hz;
          a.lchi[cell] = hx * sx + hy * sy + hz * sz;
          a.lus[cell] = -ch * hx;
          a.lus[a.bcells + cell] = -ch * hy;
          a.lus[2 * a.bcells + cell] = -ch * hz;
        }
        out[k][0] = lux;
        out[k][1] = luy;
        out[k][2] = luz;
        out[k][3] = gy * uz - gz * uy;  // lambda_G x u
        out[k][4] = gz * ux - gx * uz;
        out[k][5] = gx * uy - gy * ux;
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PMAX; ++k) {
      const int it = tid2 + k * NT;
      if (it < n * L) {
        const int x = it % n, l = it / n;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const int r = l * 6 + q;
          bufr[2 * (x * RF + (r >> 1)) + (r & 1)] = out[k][q];
        }
      }
    }
    __syncthreads();
    fft_lds<T, SF, RF, NT, MAXE, false>(buf, a.plan, tws);

    // 3) unpack the 12 real transforms, keep kx <= K
    const int tid3 = opaque((int)threadIdx.x);
    for (int it = tid3; it < 2 * SF * a.kx1; it += NT) {
      const int k = it % a.kx1, r = it / a.kx1;
      const cpx<T> zz = buf[k * RF + (r >> 1)];
      const cpx<T> zc = conj(buf[((n - k) % n) * RF + (r >> 1)]);
      cpx<T> v;
      if (!(r & 1)) v = scl(zz + zc, (T)0.5);
      else {
        const cpx<T> d = zz - zc;
        v = mk<T>((T)0.5 * d.im, (T)-0.5 * d.re);
      }
      a.spec[(r % 6) * a.sfs + (long long)(line0 + r / 6) * a.ld + k] = v;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// fused x pass of the reverse step for nx = 512: one wavefront per line pair,
// register-resident transforms (wave512.h)
// ---------------------------------------------------------------------------
//
// Per line the 9 inputs (u, omega, lambda_G) are 4 packed complex signals
// (ux + i uy, uz + i wx, wy + i wz, gx + i gy); the lambda_Gz of the two lines
// of the pair share one more.  The 6 outputs (lambda_u, lambda_omega) of a
// line are 3 packed forward transforms.  Every line is read completely before
// any of its outputs is stored, so the pass runs in place.

template <typename T>
__device__ __forceinline__ void xadj_load(const XAdjArgs<T>& a, int line, int f, int lane, Raw512<T>& w) {
  load512<T>(adj_in(a, f) + (long long)line * a.ld, adj_in(a, f + 1) + (long long)line * a.ld, lane, w);
}

// One line: inverse transforms of the 8 paired inputs (lambda_Gz given in the
// physical layout), the transposed pointwise term, the sub-box cotangents of
// chi and u_s, and the forward transforms of the 6 outputs.
template <typename T>
__device__ __forceinline__ void xadj_line(const XAdjArgs<T>& a, int line, int lane, cpx<T>* X, const cpx<T>* tIB,
                                          const cpx<T>* tC, const cpx<T>* tFB, const T (&gzl)[8]) {
  constexpr int K = 170;
  cpx<T> P[4][8];
  Raw512<T> w;
  xadj_load<T>(a, line, 0, lane, w);
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    cpx<T> v[8];
    pack512<T>(w, lane, v);
    if (p < 3) xadj_load<T>(a, line, 2 * p + 2, lane, w);  // in flight during the transform
    inv512<T>(v, X, lane, tIB, tC);
#pragma unroll
    for (int j = 0; j < 8; ++j) P[p][j] = v[j];
  }
  cpx<T> o[3][8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const T ux = P[0][j].re, uy = P[0][j].im, uz = P[1][j].re;
    const T wx = P[1][j].im, wy = P[2][j].re, wz = P[2][j].im;
    const T gx = P[3][j].re, gy = P[3][j].im, gz = gzl[j];
    o[0][j] = mk<T>(wy * gz - wz * gy, wz * gx - wx * gz);  // omega x lambda_G
    o[1][j] = mk<T>(wx * gy - wy * gx, gy * uz - gz * uy);  // ..., lambda_G x u
    o[2][j] = mk<T>(gz * ux - gx * uz, gx * uy - gy * ux);
  }
  const int z = line / a.ny, y = line - z * a.ny;
  const int qy = y - a.py0, qz = z - a.pz0;
  if (a.pnx > 0 && qy >= 0 && qy < a.pny && qz >= 0 && qz < a.pnz) {  // uniform per wave
    const long long rowcell = ((long long)qz * a.pny + qy) * a.pnx;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int qx = (lane >> 3) + 8 * (lane & 7) + 64 * j - a.px0;
      if (qx >= 0 && qx < a.pnx) {
        // p = Pi - |u|^2 / 2: lambda_u -= u lambda_p
        const T lpv = a.lp[rowcell + qx];
        o[0][j].re -= P[0][j].re * lpv;
        o[0][j].im -= P[0][j].im * lpv;
        o[1][j].re -= P[1][j].re * lpv;
      }
    }
  }
  const int by = y - a.by0, bz = z - a.bz0;
  if (a.bnx > 0 && by >= 0 && by < a.bny && bz >= 0 && bz < a.bnz) {  // uniform per wave
    const long long rowcell = ((long long)bz * a.bny + by) * a.bnx;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int bx = (lane >> 3) + 8 * (lane & 7) + 64 * j - a.bx0;
      if (bx >= 0 && bx < a.bnx) {
        const long long cell = rowcell + bx;
        const T ch = a.chi[cell];
        const T sx = P[0][j].re - a.us[cell];
        const T sy = P[0][j].im - a.us[a.bcells + cell];
        const T sz = P[1][j].re - a.us[2 * a.bcells + cell];
        // lambda_G and the force seed act on (u - u_s) through chi / eta
        const T hx = (a.g0 - P[3][j].re) * a.inv_eta;
        const T hy = (a.g1 - P[3][j].im) * a.inv_eta;
        const T hz = (a.g2 - gzl[j]) * a.inv_eta;
        o[0][j].re += ch * hx;
        o[0][j].im += ch * hy;
        o[1][j].re += ch * hz;
        a.lchi[cell] = hx * sx + hy * sy + hz * sz;
        a.lus[cell] = -ch * hx;
        a.lus[a.bcells + cell] = -ch * hy;
        a.lus[2 * a.bcells + cell] = -ch * hz;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    fwd512<T>(o[p], X, lane, tC, tFB);
    unpack_store512<T>(o[p], lane, K, a.spec + (long long)(2 * p) * a.sfs + (long long)line * a.ld,
                       a.spec + (long long)(2 * p + 1) * a.sfs + (long long)line * a.ld);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void xadj_wave512(XAdjArgs<T> a) {
  __shared__ cpx<T> xbuf[4][kXBuf];
  __shared__ cpx<T> tws[3][512];
  // the wave index is uniform: as a scalar, every line address is a scalar
  // base plus a 32-bit lane offset (no 64-bit vector address arithmetic)
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  cpx<T>* X = xbuf[wv];
  wave512_twiddles<T, 256>(tws, a.tw);
  __syncthreads();
  const int npairs = a.nlines / 2;
#pragma unroll 1
  for (int pr = blockIdx.x * 4 + wv; pr < npairs; pr += gridDim.x * 4) {
    const int l0 = opaque(lane);
    // lambda_Gz of both lines as one packed signal
    Raw512<T> w;
    load512<T>(a.spec + 8 * a.sfs + (long long)(2 * pr) * a.ld, a.spec + 8 * a.sfs + (long long)(2 * pr + 1) * a.ld,
               l0, w);
    cpx<T> v[8];
    pack512<T>(w, l0, v);
    inv512<T>(v, X, l0, tws[0], tws[1]);
    T gza[8], gzb[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      gza[j] = v[j].re;
      gzb[j] = v[j].im;
    }
    xadj_line<T>(a, 2 * pr, opaque(lane), X, tws[0], tws[1], tws[2], gza);
    xadj_line<T>(a, 2 * pr + 1, opaque(lane), X, tws[0], tws[1], tws[2], gzb);
  }
}

// ---------------------------------------------------------------------------
// mask adjoint: per-triangle vertex cotangents
// ---------------------------------------------------------------------------

__device__ __forceinline__ double profile_dchi(double d, double tw, double h, int profile) {
  if (profile == 0) {
    if (d <= tw - h || d >= tw + h) return 0.0;
    return -0.5 * sin(3.14159265358979323846 * (d - tw + h) / (2.0 * h)) * 3.14159265358979323846 / (2.0 * h);
  }
  const double th = tanh((d - tw) / h);
  return -0.5 * (1.0 - th * th) / h;
}

template <typename T>
__global__ __launch_bounds__(256) void mask_adj(MaskAdjArgs<T> a) {
  __shared__ double red[18 * 4];
  const int t = blockIdx.x;
  if (t >= a.nt) return;
  const int iv[3] = {a.tri[3 * t], a.tri[3 * t + 1], a.tri[3 * t + 2]};
  const double ax = a.x[3 * iv[0]], ay = a.x[3 * iv[0] + 1], az = a.x[3 * iv[0] + 2];
  const double bx = a.x[3 * iv[1]] - ax, by = a.x[3 * iv[1] + 1] - ay, bz = a.x[3 * iv[1] + 2] - az;
  const double cx = a.x[3 * iv[2]] - ax, cy = a.x[3 * iv[2] + 1] - ay, cz = a.x[3 * iv[2] + 2] - az;
  const double lox = fmin(fmin(0.0, bx), cx) + ax - a.rsup, hix = fmax(fmax(0.0, bx), cx) + ax + a.rsup;
  const double loy = fmin(fmin(0.0, by), cy) + ay - a.rsup, hiy = fmax(fmax(0.0, by), cy) + ay + a.rsup;
  const double loz = fmin(fmin(0.0, bz), cz) + az - a.rsup, hiz = fmax(fmax(0.0, bz), cz) + az + a.rsup;
  const int i0 = max((int)floor(lox / a.dx) - 1, a.bx0), i1 = min((int)ceil(hix / a.dx) + 1, a.bx0 + a.bnx - 1);
  const int j0 = max((int)floor(loy / a.dy) - 1, a.by0), j1 = min((int)ceil(hiy / a.dy) + 1, a.by0 + a.bny - 1);
  const int k0 = max((int)floor(loz / a.dz) - 1, a.bz0), k1 = min((int)ceil(hiz / a.dz) + 1, a.bz0 + a.bnz - 1);
  double acc[18];
#pragma unroll
  for (int q = 0; q < 18; ++q) acc[q] = 0.0;
  const double e[2][3] = {{bx, by, bz}, {cx, cy, cz}};
  if (i1 >= i0 && j1 >= j0 && k1 >= k0) {
    const int ni = i1 - i0 + 1, nj = j1 - j0 + 1, nk = k1 - k0 + 1;
    const int total = ni * nj * nk;
    for (int q = threadIdx.x; q < total; q += 256) {
      const int ii = i0 + q % ni;
      const int jj = j0 + (q / ni) % nj;
      const int kk = k0 + q / (ni * nj);
      const long long cell = ((long long)(kk - a.bz0) * a.bny + (jj - a.by0)) * a.bnx + (ii - a.bx0);
      const unsigned long long key = a.key2[cell];
      if (key == ~0ull || (int)(key & 0xffffffffull) != t) continue;
      const double p[3] = {(double)ii * a.dx - ax, (double)jj * a.dy - ay, (double)kk * a.dz - az};
      double w[3];
      TriRegion rg;
      const double d2 = closest_on_triangle<double>(p[0], p[1], p[2], bx, by, bz, cx, cy, cz, w[0], w[1], w[2], &rg);
      const double d = sqrt(d2);
      if (d >= a.rsup) continue;
      // closest point relative to vertex a
      double cp[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) cp[c] = w[1] * e[0][c] + w[2] * e[1][c];
      // distance: d delta / d x_j = -w_j (p - cp) / delta
      const double gd = (double)a.lchi[cell] * profile_dchi(d, a.tw, a.h, a.profile);
      if (gd != 0.0 && d > 0.0) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[3 * j + c] -= gd * w[j] * (p[c] - cp[c]) / d;
      }
      if ((double)a.chi[cell] == 0.0) continue;  // u_s is zero (and constant) there
      const double lu[3] = {(double)a.lus[cell], (double)a.lus[a.bcells + cell], (double)a.lus[2 * a.bcells + cell]};
      // velocities: u_s = sum_j w_j v_j
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[9 + 3 * j + c] += w[j] * lu[c];
      // positions through the barycentric weights of the closest point
      double vv[3][3];
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int c = 0; c < 3; ++c) vv[j][c] = a.v[3 * iv[j] + c];
      if (rg.kind == 0) {
        // face: (beta, gamma) = M^-1 (e0.d, e1.d), d = p - a
        const double lb = lu[0] * (vv[1][0] - vv[0][0]) + lu[1] * (vv[1][1] - vv[0][1]) + lu[2] * (vv[1][2] - vv[0][2]);
        const double lg = lu[0] * (vv[2][0] - vv[0][0]) + lu[1] * (vv[2][1] - vv[0][1]) + lu[2] * (vv[2][2] - vv[0][2]);
        const double m00 = bx * bx + by * by + bz * bz, m01 = bx * cx + by * cy + bz * cz, m11 = cx * cx + cy * cy + cz * cz;
        const double det = m00 * m11 - m01 * m01;
        const double y0 = (m11 * lb - m01 * lg) / det, y1 = (m00 * lg - m01 * lb) / det;
        const double be = w[1], ga = w[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double ge0 = y0 * p[c] - (2.0 * y0 * be * e[0][c] + (y0 * ga + y1 * be) * e[1][c]);
          const double ge1 = y1 * p[c] - ((y0 * ga + y1 * be) * e[0][c] + 2.0 * y1 * ga * e[1][c]);
          const double gdd = y0 * e[0][c] + y1 * e[1][c];
          acc[3 + c] += ge0;
          acc[6 + c] += ge1;
          acc[c] += -ge0 - ge1 - gdd;
        }
      } else if (rg.kind == 1) {
        // edge P0 = vertex i0, P1 = vertex i1, t = (p - P0).s / s.s, s = P1 - P0
        const double P0[3] = {rg.i0 == 0 ? 0.0 : e[rg.i0 - 1][0], rg.i0 == 0 ? 0.0 : e[rg.i0 - 1][1],
                              rg.i0 == 0 ? 0.0 : e[rg.i0 - 1][2]};
        const double P1[3] = {rg.i1 == 0 ? 0.0 : e[rg.i1 - 1][0], rg.i1 == 0 ? 0.0 : e[rg.i1 - 1][1],
                              rg.i1 == 0 ? 0.0 : e[rg.i1 - 1][2]};
        double s[3], d0[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          s[c] = P1[c] - P0[c];
          d0[c] = p[c] - P0[c];
        }
        const double ss = s[0] * s[0] + s[1] * s[1] + s[2] * s[2];
        if (ss > 0.0) {
          double lt = 0.0;
#pragma unroll
          for (int c = 0; c < 3; ++c) lt += lu[c] * (vv[rg.i1][c] - vv[rg.i0][c]);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const double g1 = lt * (d0[c] - 2.0 * rg.t * s[c]) / ss;
            const double g0 = lt * (-s[c] - d0[c] + 2.0 * rg.t * s[c]) / ss;
            acc[3 * rg.i1 + c] += g1;
            acc[3 * rg.i0 + c] += g0;
          }
        }
      }
    }
  }
  // fixed-order workgroup sums
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 18; ++q) {
    double v = acc[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[q * 4 + wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < 18) {
    const int q = threadIdx.x;
    a.tgrad[(long long)t * 18 + q] = ((red[q * 4] + red[q * 4 + 1]) + red[q * 4 + 2]) + red[q * 4 + 3];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <typename T>
struct XAdjCfg {
  static constexpr int NT = 512, MAXE = 10;
};

template <typename T>
int xadj_supported(int n) {
  return (n * 9 <= XAdjCfg<T>::MAXE * XAdjCfg<T>::NT) ? 1 : 0;
}

template <typename T>
hipError_t launch_xadj(const XAdjArgs<T>& a, int grid, hipStream_t s) {
  if (a.n == 512 && a.nlines % 2 == 0) {
    hipLaunchKernelGGL(xadj_wave512<T>, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
  }
  constexpr int NT = XAdjCfg<T>::NT, M = XAdjCfg<T>::MAXE;
  const size_t lds = (size_t)a.n * (PadStride<9>::value + 1) * sizeof(cpx<T>);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)xpass_adj<T, NT, M>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((xpass_adj<T, NT, M>), dim3(grid), dim3(NT), lds, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mask_adj(const MaskAdjArgs<T>& a, hipStream_t s) {
  if (a.nt <= 0) return hipSuccess;
  hipLaunchKernelGGL(mask_adj<T>, dim3(a.nt), dim3(256), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_xadj<float>(const XAdjArgs<float>&, int, hipStream_t);
template hipError_t launch_xadj<double>(const XAdjArgs<double>&, int, hipStream_t);
template int xadj_supported<float>(int);
template int xadj_supported<double>(int);
template hipError_t launch_mask_adj<float>(const MaskAdjArgs<float>&, hipStream_t);
template hipError_t launch_mask_adj<double>(const MaskAdjArgs<double>&, hipStream_t);

}  // namespace fsi
