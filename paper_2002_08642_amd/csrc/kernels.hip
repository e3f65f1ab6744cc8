// kernels.hip - the passes of the penalized pseudo-spectral step for gfx950.
//
// Sec. 4.1 (penalized Navier-Stokes in rotational form, Fourier pseudo-spectral
// discretization): every step evaluates u x omega - (chi/eta)(u - u_s) on the
// grid, transforms it back, projects it onto divergence-free fields and
// advances the velocity.  The passes below each make one round trip through
// HBM and keep the intermediate transforms in LDS.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "device_util.h"
#include "kernels.h"
#include "launch.h"
#include "wave512.h"

namespace fsi {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// column passes: FFT along the slow axis of a [rows][C] slice, W columns per WG
// ---------------------------------------------------------------------------
//
// LDS holds the W columns of the slice (n rows, row stride W) followed by the
// twiddle table of the axis.  Global loads are issued in unrolled batches
// into registers before they are written to LDS, so that each thread keeps
// all of its row loads in flight at once.

// Two adjacent complex FP32 values moved as one 16-byte access (the 512-point
// column passes: a lane carries two columns, halving the memory instructions).
struct cpx2f {
  cpx<float> a, b;
};
typedef float v4f __attribute__((ext_vector_type(4)));
// Moved through a buffer resource (a wave-uniform base and byte bound): a lane
// whose byte offset is at or beyond the bound loads zeros and its store is
// dropped, with no memory traffic and no branch (a branch around stores would
// make the next wait for prefetched loads wait for the stores).
// kOOB marks such lanes; every bound used here is below 2^31 bytes.
constexpr unsigned kOOB = 0x80000000u;
typedef unsigned v4u __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, long long bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0,
                                           (int)(bytes < (long long)kOOB ? bytes : (long long)kOOB), 0x00020000);
}
__device__ __forceinline__ cpx2f ld_buf2(__amdgpu_buffer_rsrc_t r, unsigned off) {
  const v4f w = __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, (FSI_NT & 2) ? 2 : 0));
  return cpx2f{mk<float>(w.x, w.y), mk<float>(w.z, w.w)};
}
__device__ __forceinline__ void st_buf2(__amdgpu_buffer_rsrc_t r, unsigned off, cpx2f v) {
  v4f w;
  w.x = v.a.re;
  w.y = v.a.im;
  w.z = v.b.re;
  w.w = v.b.im;
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4u, w), r, off, 0, (FSI_NT & 1) ? 2 : 0);
}
__device__ __forceinline__ cpx2f ld_lds2(const cpx<float>* p) {
  const v4f w = *reinterpret_cast<const v4f*>(p);
  return cpx2f{mk<float>(w.x, w.y), mk<float>(w.z, w.w)};
}
__device__ __forceinline__ void st_lds2(cpx<float>* p, cpx2f v) {
  v4f w;
  w.x = v.a.re;
  w.y = v.a.im;
  w.z = v.b.re;
  w.w = v.b.im;
  *reinterpret_cast<v4f*>(p) = w;
}

// f(integral_constant<int, I>) for I = B .. E - 1, in order
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// m of the e-th of the twelve rows r0 + 32 m (m = 0..5, 10..15) of a thread
// that can lie in the 2/3 band of a 512-point column
constexpr int band_slot512(int e) { return e < 6 ? e : e + 4; }

// a s - b t with both products rounded (no fused multiply-add): the stand-alone
// z-inverse pass and the one fused into the update pass then form the same bits
template <typename T>
__device__ __forceinline__ cpx<T> scaled_diff(cpx<T> a, T s, cpx<T> b, T t) {
#pragma clang fp contract(off)
  return mk<T>(a.re * s - b.re * t, a.im * s - b.im * t);
}

template <typename T, int W, int NT, int MAXE, int MODE, int N>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT >= 1024 ? 4 : NT / 128))) void col_pass(
    ColArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  constexpr int RSTEP = NT / W;
  // band rows per thread: 2K + 1 <= (2n + 1)/3 rows over RSTEP-row strides with
  // n <= MAXE RSTEP gives at most floor(2 MAXE / 3) + 1
  constexpr int MAXO = (2 * MAXE) / 3 + 1;
  const int tid = threadIdx.x;
  const int col = tid % W;
  const int r0 = tid / W;
  const int c = blockIdx.x * W + col;
  const bool cok = c < a.C && (c % a.kxp) < a.kx1;
  // N = 512: the column length and its 2/3 band are compile-time constants
  const int n = N ? N : a.n, K = N ? (N - 1) / 3 : a.K, nb = 2 * K + 1;
  // the RSTEP-row strides of a thread cover the column exactly: no row test
  constexpr bool FULL = N != 0 && N == MAXE * RSTEP;
  // two columns per lane, 16-byte loads and stores (y passes at 512 points, FP32)
  constexpr bool PAIR = FULL && N == 512 && sizeof(T) == 4 && W == 16;
  const long long ib = (long long)blockIdx.y * a.in_bs;
  const long long ob = (long long)blockIdx.y * a.out_bs;
  cpx<T>* tws = buf + n * W;
  for (int i = tid; i < n; i += NT) tws[i] = a.tw[i];

  if constexpr (MODE == COL_INV_PLAIN || MODE == COL_INV_CURL) {
    // COL_INV_CURL: outputs u (3) and omega = i k x u (3) from the three compact
    // components, produced in the order ux, wy, uz, wx, uy, wz so that two
    // register sets hold every component while it is needed (four component
    // loads per workgroup instead of nine).
    constexpr bool CURLM = (MODE == COL_INV_CURL);
    const int nout = (MODE == COL_INV_CURL) ? 6 : a.nf;
    cpx<T> RA[MAXO], RB[MAXO];
    // component loaded for output o (-1: none) and whether it goes to RB; the load
    // for output o + 1 is issued right after output o has been written to LDS, so
    // it is in flight while output o is transformed.
    // unconditional loads (clamped rows and columns), zeroed when written to LDS
    auto load_into = [&](int lq, cpx<T>(&R)[MAXO]) __attribute__((always_inline)) {
      const int tq = opaque_tid<NT>();
      const int cq = blockIdx.x * W + tq % W, rq = tq / W;
      const cpx<T>* in = a.in + lq * a.in_fs + ib + (cq < a.C ? cq : 0);
#pragma unroll
      for (int k = 0; k < MAXO; ++k) {
        const int i = rq + k * RSTEP;
        R[k] = ld_stream(in + (long long)(i < nb ? i : 0) * a.ld);
      }
    };
    auto load_for = [&](int o) {
      int lq = o, into_b = 0;
      if (CURLM) {
        lq = (o == 0) ? 0 : (o == 1) ? 2 : (o == 3) ? 1 : (o == 5) ? 0 : -1;
        into_b = (o == 1 || o == 5) ? 1 : 0;
      }
      if (lq < 0) return;
      const int tq = opaque_tid<NT>();
      const int cq = blockIdx.x * W + tq % W, rq = tq / W;
      // unconditional loads from clamped rows and columns: a load under a branch
      // makes the compiler wait for it where the branches join, which would end
      // the overlap with the transform; invalid values are replaced by zero when
      // they are written to LDS
      const cpx<T>* in = a.in + lq * a.in_fs + ib + (cq < a.C ? cq : 0);
#pragma unroll
      for (int k = 0; k < MAXO; ++k) {
        const int i = rq + k * RSTEP;
        const cpx<T> val = ld_stream(in + (long long)(i < nb ? i : 0) * a.ld);
        if (into_b) RB[k] = val;
        else RA[k] = val;
      }
    };
    // one output: LDS fill (with the curl combination), the next output's load,
    // the transform, the stores.  With a compile-time o (the static sequences
    // below) no prefetched register set is merged across branches.
    auto ostep = [&](auto oc, auto nc) __attribute__((always_inline)) {
      constexpr int o = decltype(oc)::value, NO = decltype(nc)::value;
      constexpr int fo = CURLM ? ((o == 1) ? 4 : (o == 4) ? 1 : o) : o;
      // source: 0 = A, 1 = B, 2 = curl combination of A and B
      constexpr int src = CURLM ? ((o & 1) ? 2 : (o == 2) ? 1 : 0) : (o & 1);
      // the load issued after this output is in LDS: field and set
      constexpr int nlq = CURLM ? ((o == 0) ? 2 : (o == 2) ? 1 : (o == 4) ? 0 : -1) : (o + 1 < NO ? o + 1 : -1);
      constexpr bool nb_set = CURLM ? (o == 0 || o == 4) : ((o + 1) & 1);
      const int tid = opaque_tid<NT>();
      const int col = tid % W, r0 = tid / W, c = blockIdx.x * W + col;
      const bool cok = c < a.C && (c % a.kxp) < a.kx1;
      const int ix = c % a.kxp, iy = c / a.kxp;
      const T kx = a.kfx * (T)ix;
      const T ky = a.kfy * (T)band_mode(iy, a.Ky);
#pragma unroll
      for (int k = 0; k < MAXE; ++k) {
        const int r = r0 + k * RSTEP;
        if (r > K && r < n - K) buf[r * W + col] = mk<T>(0, 0);
      }
#pragma unroll
      for (int k = 0; k < MAXO; ++k) {
        const int i = r0 + k * RSTEP;
        if (i < nb) {
          cpx<T> val = (src == 1) ? RB[k] : RA[k];
          if constexpr (src == 2) {
            const T kz = a.kfz * (T)band_mode(i, K);
            cpx<T> t;
            if constexpr (o == 1) t = scaled_diff(RA[k], kz, RB[k], kx);       // wy: kz ux - kx uz
            else if constexpr (o == 3) t = scaled_diff(RB[k], ky, RA[k], kz);  // wx: ky uz - kz uy
            else t = scaled_diff(RA[k], kx, RB[k], ky);                        // wz: kx uy - ky ux
            val = mk<T>(-t.im, t.re);  // i t
          }
          buf[band_to_row(i, K, n) * W + col] = cok ? val : mk<T>(0, 0);
        }
      }
      __syncthreads();
      if constexpr (nlq >= 0) {
        if constexpr (nb_set) {
          asm volatile("" ::: "memory");  // keeps the two load sites apart
          load_into(nlq, RB);
        } else {
          load_into(nlq, RA);
        }
      }
      col_fft<T, W, NT, MAXE, true, N>(buf, a.plan, tws);
      cpx<T>* out = a.out + fo * a.out_fs + ob;
      cpx<T> ov[MAXE];  // LDS reads first, then the stores
#pragma unroll
      for (int k = 0; k < MAXE; ++k) {
        const int r = r0 + k * RSTEP;
        ov[k] = buf[((FULL || r < n) ? r : 0) * W + col];
      }
      // 512 points: unconditional stores (columns out of the band carry zeros;
      // the launcher keeps the workgroup's columns within the row pitch), so
      // the next wait for a prefetched load does not wait for them as well
      if (N == 512 || cok) {
#pragma unroll
        for (int k = 0; k < MAXE; ++k) {
          const int r = r0 + k * RSTEP;
          if (FULL || r < n) st_stream(out + (long long)r * a.ld + c, ov[k]);
        }
      }
      __syncthreads();
    };
    using I1 = std::integral_constant<int, 1>;
    using I3 = std::integral_constant<int, 3>;
    using I6 = std::integral_constant<int, 6>;
    using I9 = std::integral_constant<int, 9>;
    // run-time output loop (other lengths and field counts)
    auto generic = [&]() {
      load_for(0);
      for (int o = 0; o < nout; ++o) {
        const int tid = opaque_tid<NT>();
        const int col = tid % W, r0 = tid / W, c = blockIdx.x * W + col;
        const bool cok = c < a.C && (c % a.kxp) < a.kx1;
        // output field and combination: o = 0 ux = A; 1 wy = i(kz A - kx B); 2 uz = B;
        // 3 wx = i(ky B - kz A); 4 uy = A; 5 wz = i(kx A - ky B)
        const int fo = CURLM ? ((o == 1) ? 4 : (o == 4) ? 1 : o) : o;
        T ka = 0, kb = 0;
        bool kza = false, kzb = false, cross = false;
        if (CURLM && (o & 1)) {
          const int ix = c % a.kxp, iy = c / a.kxp;
          const T kx = a.kfx * (T)ix;
          const T ky = a.kfy * (T)band_mode(iy, a.Ky);
          cross = true;
          if (o == 1) { kza = true; kb = kx; }
          else if (o == 3) { kb = ky; kza = true; }
          else { ka = kx; kb = ky; }
        }
        const bool useb = CURLM && (o == 2 || o == 3);
#pragma unroll
        for (int k = 0; k < MAXE; ++k) {
          const int r = r0 + k * RSTEP;
          if (r > K && r < n - K) buf[r * W + col] = mk<T>(0, 0);
        }
#pragma unroll
        for (int k = 0; k < MAXO; ++k) {
          const int i = r0 + k * RSTEP;
          if (i < nb) {
            cpx<T> val = useb ? RB[k] : RA[k];
            if (cross) {
              const T kz = a.kfz * (T)band_mode(i, K);
              // o = 1: kz A - kx B; o = 3: ky B - kz A = -(kz A - ky B); o = 5: kx A - ky B
              cpx<T> t = scl(RA[k], kza ? kz : ka) - scl(RB[k], kb);
              if (o == 3) t = mk<T>(-t.re, -t.im);
              val = mk<T>(-t.im, t.re);  // i t
            }
            buf[band_to_row(i, K, n) * W + col] = cok ? val : mk<T>(0, 0);
          }
        }
        __syncthreads();
        if (o + 1 < nout) load_for(o + 1);
        col_fft<T, W, NT, MAXE, true, N>(buf, a.plan, tws);
        cpx<T>* out = a.out + fo * a.out_fs + ob;
        // every LDS read first, then the stores: reading each value just before
        // its store would put an LDS round trip in front of every store
        cpx<T> ov[MAXE];
#pragma unroll
        for (int k = 0; k < MAXE; ++k) {
          const int r = r0 + k * RSTEP;
          ov[k] = buf[((FULL || r < n) ? r : 0) * W + col];
        }
        if (cok) {
#pragma unroll
          for (int k = 0; k < MAXE; ++k) {
            const int r = r0 + k * RSTEP;
            if (FULL || r < n) st_stream(out + (long long)r * a.ld + c, ov[k]);
          }
        }
        __syncthreads();
      }
    };
    if constexpr (N == 512 && CURLM) {
      load_into(0, RA);
      static_for<0, 6>([&](auto oc) { ostep(oc, I6{}); });
    } else if constexpr (N == 512) {
      if (nout == 1 || nout == 3 || nout == 9) load_into(0, RA);
      if (nout == 1) static_for<0, 1>([&](auto oc) { ostep(oc, I1{}); });
      else if (nout == 3) static_for<0, 3>([&](auto oc) { ostep(oc, I3{}); });
      else if (nout == 9) static_for<0, 9>([&](auto oc) { ostep(oc, I9{}); });
      else generic();
    } else {
      generic();
    }
  } else if constexpr (MODE == COL_ADJ_MU) {
    // Reverse of the update and the projection (per mode) on the thread's band
    // rows: lambda_N^n = a E lambda_u + lambda_N', the new lambda_N^{n-1} =
    // -b E E_prev lambda_u, lambda_u <- E lambda_u, mu = P(lambda_N^n)/(m_k N^3)
    // (+ i k lambda_Pi / |k|^2 with a pressure seed); then the z inverse of mu
    // from registers (three outputs), as COL_INV_PLAIN would from memory.
    const int ix = c % a.kxp, iy = c / a.kxp;
    const T kx = a.kfx * (T)ix;
    const T ky = a.kfy * (T)band_mode(iy, a.Ky);
    T an, bn;
    if (a.first) {
      an = (T)a.adt;
      bn = 0;
    } else {
      const double xi = a.adt / a.adtp;
      an = (T)(a.adt * (1.0 + 0.5 * xi));
      bn = (T)(a.adt * 0.5 * xi);
    }
    const T sc = (T)(a.invN3 / (ix == 0 ? 1.0 : 2.0));
    // FP32 512-point columns: the thread's rows r0 + 32 m (fft512_reg's
    // one-column slots; band slot e for m = band_slot512(e): m <= 4 and m >= 11
    // always in the band, m = 5 when r0 <= 10, m = 10 when r0 >= 22), so that mu
    // is in registers where the register-staged inverse transforms need it;
    // other lengths: band index r0 + k RSTEP
    constexpr bool REGM = N == 512 && sizeof(T) == 4 && RSTEP == 32 && MAXE == 16;
    constexpr int NS = REGM ? 12 : MAXO;
    const bool b5 = r0 <= 10, b10 = r0 >= 22;
    auto band_i = [&](int k, int rr) __attribute__((always_inline)) {
      if constexpr (REGM) {
        const int m = band_slot512(k);
        return m <= 5 ? rr + 32 * m : rr + 32 * m - 171;
      } else {
        return rr + k * RSTEP;
      }
    };
    auto band_ok = [&](int k) __attribute__((always_inline)) {
      if constexpr (REGM) {
        const int m = band_slot512(k);
        return (m <= 4 || m >= 11) ? true : (m == 5) ? b5 : b10;
      } else {
        return r0 + k * RSTEP < nb;
      }
    };
    cpx<T> M[3][NS];
    constexpr int KC = REGM ? 2 : sizeof(T) == 4 ? 3 : 1;
    const int cl = c < a.C ? c : 0;
#pragma unroll
    for (int k0 = 0; k0 < NS; k0 += KC) {
      cpx<T> uo[KC][3], po[KC][3];
      const int r0l = opaque(r0);  // addresses per chunk, not for all chunks ahead
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) {  // loads of the chunk before its stores
        const int k = k0 + kk;
        if (k < NS) {
          const int i = band_i(k, r0l);
          const long long idx = (long long)(i < nb ? i : 0) * a.ld + cl;
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            uo[kk][q] = a.uh[q * a.cfs + idx];
            po[kk][q] = a.nh[q * a.cfs + idx];
          }
        }
      }
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) {
        const int k = k0 + kk;
        if (k >= NS) break;
        const int i = band_i(k, r0l);
#pragma unroll
        for (int q = 0; q < 3; ++q) M[q][k] = mk<T>(0, 0);
        if (cok && band_ok(k)) {
          const T kz = a.kfz * (T)band_mode(i, K);
          const T k2 = kx * kx + ky * ky + kz * kz;
          const T en = dev_exp<T>(-a.nu * k2 * (T)a.adt);
          const T ep = a.first ? (T)0 : dev_exp<T>(-a.nu * k2 * (T)a.adtp);
          const long long idx = (long long)i * a.ld + c;
          cpx<T> ln[3];
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            ln[q] = scl(uo[kk][q], an * en) + po[kk][q];             // cotangent of N_hat^n
            a.nh[q * a.cfs + idx] = scl(uo[kk][q], -bn * en * ep);  // of N_hat^{n-1}
            a.uh[q * a.cfs + idx] = scl(uo[kk][q], en);             // update share of u_hat^n
          }
          cpx<T> extra[3] = {mk<T>(0, 0), mk<T>(0, 0), mk<T>(0, 0)};
          if (k2 > (T)0) {
            const cpx<T> sp = scl(scl(ln[0], kx) + scl(ln[1], ky) + scl(ln[2], kz), (T)1 / k2);
            ln[0] = ln[0] - scl(sp, kx);
            ln[1] = ln[1] - scl(sp, ky);
            ln[2] = ln[2] - scl(sp, kz);
            if (a.lpi) {  // Pi_hat = -i k.N'_hat / |k|^2: its transpose adds i k lambda_Pi / |k|^2
              const cpx<T> lp = a.lpi[idx];
              const T ik2 = (T)1 / k2;
              extra[0] = mk<T>(-kx * lp.im * ik2, kx * lp.re * ik2);
              extra[1] = mk<T>(-ky * lp.im * ik2, ky * lp.re * ik2);
              extra[2] = mk<T>(-kz * lp.im * ik2, kz * lp.re * ik2);
            }
          }
#pragma unroll
          for (int q = 0; q < 3; ++q) M[q][k] = scl(ln[q], sc) + extra[q];
          if (a.spadj) {
            // the sponge term T_hat = A S_hat, A = -(1/C_sp) (i k x) / |k|^2, enters
            // like N before the projection; A is Hermitian, so the cotangent
            // of S_hat over m_k N^3 is A mu
            const T f = k2 > (T)0 ? -a.csp_inv / k2 : (T)0;
            const cpx<T> t0 = scl(M[2][k], ky) - scl(M[1][k], kz);
            const cpx<T> t1 = scl(M[0][k], kz) - scl(M[2][k], kx);
            const cpx<T> t2 = scl(M[1][k], kx) - scl(M[0][k], ky);
            a.spadj[idx] = scl(mk<T>(-t0.im, t0.re), f);
            a.spadj[a.cfs + idx] = scl(mk<T>(-t1.im, t1.re), f);
            a.spadj[2 * a.cfs + idx] = scl(mk<T>(-t2.im, t2.re), f);
          }
        }
      }
    }
    if constexpr (REGM) {
      // z inverse of mu (three outputs) with the first and last stage on registers
      static_for<0, 3>([&](auto oc) __attribute__((always_inline)) {
        constexpr int o = decltype(oc)::value;
        cpx<T> v0[8], v1[8];
        static_for<0, 16>([&](auto mc) __attribute__((always_inline)) {
          constexpr int m = decltype(mc)::value;
          cpx<T> val = mk<T>(0, 0);
          if constexpr (m <= 5 || m >= 10) val = M[o][m <= 5 ? m : m - 4];
          if constexpr (m & 1) v1[m >> 1] = val;
          else v0[m >> 1] = val;
        });
        fft512_reg<T, W, true, true>(v0, v1, buf, tws);
        cpx<T>* out = a.out + o * a.out_fs + ob;
        // unconditional stores (columns out of the band carry zeros; the launcher
        // runs this kernel only for whole workgroups of columns): a store under
        // a branch makes the next wait for a prefetched load wait for the
        // stores as well
#pragma unroll
        for (int m = 0; m < 16; ++m)
          st_stream(out + (long long)(r0 + 32 * m) * a.ld + c, (m & 1) ? v1[m >> 1] : v0[m >> 1]);
      });
    } else {
      __syncthreads();
      auto mstep = [&](auto oc) {
        constexpr int o = decltype(oc)::value;
        const int tid = opaque_tid<NT>();
        const int col = tid % W, r0 = tid / W, c = blockIdx.x * W + col;
        const bool cok = c < a.C && (c % a.kxp) < a.kx1;
#pragma unroll
        for (int k = 0; k < MAXE; ++k) {
          const int r = r0 + k * RSTEP;
          if (r > K && r < n - K) buf[r * W + col] = mk<T>(0, 0);
        }
#pragma unroll
        for (int k = 0; k < MAXO; ++k) {
          const int i = r0 + k * RSTEP;
          if (i < nb) buf[band_to_row(i, K, n) * W + col] = cok ? M[o][k] : mk<T>(0, 0);
        }
        __syncthreads();
        col_fft<T, W, NT, MAXE, true, N>(buf, a.plan, tws);
        cpx<T>* out = a.out + o * a.out_fs + ob;
        cpx<T> ov[MAXE];  // LDS reads first, then the stores
#pragma unroll
        for (int k = 0; k < MAXE; ++k) {
          const int r = r0 + k * RSTEP;
          ov[k] = buf[((FULL || r < n) ? r : 0) * W + col];
        }
        if (cok) {
#pragma unroll
          for (int k = 0; k < MAXE; ++k) {
            const int r = r0 + k * RSTEP;
            if (FULL || r < n) st_stream(out + (long long)r * a.ld + c, ov[k]);
          }
        }
        __syncthreads();
      };
      static_for<0, 3>([&](auto oc) { mstep(oc); });
    }
  } else if constexpr (MODE == COL_INV_WZ && PAIR) {
    // COL_INV_WZ below with two columns per lane (same outputs, order and loads)
    // on the lane's own rows rp + 64 m (m = 0..7) of fft512_reg:
    // the band rows (K = 170) are m = 0, 1, 6, 7, m = 2 when rp <= 42 and m = 5
    // when rp >= 22 (band slot e = 0..5 for m = 0, 1, 2, 5, 6, 7), band index
    // rp + 64 m (m <= 2) or rp + 64 m - 171 (m >= 5)
    constexpr int WP = W / 2;
    cpx2f RA[6], RB[6];
    // buffer loads (a field of a z slab is below 2^31 bytes): rows out of the
    // band and column pairs wholly in the kx padding or past the last column
    // load zeros with no memory traffic
    auto load_into = [&](int lq, cpx2f(&R)[6]) __attribute__((always_inline)) {
      const int tq = opaque((int)threadIdx.x);
      const int cq = blockIdx.x * W + 2 * (tq % WP), rq = tq / WP;
      const __amdgpu_buffer_rsrc_t rin = buf_rsrc(reinterpret_cast<const cpx<float>*>(a.in) + lq * a.in_fs,
                                                  (long long)a.in_fs * 8);
      const bool cin = cq < a.C && (cq % a.kxp) < a.kx1;
      const unsigned base = (unsigned)(ib + cq) * 8u;
#pragma unroll
      for (int e = 0; e < 6; ++e) {
        const int m = e < 3 ? e : e + 2;
        const bool inb = cin && ((m == 2) ? rq <= 42 : (m == 5) ? rq >= 22 : true);
        const int i = m <= 2 ? rq + 64 * m : rq + 64 * m - 171;
        R[e] = ld_buf2(rin, inb ? base + (unsigned)(i * a.ld) * 8u : kOOB);
      }
    };
    auto step = [&](auto oc) __attribute__((always_inline)) {
      constexpr int o = decltype(oc)::value;
      constexpr int fo = (o == 2) ? 5 : (o > 2) ? o - 1 : o;
      constexpr int src = (o == 1 || o == 4) ? 1 : (o == 2) ? 2 : 0;
      constexpr int lq = (o == 0) ? 1 : (o == 2) ? 2 : (o == 3) ? 3 : (o == 4) ? 4 : -1;
      constexpr bool to_b = (o == 0 || o == 3);
      const int tid = opaque((int)threadIdx.x);
      const int cp = tid % WP, rp = tid / WP, c = blockIdx.x * W + 2 * cp;
      const bool ok0 = c < a.C && (c % a.kxp) < a.kx1, ok1 = c + 1 < a.C && ((c + 1) % a.kxp) < a.kx1;
      const float kx0 = (float)a.kfx * (float)(c % a.kxp), kx1 = kx0 + (float)a.kfx;
      const bool in2 = rp <= 42, in5 = rp >= 22;
      cpx<float> v0[8], v1[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        v0[m] = mk<float>(0, 0);
        v1[m] = mk<float>(0, 0);
      }
      static_for<0, 6>([&](auto ec) __attribute__((always_inline)) {
        constexpr int e = decltype(ec)::value, m = e < 3 ? e : e + 2;
        cpx2f val = (src == 1) ? RB[e] : RA[e];
        if constexpr (src == 2) {  // wz = i (kx uy - ky ux)
          const int i = m <= 2 ? rp + 64 * m : rp + 64 * m - 171;
          const float krow = (float)a.kfy * (float)band_mode(i, K);
          const cpx<float> t0 = scl(RB[e].a, kx0) - scl(RA[e].a, krow);
          const cpx<float> t1 = scl(RB[e].b, kx1) - scl(RA[e].b, krow);
          val = cpx2f{mk<float>(-t0.im, t0.re), mk<float>(-t1.im, t1.re)};
        }
        const bool inb = (m == 2) ? in2 : (m == 5) ? in5 : true;
        // component selects (a select of the whole pair keeps the array in memory)
        const bool k0 = ok0 && inb, k1 = ok1 && inb;
        v0[m] = mk<float>(k0 ? val.a.re : 0.f, k0 ? val.a.im : 0.f);
        v1[m] = mk<float>(k1 ? val.b.re : 0.f, k1 ? val.b.im : 0.f);
      });
      if constexpr (lq >= 0) {  // in flight during the transform
        if constexpr (to_b) {
          asm volatile("" ::: "memory");  // keeps the two load sites apart
          load_into(lq, RB);
        } else {
          load_into(lq, RA);
        }
      }
      fft512_reg<float, W, true>(v0, v1, reinterpret_cast<cpx<float>*>(buf), reinterpret_cast<const cpx<float>*>(tws));
      // unconditional stores of whole 128-byte row segments (columns out of the
      // band, padding included, carry zeros; the launcher keeps the workgroup's
      // columns within the row pitch): a store under a branch makes the next
      // wait for the prefetched field wait for these stores as well, and
      // dropping the padding columns' stores leaves partial lines (measured
      // 0.70 -> 0.73 ms)
      const __amdgpu_buffer_rsrc_t rout =
          buf_rsrc(reinterpret_cast<cpx<float>*>(a.out) + fo * a.out_fs, (long long)a.out_fs * 8);
      const unsigned base = (unsigned)(ob + c) * 8u;
#pragma unroll
      for (int m = 0; m < 8; ++m) st_buf2(rout, base + (unsigned)((rp + 64 * m) * a.ld) * 8u, cpx2f{v0[m], v1[m]});
    };
    load_into(0, RA);
    static_for<0, 6>([&](auto oc) { step(oc); });
  } else if constexpr (MODE == COL_INV_CURL5 || MODE == COL_INV_WZ) {
    // Stored fields of the forward step.  omega_z = i (kx uy - ky ux) needs no z
    // derivative, so the z pass (COL_INV_CURL5) stores ux, uy, uz, wx, wy and the
    // y pass (COL_INV_WZ) forms wz from ux, uy on the way.  Two register sets A,
    // B; the load for output o + 1 is issued right after output o is in LDS so
    // that it is in flight during that output's transform:
    //  z pass (output: value, [load issued]): ux:A [B = uz]  wy:i(kz A - kx B)
    //         uz:B [A = uy]  wx:i(ky B - kz A)  uy:A           3 loads, 5 outputs
    //  y pass: ux:A [B = uy]  uy:B  wz:i(kx B - ky A) [A = uz]  uz:A [B = wx]
    //         wx:B [A = wy]  wy:A                              5 loads, 6 outputs
    // The outputs are generated at compile time (one code path per output), so
    // that no register set is merged across branches: a merge copies the
    // registers and has to wait for loads still in flight.
    constexpr bool Z5 = (MODE == COL_INV_CURL5);
    cpx<T> RA[MAXO], RB[MAXO];
    auto load_into = [&](int lq, cpx<T>(&R)[MAXO]) {
      const int tq = opaque_tid<NT>();
      const int cq = blockIdx.x * W + tq % W, rq = tq / W;
      // unconditional loads (clamped rows and columns), zeroed when written to
      // LDS: a load under a branch would also be waited for where the branches join
      const cpx<T>* in = a.in + lq * a.in_fs + ib + (cq < a.C ? cq : 0);
#pragma unroll
      for (int k = 0; k < MAXO; ++k) {
        const int i = rq + k * RSTEP;
        R[k] = ld_stream(in + (long long)(i < nb ? i : 0) * a.ld);
      }
    };
    auto step = [&](auto oc) {
      constexpr int o = decltype(oc)::value;
      // output field, source (0: A, 1: B, 2: cross term), next load and its set
      constexpr int fo = Z5 ? ((o == 1) ? 4 : (o == 3) ? 3 : (o == 4) ? 1 : o) : ((o == 2) ? 5 : (o > 2) ? o - 1 : o);
      constexpr int src = Z5 ? ((o == 2) ? 1 : (o == 1 || o == 3) ? 2 : 0) : ((o == 1 || o == 4) ? 1 : (o == 2) ? 2 : 0);
      constexpr int lq = Z5 ? ((o == 0) ? 2 : (o == 2) ? 1 : -1) : ((o == 0) ? 1 : (o == 2) ? 2 : (o == 3) ? 3 : (o == 4) ? 4 : -1);
      constexpr bool to_b = Z5 ? (o == 0) : (o == 0 || o == 3);
      const int tid = opaque_tid<NT>();
      const int col = tid % W, r0 = tid / W, c = blockIdx.x * W + col;
      const bool cok = c < a.C && (c % a.kxp) < a.kx1;
      const int ix = c % a.kxp, iy = c / a.kxp;
      const T kx = a.kfx * (T)ix;
      const T ky = Z5 ? a.kfy * (T)band_mode(iy, a.Ky) : (T)0;
#pragma unroll
      for (int k = 0; k < MAXE; ++k) {
        const int r = r0 + k * RSTEP;
        if (r > K && r < n - K) buf[r * W + col] = mk<T>(0, 0);
      }
#pragma unroll
      for (int k = 0; k < MAXO; ++k) {
        const int i = r0 + k * RSTEP;
        if (i < nb) {
          cpx<T> val = (src == 1) ? RB[k] : RA[k];
          if constexpr (src == 2) {
            // per-row wavenumber: kz in the z pass, ky in the y pass
            const T krow = (Z5 ? a.kfz : a.kfy) * (T)band_mode(i, K);
            cpx<T> t;
            if constexpr (Z5 && o == 1) t = scaled_diff(RA[k], krow, RB[k], kx);  // wy: kz ux - kx uz
            else if constexpr (Z5) t = scaled_diff(RB[k], ky, RA[k], krow);       // wx: ky uz - kz uy
            else t = scl(RB[k], kx) - scl(RA[k], krow);                          // wz: kx uy - ky ux
            val = mk<T>(-t.im, t.re);  // i t
          }
          buf[band_to_row(i, K, n) * W + col] = cok ? val : mk<T>(0, 0);
        }
      }
      __syncthreads();
      if constexpr (lq >= 0) {
        if constexpr (to_b) load_into(lq, RB);
        else load_into(lq, RA);
      }
      col_fft<T, W, NT, MAXE, true, N>(buf, a.plan, tws);
      cpx<T>* out = a.out + fo * a.out_fs + ob;
      // every LDS read first, then the stores: reading each value just before
      // its store would put an LDS round trip in front of every store
      cpx<T> ov[MAXE];
#pragma unroll
      for (int k = 0; k < MAXE; ++k) {
        const int r = r0 + k * RSTEP;
        ov[k] = buf[((FULL || r < n) ? r : 0) * W + col];
      }
      if (N == 512 || cok) {  // 512 points: unconditional stores, as in COL_INV_PLAIN
#pragma unroll
        for (int k = 0; k < MAXE; ++k) {
          const int r = r0 + k * RSTEP;
          if (FULL || r < n) st_stream(out + (long long)r * a.ld + c, ov[k]);
        }
      }
      __syncthreads();
    };
    load_into(0, RA);
    step(std::integral_constant<int, 0>{});
    step(std::integral_constant<int, 1>{});
    step(std::integral_constant<int, 2>{});
    step(std::integral_constant<int, 3>{});
    step(std::integral_constant<int, 4>{});
    if constexpr (!Z5) step(std::integral_constant<int, 5>{});
  } else if constexpr (MODE == COL_FWD_PLAIN && PAIR) {
    // y forward (P4 and the helper transforms) with two columns per lane, on the
    // lane's own rows rp + 64 m of fft512_reg; band rows out as in
    // COL_INV_WZ above
    constexpr int WP = W / 2;
    const int nfield = a.nf;
    cpx2f tmp[8];
    // buffer accesses (a field of a y slab is below 2^31 bytes): column pairs
    // wholly in the kx padding or past the last column load zeros and are not
    // stored, nor are rows out of the y band
    auto load_field = [&](int f) __attribute__((always_inline)) {
      const int tq = opaque((int)threadIdx.x);
      const int cq = blockIdx.x * W + 2 * (tq % WP), rq = tq / WP;
      const __amdgpu_buffer_rsrc_t rin = buf_rsrc(reinterpret_cast<const cpx<float>*>(a.in) + f * a.in_fs,
                                                  (long long)a.in_fs * 8);
      const bool cin = cq < a.C && (cq % a.kxp) < a.kx1;
      const unsigned base = (unsigned)(ib + cq) * 8u;
#pragma unroll
      for (int m = 0; m < 8; ++m) tmp[m] = ld_buf2(rin, cin ? base + (unsigned)((rq + 64 * m) * a.ld) * 8u : kOOB);
    };
    auto field = [&](int f, bool prefetch) __attribute__((always_inline)) {
      cpx<float> v0[8], v1[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        v0[m] = tmp[m].a;
        v1[m] = tmp[m].b;
      }
      if (prefetch) load_field(f + 1);  // in flight during the transform
      fft512_reg<float, W, false>(v0, v1, reinterpret_cast<cpx<float>*>(buf), reinterpret_cast<const cpx<float>*>(tws));
      const int tid = opaque((int)threadIdx.x);
      const int cp = tid % WP, rp = tid / WP, c = blockIdx.x * W + 2 * cp;
      const __amdgpu_buffer_rsrc_t rout =
          buf_rsrc(reinterpret_cast<cpx<float>*>(a.out) + f * a.out_fs, (long long)a.out_fs * 8);
      const bool cin = c < a.C && (c % a.kxp) < a.kx1;
      const unsigned base = (unsigned)(ob + c) * 8u;
      const float sc = (float)a.scale;
      // stores without a branch: rows out of the band (m = 2 with rp > 42,
      // m = 5 with rp < 22) and padding pairs take the dropped offset (storing
      // the padding pairs as well, for whole 128-byte lines, measured the same)
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        if (m == 3 || m == 4) continue;
        const bool inb = cin && ((m == 2) ? rp <= 42 : (m == 5) ? rp >= 22 : true);
        const int i = m <= 2 ? rp + 64 * m : rp + 64 * m - 171;
        st_buf2(rout, inb ? base + (unsigned)(i * a.ld) * 8u : kOOB, cpx2f{scl(v0[m], sc), scl(v1[m], sc)});
      }
    };
    load_field(0);
    if (nfield == 3) {
      field(0, true);
      field(1, true);
      field(2, false);
    } else if (nfield == 6) {
      field(0, true);
      field(1, true);
      field(2, true);
      field(3, true);
      field(4, true);
      field(5, false);
    } else {
      for (int f = 0; f < nfield; ++f) {
        if (f > 0) load_field(f);
        field(f, false);
      }
    }
  } else {
    // forward modes: all n rows in, band rows out
    const int nfield = (MODE == COL_FWD_PLAIN || MODE == COL_FWD_ACC) ? a.nf : 3;
    // COL_FWD_UPDATE_Z at 512 points (FP32): the update and the next step's z
    // inverse work on the thread's rows r0 + 32 m (fft512_reg's one-column
    // slots, m = s + 2 r); the stash of the first two components follows that
    // layout (band slot e = 0..11 for m = 0..5, 10..15).  The forward
    // transforms run their first stage on the loaded registers and the other
    // two in LDS: all on registers, the three components and the prefetch
    // would not fit in 128 VGPRs
    constexpr bool REGZ = MODE == COL_FWD_UPDATE_Z && N == 512 && sizeof(T) == 4 && RSTEP == 32 && MAXE == 16;
    constexpr int NST = REGZ ? 12 : MAXO;
    cpx<T> st[2][NST];
    cpx<T> tmp[MAXE];
    // rows of field f into tmp: unconditional loads (clamped row and column);
    // columns outside the band are transformed but never stored
    auto load_field = [&](int f) __attribute__((always_inline)) {
      const int tq = opaque_tid<NT>();
      const int cq = blockIdx.x * W + tq % W, rq = tq / W;
      const cpx<T>* in = a.in + f * a.in_fs + ib + (cq < a.C ? cq : 0);
#pragma unroll
      for (int k = 0; k < MAXE; ++k) {
        const int r = rq + k * RSTEP;
        tmp[k] = ld_stream(in + (long long)((FULL || r < n) ? r : 0) * a.ld);
      }
    };
    // field f from tmp: LDS, transform, band rows out (or stashed); with
    // prefetch, the loads of field f + 1 are in flight during the transform
    auto field = [&](int f, bool prefetch) __attribute__((always_inline)) {
      const int tid = opaque_tid<NT>();
      const int col = tid % W, r0 = tid / W, c = blockIdx.x * W + col;
      if constexpr (REGZ) {
        // the loaded rows r0 + 32 m are the inputs of the span-1 butterflies
        // j = r0 and j = r0 + 32 (m = s + 2 r): that stage on registers, its
        // outputs (rows 8 j + r) to LDS, the two other stages there
        cpx<T> v0[8], v1[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          v0[r] = tmp[2 * r];
          v1[r] = tmp[2 * r + 1];
        }
        Bfly<T, 8, -1>::run(v0);
        Bfly<T, 8, -1>::run(v1);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          buf[(8 * r0 + r) * W + col] = v0[r];
          buf[(8 * (r0 + 32) + r) * W + col] = v1[r];
        }
        __syncthreads();
        if (prefetch) load_field(f + 1);
        fft_stage<T, 8, W, W, NT, MAXE, false>(buf, 512, 8, tws);
        fft_stage<T, 8, W, W, NT, MAXE, false>(buf, 512, 64, tws);
      } else {
#pragma unroll
        for (int k = 0; k < MAXE; ++k) {
          const int r = r0 + k * RSTEP;
          if (FULL || r < n) buf[r * W + col] = tmp[k];
        }
        __syncthreads();
        if (prefetch) load_field(f + 1);
        col_fft<T, W, NT, MAXE, false, N>(buf, a.plan, tws);
      }
      if (MODE == COL_FWD_PLAIN) {
        cpx<T>* out = a.out + f * a.out_fs + ob;
        cpx<T> ov[MAXO];  // LDS reads first, then the stores
#pragma unroll
        for (int k = 0; k < MAXO; ++k) {
          const int i = r0 + k * RSTEP;
          ov[k] = buf[band_to_row(i < nb ? i : 0, K, n) * W + col];
        }
        if (cok) {
#pragma unroll
          for (int k = 0; k < MAXO; ++k) {
            const int i = r0 + k * RSTEP;
            if (i < nb) st_stream(out + (long long)i * a.ld + c, scl(ov[k], a.scale));
          }
        }
        __syncthreads();
      } else if (MODE == COL_FWD_ACC) {
        cpx<T>* out = a.out + f * a.cfs;
        const T m = a.scale * (T)((c % a.kxp) == 0 ? 1 : 2);
        // all loads before the stores (a load after a store that may alias it
        // waits for the store)
        cpx<T> ov[MAXO];
        const int cl = c < a.C ? c : 0;
#pragma unroll
        for (int k = 0; k < MAXO; ++k) {
          const int i = r0 + k * RSTEP;
          ov[k] = out[(long long)(i < nb ? i : 0) * a.ld + cl];
        }
        if (cok) {
#pragma unroll
          for (int k = 0; k < MAXO; ++k) {
            const int i = r0 + k * RSTEP;
            if (i < nb) out[(long long)i * a.ld + c] = ov[k] + scl(buf[band_to_row(i, K, n) * W + col], m);
          }
        }
        __syncthreads();
      } else if (REGZ && f < 2) {
        if (f == 0) {
#pragma unroll
          for (int e = 0; e < NST; ++e) st[0][e] = scl(buf[(r0 + 32 * band_slot512(e)) * W + col], a.scale);
        } else {
#pragma unroll
          for (int e = 0; e < NST; ++e) st[1][e] = scl(buf[(r0 + 32 * band_slot512(e)) * W + col], a.scale);
        }
        __syncthreads();
      } else if (f < 2) {
        // one loop per stash (a run-time register index would go to scratch)
        if (f == 0) {
#pragma unroll
          for (int k = 0; k < MAXO; ++k) {
            const int i = r0 + k * RSTEP;
            if (i < nb) st[0][k] = scl(buf[band_to_row(i, K, n) * W + col], a.scale);
          }
        } else {
#pragma unroll
          for (int k = 0; k < MAXO; ++k) {
            const int i = r0 + k * RSTEP;
            if (i < nb) st[1][k] = scl(buf[band_to_row(i, K, n) * W + col], a.scale);
          }
        }
        __syncthreads();
      }
    };
    if constexpr (MODE != COL_FWD_PLAIN && MODE != COL_FWD_ACC) {
      // three fields in a compile-time sequence: the prefetched registers are
      // never merged across branches (a merge would wait for the loads)
      load_field(0);
      field(0, true);
      field(1, true);
      field(2, false);
    } else if constexpr (N == 512) {
      load_field(0);
      if (nfield == 3) {
        field(0, true);
        field(1, true);
        field(2, false);
      } else if (nfield == 6) {
        field(0, true);
        field(1, true);
        field(2, true);
        field(3, true);
        field(4, true);
        field(5, false);
      } else {
        for (int f = 0; f < nfield; ++f) {
          if (f > 0) load_field(f);
          field(f, false);
        }
      }
    } else {
      for (int f = 0; f < nfield; ++f) {
        load_field(f);
        field(f, false);
      }
    }
    if constexpr (MODE == COL_FWD_ACC_CURL) {
      const int ix = c % a.kxp, iy = c / a.kxp;
      const T kx = a.kfx * (T)ix;
      const T ky = a.kfy * (T)band_mode(iy, a.Ky);
      const T m = (T)(ix == 0 ? 1 : 2);  // a.scale is already in st and in v2 below
#pragma unroll
      for (int k = 0; k < MAXO; ++k) {
        const int i = r0 + k * RSTEP;
        if (cok && i < nb) {
          const T kz = a.kfz * (T)band_mode(i, K);
          const cpx<T> v0 = st[0][k], v1 = st[1][k];
          const cpx<T> v2 = scl(buf[band_to_row(i, K, n) * W + col], a.scale);
          const cpx<T> t0 = scl(v2, ky) - scl(v1, kz);  // (i k x v) = i t
          const cpx<T> t1 = scl(v0, kz) - scl(v2, kx);
          const cpx<T> t2 = scl(v1, kx) - scl(v0, ky);
          const long long idx = (long long)i * a.ld + c;
          a.out[idx] = a.out[idx] + scl(mk<T>(-t0.im, t0.re), m);
          a.out[a.cfs + idx] = a.out[a.cfs + idx] + scl(mk<T>(-t1.im, t1.re), m);
          a.out[2 * a.cfs + idx] = a.out[2 * a.cfs + idx] + scl(mk<T>(-t2.im, t2.re), m);
        }
      }
    }
    if constexpr (MODE == COL_FWD_SPONGE) {
      // T_hat = -(1/C_sp) i k x S_hat / |k|^2 (zero at k = 0), S the masked vorticity
      const int ix = c % a.kxp, iy = c / a.kxp;
      const T kx = a.kfx * (T)ix;
      const T ky = a.kfy * (T)band_mode(iy, a.Ky);
#pragma unroll
      for (int k = 0; k < MAXO; ++k) {
        const int i = r0 + k * RSTEP;
        if (cok && i < nb) {
          const T kz = a.kfz * (T)band_mode(i, K);
          const cpx<T> v0 = st[0][k], v1 = st[1][k];
          const cpx<T> v2 = scl(buf[band_to_row(i, K, n) * W + col], a.scale);
          const T k2 = kx * kx + ky * ky + kz * kz;
          const T f = k2 > (T)0 ? -a.csp_inv / k2 : (T)0;
          const cpx<T> t0 = scl(v2, ky) - scl(v1, kz);  // i k x v = i t
          const cpx<T> t1 = scl(v0, kz) - scl(v2, kx);
          const cpx<T> t2 = scl(v1, kx) - scl(v0, ky);
          const long long idx = (long long)i * a.ld + c;
          a.out[idx] = scl(mk<T>(-t0.im, t0.re), f);
          a.out[a.cfs + idx] = scl(mk<T>(-t1.im, t1.re), f);
          a.out[2 * a.cfs + idx] = scl(mk<T>(-t2.im, t2.re), f);
        }
      }
    }
    constexpr bool UPD = (MODE == COL_FWD_UPDATE || MODE == COL_FWD_UPDATE_Z);
    if constexpr (REGZ) {
      // band rows of the thread (K = 170): m <= 4 and m >= 11 always, m = 5 when
      // r0 <= 10, m = 10 when r0 >= 22, never m = 6..9; band index r0 + 32 m
      // (m <= 5) or r0 + 32 m - 171 (m >= 10), a valid compact row for every slot
      // u_x, u_z of u^{n+1} (zero outside the band and in columns out of it);
      // u_y is read back from u_hat when the inverse transforms need it (all
      // three in registers next to a transform would not fit in 128 VGPRs)
      cpx<T> U[3][NST];
      const int ix = c % a.kxp, iy = c / a.kxp;
      const T kx = a.kfx * (T)ix;
      const T ky = a.kfy * (T)band_mode(iy, a.Ky);
      const double d_n = a.sc->dt[a.cur];
      const double d_p = a.sc->dt[a.cur ^ 1];
      const T dtn = (T)d_n, dtp = (T)d_p;
      T c1, c2;
      if (a.first) {
        c1 = dtn;
        c2 = 0;
      } else {
        const double xi = d_n / d_p;
        c1 = (T)(d_n * (1.0 + 0.5 * xi));
        c2 = (T)(d_n * 0.5 * xi);
      }
      const bool b5 = r0 <= 10, b10 = r0 >= 22;
      const int cl = c < a.C ? c : 0;
      // the state through buffer resources bounded by a compact field (far
      // below 2^31 bytes at 512 points): slots out of the band, and the previous
      // nonlinear term on the first step, load zeros with no memory traffic
      constexpr int kOut = 1 << 28;  // an element index beyond every compact field
      // band slots in chunks of two: every load of a chunk before its first
      // store (a load after a store that may alias it waits for that store)
      constexpr int KCZ = 2;
      static_for<0, 12 / KCZ>([&](auto cc) __attribute__((always_inline)) {
        constexpr int e0 = KCZ * decltype(cc)::value;
        cpx<T> uo[KCZ][3], po[KCZ][3];
        const int r0l = opaque(r0);  // addresses per chunk, not for all chunks ahead
#pragma unroll
        for (int kk = 0; kk < KCZ; ++kk) {
          const int m = band_slot512(e0 + kk);
          const bool inb = (m <= 4 || m >= 11) ? true : (m == 5) ? b5 : b10;
          const int idx = (m <= 5 ? r0l + 32 * m : r0l + 32 * m - 171) * a.ld + cl;
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            uo[kk][q] = ld_band<T>(band_rsrc(a.uh + q * a.cfs, (int)a.cfs), inb ? idx : kOut);
            po[kk][q] = ld_band<T>(band_rsrc(a.nh + q * a.cfs, (int)a.cfs), (inb && !a.first) ? idx : kOut);
          }
        }
        // every lane computes its slots; slots out of the band and columns out
        // of it take the dropped offset of the buffer stores (no branch around
        // the stores) and leave zeros in U
#pragma unroll
        for (int kk = 0; kk < KCZ; ++kk) {
          const int e = e0 + kk, m = band_slot512(e);
          const bool ok = cok && ((m <= 4 || m >= 11) ? true : (m == 5) ? b5 : b10);
          const int i = m <= 5 ? r0l + 32 * m : r0l + 32 * m - 171;
          const T kz = a.kfz * (T)band_mode(i, K);
          cpx<T> n0 = st[0][e], n1 = st[1][e];
          cpx<T> n2 = scl(buf[(r0l + 32 * m) * W + col], a.scale);
          const T k2 = kx * kx + ky * ky + kz * kz;
          const int idx = ok ? i * a.ld + c : kOut;
          if (a.tsp) {  // vorticity sponge (solenoidal: the projection keeps it)
            n0 = n0 + ld_band<T>(band_rsrc(a.tsp, (int)a.cfs), idx);
            n1 = n1 + ld_band<T>(band_rsrc(a.tsp + a.cfs, (int)a.cfs), idx);
            n2 = n2 + ld_band<T>(band_rsrc(a.tsp + 2 * a.cfs, (int)a.cfs), idx);
          }
          const T ik2 = k2 > (T)0 ? (T)1 / k2 : (T)0;  // the projection is the identity at k = 0
          const cpx<T> sp = scl(scl(n0, kx) + scl(n1, ky) + scl(n2, kz), ik2);
          n0 = n0 - scl(sp, kx);
          n1 = n1 - scl(sp, ky);
          n2 = n2 - scl(sp, kz);
          if (a.pi) st_band<T>(band_rsrc(a.pi, (int)a.cfs), idx, mk<T>(sp.im, -sp.re));  // -i (k.N') / |k|^2
          const T en = dev_exp<T>(-a.nu * k2 * dtn);
          const T c2e = c2 * en * dev_exp<T>(-a.nu * k2 * dtp);
          const cpx<T> nn[3] = {n0, n1, n2};
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            const cpx<T> u1 = scl(uo[kk][q] + scl(nn[q], c1), en);
            // first step: Euler, the stored previous term is not read
            const cpx<T> u2 = a.first ? u1 : u1 - scl(po[kk][q], c2e);
            st_band<T>(band_rsrc(a.uh + q * a.cfs, (int)a.cfs), idx, u2);
            st_band<T>(band_rsrc(a.nh + q * a.cfs, (int)a.cfs), idx, nn[q]);
            if (q != 1) U[q][e] = mk<T>(ok ? u2.re : (T)0, ok ? u2.im : (T)0);
          }
        }
      });
      // the first pass of the next step on the same columns: z inverse of u^{n+1}
      // and of omega_x, omega_y = (i k x u)_x,y in the order of COL_INV_CURL5
      // (ux, wy, uz, wx, uy), from registers
      static_for<0, 5>([&](auto oc) __attribute__((always_inline)) {
        constexpr int o = decltype(oc)::value;
        constexpr int fo = (o == 1) ? 4 : (o == 4) ? 1 : o;
        cpx<T> v0[8], v1[8];
        const int r0l = opaque(r0);
        if constexpr (o == 2) {
          // u_y back from u_hat (this thread's own stores above: a load after a
          // store to the same address from the same thread returns the stored
          // value), in flight during this transform; u_x is no longer needed
#pragma unroll
          for (int e = 0; e < NST; ++e) {
            const int m = band_slot512(e);
            const bool inb = (m <= 4 || m >= 11) ? true : (m == 5) ? b5 : b10;
            U[1][e] = ld_band<T>(band_rsrc(a.uh + a.cfs, (int)a.cfs),
                                 inb ? (m <= 5 ? r0l + 32 * m : r0l + 32 * m - 171) * a.ld + cl : kOut);
          }
        }
        static_for<0, 16>([&](auto mc) __attribute__((always_inline)) {
          constexpr int m = decltype(mc)::value;
          cpx<T> val = mk<T>(0, 0);
          if constexpr (m <= 5 || m >= 10) {
            constexpr int e = m <= 5 ? m : m - 4;
            // u_y as read back (outputs 3, 4): zero outside the band and in
            // columns out of it
            auto uy = [&]() __attribute__((always_inline)) {
              const bool yok = cok && ((m <= 4 || m >= 11) ? true : (m == 5) ? b5 : b10);
              return mk<T>(yok ? U[1][e].re : (T)0, yok ? U[1][e].im : (T)0);
            };
            if constexpr (o == 0) val = U[0][e];
            else if constexpr (o == 2) val = U[2][e];
            else if constexpr (o == 4) val = uy();
            else {
              const T kz = a.kfz * (T)band_mode(m <= 5 ? r0l + 32 * m : r0l + 32 * m - 171, K);
              // wy = i (kz ux - kx uz), wx = i (ky uz - kz uy)
              cpx<T> t;
              if constexpr (o == 1) t = scaled_diff(U[0][e], kz, U[2][e], kx);
              else t = scaled_diff(U[2][e], ky, uy(), kz);
              val = mk<T>(-t.im, t.re);
            }
          }
          if constexpr (m & 1) v1[m >> 1] = val;
          else v0[m >> 1] = val;
        });
        fft512_reg<T, W, true, true>(v0, v1, buf, tws);
        cpx<T>* out = a.zout + fo * a.zout_fs;
        // unconditional stores (columns out of the band carry zeros; whole
        // workgroups of columns only): a store under a branch makes the next
        // wait for a prefetched load wait for the stores as well
#pragma unroll
        for (int m = 0; m < 16; ++m) st_stream(at_u32(out, (r0 + 32 * m) * a.ld + c), (m & 1) ? v1[m >> 1] : v0[m >> 1]);
      });
    } else if constexpr (MODE == COL_FWD_PROJECT || UPD) {
      // COL_FWD_UPDATE_Z keeps the new velocity of the thread's rows for the
      // z inverse of the next step
      cpx<T> U[3][MAXO];
      const int ix = c % a.kxp, iy = c / a.kxp;
      const T kx = a.kfx * (T)ix;
      const T ky = a.kfy * (T)band_mode(iy, a.Ky);
      T dtn = 0, dtp = 0, c1 = 0, c2 = 0;
      if constexpr (UPD) {
        const double d_n = a.sc->dt[a.cur];
        const double d_p = a.sc->dt[a.cur ^ 1];
        dtn = (T)d_n;
        dtp = (T)d_p;
        if (a.first) {
          c1 = dtn;
          c2 = 0;
        } else {
          const double xi = d_n / d_p;
          c1 = (T)(d_n * (1.0 + 0.5 * xi));
          c2 = (T)(d_n * 0.5 * xi);
        }
      }
      // Rows in chunks of KC: every load of a chunk is issued before its first
      // store.  The stores may alias the loads as far as the compiler can tell,
      // so a load placed after a store waits for that store's round trip.
      constexpr int KC = sizeof(T) == 4 ? 3 : 1;
      const int cl = c < a.C ? c : 0;  // clamped column of the unconditional loads
#pragma unroll
      for (int k0 = 0; k0 < MAXO; k0 += KC) {
        cpx<T> uo[KC][3], po[KC][3];
        if constexpr (UPD) {
#pragma unroll
          for (int kk = 0; kk < KC; ++kk) {
            const int k = k0 + kk;
            if (k < MAXO) {
              const int i = r0 + k * RSTEP;
              const long long idx = (long long)(i < nb ? i : 0) * a.ld + cl;
#pragma unroll
              for (int q = 0; q < 3; ++q) {
                uo[kk][q] = ld_state(a.uh + q * a.cfs + idx);
                po[kk][q] = ld_state(a.nh + q * a.cfs + idx);  // unused on the first step
              }
            }
          }
        }
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
          const int k = k0 + kk;
          if (k >= MAXO) break;
          const int i = r0 + k * RSTEP;
          if (cok && i < nb) {
            const T kz = a.kfz * (T)band_mode(i, K);
            cpx<T> n0 = st[0][k], n1 = st[1][k];
            cpx<T> n2 = scl(buf[band_to_row(i, K, n) * W + col], a.scale);
            const T k2 = kx * kx + ky * ky + kz * kz;
            const long long idx = (long long)i * a.ld + c;
            if constexpr (UPD) {
              if (a.tsp) {  // vorticity sponge (solenoidal: the projection keeps it)
                n0 = n0 + a.tsp[idx];
                n1 = n1 + a.tsp[a.cfs + idx];
                n2 = n2 + a.tsp[2 * a.cfs + idx];
              }
            }
            if (k2 > (T)0) {
              const T ik2 = (T)1 / k2;
              cpx<T> sp = scl(scl(n0, kx) + scl(n1, ky) + scl(n2, kz), ik2);
              n0 = n0 - scl(sp, kx);
              n1 = n1 - scl(sp, ky);
              n2 = n2 - scl(sp, kz);
              if (a.pi) a.pi[idx] = mk<T>(sp.im, -sp.re);  // -i (k.N') / |k|^2
            } else if (a.pi) {
              a.pi[idx] = mk<T>(0, 0);
            }
            if constexpr (MODE == COL_FWD_PROJECT) {
              if (a.out) {  // NULL: the total pressure only
                a.out[idx] = n0;
                a.out[a.cfs + idx] = n1;
                a.out[2 * a.cfs + idx] = n2;
              }
            } else {
              const T en = dev_exp<T>(-a.nu * k2 * dtn);
              const T c2e = c2 * en * dev_exp<T>(-a.nu * k2 * dtp);
              const cpx<T> nn[3] = {n0, n1, n2};
#pragma unroll
              for (int q = 0; q < 3; ++q) {
                const cpx<T> u1 = scl(uo[kk][q] + scl(nn[q], c1), en);
                // first step: Euler, the stored previous term is not read
                const cpx<T> u2 = a.first ? u1 : u1 - scl(po[kk][q], c2e);
                st_stream(a.uh + q * a.cfs + idx, u2);
                st_stream(a.nh + q * a.cfs + idx, nn[q]);
                if constexpr (MODE == COL_FWD_UPDATE_Z) U[q][k] = u2;
              }
            }
          }
        }
      }
      if constexpr (MODE == COL_FWD_UPDATE_Z) {
        // The first pass of the next step on the same columns: z inverse of
        // u^{n+1} and of omega_x, omega_y = (i k x u)_x,y, in the order of
        // COL_INV_CURL5 (ux, wy, uz, wx, uy), from registers instead of memory.
        __syncthreads();
        auto zstep = [&](auto oc) {
          constexpr int o = decltype(oc)::value;
          constexpr int fo = (o == 1) ? 4 : (o == 4) ? 1 : o;
          const int tid = opaque_tid<NT>();
          const int col = tid % W, r0 = tid / W, c = blockIdx.x * W + col;
          const bool cok = c < a.C && (c % a.kxp) < a.kx1;
#pragma unroll
          for (int k = 0; k < MAXE; ++k) {
            const int r = r0 + k * RSTEP;
            if (r > K && r < n - K) buf[r * W + col] = mk<T>(0, 0);
          }
#pragma unroll
          for (int k = 0; k < MAXO; ++k) {
            const int i = r0 + k * RSTEP;
            if (i < nb) {
              cpx<T> val;
              if constexpr (o == 0) val = U[0][k];
              else if constexpr (o == 2) val = U[2][k];
              else if constexpr (o == 4) val = U[1][k];
              else {
                const T kz = a.kfz * (T)band_mode(i, K);
                // wy = i (kz ux - kx uz), wx = i (ky uz - kz uy)
                const cpx<T> t = (o == 1) ? scaled_diff(U[0][k], kz, U[2][k], kx) : scaled_diff(U[2][k], ky, U[1][k], kz);
                val = mk<T>(-t.im, t.re);
              }
              buf[band_to_row(i, K, n) * W + col] = cok ? val : mk<T>(0, 0);
            }
          }
          __syncthreads();
          col_fft<T, W, NT, MAXE, true, N>(buf, a.plan, tws);
          cpx<T>* out = a.zout + fo * a.zout_fs;
          cpx<T> ov[MAXE];  // LDS reads first, then the stores
#pragma unroll
          for (int k = 0; k < MAXE; ++k) {
            const int r = r0 + k * RSTEP;
            ov[k] = buf[((FULL || r < n) ? r : 0) * W + col];
          }
          if (cok) {
#pragma unroll
            for (int k = 0; k < MAXE; ++k) {
              const int r = r0 + k * RSTEP;
              if (FULL || r < n) st_stream(out + (long long)r * a.ld + c, ov[k]);
            }
          }
          __syncthreads();
        };
        zstep(std::integral_constant<int, 0>{});
        zstep(std::integral_constant<int, 1>{});
        zstep(std::integral_constant<int, 2>{});
        zstep(std::integral_constant<int, 3>{});
        zstep(std::integral_constant<int, 4>{});
      }
    }
  }
}

// ---------------------------------------------------------------------------
// x pass: real transforms along x, two real lines packed per complex signal
// ---------------------------------------------------------------------------
//
// LDS holds n rows of packed signals with a padded row stride (odd number of
// complex values against bank conflicts), then the twiddle table.

// Penalization at one grid point with the static plane on (max rule): the
// static solid's chi, u_s at plane index sidx, replaced by the wing's at
// sub-box cell `cell` (-1: outside the sub-box) where the wing's chi is larger.
// Subtracts (chi/eta)(u - u_s) from G and adds chi (u - u_s) to the force sums
// of the solid that wins (weighted by the static force weight).
template <typename T>
__device__ __forceinline__ void penalize_static(const XArgs<T>& a, long long cell, long long sidx, T ux, T uy, T uz,
                                                T& gx, T& gy, T& gz, double& f0, double& f1, double& f2, double& s0,
                                                double& s1, double& s2) {
  const long long plane = (long long)a.ny * a.n;
  T ch = a.st_chi[sidx], u0 = a.st_us[sidx], u1 = a.st_us[plane + sidx], u2 = a.st_us[2 * plane + sidx];
  bool wing = false;
  if (cell >= 0) {
    const T cw = a.chi[cell];
    if (cw > ch) {
      ch = cw;
      u0 = a.us[cell];
      u1 = a.us[a.bcells + cell];
      u2 = a.us[2 * a.bcells + cell];
      wing = true;
    }
  }
  if (ch != (T)0) {
    const T sx = ux - u0, sy = uy - u1, sz = uz - u2;
    const T ce = ch * a.inv_eta;
    gx -= ce * sx;
    gy -= ce * sy;
    gz -= ce * sz;
    if (wing) {
      f0 += (double)(ch * sx);
      f1 += (double)(ch * sy);
      f2 += (double)(ch * sz);
    } else {
      const T cwt = ch * a.st_w[sidx];
      s0 += (double)(cwt * sx);
      s1 += (double)(cwt * sy);
      s2 += (double)(cwt * sz);
    }
  }
}

// Fused pass: C2R of (u, omega) for L lines, G = u x omega - (chi/eta)(u - u_s),
// partial sums of the diagnostics, R2C of G truncated to the x band.  N != 0:
// the line length as a compile-time constant (its plan, band and index
// arithmetic; fft_n), N = 0: the run-time length and plan.
template <typename T, int L, int NT, int MAXE, bool ST, int N>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu((N == 800 && sizeof(T) == 4) ? 4 : 1)))
void xpass_fused(XArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  __shared__ double red[8 * (NT / 64)];
  constexpr int WI = 3 * L;      // inverse: pairs (ux,uy) (uz,wx) (wy,wz) per line
  constexpr int WF = 3 * L / 2;  // forward: (Gx,Gy) per line, (Gz,Gz') per line pair
  constexpr int RI = PadStride<WI>::value;
  constexpr int RF = PadStride<WF>::value;
  static_assert(L % 2 == 0, "L must be even");
  // per-thread slots of a line: XI along the band (K + 1 <= XI NT), XP along
  // the line (n <= XP NT); an instantiation serves n <= MAXE NT / (3 L)
  constexpr int NMAX = N ? N : MAXE * NT / (3 * L);
  constexpr int XI = ((NMAX - 1) / 3 + 1 + NT - 1) / NT;
  constexpr int XP = (NMAX + NT - 1) / NT;
  const int tid = threadIdx.x;
  const int n = N ? N : a.n, K = N ? (N - 1) / 3 : a.kx1 - 1, kx1 = K + 1;
  const int ngroups = a.nlines / L;
  cpx<T>* tws = buf + n * RI;
  for (int i = tid; i < n; i += NT) tws[i] = a.tw[i];
  double aF0 = 0, aF1 = 0, aF2 = 0, aE = 0, aM = 0, aS0 = 0, aS1 = 0, aS2 = 0;

  for (int g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const int tid = opaque_tid<NT>();
    const int line0 = g * L;
    // 1) Hermitian-extended packed spectra, signal s = 3 l + p: a wave-uniform
    //    line base per field and 32-bit offsets x (no 64-bit vector address
    //    arithmetic); every load issued before the LDS writes
    {
      cpx<T> A[WI][XI], B[WI][XI];
#pragma unroll
      for (int s = 0; s < WI; ++s) {
        const int l = s / 3, p = s % 3;
        const cpx<T>* ab = a.spec + (2 * p) * a.sfs + (long long)(line0 + l) * a.ld;
        const cpx<T>* bb = a.spec + (2 * p + 1) * a.sfs + (long long)(line0 + l) * a.ld;
#pragma unroll
        for (int k = 0; k < XI; ++k) {
          const int x = tid + k * NT;
          const int xc = x < kx1 ? x : 0;  // unconditional loads (see load512)
          A[s][k] = *at_u32(ab, xc);
          B[s][k] = *at_u32(bb, xc);
        }
      }
#pragma unroll
      for (int s = 0; s < WI; ++s) {
#pragma unroll
        for (int k = 0; k < XI; ++k) {
          const int x = tid + k * NT;
          if (x < kx1) {
            const cpx<T> av = A[s][k], bv = B[s][k];
            if (x == 0) {
              buf[s] = mk<T>(av.re, bv.re);
            } else {
              buf[x * RI + s] = mk<T>(av.re - bv.im, av.im + bv.re);
              buf[(n - x) * RI + s] = mk<T>(av.re + bv.im, bv.re - av.im);
            }
          }
        }
      }
      const int gap = n - 2 * K - 1;
      for (int it = tid; it < WI * gap; it += NT) {
        const int s = it % WI, x = K + 1 + it / WI;
        buf[x * RI + s] = mk<T>(0, 0);
      }
    }
    __syncthreads();
    fft_n<T, WI, RI, NT, MAXE, true, N>(buf, a.plan, tws);
    // (y, z) of the group's first line (one division per group); line l of the
    // group is y0 + l, wrapped into the next z plane (L <= ny)
    const int z0 = line0 / a.ny, y0 = line0 - z0 * a.ny;

    // 2) pointwise nonlinear + penalization term and diagnostics, line by line
    //    (the line's y, z and its rows of the mask sub-box once per line)
    T g0[L][XP], g1[L][XP], g2[L][XP];
    const int tid2 = opaque_tid<NT>();
#pragma unroll
    for (int l = 0; l < L; ++l) {
      const int yl = y0 + l, wrap = yl >= a.ny, y = yl - (wrap ? a.ny : 0), z = z0 + wrap;
      const int by = y - a.by0, bz = z - a.bz0;
      const bool lbox = a.bnx > 0 && by >= 0 && by < a.bny && bz >= 0 && bz < a.bnz;  // uniform
      const long long rowcell = lbox ? ((long long)bz * a.bny + by) * a.bnx : 0;
      const int qy = y - a.py0, qz = z - a.pz0;
      const bool lpbox = a.pnx > 0 && qy >= 0 && qy < a.pny && qz >= 0 && qz < a.pnz;  // uniform
      const long long prow = lpbox ? ((long long)qz * a.pny + qy) * a.pnx : 0;
#pragma unroll
      for (int k = 0; k < XP; ++k) {
        const int x = tid2 + k * NT;
        g0[l][k] = g1[l][k] = g2[l][k] = (T)0;
        if (x < n) {
          const cpx<T> z1 = buf[x * RI + 3 * l], z2 = buf[x * RI + 3 * l + 1], z3 = buf[x * RI + 3 * l + 2];
          const T ux = z1.re, uy = z1.im, uz = z2.re;
          const T wx = z2.im, wy = z3.re, wz = z3.im;
          T gx = uy * wz - uz * wy;
          T gy = uz * wx - ux * wz;
          T gz = ux * wy - uy * wx;
          const int bx = x - a.bx0;
          if constexpr (ST) {
            const long long cell = (lbox && bx >= 0 && bx < a.bnx) ? rowcell + bx : -1;
            penalize_static<T>(a, cell, (long long)y * n + x, ux, uy, uz, gx, gy, gz, aF0, aF1, aF2, aS0, aS1,
                               aS2);
          } else if (lbox && bx >= 0 && bx < a.bnx) {
            const long long cell = rowcell + bx;
            const T ch = a.chi[cell];
            if (ch != (T)0) {
              const T sx = ux - a.us[cell], sy = uy - a.us[a.bcells + cell], sz = uz - a.us[2 * a.bcells + cell];
              const T ce = ch * a.inv_eta;
              gx -= ce * sx;
              gy -= ce * sy;
              gz -= ce * sz;
              aF0 += (double)(ch * sx);
              aF1 += (double)(ch * sy);
              aF2 += (double)(ch * sz);
            }
          }
          const int qx = x - a.px0;
          if (lpbox && qx >= 0 && qx < a.pnx) {
            const long long cell = prow + qx;
            a.up[cell] = ux;
            a.up[a.pcells + cell] = uy;
            a.up[2 * a.pcells + cell] = uz;
          }
          const double u2 = (double)(ux * ux + uy * uy + uz * uz);
          aE += u2;
          aM = fmax(aM, u2);
          g0[l][k] = gx;
          g1[l][k] = gy;
          g2[l][k] = gz;
        }
      }
    }
    __syncthreads();
    T* bufr = reinterpret_cast<T*>(buf);
#pragma unroll
    for (int l = 0; l < L; ++l) {
#pragma unroll
      for (int k = 0; k < XP; ++k) {
        const int x = tid2 + k * NT;
        if (x < n) {
          buf[x * RF + l] = mk<T>(g0[l][k], g1[l][k]);
          bufr[2 * (x * RF + L + (l >> 1)) + (l & 1)] = g2[l][k];
        }
      }
    }
    __syncthreads();
    fft_n<T, WF, RF, NT, MAXE, false, N>(buf, a.plan, tws);

    // 3) unpack the two real transforms of each signal, keep kx <= K; field f
    //    of line l through a wave-uniform base and 32-bit offsets
    const int tid3 = opaque_tid<NT>();
#pragma unroll
    for (int f = 0; f < 3; ++f) {
#pragma unroll
      for (int l = 0; l < L; ++l) {
        const int sig = (f < 2) ? l : L + (l >> 1);
        const bool second = (f == 1) || (f == 2 && (l & 1));
        cpx<T>* ob = a.gout + f * a.sfs + (long long)(line0 + l) * a.ld;
#pragma unroll
        for (int k = 0; k < XI; ++k) {
          const int x = tid3 + k * NT;
          if (x < kx1) {
            const cpx<T> zv = buf[x * RF + sig];
            const cpx<T> zc = conj(buf[(x == 0 ? 0 : n - x) * RF + sig]);
            cpx<T> r;
            if (!second) r = scl(zv + zc, (T)0.5);
            else {
              const cpx<T> d = zv - zc;
              r = mk<T>((T)0.5 * d.im, (T)-0.5 * d.re);
            }
            *at_u32(ob, x) = r;
          }
        }
      }
    }
    __syncthreads();
  }

  double v[7] = {aF0, aF1, aF2, aE, aS0, aS1, aS2};
  block_sum<ST ? 7 : 4, NT>(reinterpret_cast<double(&)[ST ? 7 : 4]>(v), red);
  __syncthreads();
  const double m = block_max<NT>(aM, red);
  if (tid == 0) {
    double* p = a.partials + (long long)blockIdx.x * 8;
    p[0] = v[0];
    p[1] = v[1];
    p[2] = v[2];
    p[3] = v[3];
    p[4] = m;
    p[5] = ST ? v[4] : 0.0;
    p[6] = ST ? v[5] : 0.0;
    p[7] = ST ? v[6] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// x pass for nx = 512: one wavefront per pair of lines, register-resident FFTs
// (the transforms are in wave512.h)
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ void load512_sig(const XArgs<T>& a, int line, int p, int lane, Raw512<T>& w) {
  load512<T>(a.spec + (2 * p) * a.sfs + (long long)line * a.ld, a.spec + (2 * p + 1) * a.sfs + (long long)line * a.ld,
             lane, w);
}

// One line of the fused pass: C2R of (u, omega), pointwise term and
// diagnostics, R2C of (Gx, Gy) stored; returns Gz in the physical layout.
// On entry pf holds the line's first packed signal; on exit it holds the first
// signal of line `next` (if next >= 0), loaded while this line is transformed.
template <typename T, bool ST, typename TW>
__device__ __forceinline__ void wave512_line(const XArgs<T>& a, int line, int next, int lane, cpx<T>* X,
                                             const TW& tw, Raw512<T>& pf,
                                             T (&gz)[8], double& aF0, double& aF1, double& aF2, double& aE,
                                             double& aM, double& aS0, double& aS1, double& aS2) {
  constexpr int K = 170;  // the 2/3 band of 512 points: 3 * 170 < 512
  cpx<T> P[3][8];
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    cpx<T> v[8];
    pack512<T>(pf, lane, v);
    if (p < 2) load512_sig<T>(a, line, p + 1, lane, pf);  // prefetch: in flight during the transform
    inv512<T>(v, X, lane, tw);
#pragma unroll
    for (int j = 0; j < 8; ++j) P[p][j] = v[j];
  }
  // unconditional (the last line reloads itself): see load512
  load512_sig<T>(a, next >= 0 ? next : line, 0, lane, pf);
  // pointwise: G = u x omega - (chi/eta)(u - u_s) and the diagnostics
  cpx<T> g[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const T ux = P[0][j].re, uy = P[0][j].im, uz = P[1][j].re;
    const T wx = P[1][j].im, wy = P[2][j].re, wz = P[2][j].im;
    g[j] = mk<T>(uy * wz - uz * wy, uz * wx - ux * wz);
    gz[j] = ux * wy - uy * wx;
    // |u|^2 as a product in the bulk precision, summed per lane in FP64
    const double u2 = (double)(ux * ux + uy * uy + uz * uz);
    aE += u2;
    aM = fmax(aM, u2);
  }
  const int z = line / a.ny, y = line - z * a.ny;
  const int qy = y - a.py0, qz = z - a.pz0;
  if (a.pnx > 0 && qy >= 0 && qy < a.pny && qz >= 0 && qz < a.pnz) {  // uniform per wave
    const long long rowcell = ((long long)qz * a.pny + qy) * a.pnx;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int qx = (lane >> 3) + 8 * (lane & 7) + 64 * j - a.px0;
      if (qx >= 0 && qx < a.pnx) {
        a.up[rowcell + qx] = P[0][j].re;
        a.up[a.pcells + rowcell + qx] = P[0][j].im;
        a.up[2 * a.pcells + rowcell + qx] = P[1][j].re;
      }
    }
  }
  const int by = y - a.by0, bz = z - a.bz0;
  if constexpr (ST) {  // static plane on every line, the wing's sub-box where it has one
    const bool inbox = a.bnx > 0 && by >= 0 && by < a.bny && bz >= 0 && bz < a.bnz;  // uniform per wave
    const long long rowcell = inbox ? ((long long)bz * a.bny + by) * a.bnx : 0;
    const long long srow = (long long)y * a.n;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int x = (lane >> 3) + 8 * (lane & 7) + 64 * j;
      const int bx = x - a.bx0;
      const long long cell = (inbox && bx >= 0 && bx < a.bnx) ? rowcell + bx : -1;
      penalize_static<T>(a, cell, srow + x, P[0][j].re, P[0][j].im, P[1][j].re, g[j].re, g[j].im, gz[j], aF0, aF1,
                         aF2, aS0, aS1, aS2);
    }
  } else if (a.bnx > 0 && by >= 0 && by < a.bny && bz >= 0 && bz < a.bnz) {  // uniform per wave
    const long long rowcell = ((long long)bz * a.bny + by) * a.bnx;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int bx = (lane >> 3) + 8 * (lane & 7) + 64 * j - a.bx0;
      if (bx >= 0 && bx < a.bnx) {
        const long long cell = rowcell + bx;
        const T ch = a.chi[cell];
        if (ch != (T)0) {
          const T sx = P[0][j].re - a.us[cell];
          const T sy = P[0][j].im - a.us[a.bcells + cell];
          const T sz = P[1][j].re - a.us[2 * a.bcells + cell];
          const T ce = ch * a.inv_eta;
          g[j].re -= ce * sx;
          g[j].im -= ce * sy;
          gz[j] -= ce * sz;
          aF0 += (double)(ch * sx);
          aF1 += (double)(ch * sy);
          aF2 += (double)(ch * sz);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  fwd512<T>(g, X, lane, tw);
  unpack_store512<T>(g, lane, K, a.gout + (long long)line * a.ld, a.gout + a.sfs + (long long)line * a.ld);
}

// TM = 1: the per-lane twiddle sets held in registers (44 VGPRs, 3 waves per
// SIMD) instead of read from LDS in every transform (4 waves per SIMD): no
// twiddle reads (9 transforms x 14 complex values per lane and line pair), a
// fifth of the pass's LDS instructions; TM = 2: only the set C in registers;
// TM = 0: all sets from LDS
template <typename T, bool ST, int TM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TM == 1 ? 3 : 4))) void xpass_wave512(XArgs<T> a) {
  constexpr bool RT = TM == 1;
  __shared__ cpx<T> xbuf[4][kXBuf];
  // per-lane twiddle sets, [j][lane]: exp(+2 pi i lane j / 512), exp(-2 pi i lo j / 64),
  // exp(-2 pi i (lo + 8 j) hi / 512) with lo = lane & 7, hi = lane >> 3
  __shared__ cpx<T> tws[RT ? 1 : 3][RT ? 1 : 512];
  __shared__ double red[8 * 4];
  // Gz of the first line of a pair waits here (lane-private slots) while the
  // second line is transformed: registers are what limits the waves per SIMD
  __shared__ T gzs[4][8][64];
  // the wave index is uniform: as a scalar, every line address is a scalar
  // base plus a 32-bit lane offset (no 64-bit vector address arithmetic)
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  cpx<T>* X = xbuf[wv];
  constexpr int K = 170;
  using TW = std::conditional_t<RT, Tw512Reg<T>, std::conditional_t<TM == 2, Tw512Mix<T>, Tw512Lds<T>>>;
  TW tw;
  if constexpr (RT) {
    tw.load(a.tw, lane);
  } else if constexpr (TM == 2) {
    wave512_twiddles<T, 256>(tws, a.tw);
    __syncthreads();
    tw.ib = tws[0];
    tw.fb = tws[2];
    tw.lane = opaque(lane);
#pragma unroll
    for (int j = 1; j < 8; ++j) tw.c[j - 1] = tws[1][64 * j + lane];
  } else {
    wave512_twiddles<T, 256>(tws, a.tw);
    __syncthreads();
    tw = TW{tws[0], tws[1], tws[2], opaque(lane)};
  }
  double aF0 = 0, aF1 = 0, aF2 = 0, aE = 0, aM = 0, aS0 = 0, aS1 = 0, aS2 = 0;
  const int npairs = a.nlines / 2;
  Raw512<T> pf;
  const int pr0 = blockIdx.x * 4 + wv;
  if (pr0 < npairs) load512_sig<T>(a, 2 * pr0, 0, lane, pf);
#pragma unroll 1
  for (int pr = pr0; pr < npairs; pr += gridDim.x * 4) {
    const int nxt = (pr + gridDim.x * 4 < npairs) ? 2 * (pr + gridDim.x * 4) : -1;
    const int ln = opaque(lane);
    if constexpr (!RT) tw.lane = ln;
    {
      T gza[8];
      wave512_line<T, ST>(a, 2 * pr, 2 * pr + 1, ln, X, tw, pf, gza, aF0, aF1, aF2, aE, aM, aS0, aS1, aS2);
#pragma unroll
      for (int j = 0; j < 8; ++j) gzs[wv][j][lane] = gza[j];
    }
    T gzb[8];
    const int l2 = opaque(lane);
    if constexpr (!RT) tw.lane = l2;
    wave512_line<T, ST>(a, 2 * pr + 1, nxt, l2, X, tw, pf, gzb, aF0, aF1, aF2, aE, aM, aS0, aS1, aS2);
    cpx<T> g[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) g[j] = mk<T>(gzs[wv][j][lane], gzb[j]);
    const int l3 = opaque(lane);
    if constexpr (!RT) tw.lane = l3;
    fwd512<T>(g, X, l3, tw);
    unpack_store512<T>(g, l3, K, a.gout + 2 * a.sfs + (long long)(2 * pr) * a.ld,
                       a.gout + 2 * a.sfs + (long long)(2 * pr + 1) * a.ld);
  }
  double v[7] = {aF0, aF1, aF2, aE, aS0, aS1, aS2};
  block_sum<ST ? 7 : 4, 256>(reinterpret_cast<double(&)[ST ? 7 : 4]>(v), red);
  __syncthreads();
  const double m = block_max<256>(aM, red);
  if (threadIdx.x == 0) {
    double* p = a.partials + (long long)blockIdx.x * 8;
    p[0] = v[0];
    p[1] = v[1];
    p[2] = v[2];
    p[3] = v[3];
    p[4] = m;
    p[5] = ST ? v[4] : 0.0;
    p[6] = ST ? v[5] : 0.0;
    p[7] = ST ? v[6] : 0.0;
  }
}

// Masked vorticity of the sponge at nx = 512: the x-spectral omega (fields 3-5
// of a line pair) is transformed to the grid, multiplied by chi_sp = max(gx[x],
// gy[y], gz[z]) and transformed back into the same fields.  One wavefront per
// line pair, the register transforms of the fused pass: (wx + i wy) of each
// line and (wz of line 0 + i wz of line 1), three inverse and three forward
// transforms per pair; every input of a pair is read before its outputs are
// stored, so the pass runs in place.
// FP32 holds the twiddle sets in registers (the kernel stays within 128 VGPRs),
// FP64 reads them from LDS.
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) void xsponge_wave512(
    XArgs<T> a, const T* g) {
  constexpr bool RT = sizeof(T) == 4;
  __shared__ cpx<T> xbuf[4][kXBuf];
  __shared__ cpx<T> tws[RT ? 1 : 3][RT ? 1 : 512];
  __shared__ T gxs[512];
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  cpx<T>* X = xbuf[wv];
  constexpr int K = 170;
  using TW = std::conditional_t<RT, Tw512Reg<T>, Tw512Lds<T>>;
  TW tw;
  if constexpr (RT) tw.load(a.tw, lane);
  else {
    wave512_twiddles<T, 256>(tws, a.tw);
    tw = TW{tws[0], tws[1], tws[2], lane};
  }
  for (int i = threadIdx.x; i < 512; i += 256) gxs[i] = g[i];
  __syncthreads();
  const T* gy = g + 512;
  const T* gz = gy + a.ny;
  const int npairs = a.nlines / 2;
#pragma unroll 1
  for (int pr = blockIdx.x * 4 + wv; pr < npairs; pr += gridDim.x * 4) {
    const int l0 = 2 * pr, l1 = 2 * pr + 1;
    const T m0 = fmax(gy[l0 % a.ny], gz[l0 / a.ny]);
    const T m1 = fmax(gy[l1 % a.ny], gz[l1 / a.ny]);
    Raw512<T> w0, w1, w2;
    const long long o0 = (long long)l0 * a.ld, o1 = (long long)l1 * a.ld;
    load512<T>(a.spec + 3 * a.sfs + o0, a.spec + 4 * a.sfs + o0, lane, w0);
    load512<T>(a.spec + 3 * a.sfs + o1, a.spec + 4 * a.sfs + o1, lane, w1);
    load512<T>(a.spec + 5 * a.sfs + o0, a.spec + 5 * a.sfs + o1, lane, w2);
    cpx<T> v[8];
    // lane holds the grid points x = (lane >> 3) + 8 (lane & 7) + 64 j
    pack512<T>(w0, lane, v);
    inv512<T>(v, X, lane, tw);
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = scl(v[j], fmax(gxs[(lane >> 3) + 8 * (lane & 7) + 64 * j], m0));
    fwd512<T>(v, X, lane, tw);
    unpack_store512<T>(v, lane, K, a.spec + 3 * a.sfs + o0, a.spec + 4 * a.sfs + o0);
    pack512<T>(w1, lane, v);
    inv512<T>(v, X, lane, tw);
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = scl(v[j], fmax(gxs[(lane >> 3) + 8 * (lane & 7) + 64 * j], m1));
    fwd512<T>(v, X, lane, tw);
    unpack_store512<T>(v, lane, K, a.spec + 3 * a.sfs + o1, a.spec + 4 * a.sfs + o1);
    pack512<T>(w2, lane, v);
    inv512<T>(v, X, lane, tw);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const T gxv = gxs[(lane >> 3) + 8 * (lane & 7) + 64 * j];
      v[j] = mk<T>(v[j].re * fmax(gxv, m0), v[j].im * fmax(gxv, m1));
    }
    fwd512<T>(v, X, lane, tw);
    unpack_store512<T>(v, lane, K, a.spec + 5 * a.sfs + o0, a.spec + 5 * a.sfs + o1);
  }
}

// Plain real transforms along x for NF fields of L lines: real signal r = l * NF + f,
// complex signal j packs real signals 2j (real part) and 2j + 1 (imaginary part).
template <typename T, int NF, int L, int NT, int MAXE, int MODE>
__global__ __launch_bounds__(NT) void xpass_plain(XArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  constexpr int S = NF * L / 2;
  constexpr int RSS = PadStride<S>::value;
  static_assert((NF * L) % 2 == 0, "need an even number of real signals");
  const int tid = threadIdx.x;
  const int n = a.n, K = a.kx1 - 1;
  const int ngroups = a.nlines / L;
  cpx<T>* tws = buf + n * RSS;
  for (int i = tid; i < n; i += NT) tws[i] = a.tw[i];
  for (int g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const int line0 = g * L;
    if constexpr (MODE == X_C2R) {
      for (int it = tid; it < S * n; it += NT) {
        const int x = it % n, j = it / n;
        const int ra = 2 * j, rb = 2 * j + 1;
        if (x <= K) {
          const cpx<T> A = a.spec[(ra % NF) * a.sfs + (long long)(line0 + ra / NF) * a.ld + x];
          const cpx<T> B = a.spec[(rb % NF) * a.sfs + (long long)(line0 + rb / NF) * a.ld + x];
          if (x == 0) buf[j] = mk<T>(A.re, B.re);
          else {
            buf[x * RSS + j] = mk<T>(A.re - B.im, A.im + B.re);
            buf[(n - x) * RSS + j] = mk<T>(A.re + B.im, B.re - A.im);
          }
        } else if (x < n - K) {
          buf[x * RSS + j] = mk<T>(0, 0);
        }
      }
      __syncthreads();
      fft_lds<T, S, RSS, NT, MAXE, true>(buf, a.plan, tws);
      for (int it = tid; it < 2 * S * n; it += NT) {
        const int x = it % n, r = it / n;
        const cpx<T> z = buf[x * RSS + (r >> 1)];
        a.phys[(r % NF) * a.pfs + (long long)(line0 + r / NF) * n + x] = (r & 1) ? z.im : z.re;
      }
      __syncthreads();
    } else {
      T* bufr = reinterpret_cast<T*>(buf);
      for (int it = tid; it < 2 * S * n; it += NT) {
        const int x = it % n, r = it / n;
        bufr[2 * (x * RSS + (r >> 1)) + (r & 1)] = a.phys[(r % NF) * a.pfs + (long long)(line0 + r / NF) * n + x];
      }
      __syncthreads();
      fft_lds<T, S, RSS, NT, MAXE, false>(buf, a.plan, tws);
      for (int it = tid; it < 2 * S * a.kx1; it += NT) {
        const int k = it % a.kx1, r = it / a.kx1;
        const cpx<T> z = buf[k * RSS + (r >> 1)];
        const cpx<T> zc = conj(buf[((n - k) % n) * RSS + (r >> 1)]);
        cpx<T> v;
        if (!(r & 1)) v = scl(z + zc, (T)0.5);
        else {
          const cpx<T> d = z - zc;
          v = mk<T>((T)0.5 * d.im, (T)-0.5 * d.re);
        }
        a.spec[(r % NF) * a.sfs + (long long)(line0 + r / NF) * a.ld + k] = v;
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// reductions and adaptive dt
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kNT) void finalize_kernel(FinalArgs a) {
  __shared__ double red[8 * (kNT / 64)];
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  double m = 0;
  for (int p = threadIdx.x; p < a.np; p += kNT) {
    const double* q = a.partials + (long long)p * 8;
    v[0] += q[0];
    v[1] += q[1];
    v[2] += q[2];
    v[3] += q[3];
    m = fmax(m, q[4]);
    v[4] += q[5];
    v[5] += q[6];
    v[6] += q[7];
  }
  block_sum<7, kNT>(v, red);
  __syncthreads();
  m = block_max<kNT>(m, red);
  if (threadIdx.x == 0) {
    const double umax = sqrt(m);
    double dt;
    if (a.adaptive) {
      dt = a.cap;
      if (umax > 0.0) dt = fmin(dt, a.cfl_dx / umax);
    } else {
      dt = a.dt_fixed;
    }
    const double F0 = v[0] * a.dV * a.inv_eta, F1 = v[1] * a.dV * a.inv_eta, F2 = v[2] * a.dV * a.inv_eta;
    const double E = 0.5 * a.dV * v[3];
    const bool bad = !isfinite(E) || !isfinite(F0) || !isfinite(F1) || !isfinite(F2) || !isfinite(umax);
    DevScalars* s = a.sc;
    s->dt[a.cur] = dt;
    s->t += dt;
    s->info[0] = F0;
    s->info[1] = F1;
    s->info[2] = F2;
    s->info[3] = E;
    s->info[4] = umax;
    s->info[5] = dt;
    s->info[6] = bad ? 1.0 : s->info[6];
    s->info[7] = s->t;
    s->fst[0] = v[4] * a.dV * a.inv_eta;
    s->fst[1] = v[5] * a.dV * a.inv_eta;
    s->fst[2] = v[6] * a.dV * a.inv_eta;
  }
}

// ---------------------------------------------------------------------------
// mask: distance keys per triangle, then chi and u_s per cell
// ---------------------------------------------------------------------------

__global__ void fill_keys(unsigned long long* k1, unsigned long long* k2, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    k1[i] = ~0ull;
    k2[i] = ~0ull;
  }
}

// Key of the first pass: the FP64 distance truncated to FP32 (monotone in the
// distance), triangle id in the low word.  Key of the second pass, among the
// triangles whose truncated distance equals the minimum: the 29 mantissa bits
// that the truncation dropped, triangle id in the low word.  Together they select
// the exact FP64 minimum, ties going to the lowest triangle id.
__device__ __forceinline__ unsigned trunc_bits(double d) { return __float_as_uint(__double2float_rz(d)); }
__device__ __forceinline__ unsigned low_bits(double d) {
  return (unsigned)((unsigned long long)__double_as_longlong(d) & ((1ull << 29) - 1));
}

template <typename T, int PASS>
__global__ __launch_bounds__(kNT) void mask_dist(MaskArgs<T> a) {
  const int t = blockIdx.x;
  if (t >= a.nt) return;
  const int ia = a.tri[3 * t], ib = a.tri[3 * t + 1], ic = a.tri[3 * t + 2];
  const double ax = a.x[3 * ia], ay = a.x[3 * ia + 1], az = a.x[3 * ia + 2];
  const double bx = a.x[3 * ib] - ax, by = a.x[3 * ib + 1] - ay, bz = a.x[3 * ib + 2] - az;
  const double cx = a.x[3 * ic] - ax, cy = a.x[3 * ic + 1] - ay, cz = a.x[3 * ic + 2] - az;
  const double lox = fmin(fmin(0.0, bx), cx) + ax - a.rsup, hix = fmax(fmax(0.0, bx), cx) + ax + a.rsup;
  const double loy = fmin(fmin(0.0, by), cy) + ay - a.rsup, hiy = fmax(fmax(0.0, by), cy) + ay + a.rsup;
  const double loz = fmin(fmin(0.0, bz), cz) + az - a.rsup, hiz = fmax(fmax(0.0, bz), cz) + az + a.rsup;
  // index range, one cell of margin, clipped to the sub-box
  const int i0 = max((int)floor(lox / a.dx) - 1, a.bx0), i1 = min((int)ceil(hix / a.dx) + 1, a.bx0 + a.bnx - 1);
  const int j0 = max((int)floor(loy / a.dy) - 1, a.by0), j1 = min((int)ceil(hiy / a.dy) + 1, a.by0 + a.bny - 1);
  const int k0 = max((int)floor(loz / a.dz) - 1, a.bz0), k1 = min((int)ceil(hiz / a.dz) + 1, a.bz0 + a.bnz - 1);
  if (i1 < i0 || j1 < j0 || k1 < k0) return;
  const int ni = i1 - i0 + 1, nj = j1 - j0 + 1, nk = k1 - k0 + 1;
  const int total = ni * nj * nk;
  for (int q = threadIdx.x; q < total; q += kNT) {
    const int ii = i0 + q % ni;
    const int jj = j0 + (q / ni) % nj;
    const int kk = k0 + q / (ni * nj);
    const double px = (double)ii * a.dx - ax, py = (double)jj * a.dy - ay, pz = (double)kk * a.dz - az;
    double wa, wb, wc;
    const double d = sqrt(closest_on_triangle<double>(px, py, pz, bx, by, bz, cx, cy, cz, wa, wb, wc));
    if (d < a.rsup) {
      const long long cell = ((long long)(kk - a.bz0) * a.bny + (jj - a.by0)) * a.bnx + (ii - a.bx0);
      const unsigned q1 = trunc_bits(d);
      if (PASS == 1) {
        atomicMin(a.key1 + cell, ((unsigned long long)q1 << 32) | (unsigned)t);
      } else if ((unsigned)(a.key1[cell] >> 32) == q1) {
        atomicMin(a.key2 + cell, ((unsigned long long)low_bits(d) << 32) | (unsigned)t);
      }
    }
  }
}

// GRID = false: chi, u_s into the sub-box arrays; GRID = true: into full grids
// (the caller has zeroed them outside the sub-box)
template <typename T, bool GRID>
__global__ __launch_bounds__(kNT) void mask_eval(MaskArgs<T> a) {
  for (long long cell = (long long)blockIdx.x * kNT + threadIdx.x; cell < a.bcells; cell += (long long)gridDim.x * kNT) {
    const unsigned long long key = a.key2[cell];
    double ch = 0, u0 = 0, u1 = 0, u2 = 0;
    const int bx = (int)(cell % a.bnx);
    const int by = (int)((cell / a.bnx) % a.bny);
    const int bz = (int)(cell / ((long long)a.bnx * a.bny));
    if (key != ~0ull) {
      const int t = (int)(key & 0xffffffffull);
      const int ia = a.tri[3 * t], ib = a.tri[3 * t + 1], ic = a.tri[3 * t + 2];
      const double ax = a.x[3 * ia], ay = a.x[3 * ia + 1], az = a.x[3 * ia + 2];
      const double px = (double)(bx + a.bx0) * a.dx - ax, py = (double)(by + a.by0) * a.dy - ay,
                   pz = (double)(bz + a.bz0) * a.dz - az;
      double wa, wb, wc;
      const double d = sqrt(closest_on_triangle<double>(px, py, pz, a.x[3 * ib] - ax, a.x[3 * ib + 1] - ay,
                                                        a.x[3 * ib + 2] - az, a.x[3 * ic] - ax, a.x[3 * ic + 1] - ay,
                                                        a.x[3 * ic + 2] - az, wa, wb, wc));
      if (d < a.rsup) {
        ch = profile_chi(d, a.tw, a.h, a.profile);
        if (ch != 0.0) {
          u0 = wa * a.v[3 * ia] + wb * a.v[3 * ib] + wc * a.v[3 * ic];
          u1 = wa * a.v[3 * ia + 1] + wb * a.v[3 * ib + 1] + wc * a.v[3 * ic + 1];
          u2 = wa * a.v[3 * ia + 2] + wb * a.v[3 * ib + 2] + wc * a.v[3 * ic + 2];
        }
      }
    }
    if constexpr (GRID) {
      const long long o = ((long long)(bz + a.bz0) * a.gny + (by + a.by0)) * a.gnx + (bx + a.bx0);
      a.chi[o] = (T)ch;
      a.us[o] = (T)u0;
      a.us[a.gcells + o] = (T)u1;
      a.us[2 * a.gcells + o] = (T)u2;
    } else {
      a.chi[cell] = (T)ch;
      a.us[cell] = (T)u0;
      a.us[a.bcells + cell] = (T)u1;
      a.us[2 * a.bcells + cell] = (T)u2;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kNT) void fill_zero(T* p, long long n) {
  for (long long i = (long long)blockIdx.x * kNT + threadIdx.x; i < n; i += (long long)gridDim.x * kNT) p[i] = (T)0;
}

// Writes (v, v) into the padding columns kx1 <= c < kxp of `rows` rows of pitch kxp.
template <typename T>
__global__ __launch_bounds__(kNT) void fill_pad(cpx<T>* p, long long rows, int kx1, int kxp, T v) {
  const int w = kxp - kx1;
  const long long n = rows * w;
  for (long long i = (long long)blockIdx.x * kNT + threadIdx.x; i < n; i += (long long)gridDim.x * kNT)
    p[(i / w) * kxp + kx1 + i % w] = mk<T>(v, v);
}

template <typename T>
hipError_t launch_fill_pad(cpx<T>* p, long long rows, int kx1, int kxp, T v, hipStream_t s) {
  if (!p || rows <= 0 || kxp <= kx1) return hipSuccess;
  long long blocks = (rows * (kxp - kx1) + kNT - 1) / kNT;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(fill_pad<T>, dim3((unsigned)blocks), dim3(kNT), 0, s, p, rows, kx1, kxp, v);
  return hipGetLastError();
}
template hipError_t launch_fill_pad<float>(cpx<float>*, long long, int, int, float, hipStream_t);
template hipError_t launch_fill_pad<double>(cpx<double>*, long long, int, int, double, hipStream_t);

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// pressure samples for the wing loads (FSI mode)
// ---------------------------------------------------------------------------

// 4-point delta kernel (Peskin's), phi(r) for |r| < 2 in grid units: it
// reproduces constants and linear functions and splits evenly between even
// and odd grid points.
__device__ __forceinline__ double delta4(double r) {
  r = fabs(r);
  if (r < 1.0) return 0.125 * (3.0 - 2.0 * r + sqrt(1.0 + 4.0 * r - 4.0 * r * r));
  if (r < 2.0) return 0.125 * (5.0 - 2.0 * r - sqrt(-7.0 + 12.0 * r - 4.0 * r * r));
  return 0.0;
}

// One thread per point: p(X) = sum over the 4 x 4 x 4 grid points around X of
// phi phi phi (Pi - |u|^2 / 2); the host guarantees every stencil lies in the
// pressure box.
template <typename T>
__global__ __launch_bounds__(kNT) void pressure_sample(PressArgs<T> a) {
  const int sidx = blockIdx.x * kNT + threadIdx.x;
  if (sidx >= a.ns) return;
  const double g[3] = {a.pts[3 * sidx] / a.dx, a.pts[3 * sidx + 1] / a.dy, a.pts[3 * sidx + 2] / a.dz};
  int i0[3];
  double w[3][4];
  for (int q = 0; q < 3; ++q) {
    i0[q] = (int)floor(g[q]) - 1;
    for (int m = 0; m < 4; ++m) w[q][m] = delta4(g[q] - (double)(i0[q] + m));
  }
  double acc = 0.0;
  for (int c = 0; c < 4; ++c) {
    const int z = i0[2] + c;
    for (int b = 0; b < 4; ++b) {
      const int y = i0[1] + b;
      const double wzy = w[2][c] * w[1][b];
      for (int m = 0; m < 4; ++m) {
        const int x = i0[0] + m;
        const long long cell = ((long long)(z - a.pz0) * a.pny + (y - a.py0)) * a.pnx + (x - a.px0);
        const double ux = (double)a.up[cell], uy = (double)a.up[a.pcells + cell],
                     uz = (double)a.up[2 * a.pcells + cell];
        const double pi = (double)a.pi[((long long)z * a.ny + y) * a.nx + x];
        acc += wzy * w[0][m] * (pi - 0.5 * (ux * ux + uy * uy + uz * uz));
      }
    }
  }
  a.out[sidx] = acc;
}

template <typename T>
__global__ __launch_bounds__(kNT) void pbox_pressure(BoxArgs<T> a) {
  for (long long c = (long long)blockIdx.x * kNT + threadIdx.x; c < a.pcells; c += (long long)gridDim.x * kNT) {
    const int qx = (int)(c % a.pnx), qy = (int)((c / a.pnx) % a.pny), qz = (int)(c / ((long long)a.pnx * a.pny));
    const long long g = ((long long)(qz + a.pz0) * a.ny + (qy + a.py0)) * a.nx + (qx + a.px0);
    const double ux = (double)a.up[c], uy = (double)a.up[a.pcells + c], uz = (double)a.up[2 * a.pcells + c];
    a.out[c] = (double)a.pi[g] - 0.5 * (ux * ux + uy * uy + uz * uz);
  }
}

template <typename T>
__global__ __launch_bounds__(kNT) void embed_box(BoxArgs<T> a) {
  for (long long c = (long long)blockIdx.x * kNT + threadIdx.x; c < a.pcells; c += (long long)gridDim.x * kNT) {
    const int qx = (int)(c % a.pnx), qy = (int)((c / a.pnx) % a.pny), qz = (int)(c / ((long long)a.pnx * a.pny));
    const long long g = ((long long)(qz + a.pz0) * a.ny + (qy + a.py0)) * a.nx + (qx + a.px0);
    a.grid[g] = a.in[c];
  }
}

template <typename T>
hipError_t launch_pbox(int embed, const BoxArgs<T>& a, hipStream_t s) {
  if (a.pcells <= 0) return hipSuccess;
  long long blocks = std::min((a.pcells + kNT - 1) / kNT, 4096LL);
  if (embed)
    hipLaunchKernelGGL(embed_box<T>, dim3((unsigned)blocks), dim3(kNT), 0, s, a);
  else
    hipLaunchKernelGGL(pbox_pressure<T>, dim3((unsigned)blocks), dim3(kNT), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_psample(const PressArgs<T>& a, hipStream_t s) {
  if (a.ns <= 0) return hipSuccess;
  hipLaunchKernelGGL(pressure_sample<T>, dim3((a.ns + kNT - 1) / kNT), dim3(kNT), 0, s, a);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(kNT) void sponge_mask(SpongeArgs<T> a) {
  const T* gy = a.g + a.nx;
  const T* gz = gy + a.ny;
  for (long long i = (long long)blockIdx.x * kNT + threadIdx.x; i < a.npts; i += (long long)gridDim.x * kNT) {
    const int x = (int)(i % a.nx);
    const long long r = i / a.nx;
    const int y = (int)(r % a.ny), z = (int)(r / a.ny);
    const T m = fmax(fmax(a.g[x], gy[y]), gz[z]);
    a.phys[i] *= m;
    a.phys[a.npts + i] *= m;
    a.phys[2 * a.npts + i] *= m;
  }
}

template <typename T>
hipError_t launch_xsponge(const XArgs<T>& a, const T* g, int grid, hipStream_t s) {
  if (a.n != 512 || a.nlines % 2 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(xsponge_wave512<T>, dim3(grid), dim3(256), 0, s, a, g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sponge_mask(const SpongeArgs<T>& a, hipStream_t s) {
  const long long nb = std::min((a.npts + kNT - 1) / kNT, 8192LL);
  hipLaunchKernelGGL(sponge_mask<T>, dim3((unsigned)std::max(nb, 1LL)), dim3(kNT), 0, s, a);
  return hipGetLastError();
}

template <typename K>
static hipError_t set_lds(K kernel, size_t lds) {
  if (lds > 65536) return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return hipSuccess;
}

template <typename T, int W, int NT, int MAXE>
static hipError_t launch_col_w(int mode, const ColArgs<T>& a, int slices, hipStream_t s) {
  dim3 grid((a.C + W - 1) / W, slices);
  const size_t lds = (size_t)a.n * (W + 1) * sizeof(cpx<T>);
  hipError_t e = hipSuccess;
  // the width that holds 512-point columns gets the compile-time 512 transform
  constexpr bool k512 = (W * 512 == NT * MAXE);
  // the FP32 512-point y passes and update pass address a slice or a field with
  // 32-bit byte offsets: beyond 4 GB they run the run-time-length kernels
  const bool off32 = sizeof(T) == 4 && W == 16 &&
                     (mode == COL_FWD_PLAIN || mode == COL_INV_WZ || mode == COL_FWD_UPDATE_Z);
  // the 512-point kernels store every column of their workgroup without a
  // column test: the last workgroup's columns must lie within the row pitch
  const bool whole = (long long)((a.C + W - 1) / W) * W <= a.ld;
  const bool use512 = k512 && a.n == 512 && a.K == 170 && whole &&
                      (!off32 || (long long)a.n * a.ld * (long long)sizeof(cpx<T>) < (1LL << 32));
  // the width that holds 800-point columns gets the compile-time 800 plan
  constexpr bool k800 = NT == 1024 && (W * 800 <= NT * MAXE) && (2 * W * 800 > NT * MAXE);
  const bool use800 = k800 && a.n == 800 && a.K == 266;
#define FSI_COL_CASE(M)                                                                   \
  case M:                                                                                 \
    if constexpr (k512) {                                                                 \
      if (use512) {                                                                       \
        e = set_lds(col_pass<T, W, NT, MAXE, M, 512>, lds);                               \
        if (e != hipSuccess) return e;                                                    \
        hipLaunchKernelGGL((col_pass<T, W, NT, MAXE, M, 512>), grid, dim3(NT), lds, s, a); \
        break;                                                                            \
      }                                                                                   \
    }                                                                                     \
    if constexpr (k800) {                                                                 \
      if (use800) {                                                                       \
        e = set_lds(col_pass<T, W, NT, MAXE, M, 800>, lds);                               \
        if (e != hipSuccess) return e;                                                    \
        hipLaunchKernelGGL((col_pass<T, W, NT, MAXE, M, 800>), grid, dim3(NT), lds, s, a); \
        break;                                                                            \
      }                                                                                   \
    }                                                                                     \
    if constexpr (NT == 1024) {                                                           \
      return hipErrorInvalidValue; /* the wide workgroups serve 800 points only */        \
    } else {                                                                              \
      e = set_lds(col_pass<T, W, NT, MAXE, M, 0>, lds);                                   \
      if (e != hipSuccess) return e;                                                      \
      hipLaunchKernelGGL((col_pass<T, W, NT, MAXE, M, 0>), grid, dim3(NT), lds, s, a);    \
    }                                                                                     \
    break;
  switch (mode) {
    FSI_COL_CASE(COL_INV_PLAIN)
    FSI_COL_CASE(COL_INV_CURL)
    FSI_COL_CASE(COL_INV_CURL5)
    FSI_COL_CASE(COL_INV_WZ)
    FSI_COL_CASE(COL_FWD_PLAIN)
    FSI_COL_CASE(COL_FWD_PROJECT)
    FSI_COL_CASE(COL_FWD_UPDATE)
    FSI_COL_CASE(COL_FWD_UPDATE_Z)
    FSI_COL_CASE(COL_FWD_SPONGE)
    FSI_COL_CASE(COL_ADJ_MU)
    FSI_COL_CASE(COL_FWD_ACC)
    FSI_COL_CASE(COL_FWD_ACC_CURL)
    default: return hipErrorInvalidValue;
  }
#undef FSI_COL_CASE
  return hipGetLastError();
}

template <typename T>
int col_width(int n) {
  const int cap = ColCfg<T>::MAXE * ColCfg<T>::NT;
  int w = 64;
  while (w > 4 && n * w > cap) w >>= 1;
  return n * w <= cap ? w : 0;
}

template <typename T>
hipError_t launch_col(int mode, const ColArgs<T>& a, int slices, hipStream_t s) {
  constexpr int M = ColCfg<T>::MAXE, NT = ColCfg<T>::NT;
  // 800-point columns: 128-byte row segments (16 FP32 / 8 FP64 columns, 109 KB
  // of LDS) over 1024 threads, 13 / 7 rows per thread, the compile-time plan
  if (a.n == 800 && a.K == 266)
    return launch_col_w<T, sizeof(T) == 4 ? 16 : 8, 1024, sizeof(T) == 4 ? 13 : 7>(mode, a, slices, s);
  switch (col_width<T>(a.n)) {
    case 64: return launch_col_w<T, 64, NT, M>(mode, a, slices, s);
    case 32: return launch_col_w<T, 32, NT, M>(mode, a, slices, s);
    case 16: return launch_col_w<T, 16, NT, M>(mode, a, slices, s);
    case 8: return launch_col_w<T, 8, NT, M>(mode, a, slices, s);
    case 4: return launch_col_w<T, 4, NT, M>(mode, a, slices, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
int xpass_lines(int n) {
  if (n == 800) return X800<T>::L;
  // four lines per workgroup when their 12 packed signals fit the register bound
  // and 64 KB of LDS, else two
  const bool regs = n * 12 <= XCfg<T, 4>::MAXE * XCfg<T, 4>::NT;
  const bool lds = n * (PadStride<12>::value + 1) * (int)sizeof(cpx<T>) <= 65536;
  if (regs && lds) return 4;
  return (n * 6 <= XCfg<T, 2>::MAXE * XCfg<T, 2>::NT) ? 2 : 0;
}

template <typename T, int L, bool ST, int N, int NT = XCfg<T, L>::NT, int M = XCfg<T, L>::MAXE>
static hipError_t launch_xfused_ln(const XArgs<T>& a, int grid, hipStream_t s) {
  const size_t lds = (size_t)a.n * (PadStride<3 * L>::value + 1) * sizeof(cpx<T>);
  hipError_t e = set_lds(xpass_fused<T, L, NT, M, ST, N>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((xpass_fused<T, L, NT, M, ST, N>), dim3(grid), dim3(NT), lds, s, a);
  return hipGetLastError();
}

template <typename T, int L, bool ST>
static hipError_t launch_xfused_l(const XArgs<T>& a, int grid, hipStream_t s) {
  return launch_xfused_ln<T, L, ST, 0>(a, grid, s);
}

// the static plane selects its own instantiation: without it the kernels keep
// their registers and code
template <typename T, bool ST>
static hipError_t launch_xfused_st(const XArgs<T>& a, int grid, hipStream_t s) {
  if (a.n == 512) {
    // Without the static plane, FP32 holds all twiddles in registers (166
    // VGPRs, 3 waves per SIMD; 6 % faster than in LDS) and FP64 the set used by
    // every transform (242 VGPRs, the 2 waves per SIMD it has anyway; 1 %
    // faster); the static plane's instantiations keep the LDS sets
    constexpr int tm = ST ? 0 : (sizeof(T) == 4 ? 1 : 2);
    hipLaunchKernelGGL((xpass_wave512<T, ST, tm>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
  }
  // 800 points: the compile-time plan with its own workgroup shape
  if (a.n == 800 && a.kx1 == 267)
    return launch_xfused_ln<T, X800<T>::L, ST, 800, X800<T>::NT, X800<T>::MAXE>(a, grid, s);
  if (xpass_lines<T>(a.n) == 4) return launch_xfused_l<T, 4, ST>(a, grid, s);
  return launch_xfused_l<T, 2, ST>(a, grid, s);
}

template <typename T>
hipError_t launch_xfused(const XArgs<T>& a, int grid, hipStream_t s) {
  return a.st_chi ? launch_xfused_st<T, true>(a, grid, s) : launch_xfused_st<T, false>(a, grid, s);
}

// Workgroups of the fused x pass for nlines lines of length n (bounded: each
// workgroup leaves one row of partial sums).
int xfused_grid(int n, long long nlines, int lines_per_group) {
#ifndef FSI_XGRID
#define FSI_XGRID 4096
#endif
  const long long units = (n == 512) ? nlines / 8 : nlines / lines_per_group;
  return (int)std::max(1LL, std::min(units, (long long)FSI_XGRID));
}

template <typename T, int NF, int L>
static hipError_t launch_xplain_l(int mode, const XArgs<T>& a, int grid, hipStream_t s) {
  constexpr int NT = XCfg<T, L>::NT, M = XCfg<T, L>::MAXE;
  const size_t lds = (size_t)a.n * (PadStride<NF * L / 2>::value + 1) * sizeof(cpx<T>);
  hipError_t e;
  if (mode == X_C2R) {
    e = set_lds(xpass_plain<T, NF, L, NT, M, X_C2R>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((xpass_plain<T, NF, L, NT, M, X_C2R>), dim3(grid), dim3(NT), lds, s, a);
  } else {
    e = set_lds(xpass_plain<T, NF, L, NT, M, X_R2C>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((xpass_plain<T, NF, L, NT, M, X_R2C>), dim3(grid), dim3(NT), lds, s, a);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xplain(int mode, int nf, const XArgs<T>& a, int grid, hipStream_t s) {
  const int L = xpass_lines<T>(a.n);
  if (nf == 1) return L == 4 ? launch_xplain_l<T, 1, 4>(mode, a, grid, s) : launch_xplain_l<T, 1, 2>(mode, a, grid, s);
  if (nf == 3) return L == 4 ? launch_xplain_l<T, 3, 4>(mode, a, grid, s) : launch_xplain_l<T, 3, 2>(mode, a, grid, s);
  return hipErrorInvalidValue;
}

hipError_t launch_finalize(const FinalArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kNT), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mask(const MaskArgs<T>& a, hipStream_t s) {
  long long blocks = (a.bcells + kNT - 1) / kNT;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(fill_keys, dim3((unsigned)blocks), dim3(kNT), 0, s, a.key1, a.key2, a.bcells);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.nt > 0) {
    hipLaunchKernelGGL((mask_dist<T, 1>), dim3(a.nt), dim3(kNT), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((mask_dist<T, 2>), dim3(a.nt), dim3(kNT), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((mask_eval<T, false>), dim3((unsigned)blocks), dim3(kNT), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mask_grid(const MaskArgs<T>& a, hipStream_t s) {
  // zero both grids (a fill kernel: no memset node if the caller captures the stream)
  hipLaunchKernelGGL(fill_zero<T>, dim3(8192), dim3(kNT), 0, s, a.chi, a.gcells);
  hipLaunchKernelGGL(fill_zero<T>, dim3(8192), dim3(kNT), 0, s, a.us, 3 * a.gcells);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.bcells == 0) return e;
  long long blocks = (a.bcells + kNT - 1) / kNT;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(fill_keys, dim3((unsigned)blocks), dim3(kNT), 0, s, a.key1, a.key2, a.bcells);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.nt > 0) {
    hipLaunchKernelGGL((mask_dist<T, 1>), dim3(a.nt), dim3(kNT), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((mask_dist<T, 2>), dim3(a.nt), dim3(kNT), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((mask_eval<T, true>), dim3((unsigned)blocks), dim3(kNT), 0, s, a);
  return hipGetLastError();
}

template int col_width<float>(int);
template int col_width<double>(int);
template int xpass_lines<float>(int);
template int xpass_lines<double>(int);
template hipError_t launch_col<float>(int, const ColArgs<float>&, int, hipStream_t);
template hipError_t launch_col<double>(int, const ColArgs<double>&, int, hipStream_t);
template hipError_t launch_xfused<float>(const XArgs<float>&, int, hipStream_t);
template hipError_t launch_xfused<double>(const XArgs<double>&, int, hipStream_t);
template hipError_t launch_xplain<float>(int, int, const XArgs<float>&, int, hipStream_t);
template hipError_t launch_xplain<double>(int, int, const XArgs<double>&, int, hipStream_t);
template hipError_t launch_pbox<float>(int, const BoxArgs<float>&, hipStream_t);
template hipError_t launch_pbox<double>(int, const BoxArgs<double>&, hipStream_t);
template hipError_t launch_psample<float>(const PressArgs<float>&, hipStream_t);
template hipError_t launch_sponge_mask<float>(const SpongeArgs<float>&, hipStream_t);
template hipError_t launch_xsponge<float>(const XArgs<float>&, const float*, int, hipStream_t);
template hipError_t launch_xsponge<double>(const XArgs<double>&, const double*, int, hipStream_t);
template hipError_t launch_sponge_mask<double>(const SpongeArgs<double>&, hipStream_t);
template hipError_t launch_psample<double>(const PressArgs<double>&, hipStream_t);
template hipError_t launch_mask<float>(const MaskArgs<float>&, hipStream_t);
template hipError_t launch_mask<double>(const MaskArgs<double>&, hipStream_t);
template hipError_t launch_mask_grid<float>(const MaskArgs<float>&, hipStream_t);
template hipError_t launch_mask_grid<double>(const MaskArgs<double>&, hipStream_t);

}  // namespace fsi
