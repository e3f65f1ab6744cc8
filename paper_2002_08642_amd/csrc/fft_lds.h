// fft_lds.h - batched mixed-radix complex FFT held in LDS, for gfx950.
//
// A workgroup transforms W interleaved signals of length n stored in LDS as
// buf[row * RS + col] (row = sample index, col = signal, RS >= W a row stride
// that may be padded against LDS bank conflicts).  The transform is a
// self-sorting (Stockham) decomposition n = R_0 R_1 ... R_{s-1} with radices
// 2, 3, 4, 5 and 8: stage s (span Ns = R_0 ... R_{s-1}) reads R samples spaced
// n/R apart, multiplies sample r by w^(r (j mod Ns) n/(Ns R)) with
// w = exp(-2 pi i / n), applies a radix-R DFT and writes the outputs spaced Ns
// apart from (j div Ns) Ns R + (j mod Ns).  Every stage first loads all its
// butterflies into registers, then (after a barrier) writes back, so one LDS
// buffer suffices.  Consecutive threads handle consecutive signals, so LDS
// rows are touched in contiguous runs of W complex values.
//
// Twiddles come from a table tw[k] = exp(-2 pi i k / n) computed on the host in
// extended precision; the inverse transform conjugates them (unnormalized).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fsi {

template <typename T>
struct __align__(2 * sizeof(T)) cpx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cpx<T> mk(T a, T b) {
  cpx<T> r;
  r.re = a;
  r.im = b;
  return r;
}
template <typename T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__device__ __forceinline__ cpx<T> scl(cpx<T> a, T s) { return mk(a.re * s, a.im * s); }

#ifndef FSI_NT
#define FSI_NT 3
#endif
// Streamed global accesses: every element of a pass's fields is read or written
// once.  FSI_NT bit 0 marks the stores non-temporal, bit 1 the column-pass
// loads, bit 2 the state loads of the update, bit 3 the x-pass loads (default:
// stores and column-pass loads, the fastest combination measured at 512^3).
template <typename T>
__device__ __forceinline__ void st_stream(cpx<T>* p, cpx<T> v) {
#if FSI_NT & 1
  typedef T V __attribute__((ext_vector_type(2)));
  V w;
  w.x = v.re;
  w.y = v.im;
  __builtin_nontemporal_store(w, reinterpret_cast<V*>(p));
#else
  *p = v;
#endif
}
template <bool NT, typename T>
__device__ __forceinline__ cpx<T> ld_hint(const cpx<T>* p) {
  if constexpr (NT) {
    typedef T V __attribute__((ext_vector_type(2)));
    const V w = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
    return mk<T>(w.x, w.y);
  } else {
    return *p;
  }
}
// column-pass inputs, the state read by the update, x-pass inputs
template <typename T>
__device__ __forceinline__ cpx<T> ld_stream(const cpx<T>* p) { return ld_hint<(FSI_NT & 2) != 0>(p); }
template <typename T>
__device__ __forceinline__ cpx<T> ld_state(const cpx<T>* p) { return ld_hint<(FSI_NT & 4) != 0>(p); }
template <typename T>
__device__ __forceinline__ cpx<T> ld_xin(const cpx<T>* p) { return ld_hint<(FSI_NT & 8) != 0>(p); }
template <typename T>
__device__ __forceinline__ cpx<T> conj(cpx<T> a) { return mk(a.re, -a.im); }
// multiply by +i (sgn = +1) or -i (sgn = -1)
template <typename T, int SGN>
__device__ __forceinline__ cpx<T> mul_i(cpx<T> a) {
  return SGN > 0 ? mk(-a.im, a.re) : mk(a.im, -a.re);
}

// Returns x through an empty asm statement so that the compiler treats it as a
// fresh value: address arithmetic derived from it is recomputed inside loops
// instead of being hoisted and kept live in registers for the whole kernel.
__device__ __forceinline__ int opaque(int x) {
  __asm__ volatile("" : "+v"(x));
  return x;
}
// The thread index through opaque(), with its range restated: the compiler
// then drops the bounds tests of work items that every thread has (and the
// code of items that none has), which it cannot see through the asm barrier.
template <int NT>
__device__ __forceinline__ int opaque_tid() {
  const int t = opaque((int)threadIdx.x);
  __builtin_assume(t >= 0 && t < NT);
  return t;
}

constexpr int kMaxStages = 16;

// Factorization of one transform length (host fills it; passed by value).
struct FftPlan {
  int n;
  int nst;
  int radix[kMaxStages];
};

// Radix-R DFT in place on v[0..R-1]: out_k = sum_r v_r exp(SGN 2 pi i r k / R).
template <typename T, int R, int SGN>
struct Bfly;

template <typename T, int SGN>
struct Bfly<T, 2, SGN> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    cpx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  }
};

template <typename T, int SGN>
struct Bfly<T, 4, SGN> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    cpx<T> t0 = v[0] + v[2], t1 = v[0] - v[2];
    cpx<T> t2 = v[1] + v[3], t3 = mul_i<T, SGN>(v[1] - v[3]);
    v[0] = t0 + t2;
    v[2] = t0 - t2;
    v[1] = t1 + t3;
    v[3] = t1 - t3;
  }
};

template <typename T, int SGN>
struct Bfly<T, 8, SGN> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    cpx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cpx<T> o[4] = {v[1], v[3], v[5], v[7]};
    Bfly<T, 4, SGN>::run(e);
    Bfly<T, 4, SGN>::run(o);
    const T h = (T)0.70710678118654752440084436210484903928;
    // o[k] *= exp(SGN i pi k / 4)
    cpx<T> o1 = mk(h * (o[1].re - SGN * o[1].im), h * (o[1].im + SGN * o[1].re));
    cpx<T> o2 = mul_i<T, SGN>(o[2]);
    cpx<T> o3 = mk(h * (-o[3].re - SGN * o[3].im), h * (-o[3].im + SGN * o[3].re));
    v[0] = e[0] + o[0];
    v[4] = e[0] - o[0];
    v[1] = e[1] + o1;
    v[5] = e[1] - o1;
    v[2] = e[2] + o2;
    v[6] = e[2] - o2;
    v[3] = e[3] + o3;
    v[7] = e[3] - o3;
  }
};

template <typename T, int SGN>
struct Bfly<T, 3, SGN> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    const T c = (T)-0.5;
    const T s = (T)(SGN * 0.86602540378443864676372317075293618347);
    cpx<T> a = v[1] + v[2];
    cpx<T> b = v[1] - v[2];
    cpx<T> m = mk(v[0].re + c * a.re, v[0].im + c * a.im);
    cpx<T> ib = mk(-s * b.im, s * b.re);  // i s b
    v[0] = v[0] + a;
    v[1] = m + ib;
    v[2] = m - ib;
  }
};

template <typename T, int SGN>
struct Bfly<T, 5, SGN> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    const T c1 = (T)0.30901699437494742410229341718281905886;   // cos(2 pi/5)
    const T c2 = (T)-0.80901699437494742410229341718281905886;  // cos(4 pi/5)
    const T s1 = (T)(SGN * 0.95105651629515357211643933337938214340);  // sin(2 pi/5)
    const T s2 = (T)(SGN * 0.58778525229247312916870595463907276860);  // sin(4 pi/5)
    cpx<T> a1 = v[1] + v[4], b1 = v[1] - v[4];
    cpx<T> a2 = v[2] + v[3], b2 = v[2] - v[3];
    cpx<T> m1 = mk(v[0].re + c1 * a1.re + c2 * a2.re, v[0].im + c1 * a1.im + c2 * a2.im);
    cpx<T> m2 = mk(v[0].re + c2 * a1.re + c1 * a2.re, v[0].im + c2 * a1.im + c1 * a2.im);
    // i (s1 b1 + s2 b2) and i (s2 b1 - s1 b2)
    cpx<T> n1 = mk(-(s1 * b1.im + s2 * b2.im), s1 * b1.re + s2 * b2.re);
    cpx<T> n2 = mk(-(s2 * b1.im - s1 * b2.im), s2 * b1.re - s1 * b2.re);
    v[0] = v[0] + a1 + a2;
    v[1] = m1 + n1;
    v[4] = m1 - n1;
    v[2] = m2 + n2;
    v[3] = m2 - n2;
  }
};

// One Stockham stage over W interleaved signals with LDS row stride RS >= W.
// MAXE bounds n*W/NT.  tw may live in LDS or global memory.
template <typename T, int R, int W, int RS, int NT, int MAXE, bool INV>
__device__ __forceinline__ void fft_stage(cpx<T>* buf, int n, int Ns, const cpx<T>* tw) {
  constexpr int KB = (MAXE + R - 1) / R;
  constexpr int SGN = INV ? 1 : -1;
  const int nR = n / R;
  const int nb = nR * W;
  const int tstride = n / (Ns * R);
  // An opaque copy of the thread id keeps the compiler from hoisting the LDS
  // addresses of every radix variant out of the stage loop (that costs ~100 VGPRs).
  const int tid = opaque_tid<NT>();
  cpx<T> v[KB][R];
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int q = tid + k * NT;
    if (q < nb) {
      const int col = q % W, j = q / W;
#pragma unroll
      for (int r = 0; r < R; ++r) v[k][r] = buf[(j + r * nR) * RS + col];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int q = tid + k * NT;
    if (q < nb) {
      const int col = q % W, j = q / W;
      const int jm = j % Ns;
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cpx<T> w = tw[jm * r * tstride];
          if (INV) w.im = -w.im;
          v[k][r] = cmul(v[k][r], w);
        }
      }
      Bfly<T, R, SGN>::run(v[k]);
      const int d0 = (j - jm) * R + jm;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[(d0 + r * Ns) * RS + col] = v[k][r];
    }
  }
  __syncthreads();
}

// Full transform of the W signals in buf (caller has synchronized after filling it;
// on return the result is in buf and all threads are synchronized).
template <typename T, int W, int RS, int NT, int MAXE, bool INV>
__device__ void fft_lds(cpx<T>* buf, const FftPlan& p, const cpx<T>* tw) {
  int Ns = 1;
  for (int s = 0; s < p.nst; ++s) {
    const int R = p.radix[s];
    switch (R) {
      case 8: fft_stage<T, 8, W, RS, NT, MAXE, INV>(buf, p.n, Ns, tw); break;
      case 4: fft_stage<T, 4, W, RS, NT, MAXE, INV>(buf, p.n, Ns, tw); break;
      case 2: fft_stage<T, 2, W, RS, NT, MAXE, INV>(buf, p.n, Ns, tw); break;
      case 5: fft_stage<T, 5, W, RS, NT, MAXE, INV>(buf, p.n, Ns, tw); break;
      default: fft_stage<T, 3, W, RS, NT, MAXE, INV>(buf, p.n, Ns, tw); break;
    }
    Ns *= R;
  }
}

// The transform with a compile-time length: N = 512 runs three radix-8
// stages, N = 800 the stages 8, 4, 5, 5 (the host plan of 800 = 2^5 5^2), with
// compile-time strides and index arithmetic; N = 0 the run-time plan.
template <typename T, int W, int RS, int NT, int MAXE, bool INV, int N>
__device__ __forceinline__ void fft_n(cpx<T>* buf, const FftPlan& p, const cpx<T>* tw) {
  if constexpr (N == 512) {
    fft_stage<T, 8, W, RS, NT, MAXE, INV>(buf, 512, 1, tw);
    fft_stage<T, 8, W, RS, NT, MAXE, INV>(buf, 512, 8, tw);
    fft_stage<T, 8, W, RS, NT, MAXE, INV>(buf, 512, 64, tw);
  } else if constexpr (N == 800) {
    fft_stage<T, 8, W, RS, NT, MAXE, INV>(buf, 800, 1, tw);
    fft_stage<T, 4, W, RS, NT, MAXE, INV>(buf, 800, 8, tw);
    fft_stage<T, 5, W, RS, NT, MAXE, INV>(buf, 800, 32, tw);
    fft_stage<T, 5, W, RS, NT, MAXE, INV>(buf, 800, 160, tw);
  } else {
    fft_lds<T, W, RS, NT, MAXE, INV>(buf, p, tw);
  }
}

// Column transform (row stride W).
template <typename T, int W, int NT, int MAXE, bool INV, int N>
__device__ __forceinline__ void col_fft(cpx<T>* buf, const FftPlan& p, const cpx<T>* tw) {
  fft_n<T, W, W, NT, MAXE, INV, N>(buf, p, tw);
}

// fft512_reg with one column per thread and slots at indices j and j + 32
// (see there); the same stages and swizzled LDS rows.
template <typename T, int W, bool INV>
__device__ __forceinline__ void fft512_reg_onecol(cpx<T> (&v0)[8], cpx<T> (&v1)[8], cpx<T>* buf, const cpx<T>* tw) {
  constexpr int SGN = INV ? 1 : -1;
  auto twiddle = [&](cpx<T>(&x)[8], int step) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 1; r < 8; ++r) {
      cpx<T> w = tw[step * r];
      if (INV) w.im = -w.im;
      x[r] = cmul(x[r], w);
    }
  };
  // rows 8 js + r at 8 js + (r ^ (js & 1)); rows js + 64 r at (js ^ bit 3 of js) + 64 r;
  // rows d0 + 8 r (bit 3 of d0 clear) at d0 + 8 r ^ (r & 1)
  auto put1 = [&](cpx<T>(&x)[8], int s) __attribute__((always_inline)) {
    const int t = opaque((int)threadIdx.x);
    const int cs = t % W, js = t / W + 32 * s, b = js & 1;
    cpx<T>* pe = buf + (8 * js + b) * W + cs;
    cpx<T>* po = buf + (8 * js + 1 - b) * W + cs;
#pragma unroll
    for (int r = 0; r < 8; ++r) *((r & 1) ? po + (r - 1) * W : pe + r * W) = x[r];
  };
  auto get = [&](cpx<T>(&x)[8], int s) __attribute__((always_inline)) {
    const int t = opaque((int)threadIdx.x);
    const int cs = t % W, js = t / W + 32 * s;
    const cpx<T>* p = buf + (js ^ ((js >> 3) & 1)) * W + cs;
#pragma unroll
    for (int r = 0; r < 8; ++r) x[r] = p[64 * r * W];
  };
  auto mid = [&](cpx<T>(&x)[8], int s) __attribute__((always_inline)) {
    const int t = opaque((int)threadIdx.x);
    const int cs = t % W, js = t / W + 32 * s, jm = js & 7;
    twiddle(x, 8 * jm);
    Bfly<T, 8, SGN>::run(x);
    const int d0 = (js - jm) * 8 + jm;
    cpx<T>* pe = buf + d0 * W + cs;
    cpx<T>* po = buf + (d0 ^ 1) * W + cs;
#pragma unroll
    for (int r = 0; r < 8; ++r) *(((r & 1) ? po : pe) + 8 * r * W) = x[r];
  };
  auto last = [&](cpx<T>(&x)[8], int s) __attribute__((always_inline)) {
    get(x, s);
    const int t = opaque((int)threadIdx.x);
    twiddle(x, t / W + 32 * s);
    Bfly<T, 8, SGN>::run(x);
  };
  Bfly<T, 8, SGN>::run(v0);
  Bfly<T, 8, SGN>::run(v1);
  __syncthreads();
  put1(v0, 0);
  put1(v1, 1);
  __syncthreads();
  get(v0, 0);
  get(v1, 1);
  __syncthreads();
  mid(v0, 0);
  mid(v1, 1);
  __syncthreads();
  last(v0, 0);
  // one slot at a time: both at once would hold 14 twiddles and 16 values
  __builtin_amdgcn_sched_barrier(0);
  last(v1, 1);
}

// 512-point transforms of the W columns of a workgroup (the three radix-8
// stages of col_fft, same arithmetic in the same order) with the first and the
// last stage on registers.  Thread t carries columns cs = 2 (t % (W/2)) and
// cs + 1 (arrays v0, v1) at index js = t / (W/2) in [0, 64) (NT = 32 W
// threads cover every column and index once): on entry vs[r] = x[js + 64 r],
// on return vs[r] = X[js + 64 r].  The span-1 stage needs exactly the inputs
// js + 64 r and the span-64 stage produces exactly those outputs, so only the
// middle stage goes through LDS: two buffer writes and two reads instead of
// four each, and three barriers instead of eight.  The two columns of a thread
// are adjacent in LDS (one ds_write2 / ds_read2 moves both) and share their
// twiddles.  Row R of buf lives at R ^ ((R >> 3) & 1): the rows 8 js + r that
// the lanes of a wave write in the first stage then fill both halves of the
// LDS banks instead of one (every other access touches runs of consecutive
// rows either way).  Begins with a barrier, so buf may still be being read by
// a previous transform.
//
// ONECOL = true: the two slots of a thread are one column t % W at the
// indices t / W and t / W + 32 (NT = 32 W threads), i.e. the thread's rows
// t / W + 32 m with m = s + 2 r for slot s; LDS accesses one column at a time.
template <typename T, int W, bool INV, bool ONECOL = false>
__device__ __forceinline__ void fft512_reg(cpx<T> (&v0)[8], cpx<T> (&v1)[8], cpx<T>* buf, const cpx<T>* tw) {
  constexpr int SGN = INV ? 1 : -1;
  if constexpr (ONECOL) {
    fft512_reg_onecol<T, W, INV>(v0, v1, buf, tw);
    return;
  }
  // LDS addresses from an opaque thread id: computed per stage, not hoisted
  // and kept live across the kernel
  auto slot = [&](int& cs, int& js) __attribute__((always_inline)) {
    const int t = opaque((int)threadIdx.x);
    cs = 2 * (t % (W / 2));
    js = t / (W / 2);
  };
  auto twiddle = [&](cpx<T>(&x)[8], int step) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 1; r < 8; ++r) {
      cpx<T> w = tw[step * r];
      if (INV) w.im = -w.im;
      x[r] = cmul(x[r], w);
    }
  };
  int cs, js;
  Bfly<T, 8, SGN>::run(v0);
  Bfly<T, 8, SGN>::run(v1);
  __syncthreads();
  slot(cs, js);
  {
    // rows 8 js + r: stored at 8 js + (r ^ b), b = js & 1 (bit 3 of the row),
    // from one base per parity of r and immediate offsets
    const int b = js & 1;
    cpx<T>* pe = buf + (8 * js + b) * W + cs;
    cpx<T>* po = buf + (8 * js + 1 - b) * W + cs;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      cpx<T>* p = (r & 1) ? po + (r - 1) * W : pe + r * W;
      p[0] = v0[r];
      p[1] = v1[r];
    }
  }
  // rows js + 64 r: bit 3 is that of js
  auto read_cols = [&]() __attribute__((always_inline)) {
    slot(cs, js);
    const cpx<T>* p = buf + (js ^ ((js >> 3) & 1)) * W + cs;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      v0[r] = p[64 * r * W];
      v1[r] = p[64 * r * W + 1];
    }
  };
  __syncthreads();
  read_cols();
  __syncthreads();
  slot(cs, js);
  const int jm = js & 7;
  twiddle(v0, 8 * jm);
  twiddle(v1, 8 * jm);
  Bfly<T, 8, SGN>::run(v0);
  Bfly<T, 8, SGN>::run(v1);
  {
    // rows d0 + 8 r, d0 = 64 (js >> 3) + jm (bit 3 clear): bit 3 of the row is r & 1
    const int d0 = (js - jm) * 8 + jm;
    cpx<T>* pe = buf + d0 * W + cs;
    cpx<T>* po = buf + (d0 ^ 1) * W + cs;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      cpx<T>* p = ((r & 1) ? po : pe) + 8 * r * W;
      p[0] = v0[r];
      p[1] = v1[r];
    }
  }
  __syncthreads();
  read_cols();
  twiddle(v0, js);
  twiddle(v1, js);
  Bfly<T, 8, SGN>::run(v0);
  Bfly<T, 8, SGN>::run(v1);
}

}  // namespace fsi
