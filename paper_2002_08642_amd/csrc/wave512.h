// wave512.h - 512-point complex FFTs held by one wavefront (gfx950, wave64).
//
// A 512-point transform is held by one wavefront, 8 values per lane.  With
// k = l + 64 r (lane l, register r) and x = x1 + 8 y1 + 64 y2 (lane 8 x1 + y1,
// register y2), exp(2 pi i k x / 512) splits into three radix-8 DFTs (over r,
// over the high lane digit, over the low lane digit) separated by two twiddle
// multiplications and two exchanges through a wave-private LDS buffer.  The
// inverse maps the natural spectral layout to that permuted physical layout;
// the forward transform is its exact reverse, so the pointwise work between
// them is lane-local and no workgroup barrier is needed.  Lane `lane` holds
// the physical points x = (lane >> 3) + 8 (lane & 7) + 64 j, j = 0..7.
#pragma once

#include <hip/hip_runtime.h>

#include "fft_lds.h"

namespace fsi {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// exchange slots (padded against LDS bank conflicts): 8 x 72 complex per wave
__device__ __forceinline__ int xslot1(int x1, int l) { return x1 * 72 + l; }
__device__ __forceinline__ int xslot2(int x1, int y1, int l1) { return x1 * 72 + y1 * 9 + l1; }
constexpr int kXBuf = 576;

// The inverse radix-8 butterfly over r of a band-limited spectrum: inputs
// v[3] = Z[lane + 192] and v[4] = Z[lane + 256] lie outside the 2/3 band of
// every lane (170 < lane + 192 < 342) and are zero.  Written out without them:
// IEEE rules keep the compiler from folding x + 0 and 0 - x itself.  Same
// values as Bfly<T, 8, +1> on such input (up to the sign of zero results).
template <typename T>
__device__ __forceinline__ void bfly8_inv_zero34(cpx<T> (&v)[8]) {
  // even half {v0, v2, 0, v6}
  const cpx<T> s26 = v[2] + v[6], d26 = mul_i<T, 1>(v[2] - v[6]);
  const cpx<T> e0 = v[0] + s26, e2 = v[0] - s26, e1 = v[0] + d26, e3 = v[0] - d26;
  // odd half {v1, 0, v5, v7}
  const cpx<T> s15 = v[1] + v[5], d15 = v[1] - v[5], i7 = mul_i<T, 1>(v[7]);
  const cpx<T> o0 = s15 + v[7], o2 = s15 - v[7], o1 = d15 - i7, o3 = d15 + i7;
  const T h = (T)0.70710678118654752440084436210484903928;
  const cpx<T> w1 = mk(h * (o1.re - o1.im), h * (o1.im + o1.re));
  const cpx<T> w2 = mul_i<T, 1>(o2);
  const cpx<T> w3 = mk(h * (-o3.re - o3.im), h * (-o3.im + o3.re));
  v[0] = e0 + o0;
  v[4] = e0 - o0;
  v[1] = e1 + w1;
  v[5] = e1 - w1;
  v[2] = e2 + w2;
  v[6] = e2 - w2;
  v[3] = e3 + w3;
  v[7] = e3 - w3;
}

// Twiddle sources of the transforms below: IB(j) = exp(-2 pi i lane j / 512) and
// C(j) = exp(+2 pi i lo j / 64) for j = 1..7, FB(j) = exp(+2 pi i (lo + 8 j) hi
// / 512) for j = 0..7, lo = lane & 7, hi = lane >> 3.  Tw512Lds reads the
// per-lane sets a workgroup keeps in LDS ([j][lane], wave512_twiddles);
// Tw512Reg holds them in 44 VGPRs of the lane, loaded once from the axis table
// tw[m] = exp(+2 pi i m / 512).
template <typename T>
struct Tw512Lds {
  const cpx<T>* ib;
  const cpx<T>* c;
  const cpx<T>* fb;
  int lane;
  __device__ __forceinline__ cpx<T> IB(int j) const { return ib[64 * j + lane]; }
  __device__ __forceinline__ cpx<T> C(int j) const { return c[64 * j + lane]; }
  __device__ __forceinline__ cpx<T> FB(int j) const { return fb[64 * j + lane]; }
};
template <typename T>
struct Tw512Reg {
  cpx<T> ib[7], c[7], fb[8];
  __device__ __forceinline__ void load(const cpx<T>* tw, int lane) {
    const int lo = lane & 7, hi = lane >> 3;
#pragma unroll
    for (int j = 1; j < 8; ++j) {
      ib[j - 1] = conj(tw[(lane * j) & 511]);
      c[j - 1] = tw[(8 * lo * j) & 511];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) fb[j] = tw[((lo + 8 * j) * hi) & 511];
  }
  __device__ __forceinline__ cpx<T> IB(int j) const { return ib[j - 1]; }
  __device__ __forceinline__ cpx<T> C(int j) const { return c[j - 1]; }
  __device__ __forceinline__ cpx<T> FB(int j) const { return fb[j]; }
};

// IB and FB from the LDS sets, C (used by every transform) held by the lane
template <typename T>
struct Tw512Mix {
  const cpx<T>* ib;
  const cpx<T>* fb;
  int lane;
  cpx<T> c[7];
  __device__ __forceinline__ cpx<T> IB(int j) const { return ib[64 * j + lane]; }
  __device__ __forceinline__ cpx<T> C(int j) const { return c[j - 1]; }
  __device__ __forceinline__ cpx<T> FB(int j) const { return fb[64 * j + lane]; }
};

// inverse: v[r] = Z[lane + 64 r]  ->  v[y2] = z[x1 + 8 y1 + 64 y2], lane = 8 x1 + y1;
// v[3], v[4] must be zero on entry (pack512 leaves them so)
template <typename T, typename TW>
__device__ __forceinline__ void inv512(cpx<T> (&v)[8], cpx<T>* X, int lane, const TW& tw) {
  const int hi = lane >> 3, lo = lane & 7;
  bfly8_inv_zero34<T>(v);
#pragma unroll
  for (int j = 1; j < 8; ++j) v[j] = cmul(v[j], tw.IB(j));
#pragma unroll
  for (int j = 0; j < 8; ++j) X[xslot1(j, lane)] = v[j];
  wave_sync();
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = X[xslot1(hi, lo + 8 * j)];
  wave_sync();
  Bfly<T, 8, 1>::run(v);
#pragma unroll
  for (int j = 1; j < 8; ++j) v[j] = cmul(v[j], conj(tw.C(j)));
#pragma unroll
  for (int j = 0; j < 8; ++j) X[xslot2(hi, j, lo)] = v[j];
  wave_sync();
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = X[xslot2(hi, lo, j)];
  wave_sync();
  Bfly<T, 8, 1>::run(v);
}
template <typename T>
__device__ __forceinline__ void inv512(cpx<T> (&v)[8], cpx<T>* X, int lane, const cpx<T>* tIB, const cpx<T>* tC) {
  inv512<T>(v, X, lane, Tw512Lds<T>{tIB, tC, nullptr, lane});
}

// forward: v[y2] = g[x1 + 8 y1 + 64 y2]  ->  v[r] = G[lane + 64 r] (unnormalized)
template <typename T, typename TW>
__device__ __forceinline__ void fwd512(cpx<T> (&v)[8], cpx<T>* X, int lane, const TW& tw) {
  const int hi = lane >> 3, lo = lane & 7;
  Bfly<T, 8, -1>::run(v);
#pragma unroll
  for (int j = 1; j < 8; ++j) v[j] = cmul(v[j], tw.C(j));
#pragma unroll
  for (int j = 0; j < 8; ++j) X[xslot2(hi, lo, j)] = v[j];
  wave_sync();
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = X[xslot2(hi, j, lo)];
  wave_sync();
  Bfly<T, 8, -1>::run(v);
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = cmul(v[j], tw.FB(j));
#pragma unroll
  for (int j = 0; j < 8; ++j) X[xslot1(hi, lo + 8 * j)] = v[j];
  wave_sync();
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = X[xslot1(j, lane)];
  wave_sync();
  Bfly<T, 8, -1>::run(v);
}
template <typename T>
__device__ __forceinline__ void fwd512(cpx<T> (&v)[8], cpx<T>* X, int lane, const cpx<T>* tC, const cpx<T>* tFB) {
  fwd512<T>(v, X, lane, Tw512Lds<T>{nullptr, tC, tFB, lane});
}

// One complex value through a buffer resource whose bound is the band
// [0, nk) of a line: a lane at k >= nk loads zeros and its store is dropped,
// with no branch, no clamp and no memory traffic; the address is the
// resource's scalar base plus a 32-bit lane offset.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t band_rsrc(const cpx<T>* line, int nk) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<cpx<T>*>(line), (short)0, nk * (int)sizeof(cpx<T>),
                                           0x00020000);
}
// (whole-vector bit casts only: clang reads element 0 for a bit cast of a
// vector element such as w.y)
template <typename T>
__device__ __forceinline__ cpx<T> ld_band(__amdgpu_buffer_rsrc_t r, int k) {
  const unsigned off = (unsigned)k * (unsigned)sizeof(cpx<T>);
  typedef T F __attribute__((ext_vector_type(2)));
  F w;
  if constexpr (sizeof(T) == 4) w = __builtin_bit_cast(F, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, (FSI_NT & 8) ? 2 : 0));
  else w = __builtin_bit_cast(F, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, (FSI_NT & 8) ? 2 : 0));
  return mk<T>(w.x, w.y);
}
template <typename T>
__device__ __forceinline__ void st_band(__amdgpu_buffer_rsrc_t r, int k, cpx<T> v) {
  const unsigned off = (unsigned)k * (unsigned)sizeof(cpx<T>);
  typedef T F __attribute__((ext_vector_type(2)));
  F w;
  w.x = v.re;
  w.y = v.im;
  if constexpr (sizeof(T) == 4) {
    typedef unsigned V __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, w), r, off, 0, (FSI_NT & 1) ? 2 : 0);
  } else {
    typedef unsigned V __attribute__((ext_vector_type(4)));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V, w), r, off, 0, (FSI_NT & 1) ? 2 : 0);
  }
}

// Unpack the transforms X, Y of the two real signals packed in g (natural layout,
// g[r] = G[lane + 64 r]) and store X to dx, Y to dy for k <= K (K < 192; the
// stores beyond K fall outside the lines' band resources and are dropped).
// The partner n - k of slot r is slot 7 - r of lane 64 - lane; lane 0, which is
// its own source, offers its slot (8 - r) mod 8 instead, so no lane needs a
// select after the exchange (one would wait for every exchange in flight).
template <typename T>
__device__ __forceinline__ void unpack_store512(const cpx<T> (&g)[8], int lane, int K, cpx<T>* dx, cpx<T>* dy) {
  const int src = (64 - lane) & 63;
  const bool l0 = lane == 0;
  const __amdgpu_buffer_rsrc_t rx = band_rsrc(dx, K + 1), ry = band_rsrc(dy, K + 1);
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const cpx<T> sv = l0 ? g[(8 - r) & 7] : g[7 - r];
    cpx<T> p;
    p.re = __shfl(sv.re, src, 64);
    p.im = __shfl(sv.im, src, 64);
    const int k = lane + 64 * r;
    const cpx<T> zc = conj(p);
    const cpx<T> d = g[r] - zc;
    st_band(rx, k, scl(g[r] + zc, (T)0.5));
    st_band(ry, k, mk<T>((T)0.5 * d.im, (T)-0.5 * d.re));
  }
}

// Raw spectral values a lane needs for one packed signal of one line: A, B at
// k = lane + 64 r (r = 0, 1, 2), zero outside the 2/3 band.  The Hermitian
// partners n - k of k = lane + 64 r (r = 5, 6, 7) are the same values held by
// lane 64 - lane (r = 2, 1, 0) and are fetched across lanes by pack512.
template <typename T>
struct Raw512 {
  cpx<T> a[3], b[3];
};

// base[i] through a 32-bit unsigned byte offset: with a wave-uniform base the
// address is a scalar base plus a vector offset (no 64-bit vector arithmetic)
template <typename T>
__device__ __forceinline__ const cpx<T>* at_u32(const cpx<T>* base, int i) {
  return reinterpret_cast<const cpx<T>*>(reinterpret_cast<const char*>(base) + (unsigned)i * (unsigned)sizeof(cpx<T>));
}
template <typename T>
__device__ __forceinline__ cpx<T>* at_u32(cpx<T>* base, int i) {
  return reinterpret_cast<cpx<T>*>(reinterpret_cast<char*>(base) + (unsigned)i * (unsigned)sizeof(cpx<T>));
}

// A and B are wave-uniform line bases; the slots beyond the band (k > 170)
// load zeros from the band resources (unconditional loads: a load under a
// branch leaves the number of loads in flight unknown to the compiler, which
// then waits for all of them, including a prefetch, at the next use).
template <typename T>
__device__ __forceinline__ void load512(const cpx<T>* A, const cpx<T>* B, int lane, Raw512<T>& w) {
  constexpr int K = 170;
  const __amdgpu_buffer_rsrc_t ra = band_rsrc(A, K + 1), rb = band_rsrc(B, K + 1);
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    w.a[q] = ld_band<T>(ra, lane + 64 * q);  // direct slots r = q
    w.b[q] = ld_band<T>(rb, lane + 64 * q);
  }
}

template <typename T>
__device__ __forceinline__ cpx<T> shfl_cpx(cpx<T> v, int src) {
  return mk<T>(__shfl(v.re, src, 64), __shfl(v.im, src, 64));
}

// Z[k] = A[k] + i B[k] with the Hermitian partners, in the natural layout
// v[r] = Z[lane + 64 r].  The loads left every slot outside the band zero.  The
// partner A[n - k] of k = lane + 64 (5 + q) is slot 2 - q of lane 64 - lane;
// lane 0, which is its own source, offers its slot 3 - q instead (zero for
// q = 0: n - k = 192 lies outside the band), so no lane needs a select after
// the exchange.  At k = 0 lane 0 takes the real parts of A and B: its imaginary
// parts enter as +0 and -0, for which x - (+0) = x and (-0) + x = x exactly.
template <typename T>
__device__ __forceinline__ void pack512(const Raw512<T>& w, int lane, cpx<T> (&v)[8]) {
  const int src = (64 - lane) & 63;
  const bool l0 = lane == 0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const cpx<T> oa = q > 0 ? w.a[3 - q] : mk<T>(0, 0), ob = q > 0 ? w.b[3 - q] : mk<T>(0, 0);
    const cpx<T> pa = shfl_cpx(l0 ? oa : w.a[2 - q], src), pb = shfl_cpx(l0 ? ob : w.b[2 - q], src);
    v[5 + q] = mk<T>(pa.re + pb.im, pb.re - pa.im);
  }
  const T bim0 = l0 ? (T)0 : w.b[0].im, aim0 = l0 ? (T)-0.0 : w.a[0].im;
  v[0] = mk<T>(w.a[0].re - bim0, aim0 + w.b[0].re);
#pragma unroll
  for (int q = 1; q < 3; ++q) v[q] = mk<T>(w.a[q].re - w.b[q].im, w.a[q].im + w.b[q].re);
  v[3] = mk<T>(0, 0);
  v[4] = mk<T>(0, 0);
}

// Per-lane twiddle sets [j][lane] in LDS, from the axis table tw[m] =
// exp(+2 pi i m / 512): exp(-2 pi i lane j / 512) (inverse first stage),
// exp(+2 pi i lo j / 64) and exp(+2 pi i (lo + 8 j) hi / 512), lo = lane & 7,
// hi = lane >> 3.  Called by all NT threads of the workgroup; the caller
// synchronizes afterwards.
template <typename T, int NT>
__device__ __forceinline__ void wave512_twiddles(cpx<T> (*tws)[512], const cpx<T>* tw) {
  for (int i = threadIdx.x; i < 512; i += NT) {
    const int j = i >> 6, l = i & 63;
    tws[0][i] = conj(tw[(l * j) & 511]);
    tws[1][i] = tw[(8 * (l & 7) * j) & 511];
    tws[2][i] = tw[(((l & 7) + 8 * j) * (l >> 3)) & 511];
  }
}

}  // namespace fsi
