// device_util.h - device helpers shared by the forward and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "fft_lds.h"
#include "kernels.h"

namespace fsi {

__device__ __forceinline__ int band_to_row(int i, int K, int n) { return i <= K ? i : i + n - 2 * K - 1; }
__device__ __forceinline__ int band_mode(int i, int K) { return i <= K ? i : i - 2 * K - 1; }

template <typename T>
__device__ __forceinline__ T dev_exp(T a);
template <>
__device__ __forceinline__ float dev_exp<float>(float a) { return expf(a); }
template <>
__device__ __forceinline__ double dev_exp<double>(double a) { return exp(a); }

template <typename T>
__device__ __forceinline__ T dev_sqrt(T a);
template <>
__device__ __forceinline__ float dev_sqrt<float>(float a) { return sqrtf(a); }
template <>
__device__ __forceinline__ double dev_sqrt<double>(double a) { return sqrt(a); }

// Fixed-order workgroup sum of NV doubles; result valid in thread 0.
template <int NV, int NT>
__device__ void block_sum(double (&v)[NV], double* red /* [NV][NT/64] */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_down(v[i], off, 64);
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[i * (NT / 64) + wave] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int w = 0; w < NT / 64; ++w) s += red[i * (NT / 64) + w];
      v[i] = s;
    }
  }
}

template <int NT>
__device__ __forceinline__ double block_max(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  if (lane == 0) red[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 0; w < NT / 64; ++w) v = fmax(v, red[w]);
  }
  return v;
}

template <int W>
struct PadStride {
  static constexpr int value = (W % 2 == 0) ? W + 1 : W;
};

// Closest point of triangle (a, b, c) to p by Voronoi-region classification
// (vertex, edge or face region).  Coordinates are relative to a.  Returns the
// squared distance and the barycentric weights (wa, wb, wc).
// Which feature of the triangle holds the closest point (for the mask adjoint):
// kind 0 = face (barycentrics wb = beta, wc = gamma), 1 = edge from local vertex
// i0 to i1 at parameter t, 2 = vertex.
struct TriRegion {
  int kind, i0, i1;
  double t;
};

template <typename T>
__device__ __forceinline__ T closest_on_triangle(T px, T py, T pz, T bx, T by, T bz, T cx, T cy, T cz, T& wa, T& wb,
                                                 T& wc, TriRegion* rg = nullptr) {
  TriRegion dummy;
  TriRegion& R = rg ? *rg : dummy;
  R.kind = 2;
  R.i0 = 0;
  R.i1 = 0;
  R.t = 0;
  // p, b, c are relative to vertex a
  const T d1 = bx * px + by * py + bz * pz;
  const T d2 = cx * px + cy * py + cz * pz;
  T qx, qy, qz;
  if (d1 <= (T)0 && d2 <= (T)0) {
    wa = 1; wb = 0; wc = 0;
    qx = 0; qy = 0; qz = 0;
  } else {
    const T bpx = px - bx, bpy = py - by, bpz = pz - bz;
    const T d3 = bx * bpx + by * bpy + bz * bpz;
    const T d4 = cx * bpx + cy * bpy + cz * bpz;
    const T cpx_ = px - cx, cpy = py - cy, cpz = pz - cz;
    const T d5 = bx * cpx_ + by * cpy + bz * cpz;
    const T d6 = cx * cpx_ + cy * cpy + cz * cpz;
    const T vc = d1 * d4 - d3 * d2;
    const T vb = d5 * d2 - d1 * d6;
    const T va = d3 * d6 - d5 * d4;
    if (d3 >= (T)0 && d4 <= d3) {
      R.kind = 2;
      R.i0 = 1;
      wa = 0; wb = 1; wc = 0;
      qx = bx; qy = by; qz = bz;
    } else if (vc <= (T)0 && d1 >= (T)0 && d3 <= (T)0) {
      const T t = d1 / (d1 - d3);
      R.kind = 1; R.i0 = 0; R.i1 = 1; R.t = t;
      wa = 1 - t; wb = t; wc = 0;
      qx = t * bx; qy = t * by; qz = t * bz;
    } else if (d6 >= (T)0 && d5 <= d6) {
      R.kind = 2;
      R.i0 = 2;
      wa = 0; wb = 0; wc = 1;
      qx = cx; qy = cy; qz = cz;
    } else if (vb <= (T)0 && d2 >= (T)0 && d6 <= (T)0) {
      const T t = d2 / (d2 - d6);
      R.kind = 1; R.i0 = 0; R.i1 = 2; R.t = t;
      wa = 1 - t; wb = 0; wc = t;
      qx = t * cx; qy = t * cy; qz = t * cz;
    } else if (va <= (T)0 && (d4 - d3) >= (T)0 && (d5 - d6) >= (T)0) {
      const T t = (d4 - d3) / ((d4 - d3) + (d5 - d6));
      R.kind = 1; R.i0 = 1; R.i1 = 2; R.t = t;
      wa = 0; wb = 1 - t; wc = t;
      qx = bx + t * (cx - bx); qy = by + t * (cy - by); qz = bz + t * (cz - bz);
    } else {
      const T den = va + vb + vc;
      if (den > (T)0) {
        const T vv = vb / den, ww = vc / den;
        R.kind = 0;
        wa = 1 - vv - ww; wb = vv; wc = ww;
        qx = vv * bx + ww * cx; qy = vv * by + ww * cy; qz = vv * bz + ww * cz;
      } else {
        // degenerate triangle: nearest of the three edges
        T best = (T)INFINITY;
        wa = 1; wb = 0; wc = 0;
        qx = 0; qy = 0; qz = 0;
        const T ex[3][6] = {{0, 0, 0, bx, by, bz}, {bx, by, bz, cx, cy, cz}, {cx, cy, cz, 0, 0, 0}};
        for (int e = 0; e < 3; ++e) {
          const T ax_ = ex[e][0], ay_ = ex[e][1], az_ = ex[e][2];
          const T sx = ex[e][3] - ax_, sy = ex[e][4] - ay_, sz = ex[e][5] - az_;
          const T ss = sx * sx + sy * sy + sz * sz;
          T t = ss > (T)0 ? ((px - ax_) * sx + (py - ay_) * sy + (pz - az_) * sz) / ss : (T)0;
          t = t < (T)0 ? (T)0 : (t > (T)1 ? (T)1 : t);
          const T hx = ax_ + t * sx - px, hy = ay_ + t * sy - py, hz = az_ + t * sz - pz;
          const T dd = hx * hx + hy * hy + hz * hz;
          if (dd < best) {
            best = dd;
            qx = ax_ + t * sx; qy = ay_ + t * sy; qz = az_ + t * sz;
            if (e == 0) { wa = 1 - t; wb = t; wc = 0; R.kind = 1; R.i0 = 0; R.i1 = 1; R.t = t; }
            else if (e == 1) { wa = 0; wb = 1 - t; wc = t; R.kind = 1; R.i0 = 1; R.i1 = 2; R.t = t; }
            else { wa = t; wb = 0; wc = 1 - t; R.kind = 1; R.i0 = 2; R.i1 = 0; R.t = t; }
          }
        }
      }
    }
  }
  const T hx = px - qx, hy = py - qy, hz = pz - qz;
  return hx * hx + hy * hy + hz * hz;
}

__device__ __forceinline__ double profile_chi(double d, double tw, double h, int profile) {
  if (profile == 0) {
    if (d <= tw - h) return 1.0;
    if (d >= tw + h) return 0.0;
    return 0.5 * (1.0 + cos(3.14159265358979323846 * (d - tw + h) / (2.0 * h)));
  }
  return 0.5 * (1.0 - tanh((d - tw) / h));
}


}  // namespace fsi
