// launch.h - host entry points of the device passes.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace fsi {

// Workgroup size and per-thread element bound (transform length x signals /
// threads) of the column passes: 64 KB of LDS data per workgroup.
template <typename T>
struct ColCfg;
template <>
struct ColCfg<float> {
  static constexpr int NT = 512, MAXE = 16;
};
template <>
struct ColCfg<double> {
  static constexpr int NT = 512, MAXE = 8;
};

// Same for the x pass, per number L of lines per workgroup (3L packed signals).
template <typename T, int L>
struct XCfg;
template <>
struct XCfg<float, 4> {
  static constexpr int NT = 512, MAXE = 12;
};
template <>
struct XCfg<float, 2> {
  static constexpr int NT = 512, MAXE = 20;
};
template <>
struct XCfg<double, 4> {
  static constexpr int NT = 512, MAXE = 6;
};
template <>
struct XCfg<double, 2> {
  static constexpr int NT = 512, MAXE = 10;
};

// The fused x pass at 800 points (compile-time plan): lines per workgroup,
// threads, and the per-thread element bound (3 L 800 / NT rounded up).
template <typename T>
struct X800;
template <>
struct X800<float> {
  static constexpr int L = 2, NT = 512, MAXE = 20;
};
template <>
struct X800<double> {
  static constexpr int L = 2, NT = 512, MAXE = 10;
};

// Columns per workgroup of a column pass of length n (0 if n is too long).
template <typename T>
int col_width(int n);
// Lines per workgroup of the x pass (4 or 2).
template <typename T>
int xpass_lines(int n);

template <typename T>
hipError_t launch_col(int mode, const ColArgs<T>& a, int slices, hipStream_t s);
template <typename T>
hipError_t launch_xfused(const XArgs<T>& a, int grid, hipStream_t s);
template <typename T>
hipError_t launch_xplain(int mode, int nf, const XArgs<T>& a, int grid, hipStream_t s);
hipError_t launch_finalize(const FinalArgs& a, hipStream_t s);
int xfused_grid(int n, long long nlines, int lines_per_group);
template <typename T>
hipError_t launch_mask(const MaskArgs<T>& a, hipStream_t s);
// The same kernels writing chi and u_s into full grids [nz][ny][nx] (gnx, gny,
// gcells of MaskArgs), zeroed first; key1 / key2 may be any scratch of bcells each.
template <typename T>
hipError_t launch_mask_grid(const MaskArgs<T>& a, hipStream_t s);
// (v, v) into the padding columns [kx1, kxp) of rows of pitch kxp (testing aid)
template <typename T>
hipError_t launch_fill_pad(cpx<T>* p, long long rows, int kx1, int kxp, T v, hipStream_t s);
template <typename T>
hipError_t launch_psample(const PressArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_sponge_mask(const SpongeArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_xsponge(const XArgs<T>& a, const T* g, int grid, hipStream_t s);
template <typename T>
hipError_t launch_pbox(int embed, const BoxArgs<T>& a, hipStream_t s);

template <typename T>
hipError_t launch_xadj(const XAdjArgs<T>& a, int grid, hipStream_t s);
template <typename T>
int xadj_supported(int n);
template <typename T>
hipError_t launch_mask_adj(const MaskAdjArgs<T>& a, hipStream_t s);

}  // namespace fsi
