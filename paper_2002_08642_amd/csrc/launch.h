// launch.h - host entry points of the device passes.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace fsi {

// Upper bound of (transform length x signals) / threads held per thread in a
// pass: 64 KB of LDS per workgroup for the column passes in both precisions.
template <typename T>
struct ColMaxE;
template <>
struct ColMaxE<float> {
  static constexpr int value = 32;
};
template <>
struct ColMaxE<double> {
  static constexpr int value = 16;
};

// Same bound for the x pass (the packed signals of 2 or 4 lines).
template <typename T>
struct XMaxE;
template <>
struct XMaxE<float> {
  static constexpr int value = 40;
};
template <>
struct XMaxE<double> {
  static constexpr int value = 20;
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
template <typename T>
hipError_t launch_mask(const MaskArgs<T>& a, hipStream_t s);

}  // namespace fsi
