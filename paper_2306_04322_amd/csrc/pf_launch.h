// Host-side launchers for the kernel templates.  Each returns the number of
// work-groups it launched (the number of partial-sum records written when
// the kernel accumulates), or -1 for an unsupported size.
#pragma once

#include <hip/hip_runtime.h>

#include "pf_fe.h"
#include "pf_fft.h"

namespace pf {

template <typename T> struct XArgs;
template <typename T> struct ColArgs;
template <typename T> struct AdjArgs;
template <typename T> struct FdArgs;

template <typename T> int row_launch(int nx, int p, const XArgs<T>& a, hipStream_t s);
template <typename T> int adj_row_launch(int nx, int p, const AdjArgs<T>& a, hipStream_t s);
template <typename T> int col_launch(int n, int nouter, const ColArgs<T>& a, hipStream_t s);
template <typename T> int fd_launch(int which, int p, const FdArgs<T>& a, hipStream_t s);
int reduce_launch(const double* partials, int n, int width, double* out, const double* scale4,
                  int accumulate, hipStream_t s);

}  // namespace pf
