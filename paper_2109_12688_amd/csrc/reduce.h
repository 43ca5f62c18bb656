// Relative change of a field between two iterates, the measure of the
// threshold stopping of Sec. 4 (second hyper-parameter version).
#pragma once
#include <hip/hip_runtime.h>

#include <stddef.h>

namespace nadmm {

// Most blocks of the partial pass; `part` holds 2 doubles per block.
constexpr int kChangeBlocks = 1024;
constexpr size_t kChangeScratchBytes = 2 * kChangeBlocks * sizeof(double);

// out[0] = sum_i (a_i - b_i)^2, out[1] = sum_i a_i^2 over i < n, accumulated
// in FP64 in an order fixed by n alone (repeated calls give the same bits);
// b == nullptr reads as zero.  `part` is kChangeScratchBytes of device
// scratch; `out` is device memory or mapped pinned host memory; a and b
// 16-byte aligned.  Calls sharing `part` must be stream-ordered.
hipError_t launch_change_sums(const float* a, const float* b, size_t n, double* part, double* out,
                              hipStream_t st);

}  // namespace nadmm
