// Relative change of a field between two iterates, the measure of the
// threshold stopping of Sec. 4 (second hyper-parameter version).
#pragma once
#include <hip/hip_runtime.h>

#include <stddef.h>

namespace nadmm {

// Most blocks of the pass; the partials are 2 doubles per block.
constexpr int kChangeBlocks = 1024;

// Blocks the pass uses for n floats (at most kChangeBlocks).
int change_blocks(size_t n);

// Per-block partial sums of (a_i - b_i)^2 and a_i^2 over i < n, formed in
// FP64: part[2 j] and part[2 j + 1] for block j < change_blocks(n), each
// block's share of the indices fixed by n alone.  b == nullptr reads as
// zero.  `part` is device memory or mapped pinned host memory (the reader
// adds the partials in index order, so repeated calls give the same bits);
// a and b 16-byte aligned.
hipError_t launch_change_partials(const float* a, const float* b, size_t n, double* part, hipStream_t st);

}  // namespace nadmm
