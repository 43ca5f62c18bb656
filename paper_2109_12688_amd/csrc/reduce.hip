// Sums of squares for the relative change |a - b| / |a| of two iterates
// (the measure of the threshold stopping of Sec. 4): one pass of up to
// kChangeBlocks blocks, each writing its FP64 partial sums where the caller
// reads them (mapped pinned host memory: no copy and no second launch).
// Differences and squares are formed in FP64 (the difference of two
// float32 values is exact there).
#include "reduce.h"

namespace nadmm {

namespace {

constexpr int kThreads = 256;

__device__ inline void block_sum2(double& d, double& s) {
  __shared__ double sd[kThreads], ss[kThreads];
  const int t = threadIdx.x;
  sd[t] = d;
  ss[t] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (t < w) {
      sd[t] += sd[t + w];
      ss[t] += ss[t + w];
    }
    __syncthreads();
  }
  d = sd[0];
  s = ss[0];
}

__device__ inline void acc(double& d, double& s, float x, float y) {
  const double e = (double)x - (double)y;
  d = fma(e, e, d);
  s = fma((double)x, (double)x, s);
}

__global__ void __launch_bounds__(kThreads) k_change_partial(const float* __restrict__ a,
                                                             const float* __restrict__ b, size_t n,
                                                             double* part) {
  double d = 0.0, s = 0.0;
  const size_t n4 = n / 4, stride = (size_t)gridDim.x * kThreads;
  const float4* a4 = reinterpret_cast<const float4*>(a);
  const float4* b4 = reinterpret_cast<const float4*>(b);
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n4; i += stride) {
    const float4 x = a4[i];
    const float4 y = b ? b4[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    acc(d, s, x.x, y.x);
    acc(d, s, x.y, y.y);
    acc(d, s, x.z, y.z);
    acc(d, s, x.w, y.w);
  }
  if (blockIdx.x == 0 && threadIdx.x < n - 4 * n4) {  // the last n % 4 values
    const size_t i = 4 * n4 + threadIdx.x;
    acc(d, s, a[i], b ? b[i] : 0.f);
  }
  block_sum2(d, s);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = d;
    part[2 * blockIdx.x + 1] = s;
  }
}

}  // namespace

int change_blocks(size_t n) {
  const size_t nb = (n / 4 + kThreads - 1) / kThreads;
  return nb < 1 ? 1 : (nb > (size_t)kChangeBlocks ? kChangeBlocks : (int)nb);
}

hipError_t launch_change_partials(const float* a, const float* b, size_t n, double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_change_partial, dim3((unsigned)change_blocks(n)), dim3(kThreads), 0, st, a, b, n, part);
  return hipGetLastError();
}

}  // namespace nadmm
