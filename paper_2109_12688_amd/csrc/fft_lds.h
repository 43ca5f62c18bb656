// Batched mixed-radix (2, 3, 4, 8) FFTs on lines held in LDS, for gfx950.
//
// A workgroup transforms `nlines` lines of length N in place.  Each stage is
// a Stockham autosort radix-R pass (output in natural order, no digit
// reversal): butterfly j of a line reads elements j + r*N/R, multiplies
// element r by W_{Ns R}^{(j mod Ns) r}, takes a length-R DFT and writes the
// results to ((j - j mod Ns) R + j mod Ns) + r Ns, where Ns is the product of
// the radices of the earlier stages.  A stage first loads every butterfly
// the thread owns into registers, then barriers, then writes, so a single
// LDS buffer suffices.
//
// Twiddles come from an LDS table tw[i] = exp(-2 pi i * i / N), i < N,
// generated in float64 and rounded once to float32.  Forward transforms use
// exp(-...), inverse ones exp(+...) without the 1/N factor.
#pragma once
#include <hip/hip_runtime.h>

namespace nadmm {

struct FftPlan {
  int n;
  int nstages;
  int radix[8];
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// In-register DFTs of length 2, 3, 4, 8: y_k = sum_r x_r exp(-+2 pi i r k / R).
template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<2, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV>
struct Dft<3, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    const float h = 0.8660254037844386f;  // sin(2 pi / 3)
    float2 a = v[0], b = v[1], c = v[2];
    float2 s = cadd(b, c);
    float2 d = csub(b, c);
    float2 m = make_float2(a.x - 0.5f * s.x, a.y - 0.5f * s.y);
    // forward: y1 = m - i h d, y2 = m + i h d ; inverse swaps the signs
    float2 ihd = make_float2(-h * d.y, h * d.x);
    v[0] = cadd(a, s);
    if (INV) {
      v[1] = cadd(m, ihd);
      v[2] = csub(m, ihd);
    } else {
      v[1] = csub(m, ihd);
      v[2] = cadd(m, ihd);
    }
  }
};

template <bool INV>
struct Dft<4, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    float2 t2 = cadd(v[1], v[3]), t3 = mul_mi<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <bool INV>
struct Dft<8, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    const float r2 = 0.70710678118654752f;
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, INV>::run(e);
    Dft<4, INV>::run(o);
    // o_k *= W8^k  (W8 = exp(-+ i pi / 4))
    float2 o1 = INV ? make_float2(r2 * (o[1].x - o[1].y), r2 * (o[1].x + o[1].y))
                    : make_float2(r2 * (o[1].x + o[1].y), r2 * (o[1].y - o[1].x));
    float2 o2 = mul_mi<INV>(o[2]);
    float2 o3 = INV ? make_float2(-r2 * (o[3].x + o[3].y), r2 * (o[3].x - o[3].y))
                    : make_float2(r2 * (o[3].y - o[3].x), -r2 * (o[3].x + o[3].y));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

// One Stockham radix-R stage over `nlines` lines.  Element e of line l lives
// at buf[l * ls + e * es].  LINE_FAST maps consecutive threads to consecutive
// lines (use when lines are adjacent in LDS), otherwise to consecutive
// butterflies within a line.  The caller guarantees
// nlines * N / R <= MAXB * blockDim.x.
template <int R, int MAXB, bool INV, bool LINE_FAST>
__device__ __forceinline__ void fft_stage(float2* buf, const float2* tw, int N, int Ns, int nlines,
                                          int es, int ls) {
  const int nb = N / R;
  const int total = nb * nlines;
  const int nthr = blockDim.x;
  float2 v[MAXB][R];
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int b = threadIdx.x + i * nthr;
    if (b < total) {
      const int line = LINE_FAST ? b % nlines : b / nb;
      const int j = LINE_FAST ? b / nlines : b % nb;
      const float2* src = buf + line * ls + j * es;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = src[r * nb * es];
    }
  }
  __syncthreads();
  const int twstride = N / (Ns * R);
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int b = threadIdx.x + i * nthr;
    if (b < total) {
      const int line = LINE_FAST ? b % nlines : b / nb;
      const int j = LINE_FAST ? b / nlines : b % nb;
      const int k = j % Ns;
      const int step = k * twstride;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 w = tw[r * step];
        if (INV) w.y = -w.y;
        v[i][r] = cmul(v[i][r], w);
      }
      Dft<R, INV>::run(v[i]);
      float2* dst = buf + line * ls + ((j - k) * R + k) * es;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * Ns * es] = v[i][r];
    }
  }
  __syncthreads();
}

// Full transform of every line; EPT bounds the elements per thread of any
// stage (nlines * N <= EPT * blockDim.x), which the host checks.
template <int EPT, bool INV, bool LINE_FAST>
__device__ void fft_lines(float2* buf, const float2* tw, const FftPlan& plan, int nlines, int es,
                          int ls) {
  int Ns = 1;
  for (int s = 0; s < plan.nstages; ++s) {
    const int R = plan.radix[s];
    switch (R) {
      case 8: fft_stage<8, (EPT + 7) / 8, INV, LINE_FAST>(buf, tw, plan.n, Ns, nlines, es, ls); break;
      case 4: fft_stage<4, (EPT + 3) / 4, INV, LINE_FAST>(buf, tw, plan.n, Ns, nlines, es, ls); break;
      case 3: fft_stage<3, (EPT + 2) / 3, INV, LINE_FAST>(buf, tw, plan.n, Ns, nlines, es, ls); break;
      default: fft_stage<2, (EPT + 1) / 2, INV, LINE_FAST>(buf, tw, plan.n, Ns, nlines, es, ls); break;
    }
    Ns *= R;
  }
}

// tw[i] = exp(-2 pi i * i / n) for i < n, computed in float64.
__device__ __forceinline__ void make_twiddles(float2* tw, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double s, c;
    sincospi(-2.0 * (double)i / (double)n, &s, &c);
    tw[i] = make_float2((float)c, (float)s);
  }
}

}  // namespace nadmm
