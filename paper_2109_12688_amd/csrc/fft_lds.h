// Batched mixed-radix (2, 3, 4, 6, 8, 12, 16) FFTs on lines held in LDS, for gfx950.
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
//
// All per-stage integer divisions use host-precomputed reciprocals
// (FastDiv), exact for numerators and divisors below 2^16.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nadmm {

// q = floor(n / d) = (n * m) >> 32 with m = ceil(2^32 / d); exact for n, d < 2^16.
struct FastDiv {
  uint32_t d;
  uint32_t pad;
  uint64_t m;
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  f.pad = 0;
  f.m = ((uint64_t(1) << 32) + d - 1) / d;
  return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
  return (uint32_t)(((uint64_t)n * f.m) >> 32);
}

struct FftStage {
  int R, Ns, nb, twstride;  // radix, span of earlier stages, N / R, N / (Ns R)
  FastDiv div_nb, div_ns;
};

struct FftPlan {
  int n;
  int nstages;
  FftStage st[8];
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

// Compile-time cos/sin of 2 pi m / R (Taylor series on a reduced angle, in
// double), for the constant twiddles inside composite butterflies.
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double ct_cos_red(double x) {  // |x| <= pi
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
constexpr double ct_reduce(int m, int R) {  // angle of 2 pi m / R folded into [-pi, pi]
  const int mm = ((m % R) + R) % R;
  return kTwoPi * (2 * mm > R ? mm - R : mm) / R;
}
constexpr double ct_cos(int m, int R) { return ct_cos_red(ct_reduce(m, R)); }
constexpr double ct_sin(int m, int R) { return ct_cos_red(ct_reduce(m, R) - kTwoPi / 4.0); }

// Composite in-register DFT of length R1*R2 (Cooley-Tukey with
// n = R2 n1 + n2, k = k1 + R1 k2): R2 DFTs of length R1, constant twiddles
// W_R^{n2 k1}, R1 DFTs of length R2.
template <int R1, int R2, bool INV>
struct DftComposite {
  __device__ __forceinline__ static void run(float2* v) {
    constexpr int R = R1 * R2;
    float2 a[R2][R1];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) a[n2][n1] = v[R2 * n1 + n2];
      Dft<R1, INV>::run(a[n2]);
    }
#pragma unroll
    for (int n2 = 1; n2 < R2; ++n2) {
#pragma unroll
      for (int k1 = 1; k1 < R1; ++k1) {
        const float c = (float)ct_cos(n2 * k1, R);
        const float sn = (float)ct_sin(n2 * k1, R);
        // forward: exp(-i 2 pi m / R) = (c, -sn); inverse: (c, sn)
        a[n2][k1] = cmul(a[n2][k1], make_float2(c, INV ? sn : -sn));
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      float2 b[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) b[n2] = a[n2][k1];
      Dft<R2, INV>::run(b);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = b[k2];
    }
  }
};

template <bool INV>
struct Dft<6, INV> : DftComposite<2, 3, INV> {};
template <bool INV>
struct Dft<12, INV> : DftComposite<4, 3, INV> {};
template <bool INV>
struct Dft<16, INV> : DftComposite<4, 4, INV> {};

// One Stockham radix-R stage over `nlines` lines.  Element e of line l lives
// at buf[l * ls + e * es].  Consecutive threads take consecutive lines
// (lines are laid out so that this is bank-conflict free).  The caller
// guarantees nlines * N / R <= MAXB * blockDim.x.
template <int R, int MAXB, bool INV>
__device__ __forceinline__ void fft_stage(float2* buf, const float2* tw, const FftStage& s,
                                          const FastDiv& dl, int es, int ls) {
  const int nlines = (int)dl.d;
  const int total = s.nb * nlines;
  const int nthr = blockDim.x;
  float2 v[MAXB][R];
  int base[MAXB], kk[MAXB];
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int b = threadIdx.x + i * nthr;
    if (b < total) {
      const int j = (int)fdiv((uint32_t)b, dl);
      const int line = b - j * nlines;
      const int k = j - (int)fdiv((uint32_t)j, s.div_ns) * s.Ns;
      kk[i] = k;
      base[i] = line * ls + ((j - k) * R + k) * es;
      const float2* src = buf + line * ls + j * es;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = src[r * s.nb * es];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int b = threadIdx.x + i * nthr;
    if (b < total) {
      const int step = kk[i] * s.twstride;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 w = tw[r * step];
        if (INV) w.y = -w.y;
        v[i][r] = cmul(v[i][r], w);
      }
      Dft<R, INV>::run(v[i]);
      float2* dst = buf + base[i];
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * s.Ns * es] = v[i][r];
    }
  }
  __syncthreads();
}

// Full transform of every line; EPT bounds the elements per thread of any
// stage (nlines * N <= EPT * blockDim.x), which the host checks.
template <int EPT, bool INV>
__device__ void fft_lines(float2* buf, const float2* tw, const FftPlan& plan, const FastDiv& dl,
                          int es, int ls) {
  for (int s = 0; s < plan.nstages; ++s) {
    const FftStage& st = plan.st[s];
    switch (st.R) {
      case 16: fft_stage<16, (EPT + 15) / 16, INV>(buf, tw, st, dl, es, ls); break;
      case 12: fft_stage<12, (EPT + 11) / 12, INV>(buf, tw, st, dl, es, ls); break;
      case 8: fft_stage<8, (EPT + 7) / 8, INV>(buf, tw, st, dl, es, ls); break;
      case 6: fft_stage<6, (EPT + 5) / 6, INV>(buf, tw, st, dl, es, ls); break;
      case 4: fft_stage<4, (EPT + 3) / 4, INV>(buf, tw, st, dl, es, ls); break;
      case 3: fft_stage<3, (EPT + 2) / 3, INV>(buf, tw, st, dl, es, ls); break;
      default: fft_stage<2, (EPT + 1) / 2, INV>(buf, tw, st, dl, es, ls); break;
    }
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
