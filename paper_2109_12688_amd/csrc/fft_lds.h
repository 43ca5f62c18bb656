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
  uint32_t d = 1;
  uint32_t pad = 0;
  uint64_t m = 0;
};

constexpr FastDiv make_fastdiv(uint32_t d) {
  return FastDiv{d, 0u, ((uint64_t(1) << 32) + d - 1) / d};
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
  return (uint32_t)(((uint64_t)n * f.m) >> 32);
}

struct FftStage {
  int R = 0, Ns = 0, nb = 0, twstride = 0;  // radix, span of earlier stages, N / R, N / (Ns R)
  FastDiv div_nb{}, div_ns{};
};

struct FftPlan {
  int n;
  int nstages;
  FftStage st[8];
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * b (INV false) or a * conj(b) (INV true)
template <bool INV>
__device__ __forceinline__ float2 cmul_tw(float2 a, float2 b) {
  return INV ? make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y) : cmul(a, b);
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

// a * exp(-+ 2 pi i m / R) for a compile-time m: quarter turns are exact
// swaps and negations, eighth turns use the single constant sqrt(1/2), other
// angles a complex multiply by constants rounded once from the series above.
template <int R, bool INV>
__device__ __forceinline__ float2 ctwiddle(float2 a, int m) {
  const int q8 = ((m % R) + R) % R * 8;  // angle in eighths of a turn when q8 % R == 0
  if (q8 % R == 0) {
    // forward turns clockwise: exp(-i pi e / 4); inverse counter-clockwise
    const int e = INV ? (8 - q8 / R) % 8 : q8 / R;
    const float h = 0.70710678118654752f;
    switch (e) {
      case 0: return a;
      case 1: return make_float2(h * (a.x + a.y), h * (a.y - a.x));
      case 2: return make_float2(a.y, -a.x);
      case 3: return make_float2(h * (a.y - a.x), -h * (a.x + a.y));
      case 4: return make_float2(-a.x, -a.y);
      case 5: return make_float2(-h * (a.x + a.y), h * (a.x - a.y));
      case 6: return make_float2(-a.y, a.x);
      default: return make_float2(h * (a.x - a.y), h * (a.x + a.y));
    }
  }
  const float c = (float)ct_cos(m, R);
  const float sn = (float)ct_sin(m, R);
  // forward: exp(-i 2 pi m / R) = (c, -sn); inverse: (c, sn)
  return cmul(a, make_float2(c, INV ? sn : -sn));
}

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
      for (int k1 = 1; k1 < R1; ++k1) a[n2][k1] = ctwiddle<R, INV>(a[n2][k1], n2 * k1);
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

// Prime-factor (Good-Thomas) DFT of length R1*R2 for coprime R1, R2: with
// n = (R2 n1 + R1 n2) mod R and k the index with k = k1 mod R1, k = k2 mod R2,
// exp(-+2 pi i n k / R) = exp(-+2 pi i n1 k1 / R1) exp(-+2 pi i n2 k2 / R2),
// so R2 DFTs of length R1 and R1 DFTs of length R2 need no twiddles between
// them (both index maps are compile-time register permutations).
template <int R1, int R2>
struct PfaMaps {
  int in[R2][R1];   // input index of (n1, n2)
  int out[R1][R2];  // output index of (k1, k2)
};
template <int R1, int R2>
constexpr PfaMaps<R1, R2> make_pfa_maps() {
  PfaMaps<R1, R2> m{};
  for (int n2 = 0; n2 < R2; ++n2)
    for (int n1 = 0; n1 < R1; ++n1) m.in[n2][n1] = (R2 * n1 + R1 * n2) % (R1 * R2);
  for (int k = 0; k < R1 * R2; ++k) m.out[k % R1][k % R2] = k;
  return m;
}
template <int R1, int R2, bool INV>
struct DftPfa {
  static constexpr PfaMaps<R1, R2> M = make_pfa_maps<R1, R2>();
  __device__ __forceinline__ static void run(float2* v) {
    float2 a[R2][R1];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) a[n2][n1] = v[M.in[n2][n1]];
      Dft<R1, INV>::run(a[n2]);
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      float2 b[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) b[n2] = a[n2][k1];
      Dft<R2, INV>::run(b);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) v[M.out[k1][k2]] = b[k2];
    }
  }
};

template <bool INV>
struct Dft<6, INV> : DftPfa<2, 3, INV> {};
template <bool INV>
struct Dft<12, INV> : DftPfa<4, 3, INV> {};
template <bool INV>
struct Dft<16, INV> : DftComposite<4, 4, INV> {};

// Position of element e inside a line: with PADSH > 0 one slot of padding
// follows every 2^PADSH elements (breaks the stride-R writes of early
// Stockham stages across LDS banks).
template <int PADSH>
__host__ __device__ __forceinline__ int lpad(int e) {
  return PADSH > 0 ? e + (e >> PADSH) : e;
}

// One Stockham radix-R stage over `nlines` lines.  Element e of line l lives
// at buf[l * ls + lpad<PADSH>(e) * es].  LINE_FAST maps consecutive threads
// to consecutive lines (for lines adjacent in LDS), otherwise to consecutive
// butterflies of one line.  The caller guarantees
// nlines * N / R <= MAXB * blockDim.x.
template <int R, int MAXB, bool INV, bool LINE_FAST, int PADSH>
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
      int j, line;
      if (LINE_FAST) {
        j = (int)fdiv((uint32_t)b, dl);
        line = b - j * nlines;
      } else {
        line = (int)fdiv((uint32_t)b, s.div_nb);
        j = b - line * s.nb;
      }
      const int k = j - (int)fdiv((uint32_t)j, s.div_ns) * s.Ns;
      base[i] = line * ls;
      // low 16 bits: k = j mod Ns; high bits: destination element of r = 0
      kk[i] = k | (((j - k) * R + k) << 16);
      const float2* src = buf + line * ls;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = src[lpad<PADSH>(j + r * s.nb) * es];
    }
  }
  __syncthreads();
  const int twstride = s.twstride;
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int b = threadIdx.x + i * nthr;
    if (b < total) {
      const int k = kk[i] & 0xffff;
      const int d0 = kk[i] >> 16;
      if (s.Ns > 1) {  // the first stage's twiddles are all 1
        const int step = k * twstride;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          v[i][r] = cmul_tw<INV>(v[i][r], tw[r * step]);
        }
      }
      Dft<R, INV>::run(v[i]);
      float2* dst = buf + base[i];
#pragma unroll
      for (int r = 0; r < R; ++r) dst[lpad<PADSH>(d0 + r * s.Ns) * es] = v[i][r];
    }
  }
  __syncthreads();
}

// Full transform of every line; EPT bounds the elements per thread of any
// stage (nlines * N <= EPT * blockDim.x), which the host checks.
template <int EPT, bool INV, bool LINE_FAST = true, int PADSH = 0>
__device__ void fft_lines(float2* buf, const float2* tw, const FftPlan& plan, const FastDiv& dl,
                          int es, int ls) {
  for (int s = 0; s < plan.nstages; ++s) {
    const FftStage& st = plan.st[s];
    switch (st.R) {
      case 16: fft_stage<16, (EPT + 15) / 16, INV, LINE_FAST, PADSH>(buf, tw, st, dl, es, ls); break;
      case 12: fft_stage<12, (EPT + 11) / 12, INV, LINE_FAST, PADSH>(buf, tw, st, dl, es, ls); break;
      case 8: fft_stage<8, (EPT + 7) / 8, INV, LINE_FAST, PADSH>(buf, tw, st, dl, es, ls); break;
      case 6: fft_stage<6, (EPT + 5) / 6, INV, LINE_FAST, PADSH>(buf, tw, st, dl, es, ls); break;
      case 4: fft_stage<4, (EPT + 3) / 4, INV, LINE_FAST, PADSH>(buf, tw, st, dl, es, ls); break;
      case 3: fft_stage<3, (EPT + 2) / 3, INV, LINE_FAST, PADSH>(buf, tw, st, dl, es, ls); break;
      default: fft_stage<2, (EPT + 1) / 2, INV, LINE_FAST, PADSH>(buf, tw, st, dl, es, ls); break;
    }
  }
}

// Stockham plans fixed at compile time: fewest stages for n with radices
// from {16, 12, 8, 6, 4, 3, 2}, and among plans with equally few stages the
// one with the largest leading radices.  The host builds its run-time plans
// from the same search.
struct StockhamRadices {
  int nstages = -1;
  int R[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};

constexpr bool stockham_search_ce(int m, int depth, int* out) {
  if (m == 1) return depth == 0;
  if (depth == 0) return false;
  const int radices[7] = {16, 12, 8, 6, 4, 3, 2};
  for (int i = 0; i < 7; ++i) {
    const int r = radices[i];
    if (m % r == 0 && stockham_search_ce(m / r, depth - 1, out + 1)) {
      out[0] = r;
      return true;
    }
  }
  return false;
}

constexpr StockhamRadices stockham_radices_ce(int n) {
  StockhamRadices p{};
  for (int depth = 1; depth <= 8; ++depth) {
    int rad[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (stockham_search_ce(n, depth, rad)) {
      p.nstages = depth;
      for (int i = 0; i < depth; ++i) p.R[i] = rad[i];
      return p;
    }
  }
  return p;
}

// radix of the stage whose earlier stages span ns elements (0: none)
constexpr int stockham_radix_at(int n, int ns) {
  const StockhamRadices p = stockham_radices_ce(n);
  int span = 1;
  for (int i = 0; i < p.nstages; ++i) {
    if (span == ns) return p.R[i];
    span *= p.R[i];
  }
  return 0;
}

// One radix-R stage of a length-N transform with every index constant but
// the line count; butterflies of one line on consecutive threads and
// element e of line l at buf[l * ls + lpad<PADSH>(e)].  The caller
// guarantees nlines * N / R <= MAXB * blockDim.x.
template <int R, int NS, int N, int MAXB, bool INV, int PADSH>
__device__ __forceinline__ void fft_stage_ct(float2* buf, const float2* tw, int nlines, int ls) {
  constexpr int NB = N / R, TWS = N / (NS * R);
  const uint32_t total = (uint32_t)(NB * nlines);
  const uint32_t nthr = blockDim.x;
  float2 v[MAXB][R];
  int base[MAXB], jj[MAXB];
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const uint32_t b = threadIdx.x + i * nthr;
    if (b < total) {
      const uint32_t line = b / (uint32_t)NB;
      const int j = (int)(b - line * NB);
      base[i] = (int)line * ls;
      jj[i] = j;
      const float2* src = buf + base[i];
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = src[lpad<PADSH>(j + r * NB)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const uint32_t b = threadIdx.x + i * nthr;
    if (b < total) {
      const int j = jj[i];
      const int k = (int)((uint32_t)j % (uint32_t)NS);
      if constexpr (NS > 1) {  // the first stage's twiddles are all 1
        const int step = k * TWS;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          v[i][r] = cmul_tw<INV>(v[i][r], tw[r * step]);
        }
      }
      Dft<R, INV>::run(v[i]);
      float2* dst = buf + base[i];
      const int d0 = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[lpad<PADSH>(d0 + r * NS)] = v[i][r];
    }
  }
  __syncthreads();
}

// Full length-N transform of `nlines` lines with the compile-time plan;
// nlines * N <= EPT * blockDim.x.
template <int N, int EPT, bool INV, int PADSH, int NS = 1>
__device__ __forceinline__ void fft_lines_ct(float2* buf, const float2* tw, int nlines, int ls) {
  if constexpr (NS < N) {
    constexpr int R = stockham_radix_at(N, NS);
    static_assert(R > 1, "no Stockham plan for this length");
    fft_stage_ct<R, NS, N, (EPT + R - 1) / R, INV, PADSH>(buf, tw, nlines, ls);
    fft_lines_ct<N, EPT, INV, PADSH, NS * R>(buf, tw, nlines, ls);
  }
}

// ---------------------------------------------------------------------------
// Wave-team FFTs: every line is transformed by a team of L lanes of ONE
// wavefront, so the stages of a line need no workgroup barrier; LDS
// operations of a wavefront are performed in issue order and the fences
// below only stop the compiler from moving them.  Inside a wavefront, lane
// = tl * (64 / L) + li: li picks one of the 64 / L lines the wavefront owns
// (consecutive lanes touch consecutive lines, which the LDS layouts keep on
// distinct banks), tl the team lane, which takes butterflies tl, tl + L, ...
// of every stage.  The host planner only picks radices with L | N / R.
// ---------------------------------------------------------------------------
struct TeamPlan {
  int n = 0, nstages = -1, L = 1;
  FftStage st[4] = {};
};

// Planner (usable on the host and at compile time).  Points per lane are
// bounded by kTeamEpt; the team size L <= max_lanes is a power of two and
// every stage's butterfly count n / R must be a multiple of L; plans with
// the fewest stages win, larger L on ties.
constexpr int kTeamEpt = 27;

constexpr void team_fill(TeamPlan& p, const int* rad) {
  int ns = 1;
  for (int i = 0; i < p.nstages; ++i) {
    FftStage& s = p.st[i];
    s.R = rad[i];
    s.Ns = ns;
    s.nb = p.n / s.R;
    s.twstride = p.n / (ns * s.R);
    s.div_nb = make_fastdiv(s.nb);
    s.div_ns = make_fastdiv(ns);
    ns *= s.R;
  }
}

constexpr bool team_search(int n, int m, int L, int depth, int* out) {
  const int radices[7] = {16, 12, 8, 6, 4, 3, 2};
  if (m == 1) return depth == 0;
  if (depth == 0) return false;
  for (int i = 0; i < 7; ++i) {
    const int R = radices[i];
    if (m % R == 0 && (n / R) % L == 0 && team_search(n, m / R, L, depth - 1, out + 1)) {
      out[0] = R;
      return true;
    }
  }
  return false;
}

constexpr TeamPlan make_team_plan_ce(int n, int max_lanes) {
  TeamPlan best{};
  best.n = n;
  best.nstages = -1;
  const int Ls[5] = {16, 8, 4, 2, 1};
  for (int li = 0; li < 5; ++li) {
    const int L = Ls[li];
    if (L > max_lanes || n % L || n / L > kTeamEpt) continue;
    int rad[4] = {0, 0, 0, 0};
    for (int depth = 1; depth <= 4; ++depth) {
      if (team_search(n, n, L, depth, rad)) {
        if (best.nstages < 0 || depth < best.nstages) {
          best.nstages = depth;
          best.L = L;
          team_fill(best, rad);
        }
        break;
      }
    }
  }
  return best;
}

constexpr TeamPlan reverse_team_plan_ce(const TeamPlan& p) {
  TeamPlan q = p;
  int rad[4] = {0, 0, 0, 0};
  for (int i = 0; i < p.nstages; ++i) rad[i] = p.st[p.nstages - 1 - i].R;
  team_fill(q, rad);
  return q;
}

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Butterfly j of a stage: load its R inputs of a line.
template <int R, int PADSH>
__device__ __forceinline__ void team_load(const float2* line, int es, const FftStage& s, int j,
                                          float2* v) {
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = line[lpad<PADSH>(j + r * s.nb) * es];
}

// Twiddle and DFT of butterfly j in registers.
template <int R, bool INV>
__device__ __forceinline__ void team_compute(const float2* tw, const FftStage& s, int j,
                                             float2* v) {
  if (s.Ns > 1) {
    const int k = j - (int)fdiv((uint32_t)j, s.div_ns) * s.Ns;
    const int step = k * s.twstride;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      v[r] = cmul_tw<INV>(v[r], tw[r * step]);
    }
  }
  Dft<R, INV>::run(v);
}

template <int R, int PADSH>
__device__ __forceinline__ void team_store(float2* line, int es, const FftStage& s, int j,
                                           const float2* v) {
  const int k = j - (int)fdiv((uint32_t)j, s.div_ns) * s.Ns;
  const int d0 = (j - k) * R + k;
#pragma unroll
  for (int r = 0; r < R; ++r) line[lpad<PADSH>(d0 + r * s.Ns) * es] = v[r];
}

// One stage of a team over its line: all loads, then (fenced) all stores.
// Source and destination may differ (e.g. a row in global memory and its
// padded copy in LDS); element e lives at src[lpad<PADS>(e) * ses] and
// dst[lpad<PADD>(e) * des].
template <int R, int EPT, bool INV, int PADS, int PADD>
__device__ __forceinline__ void team_stage_io(const float2* src, int ses, float2* dst, int des,
                                              const float2* tw, const FftStage& s, int L, int tl) {
  constexpr int M = EPT / R;  // nm * R = n / L <= EPT, so nm <= EPT / R
  const int nm = s.nb / L;     // butterflies per lane (exact by the plan)
  float2 v[M][R];
#pragma unroll
  for (int m = 0; m < M; ++m)
    if (m < nm) team_load<R, PADS>(src, ses, s, tl + m * L, v[m]);
  wave_lds_fence();
#pragma unroll
  for (int m = 0; m < M; ++m)
    if (m < nm) {
      team_compute<R, INV>(tw, s, tl + m * L, v[m]);
      team_store<R, PADD>(dst, des, s, tl + m * L, v[m]);
    }
  wave_lds_fence();
}

template <int R, int EPT, bool INV, int PADSH>
__device__ __forceinline__ void team_stage(float2* line, const float2* tw, const FftStage& s,
                                           int L, int tl, int es) {
  team_stage_io<R, EPT, INV, PADSH, PADSH>(line, es, line, es, tw, s, L, tl);
}

template <int EPT, bool INV, int PADS, int PADD>
__device__ __forceinline__ void team_stage_io_any(const float2* src, int ses, float2* dst, int des,
                                                  const float2* tw, const FftStage& s, int L,
                                                  int tl) {
  switch (s.R) {
    case 16: team_stage_io<16, EPT, INV, PADS, PADD>(src, ses, dst, des, tw, s, L, tl); break;
    case 12: team_stage_io<12, EPT, INV, PADS, PADD>(src, ses, dst, des, tw, s, L, tl); break;
    case 8: team_stage_io<8, EPT, INV, PADS, PADD>(src, ses, dst, des, tw, s, L, tl); break;
    case 6: team_stage_io<6, EPT, INV, PADS, PADD>(src, ses, dst, des, tw, s, L, tl); break;
    case 4: team_stage_io<4, EPT, INV, PADS, PADD>(src, ses, dst, des, tw, s, L, tl); break;
    case 3: team_stage_io<3, EPT, INV, PADS, PADD>(src, ses, dst, des, tw, s, L, tl); break;
    default: team_stage_io<2, EPT, INV, PADS, PADD>(src, ses, dst, des, tw, s, L, tl); break;
  }
}

template <int EPT, bool INV, int PADSH>
__device__ __forceinline__ void team_stage_any(float2* line, const float2* tw, const FftStage& s,
                                               int L, int tl, int es) {
  switch (s.R) {
    case 16: team_stage<16, EPT, INV, PADSH>(line, tw, s, L, tl, es); break;
    case 12: team_stage<12, EPT, INV, PADSH>(line, tw, s, L, tl, es); break;
    case 8: team_stage<8, EPT, INV, PADSH>(line, tw, s, L, tl, es); break;
    case 6: team_stage<6, EPT, INV, PADSH>(line, tw, s, L, tl, es); break;
    case 4: team_stage<4, EPT, INV, PADSH>(line, tw, s, L, tl, es); break;
    case 3: team_stage<3, EPT, INV, PADSH>(line, tw, s, L, tl, es); break;
    default: team_stage<2, EPT, INV, PADSH>(line, tw, s, L, tl, es); break;
  }
}

// Stages [s0, s1) of the plan on every line.  The plan must live in LDS (or
// other addressable memory): stages are indexed at run time.
// LINEPAD: line l starts at lpad<PADSH>(l) * ls instead of l * ls (used when
// the lines are the padded columns of a row-major plane).
template <int EPT, bool INV, int PADSH = 0, bool LINEPAD = false>
__device__ __forceinline__ void team_fft(float2* buf, const float2* tw, const TeamPlan& p,
                                         int nlines, int es, int ls, int s0 = 0, int s1 = 4) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int nlw = 64 / p.L;
  const int li = lane % nlw, tl = lane / nlw;
  const int se = s1 < p.nstages ? s1 : p.nstages;
  for (int l0 = wave * nlw; l0 < nlines; l0 += nwaves * nlw) {
    const int l = l0 + li;
    if (l < nlines) {
      float2* line = buf + (LINEPAD ? lpad<PADSH>(l) : l) * ls;
      for (int s = s0; s < se; ++s)
        team_stage_any<EPT, INV, LINEPAD ? 0 : PADSH>(line, tw, p.st[s], p.L, tl, es);
    }
  }
}

// Last forward stage, a pointwise real multiplier on the spectrum, and the
// first stage of the inverse plan (the forward radices reversed), fused in
// registers: forward butterfly j of the last stage produces elements
// j + r N/R, exactly the inputs of inverse butterfly j of the first stage.
// The multiplier of spectral element e of this line is
// theta / (theta + lambda (kq + ks[e])^order) * scale (or its derivative
// with respect to lambda).
struct SpectralMult {
  const float* ks;
  float kq, lambda, theta, scale;
  int order;
  int deriv;  // nonzero: d/dlambda of the multiplier, -theta K^n / (theta + lambda K^n)^2
  __device__ __forceinline__ float operator()(int e) const {
    const float k0 = kq + ks[e];
    float kn = k0;
    for (int i = 1; i < order; ++i) kn *= k0;
    const float rd = __builtin_amdgcn_rcpf(theta + lambda * kn);
    return deriv ? -theta * scale * kn * rd * rd : theta * scale * rd;
  }
  // The multipliers of elements j, j + ns, ..., j + (R-1) ns at once (the same
  // operations per element as operator()): all symbol reads are issued
  // together and the power is one uniform loop over the R elements.
  template <int R>
  __device__ __forceinline__ void fill(int j, int ns, float* m) const {
    float k0[R], kn[R];
#pragma unroll
    for (int r = 0; r < R; ++r) k0[r] = kq + ks[j + r * ns];
#pragma unroll
    for (int r = 0; r < R; ++r) kn[r] = k0[r];
    for (int i = 1; i < order; ++i) {
#pragma unroll
      for (int r = 0; r < R; ++r) kn[r] *= k0[r];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float rd = __builtin_amdgcn_rcpf(theta + lambda * kn[r]);
      m[r] = deriv ? -theta * scale * kn[r] * rd * rd : theta * scale * rd;
    }
  }
};

template <int R, int EPT, int PADSH>
__device__ __forceinline__ void team_fused(float2* line, const float2* tw, const FftStage& sf,
                                           const FftStage& si, int L, int tl, int es,
                                           SpectralMult mult) {
  constexpr int M = EPT / R;
  const int nm = sf.nb / L;
  float2 v[M * R];
#pragma unroll
  for (int m = 0; m < M; ++m)
    if (m < nm) team_load<R, PADSH>(line, es, sf, tl + m * L, v + m * R);
  wave_lds_fence();
#pragma unroll
  for (int m = 0; m < M; ++m)
    if (m < nm) {
      const int j = tl + m * L;
      float2* w = v + m * R;
      team_compute<R, false>(tw, sf, j, w);
      float mr[R];
      mult.template fill<R>(j, sf.Ns, mr);
#pragma unroll
      for (int r = 0; r < R; ++r) w[r] = cscale(w[r], mr[r]);
      Dft<R, true>::run(w);  // first inverse stage: all twiddles are 1
      team_store<R, PADSH>(line, es, si, j, w);
    }
  wave_lds_fence();
}

template <int EPT, int PADSH>
__device__ __forceinline__ void team_fused_any(float2* line, const float2* tw, const FftStage& sf,
                                               const FftStage& si, int L, int tl, int es,
                                               SpectralMult mult) {
  switch (sf.R) {
    case 16: team_fused<16, EPT, PADSH>(line, tw, sf, si, L, tl, es, mult); break;
    case 12: team_fused<12, EPT, PADSH>(line, tw, sf, si, L, tl, es, mult); break;
    case 8: team_fused<8, EPT, PADSH>(line, tw, sf, si, L, tl, es, mult); break;
    case 6: team_fused<6, EPT, PADSH>(line, tw, sf, si, L, tl, es, mult); break;
    case 4: team_fused<4, EPT, PADSH>(line, tw, sf, si, L, tl, es, mult); break;
    case 3: team_fused<3, EPT, PADSH>(line, tw, sf, si, L, tl, es, mult); break;
    default: team_fused<2, EPT, PADSH>(line, tw, sf, si, L, tl, es, mult); break;
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
