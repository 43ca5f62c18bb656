// gfx950 kernels of the Nesterov-accelerated ADMM registration path.
//
// Notation follows the paper (Thorley et al.): I0 fixed, I1 moving, J the
// gradient of the warped source, r = I1^w - I0, theta the ADMM penalty,
// lambda and n the regulariser weight and order (Sec. 2 Eq. (2), Sec. 3
// Eq. (4)-(6)).
//
// The ADMM iteration is carried in a two-field form.  With S the Fourier
// w-step operator (w = S(v + b_hat), linear), every iterate satisfies
// w^k = S s^k and b^k = s^k - S s^k for s^k = v^k + b_hat^k, so the Nesterov
// extrapolation of Eq. (5) becomes t^{k+1} = s^k + gamma_k (s^k - s^{k-1}),
// w_hat^{k+1} = S t^{k+1}, b_hat^{k+1} = t^{k+1} - S t^{k+1}.  One iteration
// is then: y = S t (three passes below), a = w_hat - b_hat = 2y - t,
// v = data step(a), s^{k+1} = v + t - y.  Only s^k and s^{k-1} are stored.
//
// S itself is three memory passes per iteration:
//   pass A  per x-line: t, packed real FFT along x (two real rows as one
//           complex row), half spectrum with the DC and Nyquist bins of a
//           row packed into one complex value;
//   pass B  per y-z plane of one x frequency: FFT along y and z, multiply by
//           theta / (theta + lambda K^n) / V, inverse FFTs (for the packed
//           plane the two real spectra are separated through their
//           Hermitian symmetry);
//   pass C  per x-line: inverse x FFT, then the pointwise data step and the
//           next state (or the composition of the warping's velocity).
#include <float.h>

#include "kernels.h"

namespace nadmm {

// ---------------------------------------------------------------------------
// host-side geometry helpers
// ---------------------------------------------------------------------------
int xline_rows(int ny) {
  for (int yb = 16; yb >= 2; yb -= 2)
    if (ny % yb == 0) return yb;
  return 2;
}

static int round_up(int a, int b) { return (a + b - 1) / b * b; }

int xline_threads(const Geo& g) {
  const int elems = 3 * (xline_rows(g.ny) / 2) * g.nx;
  int t = round_up((elems + 7) / 8, 64);
  if (t > 1024) t = 1024;
  if (t < 64) t = 64;
  return t;
}

int plane_threads(const Geo& g) {
  const int elems = g.ny * g.nz;
  int t = round_up((elems + 7) / 8, 64);
  if (t > 1024) t = 1024;
  if (t < 64) t = 64;
  return t;
}

FftPlan make_plan(int n) {
  FftPlan p{};
  p.n = n;
  int m = n;
  const int radices[4] = {8, 4, 3, 2};
  for (int i = 0; i < 4; ++i) {
    while (m % radices[i] == 0 && m > 1 && p.nstages < 8) {
      p.radix[p.nstages++] = radices[i];
      m /= radices[i];
    }
  }
  if (m != 1) p.nstages = -1;
  return p;
}

// ---------------------------------------------------------------------------
// periodic trilinear sampling
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wrap_index(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// Grid voxel x plus displacement u, split exactly into the integer cell
// (taken modulo n) and the fraction: floor(x + u) = x + floor(u) and
// frac(x + u) = u - floor(u) since x is an integer.  Non-finite u gives a
// valid cell and a NaN fraction, never an out-of-range index.
__device__ __forceinline__ void cell(int x, float u, int n, int& i0, int& i1, float& t) {
  const float fu = floorf(u);
  t = u - fu;
  const float cl = fminf(fmaxf(fu, -1.0e9f), 1.0e9f);
  i0 = wrap_index(x + (int)cl, n);
  i1 = (i0 + 1 == n) ? 0 : i0 + 1;
}

__device__ __forceinline__ float lerpf(float a, float b, float t) { return fmaf(t, b - a, a); }

struct Tap {
  int o000, o100, o010, o110, o001, o101, o011, o111;
  float tx, ty, tz;
};

__device__ __forceinline__ Tap make_tap(int x, int y, int z, float ux, float uy, float uz,
                                        const Geo& g) {
  int x0, x1, y0, y1, z0, z1;
  Tap t;
  cell(x, ux, g.nx, x0, x1, t.tx);
  cell(y, uy, g.ny, y0, y1, t.ty);
  cell(z, uz, g.nz, z0, z1, t.tz);
  const int r00 = (z0 * g.ny + y0) * g.nx, r01 = (z0 * g.ny + y1) * g.nx;
  const int r10 = (z1 * g.ny + y0) * g.nx, r11 = (z1 * g.ny + y1) * g.nx;
  t.o000 = r00 + x0; t.o100 = r00 + x1;
  t.o010 = r01 + x0; t.o110 = r01 + x1;
  t.o001 = r10 + x0; t.o101 = r10 + x1;
  t.o011 = r11 + x0; t.o111 = r11 + x1;
  return t;
}

__device__ __forceinline__ float sample(const float* __restrict__ f, const Tap& t) {
  const float c00 = lerpf(f[t.o000], f[t.o100], t.tx);
  const float c10 = lerpf(f[t.o010], f[t.o110], t.tx);
  const float c01 = lerpf(f[t.o001], f[t.o101], t.tx);
  const float c11 = lerpf(f[t.o011], f[t.o111], t.tx);
  return lerpf(lerpf(c00, c10, t.ty), lerpf(c01, c11, t.ty), t.tz);
}

// ---------------------------------------------------------------------------
// pointwise data steps of Eq. (6) for a = w_hat - b_hat
// ---------------------------------------------------------------------------
// s = 2: v = a - J (J.a + r) / (theta + |J|^2)  (Sherman-Morrison)
// s = 1: v = a - clip(z) J / theta,  z = theta (J.a + r) / (|J|^2 + eps)
__device__ __forceinline__ void data_step(const float a[3], const float j[3], float r, float theta,
                                          float eps, int data_term, float v[3]) {
  const float ja = j[0] * a[0] + j[1] * a[1] + j[2] * a[2];
  const float jj = j[0] * j[0] + j[1] * j[1] + j[2] * j[2];
  float f;
  if (data_term == 2) {
    f = (ja + r) / (theta + jj);
  } else {
    const float z = theta * (ja + r) / (jj + eps);
    f = (z / fmaxf(fabsf(z), 1.0f)) / theta;
  }
  v[0] = a[0] - j[0] * f;
  v[1] = a[1] - j[1] * f;
  v[2] = a[2] - j[2] * f;
}

// ---------------------------------------------------------------------------
// elementwise kernels
// ---------------------------------------------------------------------------
__global__ void k_fill(float* __restrict__ p, float value, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = value;
}

__global__ void k_scale(const float* __restrict__ in, float* __restrict__ out, float s, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = in[i] * s;
}

static int grid_for(size_t n, int threads) {
  size_t b = (n + threads - 1) / threads;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_fill(float* p, float value, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256)), dim3(256), 0, st, p, value, n);
  return hipGetLastError();
}

hipError_t launch_scale(const float* in, float* out, float s, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_scale, dim3(grid_for(n, 256)), dim3(256), 0, st, in, out, s, n);
  return hipGetLastError();
}

// out(x) = img(x + disp(x))
__global__ void k_warp(Geo g, const float* __restrict__ img, const float* __restrict__ disp,
                       float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  const int x = i % g.nx, y = (i / g.nx) % g.ny, z = i / (g.nx * g.ny);
  const Tap t = make_tap(x, y, z, disp[i], disp[g.V + i], disp[2 * g.V + i], g);
  out[i] = sample(img, t);
}

hipError_t launch_warp(const Geo& g, const float* img, const float* disp, float* out,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_warp, dim3((g.V + 255) / 256), dim3(256), 0, st, g, img, disp, out);
  return hipGetLastError();
}

// J = central differences of iw (periodic), r = iw - ref, s0 = data step from a = 0.
__global__ void k_grad_resid(Geo g, const float* __restrict__ iw, const float* __restrict__ ref,
                             float* __restrict__ grad, float* __restrict__ resid,
                             float* __restrict__ s0, float theta, float eps, int data_term) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  const int x = i % g.nx, y = (i / g.nx) % g.ny, z = i / (g.nx * g.ny);
  const int sy = g.nx, sz = g.nx * g.ny;
  const int xp = (x + 1 == g.nx) ? i - x : i + 1;
  const int xm = (x == 0) ? i + g.nx - 1 : i - 1;
  const int yp = (y + 1 == g.ny) ? i - y * sy : i + sy;
  const int ym = (y == 0) ? i + (g.ny - 1) * sy : i - sy;
  const int zp = (z + 1 == g.nz) ? i - z * sz : i + sz;
  const int zm = (z == 0) ? i + (g.nz - 1) * sz : i - sz;
  float j[3];
  j[0] = (iw[xp] - iw[xm]) * 0.5f;
  j[1] = (iw[yp] - iw[ym]) * 0.5f;
  j[2] = (iw[zp] - iw[zm]) * 0.5f;
  if (grad) {
    grad[i] = j[0];
    grad[g.V + i] = j[1];
    grad[2 * g.V + i] = j[2];
  }
  if (ref) {
    const float r = iw[i] - ref[i];
    if (resid) resid[i] = r;
    if (s0) {
      const float a[3] = {0.f, 0.f, 0.f};
      float v[3];
      data_step(a, j, r, theta, eps, data_term, v);
      s0[i] = v[0];
      s0[g.V + i] = v[1];
      s0[2 * g.V + i] = v[2];
    }
  }
}

hipError_t launch_grad_resid(const Geo& g, const float* iw, const float* ref, float* grad,
                             float* resid, float* s0, float theta, float eps, int data_term,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_grad_resid, dim3((g.V + 255) / 256), dim3(256), 0, st, g, iw, ref, grad,
                     resid, s0, theta, eps, data_term);
  return hipGetLastError();
}

// s^0 (and optionally v^0) from given J, r: the data step from a = 0.
__global__ void k_admm_init(Geo g, const float* __restrict__ J, const float* __restrict__ r,
                            float* __restrict__ s0, float* __restrict__ v_out, float theta,
                            float eps, int data_term) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  const float j[3] = {J[i], J[g.V + i], J[2 * g.V + i]};
  const float a[3] = {0.f, 0.f, 0.f};
  float v[3];
  data_step(a, j, r[i], theta, eps, data_term, v);
  for (int c = 0; c < 3; ++c) {
    s0[c * g.V + i] = v[c];
    if (v_out) v_out[c * g.V + i] = v[c];
  }
}

hipError_t launch_admm_init(const Geo& g, const float* J, const float* r, float* s0, float* v_out,
                            float theta, float eps, int data_term, hipStream_t st) {
  hipLaunchKernelGGL(k_admm_init, dim3((g.V + 255) / 256), dim3(256), 0, st, g, J, r, s0, v_out,
                     theta, eps, data_term);
  return hipGetLastError();
}

// out(x) = v(x) + u(x + v(x))
__global__ void k_compose(Geo g, const float* __restrict__ u, const float* __restrict__ v,
                          float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  const int x = i % g.nx, y = (i / g.nx) % g.ny, z = i / (g.nx * g.ny);
  const float vx = v[i], vy = v[g.V + i], vz = v[2 * g.V + i];
  const Tap t = make_tap(x, y, z, vx, vy, vz, g);
  out[i] = vx + sample(u, t);
  out[g.V + i] = vy + sample(u + g.V, t);
  out[2 * g.V + i] = vz + sample(u + 2 * g.V, t);
}

hipError_t launch_compose(const Geo& g, const float* u, const float* v, float* out,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_compose, dim3((g.V + 255) / 256), dim3(256), 0, st, g, u, v, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// pass A: t -> packed x half spectrum
// X layout: X[((c * nx/2 + p) * nz + z) * ny + y], p < nx/2; p = 0 holds
// (DC, Nyquist) of the real row as one complex value.
// ---------------------------------------------------------------------------
__global__ void k_pass_a(Geo g, FftPlan px, int yb, const float* __restrict__ s1,
                         const float* __restrict__ s2, float gamma, float2* __restrict__ X) {
  extern __shared__ float2 lds[];
  const int nx = g.nx, nh = g.nx / 2;
  const int ls = nx + 1;           // padded line stride (complex)
  const int lines = 3 * (yb / 2);  // complex lines: (component, row pair)
  float2* tw = lds;
  float2* buf = lds + nx;
  const int y0 = blockIdx.x * yb, z = blockIdx.y;
  make_twiddles(tw, nx);

  // load t = s1 + gamma (s1 - s2) and pack rows 2q, 2q+1 as re/im
  float* bf = reinterpret_cast<float*>(buf);
  const int nvox = 3 * yb * nx;
  for (int idx = threadIdx.x; idx < nvox; idx += blockDim.x) {
    const int c = idx / (yb * nx);
    const int rem = idx - c * yb * nx;
    const int yy = rem / nx, x = rem - yy * nx;
    const int gi = c * g.V + (z * g.ny + y0 + yy) * nx + x;
    float t = s1[gi];
    if (s2) t = fmaf(gamma, t - s2[gi], t);
    const int line = c * (yb / 2) + (yy >> 1);
    bf[2 * (line * ls + x) + (yy & 1)] = t;
  }
  __syncthreads();
  fft_lines<kEpt, false, true>(buf, tw, px, lines, 1, ls);

  // split into the two rows' half spectra and store (row pairs contiguous)
  const int nout = 3 * nh * (yb / 2);
  for (int idx = threadIdx.x; idx < nout; idx += blockDim.x) {
    const int yp = idx % (yb / 2);
    const int ck = idx / (yb / 2);
    const int c = ck / nh, k = ck - c * nh;
    const float2* Z = buf + (c * (yb / 2) + yp) * ls;
    float4 o;
    if (k == 0) {
      const float2 z0 = Z[0], zn = Z[nh];
      o = make_float4(z0.x, zn.x, z0.y, zn.y);
    } else {
      const float2 zk = Z[k], zm = Z[nx - k];
      // a = (Zk + conj(Zm)) / 2 ; b = -i (Zk - conj(Zm)) / 2
      o = make_float4(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y), 0.5f * (zk.y + zm.y),
                      -0.5f * (zk.x - zm.x));
    }
    float2* dst = X + ((size_t)(c * nh + k) * g.nz + z) * g.ny + y0 + 2 * yp;
    *reinterpret_cast<float4*>(dst) = o;
  }
}

static size_t pass_a_lds(const Geo& g) {
  const int yb = xline_rows(g.ny);
  return sizeof(float2) * ((size_t)g.nx + (size_t)3 * (yb / 2) * (g.nx + 1));
}

hipError_t launch_pass_a(const Geo& g, const FftPlan& px, const float* s1, const float* s2,
                         float gamma, float2* X, hipStream_t st) {
  const int yb = xline_rows(g.ny);
  hipLaunchKernelGGL(k_pass_a, dim3(g.ny / yb, g.nz), dim3(xline_threads(g)), pass_a_lds(g), st,
                     g, px, yb, s1, s2, gamma, X);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// pass B: y-z plane FFT, spectral multiply, inverse
// ---------------------------------------------------------------------------
__device__ __forceinline__ float spectral_mult(float k0, float lambda, float theta, int order,
                                               float inv_v) {
  float kn = k0;
  for (int i = 1; i < order; ++i) kn *= k0;
  return theta / (theta + lambda * kn) * inv_v;
}

__global__ void k_pass_b(Geo g, FftPlan py, FftPlan pz, float2* __restrict__ X, float lambda,
                         float theta, int order) {
  extern __shared__ float2 lds[];
  const int ny = g.ny, nz = g.nz, nh = g.nx / 2;
  const int rs = ny + 1;  // padded row stride of the [z][y] plane
  float2* twy = lds;
  float2* twz = twy + ny;
  float* sy = reinterpret_cast<float*>(twz + nz);
  float* sz = sy + ny;
  float2* buf = reinterpret_cast<float2*>(sz + nz + ((ny + nz) & 1));  // keep 8-byte alignment
  const int p = blockIdx.x, c = blockIdx.y;
  float2* plane = X + (size_t)(c * nh + p) * nz * ny;

  make_twiddles(twy, ny);
  make_twiddles(twz, nz);
  // symbol pieces 2 - 2 cos(2 pi q / n) = 4 sin^2(pi q / n), float64 then rounded
  for (int i = threadIdx.x; i < ny + nz; i += blockDim.x) {
    if (i < ny) {
      const double s = sinpi((double)i / ny);
      sy[i] = (float)(4.0 * s * s);
    } else {
      const double s = sinpi((double)(i - ny) / nz);
      sz[i - ny] = (float)(4.0 * s * s);
    }
  }
  const int n = ny * nz;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int zz = i / ny, yy = i - zz * ny;
    buf[zz * rs + yy] = plane[i];
  }
  __syncthreads();
  fft_lines<kEpt, false, true>(buf, twy, py, nz, 1, rs);  // along y
  fft_lines<kEpt, false, true>(buf, twz, pz, ny, rs, 1);  // along z

  const float inv_v = 1.0f / (float)g.V;
  if (p > 0) {
    const double sxd = sinpi((double)p / g.nx);
    const float sx = (float)(4.0 * sxd * sxd);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const int zz = i / ny, yy = i - zz * ny;
      const float m = spectral_mult(sx + sy[yy] + sz[zz], lambda, theta, order, inv_v);
      float2& e = buf[zz * rs + yy];
      e = cscale(e, m);
    }
    __syncthreads();
  } else {
    // Packed plane P = Z0 + i Zn of two real signals (x DC and x Nyquist rows):
    // result m0 Z0 + i mn Zn = (m0 + mn)/2 P + (m0 - mn)/2 conj(P(-q, -r)).
    float2 res[kEpt];
#pragma unroll
    for (int it = 0; it < kEpt; ++it) {
      const int i = threadIdx.x + it * blockDim.x;
      if (i < n) {
        const int zz = i / ny, yy = i - zz * ny;
        const int zr = (zz == 0) ? 0 : nz - zz, yr = (yy == 0) ? 0 : ny - yy;
        const float2 P = buf[zz * rs + yy];
        const float2 Pt = cconj(buf[zr * rs + yr]);
        const float m0 = spectral_mult(sy[yy] + sz[zz], lambda, theta, order, inv_v);
        const float mn = spectral_mult(4.0f + sy[yy] + sz[zz], lambda, theta, order, inv_v);
        const float A = 0.5f * (m0 + mn), B = 0.5f * (m0 - mn);
        res[it] = make_float2(A * P.x + B * Pt.x, A * P.y + B * Pt.y);
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kEpt; ++it) {
      const int i = threadIdx.x + it * blockDim.x;
      if (i < n) {
        const int zz = i / ny, yy = i - zz * ny;
        buf[zz * rs + yy] = res[it];
      }
    }
    __syncthreads();
  }
  fft_lines<kEpt, true, true>(buf, twz, pz, ny, rs, 1);
  fft_lines<kEpt, true, true>(buf, twy, py, nz, 1, rs);
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int zz = i / ny, yy = i - zz * ny;
    plane[i] = buf[zz * rs + yy];
  }
}

static size_t pass_b_lds(const Geo& g) {
  return sizeof(float2) * (size_t)(g.ny + g.nz) + sizeof(float) * (size_t)(g.ny + g.nz + 1) +
         sizeof(float2) * (size_t)g.nz * (g.ny + 1);
}

hipError_t launch_pass_b(const Geo& g, const FftPlan& py, const FftPlan& pz, float2* X,
                         float lambda, float theta, int order, hipStream_t st) {
  hipLaunchKernelGGL(k_pass_b, dim3(g.nx / 2, 3), dim3(plane_threads(g)), pass_b_lds(g), st, g,
                     py, pz, X, lambda, theta, order);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// pass C: packed half spectrum -> y = S t, then the mode's pointwise work
// ---------------------------------------------------------------------------
template <int MODE>
__global__ void k_pass_c(Geo g, FftPlan px, int yb, PassCArgs a) {
  extern __shared__ float2 lds[];
  const int nx = g.nx, nh = g.nx / 2;
  const int ls = nx + 1;
  const int lines = 3 * (yb / 2);
  float2* tw = lds;
  float2* buf = lds + nx;
  const int y0 = blockIdx.x * yb, z = blockIdx.y;
  make_twiddles(tw, nx);

  // unpack two rows' half spectra into one complex row: Z = Xa + i Xb
  const int nin = 3 * nh * (yb / 2);
  for (int idx = threadIdx.x; idx < nin; idx += blockDim.x) {
    const int yp = idx % (yb / 2);
    const int ck = idx / (yb / 2);
    const int c = ck / nh, k = ck - c * nh;
    const float4 in = *reinterpret_cast<const float4*>(
        a.X + ((size_t)(c * nh + k) * g.nz + z) * g.ny + y0 + 2 * yp);
    float2* Z = buf + (c * (yb / 2) + yp) * ls;
    // in = (a.re, a.im, b.re, b.im)
    if (k == 0) {
      Z[0] = make_float2(in.x, in.z);
      Z[nh] = make_float2(in.y, in.w);
    } else {
      Z[k] = make_float2(in.x - in.w, in.y + in.z);
      Z[nx - k] = make_float2(in.x + in.w, in.z - in.y);
    }
  }
  __syncthreads();
  fft_lines<kEpt, true, true>(buf, tw, px, lines, 1, ls);

  const float* bf = reinterpret_cast<const float*>(buf);
  const int nvox = yb * nx;
  for (int idx = threadIdx.x; idx < nvox; idx += blockDim.x) {
    const int yy = idx / nx, x = idx - yy * nx;
    const int i = (z * g.ny + y0 + yy) * nx + x;
    float yv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) yv[c] = bf[2 * ((c * (yb / 2) + (yy >> 1)) * ls + x) + (yy & 1)];

    if (MODE == kOutY) {
#pragma unroll
      for (int c = 0; c < 3; ++c) a.out[c * g.V + i] = yv[c];
    } else if (MODE == kIter) {
      float t[3], av[3], j[3], v[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float s = a.s1[c * g.V + i];
        if (a.s2) s = fmaf(a.gamma, s - a.s2[c * g.V + i], s);
        t[c] = s;
        av[c] = 2.0f * yv[c] - s;
        j[c] = a.J[c * g.V + i];
      }
      data_step(av, j, a.r[i], a.theta, a.eps, a.data_term, v);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        // s^k = v + b_hat = v + t - y
        a.out[c * g.V + i] = v[c] + (t[c] - yv[c]);
        if (a.v_out) a.v_out[c * g.V + i] = v[c];
      }
    } else if (MODE == kFinalWB) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        a.out[c * g.V + i] = yv[c];
        if (a.b_out) a.b_out[c * g.V + i] = a.s1[c * g.V + i] - yv[c];
      }
    } else {  // kCompose: u_new = w + u_old(x + w), optional warped image
      const int x0 = x, yg = y0 + yy;
      const Tap t = make_tap(x0, yg, z, yv[0], yv[1], yv[2], g);
      float un[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        un[c] = yv[c] + sample(a.u_old + c * g.V, t);
        a.out[c * g.V + i] = un[c];
        if (a.vel_out) a.vel_out[c * g.V + i] = yv[c];
      }
      if (a.iw_out) {
        const Tap t2 = make_tap(x0, yg, z, un[0], un[1], un[2], g);
        a.iw_out[i] = sample(a.img, t2);
      }
    }
  }
}

hipError_t launch_pass_c(const Geo& g, const FftPlan& px, PassCMode mode, const PassCArgs& a,
                         hipStream_t st) {
  const int yb = xline_rows(g.ny);
  const dim3 grid(g.ny / yb, g.nz), block(xline_threads(g));
  const size_t lds = pass_a_lds(g);
  switch (mode) {
    case kOutY: hipLaunchKernelGGL(k_pass_c<kOutY>, grid, block, lds, st, g, px, yb, a); break;
    case kIter: hipLaunchKernelGGL(k_pass_c<kIter>, grid, block, lds, st, g, px, yb, a); break;
    case kFinalWB: hipLaunchKernelGGL(k_pass_c<kFinalWB>, grid, block, lds, st, g, px, yb, a); break;
    default: hipLaunchKernelGGL(k_pass_c<kCompose>, grid, block, lds, st, g, px, yb, a); break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Jacobian determinant of Id + u, float64 evaluation and fixed-order reduction
// ---------------------------------------------------------------------------
struct JacAcc {
  double mn, mx, sum, cnt;
};

__device__ __forceinline__ void jac_merge(JacAcc& a, const JacAcc& b) {
  a.mn = fmin(a.mn, b.mn);
  a.mx = fmax(a.mx, b.mx);
  a.sum += b.sum;
  a.cnt += b.cnt;
}

__device__ void jac_block_reduce(JacAcc v, JacAcc* sh, JacAcc* out) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) jac_merge(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

__global__ void k_jac_partial(Geo g, const float* __restrict__ u, float* __restrict__ det,
                              JacAcc* __restrict__ partial) {
  __shared__ JacAcc sh[256];
  JacAcc acc{DBL_MAX, -DBL_MAX, 0.0, 0.0};
  const int sy = g.nx, sz = g.nx * g.ny;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.V; i += gridDim.x * blockDim.x) {
    const int x = i % g.nx, y = (i / g.nx) % g.ny, z = i / (g.nx * g.ny);
    const int xp = (x + 1 == g.nx) ? i - x : i + 1;
    const int xm = (x == 0) ? i + g.nx - 1 : i - 1;
    const int yp = (y + 1 == g.ny) ? i - y * sy : i + sy;
    const int ym = (y == 0) ? i + (g.ny - 1) * sy : i - sy;
    const int zp = (z + 1 == g.nz) ? i - z * sz : i + sz;
    const int zm = (z == 0) ? i + (g.nz - 1) * sz : i - sz;
    double A[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float* uc = u + c * g.V;
      A[c][0] = 0.5 * ((double)uc[xp] - (double)uc[xm]) + (c == 0 ? 1.0 : 0.0);
      A[c][1] = 0.5 * ((double)uc[yp] - (double)uc[ym]) + (c == 1 ? 1.0 : 0.0);
      A[c][2] = 0.5 * ((double)uc[zp] - (double)uc[zm]) + (c == 2 ? 1.0 : 0.0);
    }
    const double d = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                     A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                     A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    if (det) det[i] = (float)d;
    acc.mn = fmin(acc.mn, d);
    acc.mx = fmax(acc.mx, d);
    acc.sum += d;
    acc.cnt += (d <= 0.0) ? 1.0 : 0.0;
  }
  jac_block_reduce(acc, sh, partial + blockIdx.x);
}

__global__ void k_jac_final(int nparts, int V, const JacAcc* __restrict__ partial,
                            double* __restrict__ stats, int64_t* __restrict__ n_nonpos) {
  __shared__ JacAcc sh[256];
  JacAcc acc{DBL_MAX, -DBL_MAX, 0.0, 0.0};
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) jac_merge(acc, partial[i]);
  __shared__ JacAcc tot;
  jac_block_reduce(acc, sh, &tot);
  __syncthreads();
  if (threadIdx.x == 0) {
    stats[0] = tot.mn;
    stats[1] = tot.mx;
    stats[2] = tot.sum / (double)V;
    n_nonpos[0] = (int64_t)tot.cnt;
  }
}

hipError_t launch_jacobian(const Geo& g, const float* disp, float* det, double* partial,
                           double* stats, int64_t* n_nonpos, hipStream_t st) {
  int nb = (g.V + 255) / 256;
  if (nb > kJacBlocks) nb = kJacBlocks;
  JacAcc* part = reinterpret_cast<JacAcc*>(partial);
  hipLaunchKernelGGL(k_jac_partial, dim3(nb), dim3(256), 0, st, g, disp, det, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_jac_final, dim3(1), dim3(256), 0, st, nb, g.V, part, stats, n_nonpos);
  return hipGetLastError();
}

}  // namespace nadmm
