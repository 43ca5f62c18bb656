// gfx950 kernels of the differentiated warping: the gradient of
// L = sum (I1(x + w(x)) - I0(x))^2 with respect to I1 and lambda, w the
// velocity of one warping from u = 0 (Sec. 2) computed by the two-field
// Nesterov-ADMM iteration (Sec. 3, Eq. (5), (6)) -- reverse mode, each
// step's adjoint written out:
//   forward step k:  t = s^{k-1} + gamma (s^{k-1} - s^{k-2}),  y = S t,
//                    a = 2y - t,  v = D(a; J, r),  s^k = v + t - y
//   adjoint, given g = dL/ds^k:
//                    (ga, gJ, gr) = D^T(g)  at a,
//                    gy = 2 ga - g,  gt = g - ga + S gy,
//                    dL/dlambda += <gy, (dS/dlambda) t>,
//                    dL/ds^{k-1} += (1 + gamma) gt,  dL/ds^{k-2} -= gamma gt.
// S is self-adjoint (a real even Fourier multiplier).  D^T for s = 2 with
// q = theta + |J|^2, f = (J.a + r) / q, c = J.g / q:
//   ga = g - c J,  gr = -c,  gJ = -f g - c (a - 2 f J).
#include "kernels.h"
#include "pointwise.h"

namespace nadmm {

namespace {

__device__ __forceinline__ void load3(const float* p, int V, int i, float v[3]) {
  v[0] = p[i];
  v[1] = p[V + i];
  v[2] = p[2 * V + i];
}
__device__ __forceinline__ void store3(float* p, int V, int i, const float v[3]) {
  p[i] = v[0];
  p[V + i] = v[1];
  p[2 * V + i] = v[2];
}

}  // namespace

// The adjoint of one step at a = 2y - t (t from s1, s2, gamma), or of the
// initial data step at a = 0 when y is null.  Writes gy = 2 ga - g and
// gt = g - ga (when the outputs are non-null) and accumulates gJ, gr.
__global__ void k_adj_step(Geo g, const float* __restrict__ gs, const float* __restrict__ s1,
                           const float* __restrict__ s2, float gamma, const float* __restrict__ y,
                           const float* __restrict__ J, const float* __restrict__ r, float theta,
                           float* __restrict__ gy, float* __restrict__ gt, float* __restrict__ gJ,
                           float* __restrict__ gr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  float gv[3], j[3], a[3] = {0.f, 0.f, 0.f};
  load3(gs, g.V, i, gv);
  load3(J, g.V, i, j);
  if (y) {
    float t[3], yy[3];
    load3(y, g.V, i, yy);
    load3(s1, g.V, i, t);
    if (s2) {
      float p[3];
      load3(s2, g.V, i, p);
      for (int c = 0; c < 3; ++c) t[c] = fmaf(gamma, t[c] - p[c], t[c]);
    }
    for (int c = 0; c < 3; ++c) a[c] = 2.0f * yy[c] - t[c];
  }
  const float q = theta + (j[0] * j[0] + j[1] * j[1] + j[2] * j[2]);
  const float f = (j[0] * a[0] + j[1] * a[1] + j[2] * a[2] + r[i]) / q;
  const float cj = (j[0] * gv[0] + j[1] * gv[1] + j[2] * gv[2]) / q;
  float ga[3], dj[3];
  for (int c = 0; c < 3; ++c) {
    ga[c] = gv[c] - cj * j[c];
    dj[c] = -f * gv[c] - cj * (a[c] - 2.0f * f * j[c]);
  }
  if (gy) {
    float o[3];
    for (int c = 0; c < 3; ++c) o[c] = 2.0f * ga[c] - gv[c];
    store3(gy, g.V, i, o);
  }
  if (gt) {
    float o[3];
    for (int c = 0; c < 3; ++c) o[c] = gv[c] - ga[c];
    store3(gt, g.V, i, o);
  }
  for (int c = 0; c < 3; ++c) gJ[c * g.V + i] += dj[c];
  gr[i] -= cj;
}

// The final warp and its adjoint: resid = I1(x + w) - I0 (written), the
// image adjoint 2 resid scattered with the trilinear weights into d_img
// (vector-memory float atomics) and gw = 2 resid * d/dp I1(p) at p = x + w.
__global__ void k_warp_adjoint(Geo g, const float* __restrict__ img, const float* __restrict__ ref,
                               const float* __restrict__ w, float* __restrict__ resid,
                               float* __restrict__ d_img, float* __restrict__ gw) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  const int x = i % g.nx, y = (i / g.nx) % g.ny, z = i / (g.nx * g.ny);
  const Tap t = make_tap(x, y, z, w[i], w[g.V + i], w[2 * g.V + i], g);
  const float c000 = img[t.o000], c100 = img[t.o100], c010 = img[t.o010], c110 = img[t.o110];
  const float c001 = img[t.o001], c101 = img[t.o101], c011 = img[t.o011], c111 = img[t.o111];
  const float val = lerpf(lerpf(lerpf(c000, c100, t.tx), lerpf(c010, c110, t.tx), t.ty),
                          lerpf(lerpf(c001, c101, t.tx), lerpf(c011, c111, t.tx), t.ty), t.tz);
  const float res = val - ref[i];
  resid[i] = res;
  const float gr = 2.0f * res;
  const float ux = 1.0f - t.tx, uy = 1.0f - t.ty, uz = 1.0f - t.tz;
  atomicAdd(d_img + t.o000, gr * ux * uy * uz);
  atomicAdd(d_img + t.o100, gr * t.tx * uy * uz);
  atomicAdd(d_img + t.o010, gr * ux * t.ty * uz);
  atomicAdd(d_img + t.o110, gr * t.tx * t.ty * uz);
  atomicAdd(d_img + t.o001, gr * ux * uy * t.tz);
  atomicAdd(d_img + t.o101, gr * t.tx * uy * t.tz);
  atomicAdd(d_img + t.o011, gr * ux * t.ty * t.tz);
  atomicAdd(d_img + t.o111, gr * t.tx * t.ty * t.tz);
  gw[i] = gr * (uy * uz * (c100 - c000) + t.ty * uz * (c110 - c010) + uy * t.tz * (c101 - c001) +
                t.ty * t.tz * (c111 - c011));
  gw[g.V + i] = gr * (ux * uz * (c010 - c000) + t.tx * uz * (c110 - c100) +
                      ux * t.tz * (c011 - c001) + t.tx * t.tz * (c111 - c101));
  gw[2 * g.V + i] = gr * (ux * uy * (c001 - c000) + t.tx * uy * (c101 - c100) +
                          ux * t.ty * (c011 - c010) + t.tx * t.ty * (c111 - c110));
}

// d_img += gr - sum_c D_c gJ_c: the transposes of r = I1 - I0 and of the
// periodic central differences J = grad I1 (D^T = -D).
__global__ void k_grad_transpose(Geo g, const float* __restrict__ gJ, const float* __restrict__ gr,
                                 float* __restrict__ d_img) {
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
  const float* gx = gJ;
  const float* gyy = gJ + g.V;
  const float* gz = gJ + 2 * g.V;
  const float dt = (gx[xp] - gx[xm] + gyy[yp] - gyy[ym] + gz[zp] - gz[zm]) * 0.5f;
  d_img[i] += gr[i] - dt;
}

// Deterministic dot product in float64: fixed-size partials, then one
// workgroup sums them in a fixed order and adds to (or sets) *out.
constexpr int kDotBlocks = 512;

__global__ void k_dot_partial(size_t n, const float* __restrict__ a, const float* __restrict__ b,
                              double* __restrict__ partial) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    acc += (double)a[i] * (double)b[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void k_dot_final(const double* __restrict__ partial, int nparts, double scale,
                            int accumulate, double* __restrict__ out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += partial[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = (accumulate ? *out : 0.0) + scale * sh[0];
}

static dim3 grid1(size_t n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_adj_step(const Geo& g, const float* gs, const float* s1, const float* s2,
                           float gamma, const float* y, const float* J, const float* r,
                           float theta, float* gy, float* gt, float* gJ, float* gr,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_adj_step, grid1(g.V), dim3(256), 0, st, g, gs, s1, s2, gamma, y, J, r,
                     theta, gy, gt, gJ, gr);
  return hipGetLastError();
}

hipError_t launch_warp_adjoint(const Geo& g, const float* img, const float* ref, const float* w,
                               float* resid, float* d_img, float* gw, hipStream_t st) {
  hipLaunchKernelGGL(k_warp_adjoint, grid1(g.V), dim3(256), 0, st, g, img, ref, w, resid, d_img,
                     gw);
  return hipGetLastError();
}

hipError_t launch_grad_transpose(const Geo& g, const float* gJ, const float* gr, float* d_img,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_grad_transpose, grid1(g.V), dim3(256), 0, st, g, gJ, gr, d_img);
  return hipGetLastError();
}

size_t dot_partials() { return kDotBlocks; }

hipError_t launch_dot_final(const double* partial, int nparts, double scale, bool accumulate, double* out,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, st, partial, nparts, scale, accumulate ? 1 : 0, out);
  return hipGetLastError();
}

hipError_t launch_dot(size_t n, const float* a, const float* b, double scale, bool accumulate,
                      double* partial, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks), dim3(256), 0, st, n, a, b, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, st, partial, kDotBlocks, scale,
                     accumulate ? 1 : 0, out);
  return hipGetLastError();
}

}  // namespace nadmm
