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
// S itself is three memory passes:
//   pass A  per x-line: t, real FFT along x (two real rows as one complex
//           row), half spectrum of nx/2 + 1 bins scaled by 1 / nx; bins 0
//           and nx/2 (real) form planes of their own;
//   pass B  per y-z plane of one x frequency: FFT along y and z, multiply by
//           theta / (theta + lambda K^n) / (ny nz), inverse FFTs;
//   pass C  per x-line: inverse x FFT, then the pointwise data step and the
//           next state (or the composition of the warping's velocity).
// Inside the iteration loop pass C and the next pass A run as one kernel
// (mode kIterFwd): the new state is extrapolated and transformed along x on
// the same lines without leaving the chip.
#include <float.h>
#include <string.h>

#include <map>
#include <mutex>
#include <tuple>
#include <utility>
#include <type_traits>

#include "kernels.h"
#include "pointwise.h"

// Layout of the x-line buffers of passes A and C: butterflies of one line on
// consecutive threads and one padding slot every 2^kXlPadsh complex elements.
constexpr int kXlPadsh = 4;
static_assert(kXlPadsh >= 2, "float4 runs must not straddle a padding slot");
// Rows of one z-slice per workgroup of the x-line passes (largest even
// divisor of ny up to this; the autotuner may pick fewer).
constexpr int kXlMaxRows = 8;

namespace nadmm {

static inline int xl_pad_host(int e) { return kXlPadsh > 0 ? e + (e >> kXlPadsh) : e; }
// complex elements between consecutive x lines in LDS
static inline int xline_stride(int nx) { return xl_pad_host(nx); }

// ---------------------------------------------------------------------------
// host-side geometry helpers
// ---------------------------------------------------------------------------
// Rows per x-line workgroup: the tuned value for these sizes when one was
// set (xline_rows_set, from the autotuner), else the largest even divisor of
// ny up to kXlMaxRows and up to 1024 / nx (192 threads for the three
// components' 8-point shares; measured at nx = 192: 4 rows 52-54 us, 8 rows
// 63-69 us for the fused pass of a 192 x 192 x 128 volume).
static std::mutex g_rows_mu;
static std::map<std::tuple<int, int, int>, int> g_rows;

int xline_rows_default(const Geo& g) {
  if (ysplit(g)) {  // two groups of 8 rows (runs of 64 bytes), else of 4, else of 2
    // (measured at 192 x 192 x 128: 61.7-63.6 us for 16 rows, 63.9-66.7 for 8)
    for (int rows = 16; rows >= 4; rows /= 2)
      if ((g.ny / 2) % (rows / 2) == 0 && xline_rows_fit(g, rows, xline_threads_rows(g, rows))) return rows;
    return 4;
  }
  const int cap = 1024 / g.nx < kXlMaxRows ? 1024 / g.nx : kXlMaxRows;
  for (int yb = cap & ~1; yb >= 2; yb -= 2)
    if (g.ny % yb == 0) return yb;
  return 2;
}

int xline_rows(const Geo& g) {
  std::lock_guard<std::mutex> lk(g_rows_mu);
  auto it = g_rows.find(std::make_tuple(g.nx, g.ny, g.nz));
  return it != g_rows.end() ? it->second : xline_rows_default(g);
}

int xline_rows_tuned(const Geo& g) {
  std::lock_guard<std::mutex> lk(g_rows_mu);
  auto it = g_rows.find(std::make_tuple(g.nx, g.ny, g.nz));
  return it != g_rows.end() ? it->second : 0;
}

void xline_rows_set(const Geo& g, int rows) {
  std::lock_guard<std::mutex> lk(g_rows_mu);
  if (rows > 0)
    g_rows[std::make_tuple(g.nx, g.ny, g.nz)] = rows;
  else
    g_rows.erase(std::make_tuple(g.nx, g.ny, g.nz));
}

// The other tuned shapes, per sizes (0 or absent: the default): rows of the
// composition pass (else those of the other x-line passes) and wavefronts of
// a y-z plane workgroup (at least what the plane's team plans need).
static std::map<std::tuple<int, int, int>, int> g_rows_compose, g_plane_waves;

static int tuned(const std::map<std::tuple<int, int, int>, int>& t, const Geo& g) {
  std::lock_guard<std::mutex> lk(g_rows_mu);
  auto it = t.find(std::make_tuple(g.nx, g.ny, g.nz));
  return it != t.end() ? it->second : 0;
}
static void tune_set(std::map<std::tuple<int, int, int>, int>& t, const Geo& g, int v) {
  std::lock_guard<std::mutex> lk(g_rows_mu);
  if (v > 0)
    t[std::make_tuple(g.nx, g.ny, g.nz)] = v;
  else
    t.erase(std::make_tuple(g.nx, g.ny, g.nz));
}
int xline_rows_compose(const Geo& g) {
  const int r = tuned(g_rows_compose, g);
  return r > 0 ? r : xline_rows(g);
}
void xline_rows_compose_set(const Geo& g, int rows) { tune_set(g_rows_compose, g, rows); }
void plane_waves_set(const Geo& g, int waves) { tune_set(g_plane_waves, g, waves); }

static int round_up(int a, int b) { return (a + b - 1) / b * b; }

// dynamic LDS of pass B for row stride rs: twiddles, symbol tables, plane
size_t plane_lds_bytes(const Geo& g, int rs) {
  return sizeof(float2) * (size_t)(g.ny + g.nz) + sizeof(float) * (size_t)(g.ny + g.nz + 1) +
         sizeof(float2) * (size_t)g.nz * rs;
}

int xline_threads_rows(const Geo& g, int rows) {
  const int elems = 3 * (rows / 2) * g.nx;
  int t = round_up((elems + 7) / 8, 64);
  if (t > kXlMaxThreads) t = kXlMaxThreads;
  if (t < 64) t = 64;
  return t;
}
int xline_threads(const Geo& g) { return xline_threads_rows(g, xline_rows(g)); }

// The x-line bounds of launch_shape_ok for `rows` rows and `xt` threads.
// Half-plane sizes: a tile is two groups of rows / 2 rows, each a whole
// number of row pairs dividing ny / 2.
static bool ysplit_rows_ok(const Geo& g, int rows) {
  return !ysplit(g) || (rows % 4 == 0 && (g.ny / 2) % (rows / 2) == 0);
}

bool xline_rows_fit(const Geo& g, int rows, int xt) {
  return xt <= kXlMaxThreads && g.ny % rows == 0 && rows % 2 == 0 && ysplit_rows_ok(g, rows) &&
         3 * (rows / 2) * g.nx <= kEpt * xt &&
         3 * rows * (g.nx / 4) <= kXItems * xt && rows * (g.nx / 4) <= 2 * xt && 3 * rows * g.nx < 65536;
}

constexpr int kPlaneEptTarget = 8;  // points per thread the plane pass is sized for
int plane_threads(const Geo& g) {
  const int elems = g.ny * g.nz;
  int t = round_up((elems + kPlaneEptTarget - 1) / kPlaneEptTarget, 64);
  if (t > 1024) t = 1024;
  if (t < 64) t = 64;
  return t;
}

FftPlan make_plan(int n) {
  FftPlan p{};
  p.n = n;
  const StockhamRadices rad = stockham_radices_ce(n);
  p.nstages = rad.nstages;
  int ns = 1;
  for (int i = 0; i < p.nstages; ++i) {
    FftStage& s = p.st[i];
    s.R = rad.R[i];
    s.Ns = ns;
    s.nb = n / s.R;
    s.twstride = n / (ns * s.R);
    s.div_nb = make_fastdiv(s.nb);
    s.div_ns = make_fastdiv(ns);
    ns *= s.R;
  }
  return p;
}

// The host's plan searches are memoised (every y-z pass launch asks for its
// plans and row stride; the searches cost microseconds of host time).
TeamPlan make_team_plan(int n, int max_lanes) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, TeamPlan> memo;
  const auto key = std::make_pair(n, max_lanes);
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
  }
  const TeamPlan p = make_team_plan_ce(n, max_lanes);
  std::lock_guard<std::mutex> lk(mu);
  memo[key] = p;
  return p;
}
TeamPlan reverse_team_plan(const TeamPlan& p) { return reverse_team_plan_ce(p); }

// Row stride (complex) of the padded [z][y] plane of pass B: element (z, y)
// lives at z * rs + y + y / 16.  rs is chosen by simulating the first-stage
// LDS reads of both phases (y rows and z columns) of one wavefront, counting
// lanes of each group of 16 that share a bank pair (32 banks of 4 bytes,
// 16 lanes per cycle for 8-byte accesses), subject to fitting in LDS.
constexpr int ypad(int y) { return y + (y >> 4); }
constexpr int plane_conflicts(const TeamPlan& p, int nlines, int rs, bool rows) {
  const int nlw = 64 / p.L;
  int score = 0;
  for (int grp = 0; grp < 4; ++grp) {
    int count[16] = {0};
    for (int lane = 16 * grp; lane < 16 * grp + 16; ++lane) {
      const int li = lane % nlw, tl = lane / nlw;
      if (li >= nlines) continue;
      const int j = tl;  // first butterfly, element r = 0
      const int a = rows ? li * rs + ypad(j) : j * rs + ypad(li);
      ++count[a & 15];
    }
    int mx = 0;
    for (int b = 0; b < 16; ++b) mx = count[b] > mx ? count[b] : mx;
    score += mx;
  }
  return score;
}

// Evaluated at compile time by the fixed-size plane kernels (which then
// address LDS with constant offsets) and at run time by the host, so both
// sides agree on the stride.
constexpr int plane_row_stride_ce(int ny, int nz, const TeamPlan& py, const TeamPlan& pz) {
  const int base = ypad(ny - 1) + 1;
  int best = base, best_score = 1 << 30;
  for (int e = 0; e < 16; ++e) {
    const int rs = base + e;
    if (8 * (ny + nz) + 4 * (ny + nz + 1) + 8 * nz * rs > kMaxLds) break;
    const int sc = plane_conflicts(py, nz, rs, true) + plane_conflicts(pz, ny, rs, false);
    if (sc < best_score) {
      best_score = sc;
      best = rs;
    }
  }
  return best;
}

int plane_row_stride(const Geo& g) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, int> memo;
  const auto key = std::make_pair(g.ny, g.nz);
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
  }
  const int rs = plane_row_stride_ce(g.ny, g.nz, plane_plan_y(g), plane_plan_z(g));
  std::lock_guard<std::mutex> lk(mu);
  memo[key] = rs;
  return rs;
}

// Lane budget of one line in pass B: a 1024-thread workgroup shared by the
// lines of one axis.
static int lane_budget(int nlines) {
  const int b = 1024 / nlines;
  return b < 1 ? 1 : b;
}
TeamPlan plane_plan_y(const Geo& g) { return make_team_plan(g.ny, lane_budget(g.nz)); }
TeamPlan plane_plan_z(const Geo& g) { return make_team_plan(g.nz, lane_budget(g.ny)); }

int plane_waves_needed(const Geo& g) {
  const TeamPlan py = plane_plan_y(g), pz = plane_plan_z(g);
  const int wy = (g.nz + 64 / py.L - 1) / (64 / py.L);
  const int wz = (g.ny + 64 / pz.L - 1) / (64 / pz.L);
  int w = wy > wz ? wy : wz;
  if (w > 16) w = 16;
  if (w < 1) w = 1;
  return w;
}
// Threads of a y-z plane workgroup: the tuned wavefronts, never fewer than
// the team plans need (more only add wavefronts that share the work).
static int plane_team_threads(const Geo& g) {
  const int need = plane_waves_needed(g), t = tuned(g_plane_waves, g);
  return 64 * (t > need && t <= 16 ? t : need);
}
int plane_threads_tuned(const Geo& g) { return plane_team_threads(g); }

static bool split_shape_ok(const Geo& g);

bool launch_shape_ok(const Geo& g) {
  if (g.nx % 4 || g.ny % 2) return false;
  const int yb = xline_rows(g), xt = xline_threads(g), pt = plane_threads(g);
  const FftPlan px = make_plan(g.nx), py = make_plan(g.ny), pz = make_plan(g.nz);
  if (px.nstages < 1 || py.nstages < 1 || pz.nstages < 1) return false;
  const bool fft_a = 3 * (yb / 2) * g.nx <= kEpt * xt;       // x-line FFT elements per thread
  const bool load_a = 3 * yb * (g.nx / 4) <= kXItems * xt;    // pass A float4 loads
  const bool point_c = yb * (g.nx / 4) <= 2 * xt;             // pass C float4 runs
  (void)pt;
  const bool div_x = 3 * yb * g.nx < 65536;  // FastDiv range of the x-line index maps
  const bool bound_x = xt <= kXlMaxThreads;   // the x-line kernels' launch bound
  bool pass_b;
  if (plane_fits(g)) {
    const TeamPlan ty = plane_plan_y(g), tz = plane_plan_z(g);
    pass_b = ty.nstages > 0 && tz.nstages > 0 && g.ny * g.nz < 65536;  // team plans, FastDiv range
  } else {
    pass_b = ysplit(g) || split_shape_ok(g);
  }
  return fft_a && load_a && point_c && pass_b && div_x && bound_x && ysplit_rows_ok(g, yb);
}

static XDivs make_xdivs_rows(const Geo& g, int yb) {
  XDivs d;
  d.q4 = make_fastdiv(g.nx / 4);
  d.yb = make_fastdiv(yb);
  d.yb2 = make_fastdiv(yb / 2);
  d.nh = make_fastdiv(g.nx / 2);
  d.lines = make_fastdiv(3 * (yb / 2));
  d.ny = make_fastdiv(g.ny);
  d.nz = make_fastdiv(g.nz);
  const bool split = ysplit(g);
  d.ygrp = split ? yb / 2 : yb;
  d.yhalf = split ? g.ny / 2 : 0;
  d.yq = make_fastdiv(split ? yb / 4 : (yb / 2 > 0 ? yb / 2 : 1));
  return d;
}
XDivs make_xdivs(const Geo& g) { return make_xdivs_rows(g, xline_rows(g)); }

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

// Count of the entries of f that are NaN or infinite: per-wavefront sums
// added to *count (zeroed by the first kernel, so the pair needs no memset).
__global__ void k_zero_count(unsigned long long* count) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *count = 0ull;
}
__global__ void k_count_nonfinite(const float* __restrict__ f, size_t n,
                                  unsigned long long* __restrict__ count) {
  unsigned int c = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    c += isfinite(f[i]) ? 0u : 1u;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, (unsigned long long)c);
}
hipError_t launch_count_nonfinite(const float* f, size_t n, int64_t* count, hipStream_t st) {
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(count);
  hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(64), 0, st, cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  hipLaunchKernelGGL(k_count_nonfinite, dim3((unsigned)(blocks ? blocks : 1)), dim3(256), 0, st, f, n, cnt);
  return hipGetLastError();
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
template <typename T>
__global__ void k_warp(Geo g, const T* __restrict__ img, const float* __restrict__ disp,
                       float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  img = at_pair(img, g.V, blockIdx.y);
  disp = at_pair(disp, 3 * (size_t)g.V, blockIdx.y);
  out = at_pair(out, g.V, blockIdx.y);
  const int x = i % g.nx, y = (i / g.nx) % g.ny, z = i / (g.nx * g.ny);
  const Tap t = make_tap(x, y, z, disp[i], disp[g.V + i], disp[2 * g.V + i], g);
  store_wt(out + i, sample(img, t));
}

template <typename T>
static hipError_t warp_any(const Geo& g, const T* img, const float* disp, float* out,
                           hipStream_t st, int batch) {
  hipLaunchKernelGGL(k_warp<T>, dim3((g.V + 255) / 256, batch), dim3(256), 0, st, g, img, disp,
                     out);
  return hipGetLastError();
}
hipError_t launch_warp(const Geo& g, const float* img, const float* disp, float* out,
                       hipStream_t st, int batch) {
  return warp_any(g, img, disp, out, st, batch);
}
hipError_t launch_warp(const Geo& g, const uint16_t* img, const float* disp, float* out,
                       hipStream_t st, int batch) {
  return warp_any(g, img, disp, out, st, batch);
}

// J = central differences of iw (periodic), r = iw - ref, s0 = data step from a = 0.
template <typename T>
__global__ void k_grad_resid(Geo g, const float* __restrict__ iw, const T* __restrict__ ref,
                             float* __restrict__ grad, float* __restrict__ resid,
                             float* __restrict__ s0, float theta, float eps, int data_term) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  const int b = blockIdx.y;
  iw = at_pair(iw, g.V, b);
  ref = at_pair(ref, g.V, b);
  grad = at_pair(grad, 3 * (size_t)g.V, b);
  resid = at_pair(resid, g.V, b);
  s0 = at_pair(s0, 3 * (size_t)g.V, b);
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
    store_wt(grad + i, j[0]);
    store_wt(grad + g.V + i, j[1]);
    store_wt(grad + 2 * g.V + i, j[2]);
  }
  if (ref) {
    const float r = iw[i] - img_at(ref, i);
    if (resid) store_wt(resid + i, r);
    if (s0) {
      const float a[3] = {0.f, 0.f, 0.f};
      float v[3];
      data_step(a, j, r, theta, eps, data_term, v);
      store_wt(s0 + i, v[0]);
      store_wt(s0 + g.V + i, v[1]);
      store_wt(s0 + 2 * g.V + i, v[2]);
    }
  }
}

template <typename T>
static hipError_t grad_resid_any(const Geo& g, const float* iw, const T* ref, float* grad,
                                 float* resid, float* s0, float theta, float eps, int data_term,
                                 hipStream_t st, int batch) {
  hipLaunchKernelGGL(k_grad_resid<T>, dim3((g.V + 255) / 256, batch), dim3(256), 0, st, g, iw,
                     ref, grad, resid, s0, theta, eps, data_term);
  return hipGetLastError();
}
hipError_t launch_grad_resid(const Geo& g, const float* iw, const float* ref, float* grad,
                             float* resid, float* s0, float theta, float eps, int data_term,
                             hipStream_t st, int batch) {
  return grad_resid_any(g, iw, ref, grad, resid, s0, theta, eps, data_term, st, batch);
}
hipError_t launch_grad_resid(const Geo& g, const float* iw, const uint16_t* ref, float* grad,
                             float* resid, float* s0, float theta, float eps, int data_term,
                             hipStream_t st, int batch) {
  return grad_resid_any(g, iw, ref, grad, resid, s0, theta, eps, data_term, st, batch);
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
  store_wt(out + i, vx + sample(u, t));
  store_wt(out + g.V + i, vy + sample(u + g.V, t));
  store_wt(out + 2 * g.V + i, vz + sample(u + 2 * g.V, t));
}

hipError_t launch_compose(const Geo& g, const float* u, const float* v, float* out,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_compose, dim3((g.V + 255) / 256), dim3(256), 0, st, g, u, v, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// pyramid resampling (coarse voxel i covers fine voxels 2i and 2i + 1)
// ---------------------------------------------------------------------------
// coarse = 2x2x2 average of fine; gc is the coarse geometry
__global__ void k_downsample2(Geo gc, const float* __restrict__ fine, float* __restrict__ coarse) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= gc.V) return;
  const int x = i % gc.nx, y = (i / gc.nx) % gc.ny, z = i / (gc.nx * gc.ny);
  const int fx = 2 * gc.nx, fy = 2 * gc.ny;
  const float* p = fine + ((size_t)(2 * z) * fy + 2 * y) * fx + 2 * x;
  const size_t sy = fx, sz = (size_t)fx * fy;
  const float a = (p[0] + p[1]) + (p[sy] + p[sy + 1]);
  const float b = (p[sz] + p[sz + 1]) + (p[sz + sy] + p[sz + sy + 1]);
  coarse[i] = (a + b) * 0.125f;
}

// uf(x) = 2 uc((x - 1/2) / 2), periodic trilinear; gf is the fine geometry
__global__ void k_upsample2_disp(Geo gf, const float* __restrict__ uc, float* __restrict__ uf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= gf.V) return;
  const int x = i % gf.nx, y = (i / gf.nx) % gf.ny, z = i / (gf.nx * gf.ny);
  const Geo gc{gf.nx / 2, gf.ny / 2, gf.nz / 2, gf.V / 8};
  auto axis = [](int xf, int nc, int& i0, int& i1, float& t) {
    const float p = ((float)xf - 0.5f) * 0.5f;
    const float f = floorf(p);
    t = p - f;
    i0 = (int)f;
    if (i0 < 0) i0 += nc;
    i1 = (i0 + 1 == nc) ? 0 : i0 + 1;
  };
  int x0, x1, y0, y1, z0, z1;
  Tap t;
  axis(x, gc.nx, x0, x1, t.tx);
  axis(y, gc.ny, y0, y1, t.ty);
  axis(z, gc.nz, z0, z1, t.tz);
  const int r00 = (z0 * gc.ny + y0) * gc.nx, r01 = (z0 * gc.ny + y1) * gc.nx;
  const int r10 = (z1 * gc.ny + y0) * gc.nx, r11 = (z1 * gc.ny + y1) * gc.nx;
  t.o000 = r00 + x0; t.o100 = r00 + x1;
  t.o010 = r01 + x0; t.o110 = r01 + x1;
  t.o001 = r10 + x0; t.o101 = r10 + x1;
  t.o011 = r11 + x0; t.o111 = r11 + x1;
  for (int c = 0; c < 3; ++c) uf[(size_t)c * gf.V + i] = 2.0f * sample(uc + (size_t)c * gc.V, t);
}

hipError_t launch_downsample2(const Geo& gc, const float* fine, float* coarse, hipStream_t st) {
  hipLaunchKernelGGL(k_downsample2, dim3((gc.V + 255) / 256), dim3(256), 0, st, gc, fine, coarse);
  return hipGetLastError();
}

hipError_t launch_upsample2_disp(const Geo& gf, const float* uc, float* uf, hipStream_t st) {
  hipLaunchKernelGGL(k_upsample2_disp, dim3((gf.V + 255) / 256), dim3(256), 0, st, gf, uc, uf);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// transform tables (float64, rounded once)
// ---------------------------------------------------------------------------
static size_t a256(size_t b) { return (b + 255) / 256 * 256; }

size_t tables_bytes(const Geo& g) {
  return a256(sizeof(float2) * g.nx) + a256(sizeof(float2) * g.ny) + a256(sizeof(float2) * g.nz) +
         a256(sizeof(float) * (g.nx / 2 + 1)) + a256(sizeof(float) * g.ny) +
         a256(sizeof(float) * g.nz);
}

Tables tables_at(const Geo& g, void* base) {
  char* p = static_cast<char*>(base);
  Tables t;
  t.twx = reinterpret_cast<float2*>(p); p += a256(sizeof(float2) * g.nx);
  t.twy = reinterpret_cast<float2*>(p); p += a256(sizeof(float2) * g.ny);
  t.twz = reinterpret_cast<float2*>(p); p += a256(sizeof(float2) * g.nz);
  t.sx = reinterpret_cast<float*>(p); p += a256(sizeof(float) * (g.nx / 2 + 1));
  t.sy = reinterpret_cast<float*>(p); p += a256(sizeof(float) * g.ny);
  t.sz = reinterpret_cast<float*>(p);
  return t;
}

__device__ __forceinline__ void tables_body(const Geo& g, const Tables& t, int bx, int gx) {
  const int n_all = g.nx + g.ny + g.nz + (g.nx / 2 + 1) + g.ny + g.nz;
  for (int i = bx * blockDim.x + threadIdx.x; i < n_all; i += gx * blockDim.x) {
    int k = i;
    float2* tw = nullptr;
    float* sv = nullptr;
    int n = 0;
    if (k < g.nx) { tw = t.twx; n = g.nx; }
    else if ((k -= g.nx) < g.ny) { tw = t.twy; n = g.ny; }
    else if ((k -= g.ny) < g.nz) { tw = t.twz; n = g.nz; }
    else if ((k -= g.nz) < g.nx / 2 + 1) { sv = t.sx; n = g.nx; }
    else if ((k -= g.nx / 2 + 1) < g.ny) { sv = t.sy; n = g.ny; }
    else { k -= g.ny; sv = t.sz; n = g.nz; }
    if (tw) {
      double sn, cs;
      sincospi(-2.0 * (double)k / (double)n, &sn, &cs);
      tw[k] = make_float2((float)cs, (float)sn);
    } else {
      const double h = sinpi((double)k / (double)n);
      sv[k] = (float)(4.0 * h * h);
    }
  }
}

__global__ void k_tables(Geo g, Tables t) { tables_body(g, t, blockIdx.x, gridDim.x); }

hipError_t launch_tables(const Geo& g, const Tables& t, hipStream_t st) {
  hipLaunchKernelGGL(k_tables, dim3(4), dim3(256), 0, st, g, t);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// pass A: t -> x half spectrum
// X layout: X[((c * (nx/2 + 1) + p) * nz + z) * ny + y], p <= nx/2.
// ---------------------------------------------------------------------------
// Coordinates of a workgroup's tile: its block index and grid extent in an
// ordinary launch (of_block), or the ones a mixed-size launch decodes for it.
// z is the pair within a batch of one size; remap: x-line tiles may be
// reordered for the XCDs (see xline_tile).
struct Blk {
  int x, y, z, gx, gy;
  bool remap;
  __device__ static Blk of_block() {
    return Blk{(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z, (int)gridDim.x, (int)gridDim.y, true};
  }
};

// Tile (y-block, z) of an x-line workgroup.  Workgroups are dispatched
// round-robin over the 8 XCDs, each with its own L2; when the grid allows,
// each XCD gets one contiguous range of tiles instead, so that neighbouring
// tiles (which share 128-byte lines of the half spectrum, and z-planes for
// the gathers) meet in the same L2.
__device__ __forceinline__ void xline_tile(const Blk& bk, int& by, int& z) {
  const int nby = bk.gx, n = bk.gx * bk.gy;
  int l = bk.x + nby * bk.y;
  if (bk.remap && (n & 7) == 0) l = (l & 7) * (n >> 3) + (l >> 3);
  z = l / nby;
  by = l - z * nby;
}

// Run idx of an x-line block (four consecutive x of one row): consecutive
// runs alternate between the two rows of a pair.  The rows of a pair share
// one complex LDS line (real and imaginary parts), so the 32 lanes of a half
// wavefront reading or writing their runs' floats reach all 32 banks (one
// row per lane would reach only the 16 banks of its parity).
__device__ __forceinline__ void run_of(int idx, int q4, const XDivs& xd, int& row, int& x4) {
  const int pr = (int)fdiv((uint32_t)(idx >> 1), xd.q4);
  x4 = (idx >> 1) - pr * q4;
  row = 2 * pr + (idx & 1);
}

// x-line transform of a block: the compile-time plan when NX is one of the
// specialised lengths, else the host-made plan.
template <int NX, bool INV>
__device__ __forceinline__ void x_transform(float2* buf, const float2* tw, const FftPlan& px,
                                            const XDivs& xd, int ls) {
  if constexpr (NX > 0)
    fft_lines_ct<NX, kEpt, INV, kXlPadsh>(buf, tw, (int)xd.lines.d, ls);
  else
    fft_lines<kEpt, INV, false, kXlPadsh>(buf, tw, px, xd.lines, 1, ls);
}

// Split the transformed line pairs of one block into the two rows' half
// spectra, scaled by 1 / nx, and store them (row pairs contiguous along y).
// Bins 0 and nx/2 of a real row are real: they go to planes 0 and nx/2 with
// zero imaginary part.  With the 1 / nx here an x transform followed by the
// inverse of pass C is the identity.
// Row y of tile row t (0 <= t < rows) of x-line tile by: consecutive rows,
// or, for half-plane sizes, two groups of ygrp rows ny / 2 apart.
__device__ __forceinline__ int tile_row(const XDivs& xd, int by, int t) {
  return by * xd.ygrp + t + (t >= xd.ygrp ? xd.yhalf - xd.ygrp : 0);
}

template <int NX, bool YS = false>
__device__ __forceinline__ void store_half_spectrum(const Geo& g, const XDivs& xd, int ls,
                                                    const float2* buf, float2* __restrict__ X,
                                                    const float2* __restrict__ twy, int by, int z) {
  const int nx = NX ? NX : g.nx, nh = nx / 2;
  const int yb2 = (int)xd.yb2.d;
  const int nthr = blockDim.x;
  const float s1 = 1.0f / (float)nx, sh = 0.5f * s1;
  // bin k of the two rows of line pair yp, (a.re, a.im, b.re, b.im); for
  // k = 0 also the Nyquist bin (both real)
  auto bins = [&](int c, int yp, int k, float4& o, float4& on) {
    const float2* Z = buf + (c * yb2 + yp) * ls;
    if (k == 0) {
      const float2 z0 = Z[0], zn = Z[lpad<kXlPadsh>(nh)];
      o = make_float4(z0.x * s1, 0.f, z0.y * s1, 0.f);
      on = make_float4(zn.x * s1, 0.f, zn.y * s1, 0.f);
    } else {
      const float2 zk = Z[lpad<kXlPadsh>(k)], zm = Z[lpad<kXlPadsh>(nx - k)];
      // a = (Zk + conj(Zm)) / 2 ; b = -i (Zk - conj(Zm)) / 2
      o = make_float4(sh * (zk.x + zm.x), sh * (zk.y - zm.y), sh * (zk.y + zm.y),
                      -sh * (zk.x - zm.x));
      on = o;
    }
  };
  if constexpr (!YS) {
    const int nout = 3 * nh * yb2;
    for (int idx = threadIdx.x; idx < nout; idx += nthr) {
      const int ck = (int)fdiv((uint32_t)idx, xd.yb2);
      const int yp = idx - ck * yb2;
      const int c = (int)fdiv((uint32_t)ck, xd.nh);
      const int k = ck - c * nh;
      const int y = by * xd.ygrp + 2 * yp;
      float4 o, on;
      bins(c, yp, k, o, on);
      if (k == 0)
        store_wt(reinterpret_cast<float4*>(X + ((size_t)(c * (nh + 1) + nh) * g.nz + z) * g.ny + y), on);
      store_wt(reinterpret_cast<float4*>(X + ((size_t)(c * (nh + 1) + k) * g.nz + z) * g.ny + y), o);
    }
  } else {
    // First step of the y transform, decimation in frequency by 2 across the
    // tile's row groups: rows n (A) and n + ny/2 (B) give A + B, stored in
    // sub-plane 0 (the even y frequencies), and (A - B) W^n, W = exp(-2 pi i
    // / ny), in sub-plane 1 (the odd ones); sub-plane s of plane (c, k) holds
    // element (z, n) at s * nz * ny/2 + z * ny/2 + n.
    const int yq = (int)xd.yq.d, nyh = xd.yhalf;
    const size_t sub = (size_t)g.nz * nyh;
    const int nout = 3 * nh * yq;
    for (int idx = threadIdx.x; idx < nout; idx += nthr) {
      const int ck = (int)fdiv((uint32_t)idx, xd.yq);
      const int j = idx - ck * yq;
      const int c = (int)fdiv((uint32_t)ck, xd.nh);
      const int k = ck - c * nh;
      const int n = by * xd.ygrp + 2 * j;
      const float2 w0 = twy[n], w1 = twy[n + 1];
      float4 a, an, b, bn;
      bins(c, j, k, a, an);
      bins(c, j + yq, k, b, bn);
      auto put = [&](int plane, const float4& A, const float4& B) {
        float2* d = X + (size_t)(c * (nh + 1) + plane) * g.nz * g.ny + (size_t)z * nyh + n;
        store_wt(reinterpret_cast<float4*>(d), make_float4(A.x + B.x, A.y + B.y, A.z + B.z, A.w + B.w));
        const float ex = A.x - B.x, ey = A.y - B.y, fx = A.z - B.z, fy = A.w - B.w;
        store_wt(reinterpret_cast<float4*>(d + sub),
                 make_float4(ex * w0.x - ey * w0.y, ex * w0.y + ey * w0.x, fx * w1.x - fy * w1.y,
                             fx * w1.y + fy * w1.x));
      };
      put(k, a, b);
      if (k == 0) put(nh, an, bn);
    }
  }
}

template <int NX, bool YS = false>
__global__ void __launch_bounds__(kXlMaxThreads) k_pass_a(Geo g, FftPlan px, XDivs xd, int ls,
                                                const float2* __restrict__ twx,
                                                const float2* __restrict__ twy,
                                                const float* __restrict__ s1,
                                                const float* __restrict__ s2, float gamma,
                                                float2* __restrict__ X, float2* __restrict__ X2) {
  extern __shared__ float2 lds[];
  const int nx = NX ? NX : g.nx, q4 = nx / 4;
  s1 = at_pair(s1, 3 * (size_t)g.V, blockIdx.z);
  s2 = at_pair(s2, 3 * (size_t)g.V, blockIdx.z);
  X = at_pair(X, spectrum_elems(g), blockIdx.z);
  X2 = at_pair(X2, spectrum_elems(g), blockIdx.z);
  const int yb = (int)xd.yb.d, yb2 = (int)xd.yb2.d;
  float2* tw = lds;
  float2* buf = lds + nx;
  int by, z;
  xline_tile(Blk::of_block(), by, z);
  const int nthr = blockDim.x;
  for (int i = threadIdx.x; i < nx; i += nthr) tw[i] = twx[i];

  // load t = s1 + gamma (s1 - s2) as float4 runs along x (all loads first)
  const int items = 3 * yb * q4;
  float4 va[kXItems], vb[kXItems];
  int goff[kXItems];
#pragma unroll
  for (int it = 0; it < kXItems; ++it) {
    const int idx = threadIdx.x + it * nthr;
    if (idx < items) {
      int row, x4;
      run_of(idx, q4, xd, row, x4);
      const int c = (int)fdiv((uint32_t)row, xd.yb);
      const int yy = row - c * yb;
      goff[it] = c * g.V + (z * g.ny + tile_row(xd, by, yy)) * nx + 4 * x4;
      va[it] = *reinterpret_cast<const float4*>(s1 + goff[it]);
      if (s2) vb[it] = *reinterpret_cast<const float4*>(s2 + goff[it]);
    }
  }
  float* bf = reinterpret_cast<float*>(buf);
#pragma unroll
  for (int it = 0; it < kXItems; ++it) {
    const int idx = threadIdx.x + it * nthr;
    if (idx < items) {
      int row, x4;
      run_of(idx, q4, xd, row, x4);
      const int c = (int)fdiv((uint32_t)row, xd.yb);
      const int yy = row - c * yb;
      float4 t = va[it];
      if (s2) {
        const float4 u = vb[it];
        t = make_float4(fmaf(gamma, t.x - u.x, t.x), fmaf(gamma, t.y - u.y, t.y),
                        fmaf(gamma, t.z - u.z, t.z), fmaf(gamma, t.w - u.w, t.w));
      }
      const int line = c * yb2 + (yy >> 1);
      float* d = bf + 2 * (line * ls + lpad<kXlPadsh>(4 * x4)) + (yy & 1);
      d[0] = t.x;
      d[2] = t.y;
      d[4] = t.z;
      d[6] = t.w;
    }
  }
  __syncthreads();
  x_transform<NX, false>(buf, tw, px, xd, ls);
  store_half_spectrum<NX, YS>(g, xd, ls, buf, X, twy, by, z);
  if (X2) store_half_spectrum<NX, YS>(g, xd, ls, buf, X2, twy, by, z);  // a second copy
}

static size_t pass_a_lds_rows(const Geo& g, int yb) {
  return sizeof(float2) * ((size_t)g.nx + (size_t)3 * (yb / 2) * xline_stride(g.nx));
}
static size_t pass_a_lds(const Geo& g) { return pass_a_lds_rows(g, xline_rows(g)); }

hipError_t launch_pass_a(const Geo& g, const FftPlan& px, const Tables& t, const float* s1,
                         const float* s2, float gamma, float2* X, hipStream_t st, int batch, float2* X2) {
  const int yb = xline_rows(g);
  const dim3 grid(g.ny / yb, g.nz, batch), block(xline_threads(g));
  const size_t lds = pass_a_lds(g);
  const XDivs xd = make_xdivs(g);
  const int ls = xline_stride(g.nx);
#define NADMM_PASS_A(N) \
  hipLaunchKernelGGL(k_pass_a<N>, grid, block, lds, st, g, px, xd, ls, t.twx, t.twy, s1, s2, gamma, X, X2)
  if (ysplit(g)) {
    if (g.nx == 192)
      hipLaunchKernelGGL((k_pass_a<192, true>), grid, block, lds, st, g, px, xd, ls, t.twx, t.twy, s1, s2, gamma, X, X2);
    else
      hipLaunchKernelGGL((k_pass_a<0, true>), grid, block, lds, st, g, px, xd, ls, t.twx, t.twy, s1, s2, gamma, X, X2);
    return hipGetLastError();
  }
  switch (g.nx) {
    case 32: NADMM_PASS_A(32); break;
    case 64: NADMM_PASS_A(64); break;
    case 96: NADMM_PASS_A(96); break;
    case 128: NADMM_PASS_A(128); break;
    case 192: NADMM_PASS_A(192); break;
    default: NADMM_PASS_A(0); break;
  }
#undef NADMM_PASS_A
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// pass B: y-z plane FFT, spectral multiply, inverse
// ---------------------------------------------------------------------------
// Stage schedules of pass B.  PlansRT reads the (host-made) plans from LDS
// and dispatches every stage's radix at run time; PlansCT<NY, NZ> has the
// same plans as compile-time constants, so only the radices a size uses are
// compiled into its kernel (small code, constant index arithmetic).
struct PlansRT {
  const TeamPlan* py;
  const TeamPlan* pz;
  const TeamPlan* pzi;
  __device__ int ly() const { return py->L; }
  __device__ int lz() const { return pz->L; }
  template <bool INV>
  __device__ __forceinline__ void y_all(float2* line, const float2* tw, int tl) const {
    for (int st = 0; st < py->nstages; ++st)
      team_stage_any<kTeamEpt, INV, 4>(line, tw, py->st[st], py->L, tl, 1);
  }
  __device__ __forceinline__ void z_fused(float2* line, const float2* tw, int tl, int es,
                          const SpectralMult& mult) const {
    for (int st = 0; st + 1 < pz->nstages; ++st)
      team_stage_any<kTeamEpt, false, 0>(line, tw, pz->st[st], pz->L, tl, es);
    team_fused_any<kTeamEpt, 0>(line, tw, pz->st[pz->nstages - 1], pzi->st[0], pz->L, tl, es, mult);
    for (int st = 1; st < pzi->nstages; ++st)
      team_stage_any<kTeamEpt, true, 0>(line, tw, pzi->st[st], pzi->L, tl, es);
  }
};

constexpr int lane_budget_ce(int nlines) { return 1024 / nlines < 1 ? 1 : 1024 / nlines; }

template <int NY, int NZ>
struct PlansCT {
  static constexpr TeamPlan PY = make_team_plan_ce(NY, lane_budget_ce(NZ));
  static constexpr TeamPlan PZ = make_team_plan_ce(NZ, lane_budget_ce(NY));
  static constexpr TeamPlan PZI = reverse_team_plan_ce(PZ);
  static_assert(PY.nstages > 0 && PZ.nstages > 0, "no wave-team plan for this size");
  __device__ int ly() const { return PY.L; }
  __device__ int lz() const { return PZ.L; }

  template <int WHICH, bool INV, int PADSH, int S, int SEND>
  __device__ __forceinline__ static void stages(float2* line, const float2* tw, int tl, int es) {
    if constexpr (S < SEND) {
      constexpr TeamPlan P = WHICH == 0 ? PY : (WHICH == 1 ? PZ : PZI);
      constexpr FftStage st = P.st[S];
      team_stage<st.R, P.n / P.L, INV, PADSH>(line, tw, st, P.L, tl, es);
      stages<WHICH, INV, PADSH, S + 1, SEND>(line, tw, tl, es);
    }
  }
  template <bool INV>
  __device__ __forceinline__ void y_all(float2* line, const float2* tw, int tl) const {
    stages<0, INV, 4, 0, PY.nstages>(line, tw, tl, 1);
  }
  __device__ __forceinline__ void z_fused(float2* line, const float2* tw, int tl, int es,
                                          const SpectralMult& mult) const {
    stages<1, false, 0, 0, PZ.nstages - 1>(line, tw, tl, es);
    constexpr FftStage sf = PZ.st[PZ.nstages - 1];
    constexpr FftStage si = PZI.st[0];
    team_fused<sf.R, PZ.n / PZ.L, 0>(line, tw, sf, si, PZ.L, tl, es, mult);
    stages<2, true, 0, 1, PZI.nstages>(line, tw, tl, es);
  }
};

// NY = NZ = 0: any size (run-time plans); otherwise the sizes are fixed.
// DERIV: multiply by d/dlambda of the multiplier.
// SUB: one of the two sub-planes (even or odd y frequencies) of a plane of a
// half-plane size, bk.y = 2 c + s: the transform runs over ny / 2 (NY when
// fixed), the plane is addressed and normalised with the full g.ny, and the
// y twiddles and symbols are the full tables' at 2 q and 2 q + s.
template <int NY, int NZ, bool DERIV = false, bool SUB = false>
// tid, nthr: the thread's index within, and the size of, the thread group
// that transforms this plane (the whole workgroup, or one of several groups
// sharing it, each with its own LDS at lds); every group of a workgroup
// meets the same __syncthreads() barriers.
__device__ __forceinline__ void pass_b_body(const Geo& g, const TeamPlan& py0, const TeamPlan& pz0,
                                            const TeamPlan& pzi0, const XDivs& xd, int rs_host,
                                            const Tables& tg, float2* __restrict__ X, float lambda,
                                            float theta, int order, const Blk& bk, int tid, int nthr,
                                            float2* lds) {
  using PCT = PlansCT<NY ? NY : 32, NZ ? NZ : 32>;
  // compile-time sizes: the same row stride as the host's, as a constant
  constexpr int kRs = NY ? plane_row_stride_ce(NY ? NY : 32, NZ ? NZ : 32, PCT::PY, PCT::PZ) : 0;
  const int rs = NY ? kRs : rs_host;
  // run-time plans are indexed by stage: keep them in LDS
  __shared__ __align__(16) unsigned char plan_mem[NY == 0 ? 3 * sizeof(TeamPlan) : 16];
  TeamPlan* plans = reinterpret_cast<TeamPlan*>(plan_mem);
  using Pol = typename std::conditional<NY == 0, PlansRT, PlansCT<NY, NZ>>::type;
  Pol pol{};
  if constexpr (NY == 0) pol = PlansRT{plans, plans + 1, plans + 2};
  // plane element (z, y) at z * rs + y + y / 16 (host-chosen rs)
  const int nyf = g.ny;  // the full y length (addressing, normalisation)
  const int ny = NY ? NY : (SUB ? nyf / 2 : nyf), nz = NZ ? NZ : g.nz, np = g.nx / 2 + 1;
  const int lane = tid & 63, wave = tid >> 6, nwaves = nthr >> 6;
  float2* twy = lds;
  float2* twz = twy + ny;
  float* sy = reinterpret_cast<float*>(twz + nz);
  float* sz = sy + ny;
  float2* buf = reinterpret_cast<float2*>(sz + nz + ((ny + nz) & 1));  // keep 8-byte alignment
  const int p = bk.x, c = SUB ? bk.y >> 1 : bk.y, ks = SUB ? bk.y & 1 : 0;
  float2* plane = at_pair(X, spectrum_elems(g), bk.z) + (size_t)(c * np + p) * nz * nyf + (size_t)ks * nz * ny;
  const float4* plane4 = reinterpret_cast<const float4*>(plane);
  // the x transform of pass A already carries 1 / nx of the inverse's 1 / V
  const float inv_v = 1.0f / (float)(nyf * nz);
  const int nlw_y = 64 / (NY ? PlansCT<NY ? NY : 32, NZ ? NZ : 32>::PY.L : py0.L);
  // Compile-time sizes: the host launches at least ceil(nz / nlw_y) and
  // ceil(ny / nlw_z) wavefronts when both are <= 16, so every wavefront owns at
  // most one group of rows and one group of columns (no loop over groups).
  constexpr int kNlwY = 64 / PCT::PY.L, kNlwZ = 64 / PCT::PZ.L;
  constexpr bool ONE_PASS = NY > 0 && (NZ + kNlwY - 1) / kNlwY <= 16 && (NY + kNlwZ - 1) / kNlwZ <= 16;

  // Rows of the y transform are owned by wavefronts: lines [l0, l0 + nlw_y)
  // with l0 = wave * nlw_y (+ multiples of nwaves * nlw_y).  Issue the loads
  // of the first group and of the tables together, then store both to LDS.
  auto load_rows = [&](int l0, int b0, float4* v) {
    const int rows = (nz - l0 < nlw_y) ? nz - l0 : nlw_y;
    const int items = rows * (ny / 2);  // float4 = two complex of one row
#pragma unroll
    for (int it = 0; it < kPItems; ++it) {
      const int idx = b0 + lane + it * 64;
      if (idx < items) v[it] = plane4[l0 * (ny / 2) + idx];
    }
    return items;
  };
  auto store_rows = [&](int l0, int b0, int items, const float4* v) {
#pragma unroll
    for (int it = 0; it < kPItems; ++it) {
      const int idx = b0 + lane + it * 64;
      if (idx < items) {
        const int i = 2 * idx;
        const int zz = NY ? i / NY : (int)fdiv((uint32_t)i, xd.ny), yy = i - zz * ny;  // yy even
        float2* d = buf + (l0 + zz) * rs + lpad<4>(yy);
        d[0] = make_float2(v[it].x, v[it].y);
        d[1] = make_float2(v[it].z, v[it].w);
      }
    }
  };
  {
    float2 t2 = make_float2(0.f, 0.f);
    float t1 = 0.f;
    const int ti = tid;
    if (ti < ny) {
      t2 = tg.twy[SUB ? 2 * ti : ti];
      t1 = tg.sy[SUB ? 2 * ti + ks : ti];
    } else if (ti < ny + nz) {
      t2 = tg.twz[ti - ny];
      t1 = tg.sz[ti - ny];
    }
    float4 v[kPItems];
    const int l0 = wave * nlw_y;
    int items = 0;
    if (l0 < nz) items = load_rows(l0, 0, v);
    if (NY == 0 && tid == 0) {
      plans[0] = py0;
      plans[1] = pz0;
      plans[2] = pzi0;
    }
    if (ti < ny) {
      twy[ti] = t2;
      sy[ti] = t1;
    } else if (ti < ny + nz) {
      twz[ti - ny] = t2;
      sz[ti - ny] = t1;
    }
    for (int i = ny + nz + tid; i < 2 * (ny + nz); i += nthr) {  // blocks narrower than ny + nz
      const int k = i - (ny + nz);
      if (k < ny) {
        twy[k] = tg.twy[SUB ? 2 * k : k];
        sy[k] = tg.sy[SUB ? 2 * k + ks : k];
      } else {
        twz[k - ny] = tg.twz[k - ny];
        sz[k - ny] = tg.sz[k - ny];
      }
    }
    if (l0 < nz) {
      store_rows(l0, 0, items, v);
      for (int b0 = kPItems * 64; b0 < items; b0 += kPItems * 64) {
        load_rows(l0, b0, v);
        store_rows(l0, b0, items, v);
      }
    }
  }
  __syncthreads();

  // --- along y ---------------------------------------------------------------
  if constexpr (ONE_PASS) {
    const int l = wave * kNlwY + lane % kNlwY;
    if (l < nz) pol.template y_all<false>(buf + l * rs, twy, lane / kNlwY);
  } else {
    const int nlw = nlw_y, li = lane % nlw, tl = lane / nlw;
    for (int l0 = wave * nlw; l0 < nz; l0 += nwaves * nlw) {
      if (l0 != wave * nlw) {  // further row groups of this wavefront
        float4 v[kPItems];
        const int items = (nz - l0 < nlw ? nz - l0 : nlw) * (ny / 2);
        for (int b0 = 0; b0 < items; b0 += kPItems * 64) {
          load_rows(l0, b0, v);
          store_rows(l0, b0, items, v);
        }
        wave_lds_fence();
      }
      const int l = l0 + li;
      if (l < nz) pol.template y_all<false>(buf + l * rs, twy, tl);
    }
  }
  __syncthreads();

  // --- along z: forward, spectral multiply, inverse, fused per column ------
  {
    const int nlw = 64 / pol.lz(), li = lane % nlw, tl = lane / nlw;
    const float sx = tg.sx[p];
    for (int l0 = wave * nlw; l0 < ny; l0 += nwaves * nlw) {
      const int q = l0 + li;
      if (q < ny) {
        const SpectralMult mult{sz, sx + sy[q], lambda, theta, inv_v, order, DERIV ? 1 : 0};
        pol.z_fused(buf + lpad<4>(q), twz, tl, rs, mult);
      }
      if constexpr (ONE_PASS) break;
    }
  }
  __syncthreads();

  // --- inverse along y, every wavefront stores its own rows ----------------
  {
    const int nlw = nlw_y, li = lane % nlw, tl = lane / nlw;
    float4* out4 = reinterpret_cast<float4*>(plane);
    for (int l0 = wave * nlw; l0 < nz; l0 += nwaves * nlw) {
      if constexpr (ONE_PASS)
        if (l0 != wave * nlw) break;
      const int l = l0 + li;
      if (l < nz) pol.template y_all<true>(buf + l * rs, twy, tl);
      wave_lds_fence();
      const int items = (nz - l0 < nlw ? nz - l0 : nlw) * (ny / 2);
      for (int idx = lane; idx < items; idx += 64) {
        const int i = 2 * idx;
        const int zz = NY ? i / NY : (int)fdiv((uint32_t)i, xd.ny), yy = i - zz * ny;
        const float2* sp = buf + (l0 + zz) * rs + lpad<4>(yy);
        const float2 a = sp[0], b = sp[1];
        store_wt(out4 + l0 * (ny / 2) + idx, make_float4(a.x, a.y, b.x, b.y));
      }
    }
  }
}

template <int NY, int NZ, bool DERIV = false, bool SUB = false>
__global__ void __launch_bounds__(1024) k_pass_b(Geo g, TeamPlan py0, TeamPlan pz0, TeamPlan pzi0,
                                                 XDivs xd, int rs_host, Tables tg, float2* __restrict__ X,
                                                 float lambda, float theta, int order) {
  extern __shared__ float2 lds[];
  pass_b_body<NY, NZ, DERIV, SUB>(g, py0, pz0, pzi0, xd, rs_host, tg, X, lambda, theta, order,
                                  Blk::of_block(), threadIdx.x, blockDim.x, lds);
}

// ---------------------------------------------------------------------------
// pass B for y-z planes larger than one workgroup's LDS: three launches over
// the same half spectrum -- the forward y transform of every row, then per
// group of W columns the forward z transform, the spectral multiply and the
// inverse z transform, then the inverse y transform of every row.
// ---------------------------------------------------------------------------
template <int N, bool INV>
__device__ __forceinline__ void line_transform(float2* buf, const float2* tw, const FftPlan& plan,
                                               const FastDiv& dl, int ls) {
  if constexpr (N > 0)
    fft_lines_ct<N, kEpt, INV, 4>(buf, tw, (int)dl.d, ls);
  else
    fft_lines<kEpt, INV, false, 4>(buf, tw, plan, dl, 1, ls);
}

// dl.d rows (contiguous ny complex each) of the half spectrum per
// workgroup; rows are numbered over (component, plane, z).
template <int NY, bool INV>
__global__ void __launch_bounds__(256) k_split_rows(Geo g, FftPlan py, FastDiv dl, FastDiv dq,
                                                     const float2* __restrict__ twy,
                                                     float2* __restrict__ X) {
  extern __shared__ float2 lds[];
  const int ny = NY ? NY : g.ny, ls = lpad<4>(ny - 1) + 1, half = ny / 2;
  float2* tw = lds;
  float2* buf = lds + ny;
  const int nthr = blockDim.x;
  const int rows = (int)dl.d;
  float4* base = reinterpret_cast<float4*>(at_pair(X, spectrum_elems(g), blockIdx.y) +
                                           (size_t)blockIdx.x * rows * ny);
  for (int i = threadIdx.x; i < ny; i += nthr) tw[i] = twy[i];
  const int items = rows * half;  // float4 = two complex of one row
  for (int idx = threadIdx.x; idx < items; idx += nthr) {
    const int row = NY ? idx / (NY / 2) : (int)fdiv((uint32_t)idx, dq);
    const int e = 2 * (idx - row * half);
    const float4 v = base[idx];
    float2* d = buf + row * ls + lpad<4>(e);  // e even: e and e + 1 share a padding group
    d[0] = make_float2(v.x, v.y);
    d[1] = make_float2(v.z, v.w);
  }
  __syncthreads();
  line_transform<NY, INV>(buf, tw, py, dl, ls);
  for (int idx = threadIdx.x; idx < items; idx += nthr) {
    const int row = NY ? idx / (NY / 2) : (int)fdiv((uint32_t)idx, dq);
    const int e = 2 * (idx - row * half);
    const float2* d = buf + row * ls + lpad<4>(e);
    store_wt(base + idx, make_float4(d[0].x, d[0].y, d[1].x, d[1].y));
  }
}

// W columns (a power of two dividing ny) of one (component, plane): z lines
// of nz complex with stride ny in memory, transposed into LDS lines on load.
template <int NZ>
__global__ void __launch_bounds__(256) k_split_cols(Geo g, FftPlan pz, FastDiv dl, FastDiv dz,
                                                     Tables t, float2* __restrict__ X,
                                                     float lambda, float theta, int order,
                                                     int deriv) {
  extern __shared__ float2 lds[];
  const int ny = g.ny, nz = NZ ? NZ : g.nz, ls = lpad<4>(nz - 1) + 1, np = g.nx / 2 + 1;
  const int W = (int)dl.d, hw = W / 2;
  float2* tw = lds;
  float* szl = reinterpret_cast<float*>(tw + nz);
  float2* buf = reinterpret_cast<float2*>(szl + nz + (nz & 1));
  const int nthr = blockDim.x;
  const int q0 = blockIdx.x * W, p = blockIdx.y, c = blockIdx.z % 3;
  float2* plane = at_pair(X, spectrum_elems(g), blockIdx.z / 3) + (size_t)(c * np + p) * nz * ny;
  for (int i = threadIdx.x; i < nz; i += nthr) {
    tw[i] = t.twz[i];
    szl[i] = t.sz[i];
  }
  const int hs = __ffs(hw) - 1;  // W is a power of two: idx / hw == idx >> hs
  const int items = nz * hw;     // float4 = columns q0 + 2j, q0 + 2j + 1 of row rr
  for (int idx = threadIdx.x; idx < items; idx += nthr) {
    const int rr = idx >> hs, jj = idx - (rr << hs);
    const float4 v = *reinterpret_cast<const float4*>(plane + (size_t)rr * ny + q0 + 2 * jj);
    buf[(2 * jj) * ls + lpad<4>(rr)] = make_float2(v.x, v.y);
    buf[(2 * jj + 1) * ls + lpad<4>(rr)] = make_float2(v.z, v.w);
  }
  __syncthreads();
  line_transform<NZ, false>(buf, tw, pz, dl, ls);
  // multiply by theta / (theta + lambda K^n) / (ny nz); pass A carried 1 / nx
  const float inv = 1.0f / (float)(ny * nz), kx = t.sx[p];
  for (int idx = threadIdx.x; idx < W * nz; idx += nthr) {
    const int l = NZ ? idx / NZ : (int)fdiv((uint32_t)idx, dz);
    const int r = idx - l * nz;
    const float k0 = kx + t.sy[q0 + l] + szl[r];
    float kn = k0;
    for (int i = 1; i < order; ++i) kn *= k0;
    const float rd = __builtin_amdgcn_rcpf(theta + lambda * kn);
    const float m = deriv ? -theta * inv * kn * rd * rd : theta * inv * rd;
    float2& e = buf[l * ls + lpad<4>(r)];
    e = make_float2(e.x * m, e.y * m);
  }
  __syncthreads();
  line_transform<NZ, true>(buf, tw, pz, dl, ls);
  for (int idx = threadIdx.x; idx < items; idx += nthr) {
    const int rr = idx >> hs, jj = idx - (rr << hs);
    const float2 a = buf[(2 * jj) * ls + lpad<4>(rr)], b = buf[(2 * jj + 1) * ls + lpad<4>(rr)];
    store_wt(reinterpret_cast<float4*>(plane + (size_t)rr * ny + q0 + 2 * jj), make_float4(a.x, a.y, b.x, b.y));
  }
}

// Shapes of the split pass B: rows per row workgroup (divides the row count
// 3 (nx/2 + 1) nz) and columns per column workgroup (a power of two <= 16
// dividing ny); at most 256 threads, at most kEpt points per thread.
struct SplitShape {
  int rb, rows_threads, w, cols_threads;
};
static SplitShape split_shape(const Geo& g) {
  SplitShape sh{1, 64, 2, 64};
  const long total = 3L * (g.nx / 2 + 1) * g.nz;
  for (int rb = 8; rb >= 1; rb /= 2)
    if (total % rb == 0 && rb * g.ny <= kEpt * 256) {
      sh.rb = rb;
      break;
    }
  for (int w = 16; w >= 2; w /= 2)
    if (g.ny % w == 0 && w * g.nz <= kEpt * 256) {
      sh.w = w;
      break;
    }
  auto threads = [](int elems) {
    int t = round_up((elems + 7) / 8, 64);
    return t > 256 ? 256 : (t < 64 ? 64 : t);
  };
  sh.rows_threads = threads(sh.rb * g.ny);
  sh.cols_threads = threads(sh.w * g.nz);
  return sh;
}
static size_t split_rows_lds(const Geo& g, const SplitShape& sh) {
  return sizeof(float2) * ((size_t)g.ny + (size_t)sh.rb * (lpad<4>(g.ny - 1) + 1));
}
static size_t split_cols_lds(const Geo& g, const SplitShape& sh) {
  return sizeof(float2) * (size_t)g.nz + sizeof(float) * (size_t)(g.nz + (g.nz & 1)) +
         sizeof(float2) * (size_t)sh.w * (lpad<4>(g.nz - 1) + 1);
}

bool plane_fits(const Geo& g) {
  return g.ny * g.nz <= 16384 && plane_lds_bytes(g, plane_row_stride(g)) <= (size_t)kMaxLds;
}

static Geo half_plane_geo(const Geo& g) { return Geo{g.nx, g.ny / 2, g.nz, g.V / 2}; }

static bool ysplit_eval(const Geo& g) {
  if (g.ny % 8 || plane_fits(g)) return false;
  const Geo gs = half_plane_geo(g);
  if (!plane_fits(gs)) return false;
  const TeamPlan ty = plane_plan_y(gs), tz = plane_plan_z(gs);
  return ty.nstages > 0 && tz.nstages > 0 && gs.ny * gs.nz < 65536;
}

// Memoised per sizes: every x-line and plane launch asks, and the answer
// takes the plane planners' searches.
bool ysplit(const Geo& g) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, int>, bool> memo;
  const auto key = std::make_tuple(g.nx, g.ny, g.nz);
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
  }
  const bool v = ysplit_eval(g);
  std::lock_guard<std::mutex> lk(mu);
  memo[key] = v;
  return v;
}

static bool split_shape_ok(const Geo& g) {
  const SplitShape sh = split_shape(g);
  const FftPlan py = make_plan(g.ny), pz = make_plan(g.nz);
  return py.nstages > 0 && pz.nstages > 0 && sh.rb * g.ny <= kEpt * sh.rows_threads &&
         g.ny % sh.w == 0 && sh.w * g.nz <= kEpt * sh.cols_threads &&
         split_rows_lds(g, sh) <= (size_t)kMaxLds && split_cols_lds(g, sh) <= (size_t)kMaxLds;
}

static hipError_t launch_pass_b_split(const Geo& g, const Tables& t, float2* X, float lambda,
                                      float theta, int order, hipStream_t st, int batch,
                                      int deriv) {
  const SplitShape sh = split_shape(g);
  const FftPlan py = make_plan(g.ny), pz = make_plan(g.nz);
  const int np = g.nx / 2 + 1;
  const dim3 rgrid((unsigned)(3L * np * g.nz / sh.rb), batch), rblock(sh.rows_threads);
  const dim3 cgrid(g.ny / sh.w, np, 3 * batch), cblock(sh.cols_threads);
  const size_t rlds = split_rows_lds(g, sh), clds = split_cols_lds(g, sh);
  const FastDiv drows = make_fastdiv(sh.rb), dhalf = make_fastdiv(g.ny / 2);
  const FastDiv dw = make_fastdiv(sh.w), dz = make_fastdiv(g.nz);
#define NADMM_ROWS(N, INV)                                                                    \
  hipLaunchKernelGGL((k_split_rows<N, INV>), rgrid, rblock, rlds, st, g, py, drows, dhalf, t.twy, X)
#define NADMM_ROWS_NY(INV)               \
  switch (g.ny) {                        \
    case 128: NADMM_ROWS(128, INV); break; \
    case 192: NADMM_ROWS(192, INV); break; \
    case 256: NADMM_ROWS(256, INV); break; \
    default: NADMM_ROWS(0, INV); break;    \
  }
#define NADMM_COLS(N) \
  hipLaunchKernelGGL((k_split_cols<N>), cgrid, cblock, clds, st, g, pz, dw, dz, t, X, lambda, theta, order, \
                     (int)deriv)
  NADMM_ROWS_NY(false);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (g.nz) {
    case 96: NADMM_COLS(96); break;
    case 128: NADMM_COLS(128); break;
    case 192: NADMM_COLS(192); break;
    case 256: NADMM_COLS(256); break;
    default: NADMM_COLS(0); break;
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  NADMM_ROWS_NY(true);
#undef NADMM_COLS
#undef NADMM_ROWS_NY
#undef NADMM_ROWS
  return hipGetLastError();
}

static size_t pass_b_lds(const Geo& g) { return plane_lds_bytes(g, plane_row_stride(g)); }

// Both sub-planes of every plane of a half-plane size, one workgroup each.
static hipError_t launch_pass_b_sub(const Geo& g, const Tables& t, float2* X, float lambda, float theta,
                                    int order, hipStream_t st, int batch, bool deriv) {
  const Geo gs = half_plane_geo(g);
  const TeamPlan ty = plane_plan_y(gs), tz = plane_plan_z(gs), tzi = reverse_team_plan(tz);
  // exactly the wavefronts the sub-plane's team plans need (no tuning)
  const int waves = plane_waves_needed(gs);
  const dim3 grid(g.nx / 2 + 1, 6, batch), block(64 * waves);
  const size_t lds = pass_b_lds(gs);
  const XDivs xd = make_xdivs_rows(gs, 2);  // only its ny and nz divisors are used
  const int rs = plane_row_stride(gs);
  if (!deriv && gs.ny == 96 && gs.nz == 128)  // 192 x 128 planes
    hipLaunchKernelGGL((k_pass_b<96, 128, false, true>), grid, block, lds, st, g, ty, tz, tzi, xd, rs, t, X,
                       lambda, theta, order);
  else if (deriv)
    hipLaunchKernelGGL((k_pass_b<0, 0, true, true>), grid, block, lds, st, g, ty, tz, tzi, xd, rs, t, X,
                       lambda, theta, order);
  else
    hipLaunchKernelGGL((k_pass_b<0, 0, false, true>), grid, block, lds, st, g, ty, tz, tzi, xd, rs, t, X,
                       lambda, theta, order);
  return hipGetLastError();
}

hipError_t launch_pass_b(const Geo& g, const Tables& t, float2* X, float lambda, float theta,
                         int order, hipStream_t st, int batch, bool deriv) {
  if (!plane_fits(g)) {
    if (ysplit(g)) return launch_pass_b_sub(g, t, X, lambda, theta, order, st, batch, deriv);
    return launch_pass_b_split(g, t, X, lambda, theta, order, st, batch, deriv);
  }
  const TeamPlan ty = plane_plan_y(g), tz = plane_plan_z(g);
  const dim3 grid(g.nx / 2 + 1, 3, batch), block(plane_team_threads(g));
  const size_t lds = pass_b_lds(g);
  const XDivs xd = make_xdivs(g);
  const int rs = plane_row_stride(g);
  const TeamPlan tzi = reverse_team_plan(tz);
  // Plane sizes (ny, nz) with compile-time plans, each with the multiplier
  // and with its derivative: every pair of 32, 64, 96 and 128, and the
  // coarser levels of the three-level pyramid over 128 x 128 x 96 (64 x 48,
  // 32 x 24) and over 192 x 192 x 128 (48 x 32).  The run-time-plan kernel
  // serves every other size; at these sizes it takes 2.2-2.6x as long (14 us
  // against 5.4 us for the 51 planes of 32 x 24, 13.9 against 6.3 us for the
  // 99 planes of 64 x 48).
#define NADMM_PASS_B(NY_, NZ_)                                                                      \
  if (g.ny == NY_ && g.nz == NZ_) {                                                                 \
    if (deriv)                                                                                      \
      hipLaunchKernelGGL((k_pass_b<NY_, NZ_, true>), grid, block, lds, st, g, ty, tz, tzi, xd, rs, t, \
                         X, lambda, theta, order);                                                  \
    else                                                                                            \
      hipLaunchKernelGGL((k_pass_b<NY_, NZ_>), grid, block, lds, st, g, ty, tz, tzi, xd, rs, t, X,    \
                         lambda, theta, order);                                                     \
    return hipGetLastError();                                                                       \
  }
  NADMM_PASS_B(32, 32) NADMM_PASS_B(32, 64) NADMM_PASS_B(32, 96) NADMM_PASS_B(32, 128)
  NADMM_PASS_B(64, 32) NADMM_PASS_B(64, 64) NADMM_PASS_B(64, 96) NADMM_PASS_B(64, 128)
  NADMM_PASS_B(96, 32) NADMM_PASS_B(96, 64) NADMM_PASS_B(96, 96) NADMM_PASS_B(96, 128)
  NADMM_PASS_B(128, 32) NADMM_PASS_B(128, 64) NADMM_PASS_B(128, 96) NADMM_PASS_B(128, 128)
  NADMM_PASS_B(64, 48) NADMM_PASS_B(32, 24) NADMM_PASS_B(48, 32)
#undef NADMM_PASS_B
  if (deriv)
    hipLaunchKernelGGL((k_pass_b<0, 0, true>), grid, block, lds, st, g, ty, tz, tzi, xd, rs, t, X,
                       lambda, theta, order);
  else
    hipLaunchKernelGGL((k_pass_b<0, 0>), grid, block, lds, st, g, ty, tz, tzi, xd, rs, t, X, lambda,
                       theta, order);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// pass C: half spectrum -> y = S t, then the mode's pointwise work
// ---------------------------------------------------------------------------
__device__ __forceinline__ float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ __forceinline__ void st4(float* p, float4 v) { store_wt(reinterpret_cast<float4*>(p), v); }
__device__ __forceinline__ float f4get(const float4& v, int e) {
  return e == 0 ? v.x : (e == 1 ? v.y : (e == 2 ? v.z : v.w));
}
__device__ __forceinline__ void f4set(float4& v, int e, float s) {
  if (e == 0) v.x = s; else if (e == 1) v.y = s; else if (e == 2) v.z = s; else v.w = s;
}

// J = grad I1^w at the 4 voxels (x0 .. x0+3, y, z) of a run: periodic central
// differences with unit spacing, the same operations as k_grad_resid.
__device__ __forceinline__ void run_gradient(const Geo& g, int nx, const float* __restrict__ iw,
                                             int x0, int y, int z, float4 J[3]) {
  const uint32_t ny = g.ny, nz = g.nz, n = nx;
  const uint32_t row = ((uint32_t)z * ny + y) * n;
  const float4 c = ld4_at(iw, row + x0);
  const float xm = img_at(iw, row + (x0 == 0 ? nx - 1 : x0 - 1));
  const float xp = img_at(iw, row + (x0 + 4 == nx ? 0 : x0 + 4));
  const float4 ym = ld4_at(iw, ((uint32_t)z * ny + (y == 0 ? ny - 1 : y - 1)) * n + x0);
  const float4 yp = ld4_at(iw, ((uint32_t)z * ny + (y + 1 == (int)ny ? 0 : y + 1)) * n + x0);
  const float4 zm = ld4_at(iw, ((z == 0 ? nz - 1 : z - 1) * ny + y) * n + x0);
  const float4 zp = ld4_at(iw, ((z + 1 == (int)nz ? 0 : z + 1) * ny + y) * n + x0);
  J[0] = make_float4((c.y - xm) * 0.5f, (c.z - c.x) * 0.5f, (c.w - c.y) * 0.5f, (xp - c.z) * 0.5f);
  J[1] = make_float4((yp.x - ym.x) * 0.5f, (yp.y - ym.y) * 0.5f, (yp.z - ym.z) * 0.5f,
                     (yp.w - ym.w) * 0.5f);
  J[2] = make_float4((zp.x - zm.x) * 0.5f, (zp.y - zm.y) * 0.5f, (zp.z - zm.z) * 0.5f,
                     (zp.w - zm.w) * 0.5f);
}

// Pass A at the start of a warping, fused with the linearised data term:
// per run of 4 voxels J = grad I1^w (the differences of k_grad_resid),
// r = I1^w - I0 and s^0 = the data step from zero, stored (the first
// iteration reads both) and transformed along x as pass A transforms s^0.
template <int NX, typename T, bool YS = false>
__device__ __forceinline__ void pass_a0_body(const Geo& g, const FftPlan& px, const XDivs& xd, int ls,
                                             const float2* __restrict__ twx,
                                             const float2* __restrict__ twy,
                                             const float* __restrict__ iw,
                                             const T* __restrict__ ref, float* __restrict__ r_out,
                                             float* __restrict__ s0, float theta, float eps,
                                             int data_term, float2* __restrict__ X, const Blk& bk) {
  extern __shared__ float2 lds[];
  const int nx = NX ? NX : g.nx, q4 = nx / 4;
  iw = at_pair(iw, (size_t)g.V, bk.z);
  ref = at_pair(ref, (size_t)g.V, bk.z);
  r_out = at_pair(r_out, (size_t)g.V, bk.z);
  s0 = at_pair(s0, 3 * (size_t)g.V, bk.z);
  X = at_pair(X, spectrum_elems(g), bk.z);
  const int yb = (int)xd.yb.d, yb2 = (int)xd.yb2.d;
  float2* tw = lds;
  float2* buf = lds + nx;
  int by, z;
  xline_tile(bk, by, z);
  const int nthr = blockDim.x;
  for (int i = threadIdx.x; i < nx; i += nthr) tw[i] = twx[i];
  float* bf = reinterpret_cast<float*>(buf);
  const int nitems = yb * q4;
  for (int idx = threadIdx.x; idx < nitems; idx += nthr) {
    int yy, x4;
    run_of(idx, q4, xd, yy, x4);
    const int x0 = 4 * x4;
    const int y = tile_row(xd, by, yy);
    const uint32_t go = ((uint32_t)z * g.ny + y) * nx + x0;
    float4 J[3];
    run_gradient(g, nx, iw, x0, y, z, J);
    const float4 c = ld4_at(iw, go);
    const float4 rv = make_float4(c.x - img_at(ref, go), c.y - img_at(ref, go + 1),
                                  c.z - img_at(ref, go + 2), c.w - img_at(ref, go + 3));
    store_wt_at(r_out, go, rv);
    float4 sv[3];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float a[3] = {0.f, 0.f, 0.f};
      const float j[3] = {f4get(J[0], e), f4get(J[1], e), f4get(J[2], e)};
      float v[3];
      data_step(a, j, f4get(rv, e), theta, eps, data_term, v);
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) f4set(sv[cc], e, v[cc]);
    }
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      store_wt_at(s0 + cc * g.V, go, sv[cc]);
      float* d = bf + 2 * ((cc * yb2 + (yy >> 1)) * ls + lpad<kXlPadsh>(x0)) + (yy & 1);
      d[0] = sv[cc].x;
      d[2] = sv[cc].y;
      d[4] = sv[cc].z;
      d[6] = sv[cc].w;
    }
  }
  __syncthreads();
  x_transform<NX, false>(buf, tw, px, xd, ls);
  store_half_spectrum<NX, YS>(g, xd, ls, buf, X, twy, by, z);
}

template <int NX, typename T, bool YS = false>
__global__ void __launch_bounds__(kXlMaxThreads) k_pass_a0(Geo g, FftPlan px, XDivs xd, int ls,
                                                 const float2* __restrict__ twx,
                                                 const float2* __restrict__ twy,
                                                 const float* __restrict__ iw,
                                                 const T* __restrict__ ref, float* __restrict__ r_out,
                                                 float* __restrict__ s0, float theta, float eps,
                                                 int data_term, float2* __restrict__ X) {
  pass_a0_body<NX, T, YS>(g, px, xd, ls, twx, twy, iw, ref, r_out, s0, theta, eps, data_term, X, Blk::of_block());
}

template <typename T>
static hipError_t pass_a0_any(const Geo& g, const FftPlan& px, const Tables& t, const float* iw,
                              const T* ref, float* r, float* s0, float theta, float eps,
                              int data_term, float2* X, hipStream_t st, int batch) {
  const int yb = xline_rows(g);
  const dim3 grid(g.ny / yb, g.nz, batch), block(xline_threads(g));
  const size_t lds = pass_a_lds(g);
  const XDivs xd = make_xdivs(g);
  const int ls = xline_stride(g.nx);
#define NADMM_PASS_A0(N)                                                                     \
  hipLaunchKernelGGL((k_pass_a0<N, T>), grid, block, lds, st, g, px, xd, ls, t.twx, t.twy, iw, ref, r, \
                     s0, theta, eps, data_term, X)
  if (ysplit(g)) {
    if (g.nx == 192)
      hipLaunchKernelGGL((k_pass_a0<192, T, true>), grid, block, lds, st, g, px, xd, ls, t.twx, t.twy, iw, ref,
                         r, s0, theta, eps, data_term, X);
    else
      hipLaunchKernelGGL((k_pass_a0<0, T, true>), grid, block, lds, st, g, px, xd, ls, t.twx, t.twy, iw, ref, r,
                         s0, theta, eps, data_term, X);
    return hipGetLastError();
  }
  switch (g.nx) {
    case 32: NADMM_PASS_A0(32); break;
    case 64: NADMM_PASS_A0(64); break;
    case 96: NADMM_PASS_A0(96); break;
    case 128: NADMM_PASS_A0(128); break;
    case 192: NADMM_PASS_A0(192); break;
    default: NADMM_PASS_A0(0); break;
  }
#undef NADMM_PASS_A0
  return hipGetLastError();
}
hipError_t launch_pass_a0(const Geo& g, const FftPlan& px, const Tables& t, const float* iw,
                          const float* ref, float* r, float* s0, float theta, float eps,
                          int data_term, float2* X, hipStream_t st, int batch) {
  return pass_a0_any(g, px, t, iw, ref, r, s0, theta, eps, data_term, X, st, batch);
}
hipError_t launch_pass_a0(const Geo& g, const FftPlan& px, const Tables& t, const float* iw,
                          const uint16_t* ref, float* r, float* s0, float theta, float eps,
                          int data_term, float2* X, hipStream_t st, int batch) {
  return pass_a0_any(g, px, t, iw, ref, r, s0, theta, eps, data_term, X, st, batch);
}

template <int MODE, int NX, bool YS = false>
__device__ __forceinline__ void pass_c_body(const Geo& g, const FftPlan& px, const XDivs& xd, int ls,
                                            const float2* __restrict__ twx, PassCArgs a, const Blk& bk) {
  extern __shared__ float2 lds[];
  const int nx = NX ? NX : g.nx, nh = nx / 2, q4 = nx / 4;
  {
    const int b = bk.z;
    const size_t v1 = g.V, v3 = 3 * (size_t)g.V;
    a.X = at_pair(a.X, spectrum_elems(g), b);
    a.s1 = at_pair(a.s1, v3, b);
    a.s2 = at_pair(a.s2, v3, b);
    a.J = at_pair(a.J, v3, b);
    a.r = at_pair(a.r, v1, b);
    a.iw = at_pair(a.iw, v1, b);
    a.out = at_pair(a.out, v3, b);
    a.v_out = at_pair(a.v_out, v3, b);
    a.b_out = at_pair(a.b_out, v3, b);
    a.u_old = at_pair(a.u_old, v3, b);
    a.img = at_pair(a.img, v1, b);
    a.img_bf16 = at_pair(a.img_bf16, v1, b);
    a.iw_out = at_pair(a.iw_out, v1, b);
    a.vel_out = at_pair(a.vel_out, v3, b);
  }
  const int yb = (int)xd.yb.d, yb2 = (int)xd.yb2.d;
  const int nthr = blockDim.x;
  float2* tw = lds;
  float2* buf = lds + nx;
  int by, z;
  xline_tile(bk, by, z);

  // unpack two rows' half spectra into one complex row: Z = Xa + i Xb
  const int nin = 3 * nh * yb2;
  float4 in[kXItems], inn[kXItems];
  // half-plane sizes: items (c, k, j) over the j-th row pair of each group,
  // two sub-plane values each (in[it], inn[it]), for k = 0 also the Nyquist
  // plane's (in[it + KH], inn[it + KH])
  constexpr int KH = kXItems / 2;
  const int yq = (int)xd.yq.d, nyh = xd.yhalf;
  const size_t sub = (size_t)g.nz * nyh;
  if constexpr (!YS) {
#pragma unroll
    for (int it = 0; it < kXItems; ++it) {
      const int idx = threadIdx.x + it * nthr;
      if (idx < nin) {
        const int ck = (int)fdiv((uint32_t)idx, xd.yb2);
        const int yp = idx - ck * yb2;
        const int c = (int)fdiv((uint32_t)ck, xd.nh);
        const int k = ck - c * nh;
        const float2* src = a.X + ((size_t)(c * (nh + 1) + k) * g.nz + z) * g.ny + by * xd.ygrp + 2 * yp;
        in[it] = *reinterpret_cast<const float4*>(src);
        if (k == 0)  // the Nyquist plane
          inn[it] = *reinterpret_cast<const float4*>(src + (size_t)nh * g.nz * g.ny);
      }
    }
  } else {
#pragma unroll
    for (int it = 0; it < KH; ++it) {
      const int idx = threadIdx.x + it * nthr;
      if (idx < nin / 2) {
        const int ck = (int)fdiv((uint32_t)idx, xd.yq);
        const int jj = idx - ck * yq;
        const int c = (int)fdiv((uint32_t)ck, xd.nh);
        const int k = ck - c * nh;
        const float2* src =
            a.X + (size_t)(c * (nh + 1) + k) * g.nz * g.ny + (size_t)z * nyh + by * xd.ygrp + 2 * jj;
        in[it] = *reinterpret_cast<const float4*>(src);
        inn[it] = *reinterpret_cast<const float4*>(src + sub);
        if (k == 0) {  // the Nyquist plane
          const float2* srn = src + (size_t)nh * g.nz * g.ny;
          in[it + KH] = *reinterpret_cast<const float4*>(srn);
          inn[it + KH] = *reinterpret_cast<const float4*>(srn + sub);
        }
      }
    }
  }
  // float4 runs of 4 voxels along x for the pointwise part
  const int nitems = yb * q4;
  constexpr int MI = 2;  // runs per thread (host checks yb * nx / 4 <= 2 * threads)
  int gi[MI];
#pragma unroll
  for (int it = 0; it < MI; ++it) {
    const int idx = threadIdx.x + it * nthr;
    int yy, x4;
    run_of(idx, q4, xd, yy, x4);
    gi[it] = (z * g.ny + tile_row(xd, by, yy)) * nx + 4 * x4;
  }
  for (int i = threadIdx.x; i < nx; i += nthr) tw[i] = twx[i];
  if constexpr (YS) {
    // last step of the inverse y transform, decimation in time by 2: rows n
    // and n + ny/2 are P0 + conj(W^n) P1 and P0 - conj(W^n) P1 of the two
    // sub-planes' values P0, P1 (the inverse of the forward step in
    // store_half_spectrum, the factor 1/2 carried by the multiplier's 1/V)
#pragma unroll
    for (int it = 0; it < KH; ++it) {
      const int idx = threadIdx.x + it * nthr;
      if (idx < nin / 2) {
        const int ck = (int)fdiv((uint32_t)idx, xd.yq);
        const int jj = idx - ck * yq;
        const int c = (int)fdiv((uint32_t)ck, xd.nh);
        const int k = ck - c * nh;
        const int n = by * xd.ygrp + 2 * jj;
        const float2 w0 = a.twy[n], w1 = a.twy[n + 1];
        // A = P0 + conj(w) P1 and B = P0 - conj(w) P1, per row of the pair
        auto dit = [&](const float4& P0, const float4& P1, float4& A, float4& B) {
          const float t0x = w0.x * P1.x + w0.y * P1.y, t0y = w0.x * P1.y - w0.y * P1.x;
          const float t1x = w1.x * P1.z + w1.y * P1.w, t1y = w1.x * P1.w - w1.y * P1.z;
          A = make_float4(P0.x + t0x, P0.y + t0y, P0.z + t1x, P0.w + t1y);
          B = make_float4(P0.x - t0x, P0.y - t0y, P0.z - t1x, P0.w - t1y);
        };
        float4 qa, qb;
        dit(in[it], inn[it], qa, qb);
        float2* ZA = buf + (c * yb2 + jj) * ls;
        float2* ZB = buf + (c * yb2 + jj + yq) * ls;
        if (k == 0) {
          float4 na, nb;
          dit(in[it + KH], inn[it + KH], na, nb);
          ZA[0] = make_float2(qa.x, qa.z);
          ZA[lpad<kXlPadsh>(nh)] = make_float2(na.x, na.z);
          ZB[0] = make_float2(qb.x, qb.z);
          ZB[lpad<kXlPadsh>(nh)] = make_float2(nb.x, nb.z);
        } else {
          ZA[lpad<kXlPadsh>(k)] = make_float2(qa.x - qa.w, qa.y + qa.z);
          ZA[lpad<kXlPadsh>(nx - k)] = make_float2(qa.x + qa.w, qa.z - qa.y);
          ZB[lpad<kXlPadsh>(k)] = make_float2(qb.x - qb.w, qb.y + qb.z);
          ZB[lpad<kXlPadsh>(nx - k)] = make_float2(qb.x + qb.w, qb.z - qb.y);
        }
      }
    }
  }
#pragma unroll
  for (int it = 0; it < kXItems; ++it) {
    const int idx = threadIdx.x + it * nthr;
    if (!YS && idx < nin) {
      const int ck = (int)fdiv((uint32_t)idx, xd.yb2);
      const int yp = idx - ck * yb2;
      const int c = (int)fdiv((uint32_t)ck, xd.nh);
      const int k = ck - c * nh;
      float2* Z = buf + (c * yb2 + yp) * ls;
      const float4 q = in[it];  // (a.re, a.im, b.re, b.im)
      if (k == 0) {
        // real DC and Nyquist bins of the two rows (imaginary parts are zero)
        const float4 qn = inn[it];
        Z[0] = make_float2(q.x, q.z);
        Z[lpad<kXlPadsh>(nh)] = make_float2(qn.x, qn.z);
      } else {
        Z[lpad<kXlPadsh>(k)] = make_float2(q.x - q.w, q.y + q.z);
        Z[lpad<kXlPadsh>(nx - k)] = make_float2(q.x + q.w, q.z - q.y);
      }
    }
  }
  __syncthreads();
  x_transform<NX, true>(buf, tw, px, xd, ls);

  float* bf = reinterpret_cast<float*>(buf);
  // LDS slots of run it, component c: four consecutive x of one real row
  auto run_slot = [&](int it, int c) {
    const int idx = threadIdx.x + it * nthr;
    int yy, x4;
    run_of(idx, q4, xd, yy, x4);
    return bf + 2 * ((c * yb2 + (yy >> 1)) * ls + lpad<kXlPadsh>(4 * x4)) + (yy & 1);
  };
  constexpr bool ITER = MODE == kIterFwd || MODE == kIterFwdIw || MODE == kIterFwdIwChk;
  float4 yv[MI][3];
  if (!ITER && MODE != kAdjStep) {
#pragma unroll
    for (int it = 0; it < MI; ++it)
      if (threadIdx.x + it * nthr < nitems)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float* rowp = run_slot(it, c);
          yv[it][c] = make_float4(rowp[0], rowp[2], rowp[4], rowp[6]);
        }
  }

  if (MODE == kOutY) {
#pragma unroll
    for (int it = 0; it < MI; ++it)
      if (threadIdx.x + it * nthr < nitems)
#pragma unroll
        for (int c = 0; c < 3; ++c) st4(a.out + c * g.V + gi[it], yv[it][c]);
  } else if (MODE == kAdjStep) {
    // the same arithmetic as the step adjoint of adjoint.hip, per run of 4
    // voxels (each run read and written by one thread)
#pragma unroll
    for (int it = 0; it < MI; ++it) {
      const int idx = threadIdx.x + it * nthr;
      if (idx >= nitems) break;
      int yy, x4;
      run_of(idx, q4, xd, yy, x4);
      const int x0 = 4 * x4;
      const int y = tile_row(xd, by, yy);
      const int go = (z * g.ny + y) * nx + x0;
      float* slot[3];
      float4 yr[3], s1v[3], s2v[3], jv[3], gv[3], gjv[3], gyo[3], gto[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        slot[c] = run_slot(it, c);
        yr[c] = make_float4(slot[c][0], slot[c][2], slot[c][4], slot[c][6]);
        s1v[c] = ld4_at(a.s1 + c * g.V, go);
        s2v[c] = a.s2 ? ld4_at(a.s2 + c * g.V, go) : s1v[c];
        jv[c] = ld4_at(a.J + c * g.V, go);
        gv[c] = ld4_at(a.gs + c * g.V, go);
        gjv[c] = ld4_at(a.gJ + c * g.V, go);
      }
      const float4 rv = ld4_at(a.r, go);
      float4 grv = ld4_at(a.gr, go);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float t[3], av[3], j[3], gg[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float s = f4get(s1v[c], e);
          t[c] = a.s2 ? fmaf(a.gamma, s - f4get(s2v[c], e), s) : s;
          av[c] = 2.0f * f4get(yr[c], e) - t[c];
          j[c] = f4get(jv[c], e);
          gg[c] = f4get(gv[c], e);
        }
        const float q = a.theta + (j[0] * j[0] + j[1] * j[1] + j[2] * j[2]);
        const float f = (j[0] * av[0] + j[1] * av[1] + j[2] * av[2] + f4get(rv, e)) / q;
        const float cj = (j[0] * gg[0] + j[1] * gg[1] + j[2] * gg[2]) / q;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float ga = gg[c] - cj * j[c];
          const float dj = -f * gg[c] - cj * (av[c] - 2.0f * f * j[c]);
          f4set(gyo[c], e, 2.0f * ga - gg[c]);
          f4set(gto[c], e, gg[c] - ga);
          f4set(gjv[c], e, f4get(gjv[c], e) + dj);
        }
        f4set(grv, e, f4get(grv, e) - cj);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        store_wt_at(a.gy + c * g.V, go, gyo[c]);
        store_wt_at(a.gt + c * g.V, go, gto[c]);
        store_wt_at(a.gJ + c * g.V, go, gjv[c]);
        // gy is the next solve's input: written over the slots y came from
        slot[c][0] = gyo[c].x;
        slot[c][2] = gyo[c].y;
        slot[c][4] = gyo[c].z;
        slot[c][6] = gyo[c].w;
      }
      store_wt_at(a.gr, go, grv);
    }
    __syncthreads();
    x_transform<NX, false>(buf, tw, px, xd, ls);
    store_half_spectrum<NX, YS>(g, xd, ls, buf, a.X, a.twy, by, z);
  } else if (MODE == kAdjY) {
    const float g1w = 1.0f + a.gamma;
#pragma unroll
    for (int it = 0; it < MI; ++it)
      if (threadIdx.x + it * nthr < nitems)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const size_t o = (size_t)c * g.V + gi[it];
          const float4 y4 = yv[it][c], p4 = ld4(a.s1 + o), q1 = ld4(a.out + o);
          const float4 gt = make_float4(p4.x + y4.x, p4.y + y4.y, p4.z + y4.z, p4.w + y4.w);
          st4(a.out + o, make_float4(fmaf(g1w, gt.x, q1.x), fmaf(g1w, gt.y, q1.y), fmaf(g1w, gt.z, q1.z),
                                     fmaf(g1w, gt.w, q1.w)));
          if (a.b_out) {
            const float4 q2 = ld4(a.b_out + o);
            st4(a.b_out + o, make_float4(fmaf(-a.gamma, gt.x, q2.x), fmaf(-a.gamma, gt.y, q2.y),
                                         fmaf(-a.gamma, gt.z, q2.z), fmaf(-a.gamma, gt.w, q2.w)));
          }
          if (a.v_out) st4(a.v_out + o, make_float4(0.f, 0.f, 0.f, 0.f));
        }
  } else if (MODE == kDotY) {
    // products of two float32 values are exact in FP64
    double acc = 0.0;
#pragma unroll
    for (int it = 0; it < MI; ++it)
      if (threadIdx.x + it * nthr < nitems)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float4 o = ld4(a.s1 + c * g.V + gi[it]), y4 = yv[it][c];
          acc = fma((double)y4.x, (double)o.x, acc);
          acc = fma((double)y4.y, (double)o.y, acc);
          acc = fma((double)y4.z, (double)o.z, acc);
          acc = fma((double)y4.w, (double)o.w, acc);
        }
    // each wavefront's sum by a butterfly of shuffles, then the wavefronts'
    // in order (the same order on every run)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    double* red = reinterpret_cast<double*>(lds);
    __syncthreads();  // every thread has read its y from buf
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double sum = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) sum += red[w];
      a.chk_part[blockIdx.x + (size_t)gridDim.x * (blockIdx.y + (size_t)gridDim.y * blockIdx.z)] = sum;
    }
  } else if (ITER) {
    // change sums of the threshold check (FP64; the difference of two
    // float32 values is exact there)
    double chk_d = 0.0, chk_n = 0.0;
    // the runs one after the other (out may alias s2, so a run's loads stay
    // behind the previous run's stores; each run is read and written by the
    // same thread only); unrolled, at the same register count as a loop
    // (measured at 128x128x96: 18.88 -> 18.76 us)
#pragma unroll
    for (int it = 0; it < MI; ++it) {
      const int idx = threadIdx.x + it * nthr;
      if (idx >= nitems) break;
      int yy, x4;
      run_of(idx, q4, xd, yy, x4);
      const int x0 = 4 * x4;
      const int y = tile_row(xd, by, yy);
      const int go = (z * g.ny + y) * nx + x0;
      float4 s1v[3], s2v[3], jv[3], yr[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        s1v[c] = ld4_at(a.s1 + c * g.V, go);
        s2v[c] = a.s2 ? ld4_at(a.s2 + c * g.V, go) : s1v[c];
        if constexpr (MODE == kIterFwd) jv[c] = ld4_at(a.J + c * g.V, go);
      }
      if constexpr (MODE != kIterFwd) run_gradient(g, nx, a.iw, x0, y, z, jv);
      const float4 rv = ld4_at(a.r, go);
      float* slot[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        slot[c] = run_slot(it, c);
        yr[c] = make_float4(slot[c][0], slot[c][2], slot[c][4], slot[c][6]);
      }
      float4 so[3], vo[3];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float t[3], av[3], j[3], v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float s = f4get(s1v[c], e);
          t[c] = fmaf(a.gamma, s - f4get(s2v[c], e), s);
          av[c] = 2.0f * f4get(yr[c], e) - t[c];
          j[c] = f4get(jv[c], e);
        }
        data_step(av, j, f4get(rv, e), a.theta, a.eps, a.data_term, v);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          // s^k = v + b_hat = v + t - y
          f4set(so[c], e, v[c] + (t[c] - f4get(yr[c], e)));
          f4set(vo[c], e, v[c]);
        }
      }
      if constexpr (MODE == kIterFwdIwChk) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const double n = (double)f4get(so[c], e), dd = n - (double)f4get(s1v[c], e);
            chk_d = fma(dd, dd, chk_d);
            chk_n = fma(n, n, chk_n);
          }
      }
      const float gn = a.gamma_next;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        store_wt_at(a.out + c * g.V, go, so[c]);
        if (a.v_out) store_wt_at(a.v_out + c * g.V, go, vo[c]);
        // next solve's input t' = s^k + gamma_next (s^k - s^{k-1}), written
        // over the slots this thread read y from
        const float4 n = so[c], o = s1v[c];
        slot[c][0] = fmaf(gn, n.x - o.x, n.x);
        slot[c][2] = fmaf(gn, n.y - o.y, n.y);
        slot[c][4] = fmaf(gn, n.z - o.z, n.z);
        slot[c][6] = fmaf(gn, n.w - o.w, n.w);
      }
    }
    __syncthreads();
    x_transform<NX, false>(buf, tw, px, xd, ls);
    store_half_spectrum<NX, YS>(g, xd, ls, buf, a.X, a.twy, by, z);
    if constexpr (MODE == kIterFwdIwChk) {
      // the workgroup's sums: each wavefront's by a butterfly of shuffles,
      // then the wavefronts' in order (the same order on every run)
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        chk_d += __shfl_xor(chk_d, off);
        chk_n += __shfl_xor(chk_n, off);
      }
      __syncthreads();  // buf is free again
      double* red = reinterpret_cast<double*>(lds);
      const int wv = threadIdx.x >> 6;
      if ((threadIdx.x & 63) == 0) {
        red[2 * wv] = chk_d;
        red[2 * wv + 1] = chk_n;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        double d = 0.0, n = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
          d += red[2 * w];
          n += red[2 * w + 1];
        }
        const size_t b = blockIdx.x + (size_t)gridDim.x * (blockIdx.y + (size_t)gridDim.y * blockIdx.z);
        a.chk_part[2 * b] = d;
        a.chk_part[2 * b + 1] = n;
      }
    }
  } else if (MODE == kFinalWB) {
#pragma unroll
    for (int it = 0; it < MI; ++it) {
      if (threadIdx.x + it * nthr < nitems) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float4 y4 = yv[it][c];
          if (a.b_out) {
            const float4 s4 = ld4(a.s1 + c * g.V + gi[it]);
            st4(a.b_out + c * g.V + gi[it],
                make_float4(s4.x - y4.x, s4.y - y4.y, s4.z - y4.z, s4.w - y4.w));
          }
          st4(a.out + c * g.V + gi[it], y4);
        }
      }
    }
  } else {  // kCompose(Bf16): u_new = w + u_old(x + w), optional warped image
#pragma unroll
    for (int it = 0; it < MI; ++it) {
      const int idx = threadIdx.x + it * nthr;
      if (idx < nitems) {
        int yy, x4;
        run_of(idx, q4, xd, yy, x4);
        float4 un[3], iw;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float w0 = f4get(yv[it][0], e), w1 = f4get(yv[it][1], e), w2 = f4get(yv[it][2], e);
          float u0 = w0, u1 = w1, u2 = w2;
          if (a.u_old) {  // null: the previous displacement is zero
            const Tap t = make_tap(4 * x4 + e, tile_row(xd, by, yy), z, w0, w1, w2, g);
            u0 += sample(a.u_old, t);
            u1 += sample(a.u_old + g.V, t);
            u2 += sample(a.u_old + 2 * g.V, t);
          }
          f4set(un[0], e, u0);
          f4set(un[1], e, u1);
          f4set(un[2], e, u2);
          if (a.iw_out) {
            const Tap t2 = make_tap(4 * x4 + e, tile_row(xd, by, yy), z, u0, u1, u2, g);
            if constexpr (MODE == kComposeBf16) f4set(iw, e, sample(a.img_bf16, t2));
            else f4set(iw, e, sample(a.img, t2));
          }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          st4(a.out + c * g.V + gi[it], un[c]);
          if (a.vel_out) st4(a.vel_out + c * g.V + gi[it], yv[it][c]);
        }
        if (a.iw_out) st4(a.iw_out + gi[it], iw);
      }
    }
  }
}

template <int MODE, int NX, bool YS = false>
__global__ void __launch_bounds__(kXlMaxThreads) k_pass_c(Geo g, FftPlan px, XDivs xd, int ls,
                                                const float2* __restrict__ twx, PassCArgs a) {
  pass_c_body<MODE, NX, YS>(g, px, xd, ls, twx, a, Blk::of_block());
}

static hipError_t launch_pass_c_rows(const Geo& g, const FftPlan& px, const Tables& t, PassCMode mode,
                                     const PassCArgs& a, hipStream_t st, int batch, int yb) {
  const dim3 grid(g.ny / yb, g.nz, batch), block(xline_threads_rows(g, yb));
  const size_t lds = pass_a_lds_rows(g, yb);
  const XDivs xd = make_xdivs_rows(g, yb);
  const int ls = xline_stride(g.nx);
  PassCArgs at = a;
  at.twy = t.twy;
#define NADMM_PASS_C(M, N) \
  hipLaunchKernelGGL((k_pass_c<M, N>), grid, block, lds, st, g, px, xd, ls, t.twx, at)
#define NADMM_PASS_C_NX(M)                 \
  if (ysplit(g)) {                         \
    if (g.nx == 192)                       \
      hipLaunchKernelGGL((k_pass_c<M, 192, true>), grid, block, lds, st, g, px, xd, ls, t.twx, at); \
    else                                   \
      hipLaunchKernelGGL((k_pass_c<M, 0, true>), grid, block, lds, st, g, px, xd, ls, t.twx, at);   \
    break;                                 \
  }                                        \
  switch (g.nx) {                          \
    case 32: NADMM_PASS_C(M, 32); break;   \
    case 64: NADMM_PASS_C(M, 64); break;   \
    case 96: NADMM_PASS_C(M, 96); break;   \
    case 128: NADMM_PASS_C(M, 128); break; \
    case 192: NADMM_PASS_C(M, 192); break; \
    default: NADMM_PASS_C(M, 0); break;    \
  }
  switch (mode) {
    case kOutY: NADMM_PASS_C_NX(kOutY); break;
    case kIterFwd: NADMM_PASS_C_NX(kIterFwd); break;
    case kIterFwdIw: NADMM_PASS_C_NX(kIterFwdIw); break;
    case kIterFwdIwChk: NADMM_PASS_C_NX(kIterFwdIwChk); break;
    case kDotY: NADMM_PASS_C_NX(kDotY); break;
    case kAdjY: NADMM_PASS_C_NX(kAdjY); break;
    case kAdjStep: NADMM_PASS_C_NX(kAdjStep); break;
    case kFinalWB: NADMM_PASS_C_NX(kFinalWB); break;
    case kComposeBf16: NADMM_PASS_C_NX(kComposeBf16); break;
    default: NADMM_PASS_C_NX(kCompose); break;
  }
#undef NADMM_PASS_C_NX
#undef NADMM_PASS_C
  return hipGetLastError();
}

hipError_t launch_pass_c(const Geo& g, const FftPlan& px, const Tables& t, PassCMode mode,
                         const PassCArgs& a, hipStream_t st, int batch) {
  // the composition pass has rows of its own (tuned separately)
  const int yb = (mode == kCompose || mode == kComposeBf16) ? xline_rows_compose(g) : xline_rows(g);
  return launch_pass_c_rows(g, px, t, mode, a, st, batch, yb);
}

int pass_c_blocks(const Geo& g) { return g.ny / xline_rows(g) * g.nz; }
int pass_c_blocks_max(const Geo& g) { return g.ny / 2 * g.nz; }  // rows are even

hipError_t launch_pass_c_dot(const Geo& g, const FftPlan& px, const Tables& t, const PassCArgs& a,
                             hipStream_t st, int cap_blocks, int* blocks) {
  const int yb = xline_rows(g), nb = g.ny / yb * g.nz;  // the rows read once for both
  *blocks = 0;
  if (nb > cap_blocks || !a.chk_part || !a.s1) return hipErrorInvalidValue;
  *blocks = nb;
  return launch_pass_c_rows(g, px, t, kDotY, a, st, 1, yb);
}

hipError_t launch_pass_c_chk(const Geo& g, const FftPlan& px, const Tables& t, const PassCArgs& a,
                             hipStream_t st, int cap_blocks, int* blocks) {
  const int yb = xline_rows(g), nb = g.ny / yb * g.nz;  // the rows read once for both
  *blocks = nb <= cap_blocks && a.chk_part ? nb : 0;
  return launch_pass_c_rows(g, px, t, *blocks ? kIterFwdIwChk : kIterFwdIw, a, st, 1, yb);
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

int jacobian_blocks(const Geo& g) {
  const int nb = (g.V + 255) / 256;
  return nb > kJacBlocks ? kJacBlocks : nb;
}

hipError_t launch_jacobian(const Geo& g, const float* disp, float* det, double* partial,
                           double* stats, int64_t* n_nonpos, hipStream_t st) {
  const int nb = jacobian_blocks(g);
  JacAcc* part = reinterpret_cast<JacAcc*>(partial);
  hipLaunchKernelGGL(k_jac_partial, dim3(nb), dim3(256), 0, st, g, disp, det, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_jac_final, dim3(1), dim3(256), 0, st, nb, g.V, part, stats, n_nonpos);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// mixed-size launches: one launch per phase over pairs of several sizes
// ---------------------------------------------------------------------------
bool mixed_class_ok(const Geo& g) {
  const auto x_ok = [](int n) { return n == 64 || n == 96 || n == 128 || n == 192; };
  const auto yz_ok = [](int n) { return n == 32 || n == 64 || n == 96 || n == 128; };
  return x_ok(g.nx) && yz_ok(g.ny) && yz_ok(g.nz) && launch_shape_ok(g) && plane_fits(g);
}
int xline_stride_of(int nx) { return xline_stride(nx); }

void mixed_shapes(MixedLaunch& m) {
  MixedDesc& d = m.d;
  // x-line launch: the threads of the class that needs most (each with its
  // tuned rows); every other class then takes the rows (an even divisor of ny
  // within the kernels' bounds) whose workgroup needs the threads closest to
  // that number from below, so that few threads idle (results do not depend
  // on the rows)
  m.xthreads = 64;
  int waves = 1;
  for (int c = 0; c < d.nclasses; ++c) {
    const Geo& g = d.c[c].g;
    const int xth = xline_threads(g), pw = plane_team_threads(g) / 64;
    if (xth > m.xthreads) m.xthreads = xth;
    if (pw > waves) waves = pw;
  }
  m.xlds = 0;
  int xt = 0;
  for (int c = 0; c < d.nclasses; ++c) {
    MixedClass& k = d.c[c];
    const Geo& g = k.g;
    int rows = xline_rows(g), best = xline_threads_rows(g, rows);
    for (int r = 2; r <= 32; r += 2) {  // the autotuner's range
      const int t = xline_threads_rows(g, r);
      if (t <= m.xthreads && t > best && xline_rows_fit(g, r, m.xthreads)) {
        best = t;
        rows = r;
      }
    }
    const size_t xl = pass_a_lds_rows(g, rows);
    if (xl > m.xlds) m.xlds = xl;
    k.xd = make_xdivs_rows(g, rows);
    k.ls = xline_stride(g.nx);
    k.rs = plane_row_stride(g);
    k.nby = g.ny / rows;
    k.xtiles = k.nby * g.nz;
    k.xtile0 = xt;
    xt += k.xtiles * k.npairs;
  }
  d.xtiles = xt;
  // plane launch: `waves` wavefronts per workgroup (the largest class's need
  // rounded up to a power of two, so that smaller classes' planes can share a
  // workgroup), split into the largest number of equal groups that each hold
  // a class's plane (its wavefronts and LDS)
  int w2 = 1;
  while (w2 < waves) w2 *= 2;
  if (d.nclasses > 1) waves = w2 > 16 ? 16 : w2;  // measured: a little faster with several classes
  m.pthreads = 64 * waves;
  m.plds = 0;
  int pt = 0;
  for (int c = 0; c < d.nclasses; ++c) {
    MixedClass& k = d.c[c];
    const int need = plane_team_threads(k.g) / 64;
    const size_t lds1 = (pass_b_lds(k.g) + 15) / 16 * 16;
    int grp = 1;
    for (int gcount = waves; gcount >= 1; --gcount)
      if (waves % gcount == 0 && waves / gcount >= need && gcount * lds1 <= (size_t)kMaxLds) {
        grp = gcount;
        break;
      }
    k.pplanes = 3 * (k.g.nx / 2 + 1);
    k.pgroup = grp;
    k.psub = m.pthreads / grp;
    k.plds = (int)lds1;
    k.ptile0 = pt;
    pt += (k.npairs * k.pplanes + grp - 1) / grp;
    if (grp * lds1 > m.plds) m.plds = grp * lds1;
  }
  d.ptiles = pt;
}

// The class of workgroup l of an x-line (plane = false) or plane launch:
// classes are numbered in the order of their first workgroups.
__device__ __forceinline__ int mixed_class_of(const MixedDesc& md, int l, bool plane) {
  int c = 0;
#pragma unroll
  for (int k = 1; k < kMaxClasses; ++k)
    if (k < md.nclasses && l >= (plane ? md.c[k].ptile0 : md.c[k].xtile0)) c = k;
  return c;
}

template <typename P>
__device__ __forceinline__ P* off_by(P* p, int64_t o) {
  return p ? p + o : p;
}

// Decodes an x-line workgroup of a mixed launch: class, pair index within the
// class and the tile within the pair.  Within each class (a contiguous range
// of workgroups, dispatched round-robin over the XCDs) the workgroups are
// reordered so that each XCD gets one contiguous range of (pair, tile), as
// in the one-size launches; every class is spread over all XCDs, whose work
// then stays balanced although tiles of different classes differ in size.
struct MixedTile {
  int cls, pair;
  Blk bk;
};
__device__ __forceinline__ MixedTile mixed_xline_tile(const MixedDesc& md) {
  const int l = blockIdx.x;
  MixedTile t;
  t.cls = mixed_class_of(md, l, false);
  const MixedClass& mc = md.c[t.cls];
  const int n = mc.xtiles * mc.npairs;
  int local = l - mc.xtile0;
  if ((n & 7) == 0 && (mc.xtile0 & 7) == 0) local = (local & 7) * (n >> 3) + (local >> 3);
  t.pair = local / mc.xtiles;
  t.bk = Blk{local - t.pair * mc.xtiles, 0, 0, mc.nby, mc.g.nz, false};
  return t;
}

__global__ void k_mixed_tables(const MixedDesc md) {
  const MixedClass& mc = md.c[blockIdx.y];
  tables_body(mc.g, mc.tab, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kXlMaxThreads) k_mixed_pass_a0(const MixedDesc md, const float* __restrict__ iw,
                                                       const float* __restrict__ ref, float* __restrict__ r,
                                                       float* __restrict__ s0, float theta, float eps,
                                                       int data_term, float2* __restrict__ X) {
  const MixedTile t = mixed_xline_tile(md);
  const MixedClass& mc = md.c[t.cls];
  const Geo g = mc.g;
  const XDivs xd = mc.xd;
  const FftPlan px{};  // the compile-time x plans need none
  const int64_t o1 = mc.o1 + (int64_t)t.pair * g.V;
  iw += o1;
  ref += o1;
  r += o1;
  s0 += 3 * o1;
  X += mc.os + (int64_t)t.pair * (int64_t)spectrum_elems(g);
#define NADMM_MIXED_A0(N)                                                                                \
  case N:                                                                                                \
    pass_a0_body<N, float>(g, px, xd, mc.ls, mc.tab.twx, mc.tab.twy, iw, ref, r, s0, theta, eps, data_term, X, t.bk); \
    break;
  switch (g.nx) {
    NADMM_MIXED_A0(64) NADMM_MIXED_A0(96) NADMM_MIXED_A0(128) NADMM_MIXED_A0(192)
  }
#undef NADMM_MIXED_A0
}

template <int MODE>
__global__ void __launch_bounds__(kXlMaxThreads) k_mixed_pass_c(const MixedDesc md, PassCArgs a) {
  const MixedTile t = mixed_xline_tile(md);
  const MixedClass& mc = md.c[t.cls];
  const Geo g = mc.g;
  const XDivs xd = mc.xd;
  const FftPlan px{};
  const int64_t o1 = mc.o1 + (int64_t)t.pair * g.V, o3 = 3 * o1;
  a.X = off_by(a.X, mc.os + (int64_t)t.pair * (int64_t)spectrum_elems(g));
  a.s1 = off_by(a.s1, o3);
  a.s2 = off_by(a.s2, o3);
  a.J = off_by(a.J, o3);
  a.iw = off_by(a.iw, o1);
  a.r = off_by(a.r, o1);
  a.out = off_by(a.out, o3);
  a.v_out = off_by(a.v_out, o3);
  a.b_out = off_by(a.b_out, o3);
  a.u_old = off_by(a.u_old, o3);
  a.img = off_by(a.img, o1);
  a.img_bf16 = off_by(a.img_bf16, o1);
  a.iw_out = off_by(a.iw_out, o1);
  a.vel_out = off_by(a.vel_out, o3);
#define NADMM_MIXED_C(N)                                              \
  case N:                                                             \
    pass_c_body<MODE, N>(g, px, xd, mc.ls, mc.tab.twx, a, t.bk);      \
    break;
  switch (g.nx) {
    NADMM_MIXED_C(64) NADMM_MIXED_C(96) NADMM_MIXED_C(128) NADMM_MIXED_C(192)
  }
#undef NADMM_MIXED_C
}

__global__ void __launch_bounds__(1024) k_mixed_pass_b(const MixedDesc md, float2* __restrict__ X,
                                                       float lambda, float theta, int order) {
  extern __shared__ float2 lds[];
  const int l = blockIdx.x;
  const MixedClass& mc = md.c[mixed_class_of(md, l, true)];
  const Geo g = mc.g;
  const XDivs xd = mc.xd;
  const Tables tab = mc.tab;
  // planes pgroup * (l - ptile0) ... of the class, one per thread group; a
  // group past the class's last plane repeats that plane (the same reads
  // before the first barrier and the same values written after the last)
  const int sub = threadIdx.x / mc.psub, tid = threadIdx.x - sub * mc.psub;
  const int total = mc.npairs * mc.pplanes;
  int q = (l - mc.ptile0) * mc.pgroup + sub;
  if (q >= total) q = total - 1;
  const int j = q / mc.pplanes, tl = q - j * mc.pplanes;
  const int np = g.nx / 2 + 1, c = tl / np;
  const Blk bk{tl - c * np, c, 0, 0, 0, false};
  X += mc.os + (int64_t)j * (int64_t)spectrum_elems(g);
  float2* mine = lds + (size_t)sub * (mc.plds / sizeof(float2));
  const TeamPlan none{};  // the compile-time plane plans need none
#define NADMM_MIXED_B(NY_, NZ_)                                                                          \
  case (NY_ << 16) | NZ_:                                                                                \
    pass_b_body<NY_, NZ_>(g, none, none, none, xd, mc.rs, tab, X, lambda, theta, order, bk, tid, mc.psub, \
                          mine);                                                                         \
    break;
  switch ((g.ny << 16) | g.nz) {
    NADMM_MIXED_B(32, 32) NADMM_MIXED_B(32, 64) NADMM_MIXED_B(32, 96) NADMM_MIXED_B(32, 128)
    NADMM_MIXED_B(64, 32) NADMM_MIXED_B(64, 64) NADMM_MIXED_B(64, 96) NADMM_MIXED_B(64, 128)
    NADMM_MIXED_B(96, 32) NADMM_MIXED_B(96, 64) NADMM_MIXED_B(96, 96) NADMM_MIXED_B(96, 128)
    NADMM_MIXED_B(128, 32) NADMM_MIXED_B(128, 64) NADMM_MIXED_B(128, 96) NADMM_MIXED_B(128, 128)
  }
#undef NADMM_MIXED_B
}

hipError_t launch_mixed_tables(const MixedLaunch& m, hipStream_t st) {
  hipLaunchKernelGGL(k_mixed_tables, dim3(4, m.d.nclasses), dim3(256), 0, st, m.d);
  return hipGetLastError();
}

hipError_t launch_mixed_pass_a0(const MixedLaunch& m, const float* iw, const float* ref, float* r,
                                float* s0, float theta, float eps, int data_term, float2* X,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_mixed_pass_a0, dim3(m.d.xtiles), dim3(m.xthreads), m.xlds, st, m.d, iw, ref, r, s0,
                     theta, eps, data_term, X);
  return hipGetLastError();
}

hipError_t launch_mixed_pass_b(const MixedLaunch& m, float2* X, float lambda, float theta, int order,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_mixed_pass_b, dim3(m.d.ptiles), dim3(m.pthreads), m.plds, st, m.d, X, lambda, theta,
                     order);
  return hipGetLastError();
}

hipError_t launch_mixed_pass_c(const MixedLaunch& m, PassCMode mode, const PassCArgs& a,
                               hipStream_t st) {
  if (mode == kIterFwdIw)
    hipLaunchKernelGGL(k_mixed_pass_c<kIterFwdIw>, dim3(m.d.xtiles), dim3(m.xthreads), m.xlds, st, m.d, a);
  else if (mode == kCompose)
    hipLaunchKernelGGL(k_mixed_pass_c<kCompose>, dim3(m.d.xtiles), dim3(m.xthreads), m.xlds, st, m.d, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace nadmm
