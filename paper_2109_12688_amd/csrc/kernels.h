// Internal launch interface of the gfx950 kernels (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_lds.h"

namespace nadmm {

struct Geo {
  int nx, ny, nz;
  int V;  // nx * ny * nz
};

// Rows of the y axis handled by one x-line workgroup (even, divides ny):
// the value set for these sizes by xline_rows_set (the autotuner; 0 clears
// it), else a default.  Results do not depend on it.
int xline_rows(const Geo& g);
int xline_rows_default(const Geo& g);
void xline_rows_set(const Geo& g, int rows);
int xline_rows_tuned(const Geo& g);  // the value set for these sizes, 0 if none
// Rows of the composition pass (tuned separately; else xline_rows), and
// the wavefronts of a y-z plane workgroup (0 restores the default: what the
// team plans need).  Results do not depend on either.
int xline_rows_compose(const Geo& g);
void xline_rows_compose_set(const Geo& g, int rows);
void plane_waves_set(const Geo& g, int waves);
int plane_waves_needed(const Geo& g);
int plane_threads_tuned(const Geo& g);  // threads of a y-z plane workgroup
// Threads of an x-line workgroup of `rows` rows, and whether those rows fit
// the x-line kernels' per-thread bounds at `threads` threads.
int xline_threads_rows(const Geo& g, int rows);
bool xline_rows_fit(const Geo& g, int rows, int threads);
// Threads of the x-line passes and of the y-z plane pass for these sizes.
int xline_threads(const Geo& g);
int plane_threads(const Geo& g);
// Elements-per-thread bound every LDS FFT stage is compiled for: the host
// sizes workgroups for 8 points per thread, and a bound of 8 leaves no unused
// butterfly slot in the radix-8 stages (measured at 128x128x96: fused x-line
// pass 18.95 -> 18.84 us against a bound of 16; every supported size keeps a
// launch shape).
constexpr int kEpt = 8;
constexpr int kJacBlocks = 1024;
constexpr int kMaxLds = 160 * 1024 - 1024;  // dynamic LDS budget of a workgroup (static use reserved)

FftPlan make_plan(int n);
// Points per lane bound of the wave-team FFTs, and their planner: the team
// size L <= max_lanes (lanes per line, a power of two) and radices with
// L | n / R for every stage, fewest stages first, larger L on ties.
TeamPlan make_team_plan(int n, int max_lanes);
TeamPlan reverse_team_plan(const TeamPlan& p);
size_t plane_lds_bytes(const Geo& g, int rs);
TeamPlan plane_plan_y(const Geo& g);
TeamPlan plane_plan_z(const Geo& g);
int plane_row_stride(const Geo& g);

// Host-precomputed divisors of the x-line and y-z plane index maps.
struct XDivs {
  FastDiv q4;     // nx / 4 (float4 groups per row)
  FastDiv yb;     // rows per x-line workgroup
  FastDiv yb2;    // row pairs per workgroup
  FastDiv nh;     // nx / 2 (packed half-spectrum length)
  FastDiv lines;  // complex lines per x-line workgroup: 3 * yb / 2
  FastDiv ny, nz;
  // Rows of a tile: ygrp consecutive rows, or (half-plane y-z pass, yhalf =
  // ny / 2 > 0) two groups of ygrp = rows / 2 rows yhalf apart; yq = row
  // pairs per group.
  int ygrp, yhalf;
  FastDiv yq;
};
XDivs make_xdivs(const Geo& g);
// True when a y-z plane of the half spectrum fits one workgroup's LDS (pass B
// in one launch); otherwise pass B runs as three launches (rows, columns, rows).
bool plane_fits(const Geo& g);
// True when a y-z plane does not fit one workgroup but its two halves of
// ny / 2 x nz do: the x-line passes then take a radix-2 step of the y
// transform (tiles of two row groups ny / 2 apart; the half spectrum stored
// as two sub-planes per plane, the even and the odd y frequencies) and
// pass B transforms each sub-plane in one workgroup.
bool ysplit(const Geo& g);
// True when every kernel's compile-time per-thread bounds hold for these sizes.
bool launch_shape_ok(const Geo& g);
// Per-thread item bounds the batched loads are compiled for (checked on the host).
constexpr int kXItems = 4;   // float4 groups per thread in the x-line passes
// threads of an x-line workgroup at most: the launch bound the x-line kernels
// are compiled for (a launch with more threads is outside what the compiler
// assumed for them)
constexpr int kXlMaxThreads = 768;
// float4 (two complex) per thread and batch in the plane pass's row loads;
// a wavefront's rows of 128 points arrive in two batches of 4 (measured at
// 128x128x96: 7.10 ms per registration against 7.16 with one batch of 8,
// 7.15 with 6, 7.20 with 3 or 2)
constexpr int kPItems = 4;

// Transform tables, generated once per call into the workspace in float64
// and rounded once: tw* = exp(-2 pi i k / n), s* = 2 - 2 cos(2 pi k / n)
// = 4 sin^2(pi k / n) (the pieces of the Laplacian symbol; sx for k <= nx/2).
struct Tables {
  float2* twx;
  float2* twy;
  float2* twz;
  float* sx;
  float* sy;
  float* sz;
};
size_t tables_bytes(const Geo& g);
Tables tables_at(const Geo& g, void* base);
hipError_t launch_tables(const Geo& g, const Tables& t, hipStream_t st);

// Pass C (inverse x transform + pointwise update) output modes.
// kIterFwd: the data step and s^k, followed on the same x-lines by pass A of
// the next solve (t' = s^k + gamma_next (s^k - s^{k-1}) transformed along x
// and written back over the spectrum the pass read).
// kComposeBf16 is kCompose with the moving image stored as bfloat16.
// kIterFwdIw is kIterFwd with J recomputed from the warped source iw (the
// periodic central differences of k_grad_resid) instead of read.
// kIterFwdIwChk is kIterFwdIw that also writes, for each workgroup, the FP64
// sums of |s^k - s^{k-1}|^2 and |s^k|^2 over its voxels (the relative change
// that threshold stopping of the ADMM loop compares, Sec. 4) to chk_part.
// kDotY stores no y: each workgroup writes the FP64 sum of y . s1 over its
// voxels (three components) to chk_part (a dot product with the output of
// the solve, as the gradient's d/dlambda terms take it).
// kAdjY (the gradient's reverse pass) stores no y: with gt = s1 + y it sets
// out = out + (1 + gamma) gt, b_out = b_out - gamma gt (b_out nullable) and
// v_out = 0 (nullable), per voxel and component.
// kAdjStep (the gradient's reverse pass) is the adjoint of one forward step
// at y = S t (t = s1 + gamma (s1 - s2), s2 nullable; J, r, theta the data
// term): from gs = dL/ds^k it stores gy = 2 ga - gs and gt = gs - ga
// (ga = gs - (J.gs / q) J, q = theta + |J|^2), adds the data term's adjoints
// into gJ and gr, and transforms gy along x into the spectrum it read.
enum PassCMode {
  kOutY = 0, kIterFwd = 1, kFinalWB = 2, kCompose = 3, kComposeBf16 = 4, kIterFwdIw = 5,
  kIterFwdIwChk = 6, kDotY = 7, kAdjY = 8, kAdjStep = 9
};

struct PassCArgs {
  float2* X;         // read; kIterFwd also writes the next half spectrum here
  const float* s1;   // s^{k-1} (iteration), s (final)
  const float* s2;   // s^{k-2} or nullptr when gamma = 0
  float gamma;
  float gamma_next;  // kIterFwd: extrapolation weight of the next solve's input
  const float* J;    // kIterFwd
  const float* iw;   // kIterFwdIw: warped source; J = its central differences
  const float* r;
  float theta;
  float eps;
  int data_term;
  float* out;        // kOutY: y; kIterFwd: s^k (may alias s2); kFinalWB: w; kCompose: new u
  float* v_out;      // kIterFwd: optional v^k
  float* b_out;      // kFinalWB: optional b
  const float* u_old;  // kCompose: displacement before this warping (null: zero)
  const float* img;    // kCompose: moving image
  const uint16_t* img_bf16;  // kComposeBf16: moving image (bfloat16 bit patterns)
  float* iw_out;       // kCompose: optional moving(x + u_new(x))
  float* vel_out;      // kCompose: optional velocity of this warping
  const float2* twy;   // y twiddles (the radix-2 y step of half-plane sizes)
  const float* gs;     // kAdjStep: dL/ds^k
  float* gy;           // kAdjStep outputs
  float* gt;
  float* gJ;           // kAdjStep: accumulated
  float* gr;
  double* chk_part;    // kIterFwdIwChk: (|s^k - s^{k-1}|^2, |s^k|^2) of workgroup b at [2 b], [2 b + 1];
                       // kDotY: y . s1 of workgroup b at [b]
};

hipError_t launch_fill(float* p, float value, size_t n, hipStream_t st);
// *count = number of NaN or infinite values among f[0 .. n) (device int64).
hipError_t launch_count_nonfinite(const float* f, size_t n, int64_t* count, hipStream_t st);
hipError_t launch_scale(const float* in, float* out, float s, size_t n, hipStream_t st);
// Images are float32 or bfloat16 (uint16_t bit patterns, widened exactly to
// float32 on load); every other field is float32.
// `batch` pairs of one size stored back to back (see kernels.hip); the
// warp, gradient and pass launches cover all of them.
hipError_t launch_warp(const Geo& g, const float* img, const float* disp, float* out,
                       hipStream_t st, int batch = 1);
hipError_t launch_warp(const Geo& g, const uint16_t* img, const float* disp, float* out,
                       hipStream_t st, int batch = 1);
// grad (3V, optional), resid (optional, needs ref), s0 (3V, optional: the
// first ADMM iterate v^0 = b^0-free data step from zero, needs ref).
hipError_t launch_grad_resid(const Geo& g, const float* iw, const float* ref, float* grad,
                             float* resid, float* s0, float theta, float eps, int data_term,
                             hipStream_t st, int batch = 1);
hipError_t launch_grad_resid(const Geo& g, const float* iw, const uint16_t* ref, float* grad,
                             float* resid, float* s0, float theta, float eps, int data_term,
                             hipStream_t st, int batch = 1);
hipError_t launch_admm_init(const Geo& g, const float* J, const float* r, float* s0, float* v_out,
                            float theta, float eps, int data_term, hipStream_t st);
// X2 (nullable): a second copy of the spectrum.
hipError_t launch_pass_a(const Geo& g, const FftPlan& px, const Tables& t, const float* s1,
                         const float* s2, float gamma, float2* X, hipStream_t st, int batch = 1,
                         float2* X2 = nullptr);
// Pass A from the data term at the start of a warping: r = iw - ref and
// s^0 (the data step from zero, J = grad iw) stored, s^0 transformed along x.
hipError_t launch_pass_a0(const Geo& g, const FftPlan& px, const Tables& t, const float* iw,
                          const float* ref, float* r, float* s0, float theta, float eps,
                          int data_term, float2* X, hipStream_t st, int batch = 1);
hipError_t launch_pass_a0(const Geo& g, const FftPlan& px, const Tables& t, const float* iw,
                          const uint16_t* ref, float* r, float* s0, float theta, float eps,
                          int data_term, float2* X, hipStream_t st, int batch = 1);
// deriv: multiply by d/dlambda of the w-step multiplier instead of the multiplier.
hipError_t launch_pass_b(const Geo& g, const Tables& t, float2* X, float lambda, float theta,
                         int order, hipStream_t st, int batch = 1, bool deriv = false);
hipError_t launch_pass_c(const Geo& g, const FftPlan& px, const Tables& t, PassCMode mode,
                         const PassCArgs& a, hipStream_t st, int batch = 1);
// One pair's kIterFwdIwChk pass into a.chk_part, which holds cap_blocks
// workgroups' sums: *blocks = the workgroups that wrote theirs.  When the
// launch would need more than cap_blocks workgroups it runs kIterFwdIw
// instead and sets *blocks = 0 (the caller then measures the change apart).
hipError_t launch_pass_c_chk(const Geo& g, const FftPlan& px, const Tables& t, const PassCArgs& a,
                             hipStream_t st, int cap_blocks, int* blocks);
// Workgroups of one pair's x-line iteration pass at the current rows, and
// the most that any rows give.
int pass_c_blocks(const Geo& g);
int pass_c_blocks_max(const Geo& g);
// One pair's kDotY pass (a.s1 the other operand, a.chk_part holding
// cap_blocks doubles): *blocks = the workgroups that wrote their sums, or
// hipErrorInvalidValue (nothing launched) when more would be needed.
hipError_t launch_pass_c_dot(const Geo& g, const FftPlan& px, const Tables& t, const PassCArgs& a,
                             hipStream_t st, int cap_blocks, int* blocks);
hipError_t launch_compose(const Geo& g, const float* u, const float* v, float* out, hipStream_t st);
// Pyramid resampling: coarse (geometry gc) = 2x2x2 average of fine;
// uf (geometry gf) = 2 uc((x - 1/2) / 2), periodic trilinear, per component.
hipError_t launch_downsample2(const Geo& gc, const float* fine, float* coarse, hipStream_t st);
hipError_t launch_upsample2_disp(const Geo& gf, const float* uc, float* uf, hipStream_t st);

// Differentiated warping (adjoint.hip).  Fields are float32 vector fields
// (3V) unless noted; r, gr, resid, d_img are scalar volumes.
hipError_t launch_adj_step(const Geo& g, const float* gs, const float* s1, const float* s2,
                           float gamma, const float* y, const float* J, const float* r,
                           float theta, float* gy, float* gt, float* gJ, float* gr,
                           hipStream_t st);
hipError_t launch_warp_adjoint(const Geo& g, const float* img, const float* ref, const float* w,
                               float* resid, float* d_img, float* gw, hipStream_t st);
hipError_t launch_grad_transpose(const Geo& g, const float* gJ, const float* gr, float* d_img,
                                 hipStream_t st);
// *out (device double) = (accumulate ? *out : 0) + scale * sum a[i] b[i],
// float64, fixed summation order; `partial` holds dot_partials() doubles.
size_t dot_partials();
// *out = (accumulate ? *out : 0) + scale * the sum of partial[0 .. nparts),
// added in one block in an order fixed by nparts.
hipError_t launch_dot_final(const double* partial, int nparts, double scale, bool accumulate, double* out,
                            hipStream_t st);
hipError_t launch_dot(size_t n, const float* a, const float* b, double scale, bool accumulate,
                      double* partial, double* out, hipStream_t st);
// Blocks of the first Jacobian launch; `partial` holds 4 doubles per block
// (min, max, sum, count of det <= 0), every one written before it is read.
int jacobian_blocks(const Geo& g);
hipError_t launch_jacobian(const Geo& g, const float* disp, float* det, double* partial,
                           double* stats, int64_t* n_nonpos, hipStream_t st);

// ---------------------------------------------------------------------------
// Pairs of several sizes in one launch per phase.  A mixed launch covers every
// pair of every size: its workgroups are numbered over (size class, pair,
// tile); each finds its class in the descriptor (a kernel argument) and runs
// the same device code as the one-size launch compiled for that class's
// sizes.  Pairs of one size are consecutive, and every field holds all pairs
// back to back, so a pair's data sits at its class's offset plus its index in
// the class times the per-pair size.
// ---------------------------------------------------------------------------
constexpr int kMaxClasses = 8;
constexpr int kMaxMixedPairs = 4096;
struct MixedClass {
  Geo g;
  XDivs xd;
  int64_t o1, os;      // element offsets of the class's first pair: scalar volumes
                       // (vector fields at 3 o1) and half spectra (complex)
  int ls, rs;          // x-line LDS line stride, y-z plane row stride
  int nby;             // x-line tiles along y per z-slice (ny / rows)
  int xtile0, ptile0;  // first workgroup of the class in x-line and plane launches
  int xtiles;          // x-line workgroups per pair: nby * nz
  int pplanes;         // y-z planes per pair: 3 (nx / 2 + 1)
  int pgroup, psub;    // planes per plane-launch workgroup, and the threads of each
  int plds;            // LDS bytes of one plane's group
  int npairs;
  Tables tab;
};
struct MixedDesc {
  int nclasses;
  int xtiles, ptiles;  // workgroups of an x-line and of a plane launch
  MixedClass c[kMaxClasses];
};
// A mixed batch's descriptor and the launch shapes (threads, LDS) that fit
// every class.
struct MixedLaunch {
  MixedDesc d;
  int xthreads, pthreads;
  size_t xlds, plds;
};
// True when a class of these sizes can take part in a mixed launch: lengths
// with compile-time transforms (nx in {64, 96, 128, 192}, ny and nz in
// {32, 64, 96, 128}) and a y-z plane in one workgroup.
bool mixed_class_ok(const Geo& g);
// Launch shapes of the mixed launches: threads and LDS that fit every class;
// a plane-launch workgroup transforms several planes of a class at once (one
// thread group and LDS region each) when they fit.  Needs the classes' g and
// npairs; sets their plane fields and ptile0 and the totals.
void mixed_shapes(MixedLaunch& m);
hipError_t launch_mixed_tables(const MixedLaunch& m, hipStream_t st);
hipError_t launch_mixed_pass_a0(const MixedLaunch& m, const float* iw, const float* ref, float* r,
                                float* s0, float theta, float eps, int data_term, float2* X,
                                hipStream_t st);
hipError_t launch_mixed_pass_b(const MixedLaunch& m, float2* X, float lambda, float theta, int order,
                               hipStream_t st);
// mode kIterFwdIw or kCompose; the pointers of `a` are the fields' bases.
hipError_t launch_mixed_pass_c(const MixedLaunch& m, PassCMode mode, const PassCArgs& a,
                               hipStream_t st);
int xline_stride_of(int nx);

}  // namespace nadmm
