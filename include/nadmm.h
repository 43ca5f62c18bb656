/*
 * nadmm.h -- C ABI of the MI355X (gfx950) library for Nesterov-accelerated
 * ADMM diffeomorphic registration (Thorley et al., "Nesterov Accelerated ADMM
 * for Fast Diffeomorphic Image Registration").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.   Every array argument is a DEVICE pointer (hipMalloc'd or a torch
 *           CUDA/ROCm tensor's data pointer) unless its comment says "host".
 *           The caller owns every buffer; the library never allocates device
 *           memory.  Buffers must stay alive until the enqueued work has run.
 * Layout.   A scalar volume holds nx*ny*nz float32 values, voxel (x, y, z) at
 *           index x + nx*(y + ny*z) (x fastest; a torch tensor of shape
 *           (nz, ny, nx)).  A vector field holds three such volumes back to
 *           back: component 0 is the x displacement, 1 the y, 2 the z
 *           (torch shape (3, nz, ny, nx)).  Displacements and velocities are in
 *           voxel units.  Deformations are backward (pull): the image warped
 *           by displacement u is I(x + u(x)).  Boundaries are periodic
 *           everywhere (resampling, finite differences and the Fourier solve).
 * Alignment. Every array pointer must be 16-byte aligned.
 * Streams.   `stream` is a hipStream_t passed as void* (NULL = the null
 *           stream).  Every call except nadmm_register_threshold,
 *           nadmm_register_pyramid_threshold, nadmm_register_checked and
 *           nadmm_autotune (which wait for their own results) only enqueues
 *           work on that stream and returns; results are valid after the
 *           caller synchronises it.
 * Threads.  Calls are independent of each other: a call reads only its
 *           arguments, so calls from several host threads on different
 *           streams with separate buffers and workspaces may overlap.  The
 *           only shared state is process-wide and guarded: the launch-shape
 *           tables (nadmm_autotune, nadmm_set_shapes; a change alters speed,
 *           never results), the timing records of nadmm_profile_*, and the
 *           scratch array of nadmm_jacobian_noalloc (see there).
 * Errors.   Every entry point validates all arguments before it enqueues
 *           anything, so a call that returns an error has enqueued nothing.
 *           HIP runtime failures return NADMM_ERR_HIP.  nadmm_last_error()
 *           gives a per-thread message for the last non-OK status.
 * Sizes.    nx must be a multiple of 4 and ny even; every dimension must be 2^a * 3^b with
 *           4 <= n <= 256.  Other sizes return NADMM_ERR_UNSUPPORTED_SIZE.
 *           (y-z spectral planes of up to 16384 points are transformed in
 *           one pass in a compute unit's local memory, larger ones as two
 *           half planes when ny is a multiple of 8 and a half plane fits,
 *           else in three passes; results agree to rounding.)
 */
#ifndef NADMM_H
#define NADMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The entry points declared below are the library's only exported symbols
 * (it is built with hidden visibility for everything else). */
#if defined(__GNUC__) || defined(__clang__)
#pragma GCC visibility push(default)
#endif

#define NADMM_ABI_VERSION 1

typedef enum {
  NADMM_OK = 0,
  NADMM_ERR_INVALID_ARG = 1,      /* null/misaligned pointer, bad parameter value   */
  NADMM_ERR_UNSUPPORTED_SIZE = 2, /* dimensions outside the supported set above      */
  NADMM_ERR_WORKSPACE = 3,        /* workspace missing or smaller than required      */
  NADMM_ERR_HIP = 4,              /* a HIP runtime call failed (message in last_error) */
  NADMM_ERR_NONFINITE = 5,        /* nadmm_register_checked: NaN or infinity in the outputs */
  NADMM_ERR_DIVERGED = 6          /* nadmm_register_checked: an ADMM loop diverged (guard) */
} nadmm_status;

typedef struct {
  int32_t nx, ny, nz;
} nadmm_dims;

/* Model and loop parameters.
 *   lambda     regularisation weight lambda >= 0 of Eq. (2).
 *   theta      ADMM penalty theta > 0 of Eq. (4).
 *   order      regulariser order n, 1 <= n <= 4 (Eq. (2); the w-step divides
 *              by theta + lambda * (2(3 - cos - cos - cos))^n, Sec. 3).
 *   data_term  s of Eq. (2): 2 = squared L2 (Sherman-Morrison v-step),
 *              1 = L1 (clipped v-step, Eq. (6) top).
 *   eps        L1 only: the positive constant in the denominator of z_hat
 *              (Sec. 3, text after Eq. (6)); ignored for data_term = 2.
 *   outer      number of warpings (velocity fields composed, Eq. (1), N = 1).
 *   iters      ADMM iterations per warping (Eq. (5)), >= 1.
 */
typedef struct {
  double lambda;
  double theta;
  int32_t order;
  int32_t data_term;
  double eps;
  int32_t outer;
  int32_t iters;
} nadmm_params;

/* NADMM_ABI_VERSION of the loaded library. */
int nadmm_abi_version(void);

/* Hex SHA-256 (64 characters, static string) of the sources this library
 * was compiled from: the names and contents of the HIP sources and headers
 * of the package's csrc/ directory and of this header, in name order.  A
 * caller can compare it with the sources on disk to detect a stale build. */
const char* nadmm_source_digest(void);

/* Human-readable name of a status code (static string). */
const char* nadmm_status_string(nadmm_status s);

/* Message describing the last non-OK status returned on the calling thread
 * (static per-thread buffer, overwritten by the next failing call). */
const char* nadmm_last_error(void);

/* Size in bytes (written to host *bytes) of the workspace that every entry
 * point below accepts for these dimensions (the fields of the Sec. 2 scheme
 * and of the Sec. 3 iteration: r, the warped source, the two iteration
 * states, the half spectrum of the Eq. (6) w-step, a displacement, the
 * Jacobian partials and the transform tables).  `p` may be NULL (the size
 * does not depend on the parameters).  About 14 float32 values per voxel. */
nadmm_status nadmm_workspace_size(nadmm_dims d, const nadmm_params* p, size_t* bytes);

/* Full registration: the iterative scheme of Sec. 2 with the
 * Nesterov-accelerated ADMM of Sec. 3 (Eq. (5), (6)).
 * For c = 1..outer: warp the ORIGINAL moving image by the current
 * displacement, form the linearised data term (periodic central-difference
 * gradient of the warped image and the residual warped - fixed), run `iters`
 * ADMM iterations from zero (alpha^0 = 1), take the final w iterate as the
 * warping's velocity v_c and compose: u <- v_c + u(x + v_c(x)).
 *   fixed, moving  in, scalar volumes (I0 target, I1 source).
 *   init_disp      in, vector field or NULL (NULL = start from u = 0).
 *   disp           out, vector field: the final displacement u (phi = Id + u).
 *   warped         out, scalar volume or NULL: moving(x + u(x)).
 *   velocities     out, `outer` vector fields back to back, or NULL.
 *   workspace      device scratch of at least nadmm_workspace_size bytes.
 * Outputs must not overlap inputs or each other. */
nadmm_status nadmm_register(nadmm_dims d, const nadmm_params* p,
                            const float* fixed, const float* moving,
                            const float* init_disp, float* disp, float* warped,
                            float* velocities, void* workspace, size_t workspace_bytes,
                            void* stream);

/* nadmm_register with checks of its result, reported as status codes.
 * flags (bit set):
 *   NADMM_CHECK_FINITE      count NaN and infinite values of disp and warped
 *                           on the device; any: NADMM_ERR_NONFINITE.
 *   NADMM_CHECK_DIVERGENCE  the divergence guard of every warping with
 *                           iters >= 3.  Eq. (5) has no restart, and the
 *                           un-restarted momentum can diverge when the data
 *                           term dominates (large |grad I1|, large lambda);
 *                           the paper gives no rule, and this library reads
 *                           divergence as: the fixed-point residual of the
 *                           last iteration exceeds that of the first,
 *                           |s^{K-1} - s^{K-2}| > |s^1 - s^0| (L2 norms over
 *                           the whole field, s^k = v^k + b_hat^k the w-step's
 *                           input, sums in FP64 in a fixed order) or is not
 *                           finite.  Any warping: NADMM_ERR_DIVERGED (when
 *                           the outputs are finite or not checked).
 *   diverged   host out, p->outer int32 or NULL: 1 for each warping whose
 *              guard tripped, else 0.
 * The outputs are written in every case (the registration runs to its fixed
 * counts).  Other arguments, workspace and errors as for nadmm_register (no
 * per-warping velocities).  SYNCHRONOUS: the guard reads two sums per
 * warping back (pinned host memory as for nadmm_register_threshold and two
 * events are allocated for the call) and the call waits for the stream
 * before returning. */
#define NADMM_CHECK_FINITE 1u
#define NADMM_CHECK_DIVERGENCE 2u
nadmm_status nadmm_register_checked(nadmm_dims d, const nadmm_params* p, uint32_t flags,
                                    const float* fixed, const float* moving, const float* init_disp,
                                    float* disp, float* warped, int32_t* diverged, void* workspace,
                                    size_t workspace_bytes, void* stream);

/* nadmm_register with threshold stopping (Sec. 4, second hyper-parameter
 * version: the ADMM loop ends at a convergence threshold, the warping loop
 * once two successive warpings differ by less than a set fraction, 2 % in
 * the paper).  The paper does not define the two measures; this library
 * reads them as relative changes in the L2 norm over the whole field:
 *   - ADMM: after iteration k >= 1, stop once |s^k - s^{k-1}| <= tol_admm |s^k|,
 *     with s^k = v^k + b_hat^k the input of the w-step; the warping's
 *     velocity is then w^k (of that iteration);
 *   - warpings: after warping c >= 1 (0-based), stop once
 *     |u_c - u_{c-1}| <= tol_warp |u_c|.
 * p->iters and p->outer remain the caps.  A negative tolerance switches its
 * check off (that loop runs to its cap); NaN is NADMM_ERR_INVALID_ARG.
 * Sums of squares are accumulated in FP64 from the float32 fields, in an
 * order fixed by the sizes and the launch shapes (nadmm_tuned_shapes).
 *   iters_run    host out, p->outer int32 or NULL: ADMM iterations of each
 *                warping run (0 for warpings not run).
 *   outer_run    host out or NULL: warpings run.
 *   admm_change  host out, p->outer * (p->iters - 1) doubles or NULL: row c
 *                holds warping c's measured changes for k = 1 .. (NaN where
 *                not measured; the last iteration is not measured).
 *   warp_change  host out, p->outer - 1 doubles or NULL: the change of
 *                warping c at index c - 1 (NaN where not measured).
 * Other arguments, the workspace (nadmm_workspace_size bytes) and errors as
 * for nadmm_register (no initial displacement, no per-warping velocities).
 * SYNCHRONOUS: each check's partial sums are written into pinned host
 * memory and added there in order (an ADMM check's by the iteration's own
 * x-line pass, one pair of doubles per workgroup; a warping check's by a
 * pass of its own, at most 1024 pairs); an ADMM check is read while the
 * next iteration already runs (on a stop that iteration is discarded and
 * the result is the one of the stopping iteration), a warping check is
 * waited for.  The call allocates 32 KB of pinned host memory (32 bytes per
 * x-line workgroup of the grid where that is more) and two HIP events for
 * its duration and returns after the work is done. */
nadmm_status nadmm_register_threshold(nadmm_dims d, const nadmm_params* p, double tol_admm,
                                      double tol_warp, const float* fixed, const float* moving,
                                      float* disp, float* warped, int32_t* iters_run,
                                      int32_t* outer_run, double* admm_change, double* warp_change,
                                      void* workspace, size_t workspace_bytes, void* stream);

/* nadmm_register with the two images stored as bfloat16 (each element the
 * upper 16 bits of an IEEE float32, round-to-nearest-even from the float32
 * image being the caller's job).  Image values are widened exactly to
 * float32 where they are read (the warps of the moving image and the
 * residual against the fixed image); the warped image, its gradient, every
 * field and every transform stay float32.  Arguments, layout, workspace and
 * errors as for nadmm_register; `warped` is float32. */
nadmm_status nadmm_register_bf16(nadmm_dims d, const nadmm_params* p,
                                 const uint16_t* fixed, const uint16_t* moving,
                                 const float* init_disp, float* disp, float* warped,
                                 float* velocities, void* workspace, size_t workspace_bytes,
                                 void* stream);

/* Batched registration: `batch` (1..4096) independent pairs of one size
 * and one parameter set, stored back to back in every buffer (pair i's
 * fixed image at fixed + i*V, its displacement at disp + i*3V, ...; init_disp
 * and warped likewise, both may be NULL).  Each launch of the path covers
 * all pairs (the pair is the last grid index), so small volumes fill the
 * GPU and the launch count does not grow with the batch.  Results are those
 * of `batch` separate nadmm_register calls, bit for bit.  The workspace is
 * nadmm_workspace_size_batch bytes; no per-warping velocities.  Errors as
 * for nadmm_register, plus NADMM_ERR_INVALID_ARG for batch out of range.
 * (Pairs of several sizes: one call per size, e.g. on separate streams.) */
nadmm_status nadmm_workspace_size_batch(nadmm_dims d, int32_t batch, size_t* bytes);
nadmm_status nadmm_register_batch(nadmm_dims d, int32_t batch, const nadmm_params* p,
                                  const float* fixed, const float* moving,
                                  const float* init_disp, float* disp, float* warped,
                                  void* workspace, size_t workspace_bytes, void* stream);

/* Registration of pairs of SEVERAL sizes in one call, each launch of the
 * path (Sec. 2 scheme with the Sec. 3 iteration, as nadmm_register from
 * u = 0) covering every pair of every size: its workgroups are numbered over
 * (size class, pair, tile) and each runs the code compiled for its pair's
 * sizes, so there is one launch per phase for the whole batch.
 *   npairs     1..4096 pairs; dims (host array of npairs) gives each pair's
 *              size.  Pairs of one size must be consecutive (at most 8 runs
 *              of sizes, all different), each size with nx in
 *              {64, 96, 128, 192} and ny, nz in {32, 64, 96, 128}
 *              (NADMM_ERR_UNSUPPORTED_SIZE otherwise).
 *   fixed, moving, warped   scalar volumes of every pair back to back in
 *              pair order (pair i at offset V_0 + .. + V_{i-1} floats);
 *              warped may be NULL.
 *   disp       vector fields of every pair back to back (pair i at
 *              3 (V_0 + .. + V_{i-1}) floats).
 *   p          one parameter set for every pair.
 * Results are those of npairs separate nadmm_register calls, bit for bit
 * (each pair's arithmetic is the same; the tile autotuner's choice for a
 * size applies here as well).  Workspace: nadmm_workspace_size_mixed bytes.
 * Asynchronous; the call enqueues kernel launches only (the batch's
 * descriptor travels as a kernel argument), so it can be captured in a
 * graph. */
nadmm_status nadmm_workspace_size_mixed(int32_t npairs, const nadmm_dims* dims, size_t* bytes);
nadmm_status nadmm_register_mixed(int32_t npairs, const nadmm_dims* dims, const nadmm_params* p,
                                  const float* fixed, const float* moving, float* disp, float* warped,
                                  void* workspace, size_t workspace_bytes, void* stream);

/* Multi-resolution registration (Sec. 4: the three-level pyramid of the
 * first hyper-parameter version caps the ADMM iterations at 10, 5, 5 and the
 * warpings at 10, 10, 5, coarsest level first).  Level l of `levels` (1..4,
 * l = 0 the coarsest) has every dimension divided by 2^(levels-1-l), which
 * must divide it and give supported sizes; its images are 2x2x2 averages of
 * the next finer level's.  Each level runs nadmm_register with
 * outer[l] warpings of iters[l] iterations (p->outer / p->iters are
 * ignored; lambda, theta, n and the data term are the same at every level),
 * starting from the previous level's displacement carried to its grid:
 * u_fine(x) = 2 u_coarse((x - 1/2) / 2), periodic trilinear (coarse voxel i
 * covers fine voxels 2i and 2i + 1).  The finest level's displacement goes
 * to disp, its warped image to warped (may be NULL).  Workspace:
 * nadmm_workspace_size_pyramid bytes. */
typedef struct {
  int32_t levels;
  int32_t outer[4];
  int32_t iters[4];
} nadmm_pyramid;
nadmm_status nadmm_workspace_size_pyramid(nadmm_dims d, const nadmm_pyramid* pyr, size_t* bytes);
nadmm_status nadmm_register_pyramid(nadmm_dims d, const nadmm_params* p, const nadmm_pyramid* pyr,
                                    const float* fixed, const float* moving, float* disp,
                                    float* warped, void* workspace, size_t workspace_bytes,
                                    void* stream);

/* The pyramid with threshold stopping at every level (Sec. 4, second
 * hyper-parameter version: the three-level scheme with the ADMM and warping
 * loops ended by thresholds; measures and rules as for
 * nadmm_register_threshold, pyr->outer / pyr->iters being the caps).
 *   iters_run  host out or NULL: sum of pyr->outer[l] int32; level l's
 *              warpings start at index outer[0] + .. + outer[l-1] and hold
 *              the ADMM iterations run (0 for warpings not run).
 *   outer_run  host out or NULL: pyr->levels int32, warpings run per level.
 * Other arguments, workspace and errors as for nadmm_register_pyramid
 * (NaN tolerances: NADMM_ERR_INVALID_ARG).  Synchronous, and allocates
 * pinned host memory (sized for the finest level; a coarser level whose
 * x-line pass has more workgroups than that takes its ADMM checks from a
 * pass of their own) and two events for its duration, as
 * nadmm_register_threshold does. */
nadmm_status nadmm_register_pyramid_threshold(nadmm_dims d, const nadmm_params* p,
                                              const nadmm_pyramid* pyr, double tol_admm,
                                              double tol_warp, const float* fixed,
                                              const float* moving, float* disp, float* warped,
                                              int32_t* iters_run, int32_t* outer_run,
                                              void* workspace, size_t workspace_bytes,
                                              void* stream);

/* Tile autotuner.  Times, with HIP events on `stream` (`reps` = 20 launches
 * each; the call waits for them), every admissible choice of three launch
 * shapes and keeps the fastest of each for all later calls with these dims
 * in this process (process-wide tables; tuning while other threads run the
 * same dims changes only their speed):
 *   - y rows per workgroup of the x-line passes (even divisors of ny up to
 *     32 within the kernels' per-thread bounds), on the fused pass of the
 *     iteration;
 *   - y rows per workgroup of the composition pass (the same range), timed
 *     with a previous displacement of half a voxel everywhere;
 *   - wavefronts per y-z plane workgroup, from what the plane's transform
 *     teams need up to 16 (planes that fit one workgroup).
 * Results of every entry point are bit for bit the same for any choice.
 * `workspace` (nadmm_workspace_size_batch(d, batch) bytes) is scratch; the
 * chosen x-line rows go to host *rows (may be NULL).  Not for use inside
 * stream capture.  With the environment variable NADMM_AUTOTUNE_LOG set,
 * every candidate's mean time per launch is written to stderr. */
nadmm_status nadmm_autotune(nadmm_dims d, int32_t batch, const nadmm_params* p, void* workspace,
                            size_t workspace_bytes, void* stream, int32_t* rows);

/* The launch shapes in use for these dims (host shapes[3]): x-line rows,
 * composition-pass rows, threads per y-z plane workgroup (0 when the planes
 * do not fit one workgroup: half planes or three launches). */
nadmm_status nadmm_tuned_shapes(nadmm_dims d, int32_t* shapes);

/* Sets the three launch shapes of nadmm_tuned_shapes for these dims without
 * timing anything (host shapes[3]: x-line rows, composition-pass rows,
 * threads per y-z plane workgroup; 0 restores a shape's default), e.g. the
 * values an earlier nadmm_autotune chose, so that runs (and profiles) use
 * the same shapes.  Rows must be even divisors of ny up to 32 within the
 * kernels' per-thread bounds; plane threads a multiple of 64 from what the
 * plane's transform teams need to 1024, and only for dims whose planes fit
 * one workgroup.  Invalid values: NADMM_ERR_INVALID_ARG and nothing
 * changes.  The same process-wide tables as nadmm_autotune; results are bit
 * for bit the same for any valid shapes. */
nadmm_status nadmm_set_shapes(nadmm_dims d, const int32_t* shapes);

/* Gradient of one warping's image match (the differentiated hot path):
 *   L = sum_x (I1(x + w(x)) - I0(x))^2,
 * with w the velocity of ONE warping from u = 0 (Sec. 2): `p->iters`
 * iterations of Eq. (5) with the L2 data step of Eq. (6) for J = grad I1,
 * r = I1 - I0 (p->outer is ignored; data_term must be 2).  Writes the loss
 * and dL/dlambda to device doubles *loss and *d_lambda, and dL/dI1 to the
 * device scalar volume d_moving, by reverse-mode differentiation through
 * the unrolled iterations (the Fourier solve is self-adjoint; its lambda
 * derivative is the multiplier -theta K^n / (theta + lambda K^n)^2).  The
 * iteration states are stored every `checkpoint` (1..30) iterations and
 * recomputed in between.  The image adjoint of the final warp is a
 * scatter-add with float atomics, so d_moving may differ in the last bits
 * between runs.  d_moving and d_lambda may both be NULL: then only the loss
 * is computed (the forward iterations, no reverse pass), the same value as
 * with them.  Workspace: nadmm_workspace_size_grad bytes. */
nadmm_status nadmm_workspace_size_grad(nadmm_dims d, const nadmm_params* p, int32_t checkpoint,
                                       size_t* bytes);
nadmm_status nadmm_ssd_grad(nadmm_dims d, const nadmm_params* p, int32_t checkpoint,
                            const float* fixed, const float* moving, double* loss,
                            float* d_moving, double* d_lambda, void* workspace,
                            size_t workspace_bytes, void* stream);

/* One ADMM solve (Eq. (5), (6)) for a given linearised data term:
 * `p->iters` iterations from zero with J = grad I1^w (vector field) and
 * r = I1^w - I0 (scalar volume).  Writes the final iterates w (vector
 * field), b (vector field, may be NULL) and v (vector field, may be NULL).
 * p->outer is ignored. */
nadmm_status nadmm_admm(nadmm_dims d, const nadmm_params* p, const float* J,
                        const float* r, float* w_out, float* b_out, float* v_out,
                        void* workspace, size_t workspace_bytes, void* stream);

/* The Fourier-diagonalised w-step alone (Eq. (6) bottom, read with theta in
 * the numerator): w = F^-1[ theta F(s) / (theta + lambda (2(3 - cos(2 pi p/nx)
 * - cos(2 pi q/ny) - cos(2 pi r/nz)))^n) ] per component.  Uses lambda,
 * theta and order of `p`.  s and w are vector fields (may be the same
 * pointer). */
nadmm_status nadmm_fourier_solve(nadmm_dims d, const nadmm_params* p, const float* s,
                                 float* w, void* workspace, size_t workspace_bytes,
                                 void* stream);

/* Periodic trilinear warp (Sec. 2): out(x) = img(x + disp(x)).  If `grad` is
 * not NULL also writes the periodic central-difference gradient of `out`
 * (vector field); if `resid` is not NULL (requires `ref`) writes
 * out - ref.  `out` must not alias img or disp. */
nadmm_status nadmm_warp(nadmm_dims d, const float* img, const float* disp, const float* ref,
                        float* out, float* grad, float* resid, void* stream);

/* Composition of displacements (Eq. (1)): out(x) = v(x) + u(x + v(x)), the
 * displacement of (Id + u) o (Id + v).  out must not alias u or v. */
nadmm_status nadmm_compose(nadmm_dims d, const float* u, const float* v, float* out,
                           void* stream);

/* Scaling and squaring of a stationary velocity field (the exponential map
 * of the diffeomorphic registration framework the paper builds on, Sec. 1,
 * and of the velocity-field baselines it compares with, Sec. 4): u = vel /
 * 2^steps, then `steps` self-compositions u <- u + u(x + u(x)), each the
 * periodic trilinear composition of Eq. (1).  0 <= steps <= 30.  out must
 * not alias vel. */
nadmm_status nadmm_expmap(nadmm_dims d, const float* vel, int32_t steps, float* out,
                          void* workspace, size_t workspace_bytes, void* stream);

/* Jacobian-determinant check (Sec. 4): det(I + D disp) per voxel with periodic
 * central differences, evaluated and reduced in float64.
 *   det        out, scalar volume or NULL.
 *   stats      out, device double[3]: min, max and mean of the determinant.
 *   n_nonpos   out, device int64[1]: number of voxels with det <= 0.
 * The reduction order is fixed, so results are bitwise reproducible. */
nadmm_status nadmm_jacobian(nadmm_dims d, const float* disp, float* det, double* stats,
                            int64_t* n_nonpos, void* workspace, size_t workspace_bytes,
                            void* stream);

/* nadmm_jacobian without a workspace, for callers that cannot allocate
 * device memory (code under stream capture, serving loops that must not call
 * hipMalloc).  Same arguments, results and errors as nadmm_jacobian, bit for
 * bit; the partial sums of the reduction live in a 32 KB array of device
 * memory inside the library (one per GPU, allocated when the library's code
 * is loaded on that GPU and held until the process ends), so the call
 * allocates nothing.  Every supported size fits that array (the reduction
 * uses at most 1024 blocks); a size that did not would be rejected with
 * NADMM_ERR_UNSUPPORTED_SIZE before anything is enqueued.  All calls on one
 * GPU share the array: calls whose work overlaps in time on the same GPU
 * (different streams or threads without ordering between them) race and
 * give undefined results.  The stream must belong to the current device. */
nadmm_status nadmm_jacobian_noalloc(nadmm_dims d, const float* disp, float* det, double* stats,
                                    int64_t* n_nonpos, void* stream);

/* Output check (not an operation of the paper): the number of NaN or
 * infinite values among `count` volumes stored back to back at `field`
 * (count = 3 for a displacement or velocity field, 1 for an image), written
 * to *nonfinite (device int64).  Lets a caller test a registration's outputs
 * on the device, in stream order, without a host synchronisation inside the
 * library.  1 <= count <= 64; no workspace. */
nadmm_status nadmm_count_nonfinite(nadmm_dims d, const float* field, int32_t count,
                                   int64_t* nonfinite, void* stream);

/* Kernel timing instrumentation, for benchmarks.  While enabled (enable != 0),
 * every kernel the library launches is bracketed by two HIP events recorded
 * on its stream.  Host-side bookkeeping only; no device memory is used.
 * nadmm_profile_read() waits for the recorded events, writes for up to `max`
 * kernel kinds their static name, launch count and summed event-to-event
 * milliseconds since the previous read (host arrays, any may be NULL), clears
 * the records and returns the number of kinds (or -1 on a HIP failure). */
nadmm_status nadmm_profile_enable(int enable);
int nadmm_profile_read(int max, const char** names, int64_t* counts, double* total_ms);

/* Benchmark replay of one kernel of the ADMM iteration: launches it `reps`
 * times back to back (1 <= reps <= 10000) on the buffers that a preceding
 * nadmm_register call with the same dims and params left in `workspace`,
 * between two HIP events on `stream`, waits for them and writes the mean
 * milliseconds per launch to host *avg_ms.  kind: 0 = forward x pass of a
 * warping's first solve, 1 = y-z spectral pass, 2 = the fused x pass of the
 * iteration loop (inverse x transform, data step and new state, extrapolation
 * and forward x transform of the next solve's input; replayed with zero
 * extrapolation weights so that the state stays bounded), 3 = one whole ADMM
 * iteration (kind 2 followed by kind 1; *avg_ms is per iteration).  The
 * replayed launches overwrite the workspace's iteration state. */
nadmm_status nadmm_profile_replay(nadmm_dims d, const nadmm_params* p, int32_t kind, int32_t reps,
                                  void* workspace, size_t workspace_bytes, void* stream,
                                  double* avg_ms);

#if defined(__GNUC__) || defined(__clang__)
#pragma GCC visibility pop
#endif

#ifdef __cplusplus
}
#endif
#endif /* NADMM_H */
