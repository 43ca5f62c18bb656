// C ABI of the registration library: argument validation, workspace layout
// and the host-side loop orchestration (Sec. 2 iterative scheme, Sec. 3
// Eq. (5) recurrence).  All device work is enqueued on the caller's stream;
// nothing here allocates device memory, and only the threshold-stopped
// registration (whose loop counts depend on device results) and the tile
// autotuner synchronise.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <type_traits>
#include <vector>

#include "../../include/nadmm.h"
#include "kernels.h"
#include "reduce.h"

namespace nadmm {
// Sets the calling thread's nadmm_last_error() message and returns s
// (defined in capi.hip, where that message lives).
nadmm_status set_last_error(nadmm_status s, const char* msg);
}  // namespace nadmm

using namespace nadmm;

namespace {

thread_local char g_err[512] = "";

nadmm_status fail(nadmm_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

}  // namespace

nadmm_status nadmm::set_last_error(nadmm_status s, const char* msg) {
  snprintf(g_err, sizeof(g_err), "%s", msg);
  return s;
}

namespace {

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(NADMM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ---- optional per-kernel event timing -----------------------------------
enum KernelKind {
  KK_FILL, KK_SCALE, KK_WARP, KK_GRAD, KK_ADMM_INIT, KK_PASS_A, KK_PASS_B, KK_PASS_C_OUT,
  KK_PASS_CA_ITER, KK_PASS_C_WB, KK_PASS_C_COMPOSE, KK_COMPOSE, KK_JACOBIAN, KK_COUNT
};
const char* const kKindNames[KK_COUNT] = {
    "fill", "scale", "warp", "grad_resid", "admm_init", "pass_a_fwd_x", "pass_b_yz_solve",
    "pass_c_out", "pass_ca_iter", "pass_c_final_wb", "pass_c_compose", "compose", "jacobian"};

struct ProfRecord {
  int kind;
  hipEvent_t start, stop;
};
// Timing instrumentation: process-wide, safe to use from several threads
// (the records and the pool of reusable events are guarded by g_prof_mu).
std::atomic<bool> g_prof{false};
std::mutex g_prof_mu;
std::vector<ProfRecord> g_records;
std::vector<hipEvent_t> g_free_events;

hipEvent_t take_event() {
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_free_events.empty()) {
      hipEvent_t e = g_free_events.back();
      g_free_events.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Runs launch() and, when timing is on, brackets it with events on st.
template <class F>
hipError_t timed(int kind, hipStream_t st, F&& launch) {
  if (!g_prof.load(std::memory_order_relaxed)) return launch();
  ProfRecord r{kind, take_event(), take_event()};
  if (!r.start || !r.stop) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(r.start, st);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(r.stop, st);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_records.push_back(r);
  return hipSuccess;
}

bool fft_length_ok(int n) {
  if (n < 4 || n > 256) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

nadmm_status check_dims(const nadmm_dims& d) {
  if (!fft_length_ok(d.nx) || !fft_length_ok(d.ny) || !fft_length_ok(d.nz))
    return fail(NADMM_ERR_UNSUPPORTED_SIZE,
                "dims (%d, %d, %d): each must be 2^a 3^b in [4, 256]", d.nx, d.ny, d.nz);
  if (d.nx % 4 || d.ny % 2)
    return fail(NADMM_ERR_UNSUPPORTED_SIZE,
                "dims (%d, %d, %d): nx must be a multiple of 4 and ny even", d.nx, d.ny, d.nz);
  if (!launch_shape_ok(Geo{d.nx, d.ny, d.nz, d.nx * d.ny * d.nz}))
    return fail(NADMM_ERR_UNSUPPORTED_SIZE, "dims (%d, %d, %d): no valid launch shape", d.nx,
                d.ny, d.nz);
  return NADMM_OK;
}

nadmm_status check_params(const nadmm_params* p, bool need_outer) {
  if (!p) return fail(NADMM_ERR_INVALID_ARG, "params is NULL");
  if (!(isfinite(p->theta) && p->theta > 0))
    return fail(NADMM_ERR_INVALID_ARG, "theta must be finite and > 0 (got %g)", p->theta);
  if (!(isfinite(p->lambda) && p->lambda >= 0))
    return fail(NADMM_ERR_INVALID_ARG, "lambda must be finite and >= 0 (got %g)", p->lambda);
  if (p->order < 1 || p->order > 4)
    return fail(NADMM_ERR_INVALID_ARG, "order must be in [1, 4] (got %d)", p->order);
  if (p->data_term != 1 && p->data_term != 2)
    return fail(NADMM_ERR_INVALID_ARG, "data_term must be 1 or 2 (got %d)", p->data_term);
  if (p->data_term == 1 && !(isfinite(p->eps) && p->eps > 0))
    return fail(NADMM_ERR_INVALID_ARG, "eps must be finite and > 0 for data_term 1");
  if (p->iters < 1 || p->iters > 100000)
    return fail(NADMM_ERR_INVALID_ARG, "iters must be in [1, 100000] (got %d)", p->iters);
  if (need_outer && (p->outer < 0 || p->outer > 100000))
    return fail(NADMM_ERR_INVALID_ARG, "outer must be in [0, 100000] (got %d)", p->outer);
  return NADMM_OK;
}

nadmm_status check_ptr(const void* p, const char* name, bool nullable) {
  if (!p) return nullable ? NADMM_OK : fail(NADMM_ERR_INVALID_ARG, "%s is NULL", name);
  if (reinterpret_cast<uintptr_t>(p) & 15)
    return fail(NADMM_ERR_INVALID_ARG, "%s is not 16-byte aligned", name);
  return NADMM_OK;
}

#define CHECK(expr)                         \
  do {                                      \
    nadmm_status s_ = (expr);               \
    if (s_ != NADMM_OK) return s_;          \
  } while (0)

// Workspace: 14 float32 fields of V values (each region 256-byte aligned),
// the Jacobian partials and the transform tables (a few KB).
struct Layout {
  size_t r, iw, s1, s2, X, u, jac, tab, total;
};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Per-pair regions hold `batch` pairs back to back; tables and Jacobian
// partials are shared.
Layout layout(const nadmm_dims& d, int batch = 1) {
  const size_t V = (size_t)d.nx * d.ny * d.nz, B = (size_t)batch;
  const size_t f3 = align256(B * 3 * V * sizeof(float)), f1 = align256(B * V * sizeof(float));
  Layout L;
  size_t o = 0;
  L.r = o; o += f1;
  L.iw = o; o += f1;
  L.s1 = o; o += f3;
  L.s2 = o; o += f3;
  L.X = o; o += align256(B * 3 * (d.nx / 2 + 1) * d.ny * d.nz * 2 * sizeof(float));
  L.u = o; o += f3;
  L.jac = o; o += align256(kJacBlocks * 4 * sizeof(double));
  L.tab = o; o += align256(tables_bytes(Geo{d.nx, d.ny, d.nz, d.nx * d.ny * d.nz}));
  L.total = o;
  return L;
}

nadmm_status check_ws(const nadmm_dims& d, void* ws, size_t bytes, int batch = 1) {
  CHECK(check_ptr(ws, "workspace", false));
  const size_t need = layout(d, batch).total;
  if (bytes < need)
    return fail(NADMM_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required",
                bytes, need);
  return NADMM_OK;
}

nadmm_status check_batch(int32_t batch) {
  if (batch < 1 || batch > 4096)
    return fail(NADMM_ERR_INVALID_ARG, "batch must be in [1, 4096] (got %d)", batch);
  return NADMM_OK;
}

Geo geo(const nadmm_dims& d) { return Geo{d.nx, d.ny, d.nz, d.nx * d.ny * d.nz}; }

template <class T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// gamma_k = (alpha^k - 1) / alpha^{k+1}, alpha^0 = 1 (Eq. (5)), float64.
std::vector<double> nesterov_gammas(int n) {
  std::vector<double> g(n > 0 ? n : 0);
  double a = 1.0;
  for (int k = 0; k < n; ++k) {
    const double an = (1.0 + sqrt(1.0 + 4.0 * a * a)) / 2.0;
    g[k] = (a - 1.0) / an;
    a = an;
  }
  return g;
}

struct Plans {
  FftPlan x, y, z;
};

Plans plans(const nadmm_dims& d) { return Plans{make_plan(d.nx), make_plan(d.ny), make_plan(d.nz)}; }

// One application of the w-step operator S to t = s1 + gamma (s1 - s2)
// through passes A and B; pass C (with its mode) is issued by the caller.
hipError_t spectral_ab(const Geo& g, const Plans& pl, const Tables& tb, const nadmm_params* p,
                       const float* s1, const float* s2, float gamma, float2* X, hipStream_t st,
                       int batch = 1, bool deriv = false) {
  hipError_t e = timed(KK_PASS_A, st, [&] {
    return launch_pass_a(g, pl.x, tb, s1, s2, gamma, X, st, batch);
  });
  if (e != hipSuccess) return e;
  return timed(KK_PASS_B, st, [&] {
    return launch_pass_b(g, tb, X, (float)p->lambda, (float)p->theta, p->order, st, batch, deriv);
  });
}

// out = S t (or (dS/dlambda) t) for t = s1 + gamma (s1 - s2), one field.
hipError_t spectral_apply(const Geo& g, const Plans& pl, const Tables& tb, const nadmm_params* p,
                          const float* s1, const float* s2, float gamma, float2* X, float* out,
                          hipStream_t st, bool deriv = false) {
  hipError_t e = spectral_ab(g, pl, tb, p, s1, s2, gamma, X, st, 1, deriv);
  if (e != hipSuccess) return e;
  PassCArgs a{};
  a.X = X;
  a.out = out;
  return timed(KK_PASS_C_OUT, st, [&] { return launch_pass_c(g, pl.x, tb, kOutY, a, st); });
}

// The ADMM loop of one warping in the two-field form, with s^0 already in
// *cur.  Runs iterations k = 1 .. iters-1 (each: pass C of S t^k fused with
// pass A of the next solve's input, then pass B).  On return *cur holds
// s^{iters-1} and X the pass-B output for S s^{iters-1}, ready for the
// warping's final pass C.
// J given, or (J null) recomputed in the fused pass from the warped source iw.
// x_done: the x transform of s^0 is already in X (pass A fused with the
// data term), so the first solve starts at pass B.
// stop (nullable): threshold stopping; the loop may then end early, with X
// holding the pass-B output for S applied to the stopping iterate.
// Threshold stopping (Sec. 4, second hyper-parameter version): a loop stops
// after the first check at which |new - old| <= tol |new| (L2 norms over the
// whole field; the ADMM loop compares its w-step inputs s^k, s^{k-1} from
// k = 1 on, the warping loop the displacements u_c, u_{c-1} from c = 1 on).
// A negative tolerance switches that loop's check off.  A check's per-block
// partial sums are written into pinned host memory behind an event and
// added there in block order; the ADMM loop reads iteration k's check while
// iteration k + 1 already runs (a stop at k then finalises from s^k, which
// iteration k + 1 leaves in place), the warping loop waits for its check.
// The ADMM loop's sums come from the x-line pass that forms s^k (one pair of
// sums per workgroup), so that its check reads no field again; the other
// checks take a pass of their own over the two fields.
struct StopRule {
  double tol_admm, tol_warp;
  double* host;          // pinned host: 2 read-back slots of 2 * slot_blocks doubles
  double* host_dev;      // the same memory as the device addresses it
  int slot_blocks;       // partial sums per slot
  int nb[2];             // blocks of the check in each slot
  hipEvent_t ev[2];      // completion of each slot's partial sums
  double* admm_change;   // host, nullable: outer x (iters - 1) measured changes
  double* warp_change;   // host, nullable: outer - 1 measured changes
  int32_t* iters_run;    // host, nullable: ADMM iterations of each warping
  int outer_run;
  // divergence guard (thresholds off): |s^1 - s^0|^2 into slot 0 and
  // |s^{K-1} - s^{K-2}|^2 into slot 1 of every warping with K >= 3
  bool guard;
  int32_t* diverged;     // host, nullable: 1 for each warping whose guard tripped
  int n_diverged;
};

// Enqueue the partial sums of |a - b|^2 and |a|^2 over n floats, written by
// the kernel into read-back slot `slot`.
nadmm_status change_enqueue(const float* a, const float* b, size_t n, StopRule* stop, int slot,
                            hipStream_t st) {
  stop->nb[slot] = change_blocks(n);
  HIP_TRY(launch_change_partials(a, b, n, stop->host_dev + (size_t)2 * stop->slot_blocks * slot, st));
  HIP_TRY(hipEventRecord(stop->ev[slot], st));
  return NADMM_OK;
}

// Wait for slot `slot` and add its partials in block order: |a - b|^2 and |a|^2.
nadmm_status change_sums(StopRule* stop, int slot, double& d, double& n) {
  HIP_TRY(hipEventSynchronize(stop->ev[slot]));
  const double* part = stop->host + (size_t)2 * stop->slot_blocks * slot;
  d = 0.0;
  n = 0.0;
  for (int j = 0; j < stop->nb[slot]; ++j) {
    d += part[2 * j];
    n += part[2 * j + 1];
  }
  return NADMM_OK;
}

// Wait for slot `slot` and add its partials in block order: |a - b| / |a|
// and whether |a - b| <= tol |a|.
nadmm_status change_read(StopRule* stop, int slot, double tol, double& change, bool& below) {
  HIP_TRY(hipEventSynchronize(stop->ev[slot]));
  const double* part = stop->host + (size_t)2 * stop->slot_blocks * slot;
  double d = 0.0, n = 0.0;
  for (int j = 0; j < stop->nb[slot]; ++j) {
    d += part[2 * j];
    n += part[2 * j + 1];
  }
  change = n > 0 ? sqrt(d / n) : (d == 0 ? 0.0 : INFINITY);
  below = d <= tol * tol * n;
  return NADMM_OK;
}

// Pinned read-back slots and their events, for one threshold-stopped call
// (released when it returns; an early error return may leave a write in
// flight, so the stream is drained first).
struct CheckHost {
  hipStream_t st;
  double* host = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  ~CheckHost() {
    if (host) (void)hipStreamSynchronize(st);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (host) (void)hipHostFree(host);
  }
  // Allocates the slots (each for the larger of a separate check's blocks
  // and the x-line pass's workgroups at geometry g) and the events, and
  // points `stop` at them.
  nadmm_status init(StopRule& stop, const Geo& g) {
    const int xb = pass_c_blocks(g);
    stop.slot_blocks = xb > kChangeBlocks ? xb : kChangeBlocks;
    HIP_TRY(hipHostMalloc((void**)&host, 4 * (size_t)stop.slot_blocks * sizeof(double), hipHostMallocDefault));
    for (hipEvent_t& e : ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    stop.host = host;
    HIP_TRY(hipHostGetDevicePointer((void**)&stop.host_dev, host, 0));
    stop.ev[0] = ev[0];
    stop.ev[1] = ev[1];
    return NADMM_OK;
  }
};

nadmm_status admm_iterations(const Geo& g, const Plans& pl, const Tables& tb,
                             const nadmm_params* p, const float* J, const float* iw,
                             const float* r, float*& cur, float*& prev, float2* X, float* v_last,
                             hipStream_t st, int batch = 1, bool x_done = false,
                             StopRule* stop = nullptr, int warping = 0) {
  const std::vector<double> gam = nesterov_gammas(p->iters);
  if (stop && stop->iters_run) stop->iters_run[warping] = 1;
  if (x_done)
    HIP_TRY(timed(KK_PASS_B, st, [&] {
      return launch_pass_b(g, tb, X, (float)p->lambda, (float)p->theta, p->order, st, batch);
    }));
  else
    HIP_TRY(spectral_ab(g, pl, tb, p, cur, nullptr, 0.0f, X, st, batch));  // gamma_0 = 0: t = s^0
  for (int k = 1; k < p->iters; ++k) {
    PassCArgs a{};
    a.X = X;
    a.s1 = cur;
    a.s2 = (k == 1) ? nullptr : prev;  // s^{-1} is never read
    a.gamma = (float)gam[k - 1];
    a.gamma_next = (k + 1 < p->iters) ? (float)gam[k] : 0.0f;  // the final solve takes s as is
    a.J = J;
    a.iw = iw;
    a.r = r;
    a.theta = (float)p->theta;
    a.eps = (float)p->eps;
    a.data_term = p->data_term;
    a.out = prev;  // s^k overwrites s^{k-2} voxel by voxel
    a.v_out = (k == p->iters - 1) ? v_last : nullptr;
    // the threshold check of iteration k (not the last: it ends the loop
    // anyway) from the pass that forms s^k, when it can hold the sums
    const bool chk = stop && stop->tol_admm >= 0 && !J && batch == 1 && k + 1 < p->iters;
    int chk_blocks = 0;
    if (chk) a.chk_part = stop->host_dev + (size_t)2 * stop->slot_blocks * (k & 1);
    HIP_TRY(timed(KK_PASS_CA_ITER, st, [&] {
      if (chk) return launch_pass_c_chk(g, pl.x, tb, a, st, stop->slot_blocks, &chk_blocks);
      return launch_pass_c(g, pl.x, tb, J ? kIterFwd : kIterFwdIw, a, st, batch);
    }));
    if (chk_blocks > 0) {
      stop->nb[k & 1] = chk_blocks;
      HIP_TRY(hipEventRecord(stop->ev[k & 1], st));
    }
    HIP_TRY(timed(KK_PASS_B, st, [&] {
      return launch_pass_b(g, tb, X, (float)p->lambda, (float)p->theta, p->order, st, batch);
    }));
    float* tmp = cur;
    cur = prev;
    prev = tmp;
    if (stop && stop->iters_run) stop->iters_run[warping] = k + 1;
    if (stop && stop->guard && p->iters >= 3 && (k == 1 || k == p->iters - 1))
      CHECK(change_enqueue(cur, prev, 3 * (size_t)g.V * batch, stop, k == 1 ? 0 : 1, st));
    if (stop && stop->tol_admm >= 0) {
      // check iteration k (unless its x-line pass did), then read the check
      // of iteration k - 1, enqueued one iteration ago
      if (k + 1 < p->iters && chk_blocks == 0)
        CHECK(change_enqueue(cur, prev, 3 * (size_t)g.V, stop, k & 1, st));
      if (k >= 2) {
        double ch;
        bool below;
        CHECK(change_read(stop, (k - 1) & 1, stop->tol_admm, ch, below));
        if (stop->admm_change) stop->admm_change[(size_t)warping * (p->iters - 1) + (k - 2)] = ch;
        if (below) {
          // stop at k - 1: iteration k (and its check) ran ahead; s^{k-1} is
          // in prev, and the solve of pass B took an extrapolated input, so
          // redo it on s^{k-1} itself
          if (stop->iters_run) stop->iters_run[warping] = k;
          HIP_TRY(spectral_ab(g, pl, tb, p, prev, nullptr, 0.0f, X, st, batch));
          return NADMM_OK;
        }
      }
    }
  }
  return NADMM_OK;
}

// The registration of nadmm_register / _bf16 / _batch; T is the image
// element type (float, or uint16_t holding bfloat16 bit patterns); `batch`
// pairs of one size, back to back in every buffer (velocities only for 1).
template <typename T>
nadmm_status register_impl(nadmm_dims d, const nadmm_params* p, const T* fixed, const T* moving,
                           const float* init_disp, float* disp, float* warped, float* velocities,
                           void* workspace, size_t workspace_bytes, void* stream, int batch,
                           StopRule* stop = nullptr) {
  constexpr bool kBf16 = std::is_same<T, uint16_t>::value;
  CHECK(check_dims(d));
  CHECK(check_params(p, true));
  CHECK(check_ptr(fixed, "fixed", false));
  CHECK(check_ptr(moving, "moving", false));
  CHECK(check_ptr(init_disp, "init_disp", true));
  CHECK(check_ptr(disp, "disp", false));
  CHECK(check_ptr(warped, "warped", true));
  CHECK(check_ptr(velocities, "velocities", true));
  CHECK(check_ws(d, workspace, workspace_bytes, batch));
  const Geo g = geo(d);
  const Plans pl = plans(d);
  const Layout L = layout(d, batch);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t V = (size_t)g.V;
  float* r = at<float>(workspace, L.r);
  float* iw = at<float>(workspace, L.iw);
  float* S1 = at<float>(workspace, L.s1);
  float* S2 = at<float>(workspace, L.s2);
  float2* X = at<float2>(workspace, L.X);
  float* U = at<float>(workspace, L.u);
  const Tables tb = tables_at(g, at<char>(workspace, L.tab));
  HIP_TRY(launch_tables(g, tb, st));

  // Displacement buffers alternate between U and disp so that the last
  // warping writes disp.
  auto dst_of = [&](int c) { return ((p->outer - 1 - c) % 2 == 0) ? disp : U; };
  // u_src null: no displacement yet (u = 0).  Then the first warped image is
  // the moving image itself (sampling at the grid points is exact) and the
  // first composition has nothing to gather.
  const float* u_src = init_disp;
  if (p->outer == 0) {
    if (!u_src)
      HIP_TRY(timed(KK_FILL, st, [&] { return launch_fill(disp, 0.0f, 3 * V * batch, st); }));
    else if (u_src != disp)
      HIP_TRY(hipMemcpyAsync(disp, u_src, 3 * V * batch * sizeof(float), hipMemcpyDeviceToDevice, st));
    if (warped) HIP_TRY(timed(KK_WARP, st, [&] { return launch_warp(g, moving, disp, warped, st, batch); }));
    return NADMM_OK;
  }
  const float* iw_first = iw;  // I1^w of the first warping
  if (u_src) {
    HIP_TRY(timed(KK_WARP, st, [&] { return launch_warp(g, moving, u_src, iw, st, batch); }));
  } else if constexpr (kBf16) {
    // widen the bfloat16 image: a warp by the zero field
    float* z = dst_of(0) == disp ? U : disp;
    HIP_TRY(timed(KK_FILL, st, [&] { return launch_fill(z, 0.0f, 3 * V * batch, st); }));
    HIP_TRY(timed(KK_WARP, st, [&] { return launch_warp(g, moving, z, iw, st, batch); }));
  } else {
    iw_first = reinterpret_cast<const float*>(moving);
  }
  for (int c = 0; c < p->outer; ++c) {
    const bool last = (c == p->outer - 1);
    // linearised data term at the current warp, and s^0 (Eq. (6) from zero)
    // r and s^0 only: the iterations recompute J = grad I1^w from iw
    // (fused with the x transform of s^0)
    const float* iw_c = c == 0 ? iw_first : iw;
    HIP_TRY(timed(KK_PASS_A, st, [&] { return launch_pass_a0(g, pl.x, tb, iw_c, fixed, r, S1, (float)p->theta,
                              (float)p->eps, p->data_term, X, st, batch); }));
    float* cur = S1;
    float* prev = S2;
    CHECK(admm_iterations(g, pl, tb, p, nullptr, iw_c, r, cur, prev, X, nullptr, st, batch, true, stop, c));
    // final w = S s^{K-1}, composed onto the displacement
    PassCArgs a{};
    a.X = X;
    a.out = dst_of(c);
    a.u_old = u_src;
    if constexpr (kBf16) a.img_bf16 = moving;
    else a.img = moving;
    a.iw_out = last ? warped : iw;
    a.vel_out = velocities ? velocities + (size_t)c * 3 * V : nullptr;
    HIP_TRY(timed(KK_PASS_C_COMPOSE, st, [&] { return launch_pass_c(g, pl.x, tb, kBf16 ? kComposeBf16 : kCompose, a, st, batch); }));
    if (stop) stop->outer_run = c + 1;
    if (stop && stop->guard && p->iters >= 3) {  // read while the composition runs
      double d0, d1, n0, n1;
      CHECK(change_sums(stop, 0, d0, n0));
      CHECK(change_sums(stop, 1, d1, n1));
      const bool div = !isfinite(d1) || d1 > d0;
      if (stop->diverged) stop->diverged[c] = div ? 1 : 0;
      stop->n_diverged += div ? 1 : 0;
    }
    if (stop && stop->tol_warp >= 0 && c >= 1 && !last) {
      double ch;
      bool below;
      CHECK(change_enqueue(a.out, u_src, 3 * V, stop, 0, st));
      CHECK(change_read(stop, 0, stop->tol_warp, ch, below));
      if (stop->warp_change) stop->warp_change[c - 1] = ch;
      if (below) {
        // the buffers were laid out for `outer` warpings: this one's
        // displacement may be in U and its warped image is in iw
        if (a.out != disp)
          HIP_TRY(hipMemcpyAsync(disp, a.out, 3 * V * sizeof(float), hipMemcpyDeviceToDevice, st));
        if (warped) HIP_TRY(hipMemcpyAsync(warped, iw, V * sizeof(float), hipMemcpyDeviceToDevice, st));
        return NADMM_OK;
      }
    }
    u_src = a.out;
  }
  return NADMM_OK;
}

// ---- differentiated warping ---------------------------------------------
// Workspace of nadmm_ssd_grad: J, r, the spectrum and tables as for a
// registration, then the iteration states (checkpoint pairs and a segment
// buffer), the adjoint ring and temporaries, all float32 vector fields.
struct GradLayout {
  int nseg, nbuf;
  size_t nparts;
  size_t J, r, gr, resid, X, X2, tab, part, f3[64];
  int nf3;
  size_t total;
};

int grad_segments(int iters, int c) { return iters <= 1 ? 0 : (iters - 1 + c - 1) / c; }

GradLayout grad_layout(const nadmm_dims& d, int iters, int c) {
  const size_t V = (size_t)d.nx * d.ny * d.nz;
  const size_t f3 = align256(3 * V * sizeof(float)), f1 = align256(V * sizeof(float));
  GradLayout L{};
  L.nseg = grad_segments(iters, c);
  L.nbuf = c - 1 > 2 ? c - 1 : 2;
  // checkpoints (2 per segment), shared segment/rolling buffers, ring (3),
  // gy, gt, tmp, w, gw, gJ
  L.nf3 = 2 * (L.nseg > 0 ? L.nseg : 1) + L.nbuf + 3 + 6;
  size_t o = 0;
  L.J = o; o += f3;
  L.r = o; o += f1;
  L.gr = o; o += f1;
  L.resid = o; o += f1;
  L.X = o; o += align256((size_t)3 * (d.nx / 2 + 1) * d.ny * d.nz * 2 * sizeof(float));
  L.X2 = o; o += align256((size_t)3 * (d.nx / 2 + 1) * d.ny * d.nz * 2 * sizeof(float));
  L.tab = o; o += align256(tables_bytes(Geo{d.nx, d.ny, d.nz, d.nx * d.ny * d.nz}));
  // dot partials: the dot pass's blocks, or the x-line pass's workgroups
  // at any rows (the d/dlambda terms' sums)
  const size_t xb = (size_t)pass_c_blocks_max(Geo{d.nx, d.ny, d.nz, d.nx * d.ny * d.nz});
  L.nparts = xb > dot_partials() ? xb : dot_partials();
  L.part = o; o += align256(L.nparts * sizeof(double));
  for (int i = 0; i < L.nf3; ++i) {
    L.f3[i] = o;
    o += f3;
  }
  L.total = o;
  return L;
}

nadmm_status check_grad_args(const nadmm_params* p, int32_t checkpoint) {
  CHECK(check_params(p, false));
  if (p->data_term != 2)
    return fail(NADMM_ERR_INVALID_ARG, "the gradient supports the L2 data term (data_term 2) only");
  if (p->iters > 100000) return fail(NADMM_ERR_INVALID_ARG, "iters too large");
  if (checkpoint < 1 || checkpoint > 30)
    return fail(NADMM_ERR_INVALID_ARG, "checkpoint must be in [1, 30] (got %d)", checkpoint);
  if (2 * grad_segments(p->iters, checkpoint) + 12 + (checkpoint > 3 ? checkpoint - 1 : 2) > 64)
    return fail(NADMM_ERR_INVALID_ARG, "iters / checkpoint needs too many stored states");
  return NADMM_OK;
}

// ---- pyramid ---------------------------------------------------------------
// Workspace of nadmm_register_pyramid: the registration workspace of the
// finest level (every level's fits in it), then for each coarser level its
// two images and its displacement, and one buffer for the displacement
// carried to the next level (the finest size).
struct PyrLayout {
  size_t reg, img[4], disp[4], carry, total;
};

nadmm_dims level_dims(const nadmm_dims& d, int levels, int l) {
  const int sh = levels - 1 - l;  // l = 0 is the coarsest
  return nadmm_dims{d.nx >> sh, d.ny >> sh, d.nz >> sh};
}

PyrLayout pyr_layout(const nadmm_dims& d, int levels) {
  PyrLayout L{};
  size_t o = 0;
  L.reg = o;
  o += layout(d).total;
  for (int l = 0; l + 1 < levels; ++l) {
    const nadmm_dims dl = level_dims(d, levels, l);
    const size_t V = (size_t)dl.nx * dl.ny * dl.nz;
    L.img[l] = o;
    o += align256(2 * V * sizeof(float));
    L.disp[l] = o;
    o += align256(3 * V * sizeof(float));
  }
  L.carry = o;
  o += align256(3 * (size_t)d.nx * d.ny * d.nz * sizeof(float));
  L.total = o;
  return L;
}

nadmm_status check_pyramid(const nadmm_dims& d, const nadmm_pyramid* pyr) {
  if (!pyr) return fail(NADMM_ERR_INVALID_ARG, "pyramid is NULL");
  if (pyr->levels < 1 || pyr->levels > 4)
    return fail(NADMM_ERR_INVALID_ARG, "levels must be in [1, 4] (got %d)", pyr->levels);
  const int m = 1 << (pyr->levels - 1);
  if (d.nx % m || d.ny % m || d.nz % m)
    return fail(NADMM_ERR_UNSUPPORTED_SIZE, "dims (%d, %d, %d) must be divisible by %d for %d levels",
                d.nx, d.ny, d.nz, m, pyr->levels);
  for (int l = 0; l < pyr->levels; ++l) {
    CHECK(check_dims(level_dims(d, pyr->levels, l)));
    if (pyr->outer[l] < 0 || pyr->outer[l] > 100000 || pyr->iters[l] < 1 || pyr->iters[l] > 100000)
      return fail(NADMM_ERR_INVALID_ARG, "level %d: outer in [0, 100000], iters in [1, 100000]", l);
  }
  return NADMM_OK;
}

// ---- pairs of several sizes (one launch per phase) -----------------------
// Pairs of one size must be consecutive (a size class); every field holds all
// pairs back to back in the caller's order.
struct MixedPlan {
  MixedLaunch m{};
  size_t v_total = 0, s_total = 0;  // sum of V, sum of half-spectrum elements
};

nadmm_status mixed_plan(int32_t npairs, const nadmm_dims* dims, MixedPlan& mp) {
  if (npairs < 1 || npairs > kMaxMixedPairs)
    return fail(NADMM_ERR_INVALID_ARG, "npairs must be in [1, %d] (got %d)", kMaxMixedPairs, npairs);
  if (!dims) return fail(NADMM_ERR_INVALID_ARG, "dims is NULL");
  MixedDesc& d = mp.m.d;
  d.nclasses = 0;
  for (int i = 0; i < npairs; ++i) {
    const nadmm_dims di = dims[i];
    CHECK(check_dims(di));
    const Geo g = geo(di);
    MixedClass* k = d.nclasses ? &d.c[d.nclasses - 1] : nullptr;
    if (!k || k->g.nx != g.nx || k->g.ny != g.ny || k->g.nz != g.nz) {
      for (int c = 0; c + 1 < d.nclasses; ++c)
        if (d.c[c].g.nx == g.nx && d.c[c].g.ny == g.ny && d.c[c].g.nz == g.nz)
          return fail(NADMM_ERR_INVALID_ARG, "pair %d: pairs of one size must be consecutive", i);
      if (d.nclasses == kMaxClasses)
        return fail(NADMM_ERR_INVALID_ARG, "more than %d different sizes in one mixed batch", kMaxClasses);
      if (!mixed_class_ok(g))
        return fail(NADMM_ERR_UNSUPPORTED_SIZE,
                    "dims (%d, %d, %d) of pair %d: a mixed batch needs nx in {64, 96, 128, 192} and ny, nz in "
                    "{32, 64, 96, 128}", di.nx, di.ny, di.nz, i);
      k = &d.c[d.nclasses++];
      *k = MixedClass{};
      k->g = g;
      k->o1 = (int64_t)mp.v_total;
      k->os = (int64_t)mp.s_total;
    }
    k->npairs += 1;
    mp.v_total += (size_t)g.V;
    mp.s_total += (size_t)3 * (g.nx / 2 + 1) * g.ny * g.nz;
  }
  mixed_shapes(mp.m);
  return NADMM_OK;
}

// Workspace of a mixed batch: each class's transform tables, then r, I1^w,
// s^k, s^{k-1}, the half spectrum and the displacement ping-pong buffer of
// every pair.
struct MixedLayout {
  size_t tab[kMaxClasses], r, iw, s1, s2, X, u, total;
};

MixedLayout mixed_layout(const MixedPlan& mp) {
  MixedLayout L{};
  const size_t V = mp.v_total;
  size_t o = 0;
  for (int c = 0; c < mp.m.d.nclasses; ++c) {
    L.tab[c] = o;
    o += align256(tables_bytes(mp.m.d.c[c].g));
  }
  L.r = o; o += align256(V * sizeof(float));
  L.iw = o; o += align256(V * sizeof(float));
  L.s1 = o; o += align256(3 * V * sizeof(float));
  L.s2 = o; o += align256(3 * V * sizeof(float));
  L.X = o; o += align256(mp.s_total * sizeof(float2));
  L.u = o; o += align256(3 * V * sizeof(float));
  L.total = o;
  return L;
}

}  // namespace

extern "C" {

#ifndef NADMM_SOURCE_DIGEST
#define NADMM_SOURCE_DIGEST "unknown"
#endif
int nadmm_abi_version(void) { return NADMM_ABI_VERSION; }

const char* nadmm_source_digest(void) { return NADMM_SOURCE_DIGEST; }

const char* nadmm_status_string(nadmm_status s) {
  switch (s) {
    case NADMM_OK: return "NADMM_OK";
    case NADMM_ERR_INVALID_ARG: return "NADMM_ERR_INVALID_ARG";
    case NADMM_ERR_UNSUPPORTED_SIZE: return "NADMM_ERR_UNSUPPORTED_SIZE";
    case NADMM_ERR_WORKSPACE: return "NADMM_ERR_WORKSPACE";
    case NADMM_ERR_HIP: return "NADMM_ERR_HIP";
    case NADMM_ERR_NONFINITE: return "NADMM_ERR_NONFINITE";
    case NADMM_ERR_DIVERGED: return "NADMM_ERR_DIVERGED";
  }
  return "NADMM_ERR_UNKNOWN";
}

const char* nadmm_last_error(void) { return g_err; }

nadmm_status nadmm_workspace_size(nadmm_dims d, const nadmm_params* p, size_t* bytes) {
  (void)p;
  if (!bytes) return fail(NADMM_ERR_INVALID_ARG, "bytes is NULL");
  CHECK(check_dims(d));
  *bytes = layout(d).total;
  return NADMM_OK;
}

nadmm_status nadmm_register(nadmm_dims d, const nadmm_params* p, const float* fixed,
                            const float* moving, const float* init_disp, float* disp,
                            float* warped, float* velocities, void* workspace,
                            size_t workspace_bytes, void* stream) {
  return register_impl(d, p, fixed, moving, init_disp, disp, warped, velocities, workspace,
                       workspace_bytes, stream, 1);
}

nadmm_status nadmm_register_threshold(nadmm_dims d, const nadmm_params* p, double tol_admm,
                                      double tol_warp, const float* fixed, const float* moving,
                                      float* disp, float* warped, int32_t* iters_run,
                                      int32_t* outer_run, double* admm_change, double* warp_change,
                                      void* workspace, size_t workspace_bytes, void* stream) {
  CHECK(check_dims(d));
  CHECK(check_params(p, true));
  if (isnan(tol_admm) || isnan(tol_warp))
    return fail(NADMM_ERR_INVALID_ARG, "tolerances must not be NaN");
  CHECK(check_ws(d, workspace, workspace_bytes));
  CHECK(check_ptr(fixed, "fixed", false));
  CHECK(check_ptr(moving, "moving", false));
  CHECK(check_ptr(disp, "disp", false));
  CHECK(check_ptr(warped, "warped", true));
  StopRule stop{};
  CheckHost res{static_cast<hipStream_t>(stream)};
  CHECK(res.init(stop, geo(d)));
  stop.tol_admm = tol_admm;
  stop.tol_warp = tol_warp;
  stop.admm_change = admm_change;
  stop.warp_change = warp_change;
  stop.iters_run = iters_run;
  const int64_t cells = (int64_t)p->outer * (p->iters - 1);  // up to ~1e10: 64-bit
  for (int64_t i = 0; admm_change && i < cells; ++i) admm_change[i] = NAN;
  for (int i = 0; warp_change && i + 1 < p->outer; ++i) warp_change[i] = NAN;
  for (int i = 0; iters_run && i < p->outer; ++i) iters_run[i] = 0;
  CHECK(register_impl(d, p, fixed, moving, nullptr, disp, warped, nullptr, workspace, workspace_bytes,
                      stream, 1, &stop));
  if (outer_run) *outer_run = stop.outer_run;
  HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  return NADMM_OK;
}

nadmm_status nadmm_register_checked(nadmm_dims d, const nadmm_params* p, uint32_t flags,
                                    const float* fixed, const float* moving, const float* init_disp,
                                    float* disp, float* warped, int32_t* diverged, void* workspace,
                                    size_t workspace_bytes, void* stream) {
  CHECK(check_dims(d));
  CHECK(check_params(p, true));
  if (flags & ~(uint32_t)(NADMM_CHECK_FINITE | NADMM_CHECK_DIVERGENCE))
    return fail(NADMM_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
  CHECK(check_ws(d, workspace, workspace_bytes));
  CHECK(check_ptr(fixed, "fixed", false));
  CHECK(check_ptr(moving, "moving", false));
  CHECK(check_ptr(init_disp, "init_disp", true));
  CHECK(check_ptr(disp, "disp", false));
  CHECK(check_ptr(warped, "warped", true));
  hipStream_t st = static_cast<hipStream_t>(stream);
  StopRule stop{};
  CheckHost res{st};
  CHECK(res.init(stop, geo(d)));
  stop.tol_admm = -1.0;
  stop.tol_warp = -1.0;
  stop.guard = (flags & NADMM_CHECK_DIVERGENCE) != 0;
  stop.diverged = diverged;
  for (int i = 0; diverged && i < p->outer; ++i) diverged[i] = 0;
  CHECK(register_impl(d, p, fixed, moving, init_disp, disp, warped, nullptr, workspace, workspace_bytes,
                      stream, 1, &stop));
  int64_t bad = 0;
  if (flags & NADMM_CHECK_FINITE) {
    // counted on the device into the workspace's Jacobian partials, copied
    // into the pinned read-back slots
    const Layout L = layout(d);
    int64_t* cnt = at<int64_t>(workspace, L.jac);
    const size_t V = (size_t)d.nx * d.ny * d.nz;
    HIP_TRY(launch_count_nonfinite(disp, 3 * V, cnt, st));
    HIP_TRY(hipMemcpyAsync(stop.host, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    if (warped) {
      HIP_TRY(launch_count_nonfinite(warped, V, cnt + 1, st));
      HIP_TRY(hipMemcpyAsync(stop.host + 1, cnt + 1, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    }
  }
  HIP_TRY(hipStreamSynchronize(st));
  if (flags & NADMM_CHECK_FINITE) {
    int64_t c0 = 0, c1 = 0;
    memcpy(&c0, stop.host, sizeof(int64_t));
    if (warped) memcpy(&c1, stop.host + 1, sizeof(int64_t));
    bad = c0 + c1;
  }
  if (bad > 0)
    return fail(NADMM_ERR_NONFINITE, "%lld non-finite values in the outputs", (long long)bad);
  if (stop.n_diverged > 0)
    return fail(NADMM_ERR_DIVERGED, "the ADMM iteration diverged in %d of %d warpings (last fixed-point "
                "residual above the first)", stop.n_diverged, p->outer);
  return NADMM_OK;
}

nadmm_status nadmm_register_bf16(nadmm_dims d, const nadmm_params* p, const uint16_t* fixed,
                                 const uint16_t* moving, const float* init_disp, float* disp,
                                 float* warped, float* velocities, void* workspace,
                                 size_t workspace_bytes, void* stream) {
  return register_impl(d, p, fixed, moving, init_disp, disp, warped, velocities, workspace,
                       workspace_bytes, stream, 1);
}

nadmm_status nadmm_workspace_size_batch(nadmm_dims d, int32_t batch, size_t* bytes) {
  if (!bytes) return fail(NADMM_ERR_INVALID_ARG, "bytes is NULL");
  CHECK(check_dims(d));
  CHECK(check_batch(batch));
  *bytes = layout(d, batch).total;
  return NADMM_OK;
}

nadmm_status nadmm_register_batch(nadmm_dims d, int32_t batch, const nadmm_params* p,
                                  const float* fixed, const float* moving,
                                  const float* init_disp, float* disp, float* warped,
                                  void* workspace, size_t workspace_bytes, void* stream) {
  CHECK(check_batch(batch));
  return register_impl(d, p, fixed, moving, init_disp, disp, warped, nullptr, workspace,
                       workspace_bytes, stream, batch);
}

nadmm_status nadmm_workspace_size_mixed(int32_t npairs, const nadmm_dims* dims, size_t* bytes) {
  MixedPlan mp;
  CHECK(mixed_plan(npairs, dims, mp));
  if (!bytes) return fail(NADMM_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = mixed_layout(mp).total;
  return NADMM_OK;
}

nadmm_status nadmm_register_mixed(int32_t npairs, const nadmm_dims* dims, const nadmm_params* p,
                                  const float* fixed, const float* moving, float* disp, float* warped,
                                  void* workspace, size_t workspace_bytes, void* stream) {
  MixedPlan mp;
  CHECK(mixed_plan(npairs, dims, mp));
  CHECK(check_params(p, true));
  CHECK(check_ptr(fixed, "fixed", false));
  CHECK(check_ptr(moving, "moving", false));
  CHECK(check_ptr(disp, "disp", false));
  CHECK(check_ptr(warped, "warped", true));
  CHECK(check_ptr(workspace, "workspace", false));
  const MixedLayout L = mixed_layout(mp);
  if (workspace_bytes < L.total)
    return fail(NADMM_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required",
                workspace_bytes, L.total);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t V = mp.v_total;
  if (p->outer == 0) {  // no warping: zero displacement, the moving image as warped
    HIP_TRY(timed(KK_FILL, st, [&] { return launch_fill(disp, 0.0f, 3 * V, st); }));
    if (warped) HIP_TRY(hipMemcpyAsync(warped, moving, V * sizeof(float), hipMemcpyDeviceToDevice, st));
    return NADMM_OK;
  }
  MixedLaunch& m = mp.m;
  for (int c = 0; c < m.d.nclasses; ++c) m.d.c[c].tab = tables_at(m.d.c[c].g, at<char>(workspace, L.tab[c]));
  HIP_TRY(launch_mixed_tables(m, st));
  float* r = at<float>(workspace, L.r);
  float* iw = at<float>(workspace, L.iw);
  float* S1 = at<float>(workspace, L.s1);
  float* S2 = at<float>(workspace, L.s2);
  float2* X = at<float2>(workspace, L.X);
  float* U = at<float>(workspace, L.u);
  const std::vector<double> gam = nesterov_gammas(p->iters);
  const float lam = (float)p->lambda, theta = (float)p->theta, eps = (float)p->eps;
  // the same sequence as nadmm_register from u = 0, every launch over all pairs
  auto dst_of = [&](int c) { return ((p->outer - 1 - c) % 2 == 0) ? disp : U; };
  const float* u_src = nullptr;
  for (int c = 0; c < p->outer; ++c) {
    const bool last = (c == p->outer - 1);
    const float* iw_c = c == 0 ? moving : iw;
    HIP_TRY(timed(KK_PASS_A, st, [&] {
      return launch_mixed_pass_a0(m, iw_c, fixed, r, S1, theta, eps, p->data_term, X, st);
    }));
    HIP_TRY(timed(KK_PASS_B, st, [&] { return launch_mixed_pass_b(m, X, lam, theta, p->order, st); }));
    float* cur = S1;
    float* prev = S2;
    for (int k = 1; k < p->iters; ++k) {
      PassCArgs a{};
      a.X = X;
      a.s1 = cur;
      a.s2 = (k == 1) ? nullptr : prev;
      a.gamma = (float)gam[k - 1];
      a.gamma_next = (k + 1 < p->iters) ? (float)gam[k] : 0.0f;
      a.iw = iw_c;
      a.r = r;
      a.theta = theta;
      a.eps = eps;
      a.data_term = p->data_term;
      a.out = prev;
      HIP_TRY(timed(KK_PASS_CA_ITER, st, [&] { return launch_mixed_pass_c(m, kIterFwdIw, a, st); }));
      HIP_TRY(timed(KK_PASS_B, st, [&] { return launch_mixed_pass_b(m, X, lam, theta, p->order, st); }));
      float* t = cur;
      cur = prev;
      prev = t;
    }
    PassCArgs a{};
    a.X = X;
    a.out = dst_of(c);
    a.u_old = u_src;
    a.img = moving;
    a.iw_out = last ? warped : iw;
    HIP_TRY(timed(KK_PASS_C_COMPOSE, st, [&] { return launch_mixed_pass_c(m, kCompose, a, st); }));
    u_src = a.out;
  }
  return NADMM_OK;
}

nadmm_status nadmm_autotune(nadmm_dims d, int32_t batch, const nadmm_params* p, void* workspace,
                            size_t workspace_bytes, void* stream, int32_t* rows_out) {
  CHECK(check_dims(d));
  CHECK(check_batch(batch));
  CHECK(check_params(p, false));
  CHECK(check_ws(d, workspace, workspace_bytes, batch));
  const Geo g = geo(d);
  const Plans pl = plans(d);
  const Layout L = layout(d, batch);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t V = (size_t)g.V, B = (size_t)batch;
  const Tables tb = tables_at(g, at<char>(workspace, L.tab));
  HIP_TRY(launch_tables(g, tb, st));
  // defined contents for the timed launches (the values do not matter)
  HIP_TRY(launch_fill(at<float>(workspace, L.r), 0.0f, B * V, st));
  HIP_TRY(launch_fill(at<float>(workspace, L.iw), 0.0f, B * V, st));
  HIP_TRY(launch_fill(at<float>(workspace, L.s1), 0.0f, 3 * B * V, st));
  HIP_TRY(launch_fill(at<float>(workspace, L.s2), 0.0f, 3 * B * V, st));
  HIP_TRY(launch_fill(at<float>(workspace, L.X), 0.0f,
                      B * 3 * (size_t)(d.nx / 2 + 1) * d.ny * d.nz * 2, st));
  PassCArgs a{};
  a.X = at<float2>(workspace, L.X);
  a.s1 = at<float>(workspace, L.s1);
  a.s2 = at<float>(workspace, L.s2);
  a.iw = at<float>(workspace, L.iw);
  a.r = at<float>(workspace, L.r);
  a.theta = (float)p->theta;
  a.eps = (float)p->eps;
  a.data_term = p->data_term;
  a.out = at<float>(workspace, L.s2);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  hipError_t err = hipEventCreate(&e1);
  int best = 0;
  float best_ms = 0.f;
  const int reps = 20;
  // NADMM_AUTOTUNE_LOG set: every candidate's time per launch on stderr
  const bool log = getenv("NADMM_AUTOTUNE_LOG") != nullptr;
  auto note = [&](const char* what, int value, float ms) {
    if (log)
      fprintf(stderr, "nadmm_autotune %dx%dx%d batch %d: %s %d: %.3f us per launch\n", d.nx, d.ny, d.nz, batch,
              what, value, 1000.f * ms / reps);
  };
  for (int rows = 2; rows <= 32 && err == hipSuccess; rows += 2) {
    if (g.ny % rows) continue;
    xline_rows_set(g, rows);
    if (!launch_shape_ok(g)) continue;
    for (int i = 0; i < 2 && err == hipSuccess; ++i)
      err = launch_pass_c(g, pl.x, tb, kIterFwdIw, a, st, batch);
    if (err == hipSuccess) err = hipEventRecord(e0, st);
    for (int i = 0; i < reps && err == hipSuccess; ++i)
      err = launch_pass_c(g, pl.x, tb, kIterFwdIw, a, st, batch);
    if (err == hipSuccess) err = hipEventRecord(e1, st);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err == hipSuccess) note("fused x-line pass rows", rows, ms);
    if (err == hipSuccess && (best == 0 || ms < best_ms)) {
      best = rows;
      best_ms = ms;
    }
  }
  xline_rows_set(g, best);  // 0 (nothing timed) restores the default
  // Times `launch` (reps launches after two untimed ones) into *ms.
  auto time_it = [&](auto&& launch, float* ms) -> hipError_t {
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int i = 0; i < reps && e == hipSuccess; ++i) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    return e;
  };
  // the composition pass's rows, on the same zero state with a previous
  // displacement of half a voxel everywhere (every sample between grid
  // points, the taps of neighbouring voxels neighbouring in memory, as for a
  // smooth deformation)
  if (err == hipSuccess) err = launch_fill(at<float>(workspace, L.u), 0.5f, 3 * B * V, st);
  PassCArgs ac{};
  ac.X = at<float2>(workspace, L.X);
  ac.u_old = at<float>(workspace, L.u);
  ac.img = at<float>(workspace, L.r);
  ac.out = at<float>(workspace, L.s1);
  ac.iw_out = at<float>(workspace, L.iw);
  int best_c = 0;
  float best_c_ms = 0.f;
  for (int rows = 2; rows <= 32 && err == hipSuccess; rows += 2) {
    if (!xline_rows_fit(g, rows, xline_threads_rows(g, rows))) continue;
    xline_rows_compose_set(g, rows);
    float ms = 0.f;
    err = time_it([&] { return launch_pass_c(g, pl.x, tb, kCompose, ac, st, batch); }, &ms);
    if (err == hipSuccess) note("composition pass rows", rows, ms);
    if (err == hipSuccess && (best_c == 0 || ms < best_c_ms)) {
      best_c = rows;
      best_c_ms = ms;
    }
  }
  xline_rows_compose_set(g, best_c);
  // wavefronts of a y-z plane workgroup, from what its team plans need to 16
  // (one-launch planes only)
  int best_w = 0;
  float best_w_ms = 0.f;
  if (plane_fits(g)) {
    for (int w = plane_waves_needed(g); w <= 16 && err == hipSuccess; ++w) {
      plane_waves_set(g, w);
      float ms = 0.f;
      err = time_it([&] {
        return launch_pass_b(g, tb, at<float2>(workspace, L.X), (float)p->lambda, (float)p->theta, p->order, st,
                             batch);
      }, &ms);
      if (err == hipSuccess) note("y-z pass wavefronts", w, ms);
      if (err == hipSuccess && (best_w == 0 || ms < best_w_ms)) {
        best_w = w;
        best_w_ms = ms;
      }
    }
  }
  plane_waves_set(g, best_w);
  (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(NADMM_ERR_HIP, "autotune: %s", hipGetErrorString(err));
  if (rows_out) *rows_out = xline_rows(g);
  return NADMM_OK;
}

nadmm_status nadmm_tuned_shapes(nadmm_dims d, int32_t* shapes) {
  CHECK(check_dims(d));
  if (!shapes) return fail(NADMM_ERR_INVALID_ARG, "shapes is NULL");
  const Geo g = geo(d);
  shapes[0] = xline_rows(g);
  shapes[1] = xline_rows_compose(g);
  shapes[2] = plane_fits(g) ? plane_threads_tuned(g) : 0;
  return NADMM_OK;
}

nadmm_status nadmm_set_shapes(nadmm_dims d, const int32_t* shapes) {
  CHECK(check_dims(d));
  if (!shapes) return fail(NADMM_ERR_INVALID_ARG, "shapes is NULL");
  const Geo g = geo(d);
  const int rows = shapes[0], crows = shapes[1], threads = shapes[2];
  if (rows < 0 || crows < 0 || threads < 0) return fail(NADMM_ERR_INVALID_ARG, "shapes must be >= 0");
  auto rows_ok = [&](int r) {
    return r <= 32 && r % 2 == 0 && g.ny % r == 0 && xline_rows_fit(g, r, xline_threads_rows(g, r));
  };
  if (rows > 0 && !rows_ok(rows))
    return fail(NADMM_ERR_INVALID_ARG, "x-line rows %d: not an even divisor of ny = %d up to 32 that fits", rows,
                d.ny);
  if (crows > 0 && !rows_ok(crows))
    return fail(NADMM_ERR_INVALID_ARG, "composition rows %d: not an even divisor of ny = %d up to 32 that fits",
                crows, d.ny);
  if (threads > 0) {
    if (!plane_fits(g))
      return fail(NADMM_ERR_INVALID_ARG, "plane threads: the y-z planes of these dims take the three-launch path");
    const int w = threads / 64;
    if (threads % 64 || w < plane_waves_needed(g) || w > 16)
      return fail(NADMM_ERR_INVALID_ARG, "plane threads %d: a multiple of 64 from %d to 1024", threads,
                  64 * plane_waves_needed(g));
  }
  const int old_rows = xline_rows_tuned(g);
  xline_rows_set(g, rows);
  if (!launch_shape_ok(g)) {
    xline_rows_set(g, old_rows);
    return fail(NADMM_ERR_INVALID_ARG, "x-line rows %d do not fit these dims", rows);
  }
  xline_rows_compose_set(g, crows);
  plane_waves_set(g, threads / 64);
  return NADMM_OK;
}

nadmm_status nadmm_workspace_size_pyramid(nadmm_dims d, const nadmm_pyramid* pyr, size_t* bytes) {
  if (!bytes) return fail(NADMM_ERR_INVALID_ARG, "bytes is NULL");
  CHECK(check_dims(d));
  CHECK(check_pyramid(d, pyr));
  *bytes = pyr_layout(d, pyr->levels).total;
  return NADMM_OK;
}

// The pyramid of nadmm_register_pyramid; `stop` (nullable) adds threshold
// stopping at every level, with iters_run / outer_run (host, nullable) laid
// out as nadmm_register_pyramid_threshold documents.
nadmm_status pyramid_impl(nadmm_dims d, const nadmm_params* p, const nadmm_pyramid* pyr,
                          const float* fixed, const float* moving, float* disp, float* warped,
                          void* workspace, size_t workspace_bytes, void* stream, StopRule* stop,
                          int32_t* iters_run, int32_t* outer_run) {
  CHECK(check_dims(d));
  CHECK(check_pyramid(d, pyr));
  CHECK(check_params(p, false));
  CHECK(check_ptr(fixed, "fixed", false));
  CHECK(check_ptr(moving, "moving", false));
  CHECK(check_ptr(disp, "disp", false));
  CHECK(check_ptr(warped, "warped", true));
  CHECK(check_ptr(workspace, "workspace", false));
  const int L = pyr->levels;
  const PyrLayout PL = pyr_layout(d, L);
  if (workspace_bytes < PL.total)
    return fail(NADMM_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required",
                workspace_bytes, PL.total);
  hipStream_t st = static_cast<hipStream_t>(stream);
  // images of every level, finest first down to the coarsest
  const float* F[4];
  const float* M[4];
  F[L - 1] = fixed;
  M[L - 1] = moving;
  for (int l = L - 2; l >= 0; --l) {
    const nadmm_dims dl = level_dims(d, L, l);
    const Geo gl = geo(dl);
    float* fl = at<float>(workspace, PL.img[l]);
    float* ml = fl + gl.V;
    HIP_TRY(launch_downsample2(gl, F[l + 1], fl, st));
    HIP_TRY(launch_downsample2(gl, M[l + 1], ml, st));
    F[l] = fl;
    M[l] = ml;
  }
  const size_t reg_bytes = PL.img[0] - PL.reg;  // == layout(d).total (rounded)
  const float* u_prev = nullptr;
  int run_at = 0;
  for (int l = 0; l < L; ++l) {
    const nadmm_dims dl = level_dims(d, L, l);
    const float* init = nullptr;
    if (u_prev) {
      float* carry = at<float>(workspace, PL.carry);
      HIP_TRY(launch_upsample2_disp(geo(dl), u_prev, carry, st));
      init = carry;
    }
    float* out = (l == L - 1) ? disp : at<float>(workspace, PL.disp[l]);
    nadmm_params pl = *p;
    pl.outer = pyr->outer[l];
    pl.iters = pyr->iters[l];
    if (stop) {
      stop->iters_run = iters_run ? iters_run + run_at : nullptr;
      stop->outer_run = 0;
    }
    CHECK(register_impl(dl, &pl, F[l], M[l], init, out, l == L - 1 ? warped : nullptr, nullptr,
                        at<char>(workspace, PL.reg), L > 1 ? reg_bytes : workspace_bytes, stream,
                        1, stop));
    if (stop && outer_run) outer_run[l] = stop->outer_run;
    run_at += pyr->outer[l];
    u_prev = out;
  }
  return NADMM_OK;
}

nadmm_status nadmm_register_pyramid(nadmm_dims d, const nadmm_params* p, const nadmm_pyramid* pyr,
                                    const float* fixed, const float* moving, float* disp,
                                    float* warped, void* workspace, size_t workspace_bytes,
                                    void* stream) {
  return pyramid_impl(d, p, pyr, fixed, moving, disp, warped, workspace, workspace_bytes, stream,
                      nullptr, nullptr, nullptr);
}

nadmm_status nadmm_register_pyramid_threshold(nadmm_dims d, const nadmm_params* p,
                                              const nadmm_pyramid* pyr, double tol_admm,
                                              double tol_warp, const float* fixed,
                                              const float* moving, float* disp, float* warped,
                                              int32_t* iters_run, int32_t* outer_run,
                                              void* workspace, size_t workspace_bytes,
                                              void* stream) {
  CHECK(check_dims(d));
  CHECK(check_pyramid(d, pyr));
  CHECK(check_params(p, false));
  if (isnan(tol_admm) || isnan(tol_warp))
    return fail(NADMM_ERR_INVALID_ARG, "tolerances must not be NaN");
  CHECK(check_ptr(fixed, "fixed", false));
  CHECK(check_ptr(moving, "moving", false));
  CHECK(check_ptr(disp, "disp", false));
  CHECK(check_ptr(warped, "warped", true));
  CHECK(check_ptr(workspace, "workspace", false));
  if (workspace_bytes < pyr_layout(d, pyr->levels).total)
    return fail(NADMM_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required",
                workspace_bytes, pyr_layout(d, pyr->levels).total);
  int total = 0;
  for (int l = 0; l < pyr->levels; ++l) total += pyr->outer[l];
  for (int i = 0; iters_run && i < total; ++i) iters_run[i] = 0;
  for (int l = 0; outer_run && l < pyr->levels; ++l) outer_run[l] = 0;
  StopRule stop{};
  CheckHost res{static_cast<hipStream_t>(stream)};
  CHECK(res.init(stop, geo(d)));
  stop.tol_admm = tol_admm;
  stop.tol_warp = tol_warp;
  CHECK(pyramid_impl(d, p, pyr, fixed, moving, disp, warped, workspace, workspace_bytes, stream, &stop,
                     iters_run, outer_run));
  HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  return NADMM_OK;
}

nadmm_status nadmm_workspace_size_grad(nadmm_dims d, const nadmm_params* p, int32_t checkpoint,
                                       size_t* bytes) {
  if (!bytes) return fail(NADMM_ERR_INVALID_ARG, "bytes is NULL");
  CHECK(check_dims(d));
  CHECK(check_grad_args(p, checkpoint));
  *bytes = grad_layout(d, p->iters, checkpoint).total;
  return NADMM_OK;
}

nadmm_status nadmm_ssd_grad(nadmm_dims d, const nadmm_params* p, int32_t checkpoint,
                            const float* fixed, const float* moving, double* loss,
                            float* d_moving, double* d_lambda, void* workspace,
                            size_t workspace_bytes, void* stream) {
  CHECK(check_dims(d));
  CHECK(check_grad_args(p, checkpoint));
  CHECK(check_ptr(fixed, "fixed", false));
  CHECK(check_ptr(moving, "moving", false));
  // both gradients, or neither (the loss alone: no reverse pass)
  const bool grads = d_moving || d_lambda;
  CHECK(check_ptr(d_moving, "d_moving", !grads));
  if (!loss || (grads && !d_lambda))
    return fail(NADMM_ERR_INVALID_ARG, "loss must not be NULL, and d_moving and d_lambda are both set or both NULL");
  CHECK(check_ptr(workspace, "workspace", false));
  const GradLayout L = grad_layout(d, p->iters, checkpoint);
  if (workspace_bytes < L.total)
    return fail(NADMM_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required",
                workspace_bytes, L.total);
  const Geo g = geo(d);
  const Plans pl = plans(d);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t V = (size_t)g.V;
  const int K = p->iters, c = checkpoint;
  const float theta = (float)p->theta;
  float* J = at<float>(workspace, L.J);
  float* r = at<float>(workspace, L.r);
  float* gr = at<float>(workspace, L.gr);
  float* resid = at<float>(workspace, L.resid);
  float2* X = at<float2>(workspace, L.X);
  float2* X2 = at<float2>(workspace, L.X2);  // the spectrum of t kept for the d/dlambda solve
  double* part = at<double>(workspace, L.part);
  const Tables tb = tables_at(g, at<char>(workspace, L.tab));
  int f = 0;
  auto field = [&]() { return at<float>(workspace, L.f3[f++]); };
  const int nck = L.nseg > 0 ? L.nseg : 1;
  std::vector<float*> ck_prev(nck), ck_cur(nck), buf(L.nbuf);
  for (int j = 0; j < nck; ++j) {
    ck_prev[j] = field();
    ck_cur[j] = field();
  }
  for (int i = 0; i < L.nbuf; ++i) buf[i] = field();
  float* ring[3] = {field(), field(), field()};
  float* gy = field();
  float* gt = field();
  float* tmp = field();
  float* w = field();
  float* gw = field();
  float* gJ = field();
  const std::vector<double> gam = nesterov_gammas(K);
  HIP_TRY(launch_tables(g, tb, st));

  // forward: s^k goes to checkpoint j's slots for k = j c (and j c - 1),
  // otherwise to one of two rolling buffers (in place over s^{k-2})
  auto fwd_slot = [&](int k) -> float* {
    if (k % c == 0 && k / c < nck) return ck_cur[k / c];
    if ((k + 1) % c == 0 && (k + 1) / c < nck && k + 1 > 0) return ck_prev[(k + 1) / c];
    return buf[k % 2];
  };
  // s^k for k = k0 .. k1 from the states before them (state(k) the slot of
  // s^k): the registration's fused iteration with J read, i.e. one solve
  // started on t^{k0}, then per step the x-line pass that forms s^k from
  // S t^k and transforms the next input along x, and pass B
  auto fwd_steps = [&](int k0, int k1, auto state) -> hipError_t {
    hipError_t e = spectral_ab(g, pl, tb, p, state(k0 - 1), k0 >= 2 ? state(k0 - 2) : nullptr,
                               (float)gam[k0 - 1], X, st);
    for (int k = k0; k <= k1 && e == hipSuccess; ++k) {
      PassCArgs a{};
      a.X = X;
      a.s1 = state(k - 1);
      a.s2 = k >= 2 ? state(k - 2) : nullptr;
      a.gamma = (float)gam[k - 1];
      a.gamma_next = k < k1 ? (float)gam[k] : 0.0f;
      a.J = J;
      a.r = r;
      a.theta = theta;
      a.eps = (float)p->eps;
      a.data_term = 2;
      a.out = state(k);
      e = timed(KK_PASS_CA_ITER, st, [&] { return launch_pass_c(g, pl.x, tb, kIterFwd, a, st); });
      if (e == hipSuccess && k < k1)
        e = timed(KK_PASS_B, st, [&] {
          return launch_pass_b(g, tb, X, (float)p->lambda, (float)p->theta, p->order, st);
        });
    }
    return e;
  };
  // u = 0: the warped source is the moving image itself
  HIP_TRY(launch_grad_resid(g, moving, fixed, J, r, fwd_slot(0), theta, (float)p->eps, 2, st));
  if (K >= 2) HIP_TRY(fwd_steps(1, K - 1, [&](int k) -> float* { return k < 0 ? nullptr : fwd_slot(k); }));
  float* s_last = fwd_slot(K - 1);
  HIP_TRY(spectral_apply(g, pl, tb, p, s_last, nullptr, 0.0f, X, w, st));
  if (!grads) {  // the loss alone: the same warp and residual as the adjoint kernel's
    HIP_TRY(launch_warp(g, moving, w, tmp, st));
    HIP_TRY(launch_grad_resid(g, tmp, fixed, nullptr, resid, nullptr, theta, (float)p->eps, 2, st));
    HIP_TRY(launch_dot(V, resid, resid, 1.0, false, part, loss, st));
    return NADMM_OK;
  }

  // loss, the image adjoint of the final warp, dL/dw
  HIP_TRY(launch_fill(d_moving, 0.0f, V, st));
  HIP_TRY(launch_warp_adjoint(g, moving, fixed, w, resid, d_moving, gw, st));
  HIP_TRY(launch_dot(V, resid, resid, 1.0, false, part, loss, st));
  // <o, (dS/dlambda) t> with t = s1 + gamma (s1 - s2), set or added into
  // *d_lambda: the x-line pass of the solve sums its products with o per
  // workgroup (the partials hold the most workgroups any rows give)
  // (Xt: the x transform of t is already there, else X takes it)
  auto dot_deriv = [&](const float* s1, const float* s2, float gamma, const float* o, bool add,
                       float2* Xt = nullptr) -> hipError_t {
    hipError_t e = Xt ? timed(KK_PASS_B, st, [&] {
      return launch_pass_b(g, tb, Xt, (float)p->lambda, (float)p->theta, p->order, st, 1, true);
    }) : spectral_ab(g, pl, tb, p, s1, s2, gamma, X, st, 1, true);
    if (e != hipSuccess) return e;
    PassCArgs a{};
    a.X = Xt ? Xt : X;
    a.s1 = o;
    a.chk_part = part;
    int nb = 0;
    e = timed(KK_PASS_C_OUT, st, [&] { return launch_pass_c_dot(g, pl.x, tb, a, st, (int)L.nparts, &nb); });
    if (e != hipSuccess) return e;
    return launch_dot_final(part, nb, 1.0, add, d_lambda, st);
  };
  // w = S s^{K-1}: dL/dlambda gets <gw, (dS/dlambda) s^{K-1}>, dL/ds^{K-1} = S gw
  HIP_TRY(dot_deriv(s_last, nullptr, 0.0f, gw, false));
  for (int i = 0; i < 3; ++i) HIP_TRY(launch_fill(ring[i], 0.0f, 3 * V, st));
  HIP_TRY(spectral_apply(g, pl, tb, p, gw, nullptr, 0.0f, X, ring[(K - 1) % 3], st));
  HIP_TRY(launch_fill(gJ, 0.0f, 3 * V, st));
  HIP_TRY(launch_fill(gr, 0.0f, V, st));

  // backward, one segment of steps (b, kmax] at a time, newest first
  for (int j = L.nseg - 1; j >= 0; --j) {
    const int b = j * c, kmax = (b + c < K - 1) ? b + c : K - 1;
    auto state = [&](int k) -> float* {
      if (k < 0) return nullptr;
      if (k == b) return ck_cur[j];
      if (k == b - 1) return c == 1 ? ck_cur[j - 1] : ck_prev[j];  // c = 1 keeps every state
      return buf[k - b - 1];
    };
    if (b + 1 <= kmax - 1) HIP_TRY(fwd_steps(b + 1, kmax - 1, state));  // recompute the segment's states
    for (int k = kmax; k > b; --k) {
      const float* s1 = state(k - 1);
      const float* s2 = k >= 2 ? state(k - 2) : nullptr;
      const float gk = (float)gam[k - 1];
      float* gk_ = ring[k % 3];
      // the step's adjoint in the inverse x pass of y = S t, which also
      // transforms gy along x for the next solve; the x transform of t is
      // kept in X2 for the d/dlambda solve
      HIP_TRY(timed(KK_PASS_A, st, [&] { return launch_pass_a(g, pl.x, tb, s1, s2, gk, X, st, 1, X2); }));
      HIP_TRY(timed(KK_PASS_B, st, [&] {
        return launch_pass_b(g, tb, X, (float)p->lambda, (float)p->theta, p->order, st);
      }));
      PassCArgs as{};
      as.X = X;
      as.s1 = s1;
      as.s2 = s2;
      as.gamma = gk;
      as.J = J;
      as.r = r;
      as.theta = theta;
      as.gs = gk_;
      as.gy = gy;
      as.gt = gt;
      as.gJ = gJ;
      as.gr = gr;
      HIP_TRY(timed(KK_PASS_C_OUT, st, [&] { return launch_pass_c(g, pl.x, tb, kAdjStep, as, st); }));
      HIP_TRY(timed(KK_PASS_B, st, [&] {
        return launch_pass_b(g, tb, X, (float)p->lambda, (float)p->theta, p->order, st);
      }));
      // gt + S gy into the adjoints of s^{k-1} and s^{k-2}, and gk_ (read by
      // the step's adjoint above) cleared to become the adjoint of s^{k-3}:
      // all in the inverse x pass of the solve
      PassCArgs ac{};
      ac.X = X;
      ac.s1 = gt;
      ac.gamma = gk;
      ac.out = ring[(k - 1) % 3];
      ac.b_out = k >= 2 ? ring[(k - 2) % 3] : nullptr;
      ac.v_out = gk_;
      HIP_TRY(timed(KK_PASS_C_OUT, st, [&] { return launch_pass_c(g, pl.x, tb, kAdjY, ac, st); }));
      HIP_TRY(dot_deriv(s1, s2, gk, gy, true, X2));
    }
  }
  // s^0 = D(0; J, r)
  HIP_TRY(launch_adj_step(g, ring[0], nullptr, nullptr, 0.0f, nullptr, J, r, theta, nullptr,
                          nullptr, gJ, gr, st));
  HIP_TRY(launch_grad_transpose(g, gJ, gr, d_moving, st));
  return NADMM_OK;
}

nadmm_status nadmm_admm(nadmm_dims d, const nadmm_params* p, const float* J, const float* r,
                        float* w_out, float* b_out, float* v_out, void* workspace,
                        size_t workspace_bytes, void* stream) {
  CHECK(check_dims(d));
  CHECK(check_params(p, false));
  CHECK(check_ptr(J, "J", false));
  CHECK(check_ptr(r, "r", false));
  CHECK(check_ptr(w_out, "w_out", false));
  CHECK(check_ptr(b_out, "b_out", true));
  CHECK(check_ptr(v_out, "v_out", true));
  CHECK(check_ws(d, workspace, workspace_bytes));
  const Geo g = geo(d);
  const Plans pl = plans(d);
  const Layout L = layout(d);
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* S1 = at<float>(workspace, L.s1);
  float* S2 = at<float>(workspace, L.s2);
  float2* X = at<float2>(workspace, L.X);
  const Tables tb = tables_at(g, at<char>(workspace, L.tab));
  HIP_TRY(launch_tables(g, tb, st));
  HIP_TRY(timed(KK_ADMM_INIT, st, [&] { return launch_admm_init(g, J, r, S1, p->iters == 1 ? v_out : nullptr, (float)p->theta,
                           (float)p->eps, p->data_term, st); }));
  float* cur = S1;
  float* prev = S2;
  CHECK(admm_iterations(g, pl, tb, p, J, nullptr, r, cur, prev, X, v_out, st));
  PassCArgs a{};
  a.X = X;
  a.s1 = cur;
  a.out = w_out;
  a.b_out = b_out;
  HIP_TRY(timed(KK_PASS_C_WB, st, [&] { return launch_pass_c(g, pl.x, tb, kFinalWB, a, st); }));
  return NADMM_OK;
}

nadmm_status nadmm_fourier_solve(nadmm_dims d, const nadmm_params* p, const float* s, float* w,
                                 void* workspace, size_t workspace_bytes, void* stream) {
  CHECK(check_dims(d));
  CHECK(check_params(p, false));
  CHECK(check_ptr(s, "s", false));
  CHECK(check_ptr(w, "w", false));
  CHECK(check_ws(d, workspace, workspace_bytes));
  const Geo g = geo(d);
  const Plans pl = plans(d);
  const Layout L = layout(d);
  hipStream_t st = static_cast<hipStream_t>(stream);
  float2* X = at<float2>(workspace, L.X);
  const Tables tb = tables_at(g, at<char>(workspace, L.tab));
  HIP_TRY(launch_tables(g, tb, st));
  HIP_TRY(spectral_ab(g, pl, tb, p, s, nullptr, 0.0f, X, st));
  PassCArgs a{};
  a.X = X;
  a.out = w;
  HIP_TRY(timed(KK_PASS_C_OUT, st, [&] { return launch_pass_c(g, pl.x, tb, kOutY, a, st); }));
  return NADMM_OK;
}

nadmm_status nadmm_warp(nadmm_dims d, const float* img, const float* disp, const float* ref,
                        float* out, float* grad, float* resid, void* stream) {
  CHECK(check_dims(d));
  CHECK(check_ptr(img, "img", false));
  CHECK(check_ptr(disp, "disp", false));
  CHECK(check_ptr(ref, "ref", true));
  CHECK(check_ptr(out, "out", false));
  CHECK(check_ptr(grad, "grad", true));
  CHECK(check_ptr(resid, "resid", true));
  if (resid && !ref) return fail(NADMM_ERR_INVALID_ARG, "resid requires ref");
  if (out == img || out == disp) return fail(NADMM_ERR_INVALID_ARG, "out aliases an input");
  const Geo g = geo(d);
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(timed(KK_WARP, st, [&] { return launch_warp(g, img, disp, out, st); }));
  if (grad || resid)
    HIP_TRY(timed(KK_GRAD, st, [&] { return launch_grad_resid(g, out, resid ? ref : nullptr, grad, resid, nullptr, 1.0f, 1.0f, 2,
                              st); }));
  return NADMM_OK;
}

nadmm_status nadmm_compose(nadmm_dims d, const float* u, const float* v, float* out,
                           void* stream) {
  CHECK(check_dims(d));
  CHECK(check_ptr(u, "u", false));
  CHECK(check_ptr(v, "v", false));
  CHECK(check_ptr(out, "out", false));
  if (out == u || out == v) return fail(NADMM_ERR_INVALID_ARG, "out aliases an input");
  HIP_TRY(timed(KK_COMPOSE, static_cast<hipStream_t>(stream), [&] { return launch_compose(geo(d), u, v, out, static_cast<hipStream_t>(stream)); }));
  return NADMM_OK;
}

nadmm_status nadmm_expmap(nadmm_dims d, const float* vel, int32_t steps, float* out,
                          void* workspace, size_t workspace_bytes, void* stream) {
  CHECK(check_dims(d));
  CHECK(check_ptr(vel, "vel", false));
  CHECK(check_ptr(out, "out", false));
  if (steps < 0 || steps > 30) return fail(NADMM_ERR_INVALID_ARG, "steps must be in [0, 30]");
  if (out == vel) return fail(NADMM_ERR_INVALID_ARG, "out aliases vel");
  CHECK(check_ws(d, workspace, workspace_bytes));
  const Geo g = geo(d);
  const Layout L = layout(d);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t n = 3 * (size_t)g.V;
  float* T = at<float>(workspace, L.u);
  // ping-pong so that the last squaring writes out
  float* a = (steps % 2 == 0) ? out : T;
  float* b = (a == out) ? T : out;
  HIP_TRY(timed(KK_SCALE, st, [&] { return launch_scale(vel, a, (float)ldexp(1.0, -steps), n, st); }));
  for (int k = 0; k < steps; ++k) {
    HIP_TRY(timed(KK_COMPOSE, st, [&] { return launch_compose(g, a, a, b, st); }));
    float* t = a;
    a = b;
    b = t;
  }
  return NADMM_OK;
}

nadmm_status nadmm_jacobian(nadmm_dims d, const float* disp, float* det, double* stats,
                            int64_t* n_nonpos, void* workspace, size_t workspace_bytes,
                            void* stream) {
  CHECK(check_dims(d));
  CHECK(check_ptr(disp, "disp", false));
  CHECK(check_ptr(det, "det", true));
  CHECK(check_ptr(stats, "stats", false));
  CHECK(check_ptr(n_nonpos, "n_nonpos", false));
  CHECK(check_ws(d, workspace, workspace_bytes));
  const Layout L = layout(d);
  HIP_TRY(timed(KK_JACOBIAN, static_cast<hipStream_t>(stream), [&] { return launch_jacobian(geo(d), disp, det, at<double>(workspace, L.jac), stats, n_nonpos,
                          static_cast<hipStream_t>(stream)); }));
  return NADMM_OK;
}

nadmm_status nadmm_count_nonfinite(nadmm_dims d, const float* field, int32_t count,
                                   int64_t* nonfinite, void* stream) {
  CHECK(check_dims(d));
  CHECK(check_ptr(field, "field", false));
  CHECK(check_ptr(nonfinite, "nonfinite", false));
  if (count < 1 || count > 64) return fail(NADMM_ERR_INVALID_ARG, "count must be in [1, 64]");
  const size_t n = (size_t)count * d.nx * d.ny * d.nz;
  HIP_TRY(launch_count_nonfinite(field, n, nonfinite, static_cast<hipStream_t>(stream)));
  return NADMM_OK;
}

nadmm_status nadmm_profile_replay(nadmm_dims d, const nadmm_params* p, int32_t kind, int32_t reps,
                                  void* workspace, size_t workspace_bytes, void* stream,
                                  double* avg_ms) {
  CHECK(check_dims(d));
  CHECK(check_params(p, false));
  CHECK(check_ws(d, workspace, workspace_bytes));
  if (!avg_ms) return fail(NADMM_ERR_INVALID_ARG, "avg_ms is NULL");
  if (kind < 0 || kind > 3) return fail(NADMM_ERR_INVALID_ARG, "kind must be 0, 1, 2 or 3");
  if (reps < 1 || reps > 10000) return fail(NADMM_ERR_INVALID_ARG, "reps must be in [1, 10000]");
  const Geo g = geo(d);
  const Plans pl = plans(d);
  const Layout L = layout(d);
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* r = at<float>(workspace, L.r);
  float* S1 = at<float>(workspace, L.s1);
  float* S2 = at<float>(workspace, L.s2);
  float2* X = at<float2>(workspace, L.X);
  const Tables tb = tables_at(g, at<char>(workspace, L.tab));
  // kind 2 replays the fused pass C + A with zero extrapolation weights (the
  // same loads, arithmetic and stores) so that the repeated state stays
  // bounded without pass B in between
  PassCArgs a{};
  a.X = X;
  a.s1 = S1;
  a.s2 = S2;
  a.gamma = 0.0f;
  a.gamma_next = 0.0f;
  a.iw = at<float>(workspace, L.iw);
  a.r = r;
  a.theta = (float)p->theta;
  a.eps = (float)p->eps;
  a.data_term = p->data_term;
  a.out = S2;
  auto launch = [&]() -> hipError_t {
    if (kind == 0) return launch_pass_a(g, pl.x, tb, S1, nullptr, 0.0f, X, st);
    if (kind == 1) return launch_pass_b(g, tb, X, (float)p->lambda, (float)p->theta, p->order, st);
    if (kind == 2) return launch_pass_c(g, pl.x, tb, kIterFwdIw, a, st);
    const hipError_t e = launch_pass_c(g, pl.x, tb, kIterFwdIw, a, st);
    return e != hipSuccess ? e : launch_pass_b(g, tb, X, (float)p->lambda, (float)p->theta, p->order, st);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  hipError_t err = hipEventCreate(&e1);
  if (err == hipSuccess) err = launch();  // warm the caches once
  if (err == hipSuccess) err = hipEventRecord(e0, st);
  for (int i = 0; i < reps && err == hipSuccess; ++i) err = launch();
  if (err == hipSuccess) err = hipEventRecord(e1, st);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  float ms = 0.f;
  if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(NADMM_ERR_HIP, "replay: %s", hipGetErrorString(err));
  *avg_ms = (double)ms / reps;
  return NADMM_OK;
}

nadmm_status nadmm_profile_enable(int enable) {
  g_prof.store(enable != 0);
  return NADMM_OK;
}

int nadmm_profile_read(int max, const char** names, int64_t* counts, double* total_ms) {
  int64_t cnt[KK_COUNT] = {0};
  double ms[KK_COUNT] = {0};
  int status = KK_COUNT;
  std::vector<ProfRecord> recs;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    recs.swap(g_records);
  }
  for (const ProfRecord& r : recs) {
    float t = 0.f;
    if (hipEventSynchronize(r.stop) != hipSuccess || hipEventElapsedTime(&t, r.start, r.stop) != hipSuccess) {
      status = -1;
    } else {
      cnt[r.kind] += 1;
      ms[r.kind] += t;
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (const ProfRecord& r : recs) {
      g_free_events.push_back(r.start);
      g_free_events.push_back(r.stop);
    }
  }
  for (int k = 0; k < KK_COUNT && k < max; ++k) {
    if (names) names[k] = kKindNames[k];
    if (counts) counts[k] = cnt[k];
    if (total_ms) total_ms[k] = ms[k];
  }
  if (status < 0) fail(NADMM_ERR_HIP, "event synchronisation failed while reading timings");
  return status;
}

}  // extern "C"
