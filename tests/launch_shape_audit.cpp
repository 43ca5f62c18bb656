// Host-side audit of every launch shape the library can choose: for each
// supported grid (every length 2^a 3^b in [4, 256], nx a multiple of 4, ny
// even) and every x-line row count the shape checks admit (the default and
// each even divisor of ny up to 32, as the autotuner and nadmm_set_shapes
// offer them), the x-line workgroup must stay within the 768-thread launch
// bound its kernels are compiled for, within the LDS budget and within the
// per-thread item counts the kernels unroll; every admissible y-z plane
// workgroup size must stay within 1024 threads and the LDS budget, for whole
// planes and for the half planes of sizes whose planes do not fit; the
// three-launch split shapes within 256 threads.  Exit status 1 and a line
// per violation otherwise.  Built by tests/test_launch_shapes.py with hipcc;
// it includes the kernel source for its file-local helpers and runs on the
// host only.
#include <cstdio>
#include <vector>

#include "kernels.hip"

using namespace nadmm;

static bool length_ok(int n) {
  if (n < 4 || n > 256) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

int main() {
  std::vector<int> lengths;
  for (int n = 4; n <= 256; ++n)
    if (length_ok(n)) lengths.push_back(n);
  long sizes = 0, shapes = 0, bad = 0;
  auto report = [&](const char* what, const Geo& g, int a, long b) {
    if (++bad <= 40) printf("violation: %s at %dx%dx%d (%d, %ld)\n", what, g.nx, g.ny, g.nz, a, b);
  };
  for (int nx : lengths)
    for (int ny : lengths)
      for (int nz : lengths) {
        if (nx % 4 || ny % 2) continue;
        const Geo g{nx, ny, nz, nx * ny * nz};
        xline_rows_set(g, 0);
        xline_rows_compose_set(g, 0);
        plane_waves_set(g, 0);
        if (!launch_shape_ok(g)) continue;  // rejected by the C ABI's size check
        ++sizes;
        for (int r = 0; r <= 32; r += 2) {
          if (r && ny % r) continue;
          xline_rows_set(g, r);
          if (launch_shape_ok(g)) {
            ++shapes;
            const int rows = xline_rows(g), t = xline_threads(g);
            const size_t lds = pass_a_lds_rows(g, rows);
            if (t > 768 || t % 64) report("x-line threads", g, rows, t);
            if (lds > (size_t)kMaxLds) report("x-line LDS", g, rows, (long)lds);
            if (3 * (rows / 2) * nx > kEpt * t) report("x-line FFT points per thread", g, rows, t);
            if (3 * rows * (nx / 4) > kXItems * t) report("x-line float4 loads per thread", g, rows, t);
            if (rows * (nx / 4) > 2 * t) report("x-line runs per thread", g, rows, t);
            if ((long)(ny / rows) * nz > 0x7fffffffL || nz > 65535) report("x-line grid", g, rows, nz);
          }
          // composition rows are admitted by the same fit at their own thread count
          if (r && xline_rows_fit(g, r, xline_threads_rows(g, r))) {
            ++shapes;
            const int t = xline_threads_rows(g, r);
            if (t > 768 || pass_a_lds_rows(g, r) > (size_t)kMaxLds) report("composition shape", g, r, t);
          }
        }
        xline_rows_set(g, 0);
        if (plane_fits(g)) {
          for (int w = plane_waves_needed(g); w <= 16; ++w) {
            plane_waves_set(g, w);
            ++shapes;
            const int t = plane_threads_tuned(g);
            if (t > 1024 || t % 64 || t < 64 * plane_waves_needed(g)) report("plane threads", g, w, t);
            if (plane_lds_bytes(g, plane_row_stride(g)) > (size_t)kMaxLds) report("plane LDS", g, w, t);
          }
          plane_waves_set(g, 0);
        } else if (ysplit(g)) {
          // half planes: x-line tiles of two row groups, one workgroup per sub-plane
          const Geo gs = half_plane_geo(g);
          ++shapes;
          const int t = plane_threads_tuned(gs), rows = xline_rows(g);
          if (t > 1024 || t % 64 || t < 64 * plane_waves_needed(gs)) report("half-plane threads", g, 0, t);
          if (plane_lds_bytes(gs, plane_row_stride(gs)) > (size_t)kMaxLds) report("half-plane LDS", g, 0, t);
          if (rows % 4 || (ny / 2) % (rows / 2)) report("half-plane x-line rows", g, rows, 0);
        } else {
          const SplitShape sh = split_shape(g);
          ++shapes;
          if (sh.rows_threads > 256 || sh.cols_threads > 256) report("split threads", g, sh.rb, sh.w);
          if (split_rows_lds(g, sh) > (size_t)kMaxLds) report("split LDS", g, sh.rb, sh.w);
        }
      }
  printf("%ld sizes, %ld launch shapes, %ld violations\n", sizes, shapes, bad);
  return bad ? 1 : 0;
}
