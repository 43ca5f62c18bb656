/* A plain C99 consumer of the C ABI: the public header compiles as C, and
 * the host-only entry points link and answer from C (no device is touched:
 * sizes, status strings and argument errors only).  Prints "ok" and exits 0
 * when every check holds.  Built and run by tests/test_header_c.py. */
#include <stdio.h>
#include <string.h>

#include "nadmm.h"

static int failures = 0;
#define EXPECT(cond)                                              \
  do {                                                            \
    if (!(cond)) {                                                \
      printf("check failed: %s (line %d)\n", #cond, __LINE__);   \
      ++failures;                                                 \
    }                                                             \
  } while (0)

int main(void) {
  nadmm_dims d = {128, 128, 96};
  nadmm_dims bad = {100, 128, 96};
  nadmm_params p;
  size_t bytes = 0, bytes_batch = 0;
  int32_t shapes[3] = {0, 0, 0};
  memset(&p, 0, sizeof p);
  p.lambda = 0.01;
  p.theta = 0.1;
  p.order = 2;
  p.data_term = 2;
  p.eps = 1e-8;
  p.outer = 10;
  p.iters = 20;

  EXPECT(nadmm_abi_version() == NADMM_ABI_VERSION);
  EXPECT(strcmp(nadmm_status_string(NADMM_OK), "NADMM_OK") == 0);
  EXPECT(strlen(nadmm_source_digest()) == 64);
  EXPECT(nadmm_workspace_size(d, &p, &bytes) == NADMM_OK && bytes > 0);
  EXPECT(nadmm_workspace_size_batch(d, 2, &bytes_batch) == NADMM_OK && bytes_batch > bytes);
  EXPECT(nadmm_workspace_size(bad, &p, &bytes) == NADMM_ERR_UNSUPPORTED_SIZE);
  EXPECT(strstr(nadmm_last_error(), "100") != NULL);
  EXPECT(nadmm_workspace_size(d, &p, NULL) == NADMM_ERR_INVALID_ARG);
  EXPECT(nadmm_tuned_shapes(d, shapes) == NADMM_OK && shapes[0] > 0 && shapes[2] % 64 == 0);
  EXPECT(nadmm_register(d, &p, NULL, NULL, NULL, NULL, NULL, NULL, NULL, 0, NULL) == NADMM_ERR_INVALID_ARG);
  if (failures == 0) printf("ok\n");
  return failures ? 1 : 0;
}
