/* The C ABI from C (C99, no C++ and no Python): validation and sizing of
 * problems on the host, status strings, and the error paths that need no
 * device.  Prints one line per check and exits non-zero on the first
 * failure.  Built and run by tests/test_abi_c.py. */
#include <stdio.h>
#include <string.h>

#include "mlc.h"

static int failures = 0;
#define CHECK(cond, what)                                      \
  do {                                                         \
    if (cond) {                                                \
      printf("ok   %s\n", what);                               \
    } else {                                                   \
      printf("FAIL %s\n", what);                               \
      ++failures;                                              \
    }                                                          \
  } while (0)

static mlc_problem base(void) {
  mlc_problem p;
  memset(&p, 0, sizeof p);
  p.n_cells = 256;
  p.h = 1.0 / 256;
  p.patch = 32;
  p.alpha = 3.0;
  p.beta = 6.0;
  p.P = 4;
  p.Q = 6;
  p.conv_precision = MLC_CONV_FP32;
  return p;
}

int main(void) {
  mlc_problem p = base();
  mlc_plan_info info;
  size_t bytes = 0;
  char buf[256];

  CHECK(mlc_problem_info(&p, &info) == MLC_OK, "256^3 L27 problem is valid");
  CHECK(info.M == 160 && info.npatch == 512 && info.K == 20 && info.b == 3, "its torus, patches, modes, radius");
  CHECK(info.levels == 2 && info.rhs_order == 4 && info.skip_empty == 0, "two levels, fourth order, dense by default");
  CHECK(mlc_problem_workspace_bytes(&p, &bytes) == MLC_OK && bytes > ((size_t)6 << 30), "workspace above 6 GB");

  p.levels = 3;
  p.n_cells = 512;
  p.h = 1.0 / 512;
  p.alpha = 1.75;
  p.beta = 3.25;
  p.level_alpha[0] = 3.0;
  CHECK(mlc_problem_info(&p, &info) == MLC_OK && info.level_N == 192 && info.level_alpha[0] == 3.0,
        "three levels at 512^3 with alpha 3 at level 1");

  p = base();
  p.rhs_order = 6;
  CHECK(mlc_problem_info(&p, &info) == MLC_OK && info.rhs_order == 6, "sixth-order right-hand side with L27");
  p.Q = 4;
  CHECK(mlc_problem_info(&p, &info) == MLC_ERR_UNSUPPORTED, "sixth order refused for L19");

  p = base();
  p.n_cells = 250;
  CHECK(mlc_problem_info(&p, &info) == MLC_ERR_INVALID_ARG, "N not a multiple of the patch size is refused");
  CHECK(mlc_last_error(NULL, buf, sizeof buf) == MLC_OK && strlen(buf) > 0, "the refusal is explained");

  CHECK(strcmp(mlc_status_string(MLC_ERR_BUSY), "MLC_ERR_BUSY") == 0, "status strings");
  CHECK(mlc_problem_info(NULL, &info) == MLC_ERR_INVALID_ARG, "null problem refused");
  CHECK(mlc_plan_destroy(NULL) == MLC_ERR_INVALID_ARG, "null plan refused");
  CHECK(mlc_server_drain(NULL) == MLC_ERR_INVALID_ARG, "null server refused");

  printf("%d failure(s)\n", failures);
  return failures ? 1 : 0;
}
