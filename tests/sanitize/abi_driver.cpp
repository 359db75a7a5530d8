// Drives the library's host-only paths -- configuration defaults and
// checks, level shapes, workspace sizing and the argument checks made
// before any device work -- so that a host build with
// -fsanitize=address,undefined checks them.  No call here reaches the GPU.
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "tomg.h"

static int failures = 0;
#define CHECK(c)                                          \
  do {                                                    \
    if (!(c)) {                                           \
      std::fprintf(stderr, "FAILED: %s (line %d)\n", #c, __LINE__); \
      ++failures;                                         \
    }                                                     \
  } while (0)

int main() {
  tomg_config c;
  const int sides[] = {5, 9, 17, 33, 65, 66, 101, 129, 201, 257, 401, 1001, 1025, 4097, 8193, 3};
  size_t last = 0;
  for (int nx : sides)
    for (int ny : sides) {
      tomg_config_default(&c, nx, ny, 1.0 / (nx > 1 ? nx - 1 : 1), 1.0 / (ny > 1 ? ny - 1 : 1));
      for (int prec = 0; prec < 2; ++prec)
        for (int sm = 0; sm < 4; ++sm)
          for (int neu = 0; neu < 16; neu += 5) {
            c.precision = prec;
            c.smoother = sm;
            c.neumann = neu;
            const int L = tomg_num_levels(&c);
            const size_t w = tomg_workspace_bytes(&c);
            CHECK((L == 0) == (w == 0));
            CHECK(w % 256 == 0);
            last += w;
          }
    }
  CHECK(last > 0);
  // invalid fields
  tomg_config_default(&c, 129, 129, 1.0 / 128, 1.0 / 128);
  tomg_config bad = c;
  bad.nu1 = 0;
  CHECK(tomg_workspace_bytes(&bad) == 0);
  bad = c;
  bad.dx = -1.0;
  CHECK(tomg_workspace_bytes(&bad) == 0);
  bad = c;
  bad.coarse_op = 7;
  CHECK(tomg_workspace_bytes(&bad) == 0);
  bad = c;
  bad.precision = TOMG_FP32_IR;
  bad.ir_inner_cycles = 0;
  CHECK(tomg_workspace_bytes(&bad) == 0);
  CHECK(tomg_workspace_bytes(nullptr) == 0);
  CHECK(tomg_num_levels(nullptr) == 0);
  // create: argument checks before any device work
  const size_t need = tomg_workspace_bytes(&c);
  tomg_problem *h = nullptr;
  CHECK(tomg_create(&c, nullptr, need, nullptr, &h) == TOMG_EINVAL);
  CHECK(tomg_create(&c, (void *)(uintptr_t)0x1008, need, nullptr, &h) == TOMG_EINVAL);
  CHECK(tomg_create(&c, (void *)(uintptr_t)0x100000, need - 256, nullptr, &h) == TOMG_ENOMEM);
  CHECK(tomg_create(nullptr, (void *)(uintptr_t)0x100000, need, nullptr, &h) == TOMG_EINVAL);
  CHECK(h == nullptr);
  // calls on a null problem
  CHECK(setup_coeffs(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
        TOMG_EINVAL);
  CHECK(vcycle(nullptr, nullptr) == TOMG_EINVAL);
  CHECK(solve(nullptr, nullptr, 1e-10, 10, nullptr, nullptr) == TOMG_EINVAL);
  CHECK(residual_norm(nullptr, nullptr, nullptr, nullptr) == TOMG_EINVAL);
  CHECK(tomg_setup_check(nullptr) == TOMG_EINVAL);
  CHECK(tomg_update_rhs(nullptr, nullptr) == TOMG_EINVAL);
  CHECK(std::strcmp(tomg_last_error(nullptr), "null problem") == 0);
  tomg_map_desc m{};
  tomg_source_desc s{};
  CHECK(tomg_setup_coeffs_desc(nullptr, &m, &s, nullptr, 0) == TOMG_EINVAL);
  CHECK(tomg_update_rhs_desc(nullptr, &s) == TOMG_EINVAL);
  CHECK(tomg_solve_batch(nullptr, nullptr, 1, 1e-10, 10, nullptr, nullptr, nullptr) ==
        TOMG_EINVAL);
  CHECK(tomg_solve_batch(nullptr, nullptr, 0, 1e-10, 10, nullptr, nullptr, nullptr) ==
        TOMG_EINVAL);
  // the allocation-free entry point: configuration and size checks first
  // (a stand-in device address: these calls return before any device work)
  char err[128];
  double *fake = (double *)(uintptr_t)0x100000;
  CHECK(tomg_solve_noalloc(&c, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                           1e-10, 10, nullptr, nullptr, nullptr, err, sizeof err) ==
        TOMG_EINVAL);
  CHECK(tomg_solve_noalloc(&bad, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, fake,
                           1e-10, 10, nullptr, nullptr, nullptr, err, sizeof err) ==
        TOMG_EINVAL);
  tomg_config big;
  tomg_config_default(&big, 8193, 8193, 1.0 / 8192, 1.0 / 8192);
  CHECK(tomg_solve_noalloc(&big, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, fake,
                           1e-10, 10, nullptr, nullptr, nullptr, err, 8) == TOMG_ENOMEM);
  CHECK(std::strlen(err) == 7);  // truncated to the buffer
  if (failures) return 1;
  std::printf("abi driver: all checks ran\n");
  return 0;
}
