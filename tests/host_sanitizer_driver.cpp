// Host-side checks of the library's entry points that run without a GPU.  Built together with a
// host-only build of the library under AddressSanitizer and UndefinedBehaviorSanitizer (see
// test_host_sanitizers.py): parameter validation and workspace sizing over a sweep of shapes, plan
// creation with invalid arguments, every entry point called with a NULL plan, and the error strings.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>

#include "recon.h"
#include "recon_cnn.h"

static int failures = 0;
#define CHECK(c)                                                              \
  do {                                                                        \
    if (!(c)) {                                                               \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);     \
      ++failures;                                                             \
    }                                                                         \
  } while (0)

static recon_params_t base(int n) {
  recon_params_t p;
  std::memset(&p, 0, sizeof p);
  p.n = n;
  p.batch = 1;
  p.box_len = 1000.0;
  p.observer[0] = p.observer[1] = p.observer[2] = 500.0;
  p.bias = 2.0;
  p.growth = 0.7;
  p.smooth_r = 10.0;
  p.mask_tau = 0.1;
  return p;
}

int main() {
  const double nan = std::numeric_limits<double>::quiet_NaN(), inf = std::numeric_limits<double>::infinity();

  // valid shapes: a positive size that grows with the batch and with max_objects
  const uint32_t flag_sets[] = {0u,
                                RECON_NO_RANDOMS,
                                RECON_KEEP_DELTA | RECON_START_BUFFERS,
                                RECON_KEEP_DELTA | RECON_START_BUFFERS | RECON_CNN_BUFFERS,
                                RECON_KEEP_DELTA | RECON_START_BUFFERS | RECON_CNN_BUFFERS | RECON_CNN_HALF,
                                RECON_PASS_GRAPHS | RECON_LOGNORMAL | RECON_RELAXED};
  const int batches[] = {1, 2, 7, 256};
  const int64_t objects[] = {0, 1000, (1LL << 32) - 1};
  for (int n = 8; n <= 1024; n *= 2)
    for (int batch : batches)
      for (int64_t mo : objects)
        for (uint32_t f : flag_sets) {
          recon_params_t p = base(n);
          p.batch = batch;
          p.max_objects = mo;
          p.flags = f;
          const size_t s = recon_workspace_bytes(&p);
          const bool ok = !(f & RECON_CNN_BUFFERS) || n >= ((f & RECON_CNN_HALF) ? 32 : 16);
          CHECK((s > 0) == ok);
          if (s > 0 && batch > 1) {
            recon_params_t q = p;
            q.batch = 1;
            CHECK(recon_workspace_bytes(&q) < s);
          }
          if (s > 0 && mo > 0) {
            recon_params_t q = p;
            q.max_objects = 0;
            CHECK(recon_workspace_bytes(&q) < s);
          }
        }

  // invalid parameters: size 0
  CHECK(recon_workspace_bytes(nullptr) == 0);
  const int bad_n[] = {0, 4, 7, 12, 2048, -8};
  for (int n : bad_n) {
    recon_params_t p = base(8);
    p.n = n;
    CHECK(recon_workspace_bytes(&p) == 0);
  }
  {
    recon_params_t p = base(64);
    p.batch = 0;
    CHECK(recon_workspace_bytes(&p) == 0);
    p = base(64);
    p.batch = -3;
    CHECK(recon_workspace_bytes(&p) == 0);
    const double bad_len[] = {0.0, -1.0, nan, inf};
    for (double v : bad_len) {
      p = base(64);
      p.box_len = v;
      CHECK(recon_workspace_bytes(&p) == 0);
    }
    p = base(64);
    p.bias = 0.0;
    CHECK(recon_workspace_bytes(&p) == 0);
    p = base(64);
    p.bias = nan;
    CHECK(recon_workspace_bytes(&p) == 0);
    p = base(64);
    p.growth = -0.1;
    CHECK(recon_workspace_bytes(&p) == 0);
    p = base(64);
    p.smooth_r = -1.0;
    CHECK(recon_workspace_bytes(&p) == 0);
    p = base(64);
    p.mask_tau = nan;
    CHECK(recon_workspace_bytes(&p) == 0);
    p = base(64);
    p.observer[1] = inf;
    CHECK(recon_workspace_bytes(&p) == 0);
    p = base(64);
    p.box_origin[2] = nan;
    CHECK(recon_workspace_bytes(&p) == 0);
    p = base(64);
    p.flags = 1u << 30;
    CHECK(recon_workspace_bytes(&p) == 0);
    p = base(64);
    p.flags = RECON_CNN_HALF;
    CHECK(recon_workspace_bytes(&p) == 0);
    p = base(64);
    p.max_objects = -1;
    CHECK(recon_workspace_bytes(&p) == 0);
    p = base(64);
    p.max_objects = 1LL << 32;
    CHECK(recon_workspace_bytes(&p) == 0);
  }

  // plan creation fails on its arguments before any device call
  alignas(256) static char ws[1024];
  recon_params_t p = base(64);
  CHECK(recon_plan(nullptr, &p, ws, sizeof ws, nullptr) == RECON_EINVAL);
  recon_plan_t* pl = reinterpret_cast<recon_plan_t*>(&p);
  CHECK(recon_plan(&pl, nullptr, ws, sizeof ws, nullptr) == RECON_EINVAL);
  CHECK(pl == nullptr);
  CHECK(recon_plan(&pl, &p, nullptr, 1u << 20, nullptr) == RECON_EINVAL);
  CHECK(recon_plan(&pl, &p, ws + 16, sizeof ws - 16, nullptr) == RECON_EINVAL);   // not 256-byte aligned
  CHECK(recon_plan(&pl, &p, ws, sizeof ws, nullptr) == RECON_ENOMEM);             // far too small
  CHECK(pl == nullptr);

  // the no-allocation plan checks its arguments and its scratch size before any device call
  CHECK(recon_noalloc_limit() == (size_t)64 << 20);
  CHECK(recon_plan_noalloc(nullptr, &p, nullptr) == RECON_EINVAL);
  CHECK(recon_plan_noalloc(&pl, nullptr, nullptr) == RECON_EINVAL);
  CHECK(pl == nullptr);
  {
    recon_params_t q = base(512);                          // 512^3 needs gigabytes
    CHECK(recon_plan_noalloc(&pl, &q, nullptr) == RECON_ENOMEM);
    q = base(32);
    q.flags |= RECON_PASS_GRAPHS;
    CHECK(recon_plan_noalloc(&pl, &q, nullptr) == RECON_EINVAL);
    CHECK(pl == nullptr);
  }

  // every entry point rejects a NULL plan
  float f[4] = {0.f, 0.f, 0.f, 0.f};
  int64_t g[2] = {0, 0};
  double d[8] = {0.0};
  int32_t c[8] = {0};
  CHECK(recon_paint(nullptr, RECON_GAL, f, nullptr, 1, nullptr, 0) == RECON_EINVAL);
  CHECK(recon_solve(nullptr, RECON_START_PLAIN, nullptr) == RECON_EINVAL);
  CHECK(recon_iterate(nullptr, 3, 1e-3, c, d) == RECON_EINVAL);
  CHECK(recon_shift(nullptr, RECON_RAN, f, 1, nullptr, f, nullptr) == RECON_EINVAL);
  CHECK(recon_get_psi(nullptr, f) == RECON_EINVAL);
  {
    int64_t tc[4];
    CHECK(recon_tile_counts(nullptr, tc) == RECON_EINVAL);
  }
  CHECK(recon_get_grid(nullptr, RECON_GAL, g) == RECON_EINVAL);
  CHECK(recon_get_delta(nullptr, f) == RECON_EINVAL);
  CHECK(recon_set_delta(nullptr, f) == RECON_EINVAL);
  CHECK(recon_radial_ratio(nullptr, f, -1.0, 3.0, d) == RECON_EINVAL);
  CHECK(recon_helmholtz(nullptr, f, f, nullptr) == RECON_EINVAL);
  CHECK(recon_profile_start(nullptr) == RECON_EINVAL);
  CHECK(recon_profile_stop(nullptr, c, d, 8) == RECON_EINVAL);
  CHECK(recon_cnn_forward(nullptr, f, f, f, f) == RECON_EINVAL);
  CHECK(recon_cnn_train_step(nullptr, f, f, f, 1, 1e-3f, f, f, f, d, nullptr) == RECON_EINVAL);
  CHECK(recon_get_radial(nullptr, f) == RECON_EINVAL);
  CHECK(recon_restrict(nullptr, f, f) == RECON_EINVAL);
  CHECK(recon_prolong(nullptr, f, f) == RECON_EINVAL);
  recon_destroy(nullptr);

  // error strings and kernel names are never NULL
  for (int code = -16; code <= 16; ++code) {
    const char* s = recon_strerror(code);
    CHECK(s != nullptr && std::strlen(s) > 0);
  }
  CHECK(std::strcmp(recon_last_error(nullptr), "plan is NULL") == 0);
  for (int k = -4; k < 256; ++k) CHECK(recon_profile_kernel_name(k) != nullptr);

  if (failures) {
    std::fprintf(stderr, "%d host checks failed\n", failures);
    return 1;
  }
  std::printf("host checks passed\n");
  return 0;
}
