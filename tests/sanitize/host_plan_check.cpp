// Host-only exercise of the planner and the plan/geometry entry points of the
// C ABI, built with AddressSanitizer and UndefinedBehaviorSanitizer on the
// host side (no device calls: every plan is HDCONV_PLAN_HOST_ONLY).  Prints
// one line per family and "ok" at the end; the sanitizers abort on the first
// error.
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <initializer_list>

#include "hdconv.h"

static int fails = 0;

static void plan_one(int dims, const int64_t* L, const int64_t* M, int A, int dtype, int flags, int variant, int64_t m) {
  hdconv_options o;
  hdconv_options_init(&o);
  o.flags = flags | HDCONV_PLAN_HOST_ONLY;
  if (variant) {
    for (int d = 0; d < dims; ++d) o.variant[d] = d == dims - 1 ? variant : HDCONV_VARIANT_AUTO;
    if (m) o.m[dims - 1] = m;
  }
  hdconv_plan_t p = hdconv_plan_ex(L, M, A, 1, dims, dtype, &o);
  if (!p) return;  // unsupported shapes report an error; that path is exercised too
  hdconv_plan_info_t info;
  if (hdconv_plan_info(p, &info) != HDCONV_OK) ++fails;
  hdconv_destroy(p);
}

int main() {
  const int64_t lens[] = {1, 2, 3, 7, 8, 15, 16, 63, 64, 100, 127, 128, 255, 256, 1000, 1023, 1024, 1025,
                          2047, 2048, 3000, 4096, 5000, 8192, 10000, 65536, 100000, 1 << 20, 1500000};
  const int nl = (int)(sizeof(lens) / sizeof(lens[0]));
  int n = 0;
  for (int i = 0; i < nl; ++i)
    for (int A = 2; A <= 3; ++A)
      for (int dt = 0; dt <= 1; ++dt)
        for (int fl : {0, (int)HDCONV_PLAN_CENTERED, (int)HDCONV_PLAN_HERMITIAN}) {
          int64_t M = 0;
          if (hdconv_min_padding(lens[i], A, fl, &M) != HDCONV_OK) continue;
          for (int64_t f : {1, 2, 3}) {
            const int64_t L1[1] = {lens[i]}, M1[1] = {M * f};
            plan_one(1, L1, M1, A, dt, fl, 0, 0);
            plan_one(1, L1, M1, A, dt, fl, HDCONV_VARIANT_MULTIPASS, 1024);
            plan_one(1, L1, M1, A, dt, fl, HDCONV_VARIANT_FUSED, 0);
            n += 3;
            if (lens[i] <= 4096) {
              const int64_t L2[2] = {lens[i] | (fl == HDCONV_PLAN_HERMITIAN), lens[i]};
              int64_t Mo = 0;
              (void)hdconv_min_padding(L2[0], A, fl ? HDCONV_PLAN_CENTERED : 0, &Mo);
              const int64_t M2[2] = {Mo * f, M * f};
              plan_one(2, L2, M2, A, dt, fl, 0, 0);
              ++n;
            }
            if (lens[i] <= 256) {
              const int64_t L3[3] = {lens[i] | (fl == HDCONV_PLAN_HERMITIAN), lens[i] | (fl == HDCONV_PLAN_HERMITIAN),
                                     lens[i]};
              int64_t Mo = 0;
              (void)hdconv_min_padding(L3[0], A, fl ? HDCONV_PLAN_CENTERED : 0, &Mo);
              const int64_t M3[3] = {Mo * f, Mo * f, M * f};
              plan_one(3, L3, M3, A, dt, fl, 0, 0);
              ++n;
            }
          }
        }
  printf("plans: %d\n", n);
  // geometry entry points, including the paper's centered example (Sec. 7.2:
  // L = 2048, M = 3072, m = 16 spans 128 blocks folded onto p = 64, n = 3, q = 192)
  int ng = 0;
  for (int i = 0; i < nl; ++i)
    for (int64_t m : {8, 16, 64, 1024, 4096}) {
      hdconv_dim_info_t di;
      memset(&di, 0, sizeof(di));
      (void)hdconv_geometry(lens[i], 2 * lens[i], m, 0, 0, &di);
      (void)hdconv_geometry_ex(lens[i], 3 * lens[i] / 2 + 2, m, 0, 1, HDCONV_PLAN_CENTERED, &di);
      (void)hdconv_centered_span(lens[i], m);
      ng += 3;
    }
  {
    hdconv_dim_info_t di;
    if (hdconv_geometry_ex(2048, 3072, 16, 0, 1, HDCONV_PLAN_CENTERED, &di) != HDCONV_OK || di.p != 64 ||
        di.n != 3 || di.q != 192)
      ++fails;
  }
  printf("geometries: %d\n", ng);
  // invalid arguments: every entry point must refuse them without touching memory
  {
    const int64_t L1[1] = {0}, M1[1] = {0};
    if (hdconv_plan(L1, M1, 2, 1, 1, HDCONV_C64)) ++fails;
    if (hdconv_plan(nullptr, nullptr, 2, 1, 1, HDCONV_C64)) ++fails;
    int64_t M = 0;
    if (hdconv_min_padding(0, 2, 0, &M) == HDCONV_OK) ++fails;
    char msg[256];
    (void)hdconv_last_error(msg, sizeof(msg));
    (void)hdconv_last_error(msg, 1);
  }
  printf("%s (%d failures)\n", fails ? "FAIL" : "ok", fails);
  return fails ? 1 : 0;
}
