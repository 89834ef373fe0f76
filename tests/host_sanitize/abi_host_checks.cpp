// Host-side checks of the C ABI under AddressSanitizer and UndefinedBehavior-
// Sanitizer: every argument-validation path, the footprint arithmetic over a
// sweep of grids, and plan creation without a usable GPU (which must fail
// cleanly with GPS_E_DEVICE).  No kernel is launched.  Exit status 0 = pass.
#include <cstdio>
#include <cstring>
#include <initializer_list>

#include "gps.h"

static int failures = 0;
#define EXPECT(cond)                                                   \
  do {                                                                 \
    if (!(cond)) {                                                     \
      std::fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                      \
    }                                                                  \
  } while (0)

int main() {
  for (int st = -2; st < 12; ++st) EXPECT(gps_status_string(st) != nullptr);

  // footprint arithmetic over grids, boundary conditions and options
  const int sizes[] = {2, 3, 5, 8, 16, 33, 96, 160, 300, 512};
  size_t total_checked = 0;
  for (int nx : sizes)
    for (int ny : {2, 17, 96})
      for (int nz : {2, 24, 160})
        for (int bc = 0; bc < 4; ++bc)
          for (int prec = 0; prec < 2; ++prec)
            for (int flags = 0; flags < 4; ++flags) {
              size_t t = 0, b = 0, tr = 0;
              EXPECT(gps_plan_footprint(nx, ny, nz, bc, prec, 1000, flags & 1, flags >> 1, &t, &b,
                                        &tr) == GPS_OK);
              EXPECT(t > 0 && b > 0);
              EXPECT(gps_plan_footprint(nx, ny, nz, bc, prec, 1, 0, 0, nullptr, nullptr,
                                        nullptr) == GPS_OK);
              ++total_checked;
            }
  EXPECT(gps_plan_footprint(1, 8, 8, 0, 0, 10, 0, 0, nullptr, nullptr, nullptr) == GPS_E_INVALID);
  EXPECT(gps_plan_footprint(8, 8, 8, 4, 0, 10, 0, 0, nullptr, nullptr, nullptr) == GPS_E_INVALID);
  EXPECT(gps_plan_footprint(8, 8, 8, 0, 2, 10, 0, 0, nullptr, nullptr, nullptr) == GPS_E_INVALID);
  EXPECT(gps_plan_footprint(8, 8, 8, 0, 0, 0, 0, 0, nullptr, nullptr, nullptr) == GPS_E_INVALID);

  // plan creation: invalid arguments, unsupported lengths
  gps_plan* p = reinterpret_cast<gps_plan*>(0x1);
  EXPECT(gps_plan_create(1, 8, 8, 0.5, 0, &p) == GPS_E_INVALID && p == nullptr);
  EXPECT(gps_plan_create(8, 8, 8, -1.0, 0, &p) == GPS_E_INVALID);
  EXPECT(gps_plan_create(8, 8, 8, 0.5, 7, &p) == GPS_E_INVALID);
  EXPECT(gps_plan_create(8, 8, 8, 0.5, 0, nullptr) == GPS_E_INVALID);
  EXPECT(gps_plan_create(11, 8, 8, 0.5, 0, &p) == GPS_E_UNSUPPORTED);
  // a valid plan either builds (a GPU is present) or fails cleanly
  gps_plan* q = nullptr;
  const int st = gps_plan_create(8, 8, 8, 0.5, 0, &q);
  EXPECT(st == GPS_OK || st == GPS_E_DEVICE || st == GPS_E_NOMEM);
  EXPECT((st == GPS_OK) == (q != nullptr));
  if (q) gps_plan_destroy(q);

  // every entry point on a null plan
  gps_options o;
  std::memset(&o, 0, sizeof(o));
  gps_info info;
  double h[4];
  EXPECT(gps_plan_set_options(nullptr, &o) == GPS_E_INVALID);
  EXPECT(gps_plan_get_options(nullptr, &o) == GPS_E_INVALID);
  EXPECT(gps_plan_device_bytes(nullptr) == 0);
  EXPECT(gps_plan_release_buffers(nullptr) == GPS_E_INVALID);
  gps_plan_destroy(nullptr);
  EXPECT(gps_solve_generalized(nullptr, nullptr, nullptr, nullptr, 1e-6) == GPS_E_INVALID);
  EXPECT(gps_solve_generalized_q(nullptr, nullptr, nullptr, nullptr, nullptr, 1e-6) ==
         GPS_E_INVALID);
  EXPECT(gps_solve_pb(nullptr, nullptr, nullptr, nullptr, nullptr, 1e-6) == GPS_E_INVALID);
  EXPECT(gps_solve_vacuum(nullptr, nullptr, nullptr) == GPS_E_INVALID);
  EXPECT(gps_solve_sc(nullptr, nullptr, nullptr, nullptr, 1e-6, GPS_METHOD_SC, 0.6) ==
         GPS_E_INVALID);
  EXPECT(gps_rigid_cavity(nullptr, 1, nullptr, 0.5, 78.0, nullptr, nullptr) == GPS_E_INVALID);
  EXPECT(gps_polarization_charge(nullptr, nullptr, nullptr, nullptr, nullptr) == GPS_E_INVALID);
  EXPECT(gps_last_info(nullptr, &info) == GPS_E_INVALID);
  EXPECT(gps_last_history(nullptr, h, 1) == GPS_E_INVALID);
  EXPECT(gps_plan_set_timing(nullptr, 1) == GPS_E_INVALID);
  EXPECT(gps_plan_timing(nullptr, nullptr, nullptr, nullptr) == GPS_E_INVALID);

  // serving: invalid arguments
  gps_server* srv = nullptr;
  long long ticket = 0;
  gps_result res;
  EXPECT(gps_server_create(nullptr, nullptr) == GPS_E_INVALID);
  {
    // NULL options select the defaults: a server starts (GPU present) or fails cleanly
    const int s2 = gps_server_create(nullptr, &srv);
    EXPECT(s2 == GPS_OK || s2 == GPS_E_DEVICE);
    if (srv) gps_server_destroy(srv);
    srv = nullptr;
  }
  EXPECT(gps_server_submit(nullptr, nullptr, &ticket) == GPS_E_INVALID);
  EXPECT(gps_server_poll(nullptr, 1, &res) == GPS_E_INVALID);
  EXPECT(gps_server_wait(nullptr, 1, &res) == GPS_E_INVALID);
  EXPECT(gps_server_get_stats(nullptr, nullptr) == GPS_E_INVALID);
  gps_server_destroy(nullptr);

  std::printf("host checks: %zu footprints, %d failures\n", total_checked, failures);
  return failures == 0 ? 0 : 1;
}
