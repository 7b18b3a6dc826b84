// Exercises libcmif's host-side code under AddressSanitizer and
// UndefinedBehaviorSanitizer: plan construction and validation over valid,
// ragged, windowed and invalid descriptions (every field out of range),
// workspace sizes and plan queries, the corner-error measure, status
// strings.  cmif_plan touches no device, so no GPU is needed.  Any
// sanitizer report aborts the run.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "cmif.h"

static int plans = 0, rejected = 0;

static void try_plan(cmif_plan_desc d) {
  cmif_plan_t p = nullptr;
  const cmif_status s = cmif_plan(&d, &p);
  if (s == CMIF_OK) {
    ++plans;
    size_t a = 0, b = 0;
    if (cmif_workspace_size(p, &a, &b) != CMIF_OK) std::abort();
    cmif_plan_info info;
    if (cmif_plan_query(p, &info) != CMIF_OK) std::abort();
    (void)cmif_profile_enable(p, 1);
    cmif_stage_time t[4];
    int32_t n = 0;
    (void)cmif_profile_read(p, t, 4, &n);
    cmif_plan_free(p);
  } else {
    ++rejected;
    if (p != nullptr) std::abort();
    (void)cmif_last_error();
  }
  (void)cmif_status_string(s);
}

int main() {
  const int32_t sides[][4] = {{1, 1, 1, 1}, {64, 64, 64, 64}, {37, 53, 29, 61},
                              {300, 280, 310, 290}, {1, 2048, 1, 1},
                              {2048, 5, 1, 5}, {1025, 5, 1025, 5}, {0, 5, 5, 5},
                              {5, 5, 2049, 5}, {700, 60, 650, 80}};
  const double angles[] = {0.0, 0.3, -2.0, 3.14159, NAN};
  const int32_t windows[][4] = {{0, 0, 0, 0}, {-3, 3, -2, 2}, {500, 500, 500, 500},
                                {5, 4, 0, 0}, {-4000, 0, 0, 0}};
  for (const auto& s : sides)
    for (int qa : {0, 1, 4, 64, 65})
      for (int prec : {0, 1, 2})
        for (int mode : {0, 1, 2})
          for (int na : {1, 4, 5}) {
            cmif_plan_desc d{};
            d.n_pairs = 1;
            d.h_a = &s[0]; d.w_a = &s[1]; d.h_b = &s[2]; d.w_b = &s[3];
            d.q_a = qa; d.q_b = 5;
            d.n_angles = na; d.angles_rad = angles;
            d.gamma = 0.5; d.precision = prec; d.mode = mode;
            d.flags = (na == 4) ? CMIF_FLAG_AUTOTUNE : 0;
            try_plan(d);
            for (const auto& w : windows) {
              d.window = w;
              try_plan(d);
            }
          }
  // other fields out of range
  const int32_t s1 = 40;
  cmif_plan_desc d{};
  d.n_pairs = 1; d.h_a = d.w_a = d.h_b = d.w_b = &s1; d.q_a = d.q_b = 3;
  d.n_angles = 1; d.gamma = 0.5;
  for (double g : {-0.1, 1.5, (double)NAN}) { cmif_plan_desc e = d; e.gamma = g; try_plan(e); }
  for (int32_t c : {-1, 4097, 7}) { cmif_plan_desc e = d; e.fallback_capacity = c; try_plan(e); }
  for (uint32_t f : {1u << 9, (uint32_t)CMIF_FLAG_PLAIN_SCHEDULE,
                     (uint32_t)CMIF_FLAG_SAVE_FOR_BACKWARD}) {
    cmif_plan_desc e = d; e.flags = f; try_plan(e);
    e.mode = CMIF_MODE_SOFT; try_plan(e);
  }
  { cmif_plan_desc e = d; e.n_pairs = 0; try_plan(e); }
  { cmif_plan_desc e = d; e.h_a = nullptr; try_plan(e); }
  { cmif_plan_desc e = d; e.angle_batch = -1; try_plan(e); }
  { cmif_plan_desc e = d; e.tune_cache_path = "/nonexistent/dir/tune.txt";
    e.flags = CMIF_FLAG_AUTOTUNE; try_plan(e); }
  if (cmif_plan(nullptr, nullptr) == CMIF_OK) return 1;
  // corner error
  cmif_best b{};
  b.angle_index = 3; b.angle_rad = 0.7; b.dy = -4; b.dx = 9;
  const double truth[6] = {1, 0, 2, 0, 1, -3};
  double e = 0;
  if (cmif_corner_error(&b, 50, 60, 40, 70, truth, &e) != CMIF_OK || !(e >= 0))
    return 2;
  if (cmif_corner_error(&b, 0, 60, 40, 70, truth, &e) == CMIF_OK) return 3;
  if (cmif_corner_error(nullptr, 5, 5, 5, 5, truth, &e) == CMIF_OK) return 4;
  std::printf("plan sanitizer driver ok: %d plans, %d rejected\n", plans, rejected);
  return 0;
}
