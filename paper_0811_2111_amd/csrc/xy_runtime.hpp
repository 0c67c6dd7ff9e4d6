// xy_runtime.hpp -- runtime helpers shared by the single-lattice and batch front ends.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xy.h"
#include "xy_launch.hpp"

namespace xyr {

int hip_fail(hipError_t e, const char* what);
// Failure injection (xy_test_inject_failure): true at the launch point that is
// due to fail; the caller then reports hipErrorLaunchFailure without launching.
bool inject_due();
// `expr` (a call returning hipError_t), or an injected launch failure.
#define XY_LAUNCH(expr) (xyr::inject_due() ? hipErrorLaunchFailure : (expr))
bool valid_L(int32_t L);
bool valid_beta_delta(double beta, double delta);
xyk::SweepArgs sweep_args(uint64_t seed, int L, int precision, double beta, double delta);
xy_plan default_plan(int32_t L);
bool plan_ok(int32_t L, const xy_plan& p);
bool cache_lookup(const char* path, int32_t L, int32_t precision, xy_plan* plan);
const char* env_cache_path();

}  // namespace xyr
