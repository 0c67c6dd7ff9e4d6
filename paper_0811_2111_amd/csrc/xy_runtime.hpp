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
xy_plan default_plan(int32_t L, int32_t precision);
bool plan_ok(int32_t L, const xy_plan& p);
bool cache_lookup(const char* path, int32_t L, int32_t precision, xy_plan* plan);
const char* env_cache_path();
// xy_attach + xy_sweep on a handle that lives on the stack, with `work` as its
// workspace (zeroed counters first) and the default plan: no host or device
// allocation, no file access.  Arguments as xy_attach / xy_sweep, validated.
int sweep_on_work(uint64_t seed, int32_t L, double beta, double delta, int32_t precision, uint64_t sweep,
                  int64_t n_sweeps, int32_t measure_every, void* state_dev, size_t state_len, void* work,
                  size_t work_len, xy_obs* obs_dev, hipStream_t stream);

}  // namespace xyr
