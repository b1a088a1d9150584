// Host helpers shared by the single-problem and batched drivers of the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

#include "../../include/lqgrid.h"
#include "launch.h"

namespace lqg {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
constexpr int kMaxPasses = 64;  // outer refinement passes per solve

// Dimensions of a problem, false when a size is < 1.
bool make_dims(const lqgrid_problem_desc* d, Dims* D);
// Options with defaults filled in; validity (S >= 1, even L >= 2, tol > 0).
void opts_fill(const lqgrid_solve_opts* in, lqgrid_solve_opts* o);
bool opts_valid(const lqgrid_solve_opts& o);
// Record a HIP failure for lqgrid_last_error; returns LQGRID_EHIP.
int hip_fail(hipError_t e, const char* where);
// Drop an error left behind by earlier, unrelated runtime calls of the
// process (e.g. a not-ready status of a query) so that the checks after it
// see only this library's launches.
inline void clear_stale_error() { (void)hipGetLastError(); }

}  // namespace lqg

#define HIPCHECK(x)                                          \
  do {                                                       \
    hipError_t e_ = (x);                                     \
    if (e_ != hipSuccess) return lqg::hip_fail(e_, #x);      \
  } while (0)
