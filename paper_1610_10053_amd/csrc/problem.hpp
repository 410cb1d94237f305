// Library-internal entry points shared by the C-ABI and the serving runtime.
#pragma once
#include <cstddef>

#include "../../include/jfnk.h"

namespace jfnk {
// Device bytes a problem carved from a caller-provided range needs
// (footprint plus per-buffer alignment); 0 for an invalid problem.
size_t problem_range_bytes(const jfnk_problem_desc* desc, const jfnk_solver_opts* opts);
// Pinned host bytes a problem uses for its scalar read-backs: a staging
// area for copies and the area the device's final reductions write into.
constexpr size_t kPinnedBytes = 2 * 512 * sizeof(double);
// jfnk_create_problem, with every device buffer carved from
// [range, range + range_bytes) when range is not null, and the scalar
// read-back area at pinned_host (kPinnedBytes of pinned host memory) when it
// is not null.  Neither is freed at destruction: both stay the caller's.
int create_problem_in(const jfnk_problem_desc* desc, const jfnk_solver_opts* opts, const double* u0,
                      int on_device, void* hip_stream, void* range, size_t range_bytes, void* pinned_host,
                      jfnk_problem** out);
// Thread-local error message setter of the library.
int set_error(int code, const char* msg);
}  // namespace jfnk
