// Split-precision product (internal to libmmm).
#pragma once

#include "common.h"

namespace mmm {

constexpr int kMaxSlices = 8;

size_t split_workspace_bytes(i64 N, i64 P, i64 M, const mmm_config& c);
hipError_t run_split(const double* A, const double* B, double* C, i64 N, i64 P, i64 M, const mmm_config& c,
                     char* ws, hipStream_t s);

}  // namespace mmm
