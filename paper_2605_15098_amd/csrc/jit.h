// Block passes compiled at run time from their op lists (see jit.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "plan.h"

namespace svj {

// Source text of the kernel for pass s of plan (complex64: dtype 0).
std::string generate(const svp::Step &s, const svp::Plan &plan, int dtype);

// Compile (or fetch from the cache) the kernel of pass s; *handle identifies
// it for launch(). On a compile error, *err holds the compiler log.
hipError_t prepare(const svp::Step &s, const svp::Plan &plan, int dtype, const void **handle, std::string *err);

// Launch a prepared pass on `st` with a persistent grid.
hipError_t launch(const void *handle, void *S, const svp::K2Args &a, hipStream_t st);

size_t cache_size();

// Compile only (no device needed); "" on success, else the compiler log.
std::string compile_check(const std::string &src);

}  // namespace svj
