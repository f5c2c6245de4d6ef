// Block passes compiled at run time from their op lists (see jit.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "plan.h"

namespace svj {

// Source text of the kernel for pass s of plan (complex64: dtype 0).
std::string generate(const svp::Step &s, const svp::Plan &plan, int dtype);

// Compile (or fetch from the cache) the kernels of every block pass of the
// plan, as one module; handles[i] identifies step i's kernel for launch()
// (nullptr for steps that are not block passes). On a compile error, *err
// holds the compiler log.
// compile_ms (optional) receives the compile time, 0 on a cache hit.
hipError_t prepare_plan(const svp::Plan &plan, int dtype, std::vector<const void *> &handles, std::string *err,
                        double *compile_ms = nullptr);

// Compile the plan's passes without loading them (no device needed); the
// compiler's own on-disk cache keeps the result for later prepare_plan calls.
hipError_t precompile(const svp::Plan &plan, int dtype, std::string *err);

// Unload all but the `keep` most recently used modules (synchronizes the
// device first).
hipError_t trim_cache(size_t keep);

// Source of all block passes of a plan (what prepare_plan compiles).
std::string generate_plan(const svp::Plan &plan, int dtype);

// Launch a prepared pass on `st` with a persistent grid.
hipError_t launch(const void *handle, void *S, const svp::K2Args &a, hipStream_t st);

size_t cache_size();

// Compile only (no device needed); "" on success, else the compiler log.
std::string compile_check(const std::string &src);

}  // namespace svj
