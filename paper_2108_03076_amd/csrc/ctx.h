// Accessors of the opaque context for library parts outside api.cpp.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

struct pmc_ctx;

namespace pmc {
hipStream_t ctx_stream(const pmc_ctx* c);
int ctx_device(const pmc_ctx* c);
int ctx_fail(pmc_ctx* c, int status, const std::string& msg);
}  // namespace pmc
