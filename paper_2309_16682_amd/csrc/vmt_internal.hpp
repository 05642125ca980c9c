// vmt_internal.hpp -- context services shared by the runtime's C++ files.
#pragma once

#include <cstdint>
#include <vector>

#include "vmt.h"
#include "vmt_launch.hpp"

namespace vmt {

// Record an error message for vmt_last_error and return `code`.
int set_error(int code, const char* fmt, ...);

// Variant and lane count of a registered state (VMT_ESTATE if unknown).
int ctx_state_info(vmt_ctx* ctx, const void* d_state, int* variant, uint32_t* M);

// Device copy of t^(2^k) mod mu for `variant` (cached by the context) and its degree.
int ctx_pow2_poly(vmt_ctx* ctx, int variant, uint32_t k, const uint64_t** d_poly, uint32_t* degree);

// VMT_EINVAL (with the message set) if a state pointer occurs twice in the list.
int reject_duplicate_states(void* const* d_states, size_t count);

// Device the context runs on (-1 for a host-only context).
int ctx_device(vmt_ctx* ctx);

// Batch launch shape in force for (variant, M, out_kind), with its grid.
void ctx_batch_shape(vmt_ctx* ctx, int variant, uint32_t M, int out_kind, BatchShape* out);

// Device table of t^(c 2^v) mod mu for c = 1..need (slot c - 1, kPolyWords words each) and the degrees.
// The table stays valid while the context lives (a larger request may move later calls to a new table).
int ctx_split_polys(vmt_ctx* ctx, int variant, int v, size_t need, const uint64_t** d_table,
                    std::vector<uint32_t>* degrees);

}  // namespace vmt
