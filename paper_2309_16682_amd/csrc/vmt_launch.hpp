// vmt_launch.hpp -- host entry points into the HIP kernels (internal).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

#include "vmt_common.hpp"

namespace vmt {

// Seeding kinds for InitTask.
enum : uint32_t { kSeedGenrand = 0, kSeedByArray = 1 };

struct InitTask {
    uint8_t* state;
    const uint32_t* key;  // device array (init_by_array)
    uint64_t seed;        // init_genrand seed
    uint32_t kind;
    uint32_t key_len;
};

// Output kinds (same values as VMT_OUT_*).
enum : int { kOutU32 = 0, kOutU64 = 1, kOutF32 = 2, kOutF64 = 3 };

// Seed and de-phase `count` states: lane t of state i = X_0(i) advanced by
// t*J. lane_polys holds M slots of kPolyWords words (slot t = t^(tJ) mod mu).
// With d_tasks == nullptr the single task `one` (passed by value) is used.
hipError_t launch_init(uint32_t variant, uint32_t M, const InitTask* d_tasks, const InitTask& one, uint32_t count,
                       const uint64_t* d_lane_polys, uint32_t max_deg, hipStream_t stream);

// Jump `count` states (all of one variant and M), then fix their positions.
// d_parts: device scratch of jump_parts_bytes(variant, M, count) bytes, or
// nullptr. With it, MT jumps of few lanes split each lane's sum over several
// workgroups (partial windows in d_parts, XORed by a second launch); the
// scratch is in use until the launches have run. Tasks with a completion flag
// need d_parts == nullptr.
hipError_t launch_jump(uint32_t variant, uint32_t M, const JumpTask* d_tasks, const JumpTask& one, uint32_t count,
                       hipStream_t stream, void* d_parts = nullptr);
uint32_t jump_parts(uint32_t variant, uint32_t M, uint64_t count);       // workgroups per lane jump
size_t jump_parts_bytes(uint32_t variant, uint32_t M, uint64_t count);   // 0: no scratch needed
size_t split_jump_parts_bytes(uint32_t variant, uint32_t M, uint64_t count);  // d_parts of launch_split_jump

// Set-up of a split call: C chunks of E elements (the last n - (C-1) E) of
// eb bytes into d_out; generation tasks d_bt[C], jump tasks d_jt[C-1] (chunk
// c >= 1 jumped by d_polys slot c - 1, degree d_deg[c - 1]), and the state
// (bytes, a multiple of 16) copied to the C - 1 slots of d_copies, `stride`
// bytes apart, for chunks 0 .. C-2 (the last chunk runs on d_state); d_done
// (C counters, or nullptr) is zeroed for launch_batch_gen_mt.
hipError_t launch_split_setup(const uint8_t* d_state, uint8_t* d_copies, uint32_t bytes, uint64_t stride, uint32_t C,
                              uint8_t* d_out, uint64_t E, uint64_t n, uint32_t eb, const uint64_t* d_polys,
                              const uint32_t* d_deg, BatchTask* d_bt, JumpTask* d_jt, uint32_t* d_done,
                              hipStream_t stream);

// Jump `count` copies of one state, each by its own polynomial (the chunks of
// a split call), then fix their positions. d_src holds the window all copies
// start from and is not one of them. d_parts as for launch_jump.
hipError_t launch_split_jump(uint32_t variant, uint32_t M, const uint8_t* d_src, const JumpTask* d_tasks,
                             const JumpTask& one, uint32_t count, hipStream_t stream, void* d_parts = nullptr);

// Generate `len` elements from one state into d_out with `lpw` lanes per
// workgroup (lpw divides M; lpw == M uses one workgroup).
hipError_t launch_generate(uint32_t variant, uint32_t M, uint32_t lpw, int out_kind, uint8_t* d_state,
                           void* d_out, uint64_t len, hipStream_t stream);

// Launch shape of the persistent batch kernel: tv selects threads per
// workgroup (batch_threads), sw the bytes per output store (16 or 8), grid
// the number of resident workgroups (capped at the task count).
struct BatchShape {
    uint32_t tv = 0;
    uint32_t sw = 16;
    uint32_t grid = 0;
};

// Linear-complexity self-check: count the offsets x < nw - deg S of the
// stream's 32-bit words w (out_kind gives the element type) where the XOR of
// w[x + i S] over the set coefficients i of A is nonzero. *d_count is
// overwritten (a fill kernel, not a memset).
constexpr uint32_t kCheckChunkBits = 4096;
struct CheckPolyDev {
    uint32_t deg = 0;
    bool dense = false;                // dense form (bit pattern) or sparse form (coefficient list)
    const uint32_t* bits = nullptr;    // deg + 1 bits as uint32 words, zero-padded to kCheckChunkBits
    const uint32_t* terms = nullptr;   // set coefficients, increasing
    const uint32_t* term_off = nullptr;  // deg / kCheckChunkBits + 2 entries: terms of chunk c start at term_off[c]
};
// cus: compute units of the device (the grid is a few workgroups per CU).
hipError_t launch_check(int out_kind, const void* src, uint64_t nw, uint32_t S, const CheckPolyDev& poly,
                        unsigned long long* d_count, uint32_t cus, hipStream_t stream);

// Persistent batched generation. d_counter points to two uint32 that must be
// zero before the first launch (reset_counters); every launch leaves them zero.
hipError_t reset_counters(uint32_t* d_counter, hipStream_t stream);
hipError_t launch_batch(uint32_t variant, uint32_t M, int out_kind, const BatchShape& shape, const BatchTask* d_tasks,
                        uint32_t count, uint32_t* d_counter, hipStream_t stream);

// MT19937-32/-64 tasks by lane groups: M / lpw workgroups per task, each
// running lpw lanes (lpw a power of two dividing M, at most 16); positions
// are maintained like launch_generate's. With lpw < M the positions are fixed
// by a second launch, or, given d_done (count counters, zeroed), by the last
// workgroup of each task.
hipError_t launch_batch_gen_mt(uint32_t variant, uint32_t M, uint32_t lpw, int out_kind, const BatchTask* d_tasks,
                               uint32_t count, hipStream_t stream, uint32_t* d_done = nullptr);

// Batched SFMT generation (one lane group of lpw lanes per workgroup, tasks
// of one M); positions are maintained like launch_generate's.
hipError_t launch_batch_sfmt(uint32_t variant, uint32_t M, uint32_t lpw, int out_kind, const BatchTask* d_tasks,
                             uint32_t count, hipStream_t stream);

// Measurement only. launch_write_pattern: the batch kernel's memory traffic
// for the same tasks and shape without the twist (states unchanged;
// V-MT19937-32 M = 16 and V-MT19937-64 M = 8 integer outputs).
// launch_fill: a write of `bytes` (a multiple of 16) with 16-byte stores;
// mode bit 0: 4 KiB pieces in order (0) or two contiguous regions per CU
// (1), bit 1: nontemporal stores.
bool pattern_supported(uint32_t variant, uint32_t M, int out_kind);
hipError_t launch_write_pattern(uint32_t variant, uint32_t M, int out_kind, const BatchShape& shape,
                                const BatchTask* d_tasks, uint32_t count, uint32_t* d_counter, hipStream_t stream);
hipError_t launch_fill(void* d_buf, uint64_t bytes, int mode, uint32_t cus, hipStream_t stream);

// Allocation-free batch call. The task list and counters live in a
// file-scope device array of kNoAllocMaxTasks tasks, one per device, shared
// by every call on that device. noalloc_scratch_init looks its address up for
// `device` (which must be current) once; noalloc_scratch returns it
// (hipErrorNotInitialized before init).
constexpr uint32_t kNoAllocMaxTasks = 32768;
hipError_t noalloc_scratch_init(int device);
hipError_t noalloc_scratch(int device, BatchTask** d_tasks, uint32_t** d_counter);

// Copy states: task i copies tasks[i].src to tasks[i].dst (bytes, a multiple of 16).
hipError_t launch_copy_states(const CopyTask* d_tasks, uint32_t count, uint32_t bytes, hipStream_t stream);

// Whether the combination is compiled in; threads and occupancy of a shape.
bool generate_supported(uint32_t variant, uint32_t M, uint32_t lpw, int out_kind);
bool batch_supported(uint32_t variant, uint32_t M, int out_kind);
bool batch_shape_supported(uint32_t variant, uint32_t M, int out_kind, uint32_t tv, uint32_t sw);
uint32_t batch_threads(uint32_t variant, uint32_t M, int out_kind, uint32_t tv, uint32_t sw);
uint32_t batch_max_per_cu(uint32_t variant, uint32_t M, int out_kind, uint32_t tv, uint32_t sw);
uint32_t device_cus(int device);

}  // namespace vmt
