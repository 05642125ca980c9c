// vmt_common.hpp -- state layout shared by the host runtime and the kernels.
//
// A V-state (Sec. 3) is M base generators ("lanes") advanced in lock step.
// Device layout: a 256-byte header, then the lane-interleaved window of the
// current block, word k of lane t at index k*M + t (the paper's interleaved
// state X-hat, Sec. 3). Because the round robin of eq. (combseq) polls lane
// 0..M-1 for word k before word k+1, the window in this layout *is* the next
// n*M stream elements in stream order.
//
// Position: `pos` counts the elements of the current block already emitted
// (0..block). A fresh state holds its first twisted block with pos = 0, so
// every window word is a genuine recurrence output.
#pragma once

#include <cstdint>

namespace vmt {

enum : uint32_t { kMT32 = 0, kMT64 = 1, kSFMT = 2 };
constexpr uint32_t kMagic = 0x31544d56u;  // "VMT1"
constexpr uint32_t kVersion = 1;
constexpr uint32_t kHeaderBytes = 256;
constexpr int kMaxLanes = 64;
constexpr int kPolyWords = 320;  // device polynomial slot: 20480 coefficients

struct StateHeader {
    uint32_t magic;
    uint32_t version;
    uint32_t variant;
    uint32_t M;           // lanes
    uint32_t n;           // words per lane in a block
    uint32_t word_bytes;  // 4, 8 or 16
    uint32_t block;       // stream elements per block: n*M (MT), 4*n*M (SFMT, uint32 units)
    uint32_t pos;         // elements of the current block already emitted
    uint32_t reserved[56];
};
static_assert(sizeof(StateHeader) == kHeaderBytes, "header size");

inline uint32_t words_per_lane(uint32_t variant) { return variant == kMT32 ? 624 : variant == kMT64 ? 312 : 156; }
inline uint32_t word_bytes(uint32_t variant) { return variant == kMT32 ? 4 : variant == kMT64 ? 8 : 16; }
inline uint32_t elems_per_word(uint32_t variant) { return variant == kSFMT ? 4 : 1; }

// One unit of batched work: a state, its output buffer and element count.
// If `flag` is set (host-visible memory), the workgroup adds 1 to it with
// system-scope release once the task's outputs and state are written (several
// tasks may count into one flag).
struct BatchTask {
    uint8_t* state;
    void* out;
    uint64_t len;
    uint32_t* flag;
};

// Copy of a whole state from src to dst.
struct CopyTask {
    const uint8_t* src;
    uint8_t* dst;
};

// One jump on one state: lane t uses polynomial slot poly[t] of the table
// (the same slot for every lane of an ordinary jump). `flag` as for BatchTask.
struct JumpTask {
    uint8_t* state;
    const uint64_t* poly;  // kPolyWords words; lanes use poly + lane_stride * t
    uint32_t lane_stride;  // 0: one polynomial for all lanes
    uint32_t max_deg;      // highest degree among the lanes' polynomials
    uint32_t* flag;
};

}  // namespace vmt
