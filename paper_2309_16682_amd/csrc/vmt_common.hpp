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

// Variants: the paper's three base generators, then SFMT with the generator
// authors' parameter sets for the Mersenne exponents 607 ... 11213 (the same
// recurrence, eq. (sfmt_step), with other shifts, masks and state sizes).
enum : uint32_t {
    kMT32 = 0, kMT64 = 1, kSFMT = 2,
    kSFMT607 = 3, kSFMT1279 = 4, kSFMT2281 = 5, kSFMT4253 = 6, kSFMT11213 = 7,
    kVariants = 8
};

// An SFMT parameter set: N = mexp / 128 + 1 words of 128 bits, pick-up
// position pos1 (the paper's m), 32-bit sub-word shifts sl1 and sr1, 128-bit
// shifts by sl2 and sr2 bytes, mask msk (the paper's K), and the
// period-certification vector. SFMT19937 is eq. (sfmt_params); the parity
// vectors and the other sets are from the generator's authors (Saito and
// Matsumoto), each checked by the tests: the minimal polynomial of the
// one-step map has an irreducible factor of degree mexp, and the parity
// vector annihilates the rest.
struct SfmtSet {
    uint32_t mexp, n, pos1, sl1, sl2, sr1, sr2;
    uint32_t msk[4], parity[4];
};
constexpr SfmtSet kSfmtSets[6] = {
    {19937, 156, 122, 18, 1, 11, 1, {0xdfffffefu, 0xddfecb7fu, 0xbffaffffu, 0xbffffff6u},
     {0x00000001u, 0x00000000u, 0x00000000u, 0x13c9e684u}},
    {607, 5, 2, 15, 3, 13, 3, {0xfdff37ffu, 0xef7f3f7du, 0xff777b7du, 0x7ff7fb2fu},
     {0x00000001u, 0x00000000u, 0x00000000u, 0x5986f054u}},
    {1279, 10, 7, 14, 3, 5, 1, {0xf7fefffdu, 0x7fefcfffu, 0xaff3ef3fu, 0xb5ffff7fu},
     {0x00000001u, 0x00000000u, 0x00000000u, 0x20000000u}},
    {2281, 18, 12, 19, 1, 5, 1, {0xbff7ffbfu, 0xfdfffffeu, 0xf7ffef7fu, 0xf2f7cbbfu},
     {0x00000001u, 0x00000000u, 0x00000000u, 0x41dfa600u}},
    {4253, 34, 17, 20, 1, 7, 1, {0x9f7bffffu, 0x9fffff5fu, 0x3efffffbu, 0xfffff7bbu},
     {0xa8000001u, 0xaf5390a3u, 0xb740b3f8u, 0x6c11486du}},
    {11213, 88, 68, 14, 3, 7, 3, {0xeffff7fbu, 0xffffffefu, 0xdfdfbfffu, 0x7fffdbfdu},
     {0x00000001u, 0x00000000u, 0xe8148000u, 0xd0c7afa3u}},
};
constexpr bool is_sfmt(uint32_t variant) { return variant >= kSFMT && variant < kVariants; }
constexpr const SfmtSet& sfmt_set(uint32_t variant) { return kSfmtSets[variant - kSFMT]; }
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

inline uint32_t words_per_lane(uint32_t variant) {
    return variant == kMT32 ? 624 : variant == kMT64 ? 312 : sfmt_set(variant).n;
}
inline uint32_t word_bytes(uint32_t variant) { return variant == kMT32 ? 4 : variant == kMT64 ? 8 : 16; }
inline uint32_t elems_per_word(uint32_t variant) { return is_sfmt(variant) ? 4 : 1; }
// Mersenne exponent: the period is a multiple of 2^mexp - 1, and the lane
// distance of M lanes is J = 2^(mexp - log2 M) (Sec. 3, Table jvalues).
inline uint32_t mexp(uint32_t variant) { return is_sfmt(variant) ? sfmt_set(variant).mexp : 19937; }

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
