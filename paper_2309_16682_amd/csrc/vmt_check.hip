// vmt_check.hip -- gfx950 kernel of the linear-complexity self-check.
//
// Every output bit of an F2-linear generator, read along its stream, obeys
// the linear recurrence of a polynomial A (Sec. 4 reports the resulting
// LinearComp failures of every MT-based generator; Sec. 3.1 gives the
// polynomial view of the state map). Thirty-two bits are checked at once:
// for every offset x, XOR over the set coefficients i of A of the 32-bit
// words w[x + i S] must be zero.
//
// The work is a correlation of the word sequence with the bit pattern of A
// (about deg(A) / 2 ~ 10^4 set coefficients): plain integer ALU work, about
// 10^4 XORs per stream word, bound by the VALU and by LDS reads. No MFMA:
// the arithmetic is over GF(2).
//
// Mapping. The S phases of the stride are independent sequences; a
// workgroup takes a tile of kTile consecutive offsets of one phase, thread t
// the kR = 8 consecutive offsets kR t .. kR t + 7. The phase's words are
// staged in LDS in chunks of kChunk coefficients (kTile + kChunk words). For
// each 32-coefficient word of A (a wave-uniform scalar load) a thread reads
// its window of kR + 32 words with ds_read_b128 and, nibble by nibble, XORs
// the selected window words into its accumulators: the nibble's value picks
// one of 16 straight-line cases (a scalar branch), each combining up to four
// words per accumulator with three-input XORs, ~1.25 VALU ops per nibble and
// accumulator on average. LDS layout: word j sits in plane (j / 4) % 2 at
// 16-byte slot j / 8, so the window (five 8-word groups) is ten 16-byte
// reads at a 16-byte lane stride: no bank conflicts.
#include <hip/hip_runtime.h>

#include "vmt_launch.hpp"

namespace vmt {
namespace {

constexpr int kThreads = 256;
constexpr int kR = 8;                     // consecutive offsets per thread
constexpr int kTile = kThreads * kR;      // offsets per workgroup tile
constexpr int kChunk = kCheckChunkBits;   // coefficients staged per LDS fill
constexpr int kBuf = kTile + kChunk;      // LDS words per fill
constexpr int kWin = kR + 32;             // window words per 32 coefficients
static_assert(kChunk % 32 == 0 && kR == 8 && kBuf % 8 == 0, "window = 8-word groups");

// LDS slot of buffer word j: two planes of 4-word groups.
__device__ __forceinline__ uint32_t lds_slot(uint32_t j) {
    return ((j >> 2) & 1) * (kBuf / 2) + (j >> 3) * 4 + (j & 3);
}

// a ^ b ^ c in one VALU op (v_bitop3_b32, truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, (unsigned char)0x96);
}

// acc[r] ^= XOR over the set bits e of V of w[e + r], r < kR.
template <int V>
__device__ __forceinline__ void nibble(uint32_t (&acc)[kR], const uint32_t* w) {
    constexpr int n = __builtin_popcount(V);
    constexpr int e0 = V & 1 ? 0 : V & 2 ? 1 : V & 4 ? 2 : 3;           // lowest set bit
    constexpr int e3 = V & 8 ? 3 : V & 4 ? 2 : V & 2 ? 1 : 0;           // highest set bit
    constexpr int e1 = (V & ~(1 << e0)) & 2 ? 1 : (V & ~(1 << e0)) & 4 ? 2 : 3;  // second lowest
#pragma unroll
    for (int r = 0; r < kR; r++) {
        if constexpr (n == 1) {
            acc[r] ^= w[e0 + r];
        } else if constexpr (n == 2) {
            acc[r] = xor3(acc[r], w[e0 + r], w[e3 + r]);
        } else if constexpr (n == 3) {  // e0 < e1 < e3
            acc[r] = xor3(xor3(acc[r], w[e0 + r], w[e1 + r]), w[e3 + r], 0u);
        } else {
            acc[r] = xor3(xor3(acc[r], w[r], w[r + 1]), w[r + 2], w[r + 3]);
        }
    }
}

__device__ __forceinline__ void apply_nibble(uint32_t v, uint32_t (&acc)[kR], const uint32_t* w) {
    switch (v) {
        case 1: nibble<1>(acc, w); break;
        case 2: nibble<2>(acc, w); break;
        case 3: nibble<3>(acc, w); break;
        case 4: nibble<4>(acc, w); break;
        case 5: nibble<5>(acc, w); break;
        case 6: nibble<6>(acc, w); break;
        case 7: nibble<7>(acc, w); break;
        case 8: nibble<8>(acc, w); break;
        case 9: nibble<9>(acc, w); break;
        case 10: nibble<10>(acc, w); break;
        case 11: nibble<11>(acc, w); break;
        case 12: nibble<12>(acc, w); break;
        case 13: nibble<13>(acc, w); break;
        case 14: nibble<14>(acc, w); break;
        case 15: nibble<15>(acc, w); break;
        default: break;
    }
}

__device__ __forceinline__ uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// Word X of the stream: uint32 as is, float as its integer f 2^24, uint64 and
// double (f 2^53) as (low, high) halves. Both float maps are exact.
template <int KIND>
__device__ __forceinline__ uint32_t stream_word(const void* src, uint64_t X) {
    if constexpr (KIND == kOutU32) {
        return static_cast<const uint32_t*>(src)[X];
    } else if constexpr (KIND == kOutF32) {
        return (uint32_t)(static_cast<const float*>(src)[X] * 16777216.0f);
    } else if constexpr (KIND == kOutU64) {
        return (uint32_t)(static_cast<const uint64_t*>(src)[X >> 1] >> (32 * (X & 1)));
    } else {
        const uint64_t v = (uint64_t)(static_cast<const double*>(src)[X >> 1] * 9007199254740992.0);
        return (uint32_t)(v >> (32 * (X & 1)));
    }
}

__global__ void zero_count_kernel(unsigned long long* count) { *count = 0; }

// nw words in S phases; phase p holds words p, p + S, ...; A: deg + 1
// coefficients as uint32 words, zero-padded to a multiple of kChunk.
template <int KIND>
__global__ __launch_bounds__(kThreads) void check_kernel(const void* __restrict__ src, uint64_t nw, uint32_t S,
                                                        const uint32_t* __restrict__ A, uint32_t deg,
                                                        uint64_t tiles_per_phase, unsigned long long* count) {
    __shared__ __align__(16) uint32_t buf[kBuf];
    __shared__ unsigned long long wg_count;
    const uint32_t t = threadIdx.x;
    if (t == 0) wg_count = 0;
    unsigned long long local = 0;
    const uint64_t tiles = tiles_per_phase * S;
    for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const uint32_t p = (uint32_t)(tile / tiles_per_phase);
        const uint64_t k0 = (tile % tiles_per_phase) * kTile;
        const uint64_t nk = nw > p ? (nw - p + S - 1) / S : 0;  // words in phase p
        const uint64_t valid = nk > deg ? nk - deg : 0;          // offsets k < valid are checked
        if (k0 >= valid) continue;                               // the same for the whole workgroup
        uint32_t acc[kR] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (uint32_t i0 = 0; i0 <= deg; i0 += kChunk) {
            __syncthreads();  // the previous chunk's reads are done
            for (uint32_t j = t; j < (uint32_t)kBuf; j += kThreads) {
                const uint64_t k = k0 + i0 + j;
                buf[lds_slot(j)] = k < nk ? stream_word<KIND>(src, p + k * S) : 0u;
            }
            __syncthreads();
            const uint32_t* Ac = A + i0 / 32;
            for (int q = 0; q < kChunk / 32; q++) {
                const uint32_t a = uniform(Ac[q]);
                if (a == 0) continue;
                // window: buffer words 32 q + kR t + 0 .. kWin - 1 = 8-word groups
                // 4 q + t .. 4 q + t + 4; the last word is
                // 32 (kChunk/32 - 1) + kR (kThreads - 1) + kWin - 1 = kBuf - 1
                const uint4* lo = reinterpret_cast<const uint4*>(buf) + 4 * q + t;
                const uint4* hi = reinterpret_cast<const uint4*>(buf + kBuf / 2) + 4 * q + t;
                uint32_t w[kWin];
#pragma unroll
                for (int m = 0; m < kWin / 8; m++) {
                    const uint4 u = lo[m], v = hi[m];
                    w[8 * m] = u.x;
                    w[8 * m + 1] = u.y;
                    w[8 * m + 2] = u.z;
                    w[8 * m + 3] = u.w;
                    w[8 * m + 4] = v.x;
                    w[8 * m + 5] = v.y;
                    w[8 * m + 6] = v.z;
                    w[8 * m + 7] = v.w;
                }
#pragma unroll
                for (int n = 0; n < 8; n++) apply_nibble((a >> (4 * n)) & 15u, acc, w + 4 * n);
            }
        }
#pragma unroll
        for (int r = 0; r < kR; r++) local += (k0 + kR * t + r < valid && acc[r] != 0) ? 1u : 0u;
    }
    __syncthreads();
    if (local) atomicAdd(&wg_count, local);
    __syncthreads();
    if (t == 0 && wg_count) atomicAdd(count, wg_count);
}

}  // namespace

hipError_t launch_check(int out_kind, const void* src, uint64_t nw, uint32_t S, const uint32_t* d_A, uint32_t deg,
                        unsigned long long* d_count, uint32_t max_grid, hipStream_t stream) {
    zero_count_kernel<<<1, 1, 0, stream>>>(d_count);
    const uint64_t nk0 = (nw + S - 1) / S;  // phase 0 is the longest
    const uint64_t valid0 = nk0 > deg ? nk0 - deg : 0;
    const uint64_t tiles_per_phase = (valid0 + kTile - 1) / kTile;
    const uint64_t tiles = tiles_per_phase * S;
    if (tiles == 0) return hipGetLastError();
    const uint32_t grid = (uint32_t)(tiles < max_grid ? tiles : max_grid);
    switch (out_kind) {
        case kOutU32:
            check_kernel<kOutU32><<<grid, kThreads, 0, stream>>>(src, nw, S, d_A, deg, tiles_per_phase, d_count);
            break;
        case kOutF32:
            check_kernel<kOutF32><<<grid, kThreads, 0, stream>>>(src, nw, S, d_A, deg, tiles_per_phase, d_count);
            break;
        case kOutU64:
            check_kernel<kOutU64><<<grid, kThreads, 0, stream>>>(src, nw, S, d_A, deg, tiles_per_phase, d_count);
            break;
        default:
            check_kernel<kOutF64><<<grid, kThreads, 0, stream>>>(src, nw, S, d_A, deg, tiles_per_phase, d_count);
            break;
    }
    return hipGetLastError();
}

}  // namespace vmt
