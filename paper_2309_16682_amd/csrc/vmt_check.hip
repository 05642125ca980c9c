// vmt_check.hip -- gfx950 kernels of the linear-complexity self-check.
//
// Every output bit of an F2-linear generator, read along its stream, obeys
// the linear recurrence of a polynomial A (Sec. 4.1 reports the resulting
// LinearComp failures of every MT-based generator; Sec. 3.1 gives the
// polynomial view of the state map). Thirty-two bits are checked at once:
// for every offset x, XOR over the set coefficients i of A of the 32-bit
// words w[x + i S] must be zero.
//
// The work is a correlation of the word sequence with the coefficient
// pattern of A: plain integer ALU and LDS work (no MFMA: the arithmetic is
// over GF(2)). The S phases of the stride are independent sequences; a
// workgroup takes a tile of kTile consecutive offsets of one phase and
// stages the phase's words in LDS in chunks of kChunk coefficients
// (kTile + kChunk words). Two forms, chosen by the density of A:
//
// Sparse (MT19937-32/-64: mu has 135 / 285 set coefficients of 19,938).
// 512 threads; thread t owns the offsets t + 512 r, r < 8. For each set coefficient
// i (a wave-uniform list) it XORs buf[i + t + 512 r] into accumulator r:
// consecutive lanes read consecutive words (conflict-free ds_read_b32), two
// coefficients per three-input XOR. Every LDS byte read is used: the bound
// is LDS bandwidth, 4 bytes per coefficient and offset.
//
// Dense (SFMT19937: phi psi^M has ~9,300 set coefficients). 256 threads;
// thread t owns the 16 consecutive offsets 16 t .. 16 t + 15, so one LDS
// window of 48 words serves 32 coefficients. For each 32-coefficient word of
// A (a scalar load, the next one in flight) a thread reads its window with
// twelve ds_read_b128 and, nibble by nibble, XORs the selected window words
// into its accumulators: the nibble's value picks one of 16 straight-line
// cases (a scalar branch), each combining up to four words per accumulator
// with three-input XORs, ~1.25 VALU ops per nibble and accumulator; sixteen
// accumulators per thread amortise the branch. LDS layout: word j sits in
// plane (j / 4) % 4 at 16-byte slot j / 16, so the window (three 16-word
// groups) is twelve 16-byte reads at a 16-byte lane stride. (A sweep of
// threads x offsets per thread on one MI355X: 256 x 16 ran in 0.70 of the
// time of 512 x 8 and of 256 x 8 or 128 x 16.)
#include <hip/hip_runtime.h>

#include "vmt_launch.hpp"

namespace vmt {
namespace {

constexpr int kChunk = kCheckChunkBits;  // coefficients staged per LDS fill

// Launch geometry of the two forms; both tile 4096 offsets and stage
// kTile + kChunk words per fill.
template <bool DENSE>
struct Form {
    static constexpr int kThreads = DENSE ? 256 : 512;
    static constexpr int kR = DENSE ? 16 : 8;                // offsets per thread
    static constexpr int kTile = kThreads * kR;              // offsets per workgroup tile
    static constexpr int kBuf = kTile + kChunk;              // LDS words per fill
    static constexpr int kPer = kBuf / kThreads;             // staged words per thread
    static constexpr int kPlanes = kR / 4;                   // dense layout: planes of 4-word slots
    static constexpr int kWin = kR + 32;                     // dense window: words per 32 coefficients
    static constexpr int kGridPerCu = DENSE ? 24 : 8;        // workgroups launched per CU
    static_assert(kChunk % 32 == 0 && kBuf % (4 * kThreads) == 0 && 32 % kR == 0 && kR % 4 == 0,
                  "staging in 16-byte groups; a 32-coefficient window is whole kR-word groups");
};
static_assert(Form<true>::kTile == Form<false>::kTile, "one tiling for both forms");
constexpr int kTile = Form<true>::kTile;

__device__ __forceinline__ uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// a ^ b ^ c in one VALU op (v_bitop3_b32, truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, (unsigned char)0x96);
}

// ---- dense form: nibble cases ---------------------------------------------------

// acc[r] ^= XOR over the set bits e of V of w[e + r], r < R.
template <int R, int V>
__device__ __forceinline__ void nibble(uint32_t (&acc)[R], const uint32_t* w) {
    constexpr int n = __builtin_popcount(V);
    constexpr int e0 = V & 1 ? 0 : V & 2 ? 1 : V & 4 ? 2 : 3;                    // lowest set bit
    constexpr int e3 = V & 8 ? 3 : V & 4 ? 2 : V & 2 ? 1 : 0;                    // highest set bit
    constexpr int e1 = (V & ~(1 << e0)) & 2 ? 1 : (V & ~(1 << e0)) & 4 ? 2 : 3;  // second lowest
#pragma unroll
    for (int r = 0; r < R; r++) {
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

template <int R>
__device__ __forceinline__ void apply_nibble(uint32_t v, uint32_t (&acc)[R], const uint32_t* w) {
    switch (v) {
        case 1: nibble<R, 1>(acc, w); break;
        case 2: nibble<R, 2>(acc, w); break;
        case 3: nibble<R, 3>(acc, w); break;
        case 4: nibble<R, 4>(acc, w); break;
        case 5: nibble<R, 5>(acc, w); break;
        case 6: nibble<R, 6>(acc, w); break;
        case 7: nibble<R, 7>(acc, w); break;
        case 8: nibble<R, 8>(acc, w); break;
        case 9: nibble<R, 9>(acc, w); break;
        case 10: nibble<R, 10>(acc, w); break;
        case 11: nibble<R, 11>(acc, w); break;
        case 12: nibble<R, 12>(acc, w); break;
        case 13: nibble<R, 13>(acc, w); break;
        case 14: nibble<R, 14>(acc, w); break;
        case 15: nibble<R, 15>(acc, w); break;
        default: break;
    }
}

// LDS slot of buffer word j. Dense: word j in plane (j / 4) % kPlanes at
// 4-word slot j / kR (a thread's kR consecutive words are one slot in each
// plane). Sparse: linear.
template <bool DENSE>
__device__ __forceinline__ uint32_t lds_slot(uint32_t j) {
    using F = Form<DENSE>;
    if constexpr (DENSE) return ((j >> 2) % F::kPlanes) * (F::kBuf / F::kPlanes) + (j / F::kR) * 4 + (j & 3);
    else return j;
}

// ---- staging -------------------------------------------------------------------

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

// Words base + j, j < kBuf, of phase p, held in registers between the global
// loads and the LDS stores. Thread t takes the 4-word groups
// j = 4 (t + kThreads m): with S == 1, 32-bit elements and a 16-byte aligned
// stream a group is one 16-byte load (base is a multiple of 4), otherwise
// four word loads. Words at or beyond nk read as 0.
template <int KIND, bool DENSE>
struct Stage {
    using F = Form<DENSE>;
    uint32_t v[F::kPer];

    __device__ __forceinline__ void fetch(const void* src, bool vec, uint32_t p, uint32_t S, uint64_t base,
                                          uint64_t nk, uint32_t t) {
#pragma unroll
        for (int m = 0; m < F::kPer / 4; m++) {
            const uint64_t k = base + 4 * (t + F::kThreads * m);
            if constexpr (KIND == kOutU32 || KIND == kOutF32) {
                if (vec && k + 3 < nk) {
                    const uint4 u = *reinterpret_cast<const uint4*>(static_cast<const uint32_t*>(src) + k);
                    if constexpr (KIND == kOutU32) {
                        v[4 * m] = u.x;
                        v[4 * m + 1] = u.y;
                        v[4 * m + 2] = u.z;
                        v[4 * m + 3] = u.w;
                    } else {
                        v[4 * m] = (uint32_t)(__uint_as_float(u.x) * 16777216.0f);
                        v[4 * m + 1] = (uint32_t)(__uint_as_float(u.y) * 16777216.0f);
                        v[4 * m + 2] = (uint32_t)(__uint_as_float(u.z) * 16777216.0f);
                        v[4 * m + 3] = (uint32_t)(__uint_as_float(u.w) * 16777216.0f);
                    }
                    continue;
                }
            }
#pragma unroll
            for (int e = 0; e < 4; e++) v[4 * m + e] = k + e < nk ? stream_word<KIND>(src, p + (k + e) * S) : 0u;
        }
    }

    // The four words of a group are adjacent (and 16-byte aligned) in both layouts.
    __device__ __forceinline__ void store(uint32_t* buf, uint32_t t) const {
#pragma unroll
        for (int m = 0; m < F::kPer / 4; m++) {
            const uint32_t j = 4 * (t + F::kThreads * m);
            *reinterpret_cast<uint4*>(buf + lds_slot<DENSE>(j)) =
                make_uint4(v[4 * m], v[4 * m + 1], v[4 * m + 2], v[4 * m + 3]);
        }
    }
};

__global__ void zero_count_kernel(unsigned long long* count) { *count = 0; }

// ---- the kernel -----------------------------------------------------------------

// nw words in S phases; phase p holds words p, p + S, .... Dense: A = deg + 1
// coefficients as uint32 words, zero-padded to a multiple of kChunk bits.
// Sparse: E = the set coefficients in increasing order, E[Eoff[c] ..
// Eoff[c + 1]) those of chunk c = [c kChunk, (c + 1) kChunk).
template <int KIND, bool DENSE>
__global__ __launch_bounds__(Form<DENSE>::kThreads) void check_kernel(
    const void* __restrict__ src, uint64_t nw, uint32_t S, const uint32_t* __restrict__ A,
    const uint32_t* __restrict__ E, const uint32_t* __restrict__ Eoff, uint32_t deg, uint64_t tiles_per_phase,
    unsigned long long* count) {
    using F = Form<DENSE>;
    constexpr int kR = F::kR, kThreads = F::kThreads, kBuf = F::kBuf;
    __shared__ __align__(16) uint32_t buf[kBuf];
    __shared__ unsigned long long wg_count;
    const uint32_t t = threadIdx.x;
    if (t == 0) wg_count = 0;
    unsigned long long local = 0;
    const bool vec = S == 1 && (reinterpret_cast<uintptr_t>(src) & 15) == 0;
    const uint32_t n_chunks = deg / kChunk + 1;
    const uint64_t tiles = tiles_per_phase * S;
    Stage<KIND, DENSE> st;
    for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const uint32_t p = (uint32_t)(tile / tiles_per_phase);
        const uint64_t k0 = (tile % tiles_per_phase) * kTile;
        const uint64_t nk = nw > p ? (nw - p + S - 1) / S : 0;  // words in phase p
        const uint64_t valid = nk > deg ? nk - deg : 0;          // offsets k < valid are checked
        if (k0 >= valid) continue;                               // the same for the whole workgroup
        uint32_t acc[kR];
#pragma unroll
        for (int r = 0; r < kR; r++) acc[r] = 0;
        // Sparse: the next chunk's loads are in flight while this chunk is worked on.
        // Dense (ALU-bound): loaded right before the store, so the staging
        // registers are free during the XOR loop (occupancy).
        if constexpr (!DENSE) st.fetch(src, vec, p, S, k0, nk, t);
        for (uint32_t c = 0; c < n_chunks; c++) {
            const uint32_t i0 = c * kChunk;
            if constexpr (DENSE) st.fetch(src, vec, p, S, k0 + i0, nk, t);
            __syncthreads();  // the previous chunk's reads are done
            st.store(buf, t);
            __syncthreads();
            if constexpr (!DENSE) {
                if (c + 1 < n_chunks) st.fetch(src, vec, p, S, k0 + i0 + kChunk, nk, t);
            }
            if constexpr (DENSE) {
                const uint32_t* Ac = A + i0 / 32;
                uint32_t a = uniform(Ac[0]);
                for (int q = 0; q < kChunk / 32; q++) {
                    const uint32_t a_next = q + 1 < kChunk / 32 ? uniform(Ac[q + 1]) : 0u;
                    if (a != 0) {
                        // window: buffer words 32 q + kR t + 0 .. kWin - 1 = kR-word groups
                        // g0 .. g0 + kWin / kR - 1, g0 = 32 q / kR + t; the last group is
                        // 32 (kChunk/32 - 1) / kR + (kThreads - 1) + kWin / kR - 1 = kBuf / kR - 1
                        const uint32_t g0 = 32 * q / kR + t;
                        uint32_t w[F::kWin];
#pragma unroll
                        for (int m = 0; m < F::kWin / kR; m++) {
#pragma unroll
                            for (int pl = 0; pl < F::kPlanes; pl++) {
                                const uint4 u =
                                    reinterpret_cast<const uint4*>(buf + pl * (kBuf / F::kPlanes))[g0 + m];
                                w[kR * m + 4 * pl] = u.x;
                                w[kR * m + 4 * pl + 1] = u.y;
                                w[kR * m + 4 * pl + 2] = u.z;
                                w[kR * m + 4 * pl + 3] = u.w;
                            }
                        }
#pragma unroll
                        for (int n = 0; n < 8; n++) apply_nibble<kR>((a >> (4 * n)) & 15u, acc, w + 4 * n);
                    }
                    a = a_next;
                }
            } else {
                // coefficient offset d < kChunk, offset t + kThreads r < kTile: index < kBuf
                const uint32_t e_end = uniform(Eoff[c + 1]);
                uint32_t e = uniform(Eoff[c]);
                for (; e + 1 < e_end; e += 2) {
                    const uint32_t* b1 = buf + (uniform(E[e]) - i0) + t;
                    const uint32_t* b2 = buf + (uniform(E[e + 1]) - i0) + t;
#pragma unroll
                    for (int r = 0; r < kR; r++) acc[r] = xor3(acc[r], b1[kThreads * r], b2[kThreads * r]);
                }
                if (e < e_end) {
                    const uint32_t* b1 = buf + (uniform(E[e]) - i0) + t;
#pragma unroll
                    for (int r = 0; r < kR; r++) acc[r] ^= b1[kThreads * r];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < kR; r++) {
            const uint64_t k = k0 + (DENSE ? kR * t + r : t + kThreads * r);
            local += (k < valid && acc[r] != 0) ? 1u : 0u;
        }
    }
    __syncthreads();
    if (local) atomicAdd(&wg_count, local);
    __syncthreads();
    if (t == 0 && wg_count) atomicAdd(count, wg_count);
}

template <int KIND, bool DENSE>
void launch_form(const CheckPolyDev& poly, uint64_t tiles, uint32_t cus, hipStream_t stream, const void* src,
                 uint64_t nw, uint32_t S, uint64_t tpp, unsigned long long* count) {
    using F = Form<DENSE>;
    const uint64_t cap = (uint64_t)F::kGridPerCu * cus;
    const uint32_t grid = (uint32_t)(tiles < cap ? tiles : cap);
    check_kernel<KIND, DENSE><<<grid, F::kThreads, 0, stream>>>(src, nw, S, poly.bits, poly.terms, poly.term_off,
                                                               poly.deg, tpp, count);
}

template <int KIND>
void launch_kind(const CheckPolyDev& poly, uint64_t tiles, uint32_t cus, hipStream_t stream, const void* src,
                 uint64_t nw, uint32_t S, uint64_t tpp, unsigned long long* count) {
    if (poly.dense) launch_form<KIND, true>(poly, tiles, cus, stream, src, nw, S, tpp, count);
    else launch_form<KIND, false>(poly, tiles, cus, stream, src, nw, S, tpp, count);
}

}  // namespace

hipError_t launch_check(int out_kind, const void* src, uint64_t nw, uint32_t S, const CheckPolyDev& poly,
                        unsigned long long* d_count, uint32_t cus, hipStream_t stream) {
    zero_count_kernel<<<1, 1, 0, stream>>>(d_count);
    const uint64_t nk0 = (nw + S - 1) / S;  // phase 0 is the longest
    const uint64_t valid0 = nk0 > poly.deg ? nk0 - poly.deg : 0;
    const uint64_t tiles_per_phase = (valid0 + kTile - 1) / kTile;
    const uint64_t tiles = tiles_per_phase * S;
    if (tiles == 0) return hipGetLastError();
    switch (out_kind) {
        case kOutU32: launch_kind<kOutU32>(poly, tiles, cus, stream, src, nw, S, tiles_per_phase, d_count); break;
        case kOutF32: launch_kind<kOutF32>(poly, tiles, cus, stream, src, nw, S, tiles_per_phase, d_count); break;
        case kOutU64: launch_kind<kOutU64>(poly, tiles, cus, stream, src, nw, S, tiles_per_phase, d_count); break;
        default: launch_kind<kOutF64>(poly, tiles, cus, stream, src, nw, S, tiles_per_phase, d_count); break;
    }
    return hipGetLastError();
}

}  // namespace vmt
