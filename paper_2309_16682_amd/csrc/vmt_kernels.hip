// vmt_kernels.hip -- gfx950 kernels for the V-family generators.
//
// Paper: F. Cannizzo, "VMT19937: A SIMD-Friendly Pseudo Random Number
// Generator based on Mersenne Twister 19937" (arXiv 2309.16682).
//
// The paper vectorises the twist across M lock-stepped instances in one SIMD
// register (Sec. 3, eq. msmt19937). On CDNA4 the same idea maps onto the
// 64-wide wavefront: the lane-interleaved window sits in LDS, so row k of the
// window (word k of every lane) is contiguous, and a work item updates a
// 16-byte group of lanes of one row with one ds_read_b128 per operand.
//
// Block regeneration (Sec. 2.5, eq. stepnomod): the n new words of a block
// fall into three index ranges, [0, n-m), [n-m, 2(n-m)), [2(n-m), n). Word
// c of range 1 needs only old words; word c + (n-m) of range 2 needs the new
// word c; word c + 2(n-m) of range 3 needs the new word c + (n-m). So one
// work item owns the "column" c, c + (n-m), c + 2(n-m) and carries the
// dependency in registers: every LDS read is of the old block, every write
// happens after one barrier. The only cross-column value, new word 0 read by
// the last word of the block, is published next to the window before that
// barrier and read after it.
//
// Tempering (eq. tempering) and the optional float map are fused between
// the twist and the 16-byte global store, so each output is written once,
// in stream order, by a fully coalesced store.
//
// Jump (Sec. 3.1): the state after d steps is g(F) X with g = t^d mod mu.
// Word j of the new window is the XOR of the raw words x_{i+j} over the set
// coefficients i of g (Horner's rule unrolled over the word sequence). A
// workgroup regenerates the raw sequence two blocks at a time in LDS and each
// wavefront accumulates one lane; the loop over the coefficients of g is
// wave-uniform (scalar unit), the XORs are VALU. The reads are the cost (LDS
// bandwidth), so where LDS allows, coefficients are taken four at a time from
// derived rows (accumulate_block4).
//
// SFMT19937's recurrence is serial along each lane; a quad of threads shares
// a lane, one 32-bit sub-word each (sfmt_block_quad), laid out 4 threads apart
// within a row of 16 (sfmt_quad_thread).
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include "vmt_common.hpp"
#include "vmt_launch.hpp"

namespace vmt {
namespace {

// ---------------------------------------------------------------------------
// Parameters: Sec. 2.2 eq. (params), Sec. 2.3 eq. (params64),
// Sec. 2.4 eq. (sfmt_params).
// ---------------------------------------------------------------------------

struct MT32P {
    using W = uint32_t;
    static constexpr int N = 624, MM = 397, D = N - MM;  // D = 227
    static constexpr int V = 4;                            // lanes per 16-byte group
};
struct MT64P {
    using W = uint64_t;
    static constexpr int N = 312, MM = 156, D = N - MM;  // D = 156
    static constexpr int V = 2;
};
// SFMT parameter set of the state size N (each set has its own N).
constexpr int sfmt_index(int N) {
    for (int i = 0; i < 6; i++)
        if ((int)kSfmtSets[i].n == N) return i;
    return -1;
}
template <int N>
struct SfmtP {
    static constexpr int I = sfmt_index(N);
    static_assert(I >= 0, "no SFMT parameter set with this state size");
    static constexpr int MM = kSfmtSets[I].pos1;
    static constexpr int SL1 = kSfmtSets[I].sl1, SL2 = 8 * kSfmtSets[I].sl2;  // bits
    static constexpr int SR1 = kSfmtSets[I].sr1, SR2 = 8 * kSfmtSets[I].sr2;  // bits
    static constexpr uint32_t K0 = kSfmtSets[I].msk[0], K1 = kSfmtSets[I].msk[1], K2 = kSfmtSets[I].msk[2],
                              K3 = kSfmtSets[I].msk[3];
    static constexpr uint32_t P0 = kSfmtSets[I].parity[0], P1 = kSfmtSets[I].parity[1],
                              P2 = kSfmtSets[I].parity[2], P3 = kSfmtSets[I].parity[3];
    static_assert(MM <= N - 2 && SL2 < 32 && SR2 < 32, "in-place chain and one-neighbour funnel shifts");
};

// a ^ (b & c) in one VALU op (v_bitop3_b32, truth table 0x78)
__device__ __forceinline__ uint32_t xor_and(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, (unsigned char)0x78);
}
// (m & a) | (~m & b) in one VALU op (v_bitop3_b32, truth table 0xE4)
__device__ __forceinline__ uint32_t select_bits(uint32_t m, uint32_t a, uint32_t b) {
    return __builtin_amdgcn_bitop3_b32(a, b, m, (unsigned char)0xE4);
}
// a ^ b ^ c in one VALU op (v_bitop3_b32, truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, (unsigned char)0x96);
}
// all ones if bit 0 of x is set
__device__ __forceinline__ uint32_t lsb_mask(uint32_t x) { return (uint32_t)__builtin_amdgcn_sbfe((int)x, 0, 1); }

// Values that are equal in every lane but reach the kernel through memory a
// lane reads (LDS, a task list) must be marked uniform: loops and exits that
// contain barriers have to be scalar branches, never exec-masked ones.
__device__ __forceinline__ uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uniform(uint64_t x) {
    return ((uint64_t)uniform((uint32_t)(x >> 32)) << 32) | uniform((uint32_t)x);
}
template <class T>
__device__ __forceinline__ T* uniform(T* p) {
    return reinterpret_cast<T*>(uniform((uint64_t)reinterpret_cast<uintptr_t>(p)));
}

// ---- MT19937-32: eq. (step) with eq. (matmult); h = 0x80000000, l = 0x7fffffff.
// omega = (x_k & h) | (x_{k+1} & l); bit 0 of omega is bit 0 of x_{k+1}.
__device__ __forceinline__ uint32_t twist(uint32_t xk, uint32_t xk1, uint32_t xkm) {
    const uint32_t omega = select_bits(0x80000000u, xk, xk1);
    return xor_and(xkm ^ (omega >> 1), lsb_mask(xk1), 0x9908B0DFu);
}
// eq. (tempering), MT19937-32 constants; d = 0xFFFFFFFF needs no mask.
__device__ __forceinline__ uint32_t temper(uint32_t y) {
    y ^= y >> 11;
    y = xor_and(y, y << 7, 0x9D2C5680u);
    y = xor_and(y, y << 15, 0xEFC60000u);
    return y ^ (y >> 18);
}

// Tempering of two MT19937-32 words held as one 64-bit register pair:
// v_lshrrev_b64 / v_lshlrev_b64 shift both words at once (a 64-bit shift
// issues at about 3/4 of the rate of a 32-bit one but does two words); the
// bits that cross from one word into the other land exactly where the next
// mask is zero (the masks b and c have no bits below 15 and 17), or are
// cleared by the mask of the bitop3 that consumes them.
__device__ __forceinline__ uint64_t pair64(uint32_t lo, uint32_t hi) { return ((uint64_t)hi << 32) | lo; }
template <int S>
__device__ __forceinline__ uint64_t shr64(uint64_t v) {
    uint64_t r;
    asm("v_lshrrev_b64 %0, %2, %1" : "=v"(r) : "v"(v), "n"(S));
    return r;
}
template <int S>
__device__ __forceinline__ uint64_t shl64(uint64_t v) {
    uint64_t r;
    asm("v_lshlrev_b64 %0, %2, %1" : "=v"(r) : "v"(v), "n"(S));
    return r;
}
__device__ __forceinline__ void temper_pair(uint32_t& a, uint32_t& b) {
    uint64_t s = shr64<11>(pair64(a, b));  // a: b's low 11 bits arrive in bits 21..31
    a = xor_and(a, (uint32_t)s, 0x001FFFFFu);
    b ^= (uint32_t)(s >> 32);
    s = shl64<7>(pair64(a, b));  // b: a's top 7 bits arrive in bits 0..6, outside 0x9D2C5680
    a = xor_and(a, (uint32_t)s, 0x9D2C5680u);
    b = xor_and(b, (uint32_t)(s >> 32), 0x9D2C5680u);
    s = shl64<15>(pair64(a, b));  // bits 0..14 of b, outside 0xEFC60000
    a = xor_and(a, (uint32_t)s, 0xEFC60000u);
    b = xor_and(b, (uint32_t)(s >> 32), 0xEFC60000u);
    s = shr64<18>(pair64(a, b));  // a: bits 14..31 carry b's bits, keep 0..13
    a = xor_and(a, (uint32_t)s, 0x00003FFFu);
    b ^= (uint32_t)(s >> 32);
}

// ---- MT19937-64 on 32-bit halves (v_alignbit for the 64-bit shifts):
// h = 0xFFFFFFFF80000000, l = 0x7FFFFFFF, a = 0xB5026F5AA96619E9.
__device__ __forceinline__ uint64_t twist(uint64_t xk, uint64_t xk1, uint64_t xkm) {
    const uint32_t kh = (uint32_t)(xk >> 32), kl = (uint32_t)xk, k1 = (uint32_t)xk1;
    const uint32_t ol = select_bits(0x80000000u, kl, k1);  // omega = (kh : ol)
    const uint32_t odd = lsb_mask(k1);
    const uint32_t lo = xor_and((uint32_t)xkm ^ __builtin_amdgcn_alignbit(kh, ol, 1), odd, 0xA96619E9u);
    const uint32_t hi = xor_and((uint32_t)(xkm >> 32) ^ (kh >> 1), odd, 0xB5026F5Au);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t temper(uint64_t y) {
    uint32_t lo = (uint32_t)y, hi = (uint32_t)(y >> 32);
    // y ^= (y >> 29) & 0x5555555555555555
    const uint32_t s1l = __builtin_amdgcn_alignbit(hi, lo, 29), s1h = hi >> 29;
    lo = xor_and(lo, s1l, 0x55555555u);
    hi = xor_and(hi, s1h, 0x55555555u);
    // y ^= (y << 17) & 0x71D67FFFEDA60000
    const uint32_t s2h = __builtin_amdgcn_alignbit(hi, lo, 15), s2l = lo << 17;
    lo = xor_and(lo, s2l, 0xEDA60000u);
    hi = xor_and(hi, s2h, 0x71D67FFFu);
    // y ^= (y << 37) & 0xFFF7EEE000000000
    hi = xor_and(hi, lo << 5, 0xFFF7EEE0u);
    // y ^= y >> 43
    lo ^= hi >> 11;
    return ((uint64_t)hi << 32) | lo;
}

// ---- SFMT, eq. (sfmt_step): 128-bit words as four 32-bit sub-words,
// sub-word 0 least significant; w <<< 8 SL2 moves bits from sub-word j into
// j + 1, w >>> 8 SR2 from j + 1 into j (SFMT19937: one byte each; every set
// here shifts by at most three bytes, so only the neighbouring sub-word is
// involved). Block regeneration by a quad of threads:
// thread j of the quad owns sub-word j of every 128-bit word of one lane. The recurrence
// is serial along the words (each new word reads the two before it), so the
// quad splits each step four ways instead: the two shifts that cross
// sub-words take the neighbour's value by a quad permutation (DPP). The
// neighbour's part of w_{k+N-2} is exchanged two steps ahead, off the
// dependency chain.
//
// The block loop is unrolled and software-pipelined: the operands w_k and
// w_{k+MM} of the old block are loaded kPrefetch steps ahead, and the new
// words that the recurrence reads again (w_{k+MM} for k + MM >= N, written
// N - MM steps before) stay in registers. So no load waits for the step just
// stored: the critical path of a step is the recurrence itself (the shift of
// w_{k+N-1} and an XOR). (A chain that loads each operand right before use
// waits for an LDS round trip per step, ~200 cycles.)
// Quad layout: sub-word j of lane group q is thread 16 (q / 4) + 4 j + q % 4,
// so the four sub-words of a lane sit 4 threads apart in one row of 16. The
// neighbour's sub-word is then a row shift by 4 (DPP row_shl / row_shr), and
// the shift supplies the zero that sub-words 3 and 0 need at the row's ends
// (the source lane is outside the row), with no separate mask.
struct QuadThread {
    int q, j;
};
__device__ __forceinline__ QuadThread sfmt_quad_thread(int tid) {
    return QuadThread{((tid >> 4) << 2) | (tid & 3), (tid >> 2) & 3};
}
__device__ __forceinline__ uint32_t quad_next(uint32_t x) {  // sub-word j + 1 of the lane (j = 3: zero)
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x104, 0xF, 0xF, true);
}
__device__ __forceinline__ uint32_t quad_prev(uint32_t x) {  // sub-word j - 1 of the lane (j = 0: zero)
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);
}

constexpr int kPrefetch = 8;  // steps between an operand load and its use

// src, dst: sub-word j of word k at [k * ws + j] (u32 units); src == dst runs
// in place (every old word is loaded before the step that overwrites it).
// The four threads of a quad must run it together. emit(k, value) is called
// for every new sub-word in order.
template <int N, class Emit>
__device__ __forceinline__ void sfmt_block_quad(const uint32_t* src, uint32_t* dst, int ws, int j, Emit emit) {
    using P = SfmtP<N>;
    constexpr int MM = P::MM;
    constexpr int PD = kPrefetch < N ? kPrefetch : N;
    // the mask K of eq. (sfmt_params), sub-word j
    const uint32_t K = j == 0 ? P::K0 : j == 1 ? P::K1 : j == 2 ? P::K2 : P::K3;
    // all indices below are compile-time constants after unrolling: the arrays are registers,
    // and only the live window of each (PD loads ahead, N - MM new words back) occupies any
    uint32_t pa[N], pb[N], nw[N];
#pragma unroll
    for (int k = 0; k < PD; ++k) {
        pa[k] = src[k * ws + j];
        if (k + MM < N) pb[k] = src[(k + MM) * ws + j];
    }
    // cn, dn: the upper neighbour's sub-word of c and d, zero for sub-word 3
    uint32_t c = src[(N - 2) * ws + j], d = src[(N - 1) * ws + j];
    uint32_t cn = quad_next(c), dn = quad_next(d);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        if (k + PD < N) {  // operands of step k + PD: old words, not yet overwritten
            pa[k + PD] = src[(k + PD) * ws + j];
            if (k + PD + MM < N) pb[k + PD] = src[(k + PD + MM) * ws + j];
        }
        const uint32_t ak = pa[k], bk = k + MM < N ? pb[k] : nw[k + MM - N];
        // (a <<< SL2) and (c >>> SR2) on this sub-word: funnel shifts with the neighbour's sub-word
        const uint32_t al = __builtin_amdgcn_alignbit(ak, quad_prev(ak), 32 - P::SL2);
        const uint32_t cr = __builtin_amdgcn_alignbit(cn, c, P::SR2);
        uint32_t r = xor3(ak, al, cr);
        r = xor_and(r, bk >> P::SR1, K);
        r ^= d << P::SL1;
        nw[k] = r;
        dst[k * ws + j] = r;
        emit(k, r);
        c = d;
        cn = dn;
        d = r;
        dn = quad_next(r);
    }
}

// ---- fixed float maps (exact: the kept bits fit the significand)
__device__ __forceinline__ float to_f32(uint32_t u) { return (float)(u >> 8) * 0x1p-24f; }
__device__ __forceinline__ float to_f32(uint64_t u) { return (float)(uint32_t)(u >> 40) * 0x1p-24f; }
__device__ __forceinline__ double to_f64(uint64_t u) { return (double)(u >> 11) * 0x1p-53; }

// output element for a tempered word; OUT: 0 native, 1 f32, 2 f64
template <int OUT, class W>
struct OutOf;
template <class W>
struct OutOf<0, W> {
    using T = W;
    static __device__ __forceinline__ T map(W v) { return v; }
};
template <class W>
struct OutOf<1, W> {
    using T = float;
    static __device__ __forceinline__ T map(W v) { return to_f32(v); }
};
template <class W>
struct OutOf<2, W> {
    using T = double;
    static __device__ __forceinline__ T map(W v) { return to_f64(v); }
};

template <class T, int V>
struct alignas(sizeof(T) * V) Vec {
    T v[V];
};

// Pointers that reach a kernel through memory (task lists, headers) are
// generic; these accessors make the global address space explicit so the
// compiler emits global_load/global_store (scalar base + 32-bit offset)
// rather than flat accesses. The value travels as a vector of dwords (the
// address-space cast is kept for vector types, not for aggregates).
template <int NW>
struct DwordVec {
    typedef unsigned type __attribute__((ext_vector_type(NW)));
};
template <>
struct DwordVec<1> {
    typedef unsigned type;
};
#define VMT_GLOBAL __attribute__((address_space(1)))

#ifndef VMT_NT_STORES
#define VMT_NT_STORES 0
#endif

template <class T>
__device__ __forceinline__ void gstore(T* p, const T& v) {
    static_assert(sizeof(T) % 4 == 0 && sizeof(T) <= 16, "dword multiple");
    using D = typename DwordVec<sizeof(T) / 4>::type;
    D d;
    __builtin_memcpy(&d, &v, sizeof(T));
    if constexpr (VMT_NT_STORES) __builtin_nontemporal_store(d, (VMT_GLOBAL D*)p);
    else *(VMT_GLOBAL D*)p = d;
}
template <class T>
__device__ __forceinline__ T gload(const T* p) {
    static_assert(sizeof(T) % 4 == 0 && sizeof(T) <= 16, "dword multiple");
    using D = typename DwordVec<sizeof(T) / 4>::type;
    const D d = *(const VMT_GLOBAL D*)p;
    T v;
    __builtin_memcpy(&v, &d, sizeof(T));
    return v;
}

// The same block with the lane's window in registers: R[k] holds sub-word j
// of w_k on entry and of w_{k+N} on exit (the step that writes w_{k+N} is the
// last to read w_k, and w_{k+MM} for k + MM >= N is the new word written
// N - MM steps before, already in R). With every index a compile-time
// constant the array stays in VGPRs across blocks, so a step issues no LDS
// access: the recurrence, the two neighbour moves and the output store.
template <int N, class Emit>
__device__ __forceinline__ void sfmt_block_regs(uint32_t (&R)[N], int j, Emit emit) {
    using P = SfmtP<N>;
    constexpr int MM = P::MM;
    const uint32_t K = j == 0 ? P::K0 : j == 1 ? P::K1 : j == 2 ? P::K2 : P::K3;
    uint32_t c = R[N - 2], d = R[N - 1];
    uint32_t cn = quad_next(c), dn = quad_next(d);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const uint32_t ak = R[k];
        const uint32_t bk = R[k + MM < N ? k + MM : k + MM - N];
        const uint32_t al = __builtin_amdgcn_alignbit(ak, quad_prev(ak), 32 - P::SL2);
        const uint32_t cr = __builtin_amdgcn_alignbit(cn, c, P::SR2);
        uint32_t r = xor3(ak, al, cr);
        r = xor_and(r, bk >> P::SR1, K);
        r ^= d << P::SL1;
        R[k] = r;
        emit(k, r);
        c = d;
        cn = dn;
        d = r;
        dn = quad_next(r);
    }
}

// ---------------------------------------------------------------------------
// MT generation: one workgroup owns LPW lanes (lanes g*LPW ...) of a state.
// ---------------------------------------------------------------------------

// Threads per workgroup for LPW lanes: enough whole wavefronts that each
// thread owns at most two columns (fewer live registers, no spills). Shape
// variant TV gives each thread 2^TV times as many columns (fewer, smaller
// workgroups, so more of them fit on a compute unit).
template <class P, int LPW, int TV = 0>
constexpr int mt_threads() {
    constexpr int V = LPW < P::V ? LPW : P::V;
    constexpr int items = P::D * (LPW / V);
    constexpr int iters0 = ((items + 1023) / 1024) << TV;
    constexpr int iters = iters0 * 64 > items ? (items + 63) / 64 : iters0;
    return 64 * ((items + 64 * iters - 1) / (64 * iters));
}

// SW: bytes per global store of the output (16: dwordx4, 8: dwordx2).
template <class P, int LPW, int THREADS, int OUT, int SW = 16>
struct MtGen {
    using W = typename P::W;
    static constexpr int N = P::N, MM = P::MM, D = P::D;
    static constexpr int V = LPW < P::V ? LPW : P::V;
    static constexpr int QPR = LPW / V;  // 16-byte groups per row
    static constexpr int ITEMS = D * QPR;
    static constexpr int ITERS = (ITEMS + THREADS - 1) / THREADS;
    static constexpr bool THREE = N > 2 * D;  // MT19937-32 has a third index range
    static constexpr int RANGES = THREE ? 3 : 2;
    // The last word of a block, x_{n-1}, reads the new word 0 (its x_{k+1}
    // wraps around). It belongs to column C_LAST, in range LAST_R.
    static constexpr int LAST_R = RANGES - 1;
    static constexpr int C_LAST = N - 1 - LAST_R * D;
    using VW = Vec<W, V>;
    using Map = OutOf<OUT, W>;
    using OutT = typename Map::T;
    static constexpr int CH = SW / sizeof(OutT) > 0 ? SW / sizeof(OutT) : 1;  // output elements per store
    using VO = Vec<OutT, CH>;

    static __device__ __forceinline__ VW ld(const W* win, int row, int off) {
        return *reinterpret_cast<const VW*>(win + row * LPW + off);
    }
    static __device__ __forceinline__ void st(W* win, int row, int off, const VW& v) {
        *reinterpret_cast<VW*>(win + row * LPW + off) = v;
    }
    static __device__ __forceinline__ VW twistv(const VW& a, const VW& b, const VW& m) {
        VW r;
#pragma unroll
        for (int j = 0; j < V; j++) r.v[j] = twist(a.v[j], b.v[j], m.v[j]);
        return r;
    }
    // CH consecutive window words -> tempered, mapped output chunk
    static __device__ __forceinline__ VO temper_chunk(const W (&w)[CH]) {
        VO r;
        if constexpr (sizeof(W) == 4 && OUT == 0) {
            uint32_t t[CH];
#pragma unroll
            for (int j = 0; j < CH; j++) t[j] = w[j];
#pragma unroll
            for (int j = 0; j < CH; j += 2) temper_pair(t[j], t[j + 1]);
#pragma unroll
            for (int j = 0; j < CH; j++) r.v[j] = t[j];
        } else {
#pragma unroll
            for (int j = 0; j < CH; j++) r.v[j] = Map::map(temper(w[j]));
        }
        return r;
    }

    // Store phase, whole lanes (LPW == M): the window is the block in stream
    // order, so window words [s_lo, s_hi) go to out[o_base ...] as 16-byte
    // stores aligned to the *output*, whatever the start offset; at most
    // CH - 1 elements at either end are stored one by one.
    static __device__ __forceinline__ void store_contig(const W* win, OutT* out, uint32_t s_lo, uint32_t s_hi,
                                                        uint64_t o_base, int tid) {
        const uint32_t n = s_hi - s_lo;
        OutT* ob = uniform(out + o_base);
        const uint32_t mis = (uint32_t)(((uintptr_t)ob / sizeof(OutT)) % CH);
        const uint32_t lead = mis ? (CH - mis < n ? CH - mis : n) : 0;  // elements before the first aligned chunk
        const uint32_t nch = (n - lead) / CH;
        const uint32_t tail0 = lead + nch * CH;
        const uint32_t s0 = s_lo + lead;  // window index of the first chunk
        constexpr int L = 16 / (int)sizeof(W) < CH ? 16 / (int)sizeof(W) : CH;  // words per 16-byte LDS read
        if (s0 % CH == 0) {
            for (uint32_t i = tid; i < nch; i += THREADS) {
                W w[CH];
                const uint32_t s = s0 + i * CH;
#pragma unroll
                for (int j = 0; j < CH; j += L) {
                    const Vec<W, L> x = *reinterpret_cast<const Vec<W, L>*>(win + s + j);
#pragma unroll
                    for (int q = 0; q < L; q++) w[j + q] = x.v[q];
                }
                gstore(reinterpret_cast<VO*>(ob + lead + i * CH), temper_chunk(w));
            }
        } else {
            for (uint32_t i = tid; i < nch; i += THREADS) {
                W w[CH];
                const uint32_t s = s0 + i * CH;
#pragma unroll
                for (int j = 0; j < CH; j++) w[j] = win[s + j];
                gstore(reinterpret_cast<VO*>(ob + lead + i * CH), temper_chunk(w));
            }
        }
        const uint32_t edge = lead + (n - tail0);
        if ((uint32_t)tid < edge) {
            const uint32_t e = (uint32_t)tid < lead ? tid : tail0 + (tid - lead);
            gstore(ob + e, Map::map(temper(win[s_lo + e])));
        }
    }

    // Store phase, lane subset (LPW < M): row k holds stream elements
    // k*M + lane0 .. + LPW - 1; window words in [s_lo, s_hi) are stored.
    static __device__ __forceinline__ void store_rows(const W* win, OutT* out, uint32_t s_lo, uint32_t s_hi,
                                                      uint64_t o_base, uint32_t M, uint32_t lane0, int tid) {
        OutT* ob = uniform(out + o_base);
        const uint32_t k0 = s_lo / M, k1 = (s_hi - 1) / M;
        constexpr int G = LPW >= CH ? CH : 1;  // elements per store
        const bool vec = G == CH && ((uintptr_t)(ob + (int64_t)lane0 - (int64_t)s_lo) % 16) == 0;
        for (uint32_t i = k0 * (LPW / G) + tid; i < (k1 + 1) * (LPW / G); i += THREADS) {
            const uint32_t k = i / (LPW / G), tl = (i - k * (LPW / G)) * G;
            const uint32_t e = k * M + lane0 + tl;  // stream position of the first element
            if (vec && e >= s_lo && e + G <= s_hi) {
                W w[CH];
#pragma unroll
                for (int j = 0; j < CH; j++) w[j] = win[k * LPW + tl + j];
                gstore(reinterpret_cast<VO*>(ob + (e - s_lo)), temper_chunk(w));
            } else {
#pragma unroll
                for (int j = 0; j < G; j++)
                    if (e + j >= s_lo && e + j < s_hi) gstore(ob + (e + j - s_lo), Map::map(temper(win[k * LPW + tl + j])));
            }
        }
    }

    static __device__ __forceinline__ void store(const W* win, OutT* out, uint32_t s_lo, uint32_t s_hi,
                                                 uint64_t o_base, uint32_t M, uint32_t lane0, int tid) {
        if (LPW == M) store_contig(win, out, s_lo, s_hi, o_base, tid);
        else store_rows(win, out, s_lo, s_hi, o_base, M, lane0, tid);
    }

    // Twist one block in place: three index ranges per column, dependencies
    // carried in registers; all reads before the first barrier, all writes
    // after it.
    static __device__ __forceinline__ void twist_block(W* win, int tid) {
        W* x0new = win + N * LPW;  // new word 0 of every lane, for the last word
        VW nw[ITERS][RANGES];
        VW last_old[ITERS];
#pragma unroll
        for (int s = 0; s < ITERS; ++s) {
            const int it = tid + s * THREADS;
            if (it < ITEMS) {
                const int c = it / QPR, off = (it - (it / QPR) * QPR) * V;
                // range 1: old words only
                const VW n0 = twistv(ld(win, c, off), ld(win, c + 1, off), ld(win, c + MM, off));
                nw[s][0] = n0;
                if (c == 0) st(x0new, 0, off, n0);
                // range 2: x_{k+m-n} is the new word c
                const int r1 = c + D;
                if (THREE || c != C_LAST) nw[s][1] = twistv(ld(win, r1, off), ld(win, r1 + 1, off), n0);
                else last_old[s] = ld(win, r1, off);
                if constexpr (THREE) {
                    // range 3: x_{k+m-n} is the new word c + D
                    const int r2 = c + 2 * D;
                    if (c < C_LAST) nw[s][2] = twistv(ld(win, r2, off), ld(win, r2 + 1, off), nw[s][1]);
                    else if (c == C_LAST) last_old[s] = ld(win, r2, off);
                }
            }
            __builtin_amdgcn_sched_barrier(0);  // keep the next column's loads from piling up
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < ITERS; ++s) {
            const int it = tid + s * THREADS;
            if (it < ITEMS) {
                const int c = it / QPR, off = (it - (it / QPR) * QPR) * V;
                st(win, c, off, nw[s][0]);
                if (THREE || c != C_LAST) st(win, c + D, off, nw[s][1]);
                if constexpr (THREE) {
                    if (c < C_LAST) st(win, c + 2 * D, off, nw[s][2]);
                }
                if (c == C_LAST)  // x_{n-1}: reads the new word 0 published before the barrier
                    st(win, N - 1, off, twistv(last_old[s], ld(x0new, 0, off), nw[s][LAST_R - 1]));
            }
        }
        __syncthreads();
    }

    // Emit `len` elements from `state` (lanes g*LPW .. g*LPW + LPW - 1).
    static __device__ __forceinline__ void run(uint8_t* state, OutT* out, uint64_t len, uint32_t g, bool write_pos,
                                               W* win) {
        state = uniform(state);
        out = uniform(out);
        len = uniform(len);
        StateHeader* hdr = reinterpret_cast<StateHeader*>(state);
        const uint32_t M = uniform(gload(&hdr->M));
        const uint32_t pos = uniform(gload(&hdr->pos));
        W* gwin = reinterpret_cast<W*>(state + kHeaderBytes);
        const uint32_t B = (uint32_t)N * M;
        if (len == 0) return;
        const int tid = threadIdx.x;
        const uint32_t lane0 = g * LPW;
        const uint64_t head = len < (uint64_t)(B - pos) ? len : (uint64_t)(B - pos);
        const uint64_t rest = len - head;
        const uint64_t nblocks = (rest + B - 1) / B;

        for (int i = tid; i < N * QPR; i += THREADS) {
            const int k = i / QPR, q = i - (i / QPR) * QPR;
            st(win, k, q * V, gload(reinterpret_cast<const VW*>(gwin + (size_t)k * M + lane0 + q * V)));
        }
        __syncthreads();
        if (head) store(win, out, pos, pos + (uint32_t)head, 0, M, lane0, tid);  // rest of the current block
        for (uint64_t b = 0; b < nblocks; ++b) {
            const uint64_t o0 = head + b * B;
            twist_block(win, tid);
            const uint32_t n = (len - o0) < (uint64_t)B ? (uint32_t)(len - o0) : B;
            store(win, out, 0, n, o0, M, lane0, tid);
        }
        if (nblocks) {
            __syncthreads();
            for (int i = tid; i < N * QPR; i += THREADS) {
                const int k = i / QPR, q = i - (i / QPR) * QPR;
                gstore(reinterpret_cast<VW*>(gwin + (size_t)k * M + lane0 + q * V), ld(win, k, q * V));
            }
        }
        if (write_pos && uniform((uint32_t)tid >> 6) == 0)  // wave 0, same value from every lane
            gstore(&hdr->pos, nblocks ? (uint32_t)(rest - (nblocks - 1) * (uint64_t)B) : (uint32_t)(pos + head));
    }

    // Measurement only: run()'s memory traffic with the twist left out. The
    // window is read, every block of the request is stored from the unchanged
    // window through the same store path (the twist's two barriers kept), and
    // the window is written back unchanged; the position is not advanced, so
    // the state is left as it was.
    static __device__ __forceinline__ void run_pattern(uint8_t* state, OutT* out, uint64_t len, W* win) {
        state = uniform(state);
        out = uniform(out);
        len = uniform(len);
        StateHeader* hdr = reinterpret_cast<StateHeader*>(state);
        const uint32_t M = uniform(gload(&hdr->M));
        const uint32_t pos = uniform(gload(&hdr->pos));
        W* gwin = reinterpret_cast<W*>(state + kHeaderBytes);
        const uint32_t B = (uint32_t)N * M;
        if (len == 0) return;
        const int tid = threadIdx.x;
        const uint64_t head = len < (uint64_t)(B - pos) ? len : (uint64_t)(B - pos);
        const uint64_t rest = len - head;
        const uint64_t nblocks = (rest + B - 1) / B;
        for (int i = tid; i < N * QPR; i += THREADS) {
            const int k = i / QPR, q = i - (i / QPR) * QPR;
            st(win, k, q * V, gload(reinterpret_cast<const VW*>(gwin + (size_t)k * M + q * V)));
        }
        __syncthreads();
        if (head) store(win, out, pos, pos + (uint32_t)head, 0, M, 0, tid);
        for (uint64_t b = 0; b < nblocks; ++b) {
            const uint64_t o0 = head + b * B;
            __syncthreads();
            __syncthreads();
            const uint32_t n = (len - o0) < (uint64_t)B ? (uint32_t)(len - o0) : B;
            store(win, out, 0, n, o0, M, 0, tid);
        }
        if (nblocks) {
            __syncthreads();
            for (int i = tid; i < N * QPR; i += THREADS) {
                const int k = i / QPR, q = i - (i / QPR) * QPR;
                gstore(reinterpret_cast<VW*>(gwin + (size_t)k * M + q * V), ld(win, k, q * V));
            }
        }
    }
};

// Lane groups of one state write interleaved pieces of the same output lines
// (LPW elements of every row of M). Workgroups are dispatched to the XCDs
// round robin by linear id, and each XCD has its own L2: the groups of a
// state are therefore placed on one XCD (linear ids that agree mod kXcds), so
// that its L2 merges the pieces of a line before they go to memory. A launch
// covers `states` x `groups` work items on a grid of kXcds * groups *
// ceil(states / kXcds) workgroups; ids that map past the last state exit.
// State t goes to XCD (t + xoff) mod kXcds: single-state launches pass an
// offset taken from the state's address, so that concurrent launches for
// different states spread over the XCDs.
#ifndef VMT_XCD_MAP
#define VMT_XCD_MAP 1
#endif
constexpr uint32_t kXcds = 8;  // MI355X: 8 XCDs of 32 CUs
struct GroupSlot {
    uint32_t state, group;
};
__device__ __forceinline__ GroupSlot group_slot(uint32_t linear, uint32_t groups, uint32_t xoff) {
    if (!VMT_XCD_MAP) return GroupSlot{linear / groups, linear - (linear / groups) * groups};
    const uint32_t x = linear % kXcds, s = linear / kXcds;  // slot s on XCD x
    const uint32_t t = (x + kXcds - xoff) % kXcds;          // states t, t + kXcds, ... run on XCD x
    return GroupSlot{(s / groups) * kXcds + t, s - (s / groups) * groups};
}
inline uint32_t group_grid(uint32_t states, uint32_t groups) {
    return VMT_XCD_MAP ? kXcds * groups * ((states + kXcds - 1) / kXcds) : states * groups;
}
inline uint32_t state_xcd(const void* state) { return (uint32_t)(((uintptr_t)state >> 8) % kXcds); }

template <class P, int LPW, int OUT>
__global__ __launch_bounds__((mt_threads<P, LPW>())) void gen_mt_kernel(uint8_t* state, void* out, uint64_t len,
                                                                     int write_pos, uint32_t groups, uint32_t xoff) {
    using G = MtGen<P, LPW, mt_threads<P, LPW>(), OUT>;
    __shared__ __attribute__((aligned(16))) typename P::W win[(P::N + 1) * LPW];
    const GroupSlot gs = group_slot(blockIdx.x, groups, xoff);
    if (gs.state != 0) return;
    G::run(state, reinterpret_cast<typename G::OutT*>(out), len, gs.group, write_pos != 0, win);
}

// Persistent batched generation: each workgroup pops states from a counter;
// tasks are sorted longest first by the host. counter[0] hands out tasks,
// counter[1] counts finished workgroups; the last one to finish zeroes both,
// so the next launch (or graph replay) starts from a clean counter.
// TV and SW select the launch shape (threads per workgroup, store width);
// the autotuner times them. Fewer threads hold more columns per thread, so
// the register bound is relaxed with the expected waves per SIMD.
template <class P, int LANES, int OUT, int TV, int SW>
__global__ __launch_bounds__((mt_threads<P, LANES, TV>()), (TV >= 2 ? 4 : 8)) void batch_mt_kernel(
    const BatchTask* tasks, uint32_t count, uint32_t* counter) {
    using G = MtGen<P, LANES, mt_threads<P, LANES, TV>(), OUT, SW>;
    __shared__ __attribute__((aligned(16))) typename P::W win[(P::N + 1) * LANES];
    __shared__ uint32_t s_task;
    const uint32_t wave = uniform(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63;
    for (;;) {
        // Wave 0 takes a ticket without lane divergence (lane 0 adds 1, the
        // others 0): a lane-divergent branch next to the barriers of this loop
        // lets the compiler rotate the loop so that part of a wave re-enters
        // the barrier before the ticket is taken.
        if (wave == 0) {
            const uint32_t mine = atomicAdd(counter, lane == 0 ? 1u : 0u);
            s_task = uniform(mine);
        }
        __syncthreads();
        const uint32_t t = uniform(s_task);  // one task for the whole workgroup
        __syncthreads();
        if (t >= count) break;
        const BatchTask task = tasks[t];
        G::run(task.state, reinterpret_cast<typename G::OutT*>(task.out), task.len, 0, true, win);
        uint32_t* flag = uniform(task.flag);
        if (flag) {  // completion count: every wave's writes first, then one release add (lane 0 adds 1)
            __threadfence();
            __syncthreads();
            if (wave == 0)  // global address space: the compiler folds the wave's adds into one atomic
                __hip_atomic_fetch_add((VMT_GLOBAL uint32_t*)flag, lane == 0 ? 1u : 0u, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
    if (wave == 0) {
        const uint32_t done = uniform(atomicAdd(counter + 1, lane == 0 ? 1u : 0u));
        if (done == gridDim.x - 1 && lane == 0) {
            counter[0] = 0;
            counter[1] = 0;
        }
    }
}

// Measurement only: the output pattern of batch_mt_kernel (same queue, same
// launch shape, same stores of the same lengths to the same places) without
// the twist, i.e. the write rate that pattern allows. States are unchanged.
template <class P, int LANES, int TV, int SW>
__global__ __launch_bounds__((mt_threads<P, LANES, TV>()), (TV >= 2 ? 4 : 8)) void write_pattern_kernel(
    const BatchTask* tasks, uint32_t count, uint32_t* counter) {
    using G = MtGen<P, LANES, mt_threads<P, LANES, TV>(), 0, SW>;
    __shared__ __attribute__((aligned(16))) typename P::W win[(P::N + 1) * LANES];
    __shared__ uint32_t s_task;
    const uint32_t wave = uniform(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63;
    for (;;) {
        if (wave == 0) {
            const uint32_t mine = atomicAdd(counter, lane == 0 ? 1u : 0u);
            s_task = uniform(mine);
        }
        __syncthreads();
        const uint32_t t = uniform(s_task);
        __syncthreads();
        if (t >= count) break;
        const BatchTask task = tasks[t];
        G::run_pattern(task.state, reinterpret_cast<typename G::OutT*>(task.out), task.len, win);
    }
    if (wave == 0) {
        const uint32_t done = uniform(atomicAdd(counter + 1, lane == 0 ? 1u : 0u));
        if (done == gridDim.x - 1 && lane == 0) {
            counter[0] = 0;
            counter[1] = 0;
        }
    }
}

// Measurement only: writes of n16 16-byte words of `v` in two patterns.
// fill_pieces: one-shot workgroups of 256 threads, each storing one 4 KiB
// piece, in address order (a plain fill). fill_regions: `gridDim.x`
// persistent workgroups, each writing its own contiguous region of `per16`
// words in order (the last one the remainder), which is the output pattern
// of many independent generators at once.
template <bool NT>
__device__ __forceinline__ void fill_store(uint4* p, uint32_t v) {
    using D = DwordVec<4>::type;
    const D d = {v, v, v, v};
    if constexpr (NT) __builtin_nontemporal_store(d, (VMT_GLOBAL D*)p);
    else *(VMT_GLOBAL D*)p = d;
}
template <bool NT>
__global__ __launch_bounds__(256) void fill_pieces(uint4* p, uint64_t n16, uint32_t v) {
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n16) fill_store<NT>(p + i, v);
}
template <bool NT>
__global__ __launch_bounds__(256) void fill_regions(uint4* p, uint64_t n16, uint64_t per16, uint32_t v) {
    const uint64_t lo = (uint64_t)blockIdx.x * per16;
    const uint64_t hi = blockIdx.x + 1 == gridDim.x ? n16 : lo + per16;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += 256) fill_store<NT>(p + i, v);
}

// ---------------------------------------------------------------------------
// SFMT generation: a quad of threads per lane runs the lane's serial chain
// (the recurrence reads the two previous words, Sec. 2.6; sfmt_block_quad),
// lanes in parallel.
// ---------------------------------------------------------------------------

template <int N, int LPW, int OUT>
struct SfmtGen {
    using OutT = typename OutOf<OUT == 0 ? 0 : 1, uint32_t>::T;

    static __device__ __forceinline__ OutT map(uint32_t v) {
        if constexpr (OUT == 0) return v;
        else return to_f32(v);
    }
    static __device__ __forceinline__ uint32_t sub(const uint4& w, uint32_t j) {
        return j == 0 ? w.x : j == 1 ? w.y : j == 2 ? w.z : w.w;
    }

    // Lane group g (lanes g*LPW ...): quad q of the workgroup runs lane
    // lane0 + q, its thread j sub-word j, with the lane's window in registers
    // (sfmt_block_regs); threads past the group idle.
    static __device__ __forceinline__ void run(uint8_t* state, OutT* out, uint64_t len, uint32_t g, bool write_pos) {
        state = uniform(state);
        out = uniform(out);
        len = uniform(len);
        StateHeader* hdr = reinterpret_cast<StateHeader*>(state);
        const uint32_t M = uniform(hdr->M);
        const uint32_t pos = uniform(hdr->pos);
        uint32_t* gw32 = reinterpret_cast<uint32_t*>(state + kHeaderBytes);  // sub-word j of word k, lane t: [(k M + t) 4 + j]
        const uint32_t B = 4u * N * M;  // uint32 elements per block
        if (len == 0) return;
        const int tid = threadIdx.x & 63;  // one wavefront runs the lane group
        const uint32_t lane0 = g * LPW;
        const uint64_t head = len < (uint64_t)(B - pos) ? len : (uint64_t)(B - pos);
        const uint64_t rest = len - head;
        const uint64_t nblocks = (rest + B - 1) / B;
        const QuadThread qt = sfmt_quad_thread(tid);
        const int q = qt.q, j = qt.j;
        if (q < LPW) {
            const uint32_t o = 4u * (lane0 + q) + j;  // stream offset of this sub-word within a word row
            const uint32_t step = __builtin_amdgcn_readfirstlane(4u * M);
            uint32_t R[N];
#pragma unroll
            for (int k = 0; k < N; ++k) R[k] = gw32[k * step + o];
            if (head) {  // the rest of the current block: words of the window at stream offsets [pos, pos + head)
                uint32_t sth = step;  // opaque to the compiler, as below: the load addresses are not kept for this
                asm volatile("" : "+s"(sth));
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    const uint32_t p = k * sth + o;
                    if (p >= pos && p < pos + (uint32_t)head) gstore(out + (p - pos), map(R[k]));
                }
            }
            // Whole blocks, then at most one partial block. The output of word k's sub-word j is
            // out[o0 + step k + o]: a wave-uniform base (scalar registers, advanced by the scalar unit)
            // plus this thread's fixed offset, so a step spends no vector instruction on addressing.
            const uint64_t nfull = rest / B;
            for (uint64_t b = 0; b < nfull; ++b) {
                uint64_t base = reinterpret_cast<uint64_t>(out + (head + b * B));
                sfmt_block_regs<N>(R, j, [&](int, uint32_t r) {
                    gstore(reinterpret_cast<OutT*>(uniform(base)) + o, map(r));
                    base += (uint64_t)step * sizeof(OutT);
                });
            }
            if (nfull < nblocks) {
                const uint64_t o0 = head + nfull * B;
                const uint32_t lim = (uint32_t)(len - o0);
                const int kmax = o < lim ? (int)((lim - o + step - 1) / step) : 0;  // steps whose output is in range
                uint64_t base = reinterpret_cast<uint64_t>(out + o0);
                sfmt_block_regs<N>(R, j, [&](int k, uint32_t r) {
                    if (k < kmax) gstore(reinterpret_cast<OutT*>(uniform(base)) + o, map(r));
                    base += (uint64_t)step * sizeof(OutT);
                });
            }
            if (nblocks) {
                // a stride the compiler cannot match with the loads' above: it recomputes these
                // addresses instead of keeping N of them live through the block loop (likewise the head's)
                uint32_t st2 = step;
                asm volatile("" : "+s"(st2));
#pragma unroll
                for (int k = 0; k < N; ++k) gw32[k * st2 + o] = R[k];
            }
        }
        // the wavefront read the header above, in program order, before its lane 0 writes it here
        if (write_pos && tid == 0)
            hdr->pos = nblocks ? (uint32_t)(rest - (nblocks - 1) * (uint64_t)B) : (uint32_t)(pos + head);
    }
};

// Four wavefronts per workgroup, each running one lane group (of one task)
// on its own: the four land on the four SIMDs of a compute unit. One chain
// per SIMD matters, since a chain is issue-bound: two wavefronts on one SIMD
// halve each one's step rate, and separate one-wavefront workgroups were
// found to pair up on SIMDs.
constexpr int kSfmtWavesPerWg = 4;

template <int N, int LPW, int OUT>
__global__ __launch_bounds__(64 * kSfmtWavesPerWg, 3) void gen_sfmt_kernel(uint8_t* state, void* out, uint64_t len,
                                                                         int write_pos, uint32_t groups) {
    using G = SfmtGen<N, LPW, OUT>;
    const uint32_t g = blockIdx.x * kSfmtWavesPerWg + uniform((uint32_t)threadIdx.x >> 6);
    if (g >= groups) return;
    G::run(state, reinterpret_cast<typename G::OutT*>(out), len, g, write_pos != 0);
}

// Batched SFMT generation: workgroup (g, t) runs lane group g of task t.
// With several groups per state the positions are fixed afterwards
// (finalize_batch_pos), since every group reads the header first.
template <int N, int LPW, int OUT>
__global__ __launch_bounds__(64 * kSfmtWavesPerWg, 3) void batch_sfmt_kernel(const BatchTask* tasks, uint32_t count,
                                                                           uint32_t groups) {
    using G = SfmtGen<N, LPW, OUT>;
    const uint32_t item = blockIdx.x * kSfmtWavesPerWg + uniform((uint32_t)threadIdx.x >> 6);
    const uint32_t t = item / groups, g = item - t * groups;
    if (t >= count) return;
    const BatchTask task = tasks[t];
    G::run(task.state, reinterpret_cast<typename G::OutT*>(task.out), task.len, g, groups == 1);
}

// Position of a task's state after its len elements (from the position before).
__device__ __forceinline__ void batch_final_pos(const BatchTask& task) {
    StateHeader* hdr = reinterpret_cast<StateHeader*>(task.state);
    const uint64_t B = hdr->block, pos = hdr->pos, len = task.len;
    const uint64_t head = len < B - pos ? len : B - pos;
    const uint64_t rest = len - head;
    const uint64_t nblocks = (rest + B - 1) / B;
    hdr->pos = nblocks ? (uint32_t)(rest - (nblocks - 1) * B) : (uint32_t)(pos + head);
}

// Batched MT generation by lane groups (the chunks of a split call):
// workgroup (g, t) runs lane group g of task t with the single-state code, so
// a chunk's M lanes spread over M / LPW workgroups. With several groups per
// state the positions are fixed afterwards: by finalize_batch_pos, or, with
// `done` (one zeroed counter per task), by the last of a task's workgroups to
// finish. That one counts after every other has, and each counts after its
// own reads of the position have returned (the barrier), so no read of the old
// position follows the write, which depends on the count. The count is
// relaxed: a release would write back the L2's dirty output lines at every
// workgroup's end; the kernel's end publishes the position.
template <class P, int LPW, int OUT>
__global__ __launch_bounds__((mt_threads<P, LPW>())) void batch_gen_mt_kernel(const BatchTask* tasks, uint32_t count,
                                                                           uint32_t groups, uint32_t* done) {
    using G = MtGen<P, LPW, mt_threads<P, LPW>(), OUT>;
    __shared__ __attribute__((aligned(16))) typename P::W win[(P::N + 1) * LPW];
    const GroupSlot gs = group_slot(blockIdx.x, groups, 0);
    if (gs.state >= count) return;
    const BatchTask task = tasks[gs.state];
    G::run(task.state, reinterpret_cast<typename G::OutT*>(task.out), task.len, gs.group, groups == 1, win);
    if (done && groups > 1) {
        __syncthreads();  // the whole workgroup is past its reads of the header
        if (threadIdx.x == 0 &&
            __hip_atomic_fetch_add(done + gs.state, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == groups - 1)
            batch_final_pos(task);
    }
}

// Copy whole states (header and window; `bytes` a multiple of 16): task y
// copies tasks[y].src to tasks[y].dst.
__global__ void copy_states(const CopyTask* tasks, uint32_t bytes) {
    const CopyTask t = tasks[blockIdx.y];
    const uint4* s = reinterpret_cast<const uint4*>(t.src);
    uint4* d = reinterpret_cast<uint4*>(t.dst);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < bytes / 16; i += gridDim.x * blockDim.x) d[i] = s[i];
}

// Set-up of a split call in one launch: the chunks' generation tasks, the
// jump tasks of chunks 1 .. C-1 and the copies of the state (header and
// window) that chunks 0 .. C-2 run on. Chunk c covers output elements
// [c E, (c + 1) E), the last one the rest of n, and runs on copy c (the last
// chunk on the state itself); chunk c >= 1 is jumped by slot c - 1 of `polys`
// (degree deg[c - 1]). Workgroup (x, c) copies its share of copy c, and
// thread 0 of workgroup (0, c) writes chunk c's tasks and zeroes its counter
// in `done` (if given) for the generation's workgroups.
__global__ void split_setup(const uint8_t* state, uint8_t* copies, uint32_t bytes, uint64_t stride, uint32_t C,
                            uint8_t* out, uint64_t E, uint64_t n, uint32_t eb, const uint64_t* polys,
                            const uint32_t* deg, BatchTask* bt, JumpTask* jt, uint32_t* done) {
    const uint32_t c = blockIdx.y;
    uint8_t* st = c + 1 == C ? const_cast<uint8_t*>(state) : copies + stride * c;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        bt[c] = BatchTask{st, out + (uint64_t)c * E * eb, c + 1 < C ? E : n - (uint64_t)c * E, nullptr};
        if (c) jt[c - 1] = JumpTask{st, polys + (size_t)(c - 1) * kPolyWords, 0u, deg[c - 1], nullptr};
        if (done) done[c] = 0;
    }
    if (c + 1 == C) return;
    const uint4* s = reinterpret_cast<const uint4*>(state);
    uint4* d = reinterpret_cast<uint4*>(st);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < bytes / 16; i += gridDim.x * blockDim.x) d[i] = s[i];
}

// Position after a call that emitted `len` elements, for launches with several
// workgroups per state (none of them may touch the header while others read it).
__global__ void finalize_gen_pos(uint8_t* state, uint64_t len) {
    StateHeader* hdr = reinterpret_cast<StateHeader*>(state);
    const uint64_t B = hdr->block, pos = hdr->pos;
    const uint64_t head = len < B - pos ? len : B - pos;
    const uint64_t rest = len - head;
    const uint64_t nblocks = (rest + B - 1) / B;
    hdr->pos = nblocks ? (uint32_t)(rest - (nblocks - 1) * B) : (uint32_t)(pos + head);
}

__global__ void reset_counter(uint32_t* c) { c[threadIdx.x] = 0; }

__global__ void finalize_batch_pos(const BatchTask* tasks, uint32_t count) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    batch_final_pos(tasks[i]);
}

// ---------------------------------------------------------------------------
// Raw-sequence regeneration for the jump: rows of a lane-major buffer,
// `src` -> `dst` (different buffers, so there is no read/write hazard).
// ---------------------------------------------------------------------------

template <class P>
__device__ void raw_twist_rows(const typename P::W* src, typename P::W* dst, int rows, int stride, int tid, int nthr) {
    using W = typename P::W;
    constexpr int N = P::N, MM = P::MM, D = P::D;
    for (int it = tid; it < rows * D; it += nthr) {
        const int row = it / D, c = it - (it / D) * D;
        const W* s = src + row * stride;
        W* d = dst + row * stride;
        const W n0 = twist(s[c], s[c + 1], s[c + MM]);
        d[c] = n0;
        const int r1 = c + D;
        const W b1 = (r1 + 1 < N) ? s[r1 + 1] : twist(s[0], s[1], s[MM]);
        const W n1 = twist(s[r1], b1, n0);
        d[r1] = n1;
        const int r2 = c + 2 * D;
        if (r2 < N) {
            const W b2 = (r2 + 1 < N) ? s[r2 + 1] : twist(s[0], s[1], s[MM]);
            d[r2] = twist(s[r2], b2, n1);
        }
    }
}


template <int N>
__device__ void raw_twist_rows_sfmt(const uint4* src, uint4* dst, int rows, int stride, int tid) {
    const QuadThread qt = sfmt_quad_thread(tid);  // one quad of threads per row
    const int row = qt.q, j = qt.j;
    if (row >= rows) return;
    sfmt_block_quad<N>(reinterpret_cast<const uint32_t*>(src + row * stride), reinterpret_cast<uint32_t*>(dst + row * stride),
                       4, j, [](int, uint32_t) {});
}

__device__ __forceinline__ uint32_t xorw(uint32_t a, uint32_t b) { return a ^ b; }
__device__ __forceinline__ uint64_t xorw(uint64_t a, uint64_t b) { return a ^ b; }
__device__ __forceinline__ uint4 xorw(uint4 a, uint4 b) { return make_uint4(a.x ^ b.x, a.y ^ b.y, a.z ^ b.z, a.w ^ b.w); }
// a ^ b ^ c as one three-input bitwise operation per 32 bits (truth table 0x96)
__device__ __forceinline__ uint32_t xorw3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint64_t xorw3(uint64_t a, uint64_t b, uint64_t c) {
    return (uint64_t)xorw3((uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32)) << 32 |
           xorw3((uint32_t)a, (uint32_t)b, (uint32_t)c);
}
__device__ __forceinline__ uint4 xorw3(uint4 a, uint4 b, uint4 c) {
    return make_uint4(xorw3(a.x, b.x, c.x), xorw3(a.y, b.y, c.y), xorw3(a.z, b.z, c.z), xorw3(a.w, b.w, c.w));
}
template <class W>
__device__ __forceinline__ W zero_w() { return W(0); }
template <>
__device__ __forceinline__ uint4 zero_w<uint4>() { return make_uint4(0, 0, 0, 0); }

// acc[s] ^= row[s0 + lane + 64 s] for every set coefficient i of poly with
// window start s0 = k + i - b*N inside [0, N).
template <class W, int N>
__device__ __forceinline__ void accumulate_block(W (&acc)[(N + 63) / 64], const W* row, const uint64_t* poly,
                                                 int k, int b, int max_deg, int lane) {
    constexpr int S = (N + 63) / 64;
    int lo = b * N - k, hi = (b + 1) * N - k;  // coefficient range for this block
    if (lo < 0) lo = 0;
    if (hi > max_deg + 1) hi = max_deg + 1;
    if (lo >= hi) return;
    for (int wi = lo >> 6; wi <= (hi - 1) >> 6; ++wi) {
        uint64_t bits = uniform(poly[wi]);  // scalar: the loop over coefficients runs on the scalar unit
        const int base = wi * 64;
        if (base < lo) bits &= ~0ull << (lo - base);
        if (base + 64 > hi) bits &= (hi - base >= 64) ? ~0ull : ((1ull << (hi - base)) - 1);
        while (bits) {
            const int p = __builtin_ctzll(bits);
            bits &= bits - 1;
            const W* src = row + (k + base + p - b * N) + lane;
#pragma unroll
            for (int s = 0; s < S; ++s)
                if (s < S - 1 || lane + 64 * s < N) acc[s] = xorw(acc[s], src[64 * s]);
        }
    }
}

// Grouped form: coefficients are taken four at a time. For a group with
// pattern p (bits of g at 4u .. 4u+3) the contribution to word j is the XOR
// of x_{4u+e+j} over the set bits e of p, which is word (4u + e0 + j) of the
// derived row D[p >> e0] (e0 the lowest set bit): D[q]_m = XOR of x_{m+e}
// over the set bits e of the odd pattern q. One LDS read per non-zero group
// instead of one per set coefficient: about 15/32 of the reads for a dense g.
// rows: the eight derived rows (q = 1, 3, .., 15), `rstride` words apart.
// Part `part` of `parts` takes the part-th contiguous slice of the block's
// coefficient range (XOR is linear: the parts' sums add up to the block's).
// PADDED: the buffer extends jump_pad_words<N>() words past the last derived
// row, so the reads of the last partial wavefront row need no range test
// (lanes past the window read words they never store). [clo, chi) further
// limits the coefficients taken (a part of a lane jump split by coefficient
// range).
template <class W, int N, bool PADDED = false>
__device__ __forceinline__ void accumulate_block4(W (&acc)[(N + 63) / 64], const W* rows, int rstride,
                                                  const uint64_t* poly, int k, int b, int max_deg, int lane,
                                                  int part, int parts, int clo = 0, int chi = 1 << 30) {
    constexpr int S = (N + 63) / 64;
    int lo = b * N - k, hi = (b + 1) * N - k;  // coefficient range for this block
    if (lo < clo) lo = clo;
    if (lo < 0) lo = 0;
    if (hi > chi) hi = chi;
    if (hi > max_deg + 1) hi = max_deg + 1;
    if (lo >= hi) return;
    if (parts > 1) {
        const int len = hi - lo;
        hi = lo + (len * (part + 1)) / parts;
        lo = lo + (len * part) / parts;
        if (lo >= hi) return;
    }
    const int off0 = k - b * N + lane;
    // The 16 groups of a 64-coefficient word are decoded side by side, lane u
    // taking group u (lanes 16 .. 63 repeat them): its pattern, lowest set bit
    // e0 and row offset. The scalar loop then walks the mask of non-zero groups
    // and reads each offset from its lane.
    const int u = lane & 15;
    for (int wi = lo >> 6; wi <= (hi - 1) >> 6; ++wi) {
        uint64_t bits = uniform(poly[wi]);
        const int base = wi * 64;
        if (base < lo) bits &= ~0ull << (lo - base);
        if (base + 64 > hi) bits &= (hi - base >= 64) ? ~0ull : ((1ull << (hi - base)) - 1);
        if (!bits) continue;
        const uint32_t pat = (uint32_t)(bits >> (4 * u)) & 0xFu;
        const int e0 = __builtin_ctz(pat | 0x10u);
        const int grp_off = (int)((pat >> e0) >> 1) * rstride + 4 * u + e0;  // odd pattern from e0 up
        uint64_t live = __ballot(pat != 0) & 0xFFFFull;  // non-zero groups (lanes 0 .. 15)
        auto next_group = [&]() {  // row offset of the lowest remaining group; clears it
            const int g = __builtin_ctzll(live);
            live &= live - 1;
            return base + __builtin_amdgcn_readlane(grp_off, g);
        };
        while (live) {
            // two groups per round: the second group's reads are in flight with the first's
            const W* sa = rows + off0 + next_group();
            W va[S], vb[S];
#pragma unroll
            for (int s = 0; s < S; ++s)
                va[s] = (PADDED || s < S - 1 || lane + 64 * s < N) ? sa[64 * s] : zero_w<W>();
            if (live) {
                const W* sb = rows + off0 + next_group();
#pragma unroll
                for (int s = 0; s < S; ++s)
                    vb[s] = (PADDED || s < S - 1 || lane + 64 * s < N) ? sb[64 * s] : zero_w<W>();
#pragma unroll
                for (int s = 0; s < S; ++s) acc[s] = xorw3(acc[s], va[s], vb[s]);
            } else {
#pragma unroll
                for (int s = 0; s < S; ++s) acc[s] = xorw(acc[s], va[s]);
            }
        }
    }
}

// Groups of five coefficients: as accumulate_block4, with the derived rows of
// the 16 odd 5-bit patterns (derive_rows5). The coefficients are decoded 60 at
// a time (12 groups, from two polynomial words), so no group straddles a
// decoding step; the block's range [lo, hi) masks each pattern, so every term
// taken lies in the block. Fewer window reads (one per nonzero group of 5)
// for twice the derived rows.
template <class W, int N>
__device__ __forceinline__ void accumulate_block5(W (&acc)[(N + 63) / 64], const W* rows, int rstride,
                                                  const uint64_t* poly, int k, int b, int max_deg, int lane, int clo,
                                                  int chi) {
    constexpr int S = (N + 63) / 64;
    int lo = b * N - k, hi = (b + 1) * N - k;
    if (lo < clo) lo = clo;
    if (lo < 0) lo = 0;
    if (hi > chi) hi = chi;
    if (hi > max_deg + 1) hi = max_deg + 1;
    if (lo >= hi) return;
    const int off0 = k - b * N + lane;
    const int u = lane < 12 ? lane : 0;
    for (int base = lo / 60 * 60; base < hi; base += 60) {
        const int w0 = base >> 6, sh = base & 63;
        uint64_t bits = uniform(poly[w0]) >> sh;
        if (sh > 4) bits |= uniform(poly[w0 + 1]) << (64 - sh);
        bits &= (1ull << 60) - 1;
        if (base < lo) bits &= ~0ull << (lo - base);
        if (base + 60 > hi) bits &= (1ull << (hi - base)) - 1;
        if (!bits) continue;
        const uint32_t pat = (uint32_t)(bits >> (5 * u)) & 31u;
        const int e0 = __builtin_ctz(pat | 32u);
        const int grp_off = (int)((pat >> e0) >> 1) * rstride + 5 * u + e0;
        uint64_t live = __ballot(lane < 12 && pat != 0) & 0xFFFull;
        auto next_group = [&]() {
            const int g = __builtin_ctzll(live);
            live &= live - 1;
            return base + __builtin_amdgcn_readlane(grp_off, g);
        };
        while (live) {
            const W* sa = rows + off0 + next_group();
            W va[S], vb[S];
#pragma unroll
            for (int s = 0; s < S; ++s) va[s] = sa[64 * s];
            if (live) {
                const W* sb = rows + off0 + next_group();
#pragma unroll
                for (int s = 0; s < S; ++s) vb[s] = sb[64 * s];
#pragma unroll
                for (int s = 0; s < S; ++s) acc[s] = xorw3(acc[s], va[s], vb[s]);
            } else {
#pragma unroll
                for (int s = 0; s < S; ++s) acc[s] = xorw(acc[s], va[s]);
            }
        }
    }
}

// Derived rows of the 16 odd 5-bit patterns q = 1, 3, .., 31 (row q >> 1;
// row 0 is the raw row), for m in [0, 2N), words past the window counting as
// zero: D[q + 16]_m = D[q]_m ^ x_{m+4}.
template <class W, int N>
__device__ __forceinline__ void derive_rows5(W* x, int rstride, int tid, int nthr) {
    for (int m = tid; m < 2 * N; m += nthr) {
        const W z = zero_w<W>();
        const W x0 = x[m], x1 = m + 1 < 2 * N ? x[m + 1] : z, x2 = m + 2 < 2 * N ? x[m + 2] : z,
                x3 = m + 3 < 2 * N ? x[m + 3] : z, x4 = m + 4 < 2 * N ? x[m + 4] : z;
        W d[8];
        d[0] = x0;
        d[1] = xorw(x0, x1);
        d[2] = xorw(x0, x2);
        d[3] = xorw(d[1], x2);
        d[4] = xorw(x0, x3);
        d[5] = xorw(d[1], x3);
        d[6] = xorw(d[2], x3);
        d[7] = xorw(d[3], x3);
#pragma unroll
        for (int r = 1; r < 8; ++r) x[r * rstride + m] = d[r];
#pragma unroll
        for (int r = 0; r < 8; ++r) x[(r + 8) * rstride + m] = xorw(d[r], x4);
    }
}

// Derived rows D[q]_m, q = 3, 5, .., 15, for m in [0, 2N) of every row (the
// raw row is D[1]); words past the window count as zero (no read of a valid
// group reaches them: the group's highest set coefficient is in range).
template <class W, int N>
__device__ __forceinline__ void derive_rows(W* buf, int rows, int rstride, int row_stride, int tid, int nthr) {
    for (int it = tid; it < rows * 2 * N; it += nthr) {
        const int r = it / (2 * N), m = it - r * (2 * N);
        W* x = buf + r * row_stride;
        const W z = zero_w<W>();
        const W x0 = x[m], x1 = m + 1 < 2 * N ? x[m + 1] : z, x2 = m + 2 < 2 * N ? x[m + 2] : z,
                x3 = m + 3 < 2 * N ? x[m + 3] : z;
        const W d3 = xorw(x0, x1), d5 = xorw(x0, x2), d7 = xorw(d3, x2);
        x[1 * rstride + m] = d3;
        x[2 * rstride + m] = d5;
        x[3 * rstride + m] = d7;
        x[4 * rstride + m] = xorw(x0, x3);
        x[5 * rstride + m] = xorw(d3, x3);
        x[6 * rstride + m] = xorw(d5, x3);
        x[7 * rstride + m] = xorw(d7, x3);
    }
}

// ---- seeding (the base generators' published init_genrand / init_by_array;
// the paper starts from a given state and leaves seeding open)
__device__ void seed_mt32(uint32_t* x, const InitTask& t) {
    if (t.kind == kSeedGenrand) {
        x[0] = (uint32_t)t.seed;
        for (uint32_t i = 1; i < 624; i++) x[i] = 1812433253u * (x[i - 1] ^ (x[i - 1] >> 30)) + i;
        return;
    }
    x[0] = 19650218u;
    for (uint32_t i = 1; i < 624; i++) x[i] = 1812433253u * (x[i - 1] ^ (x[i - 1] >> 30)) + i;
    uint32_t i = 1, j = 0;
    const uint32_t klen = t.key_len;
    for (uint32_t s = (624 > klen ? 624 : klen); s; --s) {
        x[i] = (x[i] ^ ((x[i - 1] ^ (x[i - 1] >> 30)) * 1664525u)) + t.key[j] + j;
        if (++i >= 624) {
            x[0] = x[623];
            i = 1;
        }
        if (++j >= klen) j = 0;
    }
    for (uint32_t s = 623; s; --s) {
        x[i] = (x[i] ^ ((x[i - 1] ^ (x[i - 1] >> 30)) * 1566083941u)) - i;
        if (++i >= 624) {
            x[0] = x[623];
            i = 1;
        }
    }
    x[0] = 0x80000000u;
}
__device__ void seed_mt64(uint64_t* x, const InitTask& t) {
    x[0] = t.seed;
    for (uint64_t i = 1; i < 312; i++) x[i] = 6364136223846793005ull * (x[i - 1] ^ (x[i - 1] >> 62)) + i;
}
template <int N>
__device__ void seed_sfmt(uint4* w, const InitTask& t) {
    using P = SfmtP<N>;
    uint32_t* x = reinterpret_cast<uint32_t*>(w);
    x[0] = (uint32_t)t.seed;
    for (uint32_t i = 1; i < 4 * N; i++) x[i] = 1812433253u * (x[i - 1] ^ (x[i - 1] >> 30)) + i;
    // period certification: if <PARITY, word 0> is even, flip the lowest set bit of PARITY
    const uint32_t inner = (x[0] & P::P0) ^ (x[1] & P::P1) ^ (x[2] & P::P2) ^ (x[3] & P::P3);
    if ((__builtin_popcount(inner) & 1) == 0) {
        const uint32_t pv[4] = {P::P0, P::P1, P::P2, P::P3};
        for (int j = 0; j < 4; j++)
            if (pv[j]) {
                x[j] ^= pv[j] & (0u - pv[j]);
                break;
            }
    }
}

template <class W, int N>
__device__ void seed_state(W* x, const InitTask& t) {
    if constexpr (std::is_same<W, uint32_t>::value) seed_mt32(x, t);
    else if constexpr (std::is_same<W, uint64_t>::value) seed_mt64(x, t);
    else seed_sfmt<N>(x, t);
}

template <class W, int N>
__device__ void twist_rows(const W* src, W* dst, int rows, int stride, int tid, int nthr) {
    if constexpr (std::is_same<W, uint32_t>::value) raw_twist_rows<MT32P>(src, dst, rows, stride, tid, nthr);
    else if constexpr (std::is_same<W, uint64_t>::value) raw_twist_rows<MT64P>(src, dst, rows, stride, tid, nthr);
    else raw_twist_rows_sfmt<N>(src, dst, rows, stride, tid);
}

// ---------------------------------------------------------------------------
// Init and jump. G lanes per workgroup, one wavefront per lane.
//   init: the raw sequence is the seeded base generator's (one shared row),
//         lane t uses polynomial slot t, offset k = N (start one block in).
//   jump: each lane regenerates its own row from its window, all lanes use
//         the same polynomial, offset k = pos / M (whole words consumed).
// Buffer: rows of 2N words (lower = block b, upper = block b + 1).
// ---------------------------------------------------------------------------

// Words of LDS per raw row: the 2N-word window, and with grouped
// accumulation its seven derived rows after it. Grouped accumulation reads
// LDS about half as often but needs eight times the LDS per row: it is used
// where the raw row is shared (seeding: one row for all lanes of a
// workgroup) and for jumps of few lanes, where latency matters; many lanes
// at once run faster per coefficient (more of them fit on a compute unit).
template <int N, bool GROUPED>
constexpr int jump_row_words() {
    return GROUPED ? 8 * 2 * N : 2 * N;
}
// Words past the last derived row that the unguarded reads of a padded
// buffer can reach: a wavefront row reads 64 * ceil(N / 64) words from a
// start below N in the last row.
template <int N>
constexpr int jump_pad_words() {
    return 64 * ((N + 63) / 64) - N;
}
// uint64 polynomial words staged in LDS by a sliced jump, in units of W
template <class W>
constexpr int jump_poly_stage_words() {
    return (int)((kPolyWords * sizeof(uint64_t) + sizeof(W) - 1) / sizeof(W));
}

// WPL wavefronts per lane (jumps of few lanes): they share the lane's raw
// row, each sums its slice of every block's coefficients, and the slices'
// sums are XORed together at the end.
template <class W, int N, int G, bool INIT, bool GROUPED, int WPL = 1>
__device__ void dephase(uint8_t* state, uint32_t M, uint32_t g, const uint64_t* poly, uint32_t lane_stride,
                        int max_deg, int k, const InitTask* init, W* buf) {
    constexpr int S = (N + 63) / 64;
    constexpr int ROWS = INIT ? 1 : G;
    constexpr int RW = jump_row_words<N, GROUPED>();  // words from one raw row to the next
    static_assert(WPL == 1 || (GROUPED && !INIT && G == 1 && WPL * N <= RW), "sliced sums need the grouped jump's LDS");
    // Sliced jumps: the buffer is padded (unguarded reads), and with 8 or more
    // wavefronts the lane's polynomial is staged in LDS after the pad, so that
    // each block's first coefficient word is an LDS read rather than a global
    // one on the critical path.
    constexpr bool PADDED = WPL > 1;
    constexpr bool STAGED = WPL >= 8;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int w = wave / WPL;             // lane of the group handled by this wave
    const int part = wave - w * WPL;      // its slice of the coefficients
    state = uniform(state);
    poly = uniform(poly);
    k = (int)uniform((uint32_t)k);
    max_deg = (int)uniform((uint32_t)max_deg);
    M = uniform(M);
    W* gwin = reinterpret_cast<W*>(state + kHeaderBytes);
    const uint32_t lane0 = g * G;

    if constexpr (INIT) {
        if (tid == 0) seed_state<W, N>(buf, *init);
    } else {
        for (int i = tid; i < N * G; i += nthr) {
            const int j = i / G, r = i - (i / G) * G;
            buf[r * RW + j] = gwin[(size_t)j * M + lane0 + r];
        }
    }
    uint64_t* spoly = reinterpret_cast<uint64_t*>(buf + RW * G + jump_pad_words<N>());
    if constexpr (STAGED) {
        const uint64_t* src = poly + (size_t)lane_stride * lane0;
        for (int i = tid; i <= (max_deg >> 6); i += nthr) spoly[i] = src[i];
    }
    __syncthreads();
    twist_rows<W, N>(buf, buf + N, ROWS, RW, tid, nthr);
    __syncthreads();
    if constexpr (GROUPED) {
        derive_rows<W, N>(buf, ROWS, 2 * N, RW, tid, nthr);
        __syncthreads();
    }

    W acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = zero_w<W>();
    const uint64_t* mypoly = STAGED ? spoly : poly + (size_t)lane_stride * (lane0 + w);
    const W* myrow = buf + (INIT ? 0 : w * RW);
    const int last_b = (k + max_deg) / N;
    for (int b = 0; b <= last_b; ++b) {
        if (w < G) {
            if constexpr (GROUPED)
                accumulate_block4<W, N, PADDED>(acc, myrow, 2 * N, mypoly, k, b, max_deg, lane, part, WPL);
            else accumulate_block<W, N>(acc, myrow, mypoly, k, b, max_deg, lane);
        }
        if (b == last_b) break;
        __syncthreads();
        for (int i = tid; i < ROWS * N; i += nthr) {  // upper -> lower
            const int r = i / N, j = i - (i / N) * N;
            buf[r * RW + j] = buf[r * RW + N + j];
        }
        __syncthreads();
        twist_rows<W, N>(buf, buf + N, ROWS, RW, tid, nthr);
        __syncthreads();
        if constexpr (GROUPED) {
            derive_rows<W, N>(buf, ROWS, 2 * N, RW, tid, nthr);
            __syncthreads();
        }
    }
    __syncthreads();
    if constexpr (WPL > 1) {  // XOR the slices' sums and store rows of G contiguous words
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int j = lane + 64 * s;
            if (j < N) buf[wave * N + j] = acc[s];
        }
        __syncthreads();
        for (int i = tid; i < N * G; i += nthr) {
            const int j = i / G, r = i - (i / G) * G;
            W v = buf[(r * WPL) * N + j];
#pragma unroll
            for (int q = 1; q < WPL; ++q) v = xorw(v, buf[(r * WPL + q) * N + j]);
            gwin[(size_t)j * M + lane0 + r] = v;
        }
        return;
    }
    // stage as [j][lane] and store rows of G contiguous words
    if (w < G) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int j = lane + 64 * s;
            if (j < N) buf[j * G + w] = acc[s];
        }
    }
    __syncthreads();
    for (int i = tid; i < N * G; i += nthr) {
        const int j = i / G, r = i - (i / G) * G;
        gwin[(size_t)j * M + lane0 + r] = buf[i];
    }
}

template <class W, int N, int G>
__global__ __launch_bounds__(G * 64) void init_kernel(const InitTask* tasks, InitTask one, uint32_t M,
                                                      const uint64_t* lane_polys, uint32_t max_deg, uint32_t variant) {
    constexpr int BUF = (jump_row_words<N, true>() > N * G) ? jump_row_words<N, true>() : N * G;
    __shared__ __attribute__((aligned(16))) W buf[BUF];
    const uint32_t groups = M / G;
    const uint32_t ti = blockIdx.x / groups, g = blockIdx.x - ti * groups;
    const InitTask task = tasks ? tasks[ti] : one;
    dephase<W, N, G, true, true>(task.state, M, g, lane_polys, kPolyWords, (int)max_deg, N, &task, buf);
    if (g == 0 && threadIdx.x == 0) {
        StateHeader* h = reinterpret_cast<StateHeader*>(task.state);
        h->magic = kMagic;
        h->version = kVersion;
        h->variant = variant;
        h->M = M;
        h->n = N;
        h->word_bytes = sizeof(W);
        h->block = (uint32_t)(N * M * (sizeof(W) == 16 ? 4 : 1));
        h->pos = 0;
        for (int i = 0; i < (int)(sizeof(h->reserved) / sizeof(h->reserved[0])); ++i) h->reserved[i] = 0;
    }
}

// One lane's jump by a workgroup of 16 wavefronts, pipelined over two LDS
// row sets (raw window of two blocks and its derived rows, padded): while
// wavefronts 1 .. 15 sum their slices of block b's coefficients from one set,
// wavefront 0 builds block b + 1's window in the other (its lower half is the
// current upper half, its upper half the next twist, then the derived rows),
// so a block costs one barrier. Wavefront 0 works alone on its set: its LDS
// writes and later reads of them are ordered by a wavefront-scope fence.
template <class W, int N>
__device__ void jump_pipelined(uint8_t* state, uint32_t M, uint32_t lane0, const uint64_t* poly, int max_deg, int k,
                               W* buf) {
    constexpr int S = (N + 63) / 64;
    constexpr int RW = jump_row_words<N, true>();
    constexpr int SET = RW + jump_pad_words<N>();  // words of one row set
    constexpr int PARTS = 15;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    state = uniform(state);
    poly = uniform(poly);
    k = (int)uniform((uint32_t)k);
    max_deg = (int)uniform((uint32_t)max_deg);
    M = uniform(M);
    W* gwin = reinterpret_cast<W*>(state + kHeaderBytes);
    uint64_t* spoly = reinterpret_cast<uint64_t*>(buf + 2 * SET);
    W* cur = buf;
    W* nxt = buf + SET;
    for (int j = tid; j < N; j += nthr) cur[j] = gwin[(size_t)j * M + lane0];
    for (int i = tid; i <= (max_deg >> 6); i += nthr) spoly[i] = poly[i];
    __syncthreads();
    twist_rows<W, N>(cur, cur + N, 1, RW, tid, nthr);
    __syncthreads();
    derive_rows<W, N>(cur, 1, 2 * N, RW, tid, nthr);
    __syncthreads();

    W acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = zero_w<W>();
    const int last_b = (k + max_deg) / N;
    for (int b = 0; b <= last_b; ++b) {
        if (wave > 0) {
            accumulate_block4<W, N, true>(acc, cur, 2 * N, spoly, k, b, max_deg, lane, wave - 1, PARTS);
        } else if (b < last_b) {
            for (int j = lane; j < N; j += 64) nxt[j] = cur[N + j];  // lower half: the current upper block
            twist_rows<W, N>(cur + N, nxt + N, 1, RW, lane, 64);     // upper half: the next block
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): this wavefront's window writes are done
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            derive_rows<W, N>(nxt, 1, 2 * N, RW, lane, 64);
        }
        __syncthreads();
        W* t = cur;
        cur = nxt;
        nxt = t;
    }
    // XOR the slices' sums (wavefronts 1 .. 15) and store the lane's window
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int j = lane + 64 * s;
        if (wave > 0 && j < N) buf[(wave - 1) * N + j] = acc[s];
    }
    __syncthreads();
    for (int j = tid; j < N; j += nthr) {
        W v = buf[j];
#pragma unroll
        for (int q = 1; q < PARTS; ++q) v = xorw(v, buf[q * N + j]);
        gwin[(size_t)j * M + lane0] = v;
    }
}

template <class W, int N, int G, bool GROUPED, int WPL = 1>
__global__ __launch_bounds__(G * WPL * 64) void jump_kernel(const JumpTask* tasks, JumpTask one, uint32_t M) {
    // SFMT: two row sets (jump_pipelined), the serial chain of the next block
    // overlapping the sums of this one. MT regenerates its rows in parallel:
    // one wavefront building them alone is slower than all of them in turn.
    constexpr bool PIPE = GROUPED && G == 1 && WPL == 16 && sizeof(W) == 16;
    constexpr int EXTRA = (WPL > 1 ? jump_pad_words<N>() : 0) + (WPL >= 8 ? jump_poly_stage_words<W>() : 0) +
                          (PIPE ? jump_row_words<N, true>() + jump_pad_words<N>() : 0);
    __shared__ __attribute__((aligned(16))) W buf[jump_row_words<N, GROUPED>() * G + EXTRA];
    const uint32_t groups = M / G;
    const uint32_t ti = blockIdx.x / groups, g = blockIdx.x - ti * groups;
    const JumpTask task = tasks ? tasks[ti] : one;
    const StateHeader* h = reinterpret_cast<const StateHeader*>(task.state);
    const uint32_t per = sizeof(W) == 16 ? 4u : 1u;
    const int k = (int)(h->pos / (per * M));  // words of every lane already consumed
    if constexpr (PIPE) {
        jump_pipelined<W, N>(task.state, M, g, task.poly + (size_t)task.lane_stride * g, (int)task.max_deg, k, buf);
    } else {
        dephase<W, N, G, false, GROUPED, WPL>(task.state, M, g, task.poly, task.lane_stride, (int)task.max_deg, k,
                                              nullptr, buf);
    }
}

#ifndef VMT_PART_RATIO_MT32
#define VMT_PART_RATIO_MT32 0.06f
#endif
#ifndef VMT_PART_RATIO_MT64
#define VMT_PART_RATIO_MT64 0.1f
#endif

// First coefficient of part p of `parts` over the nb coefficients of a lane
// jump. A part whose first coefficient lies in block b first twists its raw
// row b times without summing, so later parts get fewer coefficients: with r
// the cost of a bare twist relative to summing a block, part p's share is q^p
// (q = 1 - r) of the first part's, and each part's twists plus sums come to
// about the same time. Every workgroup of a lane jump evaluates this in the
// same order, so the parts tile the coefficients exactly.
__device__ __forceinline__ int part_start(int p, int parts, int nb, float r) {
    const float q = 1.0f - r;
    float c = 0.0f, total = 0.0f, w = 1.0f;
    for (int i = 0; i < parts; ++i) {
        if (i == p) c = total;
        total += w;
        w *= q;
    }
    if (p >= parts) return nb;
    const int b = (int)(nb * (c / total) + 0.5f);
    return b < nb ? b : nb;
}

// One part of an MT lane jump (jumps of few lanes). The sum over g's
// coefficients is linear, so it splits over coefficient ranges: workgroup
// (task, lane t, part p) sums coefficients [c0, c1) over blocks [b0, b1) of
// lane t's raw sequence, its WPL wavefronts slicing each block's groups as in
// the sliced jump, and writes the partial window (N contiguous words) to
// `partial`. Before its first block it twists the lane's row from the window
// b0 times (two N-word halves of LDS in turn, one barrier per block). A separate launch XORs the
// parts into the state (reduce_jump_parts). All parts read the window and the
// position before any of them is replaced.
template <class P, int WPL>
__global__ __launch_bounds__(WPL * 64) void jump_part_kernel(const JumpTask* tasks, JumpTask one, uint32_t M,
                                                             uint32_t parts, typename P::W* partial, float ratio) {
    using W = typename P::W;
    constexpr int N = P::N;
    constexpr int S = (N + 63) / 64;
    constexpr int RW = jump_row_words<N, true>();
    static_assert(WPL * N <= RW, "the wavefronts' partial sums are staged in the row buffer");
    __shared__ __attribute__((aligned(16))) W buf[RW + jump_pad_words<N>() + jump_poly_stage_words<W>()];
    const uint32_t per_task = M * parts;
    const uint32_t ti = blockIdx.x / per_task, rem = blockIdx.x - ti * per_task;
    const uint32_t t = rem / parts, part = rem - t * parts;
    const JumpTask task = tasks ? tasks[ti] : one;
    uint8_t* state = uniform(task.state);
    const StateHeader* h = reinterpret_cast<const StateHeader*>(state);
    const int k = (int)uniform(h->pos / M);  // words of every lane already consumed
    const int max_deg = (int)uniform(task.max_deg);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // coefficients [c0, c1) of the lane's polynomial, in blocks [b0, b1)
    const int c0 = part_start((int)part, (int)parts, max_deg + 1, ratio);
    const int c1 = part_start((int)part + 1, (int)parts, max_deg + 1, ratio);
    const int b0 = (c0 + k) / N, b1 = c1 > c0 ? (c1 - 1 + k) / N + 1 : b0;

    const W* gwin = reinterpret_cast<const W*>(state + kHeaderBytes);
    for (int j = tid; j < N; j += nthr) buf[j] = gwin[(size_t)j * M + t];
    uint64_t* spoly = reinterpret_cast<uint64_t*>(buf + RW + jump_pad_words<N>());
    const uint64_t* src = uniform(task.poly) + (size_t)task.lane_stride * t;
    for (int i = tid; i <= (max_deg >> 6); i += nthr) spoly[i] = src[i];
    __syncthreads();
    // bare twists up to block b0, alternating between the two halves of the window
    for (int i = 0; i < b0; ++i) {
        const W* a = buf + (i & 1) * N;
        raw_twist_rows<P>(a, buf + N - (i & 1) * N, 1, 0, tid, nthr);
        __syncthreads();
    }
    if (b0 & 1) {  // block b0 sits in the upper half: move it down
        for (int j = tid; j < N; j += nthr) buf[j] = buf[N + j];
        __syncthreads();
    }

    W acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = zero_w<W>();
    if (b0 < b1) {
        raw_twist_rows<P>(buf, buf + N, 1, 0, tid, nthr);
        __syncthreads();
        derive_rows<W, N>(buf, 1, 2 * N, RW, tid, nthr);
        __syncthreads();
        for (int b = b0;; ++b) {
            accumulate_block4<W, N, true>(acc, buf, 2 * N, spoly, k, b, max_deg, lane, wave, WPL, c0, c1);
            if (b + 1 == b1) break;
            __syncthreads();
            for (int j = tid; j < N; j += nthr) buf[j] = buf[N + j];  // upper -> lower
            __syncthreads();
            raw_twist_rows<P>(buf, buf + N, 1, 0, tid, nthr);
            __syncthreads();
            derive_rows<W, N>(buf, 1, 2 * N, RW, tid, nthr);
            __syncthreads();
        }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int j = lane + 64 * s;
        if (j < N) buf[wave * N + j] = acc[s];
    }
    __syncthreads();
    W* dst = partial + ((size_t)(ti * M + t) * parts + part) * N;
    for (int j = tid; j < N; j += nthr) {
        W v = buf[j];
#pragma unroll
        for (int q = 1; q < WPL; ++q) v = xorw(v, buf[q * N + j]);
        dst[j] = v;
    }
}

// XOR of a lane jump's parts into lane t's window of the state, and the
// position fix of finalize_jump_pos (by the workgroup of lane 0). One
// workgroup per (task, lane). Tasks that carry a completion flag do not come
// here: no workgroup of a task knows when the task's other lanes are done.
// PARTS is a compile-time count, so that a thread's loads of all parts are in
// flight together.
template <class W, int N, int PARTS>
__global__ __launch_bounds__(256) void reduce_jump_parts(const JumpTask* tasks, JumpTask one, uint32_t M,
                                                         const W* partial) {
    const uint32_t ti = blockIdx.x / M, t = blockIdx.x - ti * M;
    const JumpTask task = tasks ? tasks[ti] : one;
    W* gwin = reinterpret_cast<W*>(task.state + kHeaderBytes);
    const W* src = partial + (size_t)blockIdx.x * PARTS * N;
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
        W v[PARTS];
#pragma unroll
        for (int q = 0; q < PARTS; ++q) v[q] = src[(size_t)q * N + j];
#pragma unroll
        for (int q = 1; q < PARTS; ++q) v[0] = xorw(v[0], v[q]);
        gwin[(size_t)j * M + t] = v[0];
    }
    if (t == 0 && threadIdx.x == 0) {
        StateHeader* h = reinterpret_cast<StateHeader*>(task.state);
        h->pos = h->pos % M;
    }
}

// Jumps of one state's copies by different distances (the chunks of a split
// call): every copy starts from the same window, so lane t's raw sequence is
// the same for all of them. One workgroup per (lane t, CPW copies): the raw
// rows are regenerated and derived once, and wavefront w sums copy w's
// polynomial over them (grouped form) and writes lane t of that copy. `src`
// holds the common window and is not among the copies jumped.
template <class W, int N, int CPW>
__global__ __launch_bounds__(CPW * 64) void split_jump_kernel(const uint8_t* src, const JumpTask* tasks, uint32_t count,
                                                              uint32_t M) {
    constexpr int S = (N + 63) / 64;
    constexpr int RW = jump_row_words<N, true>();
    __shared__ __attribute__((aligned(16))) W buf[RW + jump_pad_words<N>()];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63;
    const uint32_t w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint32_t t = blockIdx.x % M;  // lane of the state
    const uint32_t first = (blockIdx.x / M) * CPW;
    const uint32_t mine = first + w;
    const bool active = mine < count;
    const StateHeader* h = reinterpret_cast<const StateHeader*>(src);
    const uint32_t per = sizeof(W) == 16 ? 4u : 1u;
    const int k = (int)uniform((uint32_t)(h->pos / (per * M)));  // words of every lane already consumed
    int max_deg = 0;  // the workgroup's blocks run to the highest degree among its copies' polynomials
    for (uint32_t i = first; i < first + CPW && i < count; ++i) max_deg = max(max_deg, (int)tasks[i].max_deg);
    max_deg = (int)uniform((uint32_t)max_deg);
    uint8_t* dst = nullptr;
    const uint64_t* poly = nullptr;
    int my_deg = -1;
    if (active) {
        dst = uniform(tasks[mine].state);
        poly = uniform(tasks[mine].poly);
        my_deg = (int)uniform(tasks[mine].max_deg);
    }
    const W* gsrc = reinterpret_cast<const W*>(src + kHeaderBytes);
    for (int j = tid; j < N; j += nthr) buf[j] = gsrc[(size_t)j * M + t];
    __syncthreads();
    twist_rows<W, N>(buf, buf + N, 1, RW, tid, nthr);
    __syncthreads();
    derive_rows<W, N>(buf, 1, 2 * N, RW, tid, nthr);
    __syncthreads();
    W acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = zero_w<W>();
    const int last_b = (k + max_deg) / N;
    for (int b = 0; b <= last_b; ++b) {
        if (active) accumulate_block4<W, N, true>(acc, buf, 2 * N, poly, k, b, my_deg, lane, 0, 1);
        if (b == last_b) break;
        __syncthreads();
        for (int j = tid; j < N; j += nthr) buf[j] = buf[N + j];  // upper -> lower
        __syncthreads();
        twist_rows<W, N>(buf, buf + N, 1, RW, tid, nthr);
        __syncthreads();
        derive_rows<W, N>(buf, 1, 2 * N, RW, tid, nthr);
        __syncthreads();
    }
    if (active) {
        W* gdst = reinterpret_cast<W*>(dst + kHeaderBytes);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int j = lane + 64 * s;
            if (j < N) gdst[(size_t)j * M + t] = acc[s];
        }
    }
}

// The shared-row split jump with each lane's coefficients split over `parts`
// workgroups (MT): workgroup (copy group, lane t, part p) regenerates lane
// t's raw rows for the blocks of coefficients [c0, c1) once, after bare
// twists up to the first, and wavefront w sums copy w's polynomial over them,
// writing its partial window to `partial` for reduce_jump_parts. The parts of
// a copy group take the same boundaries (all compute them from the group's
// highest degree). Few
// copies per lane then still fill the chip, while the rows are derived once
// per block for all copies of the workgroup.
template <class P, int CPW, bool G5 = false>
__global__ __launch_bounds__(CPW * 64) void split_part_jump_kernel(const uint8_t* src, const JumpTask* tasks,
                                                                   uint32_t count, uint32_t M, uint32_t parts,
                                                                   typename P::W* partial, float ratio) {
    using W = typename P::W;
    constexpr int N = P::N;
    constexpr int S = (N + 63) / 64;
    constexpr int RW = (G5 ? 16 : 8) * 2 * N;  // the raw row and its derived rows
    __shared__ __attribute__((aligned(16))) W buf[RW + jump_pad_words<N>()];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63;
    const uint32_t w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint32_t part = blockIdx.x % parts, rest = blockIdx.x / parts;
    const uint32_t t = rest % M;  // lane of the state
    const uint32_t first = (rest / M) * CPW;
    const uint32_t mine = first + w;
    const bool active = mine < count;
    const StateHeader* h = reinterpret_cast<const StateHeader*>(src);
    const int k = (int)uniform((uint32_t)(h->pos / M));  // words of every lane already consumed
    int max_deg = 0;
    for (uint32_t i = first; i < first + CPW && i < count; ++i) max_deg = max(max_deg, (int)tasks[i].max_deg);
    max_deg = (int)uniform((uint32_t)max_deg);
    const uint64_t* poly = nullptr;
    int my_deg = -1;
    if (active) {
        poly = uniform(tasks[mine].poly);
        my_deg = (int)uniform(tasks[mine].max_deg);
    }
    const int c0 = part_start((int)part, (int)parts, max_deg + 1, ratio);
    const int c1 = part_start((int)part + 1, (int)parts, max_deg + 1, ratio);
    const int b0 = (c0 + k) / N, b1 = c1 > c0 ? (c1 - 1 + k) / N + 1 : b0;

    const W* gsrc = reinterpret_cast<const W*>(src + kHeaderBytes);
    for (int j = tid; j < N; j += nthr) buf[j] = gsrc[(size_t)j * M + t];
    __syncthreads();
    for (int i = 0; i < b0; ++i) {  // bare twists up to block b0, between the two halves of the window
        raw_twist_rows<P>(buf + (i & 1) * N, buf + N - (i & 1) * N, 1, 0, tid, nthr);
        __syncthreads();
    }
    if (b0 & 1) {
        for (int j = tid; j < N; j += nthr) buf[j] = buf[N + j];
        __syncthreads();
    }
    W acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = zero_w<W>();
    if (b0 < b1) {
        raw_twist_rows<P>(buf, buf + N, 1, 0, tid, nthr);
        __syncthreads();
        if constexpr (G5) derive_rows5<W, N>(buf, 2 * N, tid, nthr);
        else derive_rows<W, N>(buf, 1, 2 * N, RW, tid, nthr);
        __syncthreads();
        for (int b = b0;; ++b) {
            if (active) {
                if constexpr (G5) accumulate_block5<W, N>(acc, buf, 2 * N, poly, k, b, my_deg, lane, c0, c1);
                else accumulate_block4<W, N, true>(acc, buf, 2 * N, poly, k, b, my_deg, lane, 0, 1, c0, c1);
            }
            if (b + 1 == b1) break;
            __syncthreads();
            for (int j = tid; j < N; j += nthr) buf[j] = buf[N + j];  // upper -> lower
            __syncthreads();
            raw_twist_rows<P>(buf, buf + N, 1, 0, tid, nthr);
            __syncthreads();
            if constexpr (G5) derive_rows5<W, N>(buf, 2 * N, tid, nthr);
            else derive_rows<W, N>(buf, 1, 2 * N, RW, tid, nthr);
            __syncthreads();
        }
    }
    if (active) {
        W* dst = partial + ((size_t)(mine * M + t) * parts + part) * N;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int j = lane + 64 * s;
            if (j < N) dst[j] = acc[s];
        }
    }
}

// Derived rows of window b from two raw blocks held elsewhere (x[m] is
// lo[m] for m < N, hi[m - N] above): row 0 receives the raw words of the
// window, rows 1 .. 7 the patterns as in derive_rows.
template <class W, int N>
__device__ __forceinline__ void derive_rows_from(W* rows, int rstride, const W* lo, const W* hi, int tid, int nthr) {
    for (int m = tid; m < 2 * N; m += nthr) {
        const W z = zero_w<W>();
        auto x = [&](int i) { return i < N ? lo[i] : (i < 2 * N ? hi[i - N] : z); };
        const W x0 = x(m), x1 = x(m + 1), x2 = x(m + 2), x3 = x(m + 3);
        const W d3 = xorw(x0, x1), d5 = xorw(x0, x2), d7 = xorw(d3, x2);
        rows[m] = x0;
        rows[1 * rstride + m] = d3;
        rows[2 * rstride + m] = d5;
        rows[3 * rstride + m] = d7;
        rows[4 * rstride + m] = xorw(x0, x3);
        rows[5 * rstride + m] = xorw(d3, x3);
        rows[6 * rstride + m] = xorw(d5, x3);
        rows[7 * rstride + m] = xorw(d7, x3);
    }
}

// One raw block of one lane by the chain (the four threads of a quad), as a
// call: its registers are then not allocated alongside the summing code's,
// which keeps the split jump's workgroups small enough for two per CU.
template <int N>
__device__ __attribute__((noinline)) void sfmt_chain_block(const uint32_t* src, uint32_t* dst, int j) {
    sfmt_block_quad<N>(src, dst, 4, j, [](int, uint32_t) {});
}

// split_jump_kernel for SFMT, whose raw rows come from the serial 128-bit
// chain: the workgroup has one more wavefront, which runs the lane's chain
// one block ahead into a ring of three raw blocks in LDS while the CPW other
// wavefronts sum their copies' polynomials over the current window's derived
// rows. Window b is raw blocks b and b + 1; the chain writes block b + 2 into
// the ring slot that held block b - 1, which no one reads any more (window b's
// rows were derived before its sums began). Per block: sums and chain side
// by side, a barrier, the rows of window b + 1 derived by every wavefront, a
// barrier.
template <int N, int CPW>
__global__ __launch_bounds__((CPW + 1) * 64) void split_jump_sfmt_kernel(const uint8_t* src, const JumpTask* tasks,
                                                                         uint32_t count, uint32_t M) {
    using W = uint4;
    constexpr int S = (N + 63) / 64;
    constexpr int RW = jump_row_words<N, true>();
    __shared__ __attribute__((aligned(16))) W rows[RW + jump_pad_words<N>()];
    __shared__ __attribute__((aligned(16))) W ring[3 * N];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63;
    const uint32_t w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool chain_wave = w == CPW;
    const uint32_t t = blockIdx.x % M;  // lane of the state
    const uint32_t first = (blockIdx.x / M) * CPW;
    const uint32_t mine = first + w;
    const bool active = !chain_wave && mine < count;
    const StateHeader* h = reinterpret_cast<const StateHeader*>(src);
    const int k = (int)uniform((uint32_t)(h->pos / (4u * M)));  // words of every lane already consumed
    int max_deg = 0;  // the workgroup's blocks run to the highest degree among its copies' polynomials
    for (uint32_t i = first; i < first + CPW && i < count; ++i) max_deg = max(max_deg, (int)tasks[i].max_deg);
    max_deg = (int)uniform((uint32_t)max_deg);
    uint8_t* dst = nullptr;
    const uint64_t* poly = nullptr;
    int my_deg = -1;
    if (active) {
        dst = uniform(tasks[mine].state);
        poly = uniform(tasks[mine].poly);
        my_deg = (int)uniform(tasks[mine].max_deg);
    }
    // the chain: quad 0 of the chain wavefront, thread j holding sub-word j
    const QuadThread qt = sfmt_quad_thread(lane);
    const bool chainer = chain_wave && qt.q == 0;
    auto chain_block = [&](int from, int to) {  // raw block `to` (a ring slot) from block `from`
        if (chainer)
            sfmt_chain_block<N>(reinterpret_cast<const uint32_t*>(ring + from * N), reinterpret_cast<uint32_t*>(ring + to * N),
                                qt.j);
    };
    const W* gsrc = reinterpret_cast<const W*>(src + kHeaderBytes);
    for (int j = tid; j < N; j += nthr) ring[j] = gsrc[(size_t)j * M + t];
    __syncthreads();
    chain_block(0, 1);
    __syncthreads();
    derive_rows_from<W, N>(rows, 2 * N, ring, ring + N, tid, nthr);
    __syncthreads();
    W acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = zero_w<W>();
    const int last_b = (k + max_deg) / N;
    for (int b = 0; b <= last_b; ++b) {
        if (active) accumulate_block4<W, N, true>(acc, rows, 2 * N, poly, k, b, my_deg, lane, 0, 1);
        if (b < last_b) chain_block((b + 1) % 3, (b + 2) % 3);  // window b + 1 needs block b + 2
        __syncthreads();
        if (b == last_b) break;
        derive_rows_from<W, N>(rows, 2 * N, ring + ((b + 1) % 3) * N, ring + ((b + 2) % 3) * N, tid, nthr);
        __syncthreads();
    }
    if (active) {
        W* gdst = reinterpret_cast<W*>(dst + kHeaderBytes);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int j = lane + 64 * s;
            if (j < N) gdst[(size_t)j * M + t] = acc[s];
        }
    }
}

__global__ void finalize_jump_pos(const JumpTask* tasks, JumpTask one, uint32_t count) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const JumpTask task = tasks ? tasks[i] : one;
    StateHeader* h = reinterpret_cast<StateHeader*>(task.state);
    const uint32_t per = h->word_bytes == 16 ? 4u : 1u;
    h->pos = h->pos % (per * h->M);
    if (task.flag) {
        __threadfence();
        __hip_atomic_fetch_add(task.flag, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

static int lanes_per_group(uint32_t variant, uint32_t M) {
    // one wavefront per lane; at most 16 lanes (1024 threads) per workgroup
    (void)variant;
    return M < 16 ? (int)M : 16;
}

// SFMT variant -> its state size NN (the kernels' template parameter)
#define VMT_SFMT_CASE(V, ...)                                                 \
    case V: {                                                                 \
        constexpr int NN = (int)kSfmtSets[V - kSFMT].n;                       \
        __VA_ARGS__;                                                          \
        break;                                                                \
    }
#define VMT_SFMT_SWITCH(variant, ...)                \
    switch (variant) {                               \
        VMT_SFMT_CASE(kSFMT607, __VA_ARGS__)         \
        VMT_SFMT_CASE(kSFMT1279, __VA_ARGS__)        \
        VMT_SFMT_CASE(kSFMT2281, __VA_ARGS__)        \
        VMT_SFMT_CASE(kSFMT4253, __VA_ARGS__)        \
        VMT_SFMT_CASE(kSFMT11213, __VA_ARGS__)       \
        default: {                                   \
            constexpr int NN = (int)kSfmtSets[0].n;  \
            __VA_ARGS__;                             \
            break;                                   \
        }                                            \
    }

#define VMT_G_SWITCH(G, ...)                                 \
    switch (G) {                                             \
        case 1: { constexpr int GG = 1; __VA_ARGS__; break; } \
        case 2: { constexpr int GG = 2; __VA_ARGS__; break; } \
        case 4: { constexpr int GG = 4; __VA_ARGS__; break; } \
        case 8: { constexpr int GG = 8; __VA_ARGS__; break; } \
        default: { constexpr int GG = 16; __VA_ARGS__; break; } \
    }

#define VMT_WPL_SWITCH(W, ...)                                \
    switch (W) {                                              \
        case 4: { constexpr int WW = 4; __VA_ARGS__; break; }  \
        case 8: { constexpr int WW = 8; __VA_ARGS__; break; }  \
        default: { constexpr int WW = 16; __VA_ARGS__; break; } \
    }
#define VMT_CPW_SWITCH(C, ...)                                \
    switch (C) {                                              \
        case 4: { constexpr int CC = 4; __VA_ARGS__; break; }  \
        case 8: { constexpr int CC = 8; __VA_ARGS__; break; }  \
        default: { constexpr int CC = 16; __VA_ARGS__; break; } \
    }
constexpr uint64_t kSplitSharedLanes = 1024;  // up to this many lane jumps a split call jumps each lane alone
#define VMT_G8_SWITCH(G, ...)                                 \
    switch (G) {                                              \
        case 1: { constexpr int GG = 1; __VA_ARGS__; break; }  \
        case 2: { constexpr int GG = 2; __VA_ARGS__; break; }  \
        case 4: { constexpr int GG = 4; __VA_ARGS__; break; }  \
        default: { constexpr int GG = 8; __VA_ARGS__; break; } \
    }

hipError_t launch_init(uint32_t variant, uint32_t M, const InitTask* d_tasks, const InitTask& one, uint32_t count,
                       const uint64_t* d_lane_polys, uint32_t max_deg, hipStream_t stream) {
    const int G = lanes_per_group(variant, M);
    const dim3 grid(count * (M / G)), block(G * 64);
    if (variant == kMT32) {
        VMT_G_SWITCH(G, init_kernel<uint32_t, 624, GG><<<grid, block, 0, stream>>>(d_tasks, one, M, d_lane_polys, max_deg, variant))
    } else if (variant == kMT64) {
        VMT_G_SWITCH(G, init_kernel<uint64_t, 312, GG><<<grid, block, 0, stream>>>(d_tasks, one, M, d_lane_polys, max_deg, variant))
    } else {
        VMT_SFMT_SWITCH(variant, VMT_G_SWITCH(G, init_kernel<uint4, NN, GG><<<grid, block, 0, stream>>>(d_tasks, one, M, d_lane_polys, max_deg, variant)))
    }
    return hipGetLastError();
}

#ifndef VMT_JUMP_PARTS_MAX
#define VMT_JUMP_PARTS_MAX 8
#endif
#ifndef VMT_JUMP_PARTS_WGS
#define VMT_JUMP_PARTS_WGS 512
#endif

#define VMT_PARTS_SWITCH(PS, ...)                                 \
    switch (PS) {                                                 \
        case 2: { constexpr int PP = 2; __VA_ARGS__; break; }     \
        case 4: { constexpr int PP = 4; __VA_ARGS__; break; }     \
        case 8: { constexpr int PP = 8; __VA_ARGS__; break; }     \
        case 16: { constexpr int PP = 16; __VA_ARGS__; break; }   \
        default: { constexpr int PP = 32; __VA_ARGS__; break; }   \
    }

// XOR the parts of `count` tasks' lane jumps into their states (parts: 2, 4, 8, 16 or 32)
static void launch_reduce_parts(uint32_t variant, uint32_t M, const JumpTask* d_tasks, const JumpTask& one,
                                uint32_t count, uint32_t parts, const void* d_parts, hipStream_t stream) {
    const dim3 grid(count * M), block(256);
    if (variant == kMT32) {
        VMT_PARTS_SWITCH(parts, (reduce_jump_parts<uint32_t, 624, PP><<<grid, block, 0, stream>>>(
                                    d_tasks, one, M, static_cast<const uint32_t*>(d_parts))))
    } else {
        VMT_PARTS_SWITCH(parts, (reduce_jump_parts<uint64_t, 312, PP><<<grid, block, 0, stream>>>(
                                    d_tasks, one, M, static_cast<const uint64_t*>(d_parts))))
    }
}

uint32_t jump_parts(uint32_t variant, uint32_t M, uint64_t count) {
    // MT jumps of up to 256 lanes (one 1,024-thread workgroup each) leave most
    // compute units idle or one lane jump per unit: split each lane's blocks
    // over up to 8 workgroups, so that about 512 of them (two per compute unit)
    // run. SFMT regenerates its rows by a serial chain, which a later part
    // would have to rerun from the start.
    if (variant != kMT32 && variant != kMT64) return 1;
    const uint64_t lanes = count * M;
    if (lanes == 0 || lanes > 256) return 1;
    uint32_t parts = 1;
    while (parts < VMT_JUMP_PARTS_MAX && lanes * parts * 2 <= VMT_JUMP_PARTS_WGS) parts *= 2;
    return parts;
}

size_t jump_parts_bytes(uint32_t variant, uint32_t M, uint64_t count) {
    const uint32_t parts = jump_parts(variant, M, count);
    if (parts == 1) return 0;
    const size_t win = variant == kMT32 ? 624 * 4 : 312 * 8;  // one lane's window
    return (size_t)count * M * parts * win;
}

#ifndef VMT_SPLIT_SHARE_PARTS
#define VMT_SPLIT_SHARE_PARTS 1
#endif
// A shared-row block carries the sums of up to 16 copies, so a bare twist
// costs far less of it than of a sliced block: near-equal parts.
#ifndef VMT_SHARE_RATIO
#define VMT_SHARE_RATIO 0.005f
#endif
#ifndef VMT_SHARE_PARTS_MAX
#define VMT_SHARE_PARTS_MAX 16
#endif
#ifndef VMT_SHARE_WGS
#define VMT_SHARE_WGS 512
#endif
static_assert(VMT_JUMP_PARTS_MAX <= 32 && VMT_SHARE_PARTS_MAX <= 32, "launch_reduce_parts instantiates up to 32 parts");
#ifndef VMT_SHARE_G5
#define VMT_SHARE_G5 1
#endif

uint32_t split_share_parts(uint32_t variant, uint32_t M, uint64_t count) {
    // MT split jumps whose copies, 16 per workgroup, give each lane fewer than
    // 512 workgroups: split every lane's blocks over up to 16 of them, when
    // that reaches at least 256 workgroups (one per compute unit). Fewer
    // lanes and copies run faster sliced (jump_part_kernel).
    if (!VMT_SPLIT_SHARE_PARTS || (variant != kMT32 && variant != kMT64)) return 1;
    const uint64_t wgs = (uint64_t)M * ((count + 15) / 16);
    uint32_t parts = 1;
    while (parts < VMT_SHARE_PARTS_MAX && wgs * parts * 2 <= VMT_SHARE_WGS) parts *= 2;
    return wgs * parts >= 256 ? parts : 1;
}

size_t split_jump_parts_bytes(uint32_t variant, uint32_t M, uint64_t count) {
    const size_t win = variant == kMT32 ? 624 * 4 : 312 * 8;
    const uint32_t sp = split_share_parts(variant, M, count);
    if (sp > 1) return (size_t)count * M * sp * win;
    if ((uint64_t)count * M <= 1024) return jump_parts_bytes(variant, M, count);
    return 0;
}

hipError_t launch_jump(uint32_t variant, uint32_t M, const JumpTask* d_tasks, const JumpTask& one, uint32_t count,
                       hipStream_t stream, void* d_parts) {
    const uint32_t parts = d_parts ? jump_parts(variant, M, count) : 1;
    if (parts > 1) {
        const dim3 grid(count * M * parts), block(16 * 64);
        if (variant == kMT32)
            jump_part_kernel<MT32P, 16><<<grid, block, 0, stream>>>(d_tasks, one, M, parts,
                                                                   static_cast<uint32_t*>(d_parts), VMT_PART_RATIO_MT32);
        else
            jump_part_kernel<MT64P, 16><<<grid, block, 0, stream>>>(d_tasks, one, M, parts,
                                                                   static_cast<uint64_t*>(d_parts), VMT_PART_RATIO_MT64);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        launch_reduce_parts(variant, M, d_tasks, one, count, parts, d_parts, stream);
        return hipGetLastError();
    }
    // Up to 1024 lanes: grouped accumulation, one lane per workgroup (40 KB of
    // LDS) and WPL wavefronts per lane, each summing a slice of the
    // coefficients: 16 for up to 256 lanes (one workgroup of 1024 threads per
    // lane), 8 up to 512, 4 up to 1024 (four lanes' workgroups per compute
    // unit). More lanes: one coefficient at a time, eight lanes (four for
    // SFMT) per workgroup in 40 KB, so that many more lanes share each
    // compute unit.
    const uint64_t lanes = (uint64_t)count * M;
    const bool grouped = lanes <= 1024;
    if (grouped) {
        const int wpl = lanes <= 256 ? 16 : (lanes <= 512 ? 8 : 4);
        const dim3 grid(count * M), block(wpl * 64);
        if (variant == kMT32) {
            VMT_WPL_SWITCH(wpl, jump_kernel<uint32_t, 624, 1, true, WW><<<grid, block, 0, stream>>>(d_tasks, one, M))
        } else if (variant == kMT64) {
            VMT_WPL_SWITCH(wpl, jump_kernel<uint64_t, 312, 1, true, WW><<<grid, block, 0, stream>>>(d_tasks, one, M))
        } else {
            VMT_SFMT_SWITCH(variant, VMT_WPL_SWITCH(wpl, jump_kernel<uint4, NN, 1, true, WW><<<grid, block, 0, stream>>>(d_tasks, one, M)))
        }
    } else {
        int G = lanes_per_group(variant, M);
        const int cap = is_sfmt(variant) ? 4 : 8;
        if (G > cap) G = cap;
        const dim3 grid(count * (M / G)), block(G * 64);
        if (variant == kMT32) {
            VMT_G8_SWITCH(G, jump_kernel<uint32_t, 624, GG, false><<<grid, block, 0, stream>>>(d_tasks, one, M))
        } else if (variant == kMT64) {
            VMT_G8_SWITCH(G, jump_kernel<uint64_t, 312, GG, false><<<grid, block, 0, stream>>>(d_tasks, one, M))
        } else {
            VMT_SFMT_SWITCH(variant, VMT_G8_SWITCH(G, jump_kernel<uint4, NN, GG, false><<<grid, block, 0, stream>>>(d_tasks, one, M)))
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    finalize_jump_pos<<<(count + 255) / 256, 256, 0, stream>>>(d_tasks, one, count);
    return hipGetLastError();
}


hipError_t launch_split_jump(uint32_t variant, uint32_t M, const uint8_t* d_src, const JumpTask* d_tasks,
                             const JumpTask& one, uint32_t count, hipStream_t stream, void* d_parts) {
    // Few lanes: each lane jump on its own, sliced over wavefronts. More: the
    // copies share each lane's raw rows, CPW copies per workgroup (fewer when
    // that leaves under 512 workgroups). States of fewer than 16 words (SFMT607,
    // SFMT1279) keep a row per lane jump: their blocks are so short that the
    // barriers of a wide workgroup cost more than regenerating the rows.
    const uint64_t lanes = (uint64_t)count * M;
    const uint32_t sp = d_parts ? split_share_parts(variant, M, count) : 1;
    if (sp > 1) {
        const dim3 grid((uint32_t)(M * ((count + 15) / 16) * sp)), block(16 * 64);
        if (variant == kMT32 && VMT_SHARE_G5 && grid.x <= 256)  // 80 KB of rows: one workgroup per CU
            split_part_jump_kernel<MT32P, 16, true><<<grid, block, 0, stream>>>(
                d_src, d_tasks, count, M, sp, static_cast<uint32_t*>(d_parts), VMT_SHARE_RATIO);
        else if (variant == kMT32)
            split_part_jump_kernel<MT32P, 16><<<grid, block, 0, stream>>>(
                d_src, d_tasks, count, M, sp, static_cast<uint32_t*>(d_parts), VMT_SHARE_RATIO);
        else
            split_part_jump_kernel<MT64P, 16><<<grid, block, 0, stream>>>(
                d_src, d_tasks, count, M, sp, static_cast<uint64_t*>(d_parts), VMT_SHARE_RATIO);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        launch_reduce_parts(variant, M, d_tasks, one, count, sp, d_parts, stream);
        return hipGetLastError();
    }
    if (lanes <= kSplitSharedLanes || words_per_lane(variant) < 16)
        return launch_jump(variant, M, d_tasks, one, count, stream, d_parts);
    int cpw = 16;
    while (cpw > 4 && (uint64_t)M * ((count + cpw - 1) / cpw) < 512) cpw /= 2;
    const dim3 grid(M * ((count + cpw - 1) / cpw)), block(cpw * 64);
    if (variant == kMT32) {
        VMT_CPW_SWITCH(cpw, split_jump_kernel<uint32_t, 624, CC><<<grid, block, 0, stream>>>(d_src, d_tasks, count, M))
    } else if (variant == kMT64) {
        VMT_CPW_SWITCH(cpw, split_jump_kernel<uint64_t, 312, CC><<<grid, block, 0, stream>>>(d_src, d_tasks, count, M))
    } else {
        // at most 8 copies per workgroup here: one more wavefront runs the chain, within 1,024 threads
        const int scpw = cpw > 8 ? 8 : cpw;
        const dim3 sgrid(M * ((count + scpw - 1) / scpw)), sblock((scpw + 1) * 64);
        if (scpw == 4)
            VMT_SFMT_SWITCH(variant, (split_jump_sfmt_kernel<NN, 4><<<sgrid, sblock, 0, stream>>>(d_src, d_tasks, count, M)))
        else
            VMT_SFMT_SWITCH(variant, (split_jump_sfmt_kernel<NN, 8><<<sgrid, sblock, 0, stream>>>(d_src, d_tasks, count, M)))
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    finalize_jump_pos<<<(count + 255) / 256, 256, 0, stream>>>(d_tasks, one, count);
    return hipGetLastError();
}

bool generate_supported(uint32_t variant, uint32_t M, uint32_t lpw, int out_kind) {
    if (lpw == 0 || lpw > 16 || (lpw & (lpw - 1)) || M % lpw) return false;
    if (variant == kMT32) return out_kind == kOutU32 || out_kind == kOutF32;
    if (variant == kMT64) return out_kind == kOutU64 || out_kind == kOutF64 || out_kind == kOutF32;
    return out_kind == kOutU32 || out_kind == kOutF32;
}

#define VMT_LPW_SWITCH(L, ...)                                \
    switch (L) {                                              \
        case 1: { constexpr int LL = 1; __VA_ARGS__; break; }  \
        case 2: { constexpr int LL = 2; __VA_ARGS__; break; }  \
        case 4: { constexpr int LL = 4; __VA_ARGS__; break; }  \
        case 8: { constexpr int LL = 8; __VA_ARGS__; break; }  \
        default: { constexpr int LL = 16; __VA_ARGS__; break; } \
    }

hipError_t launch_generate(uint32_t variant, uint32_t M, uint32_t lpw, int out_kind, uint8_t* d_state, void* d_out,
                           uint64_t len, hipStream_t stream) {
    const uint32_t groups = M / lpw;
    const dim3 grid(is_sfmt(variant) ? groups : group_grid(1, groups));
    const uint32_t xoff = state_xcd(d_state);
    const int wp = (lpw == M) ? 1 : 0;
    if (variant == kMT32) {
        if (out_kind == kOutU32) {
            VMT_LPW_SWITCH(lpw, gen_mt_kernel<MT32P, LL, 0><<<grid, mt_threads<MT32P, LL>(), 0, stream>>>(d_state, d_out, len, wp, groups, xoff))
        } else {
            VMT_LPW_SWITCH(lpw, gen_mt_kernel<MT32P, LL, 1><<<grid, mt_threads<MT32P, LL>(), 0, stream>>>(d_state, d_out, len, wp, groups, xoff))
        }
    } else if (variant == kMT64) {
        if (out_kind == kOutU64) {
            VMT_LPW_SWITCH(lpw, gen_mt_kernel<MT64P, LL, 0><<<grid, mt_threads<MT64P, LL>(), 0, stream>>>(d_state, d_out, len, wp, groups, xoff))
        } else if (out_kind == kOutF64) {
            VMT_LPW_SWITCH(lpw, gen_mt_kernel<MT64P, LL, 2><<<grid, mt_threads<MT64P, LL>(), 0, stream>>>(d_state, d_out, len, wp, groups, xoff))
        } else {
            VMT_LPW_SWITCH(lpw, gen_mt_kernel<MT64P, LL, 1><<<grid, mt_threads<MT64P, LL>(), 0, stream>>>(d_state, d_out, len, wp, groups, xoff))
        }
    } else {
        const dim3 sgrid((groups + kSfmtWavesPerWg - 1) / kSfmtWavesPerWg), block(64 * kSfmtWavesPerWg);
        if (out_kind == kOutU32) {
            VMT_SFMT_SWITCH(variant, VMT_LPW_SWITCH(lpw, gen_sfmt_kernel<NN, LL, 0><<<sgrid, block, 0, stream>>>(d_state, d_out, len, wp, groups)))
        } else {
            VMT_SFMT_SWITCH(variant, VMT_LPW_SWITCH(lpw, gen_sfmt_kernel<NN, LL, 1><<<sgrid, block, 0, stream>>>(d_state, d_out, len, wp, groups)))
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || wp) return e;
    finalize_gen_pos<<<1, 1, 0, stream>>>(d_state, len);
    return hipGetLastError();
}

bool batch_supported(uint32_t variant, uint32_t M, int out_kind) {
    if (is_sfmt(variant)) return false;
    return generate_supported(variant, M, M, out_kind);
}

// Shape variants are compiled for 8 and 16 lanes (whole generators of the
// common widths); other widths have the default shape only.
bool batch_shape_supported(uint32_t variant, uint32_t M, int out_kind, uint32_t tv, uint32_t sw) {
    if (!batch_supported(variant, M, out_kind) || tv > 2 || (sw != 16 && sw != 8)) return false;
    return (tv == 0 && sw == 16) || M == 8 || M == 16;
}

template <class P, int OUTK, int LL>
static const void* batch_shape_kernel(uint32_t tv, uint32_t sw, int* threads) {
    if (tv == 0 && sw == 16) {
        *threads = mt_threads<P, LL, 0>();
        return reinterpret_cast<const void*>(batch_mt_kernel<P, LL, OUTK, 0, 16>);
    }
    if constexpr (LL >= 8) {
        if (tv == 0) {
            *threads = mt_threads<P, LL, 0>();
            return reinterpret_cast<const void*>(batch_mt_kernel<P, LL, OUTK, 0, 8>);
        }
        if (tv == 1) {
            *threads = mt_threads<P, LL, 1>();
            return sw == 16 ? reinterpret_cast<const void*>(batch_mt_kernel<P, LL, OUTK, 1, 16>)
                            : reinterpret_cast<const void*>(batch_mt_kernel<P, LL, OUTK, 1, 8>);
        }
        *threads = mt_threads<P, LL, 2>();
        return sw == 16 ? reinterpret_cast<const void*>(batch_mt_kernel<P, LL, OUTK, 2, 16>)
                        : reinterpret_cast<const void*>(batch_mt_kernel<P, LL, OUTK, 2, 8>);
    }
    return nullptr;
}

#define VMT_BATCH_KERNEL(P, OUTK) VMT_LPW_SWITCH(M, kern = batch_shape_kernel<P, OUTK, LL>(tv, sw, &threads))

static const void* batch_kernel_ptr(uint32_t variant, uint32_t M, int out_kind, uint32_t tv, uint32_t sw,
                                    int* threads_out) {
    const void* kern = nullptr;
    int threads = 0;
    if (!batch_shape_supported(variant, M, out_kind, tv, sw)) return nullptr;
    if (variant == kMT32) {
        if (out_kind == kOutU32) { VMT_BATCH_KERNEL(MT32P, 0) }
        else { VMT_BATCH_KERNEL(MT32P, 1) }
    } else {
        if (out_kind == kOutU64) { VMT_BATCH_KERNEL(MT64P, 0) }
        else if (out_kind == kOutF64) { VMT_BATCH_KERNEL(MT64P, 2) }
        else { VMT_BATCH_KERNEL(MT64P, 1) }
    }
    *threads_out = threads;
    return kern;
}

uint32_t batch_threads(uint32_t variant, uint32_t M, int out_kind, uint32_t tv, uint32_t sw) {
    int threads = 0;
    return batch_kernel_ptr(variant, M, out_kind, tv, sw, &threads) ? (uint32_t)threads : 0;
}

uint32_t batch_max_per_cu(uint32_t variant, uint32_t M, int out_kind, uint32_t tv, uint32_t sw) {
    int threads = 0, per_cu = 0;
    const void* kern = batch_kernel_ptr(variant, M, out_kind, tv, sw, &threads);
    if (!kern || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0) != hipSuccess || per_cu < 1)
        return 1;
    return (uint32_t)per_cu;
}

uint32_t device_cus(int device) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 256;
    return (uint32_t)cus;
}

hipError_t launch_batch_sfmt(uint32_t variant, uint32_t M, uint32_t lpw, int out_kind, const BatchTask* d_tasks,
                             uint32_t count, hipStream_t stream) {
    if (count == 0) return hipSuccess;
    const uint32_t groups = M / lpw;
    const uint64_t items = (uint64_t)count * groups;
    const dim3 grid((uint32_t)((items + kSfmtWavesPerWg - 1) / kSfmtWavesPerWg)), block(64 * kSfmtWavesPerWg);
    if (out_kind == kOutU32) {
        VMT_SFMT_SWITCH(variant, VMT_LPW_SWITCH(lpw, batch_sfmt_kernel<NN, LL, 0><<<grid, block, 0, stream>>>(d_tasks, count, groups)))
    } else {
        VMT_SFMT_SWITCH(variant, VMT_LPW_SWITCH(lpw, batch_sfmt_kernel<NN, LL, 1><<<grid, block, 0, stream>>>(d_tasks, count, groups)))
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || lpw == M) return e;
    finalize_batch_pos<<<(count + 255) / 256, 256, 0, stream>>>(d_tasks, count);
    return hipGetLastError();
}

hipError_t launch_batch_gen_mt(uint32_t variant, uint32_t M, uint32_t lpw, int out_kind, const BatchTask* d_tasks,
                               uint32_t count, hipStream_t stream, uint32_t* d_done) {
    if (count == 0) return hipSuccess;
    const uint32_t groups = M / lpw;
    const dim3 grid(group_grid(count, groups));
    if (variant == kMT32) {
        if (out_kind == kOutU32) {
            VMT_LPW_SWITCH(lpw, batch_gen_mt_kernel<MT32P, LL, 0><<<grid, mt_threads<MT32P, LL>(), 0, stream>>>(d_tasks, count, groups, d_done))
        } else {
            VMT_LPW_SWITCH(lpw, batch_gen_mt_kernel<MT32P, LL, 1><<<grid, mt_threads<MT32P, LL>(), 0, stream>>>(d_tasks, count, groups, d_done))
        }
    } else {
        if (out_kind == kOutU64) {
            VMT_LPW_SWITCH(lpw, batch_gen_mt_kernel<MT64P, LL, 0><<<grid, mt_threads<MT64P, LL>(), 0, stream>>>(d_tasks, count, groups, d_done))
        } else if (out_kind == kOutF64) {
            VMT_LPW_SWITCH(lpw, batch_gen_mt_kernel<MT64P, LL, 2><<<grid, mt_threads<MT64P, LL>(), 0, stream>>>(d_tasks, count, groups, d_done))
        } else {
            VMT_LPW_SWITCH(lpw, batch_gen_mt_kernel<MT64P, LL, 1><<<grid, mt_threads<MT64P, LL>(), 0, stream>>>(d_tasks, count, groups, d_done))
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || lpw == M || d_done) return e;
    finalize_batch_pos<<<(count + 255) / 256, 256, 0, stream>>>(d_tasks, count);
    return hipGetLastError();
}

hipError_t launch_split_setup(const uint8_t* d_state, uint8_t* d_copies, uint32_t bytes, uint64_t stride, uint32_t C,
                              uint8_t* d_out, uint64_t E, uint64_t n, uint32_t eb, const uint64_t* d_polys,
                              const uint32_t* d_deg, BatchTask* d_bt, JumpTask* d_jt, uint32_t* d_done,
                              hipStream_t stream) {
    if (C == 0) return hipSuccess;
    const uint32_t per = (bytes / 16 + 255) / 256;
    split_setup<<<dim3(per < 64 ? per : 64, C), 256, 0, stream>>>(d_state, d_copies, bytes, stride, C, d_out, E, n, eb,
                                                                  d_polys, d_deg, d_bt, d_jt, d_done);
    return hipGetLastError();
}

hipError_t launch_copy_states(const CopyTask* d_tasks, uint32_t count, uint32_t bytes, hipStream_t stream) {
    if (count == 0) return hipSuccess;
    const uint32_t per = (bytes / 16 + 255) / 256;
    copy_states<<<dim3(per < 64 ? per : 64, count), 256, 0, stream>>>(d_tasks, bytes);
    return hipGetLastError();
}

hipError_t reset_counters(uint32_t* d_counter, hipStream_t stream) {
    reset_counter<<<1, 2, 0, stream>>>(d_counter);
    return hipGetLastError();
}

hipError_t launch_batch(uint32_t variant, uint32_t M, int out_kind, const BatchShape& shape, const BatchTask* d_tasks,
                        uint32_t count, uint32_t* d_counter, hipStream_t stream) {
    uint32_t grid = shape.grid > count ? count : shape.grid;
    if (grid == 0) return hipSuccess;
    int threads = 0;
    const void* kern = batch_kernel_ptr(variant, M, out_kind, shape.tv, shape.sw, &threads);
    if (!kern) return hipErrorInvalidValue;
    void* args[] = {(void*)&d_tasks, (void*)&count, (void*)&d_counter};
    return hipLaunchKernel(kern, dim3(grid), dim3(threads), args, 0, stream);
}

template <class P, int LL>
static const void* pattern_shape_kernel(uint32_t tv, uint32_t sw) {
    if (tv == 0) return sw == 16 ? reinterpret_cast<const void*>(write_pattern_kernel<P, LL, 0, 16>)
                                 : reinterpret_cast<const void*>(write_pattern_kernel<P, LL, 0, 8>);
    if (tv == 1) return sw == 16 ? reinterpret_cast<const void*>(write_pattern_kernel<P, LL, 1, 16>)
                                 : reinterpret_cast<const void*>(write_pattern_kernel<P, LL, 1, 8>);
    return sw == 16 ? reinterpret_cast<const void*>(write_pattern_kernel<P, LL, 2, 16>)
                    : reinterpret_cast<const void*>(write_pattern_kernel<P, LL, 2, 8>);
}

bool pattern_supported(uint32_t variant, uint32_t M, int out_kind) {
    return (variant == kMT32 && M == 16 && out_kind == kOutU32) || (variant == kMT64 && M == 8 && out_kind == kOutU64);
}

hipError_t launch_write_pattern(uint32_t variant, uint32_t M, int out_kind, const BatchShape& shape,
                                const BatchTask* d_tasks, uint32_t count, uint32_t* d_counter, hipStream_t stream) {
    if (!pattern_supported(variant, M, out_kind) || !batch_shape_supported(variant, M, out_kind, shape.tv, shape.sw))
        return hipErrorInvalidValue;
    uint32_t grid = shape.grid > count ? count : shape.grid;
    if (grid == 0) return hipSuccess;
    int threads = 0;
    (void)batch_kernel_ptr(variant, M, out_kind, shape.tv, shape.sw, &threads);  // same threads as the batch kernel
    const void* kern = variant == kMT32 ? pattern_shape_kernel<MT32P, 16>(shape.tv, shape.sw)
                                        : pattern_shape_kernel<MT64P, 8>(shape.tv, shape.sw);
    void* args[] = {(void*)&d_tasks, (void*)&count, (void*)&d_counter};
    return hipLaunchKernel(kern, dim3(grid), dim3(threads), args, 0, stream);
}

hipError_t launch_fill(void* d_buf, uint64_t bytes, int mode, uint32_t cus, hipStream_t stream) {
    const uint64_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    uint4* p = static_cast<uint4*>(d_buf);
    const bool nt = (mode & 2) != 0;
    if ((mode & 1) == 0) {  // 4 KiB pieces, one per workgroup
        const uint64_t grid = (n16 + 255) / 256;
        if (grid > 0x7fffffffull) return hipErrorInvalidValue;
        if (nt) fill_pieces<true><<<(uint32_t)grid, 256, 0, stream>>>(p, n16, 0x5a5a5a5au);
        else fill_pieces<false><<<(uint32_t)grid, 256, 0, stream>>>(p, n16, 0x5a5a5a5au);
    } else {  // two regions per compute unit, like two resident generators per CU
        const uint32_t grid = 2 * cus;
        const uint64_t per16 = n16 / grid;
        if (nt) fill_regions<true><<<grid, 256, 0, stream>>>(p, n16, per16, 0x5a5a5a5au);
        else fill_regions<false><<<grid, 256, 0, stream>>>(p, n16, per16, 0x5a5a5a5au);
    }
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Scratch of the allocation-free batch call: the task list (up to
// kNoAllocMaxTasks entries) and the queue's two counters, in one file-scope
// device array. In host code `scratch` names a host-side stand-in, so its
// device address is looked up once per device (hipGetSymbolAddress, with
// that device current) and only that address is ever handed to kernels or
// copies. Every call on a device shares that device's array.
// ---------------------------------------------------------------------------

constexpr size_t kNoAllocTaskBytes = (size_t)kNoAllocMaxTasks * sizeof(BatchTask);
static_assert(kNoAllocTaskBytes % 256 == 0, "the counters start on a 256-byte boundary");
static __device__ __align__(256) uint8_t scratch[kNoAllocTaskBytes + 256];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes the device current first
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch[device] = static_cast<uint8_t*>(ptr);
    return hipSuccess;
}

hipError_t noalloc_scratch(int device, BatchTask** d_tasks, uint32_t** d_counter) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    uint8_t* base;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = g_scratch[device];
    }
    if (!base) return hipErrorNotInitialized;
    *d_tasks = reinterpret_cast<BatchTask*>(base);
    *d_counter = reinterpret_cast<uint32_t*>(base + kNoAllocTaskBytes);
    return hipSuccess;
}

}  // namespace vmt
