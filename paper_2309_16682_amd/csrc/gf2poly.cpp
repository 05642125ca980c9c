// gf2poly.cpp -- host GF(2)[t] arithmetic for the jump-ahead (Sec. 3.1).
#include "gf2poly.hpp"

#include <immintrin.h>

#include "vmt_common.hpp"

#include <algorithm>
#include <cstring>
#include <stdexcept>

namespace vmt {

int poly_degree(const Words& a) {
    for (size_t i = a.size(); i-- > 0;)
        if (a[i]) return int(i * 64 + 63 - __builtin_clzll(a[i]));
    return -1;
}

void poly_trim(Words& a) {
    while (!a.empty() && a.back() == 0) a.pop_back();
}

// ---- carry-less multiplication -------------------------------------------

// r[0..2n) = a[0..n) * b[0..n), schoolbook on 64x64 -> 128 carry-less products.
static void mul_base(const uint64_t* a, const uint64_t* b, size_t n, uint64_t* r) {
    std::memset(r, 0, 2 * n * sizeof(uint64_t));
    for (size_t i = 0; i < n; i++) {
        if (!a[i]) continue;
        const __m128i ai = _mm_cvtsi64_si128((long long)a[i]);
        __m128i carry = _mm_setzero_si128();
        for (size_t j = 0; j < n; j++) {
            __m128i p = _mm_clmulepi64_si128(ai, _mm_cvtsi64_si128((long long)b[j]), 0x00);
            p = _mm_xor_si128(p, carry);
            r[i + j] ^= (uint64_t)_mm_cvtsi128_si64(p);
            carry = _mm_srli_si128(p, 8);
        }
        r[i + n] ^= (uint64_t)_mm_cvtsi128_si64(carry);
    }
}

// Karatsuba over word halves; tmp needs 8n + 64 words.
static void mul_kara(const uint64_t* a, const uint64_t* b, size_t n, uint64_t* r, uint64_t* tmp) {
    if (n <= 20) {
        mul_base(a, b, n, r);
        return;
    }
    const size_t h = n / 2, hh = n - h;  // low h words, high hh >= h words
    mul_kara(a, b, h, r, tmp);                   // a0 b0 -> r[0, 2h)
    mul_kara(a + h, b + h, hh, r + 2 * h, tmp);  // a1 b1 -> r[2h, 2n)
    uint64_t* sa = tmp;
    uint64_t* sb = tmp + hh;
    uint64_t* mid = tmp + 2 * hh;
    uint64_t* rest = tmp + 4 * hh;
    for (size_t i = 0; i < hh; i++) {
        sa[i] = (i < h ? a[i] : 0) ^ a[h + i];
        sb[i] = (i < h ? b[i] : 0) ^ b[h + i];
    }
    mul_kara(sa, sb, hh, mid, rest);  // (a0+a1)(b0+b1)
    for (size_t i = 0; i < 2 * h; i++) mid[i] ^= r[i];
    for (size_t i = 0; i < 2 * hh; i++) mid[i] ^= r[2 * h + i];
    for (size_t i = 0; i < 2 * hh; i++) r[h + i] ^= mid[i];
}

Words poly_mul(const Words& a, const Words& b) {
    const size_t n = std::max(a.size(), b.size());
    if (n == 0) return {};
    Words pa(a), pb(b);
    pa.resize(n, 0);
    pb.resize(n, 0);
    Words r(2 * n, 0), tmp(8 * n + 64, 0);
    mul_kara(pa.data(), pb.data(), n, r.data(), tmp.data());
    return r;
}

// ---- shifts -----------------------------------------------------------------

static Words shr_bits(const Words& a, int s) {  // floor(a / t^s)
    const size_t wo = size_t(s) / 64;
    const int bo = s % 64;
    if (wo >= a.size()) return {};
    Words r(a.size() - wo, 0);
    for (size_t i = 0; i < r.size(); i++) {
        uint64_t lo = a[i + wo] >> bo;
        uint64_t hi = (bo && i + wo + 1 < a.size()) ? a[i + wo + 1] << (64 - bo) : 0;
        r[i] = lo | hi;
    }
    return r;
}

// ---- arithmetic modulo mu ---------------------------------------------------

PolyMod::PolyMod(const Words& mu) : mu_(mu) {
    poly_trim(mu_);
    D_ = poly_degree(mu_);
    if (D_ < 64) throw std::invalid_argument("modulus degree too small");
    nw_ = size_t(D_ + 63) / 64;
    // barrett_ = floor(t^(2D) / mu) by long division, highest quotient bit first.
    Words rem((size_t(2 * D_) / 64) + 2, 0);
    rem[size_t(2 * D_) / 64] |= 1ull << (2 * D_ % 64);
    Words q(size_t(D_) / 64 + 2, 0);
    for (int i = 2 * D_; i >= D_; i--) {
        if (!((rem[size_t(i) / 64] >> (i % 64)) & 1u)) continue;
        const int s = i - D_;
        q[size_t(s) / 64] |= 1ull << (s % 64);
        const size_t wo = size_t(s) / 64;
        const int bo = s % 64;
        for (size_t j = 0; j < mu_.size(); j++) {
            rem[j + wo] ^= mu_[j] << bo;
            if (bo && j + wo + 1 < rem.size()) rem[j + wo + 1] ^= mu_[j] >> (64 - bo);
        }
    }
    poly_trim(q);
    barrett_ = q;
}

Words PolyMod::reduce(const Words& a_in) const {
    Words a(a_in);
    poly_trim(a);
    if (poly_degree(a) < D_) {
        a.resize(nw_, 0);
        return a;
    }
    // quotient = floor(floor(a / t^D) * floor(t^2D / mu) / t^D), exact for deg a < 2D
    Words hi = shr_bits(a, D_);
    Words q = shr_bits(poly_mul(hi, barrett_), D_);
    poly_trim(q);
    Words qm = poly_mul(q, mu_);
    Words r(nw_, 0);
    for (size_t i = 0; i < nw_; i++) r[i] = (i < a.size() ? a[i] : 0) ^ (i < qm.size() ? qm[i] : 0);
    if (D_ % 64) r[nw_ - 1] &= (1ull << (D_ % 64)) - 1;
    return r;
}

Words PolyMod::sqr(const Words& a) const {
    // squaring over GF(2) spreads the bits: (sum a_i t^i)^2 = sum a_i t^(2i)
    Words s(2 * a.size(), 0);
    for (size_t i = 0; i < a.size(); i++) {
        __m128i v = _mm_cvtsi64_si128((long long)a[i]);
        __m128i p = _mm_clmulepi64_si128(v, v, 0x00);
        s[2 * i] = (uint64_t)_mm_cvtsi128_si64(p);
        s[2 * i + 1] = (uint64_t)_mm_extract_epi64(p, 1);
    }
    return reduce(s);
}

Words PolyMod::mul(const Words& a, const Words& b) const { return reduce(poly_mul(a, b)); }

Words PolyMod::mul_t(const Words& a_in) const {
    Words a(a_in);
    a.resize(nw_ + 1, 0);
    for (size_t i = a.size(); i-- > 1;) a[i] = (a[i] << 1) | (a[i - 1] >> 63);
    a[0] <<= 1;
    if ((a[size_t(D_) / 64] >> (D_ % 64)) & 1u)
        for (size_t j = 0; j < mu_.size(); j++) a[j] ^= mu_[j];
    a.resize(nw_);
    return a;
}

Words PolyMod::t_pow2(uint64_t k, const Words* start) const {
    Words cur;
    if (start) {
        cur = reduce(*start);
    } else {
        cur.assign(nw_, 0);
        cur[0] = 2;
    }
    for (uint64_t i = 0; i < k; i++) cur = sqr(cur);
    return cur;
}

Words PolyMod::t_pow(const uint64_t* e, size_t e_words) const {
    Words acc(nw_, 0);
    acc[0] = 1;
    int top = -1;
    for (size_t i = e_words; i-- > 0;)
        if (e[i]) {
            top = int(i * 64 + 63 - __builtin_clzll(e[i]));
            break;
        }
    for (int i = top; i >= 0; i--) {
        acc = sqr(acc);
        if ((e[size_t(i) / 64] >> (i % 64)) & 1u) acc = mul_t(acc);
    }
    return acc;
}

// ---- inverse and square root ----------------------------------------------------

// a ^= b * t^s (a grows as needed)
static void xor_shifted(Words& a, const Words& b, int s) {
    const size_t wo = size_t(s) / 64;
    const int bo = s % 64;
    if (a.size() < b.size() + wo + 1) a.resize(b.size() + wo + 1, 0);
    for (size_t j = 0; j < b.size(); j++) {
        a[j + wo] ^= b[j] << bo;
        if (bo) a[j + wo + 1] ^= b[j] >> (64 - bo);
    }
}

// ---- gcd and division (schoolbook: used once per table, not per call) ------------

Words poly_div(const Words& a, const Words& b, Words* rem) {
    const int db = poly_degree(b);
    if (db < 0) throw std::invalid_argument("division by zero");
    Words r = a, q;
    poly_trim(r);
    for (int dr = poly_degree(r); dr >= db; dr = poly_degree(r)) {
        const int s = dr - db;
        if (q.size() <= size_t(s) / 64) q.resize(size_t(s) / 64 + 1, 0);
        q[size_t(s) / 64] ^= 1ull << (s % 64);
        xor_shifted(r, b, s);
        poly_trim(r);
    }
    if (rem) *rem = r;
    return q;
}

Words poly_gcd(Words a, Words b) {
    poly_trim(a);
    poly_trim(b);
    while (poly_degree(b) >= 0) {
        Words r;
        poly_div(a, b, &r);
        a = std::move(b);
        b = std::move(r);
    }
    return a;
}

Words PolyMod::inverse(const Words& a) const {
    // invariant: g1 a = u and g2 a = v (mod mu); deg u + deg v falls at every step
    Words u = reduce(a), v = mu_, g1(1, 1), g2;
    poly_trim(u);
    int du = poly_degree(u), dv = poly_degree(v);
    if (du < 0) throw std::invalid_argument("inverse of zero");
    while (du > 0) {
        int j = du - dv;
        if (j < 0) {
            std::swap(u, v);
            std::swap(g1, g2);
            std::swap(du, dv);
            j = -j;
        }
        xor_shifted(u, v, j);
        xor_shifted(g1, g2, j);
        poly_trim(u);
        poly_trim(g1);
        du = poly_degree(u);
        if (du < 0) throw std::invalid_argument("not invertible modulo mu");
    }
    return reduce(g1);
}

// even / odd coefficients of a 64-bit word, packed into 32 bits each
static inline uint32_t even_bits(uint64_t x) {
    x &= 0x5555555555555555ull;
    x = (x | (x >> 1)) & 0x3333333333333333ull;
    x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
    x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
    x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
    return (uint32_t)x;
}

// (even part, odd part) of a: a = ae(t^2) + t ao(t^2)
static void split_even_odd(const Words& a, Words& ae, Words& ao) {
    const size_t n = (a.size() + 1) / 2;
    ae.assign(n, 0);
    ao.assign(n, 0);
    for (size_t i = 0; i < a.size(); i++) {
        const uint64_t e = even_bits(a[i]), o = even_bits(a[i] >> 1);
        ae[i / 2] |= e << (32 * (i % 2));
        ao[i / 2] |= o << (32 * (i % 2));
    }
}

Words PolyMod::sqrt(const Words& a) const {
    if (sqrt_t_.empty()) {
        Words me, mo;
        split_even_odd(mu_, me, mo);
        sqrt_t_ = mul(me, inverse(mo));
    }
    Words ae, ao;
    split_even_odd(reduce(a), ae, ao);
    Words r = mul(ao, sqrt_t_);
    for (size_t i = 0; i < ae.size() && i < r.size(); i++) r[i] ^= ae[i];
    return r;
}

// ---- Berlekamp-Massey ---------------------------------------------------------

Words berlekamp_massey(const std::vector<uint8_t>& s) {
    const size_t N = s.size();
    const size_t W = N / 64 + 2;
    // rev: bit (N - 1 - i) holds s_i, so bits [N-1-n, N-1-n+L] read s_n, s_{n-1}, ..., s_{n-L}
    Words rev(W + 1, 0);
    for (size_t i = 0; i < N; i++)
        if (s[i]) {
            const size_t b = N - 1 - i;
            rev[b / 64] |= 1ull << (b % 64);
        }
    Words C(W, 0), B(W, 0), T;
    C[0] = 1;
    B[0] = 1;
    size_t L = 0, m = 1;
    for (size_t n = 0; n < N; n++) {
        // d = sum_{i=0..L} c_i s_{n-i}
        const size_t base = N - 1 - n;
        const size_t nw = L / 64 + 1;
        uint64_t acc = 0;
        for (size_t w = 0; w < nw; w++) {
            const size_t bit = base + 64 * w;
            const size_t wi = bit / 64, bo = bit % 64;
            uint64_t win = rev[wi] >> bo;
            if (bo && wi + 1 < rev.size()) win |= rev[wi + 1] << (64 - bo);
            acc ^= C[w] & win;
        }
        if (!__builtin_parityll(acc)) {
            m++;
            continue;
        }
        const bool grow = 2 * L <= n;
        if (grow) T = C;
        const size_t wo = m / 64, bo = m % 64;
        for (size_t w = 0; w + wo < W; w++) {
            C[w + wo] ^= B[w] << bo;
            if (bo && w + wo + 1 < W) C[w + wo + 1] ^= B[w] >> (64 - bo);
        }
        if (grow) {
            L = n + 1 - L;
            B.swap(T);
            m = 1;
        } else {
            m++;
        }
    }
    // characteristic orientation: mu_j = c_{L-j}
    Words mu(L / 64 + 1, 0);
    for (size_t j = 0; j <= L; j++) {
        const size_t i = L - j;
        if ((C[i / 64] >> (i % 64)) & 1u) mu[j / 64] |= 1ull << (j % 64);
    }
    return mu;
}

// ---- raw bit sequences of the base generators (block regeneration form) ------

static std::vector<uint8_t> raw_bits(int variant, size_t count, uint32_t seed) {
    std::vector<uint8_t> bits;
    bits.reserve(count);
    if (variant == 0) {
        const int n = 624, m = 397;
        uint32_t x[624];
        x[0] = seed;
        for (int i = 1; i < n; i++) x[i] = 1812433253u * (x[i - 1] ^ (x[i - 1] >> 30)) + uint32_t(i);
        while (bits.size() < count) {
            for (int k = 0; k < n; k++) {  // eq. (stepnomod): in place, indices mod n
                const uint32_t y = (x[k] & 0x80000000u) | (x[(k + 1) % n] & 0x7fffffffu);
                x[k] = x[(k + m) % n] ^ (y >> 1) ^ ((y & 1u) ? 0x9908B0DFu : 0u);
            }
            for (int k = 0; k < n && bits.size() < count; k++) bits.push_back(uint8_t(x[k] & 1u));
        }
    } else if (variant == 1) {
        const int n = 312, m = 156;
        uint64_t x[312];
        x[0] = seed;
        for (int i = 1; i < n; i++)
            x[i] = 6364136223846793005ull * (x[i - 1] ^ (x[i - 1] >> 62)) + uint64_t(i);
        while (bits.size() < count) {
            for (int k = 0; k < n; k++) {
                const uint64_t y = (x[k] & 0xFFFFFFFF80000000ull) | (x[(k + 1) % n] & 0x7FFFFFFFull);
                x[k] = x[(k + m) % n] ^ (y >> 1) ^ ((y & 1u) ? 0xB5026F5AA96619E9ull : 0ull);
            }
            for (int k = 0; k < n && bits.size() < count; k++) bits.push_back(uint8_t(x[k] & 1u));
        }
    } else {
        // SFMT, eq. (sfmt_step), with the variant's parameter set
        const SfmtSet& P = sfmt_set((uint32_t)variant);
        const int N = (int)P.n, m = (int)P.pos1;
        const int sl2 = 8 * (int)P.sl2, sr2 = 8 * (int)P.sr2;
        std::vector<unsigned __int128> w(N);
        std::vector<uint32_t> s32(4 * N);
        s32[0] = seed;
        for (int i = 1; i < 4 * N; i++) s32[i] = 1812433253u * (s32[i - 1] ^ (s32[i - 1] >> 30)) + uint32_t(i);
        for (int k = 0; k < N; k++)
            w[k] = (unsigned __int128)s32[4 * k] | ((unsigned __int128)s32[4 * k + 1] << 32) |
                   ((unsigned __int128)s32[4 * k + 2] << 64) | ((unsigned __int128)s32[4 * k + 3] << 96);
        auto sub = [](unsigned __int128 v, int j) { return uint32_t(v >> (32 * j)); };
        while (bits.size() < count) {
            for (int k = 0; k < N; k++) {
                const unsigned __int128 a = w[k], b = w[(k + m) % N], c = w[(k + N - 2) % N], d = w[(k + N - 1) % N];
                unsigned __int128 bm = 0, dl = 0;
                for (int j = 0; j < 4; j++) {
                    bm |= (unsigned __int128)((sub(b, j) >> P.sr1) & P.msk[j]) << (32 * j);
                    dl |= (unsigned __int128)(sub(d, j) << P.sl1) << (32 * j);
                }
                w[k] = a ^ (a << sl2) ^ bm ^ (c >> sr2) ^ dl;
            }
            for (int k = 0; k < N && bits.size() < count; k++) bits.push_back(uint8_t(uint32_t(w[k]) & 1u));
        }
    }
    return bits;
}

// Sequence <mask, X_i>, i < count, of an SFMT set's states X_i from a
// pseudo-random full state X_0 (splitmix64 words from `seed`, which also
// gives the mask): X_i is the window of the N words w_i .. w_{i+N-1}.
static std::vector<uint8_t> masked_bits(int variant, size_t count, uint64_t seed) {
    const SfmtSet& P = sfmt_set((uint32_t)variant);
    const int N = (int)P.n, m = (int)P.pos1;
    const int sl2 = 8 * (int)P.sl2, sr2 = 8 * (int)P.sr2;
    auto next = [&seed]() {
        uint64_t z = (seed += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    auto word = [&next]() { return (unsigned __int128)next() | ((unsigned __int128)next() << 64); };
    std::vector<unsigned __int128> w(N + count), mask(N);
    for (int k = 0; k < N; k++) w[k] = word();
    for (int k = 0; k < N; k++) mask[k] = word();
    auto sub = [](unsigned __int128 v, int j) { return uint32_t(v >> (32 * j)); };
    for (size_t k = N; k < N + count; k++) {  // eq. (sfmt_step) on the growing sequence
        const unsigned __int128 a = w[k - N], b = w[k - N + m], c = w[k - 2], d = w[k - 1];
        unsigned __int128 bm = 0, dl = 0;
        for (int j = 0; j < 4; j++) {
            bm |= (unsigned __int128)((sub(b, j) >> P.sr1) & P.msk[j]) << (32 * j);
            dl |= (unsigned __int128)(sub(d, j) << P.sl1) << (32 * j);
        }
        w[k] = a ^ (a << sl2) ^ bm ^ (c >> sr2) ^ dl;
    }
    std::vector<uint8_t> bits(count);
    for (size_t i = 0; i < count; i++) {
        uint64_t acc = 0;
        for (int k = 0; k < N; k++) {
            const unsigned __int128 v = w[i + k] & mask[k];
            acc ^= (uint64_t)v ^ (uint64_t)(v >> 64);
        }
        bits[i] = uint8_t(__builtin_parityll(acc));
    }
    return bits;
}

// The minimal polynomial of the map is the lcm of those of the sequences it
// drives; one output bit, or one state, may miss a factor (SFMT's mu is not
// irreducible). MT19937-32/-64: mu is irreducible, bit 0 of one state gives
// it. SFMT19937: bit 0 of the seeded state reaches the state dimension 19968,
// so it is mu. The other SFMT sets: the lcm over random functionals
// <mask, X_i> of random states until the degree reaches the dimension or 16
// in a row add nothing (a factor is missed with probability at most 2^-16).
Words generator_minpoly(int variant) {
    const bool sfmt = is_sfmt((uint32_t)variant);
    const size_t dim = sfmt ? 128 * (size_t)sfmt_set((uint32_t)variant).n : 19968;
    const size_t terms = 2 * dim + 256;
    Words mu = variant <= (int)kSFMT ? berlekamp_massey(raw_bits(variant, terms, 20230928u))
                                     : berlekamp_massey(masked_bits(variant, terms, 20230928u));
    poly_trim(mu);
    int quiet = 0;
    for (uint64_t s = 1; sfmt && (size_t)poly_degree(mu) < dim && quiet < 16; s++) {
        Words m2 = berlekamp_massey(masked_bits(variant, terms, 20230928u + 7919u * s));
        poly_trim(m2);
        Words rem;
        poly_div(mu, m2, &rem);
        if (poly_degree(rem) < 0) {
            quiet++;
            continue;
        }
        mu = poly_mul(mu, poly_div(m2, poly_gcd(mu, m2)));
        poly_trim(mu);
        quiet = 0;
    }
    return mu;
}

}  // namespace vmt
