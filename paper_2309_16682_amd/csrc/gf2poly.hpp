// gf2poly.hpp -- host-side GF(2)[t] arithmetic for the jump-ahead of Sec. 3.1.
//
// The state after d steps of an F2-linear generator is g(F) X with
// g = t^d mod mu, mu the minimal polynomial of the one-step map F (Cayley-
// Hamilton); the paper's matrix power F^J is replaced by this polynomial,
// which gives the same state at a tiny fraction of the cost. This file
// computes mu (Berlekamp-Massey) and powers of t modulo mu; the device
// applies g to the state.
//
// Representation: little-endian uint64 words, bit i = coefficient of t^i.
// Multiplication uses carry-less multiply (PCLMULQDQ) with Karatsuba,
// reduction uses Barrett's method with a precomputed quotient.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace vmt {

using Words = std::vector<uint64_t>;

int poly_degree(const Words& a);  // -1 for the zero polynomial
void poly_trim(Words& a);

// Full (unreduced) product.
Words poly_mul(const Words& a, const Words& b);

// Greatest common divisor (monic, as every nonzero polynomial over GF(2)).
Words poly_gcd(Words a, Words b);

// Quotient a / b; *rem (optional) receives the remainder. b must be nonzero.
Words poly_div(const Words& a, const Words& b, Words* rem = nullptr);

// Arithmetic modulo a fixed polynomial mu of degree D >= 64.
class PolyMod {
public:
    explicit PolyMod(const Words& mu);
    int degree() const { return D_; }
    size_t words() const { return nw_; }  // words of a reduced element
    const Words& modulus() const { return mu_; }

    Words reduce(const Words& a) const;   // any degree < 2D
    Words sqr(const Words& a) const;      // a^2 mod mu
    Words mul(const Words& a, const Words& b) const;
    Words mul_t(const Words& a) const;    // a * t mod mu
    Words t_pow2(uint64_t k, const Words* start = nullptr) const;  // start^(2^k), start = t by default
    Words t_pow(const uint64_t* e, size_t e_words) const;           // t^e mod mu

    // Inverse modulo mu (extended Euclid); a must be coprime to mu.
    Words inverse(const Words& a) const;
    // The square root modulo a square-free mu: a = ae(t^2) + t ao(t^2) gives
    // sqrt(a) = ae(t) + sqrt(t) ao(t), and sqrt(t) = me(t) / mo(t) for
    // mu = me(t^2) + t mo(t^2) (since mu(t) = 0). Squaring is a bijection
    // modulo a square-free mu, so the root is unique.
    Words sqrt(const Words& a) const;

private:
    Words mu_;
    Words barrett_;  // floor(t^(2D) / mu)
    mutable Words sqrt_t_;  // sqrt(t) mod mu, computed on first use
    int D_;
    size_t nw_;
};

// Minimal polynomial of a bit sequence by Berlekamp-Massey; returned in
// "characteristic" orientation: sum_j mu_j s_{i+j} = 0 for all i.
Words berlekamp_massey(const std::vector<uint8_t>& s);

// Minimal polynomial of the one-step map of a base generator
// (0 = MT19937-32, 1 = MT19937-64, 2 = SFMT19937), from a fixed internal
// seed state.
Words generator_minpoly(int variant);

}  // namespace vmt
