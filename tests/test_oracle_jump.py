"""Pins of the oracle's jump-ahead (Sec. 3.1) and V-stream (Sec. 3).

Nothing here compares the oracle with itself by retyping a formula: the jump
is checked against brute-force stepping, composition, the period of the base
generator (Sec. 2.2: 2^19937 - 1), the Frobenius identity of the lane
polynomials, and the C++ library stream.
"""
import multiprocessing as mp
import os

import numpy as np
import pytest

from oracle import pyoracle as O
from tests import golden_io, stdpins

VARIANTS = [O.MT32, O.MT64, O.SFMT]
N_WORDS = {O.MT32: 624, O.MT64: 312, O.SFMT: 156}


def _random_state(variant, seed):
    rng = np.random.default_rng(seed)
    if variant == O.MT64:
        return rng.integers(0, 2**64, 312, dtype=np.uint64)
    return rng.integers(0, 2**32, 624, dtype=np.uint64).astype(np.uint32)


def _next_words(variant, canon, count):
    g = O.Scalar(variant, canon)
    return g.out(count)


@pytest.mark.parametrize("variant", VARIANTS)
def test_minpoly_degree_and_annihilation(variant):
    # MT: effective state nw - r = 19937 bits (Sec. 2.1-2.3); SFMT: 156 * 128.
    mu = golden_io.minpoly(variant)
    assert mu.bit_length() - 1 == (19968 if variant == O.SFMT else 19937)
    # recomputing from a different (random) state gives the same polynomial
    assert O.minpoly(variant, _random_state(variant, 1)) == mu
    # mu(F) X = 0: every output bit after the jump by mu is zero
    for s in range(3):
        y = O.jump_canon(variant, _random_state(variant, 100 + s), mu)
        if variant == O.SFMT:
            assert not y.any()
        else:
            # only the r = 31 unused low bits of the oldest word may survive
            assert not y[1:].any() and int(y[0]) >> 31 == 0
            assert not _next_words(variant, y, 2 * N_WORDS[variant]).any()


@pytest.mark.parametrize("variant", VARIANTS)
def test_minpoly_squarefree(variant):
    # gcd(mu, mu') = 1, so Frobenius is injective mod mu and 2^s-th roots are unique
    mu = golden_io.minpoly(variant)
    deriv = 0
    for i in range(1, mu.bit_length()):
        if (mu >> i) & 1 and i & 1:
            deriv |= 1 << (i - 1)
    assert O.poly_gcd(mu, deriv) == 1


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("d", [0, 1, 2, 155, 156, 157, 311, 312, 313, 623, 624, 625, 1248, 100000, 1000007])
def test_jump_matches_brute_force(variant, d):
    mu = golden_io.minpoly(variant)
    x = _random_state(variant, 7 + d)
    g = O.poly_powmod_t(d, mu)
    ref = O.Scalar(variant, x)
    ref.skip(d)
    jumped = O.Scalar(variant, O.jump_canon(variant, x, g))
    np.testing.assert_array_equal(jumped.out(3 * N_WORDS[variant]), ref.out(3 * N_WORDS[variant]))


@pytest.mark.parametrize("variant", [O.MT32, O.MT64])
def test_jump_from_seeded_state_matches_library_stream(variant):
    bits = 32 if variant == O.MT32 else 64
    mu = golden_io.minpoly(variant)
    ref = stdpins.std_stream(bits, 5489, 20000)
    x = O.seed_state(variant, 5489)
    for d in (1, 624, 12345):
        y = O.jump_canon(variant, x, O.poly_powmod_t(d, mu))
        np.testing.assert_array_equal(O.Scalar(variant, y).out(1000), ref[d : d + 1000])


@pytest.mark.parametrize("variant", VARIANTS)
def test_jump_composition(variant):
    mu = golden_io.minpoly(variant)
    x = _random_state(variant, 21)
    d1, d2 = 2**70 + 5, 3**40
    a = O.jump_canon(variant, O.jump_canon(variant, x, O.poly_powmod_t(d1, mu)), O.poly_powmod_t(d2, mu))
    b = O.jump_canon(variant, x, O.poly_powmod_t(d1 + d2, mu))
    np.testing.assert_array_equal(_next_words(variant, a, 700), _next_words(variant, b, 700))


@pytest.mark.parametrize("variant", VARIANTS)
def test_lane_polys_frobenius(variant):
    # The fixture rows are one squaring chain: row q+1 = (row q)^2.
    mu = golden_io.minpoly(variant)
    rows = golden_io.tpow2(variant)
    for q in range(19931, 19937):
        assert O.poly_sqrmod(rows[q], mu) == rows[q + 1]
    if variant != O.SFMT:
        # Period 2^19937 - 1 (Sec. 2.2) <=> t^(2^19937) = t mod phi; then each
        # t^J is the unique 2^s-th root of t (mu is squarefree).
        assert rows[19937] == 2


@pytest.mark.parametrize("variant,M", [(O.MT32, 16), (O.MT32, 4), (O.MT64, 8), (O.MT64, 2)])
def test_M_lane_jumps_are_one_step(variant, M):
    # M * J = 2^19937 = 1 + (2^19937 - 1): M jumps by J equal a single step.
    gJ = golden_io.lane_poly(variant, M)
    x = _random_state(variant, 5)
    y = x.copy()
    for _ in range(M):
        y = O.jump_canon(variant, y, gJ)
    ref = O.Scalar(variant, x)
    ref.skip(1)
    np.testing.assert_array_equal(_next_words(variant, y, 1000), ref.out(1000))


def _chain_job(variant):
    mu = golden_io.minpoly(variant)
    x = O.seed_state(variant, 5489 if variant != O.SFMT else 1234)
    assert O.minpoly(variant, x) == mu
    out = {}
    cur, q = 2, 0
    for target in list(range(19931, 19937)) + [19937]:
        cur = O.poly_sqr_chain(target - q, mu, start=cur)
        q = target
        out[q] = cur
    return variant, out


@pytest.mark.skipif(os.environ.get("VMT_SKIP_CHAIN") == "1", reason="full squaring chain skipped on request")
def test_full_squaring_chain_reproduces_fixtures():
    # ~90 s: recompute t -> t^2 -> ... -> t^(2^19937) mod mu for all three
    # generators in parallel, check the stored lane polynomials and, for MT,
    # that t^(2^19937) = t (phi irreducible of prime degree 19937, hence
    # primitive: the period of Sec. 2.2).
    with mp.get_context("fork").Pool(3) as pool:
        for variant, out in pool.imap_unordered(_chain_job, VARIANTS):
            assert out == golden_io.tpow2(variant)
            if variant != O.SFMT:
                assert out[19937] == 2
