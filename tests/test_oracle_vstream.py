"""Pins of the oracle's V-stream (Sec. 3, eq. combseq and Table jvalues)."""
import numpy as np
import pytest

from oracle import pyoracle as O
from tests import golden_io, stdpins


@pytest.mark.parametrize("variant,M", [(O.MT32, 16), (O.MT32, 4), (O.MT64, 8), (O.MT64, 2)])
def test_lane0_is_the_library_stream(variant, M):
    # lane 0 starts at X_0, so S[0::M] is the base generator's own stream
    bits = 32 if variant == O.MT32 else 64
    v = O.VStream(variant, M, O.seed_state(variant, 5489), golden_io.lane_poly(variant, M))
    s = v.generate(M * 3000)
    np.testing.assert_array_equal(s[0::M], stdpins.std_stream(bits, 5489, 3000))


@pytest.mark.parametrize("variant,M", [(O.MT32, 16), (O.MT64, 8)])
def test_lane_after_last_wraps_to_lane0_plus_one(variant, M):
    # lane M would start at M*J = 2^19937 = 1 + period: lane 0 shifted by one
    bits = 32 if variant == O.MT32 else 64
    gJ = golden_io.lane_poly(variant, M)
    v = O.VStream(variant, M, O.seed_state(variant, 5489), gJ)
    last = v.lane_canon(M - 1)
    nxt = O.Scalar(variant, O.jump_canon(variant, last, gJ)).out(2000)
    np.testing.assert_array_equal(nxt, stdpins.std_stream(bits, 5489, 2001)[1:])


@pytest.mark.parametrize("variant,M", [(O.MT32, 8), (O.MT64, 4), (O.SFMT, 4)])
def test_lane_t_by_power_of_lane_poly(variant, M):
    # lane t = X_0 advanced by t*J: check lane 3 against g_J^3 mod mu applied once
    mu = golden_io.minpoly(variant)
    gJ = golden_io.lane_poly(variant, M)
    x0 = O.seed_state(variant, 5489 if variant != O.SFMT else 1234)
    v = O.VStream(variant, M, x0, gJ)
    g3 = O.poly_mulmod(O.poly_mulmod(gJ, gJ, mu), gJ, mu)
    ref = O.Scalar(variant, O.jump_canon(variant, x0, g3)).out(1500)
    got = O.Scalar(variant, v.lane_canon(3)).out(1500)
    np.testing.assert_array_equal(got, ref)


def test_sfmt_interleave_is_per_128bit_word():
    M = 4
    gJ = golden_io.lane_poly(O.SFMT, M)
    x0 = O.seed_state(O.SFMT, 1234)
    v = O.VStream(O.SFMT, M, x0, gJ)
    s = v.generate(4 * M * 500).reshape(500, M, 4)
    lane = x0.copy()
    for t in range(M):
        np.testing.assert_array_equal(s[:, t, :], O.Scalar(O.SFMT, lane).out(500))
        lane = O.jump_canon(O.SFMT, lane, gJ)


_VJUMP_CASES = [(v, M, first) for v, M in ((O.MT32, 16), (O.MT64, 8), (O.SFMT, 4))
                for first in (0, 5, 1000, 9983, 9984)] + [(O.SFMT, 64, 5)]  # 64 lanes: one offset (CPU time)


@pytest.mark.parametrize("variant,M,first", _VJUMP_CASES)
def test_vjump_skips_d_times_M_words(variant, M, first):
    # every lane advances d steps: the stream skips d*M elements (d*M*4 uint32 for SFMT)
    mu = golden_io.minpoly(variant)
    gJ = golden_io.lane_poly(variant, M)
    x0 = O.seed_state(variant, 77)
    per = 4 if variant == O.SFMT else 1
    for d in (1, 3, 700):
        a = O.VStream(variant, M, x0, gJ)
        b = O.VStream(variant, M, x0, gJ)
        a.generate(first)
        b.generate(first)
        a.jump(O.poly_powmod_t(d, mu))
        b.generate(d * M * per)
        np.testing.assert_array_equal(a.generate(3000), b.generate(3000))


def test_chunked_generation_equals_one_call():
    gJ = golden_io.lane_poly(O.MT32, 16)
    x0 = O.seed_state(O.MT32, 5489)
    a = O.VStream(O.MT32, 16, x0, gJ)
    b = O.VStream(O.MT32, 16, x0, gJ)
    whole = a.generate(30000)
    parts = [b.generate(n) for n in (1, 15, 16, 9983, 9985, 7, 9993)]
    np.testing.assert_array_equal(np.concatenate(parts), whole)
