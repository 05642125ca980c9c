"""Pins of the oracle's SFMT with the other published parameter sets
(Mersenne exponents 607, 1279, 2281, 4253, 11213): the recurrence of
eq. (sfmt_step) with each set's shifts, masks and state size N = MEXP/128 + 1.

None of these sets is printed in the paper (it gives SFMT19937). They are
pinned structurally, which a wrong constant breaks almost surely:

* the oracle's step equals an independent 128-bit-integer formulation;
* the minimal polynomial mu of the one-step map has exactly one irreducible
  factor of degree MEXP (MEXP is prime, so t^(2^MEXP) - t is the product of
  the irreducibles of degree 1 and MEXP; mu has degree < 2 MEXP);
* the stored mu annihilates fresh random states (it is the map's minimal
  polynomial, not one state's);
* the set's period-certification vector annihilates the part of the state
  outside the degree-MEXP factor, and certified seeded states have a nonzero
  component along it (period a multiple of 2^MEXP - 1);
* jumps (Horner's rule) equal stepping, and the lane distance J = 2^(MEXP -
  log2 M) applied M times equals one jump by 2^MEXP.
"""
import numpy as np
import pytest

from oracle import pyoracle as O
from tests import golden_io
from tests.linear_ref import pdivmod

SETS = [O.SFMT607, O.SFMT1279, O.SFMT2281, O.SFMT4253, O.SFMT11213]
# (POS1, SL1, SL2 bytes, SR1, SR2 bytes, MSK) per set, typed independently of the oracle's table
PARAMS = {
    O.SFMT607: (2, 15, 3, 13, 3, (0xFDFF37FF, 0xEF7F3F7D, 0xFF777B7D, 0x7FF7FB2F)),
    O.SFMT1279: (7, 14, 3, 5, 1, (0xF7FEFFFD, 0x7FEFCFFF, 0xAFF3EF3F, 0xB5FFFF7F)),
    O.SFMT2281: (12, 19, 1, 5, 1, (0xBFF7FFBF, 0xFDFFFFFE, 0xF7FFEF7F, 0xF2F7CBBF)),
    O.SFMT4253: (17, 20, 1, 7, 1, (0x9F7BFFFF, 0x9FFFFF5F, 0x3EFFFFFB, 0xFFFFF7BB)),
    O.SFMT11213: (68, 14, 3, 7, 3, (0xEFFFF7FB, 0xFFFFFFEF, 0xDFDFBFFF, 0x7FFFDBFD)),
}


def random_state(variant, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2**32, O.STATE_LEN[variant], dtype=np.uint64).astype(np.uint32)


def words128(x):
    return [sum(int(x[4 * k + j]) << (32 * j) for j in range(4)) for k in range(len(x) // 4)]


def step_bigint(variant, x, count):
    pos1, sl1, sl2, sr1, sr2, msk = PARAMS[variant]
    N = O.STATE_WORDS[variant]
    W = words128(x)
    M32, M128 = (1 << 32) - 1, (1 << 128) - 1

    def per_sub(v, f):
        return sum((f(j, (v >> (32 * j)) & M32) & M32) << (32 * j) for j in range(4))

    out = []
    for k in range(count):
        a, b, c, d = W[k], W[k + pos1], W[k + N - 2], W[k + N - 1]
        r = a ^ ((a << (8 * sl2)) & M128) ^ per_sub(b, lambda j, s: (s >> sr1) & msk[j]) ^ (c >> (8 * sr2))
        r ^= per_sub(d, lambda j, s: s << sl1)
        W.append(r)
        out.append(r)
    return out


def factors(variant):
    """(mu, phi_p) with phi_p the irreducible factor of degree MEXP."""
    mu = golden_io.minpoly(variant)
    mexp = O.MEXP[variant]
    g = O.poly_gcd(mu, golden_io.tpow2(variant)[mexp] ^ 2)  # irreducible factors of degree 1 and MEXP
    lin = O.poly_gcd(g, 0b110)                                # the degree-1 ones: t, t + 1
    phi, rem = pdivmod(g, lin)
    assert rem == 0
    return mu, phi


def parity_of(x, vec):
    v = 0
    for j in range(4):
        v ^= int(x[j]) & int(vec[j])
    return bin(v).count("1") & 1


@pytest.mark.parametrize("variant", SETS)
def test_step_matches_bigint_formulation(variant):
    x = random_state(variant, 3)
    got = O.Scalar(variant, x).out(3 * O.STATE_WORDS[variant] + 17)
    ref = step_bigint(variant, x, len(got))
    for k in range(len(got)):
        assert sum(int(got[k][j]) << (32 * j) for j in range(4)) == ref[k], k


@pytest.mark.parametrize("variant", SETS)
def test_minpoly_has_one_irreducible_factor_of_degree_mexp(variant):
    mu, phi = factors(variant)
    mexp = O.MEXP[variant]
    assert phi.bit_length() - 1 == mexp
    assert mu.bit_length() - 1 <= 128 * O.STATE_WORDS[variant] < 2 * mexp
    # phi irreducible: t^(2^MEXP) = t mod phi, prime degree, no linear factor
    assert O.poly_mod(golden_io.tpow2(variant)[mexp], phi) == 2
    assert O.poly_gcd(phi, 0b110) == 1


@pytest.mark.parametrize("variant", SETS)
def test_minpoly_annihilates_fresh_states(variant):
    mu = golden_io.minpoly(variant)
    for s in range(4):
        assert not O.jump_canon(variant, random_state(variant, 500 + s), mu).any()
    # a proper divisor does not: dropping a factor leaves some state alive
    mu_div, phi = factors(variant)
    rest, rem = pdivmod(mu, phi)
    assert rem == 0
    assert O.jump_canon(variant, random_state(variant, 77), rest).any()


@pytest.mark.parametrize("variant", SETS)
def test_parity_vector_annihilates_the_rest(variant):
    # Period certification can only force a component along phi if <PARITY, w_0>
    # vanishes on the image of phi(F) (the states with no phi component).
    mu, phi = factors(variant)
    par = O.sfmt_parity(variant)
    ys = [O.jump_canon(variant, random_state(variant, 900 + s), phi) for s in range(12)]
    for y in ys:
        assert parity_of(y, par) == 0
    # not vacuous: word 0 of that image is not identically zero, and flipping a
    # bit of PARITY that some image state has set breaks the property
    w0 = [sum(int(y[j]) << (32 * j) for j in range(4)) for y in ys]
    assert any(w0)
    b = (next(v for v in w0 if v) & -next(v for v in w0 if v)).bit_length() - 1
    wrong = par.copy()
    wrong[b // 32] ^= np.uint32(1 << (b % 32))
    assert any(parity_of(y, wrong) for y in ys)


@pytest.mark.parametrize("variant", SETS)
@pytest.mark.parametrize("seed", [1234, 0, 4321])
def test_certified_states_have_a_phi_component(variant, seed):
    mu, phi = factors(variant)
    rest, _ = pdivmod(mu, phi)
    x = O.seed_state(variant, seed)
    assert parity_of(x, O.sfmt_parity(variant)) == 1
    assert O.jump_canon(variant, x, rest).any()  # rest(F) x != 0: the phi component is nonzero


@pytest.mark.parametrize("variant", SETS)
@pytest.mark.parametrize("d", [0, 1, 2, 7, 1000, 12345])
def test_jump_matches_stepping(variant, d):
    x = random_state(variant, 11)
    y = O.jump_canon(variant, x, O.poly_powmod_t(d, golden_io.minpoly(variant)))
    ref = O.Scalar(variant, x)
    ref.skip(d)
    np.testing.assert_array_equal(O.Scalar(variant, y).out(50), ref.out(50))


@pytest.mark.parametrize("variant", SETS)
@pytest.mark.parametrize("M", [2, 4, 64])
def test_lane_distance_composes_to_2_pow_mexp(variant, M):
    # M jumps by J = 2^(MEXP - log2 M) equal one jump by 2^MEXP (composition;
    # the psi part need not have period 2^MEXP - 1, so no period identity here)
    mu = golden_io.minpoly(variant)
    x = random_state(variant, 21)
    y = x.copy()
    for _ in range(M):
        y = O.jump_canon(variant, y, golden_io.lane_poly(variant, M))
    z = O.jump_canon(variant, x, golden_io.tpow2(variant)[O.MEXP[variant]])
    np.testing.assert_array_equal(y, z)
    del mu


@pytest.mark.parametrize("variant", SETS)
def test_vstream_lanes_are_jumped_base_streams(variant):
    M = 4
    x = O.seed_state(variant, 1234)
    v = O.VStream(variant, M, x, golden_io.lane_poly(variant, M))
    s = v.generate(4 * M * 300).reshape(-1, M, 4)  # [k][lane][sub-word]
    for t in range(M):
        lane = x.copy()
        for _ in range(t):
            lane = O.jump_canon(variant, lane, golden_io.lane_poly(variant, M))
        np.testing.assert_array_equal(s[:, t, :], O.Scalar(variant, lane).out(300), err_msg=f"lane {t}")
