"""Pins of the linear-complexity self-check (Sec. 4.1: LinearComp; Sec. 3, eq.
combseq; Sec. 3.1).

The oracle's Berlekamp-Massey is pinned to closed forms (a known LFSR, the
all-zero and all-one sequences, a single 1, whose linear complexity is its
length) and to the minimal polynomials of the base generators. It then
measures the linear complexity of V-stream bits directly: for MT19937-32/-64
every bit of the interleaved stream obeys the base generator's minimal
polynomial mu itself (degree 19937, for every M), because lane t starts
t * 2^(19937 - log2 M) steps in; with any other lane spacing (a mistake
planted in the oracle) the complexity is 19937 M. For SFMT19937 the bits of
the sequence of 128-bit words obey phi(t) psi(t^M) (phi the degree-19937
factor of mu, psi = mu / phi). The library's vmt_check_poly must return
exactly these polynomials.
"""
import numpy as np
import pytest

from oracle import pyoracle as O
from tests import golden_io
from tests.linear_ref import check_poly, pdivmod, pmul, sfmt_factors

D = 19937


def lfsr_bits(poly: int, init, count):
    """Bits of the recurrence sum_j poly_j s_{i+j} = 0 (poly monic, degree L)."""
    L = poly.bit_length() - 1
    s = list(init)
    assert len(s) == L
    taps = [j for j in range(L) if (poly >> j) & 1]
    while len(s) < count:
        i = len(s) - L
        v = 0
        for j in taps:
            v ^= s[i + j]
        s.append(v)
    return np.array(s, np.uint8)


def vstream(variant, M, seed, count, skip=0, lane_poly=None):
    g = golden_io.lane_poly(variant, M) if lane_poly is None else lane_poly
    v = O.VStream(variant, M, O.seed_state(variant, seed=seed), g)
    if skip:
        v.generate(skip)
    return v.generate(count)


def bit_seq(u, b):
    return ((u >> type(u[0])(b)) & 1).astype(np.uint8)


# ---- Berlekamp-Massey against closed forms ------------------------------------


def test_bm_known_lfsr():
    # s_{i+3} = s_{i+1} + s_i: minimal polynomial t^3 + t + 1
    assert O.berlekamp_massey(lfsr_bits(0b1011, [1, 0, 0], 40)) == 0b1011
    # t^61 + t^5 + t^2 + t + 1 is irreducible (prime degree, t^(2^61) = t mod p,
    # no root), so every nonzero sequence it generates has it as minimal polynomial
    p = (1 << 61) | (1 << 5) | (1 << 2) | (1 << 1) | 1
    assert O.poly_sqr_chain(61, p) == 2 and O.poly_gcd(p, 0b110) == 1
    rng = np.random.default_rng(3)
    init = list(rng.integers(0, 2, 61))
    init[0] = 1
    assert O.berlekamp_massey(lfsr_bits(p, init, 300)) == p


def test_bm_degenerate_sequences():
    assert O.berlekamp_massey(np.zeros(100, np.uint8)) == 1          # complexity 0
    assert O.berlekamp_massey(np.ones(100, np.uint8)) == 0b11        # s_{i+1} = s_i
    for n in (1, 2, 7, 64, 65, 200):
        s = np.zeros(n, np.uint8)
        s[-1] = 1
        assert O.berlekamp_massey(s).bit_length() - 1 == n           # a single 1 at the end: complexity n


@pytest.mark.parametrize("variant,seed", [(O.MT32, 77), (O.MT64, 77), (O.SFMT, 1234), (O.SFMT, 77)])
def test_bm_reproduces_base_minpoly(variant, seed):
    # bit 0 of the base generator's raw words (the fixture was made from another state)
    x = O.seed_state(variant, seed=seed)
    raw = O.Scalar(variant, x).raw(2 * 19968 + 64)
    b = raw[:, 0] if variant == O.SFMT else raw  # SFMT: sub-word 0 of each 128-bit word
    p = O.berlekamp_massey(b & 1)
    mu = golden_io.minpoly(variant)
    if (variant, seed) == (O.SFMT, 77):
        # mu = phi psi is not irreducible: a state whose psi part lies in a smaller
        # invariant subspace has a proper divisor of mu (here of degree 19965)
        q, rem = pdivmod(mu, p)
        assert rem == 0 and p.bit_length() - 1 == 19965
    else:
        assert p == mu


# ---- linear complexity of the V-stream --------------------------------------------


@pytest.mark.parametrize("variant", [O.MT32, O.MT64])
@pytest.mark.parametrize("M", [1, 2, 4, 16])
def test_vstream_bits_obey_mu(variant, M):
    mu = golden_io.minpoly(variant)
    u = vstream(variant, M, 5489, 2 * D + 100, skip=12345)
    for b in ((0, 13, 31) if variant == O.MT32 else (0, 31, 40, 63)):
        assert O.berlekamp_massey(bit_seq(u, b)) == mu, (variant, M, b)


@pytest.mark.parametrize("M", [2, 4])
def test_planted_lane_spacing_raises_complexity(M):
    # lanes spaced J + 1 instead of J: the bits' complexity becomes 19937 M
    mu = golden_io.minpoly(O.MT32)
    wrong = O.poly_mulmod(golden_io.lane_poly(O.MT32, M), 2, mu)
    u = vstream(O.MT32, M, 5489, 2 * D * M + 200, lane_poly=wrong)
    assert O.berlekamp_massey(u & 1).bit_length() - 1 == D * M


def test_sfmt_factorisation():
    mu, phi, psi = sfmt_factors()
    assert phi.bit_length() - 1 == D and psi.bit_length() - 1 == 31
    # phi irreducible of prime degree: t^(2^19937) = t mod phi and phi has no root
    assert O.poly_mod(golden_io.tpow2(O.SFMT)[D], phi) == 2
    assert phi & 1 and bin(phi).count("1") % 2 == 1


@pytest.mark.parametrize("M", [1, 4, 8])
def test_sfmt_vstream_bits_obey_phi_psiM(M):
    A = check_poly(O.SFMT, M)
    n128 = 2 * (A.bit_length() - 1) + 100
    u = vstream(O.SFMT, M, 1234, 4 * n128, skip=4 * 777).reshape(-1, 4)
    for j, b in ((0, 0), (1, 7), (3, 31)):
        assert O.berlekamp_massey(bit_seq(u[:, j], b)) == A, (M, j, b)
    if M == 4:
        # the uint32 stream interleaves four such sequences: complexity 4 deg A
        w = u.reshape(-1)[: 8 * (A.bit_length() - 1) + 100]
        assert O.berlekamp_massey(w & 1).bit_length() - 1 == 4 * (A.bit_length() - 1)


# ---- the library's polynomials ----------------------------------------------------


@pytest.mark.parametrize("M,variant", [(4, O.SFMT607), (16, O.SFMT1279), (2, O.SFMT4253), (8, O.SFMT11213)])
def test_sfmt_sets_vstream_bits_obey_check_poly(variant, M):
    # The same collapse for the other SFMT parameter sets (phi here also holds
    # the linear factors of mu: their roots satisfy alpha^(2^MEXP) = alpha too).
    # A seeded state and one bit need not see every factor of psi, so the
    # measured minimal polynomial divides A; it always holds the degree-MEXP
    # factor (the certified state has a component along it).
    A = check_poly(variant, M)
    mexp = O.MEXP[variant]
    frob = golden_io.tpow2(variant)[mexp]
    g = O.poly_gcd(golden_io.minpoly(variant), frob ^ 2)
    phi_p, rem = pdivmod(g, O.poly_gcd(g, 0b110))  # the irreducible factor of degree MEXP
    assert rem == 0 and phi_p.bit_length() - 1 == mexp
    n128 = 2 * (A.bit_length() - 1) + 100
    u = vstream(variant, M, 1234, 4 * n128, skip=4 * 55).reshape(-1, 4)
    for j, b in ((0, 0), (2, 21)):
        p = O.berlekamp_massey(bit_seq(u[:, j], b))
        assert pdivmod(A, p)[1] == 0, (variant, M, j, b)
        assert pdivmod(p, phi_p)[1] == 0, (variant, M, j, b)
    # with the lane spacing planted one step off, A no longer annihilates the stream
    wrong = O.poly_mulmod(golden_io.lane_poly(variant, M), 2, golden_io.minpoly(variant))
    w = vstream(variant, M, 1234, 4 * n128, lane_poly=wrong).reshape(-1, 4)
    assert pdivmod(A, O.berlekamp_massey(bit_seq(w[:, 0], 0)))[1] != 0


@pytest.mark.parametrize("variant,M", [(0, 1), (0, 16), (1, 8), (2, 1), (2, 4), (2, 64), (3, 4), (4, 16), (6, 2),
                                       (7, 8)])
def test_library_check_poly_equals_oracle(variant, M):
    from paper_2309_16682_amd import vmt

    ctx = vmt.vmt_ctx_create(-1)
    try:
        assert vmt.vmt_check_poly(ctx, variant, M) == check_poly(variant, M)
    finally:
        vmt.vmt_ctx_destroy(ctx)
