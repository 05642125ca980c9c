"""Recurrence polynomials of the V-stream's bits, from the oracle's fixtures
(test infrastructure: plain Python integer arithmetic over GF(2)).

MT19937-32/-64: every bit of the V-stream obeys mu, the base minimal
polynomial. SFMT (any parameter set): mu = phi psi with phi = gcd(mu,
t^(2^MEXP) - t); the bits of the sequence of 128-bit words obey
phi(t) psi(t^M) = phi psi^M.
"""
from oracle import pyoracle as O
from tests import golden_io

D = 19937


def pdivmod(a: int, b: int):
    q, db = 0, b.bit_length() - 1
    while a and a.bit_length() - 1 >= db:
        sh = a.bit_length() - 1 - db
        q |= 1 << sh
        a ^= b << sh
    return q, a


def pmul(a: int, b: int) -> int:
    r = 0
    while b:
        low = b & -b
        r ^= a << (low.bit_length() - 1)
        b ^= low
    return r


def sfmt_factors(variant: int = O.SFMT):
    """phi = gcd(mu, t^(2^MEXP) - t) and psi = mu / phi from the fixtures (phi
    collects the factors whose roots alpha satisfy alpha^(2^MEXP) = alpha)."""
    mu = golden_io.minpoly(variant)
    frob = golden_io.tpow2(variant)[O.MEXP[variant]]  # t^(2^MEXP) mod mu
    phi = O.poly_gcd(mu, frob ^ 2)
    psi, rem = pdivmod(mu, phi)
    assert rem == 0
    return mu, phi, psi


def check_poly(variant: int, M: int) -> int:
    if not O.is_sfmt(variant):
        return golden_io.minpoly(variant)
    mu, phi, psi = sfmt_factors(variant)
    psiM = psi
    for _ in range(M.bit_length() - 1):
        psiM = pmul(psiM, psiM)  # psi(t)^2 = psi(t^2) over GF(2)
    return pmul(phi, psiM)
