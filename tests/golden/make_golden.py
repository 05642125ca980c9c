"""Write the polynomial fixtures under tests/golden/ using only the oracle.

    python tests/golden/make_golden.py

For each base generator (MT19937-32, MT19937-64, SFMT19937, and SFMT with the
parameter sets of Mersenne exponents 607, 1279, 2281, 4253, 11213) it computes,
with the oracle's plain GF(2) arithmetic:

  minpoly_<v>.txt   the minimal polynomial mu of the one-step map F, found by
                    Berlekamp-Massey on the raw bit sequence of a seeded state
                    (the 19937 generators), or for the other SFMT sets the lcm
                    of those of random functionals <mask, X_i> of pseudo-random
                    full states (numpy default_rng; one bit or one state may
                    miss a factor of mu).
  tpow2_<v>.txt     t^(2^q) mod mu for q = MEXP - 6 ... MEXP - 1, the lane
                    distance J = 2^(MEXP - log2 M) of Sec. 3 (Table jvalues;
                    M = 64 ... 2), plus t^(2^MEXP) mod mu, all from one chain of
                    squarings t -> t^2 -> t^4 -> ...

    python tests/golden/make_golden.py [name ...]   # e.g. sfmt607 (default: all)

The files are plain text: '#' comment lines, then 'key hex' lines where hex is
the polynomial as an integer (bit i = coefficient of t^i).
"""
from __future__ import annotations

import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import pyoracle as O  # noqa: E402

import numpy as np  # noqa: E402

NAMES = {O.MT32: "mt32", O.MT64: "mt64", O.SFMT: "sfmt", O.SFMT607: "sfmt607", O.SFMT1279: "sfmt1279",
         O.SFMT2281: "sfmt2281", O.SFMT4253: "sfmt4253", O.SFMT11213: "sfmt11213"}
SEED_STATE = {O.MT32: ("init_genrand", 5489), O.MT64: ("init_genrand", 5489), O.SFMT: ("init_genrand", 1234),
              **{v: ("default_rng", 2024) for v in (O.SFMT607, O.SFMT1279, O.SFMT2281, O.SFMT4253, O.SFMT11213)}}


def start_state(variant: int):
    kind, seed = SEED_STATE[variant]
    if kind == "init_genrand":
        return O.seed_state(variant, seed)
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2**32, O.STATE_LEN[variant], dtype=np.uint64).astype(np.uint32)


def _pmul(a: int, b: int) -> int:
    r = 0
    while b:
        low = b & -b
        r ^= a << (low.bit_length() - 1)
        b ^= low
    return r


def _pdivmod(a: int, b: int):
    q, db = 0, b.bit_length() - 1
    while a and a.bit_length() - 1 >= db:
        sh = a.bit_length() - 1 - db
        q |= 1 << sh
        a ^= b << sh
    return q, a


def map_minpoly(variant: int) -> int:
    """The 19937 generators: the minimal polynomial of bit 0 from the seeded state
    (it has the full degree: MT's mu is irreducible, SFMT19937's reaches the state
    dimension 19968). Other SFMT sets: the lcm of the minimal polynomials of
    <mask, X_i> for pseudo-random full states X_0 and masks, until 16 pairs in a
    row add nothing (one bit, or one state, may miss a factor of mu)."""
    mu = O.minpoly(variant, start_state(variant))
    if SEED_STATE[variant][0] == "init_genrand":
        return mu
    rng = np.random.default_rng(SEED_STATE[variant][1] + 1)
    quiet = 0
    while quiet < 16:
        x = rng.integers(0, 2**32, O.STATE_LEN[variant], dtype=np.uint64).astype(np.uint32)
        mask = rng.integers(0, 2**32, O.STATE_LEN[variant], dtype=np.uint64).astype(np.uint32)
        m2 = O.minpoly_masked(variant, x, mask)
        if _pdivmod(mu, m2)[1] == 0:
            quiet += 1
            continue
        mu = _pmul(mu, _pdivmod(m2, O.poly_gcd(mu, m2))[0])
        quiet = 0
    return mu


def _chain(variant: int):
    t0 = time.time()
    mu = map_minpoly(variant)
    out = {}
    cur = 2  # t
    q = 0
    mexp = O.MEXP[variant]
    for target in list(range(mexp - 6, mexp + 1)):
        cur = O.poly_sqr_chain(target - q, mu, start=cur)
        q = target
        out[q] = cur
    return variant, mu, out, time.time() - t0


def write(variant, mu, out, secs):
    name = NAMES[variant]
    kind, seed = SEED_STATE[variant]
    with open(os.path.join(HERE, f"minpoly_{name}.txt"), "w") as f:
        f.write(f"# Minimal polynomial of the one-step map of {name} (Sec. 2, eq. step / sfmt_step),\n")
        if kind == "init_genrand":
            f.write(f"# Berlekamp-Massey on bit 0 of the raw words from {kind}({seed}).\n")
        else:
            f.write(f"# lcm of Berlekamp-Massey on random functionals of states from {kind}({seed}).\n")
        f.write(f"# Written by tests/golden/make_golden.py with the oracle only.\n")
        f.write(f"degree {mu.bit_length() - 1}\n")
        f.write(f"mu {mu:x}\n")
    with open(os.path.join(HERE, f"tpow2_{name}.txt"), "w") as f:
        mexp = O.MEXP[variant]
        f.write(f"# t^(2^q) mod mu for {name}: lane distance J = 2^q of Sec. 3, Table jvalues\n")
        f.write(f"# (q = {mexp} - log2 M). Row {mexp} is t^(2^{mexp}) mod mu.\n")
        f.write(f"# Written by tests/golden/make_golden.py with the oracle only ({secs:.0f} s).\n")
        for q, p in sorted(out.items()):
            f.write(f"{q} {p:x}\n")


def main():
    O.build()
    pick = [v for v, n in NAMES.items() if len(sys.argv) < 2 or n in sys.argv[1:]]
    with mp.Pool(min(len(pick), 4)) as pool:
        for variant, mu, out, secs in pool.imap_unordered(_chain, pick):
            write(variant, mu, out, secs)
            print(NAMES[variant], "deg", mu.bit_length() - 1, f"{secs:.1f}s", flush=True)


if __name__ == "__main__":
    main()
