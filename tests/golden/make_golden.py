"""Write the polynomial fixtures under tests/golden/ using only the oracle.

    python tests/golden/make_golden.py

For each base generator (MT19937-32, MT19937-64, SFMT19937) it computes, with
the oracle's plain GF(2) arithmetic:

  minpoly_<v>.txt   the minimal polynomial mu of the one-step map F, found by
                    Berlekamp-Massey on a seeded state's raw bit sequence.
  tpow2_<v>.txt     t^(2^q) mod mu for q = 19931 ... 19936, the lane distance
                    J = 2^(19937 - log2 M) of Sec. 3 (Table jvalues; M = 64 ...
                    2), plus t^(2^19937) mod mu, all from one chain of squarings
                    t -> t^2 -> t^4 -> ...

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

NAMES = {O.MT32: "mt32", O.MT64: "mt64", O.SFMT: "sfmt"}
SEED_STATE = {O.MT32: ("init_genrand", 5489), O.MT64: ("init_genrand", 5489), O.SFMT: ("init_genrand", 1234)}
Q_LIST = list(range(19931, 19937))


def _chain(variant: int):
    t0 = time.time()
    kind, seed = SEED_STATE[variant]
    x = O.seed_state(variant, seed)
    mu = O.minpoly(variant, x)
    out = {}
    cur = 2  # t
    q = 0
    for target in Q_LIST + [19937]:
        cur = O.poly_sqr_chain(target - q, mu, start=cur)
        q = target
        out[q] = cur
    return variant, mu, out, time.time() - t0


def write(variant, mu, out, secs):
    name = NAMES[variant]
    kind, seed = SEED_STATE[variant]
    with open(os.path.join(HERE, f"minpoly_{name}.txt"), "w") as f:
        f.write(f"# Minimal polynomial of the one-step map of {name} (Sec. 2, eq. step / sfmt_step),\n")
        f.write(f"# Berlekamp-Massey on bit 0 of the raw words from {kind}({seed}).\n")
        f.write(f"# Written by tests/golden/make_golden.py with the oracle only.\n")
        f.write(f"degree {mu.bit_length() - 1}\n")
        f.write(f"mu {mu:x}\n")
    with open(os.path.join(HERE, f"tpow2_{name}.txt"), "w") as f:
        f.write(f"# t^(2^q) mod mu for {name}: lane distance J = 2^q of Sec. 3, Table jvalues\n")
        f.write(f"# (q = 19937 - log2 M). Row 19937 is t^(2^19937) mod mu.\n")
        f.write(f"# Written by tests/golden/make_golden.py with the oracle only ({secs:.0f} s).\n")
        for q, p in sorted(out.items()):
            f.write(f"{q} {p:x}\n")


def main():
    O.build()
    with mp.Pool(3) as pool:
        for variant, mu, out, secs in pool.imap_unordered(_chain, [O.MT32, O.MT64, O.SFMT]):
            write(variant, mu, out, secs)
            print(NAMES[variant], "deg", mu.bit_length() - 1, f"{secs:.1f}s", flush=True)


if __name__ == "__main__":
    main()
