"""Readers for the fixtures under tests/golden/ (written by make_golden.py)."""
import functools
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
NAMES = {0: "mt32", 1: "mt64", 2: "sfmt", 3: "sfmt607", 4: "sfmt1279", 5: "sfmt2281", 6: "sfmt4253", 7: "sfmt11213"}
MEXP = {0: 19937, 1: 19937, 2: 19937, 3: 607, 4: 1279, 5: 2281, 6: 4253, 7: 11213}


@functools.lru_cache(maxsize=None)
def minpoly(variant: int) -> int:
    with open(os.path.join(GOLDEN, f"minpoly_{NAMES[variant]}.txt")) as f:
        for line in f:
            if line.startswith("mu "):
                return int(line.split()[1], 16)
    raise ValueError("no mu line")


@functools.lru_cache(maxsize=None)
def tpow2(variant: int) -> dict:
    """{q: t^(2^q) mod mu} for q = MEXP - 6 .. MEXP."""
    out = {}
    with open(os.path.join(GOLDEN, f"tpow2_{NAMES[variant]}.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            out[int(k)] = int(v, 16)
    return out


def lane_poly(variant: int, M: int) -> int:
    """t^J mod mu with J = 2^(MEXP - log2 M), Sec. 3 (Table jvalues)."""
    if M == 1:
        return 1
    q = MEXP[variant] - (M.bit_length() - 1)
    return tpow2(variant)[q]
