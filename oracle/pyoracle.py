"""ctypes wrapper around the scalar oracle (oracle/vmt_oracle.c).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg import this module; the product package never does.

Polynomials cross this wrapper as Python ints (bit i = coefficient of t^i).
States cross as numpy arrays in canonical order (oldest word first):
uint32[624] for MT19937-32, uint64[312] for MT19937-64, uint32[624] for
SFMT19937 (156 words of four sub-words, sub-word 0 least significant).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
OR_PW = 640

MT32, MT64, SFMT = 0, 1, 2
# SFMT with the other published parameter sets (same recurrence, Mersenne exponent in the name)
SFMT607, SFMT1279, SFMT2281, SFMT4253, SFMT11213 = 3, 4, 5, 6, 7
SFMT_FAMILY = (SFMT, SFMT607, SFMT1279, SFMT2281, SFMT4253, SFMT11213)
MEXP = {MT32: 19937, MT64: 19937, SFMT: 19937, SFMT607: 607, SFMT1279: 1279, SFMT2281: 2281, SFMT4253: 4253,
        SFMT11213: 11213}
STATE_WORDS = {MT32: 624, MT64: 312, **{v: MEXP[v] // 128 + 1 for v in SFMT_FAMILY}}
STATE_DTYPE = {MT32: np.uint32, MT64: np.uint64, **{v: np.uint32 for v in SFMT_FAMILY}}
STATE_LEN = {MT32: 624, MT64: 312, **{v: 4 * STATE_WORDS[v] for v in SFMT_FAMILY}}  # numpy elements per state
OUT_DTYPE = {MT32: np.uint32, MT64: np.uint64, **{v: np.uint32 for v in SFMT_FAMILY}}


def is_sfmt(variant: int) -> bool:
    return variant in SFMT_FAMILY


def build(force: bool = False) -> str:
    """Compile the oracle with the system C compiler (plain -O2, no intrinsics)."""
    src = os.path.join(HERE, "vmt_oracle.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < max(
        os.path.getmtime(src), os.path.getmtime(os.path.join(HERE, "vmt_oracle.h"))
    ):
        tmp = LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, src]
        )
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.or_state_words.argtypes = [ctypes.c_int]
        L.or_word_bytes.argtypes = [ctypes.c_int]
        L.or_mt32_init_genrand.argtypes = [P, ctypes.c_uint32]
        L.or_mt32_init_by_array.argtypes = [P, P, ctypes.c_int]
        L.or_mt64_init_genrand.argtypes = [P, ctypes.c_uint64]
        L.or_sfmt_init_genrand.argtypes = [P, ctypes.c_uint32]
        L.or_sfmt_init_genrand.restype = ctypes.c_int
        L.or_sfmt_init.argtypes = [ctypes.c_int, P, ctypes.c_uint32]
        L.or_sfmt_init.restype = ctypes.c_int
        L.or_sfmt_parity.argtypes = [ctypes.c_int, P]
        L.or_mexp.argtypes = [ctypes.c_int]
        L.or_mexp.restype = ctypes.c_int
        L.or_mt32_temper.argtypes = [ctypes.c_uint32]
        L.or_mt32_temper.restype = ctypes.c_uint32
        L.or_mt64_temper.argtypes = [ctypes.c_uint64]
        L.or_mt64_temper.restype = ctypes.c_uint64
        L.or_step.argtypes = [ctypes.c_int, P, ctypes.POINTER(ctypes.c_int), P, ctypes.c_size_t, ctypes.c_int]
        L.or_canon.argtypes = [ctypes.c_int, P, ctypes.c_int, P]
        L.or_poly_deg.argtypes = [P]
        L.or_poly_mod.argtypes = [P, P]
        L.or_poly_mulmod.argtypes = [P, P, P, P]
        L.or_poly_sqrmod.argtypes = [P, P, P]
        L.or_poly_sqr_chain.argtypes = [P, P, ctypes.c_uint64, P]
        L.or_poly_powmod_t.argtypes = [P, P, ctypes.c_int, P]
        L.or_poly_gcd.argtypes = [P, P, P]
        L.or_berlekamp_massey.argtypes = [P, ctypes.c_size_t, P, ctypes.c_size_t]
        L.or_berlekamp_massey.restype = ctypes.c_int
        L.or_minpoly_masked.argtypes = [ctypes.c_int, P, P, P]
        L.or_minpoly_masked.restype = ctypes.c_int
        L.or_minpoly.argtypes = [ctypes.c_int, P, P]
        L.or_minpoly.restype = ctypes.c_int
        L.or_jump.argtypes = [ctypes.c_int, P, P]
        L.or_vgen_new.argtypes = [ctypes.c_int, ctypes.c_int, P, P]
        L.or_vgen_new.restype = P
        L.or_vgen_free.argtypes = [P]
        L.or_vgen_generate.argtypes = [P, P, ctypes.c_size_t]
        L.or_vgen_jump.argtypes = [P, P]
        L.or_vgen_pos.argtypes = [P]
        L.or_vgen_pos.restype = ctypes.c_uint64
        L.or_vgen_lane_canon.argtypes = [P, ctypes.c_int, P]
        L.or_map_f32.argtypes = [P, P, ctypes.c_size_t]
        L.or_map_f64.argtypes = [P, P, ctypes.c_size_t]
        L.or_u32pair_to_f64.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.or_u32pair_to_f64.restype = ctypes.c_double
        L.or_u64_to_f32.argtypes = [ctypes.c_uint64]
        L.or_u64_to_f32.restype = ctypes.c_float
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


# ---- polynomials ---------------------------------------------------------


def poly_to_words(p: int) -> np.ndarray:
    assert p >= 0 and p.bit_length() <= OR_PW * 64
    b = p.to_bytes(OR_PW * 8, "little")
    return np.frombuffer(b, dtype=np.uint64).copy()


def words_to_poly(w: np.ndarray) -> int:
    return int.from_bytes(np.ascontiguousarray(w, dtype=np.uint64).tobytes(), "little")


def poly_mod(a: int, mu: int) -> int:
    w = poly_to_words(a)
    lib().or_poly_mod(_ptr(w), _ptr(poly_to_words(mu)))
    return words_to_poly(w)


def poly_mulmod(a: int, b: int, mu: int) -> int:
    r = np.zeros(OR_PW, np.uint64)
    lib().or_poly_mulmod(_ptr(r), _ptr(poly_to_words(a)), _ptr(poly_to_words(b)), _ptr(poly_to_words(mu)))
    return words_to_poly(r)


def poly_sqrmod(a: int, mu: int) -> int:
    r = np.zeros(OR_PW, np.uint64)
    lib().or_poly_sqrmod(_ptr(r), _ptr(poly_to_words(a)), _ptr(poly_to_words(mu)))
    return words_to_poly(r)


def poly_sqr_chain(k: int, mu: int, start: int | None = None) -> int:
    """t^(2^k) mod mu (or start^(2^k) mod mu)."""
    r = np.zeros(OR_PW, np.uint64)
    s = poly_to_words(start) if start is not None else None
    lib().or_poly_sqr_chain(_ptr(r), _ptr(s) if s is not None else None, k, _ptr(poly_to_words(mu)))
    return words_to_poly(r)


def poly_powmod_t(e: int, mu: int) -> int:
    """t^e mod mu."""
    nw = max(1, (e.bit_length() + 63) // 64)
    ew = np.frombuffer(e.to_bytes(nw * 8, "little"), dtype=np.uint64).copy()
    r = np.zeros(OR_PW, np.uint64)
    lib().or_poly_powmod_t(_ptr(r), _ptr(ew), nw, _ptr(poly_to_words(mu)))
    return words_to_poly(r)


def poly_gcd(a: int, b: int) -> int:
    r = np.zeros(OR_PW, np.uint64)
    lib().or_poly_gcd(_ptr(r), _ptr(poly_to_words(a)), _ptr(poly_to_words(b)))
    return words_to_poly(r)


def berlekamp_massey(bits: np.ndarray) -> int:
    """Minimal polynomial (characteristic orientation) of a bit sequence; its
    degree is the sequence's linear complexity. bits: one bit per element."""
    s = np.ascontiguousarray(np.asarray(bits) & 1, dtype=np.uint8)
    pw = s.size // 64 + 2
    poly = np.zeros(pw, np.uint64)
    L = lib().or_berlekamp_massey(_ptr(s), s.size, _ptr(poly), pw)
    assert L >= 0
    return words_to_poly(poly)


def minpoly(variant: int, canon: np.ndarray) -> int:
    mu = np.zeros(OR_PW, np.uint64)
    c = np.ascontiguousarray(canon, dtype=STATE_DTYPE[variant])
    lib().or_minpoly(variant, _ptr(c), _ptr(mu))
    return words_to_poly(mu)


def minpoly_masked(variant: int, canon: np.ndarray, mask: np.ndarray) -> int:
    """Minimal polynomial of the sequence <mask, X_i> (mask: the state's layout as uint32)."""
    mu = np.zeros(OR_PW, np.uint64)
    c = np.ascontiguousarray(canon, dtype=STATE_DTYPE[variant])
    m = np.ascontiguousarray(mask, dtype=np.uint32)
    assert m.nbytes == c.nbytes
    lib().or_minpoly_masked(variant, _ptr(c), _ptr(m), _ptr(mu))
    return words_to_poly(mu)


# ---- seeding ----------------------------------------------------------------


def seed_state(variant: int, seed: int | None = None, key=None) -> np.ndarray:
    """Canonical seeded state. MT32 supports init_genrand(seed) and
    init_by_array(key); MT64 and SFMT support init_genrand(seed)."""
    x = np.zeros(STATE_LEN[variant], STATE_DTYPE[variant])
    if key is not None:
        assert variant == MT32
        k = np.ascontiguousarray(key, dtype=np.uint32)
        lib().or_mt32_init_by_array(_ptr(x), _ptr(k), len(k))
    elif variant == MT32:
        lib().or_mt32_init_genrand(_ptr(x), seed)
    elif variant == MT64:
        lib().or_mt64_init_genrand(_ptr(x), seed)
    else:
        lib().or_sfmt_init(variant, _ptr(x), seed)
    return x


def sfmt_certification_flipped(seed: int, variant: int = SFMT) -> bool:
    x = np.zeros(STATE_LEN[variant], np.uint32)
    return bool(lib().or_sfmt_init(variant, _ptr(x), seed))


def sfmt_parity(variant: int) -> np.ndarray:
    p = np.zeros(4, np.uint32)
    lib().or_sfmt_parity(variant, _ptr(p))
    return p


# ---- scalar generators ----------------------------------------------------


class Scalar:
    """One base generator on a circular buffer (eq. staterec / stepmod)."""

    def __init__(self, variant: int, canon: np.ndarray):
        self.variant = variant
        self.buf = np.ascontiguousarray(canon, dtype=STATE_DTYPE[variant]).copy()
        self.k = ctypes.c_int(0)

    def _run(self, count: int, temper: int) -> np.ndarray:
        shape = (count, 4) if is_sfmt(self.variant) else (count,)
        out = np.zeros(shape, OUT_DTYPE[self.variant])
        lib().or_step(self.variant, _ptr(self.buf), ctypes.byref(self.k), _ptr(out), count, temper)
        return out

    def raw(self, count: int) -> np.ndarray:
        return self._run(count, 0)

    def out(self, count: int) -> np.ndarray:
        """Tempered outputs (SFMT: the new words, shape (count, 4))."""
        return self._run(count, 1)

    def skip(self, count: int) -> None:
        lib().or_step(self.variant, _ptr(self.buf), ctypes.byref(self.k), None, count, 0)

    def canon(self) -> np.ndarray:
        c = np.zeros_like(self.buf)
        lib().or_canon(self.variant, _ptr(self.buf), self.k.value, _ptr(c))
        return c

    def jump(self, g: int) -> None:
        c = self.canon()
        lib().or_jump(self.variant, _ptr(c), _ptr(poly_to_words(g)))
        self.buf = c
        self.k = ctypes.c_int(0)


def jump_canon(variant: int, canon: np.ndarray, g: int) -> np.ndarray:
    c = np.ascontiguousarray(canon, dtype=STATE_DTYPE[variant]).copy()
    lib().or_jump(variant, _ptr(c), _ptr(poly_to_words(g)))
    return c


# ---- V-stream -------------------------------------------------------------------


class VStream:
    """The interleaved V-stream of Sec. 3: lane t = base stream advanced by t*J."""

    def __init__(self, variant: int, M: int, canon0: np.ndarray, gJ: int):
        self.variant, self.M = variant, M
        c = np.ascontiguousarray(canon0, dtype=STATE_DTYPE[variant])
        self._h = lib().or_vgen_new(variant, M, _ptr(c), _ptr(poly_to_words(gJ)))

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_vgen_free(self._h)
            self._h = None

    def generate(self, count: int) -> np.ndarray:
        out = np.zeros(count, OUT_DTYPE[self.variant])
        if count:
            lib().or_vgen_generate(self._h, _ptr(out), count)
        return out

    def jump(self, g: int) -> None:
        lib().or_vgen_jump(self._h, _ptr(poly_to_words(g)))

    @property
    def pos(self) -> int:
        return int(lib().or_vgen_pos(self._h))

    def lane_canon(self, t: int) -> np.ndarray:
        c = np.zeros(STATE_LEN[self.variant], STATE_DTYPE[self.variant])
        lib().or_vgen_lane_canon(self._h, t, _ptr(c))
        return c


# ---- maps -------------------------------------------------------------------------


def map_f32(u: np.ndarray) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.uint32)
    f = np.zeros(u.shape, np.float32)
    lib().or_map_f32(_ptr(u), _ptr(f), u.size)
    return f


def map_f64(u: np.ndarray) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.uint64)
    f = np.zeros(u.shape, np.float64)
    lib().or_map_f64(_ptr(u), _ptr(f), u.size)
    return f


def u32pair_to_f64(a: int, b: int) -> float:
    return float(lib().or_u32pair_to_f64(a, b))


def u64_to_f32(u: int) -> float:
    return float(lib().or_u64_to_f32(u))
