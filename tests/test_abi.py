"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and its host-side polynomial helpers agree with the oracle's fixtures."""
import ctypes
import os
import re

import pytest

from tests import golden_io

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "vmt.h")).read()
    return sorted(set(re.findall(r"\b(vmt_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2309_16682_amd import vmt

    lib = vmt.lib()
    names = declared_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    assert set(vmt.exported_symbols()) == set(names)


def test_every_declaration_cites_its_passage():
    # each declaration's comment names the passage of the paper that defines
    # the operation, or says that the paper is silent on it
    text = open(os.path.join(ROOT, "include", "vmt.h")).read()
    lines = text.split("\n")
    for name in declared_functions():
        k = next(i for i, l in enumerate(lines) if re.match(r"^[a-z].*\b" + name + r"\s*\(", l))
        end = max(i for i in range(k) if "*/" in lines[i])
        start = max(i for i in range(end + 1) if lines[i].lstrip().startswith("/*"))
        block = " ".join(lines[start : end + 1])
        assert "Cite:" in block, name
        cite = block[block.index("Cite:"):]
        assert re.search(r"Sec\. \d|eq\. \(|paper silent|as vmt_|callers that cannot allocate", cite), name


def test_host_only_context_and_error_paths():
    from paper_2309_16682_amd import vmt

    ctx = vmt.vmt_ctx_create(-1)
    try:
        assert vmt.vmt_state_bytes(vmt.VMT_MT32, 16) == 256 + 624 * 16 * 4
        assert vmt.vmt_state_bytes(vmt.VMT_MT64, 8) == 256 + 312 * 8 * 8
        assert vmt.vmt_state_bytes(vmt.VMT_SFMT, 64) == 256 + 156 * 64 * 16
        assert vmt.vmt_state_bytes(vmt.VMT_MT32, 3) == 0
        assert vmt.vmt_state_bytes(vmt.VMT_SFMT607, 4) == 256 + 5 * 4 * 16
        assert vmt.vmt_state_bytes(vmt.VMT_SFMT11213, 64) == 256 + 88 * 64 * 16
        assert vmt.vmt_state_bytes(8, 4) == 0
        # device calls on a host-only context fail cleanly
        r = vmt.lib().vmt_init_genrand(ctx, 0, 1, 4, ctypes.c_void_p(256), None)
        assert r == vmt.VMT_EDEVICE
        assert b"host-only" in vmt.lib().vmt_last_error()
        # a server needs states, an arena and a device; the server calls reject null handles
        st = ctypes.c_int(0)
        assert not vmt.lib().vmt_server_create(ctx, None, 0, None, 0, 0, 0, 1, 0, 0, ctypes.byref(st))
        assert st.value == vmt.VMT_EINVAL
        two = (ctypes.c_void_p * 2)(256, 512)
        assert not vmt.lib().vmt_server_create(ctx, two, 2, ctypes.c_void_p(4096), 4096, 4096, 0, 1, 0, 0,
                                               ctypes.byref(st))
        assert st.value == vmt.VMT_EDEVICE
        assert vmt.lib().vmt_server_set_watchdog(None, 1.0) == vmt.VMT_EINVAL
        assert vmt.lib().vmt_server_destroy(None) == vmt.VMT_EINVAL
    finally:
        vmt.vmt_ctx_destroy(ctx)


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6, 7])
def test_library_minpoly_equals_oracle_fixture(variant):
    from paper_2309_16682_amd import vmt

    ctx = vmt.vmt_ctx_create(-1)
    try:
        assert vmt.vmt_minpoly(ctx, variant) == golden_io.minpoly(variant)
    finally:
        vmt.vmt_ctx_destroy(ctx)


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6, 7])
def test_library_lane_polynomials_equal_oracle_fixtures(variant):
    from paper_2309_16682_amd import vmt

    ctx = vmt.vmt_ctx_create(-1)
    try:
        rows = golden_io.tpow2(variant)
        mexp = golden_io.MEXP[variant]
        for q in (mexp - 6, mexp - 3, mexp - 1, mexp):
            assert vmt.vmt_jump_poly(ctx, variant, 1 << q) == rows[q]
    finally:
        vmt.vmt_ctx_destroy(ctx)


def test_library_jump_poly_small_distances_match_oracle():
    from oracle import pyoracle as O
    from paper_2309_16682_amd import vmt

    ctx = vmt.vmt_ctx_create(-1)
    try:
        for variant in (0, 1, 2, 3, 7):
            mu = golden_io.minpoly(variant)
            for d in (0, 1, 19936, 19937, 19968, 40000, 2**64 + 3, 3**50):
                assert vmt.vmt_jump_poly(ctx, variant, d) == O.poly_powmod_t(d, mu), (variant, d)
    finally:
        vmt.vmt_ctx_destroy(ctx)


def test_library_jump_poly_lane_distances_match_oracle_fixtures():
    # the general distance path at the sizes of real jumps: J + d for the lane distance J = 2^(MEXP - 4) of M = 16
    # (square-and-multiply over ~20k bits in the library) against the oracle's stored t^J times t^d
    from oracle import pyoracle as O
    from paper_2309_16682_amd import vmt

    ctx = vmt.vmt_ctx_create(-1)
    try:
        for variant, d in ((0, 12345), (1, 7), (2, 99999), (7, 3)):
            mu = golden_io.minpoly(variant)
            J = 1 << (golden_io.MEXP[variant] - 4)
            ref = O.poly_mulmod(golden_io.lane_poly(variant, 16), O.poly_powmod_t(d, mu), mu)
            assert vmt.vmt_jump_poly(ctx, variant, J + d) == ref, variant
    finally:
        vmt.vmt_ctx_destroy(ctx)


def test_calls_on_several_states_reject_a_state_given_twice():
    # two workgroups seeding, jumping or serving one window in place at once would race: every call that
    # takes a list of states rejects a repeated pointer before it touches the device
    from paper_2309_16682_amd import vmt

    L = vmt.lib()
    ctx = vmt.vmt_ctx_create(-1)
    try:
        dup = (ctypes.c_void_p * 3)(256, 512, 256)
        keys = (ctypes.c_uint32 * 12)(*range(12))
        ks = (ctypes.c_uint32 * 3)(40, 41, 42)
        lens = (ctypes.c_uint64 * 3)(1, 1, 1)
        outs = (ctypes.c_void_p * 3)(4096, 8192, 12288)
        assert L.vmt_init_by_array_batch(ctx, keys, 4, 3, 16, dup, None) == vmt.VMT_EINVAL
        assert b"twice" in L.vmt_last_error()
        assert L.vmt_jump_pow2_batch(ctx, dup, ks, 3, None) == vmt.VMT_EINVAL
        assert b"twice" in L.vmt_last_error()
        seeds = (ctypes.c_uint64 * 3)(1, 2, 3)
        assert L.vmt_init_genrand_batch(ctx, 1, seeds, 3, 8, dup, None) == vmt.VMT_EINVAL
        assert b"twice" in L.vmt_last_error()
        st = ctypes.c_int(0)
        assert not L.vmt_server_create(ctx, dup, 3, ctypes.c_void_p(4096), 4096, 4096, 0, 1, 0, 0, ctypes.byref(st))
        assert st.value == vmt.VMT_EINVAL and b"twice" in L.vmt_last_error()
        # the same lists without the repeat get as far as the device check
        ok = (ctypes.c_void_p * 3)(256, 512, 768)
        assert L.vmt_init_by_array_batch(ctx, keys, 4, 3, 16, ok, None) == vmt.VMT_EDEVICE
        assert L.vmt_jump_pow2_batch(ctx, ok, ks, 3, None) == vmt.VMT_EDEVICE
        assert L.vmt_init_genrand_batch(ctx, 1, seeds, 3, 8, ok, None) == vmt.VMT_EDEVICE
        assert L.vmt_init_genrand_batch(ctx, 8, seeds, 3, 8, ok, None) == vmt.VMT_EINVAL
        # vmt_batch_generate checks registration first; unknown states are a state error, never a race
        assert L.vmt_batch_generate(ctx, dup, lens, outs, 3, 0, None) in (vmt.VMT_EDEVICE, vmt.VMT_ESTATE)
    finally:
        vmt.vmt_ctx_destroy(ctx)


def test_noalloc_batch_rejects_oversized_calls_before_the_device():
    # the allocation-free batch call holds its task list in a fixed scratch array: a larger call is an argument
    # error, reported before anything is enqueued (here on a host-only context, whose device calls fail otherwise)
    from paper_2309_16682_amd import vmt

    L = vmt.lib()
    ctx = vmt.vmt_ctx_create(-1)
    try:
        G = vmt.VMT_NOALLOC_MAX_TASKS + 1
        sp = (ctypes.c_void_p * G)(*[256 * (i + 1) for i in range(G)])
        lens = (ctypes.c_uint64 * G)(*([1] * G))
        assert L.vmt_batch_generate_noalloc(ctx, sp, lens, sp, G, 0, None) == vmt.VMT_EINVAL
        assert b"at most 32768" in L.vmt_last_error()
        assert L.vmt_batch_generate_noalloc(ctx, sp, lens, sp, 3, 0, None) == vmt.VMT_EDEVICE
        assert L.vmt_batch_generate_noalloc(None, sp, lens, sp, 3, 0, None) == vmt.VMT_EINVAL
    finally:
        vmt.vmt_ctx_destroy(ctx)
