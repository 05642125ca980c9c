"""V-SFMT with the other published parameter sets (Mersenne exponents 607,
1279, 2281, 4253, 11213) on the GPU: the same kernels, instantiated per set,
against the oracle (tolerance 0) -- seeding with period certification and
lane de-phasing by J = 2^(MEXP - log2 M), generation in one call and in
chunks, float maps, jumps from every position class, 2^k jumps, batched
generation, lanes split over workgroups, splitting one call by jump-ahead, and
the linear-complexity check."""
import numpy as np
import pytest

from oracle import pyoracle as O
from tests import golden_io
from tests.gpu_helpers import as_u, oracle_prefix, oracle_stream, pow2_poly, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_16682_amd import vmt  # noqa: E402

SETS = [vmt.VMT_SFMT607, vmt.VMT_SFMT1279, vmt.VMT_SFMT2281, vmt.VMT_SFMT4253, vmt.VMT_SFMT11213]
U32, F32 = vmt.VMT_OUT_U32, vmt.VMT_OUT_F32


def block(variant, M):
    return 4 * vmt.STATE_WORDS[variant] * M  # uint32 elements per block


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = vmt.vmt_ctx_create(0)
    yield c
    torch.cuda.synchronize()
    vmt.vmt_ctx_destroy(c)


def new_init(ctx, variant, M, seed):
    st = vmt.new_state(variant, M)
    vmt.vmt_init_genrand(ctx, variant, seed, M, st)
    return st


def gen(ctx, st, variant, n, kind=U32):
    out = torch.empty(max(n, 1), dtype=torch.int32 if kind == U32 else torch.float32, device="cuda")
    (vmt.vmt_generate_u32 if kind == U32 else vmt.vmt_uniform_f32)(ctx, st, n, out)
    torch.cuda.synchronize()
    return as_u(out[:n].cpu(), variant) if kind == U32 else out[:n].cpu().numpy()


@pytest.mark.parametrize("variant", SETS)
@pytest.mark.parametrize("M", [1, 4, 16, 64])
def test_init_and_generate_matches_oracle(ctx, variant, M):
    n = 3 * block(variant, M) + 7
    say(f"case sfmt-set init+generate variant={variant} M={M} n={n}")
    st = new_init(ctx, variant, M, 1234)
    np.testing.assert_array_equal(gen(ctx, st, variant, n), oracle_prefix(variant, M, 1234, n))


@pytest.mark.parametrize("variant", SETS)
def test_chunked_calls_and_floats(ctx, variant):
    M = 4
    B = block(variant, M)
    rng = np.random.default_rng(5)
    sizes = [0, 1, 3, B - 5, B, B + 1, 2 * B + 3, 17] + [int(x) for x in rng.integers(1, 3 * B, 5)]
    say(f"case sfmt-set chunked variant={variant} sizes={sizes}")
    st = new_init(ctx, variant, M, 99)
    got = np.concatenate([gen(ctx, st, variant, s) for s in sizes])
    np.testing.assert_array_equal(got, oracle_prefix(variant, M, 99, len(got)))
    f = gen(ctx, new_init(ctx, variant, M, 99), variant, 2 * B + 11, kind=F32)
    np.testing.assert_array_equal(f, O.map_f32(oracle_prefix(variant, M, 99, 2 * B + 11)))


@pytest.mark.parametrize("variant", SETS)
@pytest.mark.parametrize("M,first", [(4, 0), (4, 1), (4, 13), (4, "block"), (64, 13)])
def test_jump_matches_oracle(ctx, variant, M, first):
    mu = golden_io.minpoly(variant)
    B = block(variant, M)
    first = B if first == "block" else first
    for d in (1, 5, 1000, 123457):
        say(f"case sfmt-set jump variant={variant} M={M} first={first} d={d}")
        st = new_init(ctx, variant, M, 2024)
        ref = oracle_stream(variant, M, seed=2024)
        np.testing.assert_array_equal(gen(ctx, st, variant, first), ref.generate(first))
        vmt.vmt_jump(ctx, st, d)
        ref.jump(O.poly_powmod_t(d, mu))
        np.testing.assert_array_equal(gen(ctx, st, variant, 2 * B + 9), ref.generate(2 * B + 9))


@pytest.mark.parametrize("variant", SETS)
def test_jump_pow2(ctx, variant):
    M = 16
    say(f"case sfmt-set jump_pow2 variant={variant}")
    st = new_init(ctx, variant, M, 77)
    ref = oracle_stream(variant, M, seed=77)
    gen(ctx, st, variant, 101)
    ref.generate(101)
    for k in (0, 1, 32, 100, 256):
        vmt.vmt_jump_pow2(ctx, st, k)
        ref.jump(pow2_poly(variant, k))
        np.testing.assert_array_equal(gen(ctx, st, variant, 777), ref.generate(777))


@pytest.mark.parametrize("variant", SETS)
def test_batch_generate_and_split(ctx, variant):
    M = 4
    B = block(variant, M)
    rng = np.random.default_rng(3)
    count = 24
    lens = [0, 1, B - 1, B, B + 1] + [int(x) for x in rng.integers(1, 6 * B, count - 5)]
    say(f"case sfmt-set batch variant={variant}")
    seeds = list(range(3000, 3000 + count))
    states = [new_init(ctx, variant, M, s) for s in seeds]
    outs = [torch.empty(max(n, 1), dtype=torch.int32, device="cuda") for n in lens]
    refs = [oracle_stream(variant, M, seed=s) for s in seeds]
    for rep in range(2):
        vmt.vmt_batch_generate(ctx, states, lens, outs, U32)
        torch.cuda.synchronize()
        for i in range(count):
            np.testing.assert_array_equal(as_u(outs[i][: lens[i]].cpu(), variant), refs[i].generate(lens[i]),
                                          err_msg=f"rep {rep} task {i}")
    # one call split by jump-ahead into chunks of 2^6 or 2^4 lane steps (many chunks; the last call makes more than
    # 1024 lane jumps), then lanes 2 per workgroup
    for shape in ({"split_log2": 6, "lanes_per_wg": 4}, {"split_log2": 4, "lanes_per_wg": 4},
                  {"split_log2": 255, "lanes_per_wg": 2}):
        say(f"case sfmt-set split variant={variant} shape={shape}")
        vmt.vmt_shape_set(ctx, vmt.VMT_FAMILY_GENERATE, variant, M, U32, **shape)
        try:
            st = new_init(ctx, variant, M, 31)
            sizes = [5, 40 * B + 3, 7, 3 * B, 80001]
            got = np.concatenate([gen(ctx, st, variant, s) for s in sizes])
            np.testing.assert_array_equal(got, oracle_prefix(variant, M, 31, len(got)))
        finally:
            vmt.vmt_shape_set(ctx, vmt.VMT_FAMILY_GENERATE, variant, M, U32)


@pytest.mark.parametrize("variant", SETS)
def test_linear_complexity_check(ctx, variant):
    from tests.linear_ref import check_poly

    M = 8
    deg = check_poly(variant, M).bit_length() - 1
    n = 4 * deg + 200_003
    say(f"case sfmt-set check variant={variant} n={n}")
    st = new_init(ctx, variant, M, 1234)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    vmt.vmt_generate_u32(ctx, st, n, out)
    cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    vmt.vmt_check_stream(ctx, variant, M, U32, out, n, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0
    assert vmt.vmt_check_poly(ctx, variant, M) == check_poly(variant, M)


def test_state_sizes_and_export(ctx):
    for v in SETS:
        st = new_init(ctx, v, 4, 1)
        h = vmt.header(st.cpu().numpy())
        assert (h["variant"], h["n"], h["word_bytes"], h["block"]) == (v, vmt.STATE_WORDS[v], 16, block(v, 4))
        assert h["n"] == golden_io.MEXP[v] // 128 + 1
