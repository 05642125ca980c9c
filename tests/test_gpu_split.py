"""One stream split over many workgroups by jump-ahead: the chunks of a call
start from copies of the state jumped by c * 2^v lane steps, run in one
batched launch, and the state ends where the last chunk ends. The output and
everything generated afterwards must equal the oracle's single stream
(tolerance 0) for every variant, output kind, chunk length and start position."""
import numpy as np
import pytest

from oracle import pyoracle as O
from tests.gpu_helpers import as_u, oracle_stream, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_16682_amd import vmt  # noqa: E402

MT32, MT64, SFMT = vmt.VMT_MT32, vmt.VMT_MT64, vmt.VMT_SFMT
GEN = vmt.VMT_FAMILY_GENERATE
EPW = {MT32: 1, MT64: 1, SFMT: 4}
BLOCK = {MT32: 624, MT64: 312, SFMT: 156 * 4}
DT = {vmt.VMT_OUT_U32: torch.int32, vmt.VMT_OUT_U64: torch.int64, vmt.VMT_OUT_F32: torch.float32,
      vmt.VMT_OUT_F64: torch.float64}
CALL = {vmt.VMT_OUT_U32: vmt.vmt_generate_u32, vmt.VMT_OUT_U64: vmt.vmt_generate_u64,
        vmt.VMT_OUT_F32: vmt.vmt_uniform_f32, vmt.VMT_OUT_F64: vmt.vmt_uniform_f64}


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = vmt.vmt_ctx_create(0)
    yield c
    torch.cuda.synchronize()
    vmt.vmt_ctx_destroy(c)


def native(variant):
    return vmt.VMT_OUT_U64 if variant == MT64 else vmt.VMT_OUT_U32


def run(ctx, st, variant, kind, n):
    out = torch.zeros(max(n, 1), dtype=DT[kind], device="cuda")
    CALL[kind](ctx, st, n, out)
    torch.cuda.synchronize()
    t = out[:n].cpu()
    return as_u(t, variant) if kind in (vmt.VMT_OUT_U32, vmt.VMT_OUT_U64) else t.numpy()


def expect(variant, kind, raw):
    if kind in (vmt.VMT_OUT_U32, vmt.VMT_OUT_U64):
        return raw
    if kind == vmt.VMT_OUT_F64:
        return O.map_f64(raw)
    if variant == MT64:
        return np.array([O.u64_to_f32(int(u)) for u in raw], np.float32)
    return O.map_f32(raw)


CASES = [
    # variant, M, kind, split_log2, chunks, start position
    (MT32, 16, vmt.VMT_OUT_U32, 4, 37.3, 0),
    (MT32, 16, vmt.VMT_OUT_U32, 12, 3.5, 4321),
    (MT32, 16, vmt.VMT_OUT_F32, 6, 9.01, 9983),
    (MT32, 4, vmt.VMT_OUT_U32, 9, 5.5, 17),
    (MT32, 1, vmt.VMT_OUT_U32, 10, 4.2, 623),
    (MT64, 8, vmt.VMT_OUT_U64, 5, 20.7, 1),
    (MT64, 8, vmt.VMT_OUT_F64, 11, 3.1, 2495),
    (MT64, 16, vmt.VMT_OUT_F32, 7, 6.6, 100),
    (SFMT, 4, vmt.VMT_OUT_U32, 4, 50.2, 0),
    (SFMT, 4, vmt.VMT_OUT_F32, 10, 4.5, 2497),
    (SFMT, 64, vmt.VMT_OUT_U32, 6, 7.7, 333),
    (SFMT, 1, vmt.VMT_OUT_U32, 12, 3.3, 2),
    # more than 1024 lane jumps: the copies share each lane's raw rows, 4 / 8 / 16 copies per workgroup
    (MT32, 16, vmt.VMT_OUT_U32, 4, 100.5, 7),
    (MT32, 16, vmt.VMT_OUT_U32, 4, 600.2, 3000),
    (MT32, 1, vmt.VMT_OUT_U32, 4, 1500.5, 100),
    (MT64, 8, vmt.VMT_OUT_F64, 4, 150.3, 311),
    (MT64, 4, vmt.VMT_OUT_U64, 5, 1100.9, 2),
    (SFMT, 4, vmt.VMT_OUT_U32, 4, 300.7, 5),
    (SFMT, 64, vmt.VMT_OUT_F32, 4, 20.2, 1000),
    (SFMT, 2, vmt.VMT_OUT_U32, 4, 4200.1, 9),
    # MT copies whose lanes' blocks are split over 2 workgroups (16 copies per workgroup; 4, 8 and 16 above)
    (MT32, 16, vmt.VMT_OUT_U32, 4, 150.6, 11),
    (MT64, 8, vmt.VMT_OUT_U64, 4, 260.4, 5),
]


# MT chunks by lane groups (lanes per workgroup below M): variant, M, kind, split_log2, chunks, start, lanes per workgroup
LANE_GROUP_CASES = [
    (MT32, 16, vmt.VMT_OUT_U32, 6, 9.3, 4321, 1),
    (MT32, 16, vmt.VMT_OUT_F32, 5, 33.7, 17, 4),
    (MT32, 8, vmt.VMT_OUT_U32, 7, 12.2, 0, 2),
    (MT32, 2, vmt.VMT_OUT_U32, 9, 5.01, 623, 1),
    (MT64, 8, vmt.VMT_OUT_U64, 5, 20.7, 1, 1),
    (MT64, 8, vmt.VMT_OUT_F64, 6, 11.1, 2495, 4),
    (MT64, 16, vmt.VMT_OUT_F32, 7, 6.6, 100, 8),
    (MT32, 16, vmt.VMT_OUT_U32, 4, 100.5, 7, 2),  # more than 1024 lane jumps as well
]


@pytest.mark.parametrize("variant,M,kind,v,chunks,pre,lpw",
                         [c + (min(c[1], 16),) for c in CASES] + LANE_GROUP_CASES)
def test_split_call_equals_oracle_stream(ctx, variant, M, kind, v, chunks, pre, lpw):
    n = int(chunks * (1 << v) * M * EPW[variant])
    say(f"case split variant={variant} M={M} kind={kind} v={v} n={n} pre={pre} lanes_per_wg={lpw}")
    seed = 1000 + v
    st = vmt.new_state(variant, M)
    vmt.vmt_init_genrand(ctx, variant, seed, M, st)
    ref = oracle_stream(variant, M, seed=seed)
    if pre:
        run(ctx, st, variant, native(variant), pre)  # any start position, single launch
        ref.generate(pre)
    vmt.vmt_shape_set(ctx, GEN, variant, M, kind, lanes_per_wg=lpw, split_log2=v)
    try:
        got = run(ctx, st, variant, kind, n)
    finally:
        vmt.vmt_shape_set(ctx, GEN, variant, M, kind)
    np.testing.assert_array_equal(got, expect(variant, kind, ref.generate(n)))
    # the state continues where the split call ended
    tail = 3 * BLOCK[variant] * M + 5
    np.testing.assert_array_equal(run(ctx, st, variant, native(variant), tail), ref.generate(tail))


@pytest.mark.parametrize("variant,M,mib", [(MT32, 16, 10), (MT32, 16, 40), (MT64, 8, 10), (MT64, 8, 40), (SFMT, 4, 6),
                                           (SFMT, 64, 6), (MT32, 16, 300)])
def test_automatic_split_of_a_long_call(ctx, variant, M, mib):
    # lengths the library splits by itself (MT19937 from 8 MiB into up to 256, 512 or 1024 lane jumps by size;
    # SFMT19937 from M MiB), from a mid-block position
    n = (mib << 20) // (8 if variant == MT64 else 4) + 12345
    say(f"case auto split variant={variant} M={M} n={n}")
    seed = 77
    st = vmt.new_state(variant, M)
    vmt.vmt_init_genrand(ctx, variant, seed, M, st)
    ref = oracle_stream(variant, M, seed=seed)
    run(ctx, st, variant, native(variant), 999)
    ref.generate(999)
    got = run(ctx, st, variant, native(variant), n)
    np.testing.assert_array_equal(got, ref.generate(n))
    np.testing.assert_array_equal(run(ctx, st, variant, native(variant), 5000), ref.generate(5000))


@pytest.mark.parametrize("variant,M", [(MT32, 16), (MT64, 8)])
def test_automatic_lanes_per_workgroup(ctx, variant, M):
    # unsplit calls of 256 KiB or more run one lane per workgroup when the shape leaves it open
    assert vmt.vmt_shape_get(ctx, GEN, variant, M, native(variant)).lanes_per_wg == 0
    seed = 9
    st = vmt.new_state(variant, M)
    vmt.vmt_init_genrand(ctx, variant, seed, M, st)
    ref = oracle_stream(variant, M, seed=seed)
    for n in (1000, (300 << 10) // (8 if variant == MT64 else 4) + 3, 777):
        np.testing.assert_array_equal(run(ctx, st, variant, native(variant), n), ref.generate(n))


def test_split_setting_is_validated(ctx):
    with pytest.raises(vmt.VmtError):
        vmt.vmt_shape_set(ctx, GEN, MT32, 16, vmt.VMT_OUT_U32, lanes_per_wg=16, split_log2=2)
    vmt.vmt_shape_set(ctx, GEN, MT32, 16, vmt.VMT_OUT_U32, lanes_per_wg=16, split_log2=255)
    assert vmt.vmt_shape_get(ctx, GEN, MT32, 16, vmt.VMT_OUT_U32).split_log2 == 255
    vmt.vmt_shape_set(ctx, GEN, MT32, 16, vmt.VMT_OUT_U32)
    assert vmt.vmt_shape_get(ctx, GEN, MT32, 16, vmt.VMT_OUT_U32).split_log2 == 0


def test_split_calls_on_two_streams_with_growing_workspaces(ctx):
    # each stream has its own workspace in the context, grown as calls get larger; two states split side by side
    # on two streams must each equal their oracle stream
    M = 16
    n_small, n_large = 3 * (1 << 16) * M + 77, 9 * (1 << 16) * M + 5
    say(f"case split on two streams n={n_small},{n_large}")
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    sts, refs = [], []
    for seed in (31, 32):
        st = vmt.new_state(MT32, M)
        vmt.vmt_init_genrand(ctx, MT32, seed, M, st)
        sts.append(st)
        refs.append(oracle_stream(MT32, M, seed=seed))
    torch.cuda.synchronize()
    vmt.vmt_shape_set(ctx, GEN, MT32, M, vmt.VMT_OUT_U32, lanes_per_wg=1, split_log2=16)
    try:
        for n in (n_small, n_large, n_small):
            outs = [torch.zeros(n, dtype=torch.int32, device="cuda") for _ in streams]
            for st, out, s in zip(sts, outs, streams):
                vmt.vmt_generate_u32(ctx, st, n, out, stream=s.cuda_stream)
            torch.cuda.synchronize()
            for out, ref in zip(outs, refs):
                np.testing.assert_array_equal(as_u(out.cpu(), MT32), ref.generate(n))
    finally:
        vmt.vmt_shape_set(ctx, GEN, MT32, M, vmt.VMT_OUT_U32)


def test_split_calls_from_two_host_threads_on_one_stream(ctx):
    # two host threads issue split calls for their own states on one stream: the stream's workspace serves both,
    # one call at a time, and each state's outputs equal its oracle stream call after call
    import threading

    M, calls = 16, 4
    n = 3 * (1 << 16) * M + 7
    say(f"case split from two threads n={n} calls={calls}")
    stream = torch.cuda.Stream()
    sts, outs = [], []
    for seed in (41, 42):
        st = vmt.new_state(MT32, M)
        vmt.vmt_init_genrand(ctx, MT32, seed, M, st)
        sts.append(st)
        outs.append([torch.zeros(n, dtype=torch.int32, device="cuda") for _ in range(calls)])
    torch.cuda.synchronize()
    vmt.vmt_shape_set(ctx, GEN, MT32, M, vmt.VMT_OUT_U32, lanes_per_wg=1, split_log2=16)
    errors = []

    def work(i):
        try:
            for out in outs[i]:
                vmt.vmt_generate_u32(ctx, sts[i], n, out, stream=stream.cuda_stream)
        except Exception as exc:  # reported by the main thread
            errors.append(exc)

    try:
        threads = [threading.Thread(target=work, args=(i,)) for i in range(2)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        torch.cuda.synchronize()
    finally:
        vmt.vmt_shape_set(ctx, GEN, MT32, M, vmt.VMT_OUT_U32)
    assert not errors, errors
    for i, seed in enumerate((41, 42)):
        ref = oracle_stream(MT32, M, seed=seed)
        for out in outs[i]:
            np.testing.assert_array_equal(as_u(out.cpu(), MT32), ref.generate(n))
