"""The linear-complexity self-check on the GPU (vmt_check_stream).

Every bit of a generated V-stream obeys the recurrence of the polynomial the
oracle's Berlekamp-Massey finds (tests/test_oracle_linear.py): mu for
MT19937-32/-64, phi(t) psi(t^M) over 128-bit words for SFMT19937. The check
kernel must report 0 failing offsets on intact streams of every variant and
output kind (at the smallest checkable length, ragged lengths, from the middle
of a stream, from batched generation, at full size), exactly the number the
oracle's polynomial predicts for a single flipped bit, and almost every offset
for a V-stream assembled with the wrong lane spacing.
"""
import numpy as np
import pytest

from tests.gpu_helpers import say
from tests.linear_ref import check_poly

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_16682_amd import vmt  # noqa: E402

MT32, MT64, SFMT = vmt.VMT_MT32, vmt.VMT_MT64, vmt.VMT_SFMT
U32, U64, F32, F64 = vmt.VMT_OUT_U32, vmt.VMT_OUT_U64, vmt.VMT_OUT_F32, vmt.VMT_OUT_F64
DT = {U32: torch.int32, U64: torch.int64, F32: torch.float32, F64: torch.float64}
WPE = {U32: 1, F32: 1, U64: 2, F64: 2}  # 32-bit words per element


def stride(variant, kind):
    return 4 if variant == SFMT else WPE[kind]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = vmt.vmt_ctx_create(0)
    yield c
    torch.cuda.synchronize()
    vmt.vmt_ctx_destroy(c)


def fresh(ctx, variant, M, seed):
    st = vmt.new_state(variant, M)
    vmt.vmt_init_genrand(ctx, variant, seed, M, st)
    return st


def generate(ctx, st, variant, kind, n):
    out = torch.empty(max(n, 1), dtype=DT[kind], device="cuda")
    if kind == U32:
        vmt.vmt_generate_u32(ctx, st, n, out)
    elif kind == U64:
        vmt.vmt_generate_u64(ctx, st, n, out)
    elif kind == F32:
        vmt.vmt_uniform_f32(ctx, st, n, out)
    else:
        vmt.vmt_uniform_f64(ctx, st, n, out)
    return out


def failing(ctx, variant, M, kind, out, n):
    cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    vmt.vmt_check_stream(ctx, variant, M, kind, out, n, cnt)
    torch.cuda.synchronize()
    return int(cnt.item())


def min_len(variant, M, kind):
    """Smallest n with n_words > deg(A) * S."""
    deg = check_poly(variant, M).bit_length() - 1
    return deg * stride(variant, kind) // WPE[kind] + 1


def expected_flip_count(A, S, nw, P):
    """Offsets x = P - i S (A_i = 1) with 0 <= x and x + deg S < nw."""
    deg = A.bit_length() - 1
    bits = bin(A)[2:][::-1]
    return sum(1 for i, c in enumerate(bits) if c == "1" and 0 <= P - i * S and P - i * S + deg * S < nw)


CASES = [
    (MT32, 16, U32, "min"), (MT32, 16, U32, 300_001), (MT32, 1, U32, 100_000), (MT32, 4, F32, 250_007),
    (MT64, 8, U64, "min"), (MT64, 8, U64, 200_003), (MT64, 8, F64, 100_000), (MT64, 8, F32, 100_001),
    (MT64, 2, U64, 64_000),
    (SFMT, 4, U32, "min"), (SFMT, 4, U32, 1_000_003), (SFMT, 64, U32, 4 * 21921 + 5_000), (SFMT, 1, F32, 200_000),
    (SFMT, 8, F32, 333_333),
]


@pytest.mark.parametrize("variant,M,kind,n", CASES)
def test_intact_stream_passes(ctx, variant, M, kind, n):
    n = min_len(variant, M, kind) if n == "min" else n
    say(f"case check intact variant={variant} M={M} kind={kind} n={n}")
    st = fresh(ctx, variant, M, 1234 + M)
    generate(ctx, st, variant, kind, 4099)  # start in the middle of the stream
    out = generate(ctx, st, variant, kind, n)
    assert failing(ctx, variant, M, kind, out, n) == 0


@pytest.mark.parametrize("variant,M,kind", [(MT32, 16, U32), (MT64, 8, U64), (SFMT, 4, U32), (MT32, 4, F32)])
def test_single_flipped_bit_is_counted_exactly(ctx, variant, M, kind):
    n = 150_000
    st = fresh(ctx, variant, M, 99)
    out = generate(ctx, st, variant, kind, n)
    torch.cuda.synchronize()
    good = out.clone()
    A, S, nw = check_poly(variant, M), stride(variant, kind), n * WPE[kind]
    for P, bit in ((0, 5), (nw // 2 + 1, 31), (nw - 1, 0), (12345, 17)):
        say(f"case check flip variant={variant} M={M} kind={kind} word={P} bit={bit}")
        out.copy_(good)
        if kind == F32:  # a low mantissa bit of (u >> 8) 2^-24: flip bit `bit` of the 24-bit integer
            v = out[P : P + 1].cpu().numpy()
            k = (v.astype(np.float64) * 2.0**24).astype(np.uint32) ^ np.uint32(1 << (bit % 24))
            out[P] = float(k[0]) * 2.0**-24
        else:
            w = out.view(torch.int32)
            w[P] = w[P] ^ int(np.array([1 << bit], np.uint32).view(np.int32)[0])
        got = failing(ctx, variant, M, kind, out, n)
        assert got == expected_flip_count(A, S, nw, P) and got > 0, (P, bit, got)
    out.copy_(good)
    assert failing(ctx, variant, M, kind, out, n) == 0


@pytest.mark.parametrize("M", [2, 4])
def test_lane_spacing(ctx, M):
    # lanes built one by one: jumps of t J give the library's V-stream and pass;
    # jumps of t (J + 1) fail at almost every offset
    J = 1 << (19937 - (M.bit_length() - 1))
    n_lane = 60_000
    ref = generate(ctx, fresh(ctx, MT32, M, 555), MT32, U32, n_lane * M)
    for spacing, ok in ((J, True), (J + 1, False)):
        say(f"case check lanes M={M} spacing={'J' if ok else 'J+1'}")
        lanes = []
        for t in range(M):
            st = fresh(ctx, MT32, 1, 555)
            if t:
                vmt.vmt_jump(ctx, st, t * spacing)
            lanes.append(generate(ctx, st, MT32, U32, n_lane))
        v = torch.stack(lanes, dim=1).reshape(-1).contiguous()
        got = failing(ctx, MT32, M, U32, v, v.numel())
        if ok:
            assert torch.equal(v, ref)
            assert got == 0
        else:
            valid = v.numel() - 19937
            assert got > 0.999 * valid, (got, valid)


def test_batch_outputs_pass(ctx):
    M, count = 16, 6
    lens = [19938, 20000, 65_537, 100_000, 31_337, 250_000]
    states = [fresh(ctx, MT32, M, 800 + i) for i in range(count)]
    outs = [torch.empty(n, dtype=torch.int32, device="cuda") for n in lens]
    vmt.vmt_batch_generate(ctx, states, lens, outs, U32)
    for i, (o, n) in enumerate(zip(outs, lens)):
        say(f"case check batch output {i} n={n}")
        assert failing(ctx, MT32, M, U32, o, n) == 0


@pytest.mark.parametrize("variant,M,kind,n", [(MT32, 16, U32, 1 << 24), (MT64, 8, U64, 1 << 26),
                                              (MT64, 8, F64, 1 << 26), (SFMT, 4, U32, 1 << 28)])
def test_full_size_streams_pass(ctx, variant, M, kind, n):
    say(f"case check full size variant={variant} M={M} kind={kind} n={n}")
    st = fresh(ctx, variant, M, 5489 if variant != SFMT else 1234)
    out = generate(ctx, st, variant, kind, n)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    start.record()
    vmt.vmt_check_stream(ctx, variant, M, kind, out, n, cnt)
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    say(f"  {n * WPE[kind]} words checked in {ms:.2f} ms")
    assert int(cnt.item()) == 0


def test_errors(ctx):
    out = torch.empty(100_000, dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(vmt.VmtError) as e:
        vmt.vmt_check_stream(ctx, MT32, 16, U64, out, 1000, cnt)
    assert e.value.code == vmt.VMT_EVARIANT
    with pytest.raises(vmt.VmtError) as e:  # n_words = deg: nothing to check
        vmt.vmt_check_stream(ctx, MT32, 16, U32, out, 19937, cnt)
    assert e.value.code == vmt.VMT_EINVAL
    with pytest.raises(vmt.VmtError) as e:
        vmt.vmt_check_stream(ctx, MT32, 3, U32, out, 50_000, cnt)
    assert e.value.code == vmt.VMT_EINVAL
    with pytest.raises(vmt.VmtError) as e:  # misaligned uint64 stream
        vmt.vmt_check_stream(ctx, MT64, 8, U64, out.view(torch.int32)[1:], 40_000, cnt)
    assert e.value.code == vmt.VMT_EINVAL
    vmt.vmt_check_stream(ctx, MT32, 16, U32, out, 19938, cnt)  # smallest checkable length is accepted
