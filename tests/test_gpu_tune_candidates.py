"""Every launch shape the generate-family autotuner times for the single-stream
workloads (lanes per workgroup without splitting; chunk length x lanes per
workgroup with splitting) gives the oracle's stream: the candidates are the
ones vmt_autotune itself reports for the benchmark's call size, each run at a
small size (a ragged start, then at least 3 chunks plus a partial one, then
a continuation), tolerance 0."""
import numpy as np
import pytest

from oracle import pyoracle as O
from tests.gpu_helpers import as_u, oracle_stream, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_16682_amd import vmt  # noqa: E402

GEN = vmt.VMT_FAMILY_GENERATE
U32, U64, F32, F64 = vmt.VMT_OUT_U32, vmt.VMT_OUT_U64, vmt.VMT_OUT_F32, vmt.VMT_OUT_F64
DT = {U32: torch.int32, U64: torch.int64, F32: torch.float32, F64: torch.float64}
CALL = {U32: vmt.vmt_generate_u32, U64: vmt.vmt_generate_u64, F32: vmt.vmt_uniform_f32, F64: vmt.vmt_uniform_f64}

# the benchmark's single-stream workloads: variant, M, output kind, elements per call
CONFIGS = [
    (vmt.VMT_MT32, 16, U32, 1 << 24),
    (vmt.VMT_MT32, 1, U32, 1 << 24),
    (vmt.VMT_MT64, 8, U64, 1 << 26),
    (vmt.VMT_MT64, 8, F64, 1 << 26),
    (vmt.VMT_SFMT, 4, U32, 1 << 28),
    (vmt.VMT_SFMT, 64, U32, 1 << 28),
    (vmt.VMT_SFMT, 64, F32, 1 << 28),
    (vmt.VMT_SFMT607, 64, U32, 1 << 28),
    (vmt.VMT_SFMT11213, 16, U32, 1 << 28),
]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = vmt.vmt_ctx_create(0)
    yield c
    torch.cuda.synchronize()
    vmt.vmt_ctx_destroy(c)


def run(ctx, st, variant, kind, n):
    out = torch.zeros(max(n, 1), dtype=DT[kind], device="cuda")
    CALL[kind](ctx, st, n, out)
    torch.cuda.synchronize()
    t = out[:n].cpu()
    return as_u(t, variant) if kind in (U32, U64) else t.numpy()


def expect(kind, raw):
    return O.map_f64(raw) if kind == F64 else O.map_f32(raw) if kind == F32 else raw


@pytest.mark.parametrize("variant,M,kind,n_bench", CONFIGS,
                         ids=[f"v{c[0]}-M{c[1]}-k{c[2]}" for c in CONFIGS])
def test_every_autotuner_candidate_equals_oracle(ctx, variant, M, kind, n_bench):
    native = U64 if variant == vmt.VMT_MT64 else U32
    _, tried = vmt.vmt_autotune(ctx, GEN, variant, M, kind, [n_bench], reps=1)
    assert tried, "the autotuner timed no candidate"
    epw = 4 if variant in vmt.SFMT_FAMILY else 1
    block = vmt.STATE_WORDS[variant] * M * epw
    pre = 4321 % block + 1
    sizes = []
    for t in tried:
        if t.split_log2 == 255:
            n = 3 * block + 17
        else:
            n = int(3.37 * (1 << t.split_log2) * M * epw)
        sizes.append(n)
    tail = block + 5
    seed = 4000 + variant
    say(f"case autotuner candidates variant={variant} M={M} kind={kind}: {len(tried)} shapes, largest call {max(sizes)}")
    ref_all = oracle_stream(variant, M, seed=seed).generate(pre + max(sizes) + tail)
    try:
        for t, n in zip(tried, sizes):
            say(f"case candidate lanes_per_wg={t.lanes_per_wg} split_log2={t.split_log2} n={n}")
            vmt.vmt_shape_set(ctx, GEN, variant, M, kind, lanes_per_wg=t.lanes_per_wg, split_log2=t.split_log2)
            st = vmt.new_state(variant, M)
            vmt.vmt_init_genrand(ctx, variant, seed, M, st)
            head = run(ctx, st, variant, native, pre)
            np.testing.assert_array_equal(head, ref_all[:pre])
            got = run(ctx, st, variant, kind, n)
            np.testing.assert_array_equal(got, expect(kind, ref_all[pre : pre + n]),
                                          err_msg=f"lanes_per_wg={t.lanes_per_wg} split_log2={t.split_log2}")
            after = run(ctx, st, variant, native, tail)
            np.testing.assert_array_equal(after, ref_all[pre + n : pre + n + tail],
                                          err_msg=f"continuation after lanes_per_wg={t.lanes_per_wg} "
                                          f"split_log2={t.split_log2}")
            del st
    finally:
        vmt.vmt_shape_set(ctx, GEN, variant, M, kind)
