"""Launch shapes, the autotuner and graph replay on the GPU: every batch shape
(threads per workgroup, store width, resident workgroups) writes exactly the
oracle's stream (tolerance 0), the autotuner stores the fastest shape it
timed, and a batch plan captured in a HIP graph gives on every replay the
same bits as the same plan launched eagerly."""
import numpy as np
import pytest

from oracle import pyoracle as O
from tests.gpu_helpers import as_u, oracle_stream, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_16682_amd import vmt  # noqa: E402

MT32, MT64 = vmt.VMT_MT32, vmt.VMT_MT64
BLOCK = {MT32: 624, MT64: 312}
BATCH = vmt.VMT_FAMILY_BATCH
DT = {vmt.VMT_OUT_U32: torch.int32, vmt.VMT_OUT_U64: torch.int64, vmt.VMT_OUT_F32: torch.float32,
      vmt.VMT_OUT_F64: torch.float64}


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = vmt.vmt_ctx_create(0)
    yield c
    torch.cuda.synchronize()
    vmt.vmt_ctx_destroy(c)


def mapped(variant, kind, raw):
    if kind in (vmt.VMT_OUT_U32, vmt.VMT_OUT_U64):
        return raw
    if kind == vmt.VMT_OUT_F64:
        return O.map_f64(raw)
    if variant == MT64:
        return np.array([O.u64_to_f32(int(u)) for u in raw], np.float32)
    return O.map_f32(raw)


def host(out, n, variant, kind):
    t = out[:n].cpu()
    return as_u(t, variant) if kind in (vmt.VMT_OUT_U32, vmt.VMT_OUT_U64) else t.numpy()


def make_states(ctx, variant, M, seeds):
    states = []
    for s in seeds:
        st = vmt.new_state(variant, M)
        vmt.vmt_init_genrand(ctx, variant, s, M, st)
        states.append(st)
    return states


SHAPES = [(tv, sw, wpc) for tv in (0, 1, 2) for sw in (16, 8) for wpc in (0, 1)]


@pytest.mark.parametrize("variant,M,kind", [(MT32, 16, vmt.VMT_OUT_U32), (MT32, 16, vmt.VMT_OUT_F32),
                                            (MT32, 8, vmt.VMT_OUT_U32), (MT64, 8, vmt.VMT_OUT_U64),
                                            (MT64, 8, vmt.VMT_OUT_F64), (MT64, 8, vmt.VMT_OUT_F32),
                                            (MT64, 16, vmt.VMT_OUT_U64)])
def test_every_batch_shape_matches_oracle(ctx, variant, M, kind):
    rng = np.random.default_rng(21)
    B = BLOCK[variant] * M
    count = 10
    lens = [0, 1, B - 1, B + 3, 2 * B + 5] + [int(x) for x in rng.integers(1, 3 * B, count - 5)]
    pre = [int(x) for x in rng.integers(0, B, count)]
    seeds = list(range(300, 300 + count))
    refs = []
    for i in range(count):
        o = oracle_stream(variant, M, seed=seeds[i])
        o.generate(pre[i])
        refs.append(o)
    states = make_states(ctx, variant, M, seeds)
    for st, p in zip(states, pre):  # a different start position per state
        if p:
            tmp = torch.empty(p, dtype=torch.int64 if variant == MT64 else torch.int32, device="cuda")
            (vmt.vmt_generate_u64 if variant == MT64 else vmt.vmt_generate_u32)(ctx, st, p, tmp)
    outs = [torch.empty(max(n, 1), dtype=DT[kind], device="cuda") for n in lens]
    try:
        for tv, sw, wpc in SHAPES:
            say(f"case shape variant={variant} M={M} kind={kind} tv={tv} sw={sw} wpc={wpc}")
            vmt.vmt_shape_set(ctx, BATCH, variant, M, kind, threads_variant=tv, store_bytes=sw, wg_per_cu=wpc)
            sh = vmt.vmt_shape_get(ctx, BATCH, variant, M, kind)
            assert (sh.threads_variant, sh.store_bytes, sh.wg_per_cu) == (tv, sw, wpc) and sh.threads % 64 == 0
            for o in outs:
                o.zero_()
            vmt.vmt_batch_generate(ctx, states, lens, outs, kind)
            torch.cuda.synchronize()
            for i in range(count):
                ref = mapped(variant, kind, refs[i].generate(lens[i]))
                np.testing.assert_array_equal(host(outs[i], lens[i], variant, kind), ref,
                                              err_msg=f"shape {(tv, sw, wpc)} task {i}")
    finally:
        vmt.vmt_shape_set(ctx, BATCH, variant, M, kind)


def test_shape_errors(ctx):
    with pytest.raises(vmt.VmtError) as e:
        vmt.vmt_shape_set(ctx, BATCH, MT32, 4, vmt.VMT_OUT_U32, threads_variant=1, store_bytes=16)
    assert e.value.code == vmt.VMT_EINVAL  # shape variants exist for 8 and 16 lanes only
    with pytest.raises(vmt.VmtError):
        vmt.vmt_shape_set(ctx, BATCH, MT32, 16, vmt.VMT_OUT_U32, threads_variant=0, store_bytes=4)
    with pytest.raises(vmt.VmtError):
        vmt.vmt_shape_set(ctx, vmt.VMT_FAMILY_GENERATE, MT32, 16, vmt.VMT_OUT_U32, lanes_per_wg=32)
    d = vmt.vmt_shape_get(ctx, BATCH, MT32, 16, vmt.VMT_OUT_U32)
    assert (d.threads_variant, d.store_bytes, d.wg_per_cu) == (0, 16, 0)


@pytest.mark.parametrize("family", [vmt.VMT_FAMILY_GENERATE, BATCH])
def test_autotune_stores_the_fastest_shape(ctx, family):
    variant, M, kind = MT32, 16, vmt.VMT_OUT_U32
    lens = [1 << 20] if family == vmt.VMT_FAMILY_GENERATE else list(
        np.random.default_rng(4).integers(1000, 200000, 2048))
    say(f"case autotune family={family}")
    try:
        best, tried = vmt.vmt_autotune(ctx, family, variant, M, kind, lens, reps=2)
        assert len(tried) >= 2 and best.gbps > 0
        assert best.gbps == max(t.gbps for t in tried)
        cur = vmt.vmt_shape_get(ctx, family, variant, M, kind)
        if family == BATCH:
            assert (cur.threads_variant, cur.store_bytes, cur.wg_per_cu) == (best.threads_variant, best.store_bytes,
                                                                             best.wg_per_cu)
        else:
            assert cur.lanes_per_wg == best.lanes_per_wg
        # the tuned shape still writes the oracle's stream
        st = make_states(ctx, variant, M, [77])[0]
        out = torch.empty(5 * BLOCK[variant] * M + 3, dtype=torch.int32, device="cuda")
        if family == BATCH:
            vmt.vmt_batch_generate(ctx, [st], [out.numel()], [out], kind)
        else:
            vmt.vmt_generate_u32(ctx, st, out.numel(), out)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(as_u(out.cpu(), variant),
                                      oracle_stream(variant, M, seed=77).generate(out.numel()))
    finally:
        vmt.vmt_shape_set(ctx, family, variant, M, kind)


def test_plan_replayed_from_a_graph_equals_eager_launches(ctx):
    variant, M, kind = MT32, 16, vmt.VMT_OUT_U32
    count = 24
    rng = np.random.default_rng(8)
    lens = [int(x) for x in rng.integers(1, 5 * BLOCK[variant] * M, count)]
    seeds = list(range(500, 500 + count))
    a = make_states(ctx, variant, M, seeds)  # replayed from the graph
    b = make_states(ctx, variant, M, seeds)  # launched eagerly
    outs_a = [torch.zeros(n, dtype=torch.int32, device="cuda") for n in lens]
    outs_b = [torch.zeros(n, dtype=torch.int32, device="cuda") for n in lens]
    pa = vmt.vmt_batch_plan_create(ctx, a, lens, outs_a, kind)
    pb = vmt.vmt_batch_plan_create(ctx, b, lens, outs_b, kind)
    refs = [oracle_stream(variant, M, seed=s) for s in seeds]
    try:
        torch.cuda.synchronize()
        side = torch.cuda.Stream()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                vmt.vmt_batch_plan_launch(pa)
        torch.cuda.synchronize()
        # capture does not run the kernel: the states have not moved yet
        for rep in range(3):
            say(f"case graph replay {rep}")
            g.replay()
            vmt.vmt_batch_plan_launch(pb)
            junk = torch.randn(1 << 16, device="cuda").sum()  # eager work between replays
            torch.cuda.synchronize()
            assert torch.isfinite(junk)
            for i in range(count):
                ga = as_u(outs_a[i].cpu(), variant)
                np.testing.assert_array_equal(ga, as_u(outs_b[i].cpu(), variant), err_msg=f"replay {rep} task {i}")
                np.testing.assert_array_equal(ga, refs[i].generate(lens[i]), err_msg=f"replay {rep} task {i}")
    finally:
        torch.cuda.synchronize()
        vmt.vmt_batch_plan_destroy(pa)
        vmt.vmt_batch_plan_destroy(pb)
