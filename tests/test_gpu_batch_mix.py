"""A scaled-down batched mix checked in full: 512 V-MT19937-32 (M = 16)
generators seeded by init_by_array with splitmix64 keys, log-uniform lengths
in [1e3, 1e5), run as one batch plan captured in a HIP graph and replayed
twice (the second replay continues every stream), for each store width the
autotuner can pick. Every output of every generator equals the oracle's
V-stream (tolerance 0)."""
import numpy as np
import pytest

from tests.gpu_helpers import as_u, oracle_key_prefixes, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_16682_amd import vmt  # noqa: E402
from paper_2309_16682_amd.workload import batch_keys, batch_lengths  # noqa: E402

MT32 = vmt.VMT_MT32
BATCH = vmt.VMT_FAMILY_BATCH


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = vmt.vmt_ctx_create(0)
    yield c
    torch.cuda.synchronize()
    vmt.vmt_ctx_destroy(c)


def test_scaled_batched_mix_in_full(ctx):
    G, M, kind = 512, 16, vmt.VMT_OUT_U32
    keys = batch_keys(G, seed=44)
    lens = [int(x) for x in batch_lengths(G, seed=45, lo=1e3, hi=1e5)]
    widths = (16, 8)
    reps = 2
    say(f"case batched mix: {G} generators, {sum(lens)} elements per replay, oracle references")
    refs = oracle_key_prefixes(MT32, M, keys, [len(widths) * reps * n for n in lens])
    sb = vmt.vmt_state_bytes(MT32, M)
    pool = torch.empty(G * sb, dtype=torch.uint8, device="cuda")
    states = [pool[i * sb : (i + 1) * sb] for i in range(G)]
    vmt.vmt_init_by_array_batch(ctx, keys, M, states)
    offs = np.concatenate([[0], np.cumsum(lens)])
    arena = torch.empty(int(offs[-1]), dtype=torch.int32, device="cuda")
    seg = 0
    try:
        for sw in widths:
            vmt.vmt_shape_set(ctx, BATCH, MT32, M, kind, store_bytes=sw)
            plan = vmt.vmt_batch_plan_create(ctx, states, lens, [arena.data_ptr() + 4 * int(o) for o in offs[:-1]],
                                             kind)
            try:
                side = torch.cuda.Stream()
                g = torch.cuda.CUDAGraph()
                torch.cuda.synchronize()
                with torch.cuda.stream(side):
                    with torch.cuda.graph(g, stream=side):
                        vmt.vmt_batch_plan_launch(plan)
                for rep in range(reps):
                    say(f"case batched mix: store width {sw}, replay {rep}")
                    arena.fill_(0)
                    torch.cuda.synchronize()
                    g.replay()
                    torch.cuda.synchronize()
                    host = as_u(arena.cpu(), MT32)
                    for i, n in enumerate(lens):
                        np.testing.assert_array_equal(host[offs[i] : offs[i + 1]], refs[i][seg * n : (seg + 1) * n],
                                                      err_msg=f"store width {sw} replay {rep} generator {i}")
                    seg += 1
            finally:
                torch.cuda.synchronize()
                vmt.vmt_batch_plan_destroy(plan)
    finally:
        vmt.vmt_shape_set(ctx, BATCH, MT32, M, kind)
