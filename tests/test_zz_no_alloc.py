"""The allocation-free batch call (vmt_batch_generate_noalloc) against the
allocating one (vmt_batch_generate): the same states, lengths and output
kinds give bit-identical outputs and states, on two calls in a row, the
second with fewer states and shorter requests (the scratch array keeps the
first call's longer task list, which must not leak into the second)."""
import numpy as np
import pytest

from tests.gpu_helpers import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_16682_amd import vmt  # noqa: E402
from paper_2309_16682_amd.workload import batch_keys  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = vmt.vmt_ctx_create(0)
    yield c
    torch.cuda.synchronize()
    vmt.vmt_ctx_destroy(c)


def _pools(ctx, variant, M, G):
    """Two pools of G states seeded alike (init_by_array keys for MT19937-32,
    init_genrand(i + 1) otherwise)."""
    sb = vmt.vmt_state_bytes(variant, M)
    pools = []
    for _ in range(2):
        pool = torch.empty(G * sb, dtype=torch.uint8, device="cuda")
        states = [pool[i * sb : (i + 1) * sb] for i in range(G)]
        if variant == vmt.VMT_MT32:
            vmt.vmt_init_by_array_batch(ctx, batch_keys(G, seed=46), M, states)
        else:
            for i, st in enumerate(states):
                vmt.vmt_init_genrand(ctx, variant, i + 1, M, st)
        pools.append((pool, states))
    return pools


def _run(ctx, fn, states, lens, kind, esz):
    offs = np.concatenate([[0], np.cumsum([(n * esz + 255) // 256 * 256 for n in lens])]).astype(np.int64)
    arena = torch.full((int(offs[-1]) + 256,), 0x5A, dtype=torch.uint8, device="cuda")
    outs = [arena.data_ptr() + int(o) for o in offs[:-1]]
    fn(ctx, states, lens, outs, kind)
    torch.cuda.synchronize()
    host = arena.cpu().numpy()
    return [host[offs[i] : offs[i] + n * esz] for i, n in enumerate(lens)]


@pytest.mark.parametrize("variant,M,kind,esz", [
    (vmt.VMT_MT32, 16, vmt.VMT_OUT_U32, 4),
    (vmt.VMT_MT64, 8, vmt.VMT_OUT_F64, 8),
    (vmt.VMT_SFMT, 4, vmt.VMT_OUT_U32, 4),
])
def test_noalloc_batch_equals_allocating_batch(ctx, variant, M, kind, esz):
    G = 96
    rng = np.random.default_rng(1000 + variant)
    per = 4 if variant in vmt.SFMT_FAMILY else 1
    block = vmt.STATE_WORDS[variant] * M * per
    (pa, sa), (pb, sb) = _pools(ctx, variant, M, G)
    # call 1: every state, ragged lengths from 0 to ~5 blocks; call 2: a third of the states in another order,
    # shorter requests (their states continue from call 1)
    lens1 = [0, 1, block - 1, block, block + 1] + [int(x) for x in rng.integers(1, 5 * block, G - 5)]
    pick = [int(i) for i in rng.permutation(G)[: G // 3]]
    lens2 = [int(x) for x in rng.integers(0, 2 * block, len(pick))]
    for call, (idx, lens) in enumerate(((list(range(G)), lens1), (pick, lens2))):
        say(f"case noalloc: variant {variant} M={M} kind {kind} call {call + 1}: {len(idx)} states, {sum(lens)} elements")
        ref = _run(ctx, vmt.vmt_batch_generate, [sa[i] for i in idx], lens, kind, esz)
        got = _run(ctx, vmt.vmt_batch_generate_noalloc, [sb[i] for i in idx], lens, kind, esz)
        for j, i in enumerate(idx):
            np.testing.assert_array_equal(got[j], ref[j], err_msg=f"call {call + 1} state {i} ({lens[j]} elements)")
        assert torch.equal(pa, pb), f"call {call + 1}: states differ after the call"


def test_noalloc_rejects_more_tasks_than_the_scratch_holds(ctx):
    G = vmt.VMT_NOALLOC_MAX_TASKS + 1
    with pytest.raises(vmt.VmtError) as e:
        vmt.vmt_batch_generate_noalloc(ctx, [256 * (i + 1) for i in range(G)], [1] * G,
                                       [1 << 20] * G, vmt.VMT_OUT_U32)
    assert e.value.code == vmt.VMT_EINVAL and "at most" in str(e.value)
