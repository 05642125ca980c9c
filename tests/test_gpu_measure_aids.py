"""The measurement aids the benchmark times against: the calibration fills
write exactly the requested bytes in every mode, and the write-pattern launch
of a batch plan stores to the plan's outputs only and leaves its states as
they were."""
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


@pytest.mark.parametrize("regions", [False, True])
@pytest.mark.parametrize("nontemporal", [False, True])
def test_calib_fill_writes_exactly_the_buffer(ctx, regions, nontemporal):
    n = (3 << 20) + 16 * 1234  # not a multiple of a piece or of the region count
    guard = 4096
    say(f"case calib fill regions={regions} nontemporal={nontemporal} bytes={n}")
    buf = torch.zeros(n + guard, dtype=torch.uint8, device="cuda")
    vmt.vmt_calib_fill(ctx, buf, nbytes=n, regions=regions, nontemporal=nontemporal)
    torch.cuda.synchronize()
    h = buf.cpu().numpy()
    assert (h[:n] == 0x5A).all()
    assert (h[n:] == 0).all()


def test_calib_fill_rejects_bad_arguments(ctx):
    buf = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(vmt.VmtError):
        vmt.vmt_calib_fill(ctx, buf, nbytes=100)
    with pytest.raises(vmt.VmtError):
        vmt._check(vmt.lib().vmt_calib_fill(ctx, vmt._dptr(buf), 4096, 4, vmt._stream(None)))


def test_write_pattern_stores_only_to_the_outputs_and_keeps_states(ctx):
    G, M = 40, 16
    lens = [0, 1, 9983, 9984, 9985] + [int(x) for x in np.random.default_rng(8).integers(1, 40000, G - 5)]
    sb = vmt.vmt_state_bytes(vmt.VMT_MT32, M)
    pool = torch.zeros(G * sb, dtype=torch.uint8, device="cuda")
    states = [pool[i * sb : (i + 1) * sb] for i in range(G)]
    vmt.vmt_init_by_array_batch(ctx, batch_keys(G, seed=50), M, states)
    offs = np.concatenate([[0], np.cumsum([(4 * n + 255) // 256 * 256 + 256 for n in lens])]).astype(np.int64)
    arena = torch.zeros(int(offs[-1]), dtype=torch.uint8, device="cuda")
    outs = [arena.data_ptr() + int(o) for o in offs[:-1]]
    before = pool.clone()
    plan = vmt.vmt_batch_plan_create(ctx, states, lens, outs, vmt.VMT_OUT_U32)
    try:
        say("case write pattern: 40 states")
        vmt.vmt_batch_plan_write_pattern(plan)
        vmt.vmt_batch_plan_write_pattern(plan)  # the queue counters are left clean for the next launch
        torch.cuda.synchronize()
    finally:
        vmt.vmt_batch_plan_destroy(plan)
    assert torch.equal(pool, before)
    h = arena.cpu().numpy()
    for i, n in enumerate(lens):
        seg = h[offs[i] : offs[i + 1]]
        assert (seg[4 * n :] == 0).all(), f"task {i} wrote past its {n} elements"
