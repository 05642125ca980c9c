"""Sizes at the limits of the index arithmetic: one call of more than 2^32
elements (a 16 GiB output), split automatically and in one launch, checked
against the oracle at the start, around 2^31 and 2^32 and at the end, and the
stream after the call (tolerance 0; the oracle reaches far positions by its
own jump-ahead, Horner's rule on the scalar lanes)."""
import numpy as np
import pytest

from oracle import pyoracle as O
from tests import golden_io
from tests.gpu_helpers import as_u, oracle_stream, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_16682_amd import vmt  # noqa: E402

MT32 = vmt.VMT_MT32
M = 16
N_BIG = (1 << 32) + 4099


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = vmt.vmt_ctx_create(0)
    yield c
    torch.cuda.synchronize()
    vmt.vmt_ctx_destroy(c)


def oracle_at(seed, start, count):
    """count elements of the V-stream from position start (jump by start // M lane steps)."""
    ref = oracle_stream(MT32, M, seed=seed)
    q, r = divmod(start, M)
    if q:
        ref.jump(O.poly_powmod_t(q, golden_io.minpoly(MT32)))
    return ref.generate(r + count)[r:]


@pytest.mark.parametrize("split", [0, 255])  # automatic splitting, one launch
def test_call_longer_than_2_pow_32(ctx, split):
    seed = 4242
    say(f"case mt32 M=16 n=2^32+4099 split={split}")
    vmt.vmt_shape_set(ctx, vmt.VMT_FAMILY_GENERATE, MT32, M, vmt.VMT_OUT_U32, lanes_per_wg=1 if split else 16,
                      split_log2=split)
    try:
        st = vmt.new_state(MT32, M)
        vmt.vmt_init_genrand(ctx, MT32, seed, M, st)
        out = torch.empty(N_BIG, dtype=torch.int32, device="cuda")
        vmt.vmt_generate_u32(ctx, st, N_BIG, out)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(as_u(out[:50000].cpu(), MT32), oracle_stream(MT32, M, seed=seed).generate(50000))
        for start in ((1 << 31) - 777, (1 << 32) - 3000, N_BIG - 5000):
            got = as_u(out[start : start + 5000].cpu(), MT32)
            np.testing.assert_array_equal(got, oracle_at(seed, start, 5000), err_msg=f"at {start}")
        del out
        more = torch.empty(3000, dtype=torch.int32, device="cuda")
        vmt.vmt_generate_u32(ctx, st, 3000, more)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(as_u(more.cpu(), MT32), oracle_at(seed, N_BIG, 3000))
    finally:
        vmt.vmt_shape_set(ctx, vmt.VMT_FAMILY_GENERATE, MT32, M, vmt.VMT_OUT_U32)
