"""Serving loop on the GPU: every request's result in the mix equals the same
state's requests replayed alone by the oracle (tolerance 0), the memory budget
holds, and unservable requests are reported without disturbing the rest."""
import numpy as np
import pytest

from oracle import pyoracle as O
from tests import golden_io
from tests.gpu_helpers import pow2_poly, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_16682_amd import vmt  # noqa: E402
from paper_2309_16682_amd.workload import serving_trace  # noqa: E402

MT64 = vmt.VMT_MT64
M = 8


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = vmt.vmt_ctx_create(0)
    yield c
    torch.cuda.synchronize()
    vmt.vmt_ctx_destroy(c)


def make_states(ctx, n, variant=MT64, lanes=M):
    sb = vmt.vmt_state_bytes(variant, lanes)
    pool = torch.empty(n * sb, dtype=torch.uint8, device="cuda")
    states = [pool[i * sb : (i + 1) * sb] for i in range(n)]
    for i, st in enumerate(states):
        vmt.vmt_init_genrand(ctx, variant, i + 1, lanes, st)
    torch.cuda.synchronize()
    return pool, states


def small_trace(n_states, seconds, rate, seed, elem_bytes=8):
    tr = serving_trace(seconds, rate_per_s=rate, n_states=n_states, min_bytes=8, max_bytes=64 << 10,
                       elem_bytes=elem_bytes, jump_fraction=0.15, kmin=32, kmax=80, seed=seed)
    return [(r.t_arrival, r.state, 0 if r.kind == "gen" else 1, r.nelem if r.kind == "gen" else 0, r.k) for r in tr]


def check_against_oracle(reqs, res, arena, variant=MT64, lanes=M):
    gJ = golden_io.lane_poly(variant, lanes)
    eb, dt = (8, np.uint64) if variant == MT64 else (4, np.uint32)
    host = arena.cpu().numpy()
    by_state = {}
    for i, r in enumerate(reqs):
        by_state.setdefault(r[1], []).append(i)
    for st, idx in by_state.items():
        ref = O.VStream(variant, lanes, O.seed_state(variant, st + 1), gJ)
        for i in sorted(idx, key=lambda j: (reqs[j][0], j)):
            t, _, kind, count, k = reqs[i]
            assert res[i]["status"] == 0
            if kind == 1:
                ref.jump(pow2_poly(variant, k))
            else:
                off = int(res[i]["out_offset"])
                got = host[off : off + eb * count].view(dt)
                np.testing.assert_array_equal(got, ref.generate(count), err_msg=f"request {i} state {st}")


@pytest.mark.parametrize("mode,chunk", [(0, 0), (0, 1000), (1, 0), (1, 1000), (4, 1000), (4, 200)])
@pytest.mark.parametrize("realtime", [False, True])
def test_results_in_the_mix_equal_each_state_alone(ctx, mode, realtime, chunk):
    # mode 4: large requests split into chunks that run side by side from jumped copies of the state
    n_states = 24
    reqs = small_trace(n_states, 0.05, 8000.0, seed=3 + mode)
    say(f"case serving mode={mode} chunk={chunk} realtime={realtime} requests={len(reqs)}")
    total = sum(8 * r[3] for r in reqs) + 256 * len(reqs) + (1 << 20)
    pool, states = make_states(ctx, n_states)
    arena = torch.zeros(total, dtype=torch.uint8, device="cuda")
    srv = vmt.vmt_server_create(ctx, states, arena, total, total, vmt.VMT_OUT_U64, n_streams=4, mode=mode | 2,
                                chunk_elems=chunk)
    try:
        res, wall = vmt.vmt_server_run(srv, reqs, realtime=realtime)
    finally:
        vmt.vmt_server_destroy(srv)
    assert (res["t_done"] >= res["t_launch"]).all() and (res["t_launch"] >= res["t_admit"]).all()
    # a state's requests ran one at a time, in arrival order
    for st in range(n_states):
        idx = [i for i, r in enumerate(reqs) if r[1] == st]
        for a, b in zip(idx, idx[1:]):
            assert res[b]["t_admit"] >= res[a]["t_done"]
    check_against_oracle(reqs, res, arena)


@pytest.mark.parametrize("chunk", [300, 2000])
def test_split_requests_of_v_mt19937_32(ctx, chunk):
    # V-MT19937-32, M = 16, large requests split into chunks (up to 31 jumped copies per request)
    n_states, lanes = 12, 16
    reqs = small_trace(n_states, 0.05, 6000.0, seed=21 + chunk, elem_bytes=4)
    say(f"case serving MT32 split chunk={chunk} requests={len(reqs)}")
    total = sum(4 * r[3] for r in reqs) + 256 * len(reqs) + (1 << 20)
    pool, states = make_states(ctx, n_states, vmt.VMT_MT32, lanes)
    arena = torch.zeros(total, dtype=torch.uint8, device="cuda")
    srv = vmt.vmt_server_create(ctx, states, arena, total, total, vmt.VMT_OUT_U32, n_streams=4, mode=4 | 2,
                                chunk_elems=chunk)
    try:
        res, _ = vmt.vmt_server_run(srv, reqs, realtime=False)
    finally:
        vmt.vmt_server_destroy(srv)
    assert (res["status"] == 0).all()
    check_against_oracle(reqs, res, arena, vmt.VMT_MT32, lanes)


@pytest.mark.parametrize("mode", [2, 6])
def test_budget_bounds_outputs_in_flight(ctx, mode):
    n_states = 16
    reqs = small_trace(n_states, 0.05, 6000.0, seed=9)
    biggest = max(8 * r[3] for r in reqs)
    budget = ((biggest + 255) // 256) * 256 * 3  # room for about three outputs at a time
    say(f"case serving budget={budget} mode={mode} requests={len(reqs)}")
    pool, states = make_states(ctx, n_states)
    total = sum(((8 * r[3] + 255) // 256) * 256 for r in reqs) + 256
    arena = torch.zeros(total, dtype=torch.uint8, device="cuda")
    srv = vmt.vmt_server_create(ctx, states, arena, total, budget, vmt.VMT_OUT_U64, n_streams=4, mode=mode,
                                chunk_elems=777)
    try:
        res, wall = vmt.vmt_server_run(srv, reqs, realtime=False)
    finally:
        vmt.vmt_server_destroy(srv)
    assert (res["status"] == 0).all()
    check_against_oracle(reqs, res, arena)
    ev = []
    for i, r in enumerate(reqs):
        if r[2] == 0:
            b = ((8 * r[3] + 255) // 256) * 256
            ev.append((res[i]["t_admit"], 1, b))
            ev.append((res[i]["t_done"], 0, -b))
    level = 0
    for t, order, b in sorted(ev):  # releases before admissions at equal times
        level += b
        assert level <= budget


def test_unservable_requests_are_reported(ctx):
    pool, states = make_states(ctx, 4)
    arena = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda")
    reqs = [(0.0, 0, 0, 100, 0), (0.0, 7, 0, 10, 0), (0.0, 1, 0, 1 << 20, 0), (0.0, 2, 1, 0, 1 << 20), (0.0, 3, 0, 5, 0)]
    srv = vmt.vmt_server_create(ctx, states, arena, 1 << 16, 1 << 16, vmt.VMT_OUT_U64, n_streams=2, mode=0)
    try:
        res, wall = vmt.vmt_server_run(srv, reqs, realtime=False)
    finally:
        vmt.vmt_server_destroy(srv)
    assert list(res["status"]) == [0, vmt.VMT_EINVAL, vmt.VMT_EINVAL, vmt.VMT_EINVAL, 0]
    host = arena.cpu().numpy()
    gJ = golden_io.lane_poly(MT64, M)
    for i, st in ((0, 0), (4, 3)):
        ref = O.VStream(MT64, M, O.seed_state(MT64, st + 1), gJ).generate(reqs[i][3])
        off = int(res[i]["out_offset"])
        np.testing.assert_array_equal(host[off : off + 8 * reqs[i][3]].view(np.uint64), ref)


def test_split_mode_arguments_are_checked(ctx):
    pool, states = make_states(ctx, 2)
    arena = torch.zeros(1 << 12, dtype=torch.uint8, device="cuda")
    for mode, chunk in ((5, 100), (4, 0)):  # plain form with splitting; splitting without a chunk size
        with pytest.raises(vmt.VmtError) as e:
            vmt.vmt_server_create(ctx, states, arena, 1 << 12, 1 << 12, vmt.VMT_OUT_U64, mode=mode, chunk_elems=chunk)
        assert e.value.code == vmt.VMT_EINVAL


def test_server_rejects_mixed_states(ctx):
    a = vmt.new_state(MT64, 8)
    b = vmt.new_state(MT64, 4)
    vmt.vmt_init_genrand(ctx, MT64, 1, 8, a)
    vmt.vmt_init_genrand(ctx, MT64, 1, 4, b)
    arena = torch.zeros(1 << 12, dtype=torch.uint8, device="cuda")
    with pytest.raises(vmt.VmtError) as e:
        vmt.vmt_server_create(ctx, [a, b], arena, 1 << 12, 1 << 12, vmt.VMT_OUT_U64)
    assert e.value.code == vmt.VMT_EINVAL


@pytest.mark.parametrize("mode", [0, 1])
def test_a_run_that_gives_up_reports_what_ran_and_the_server_recovers(ctx, mode):
    # The give-up path, forced from the host: with a watchdog of 0 s the run gives up at its first check with work
    # in flight. Every kernel still runs to its end; no request completes within the run.
    n_states = 12
    rng = np.random.default_rng(30 + mode)
    reqs = []
    for st in range(n_states):
        for j in range(3):
            if j == 1 and st % 3 == 0:
                reqs.append((0.0, st, 1, 0, int(rng.integers(32, 80))))
            else:
                reqs.append((0.0, st, 0, int(rng.integers(1, 20000)), 0))
    total = sum(((8 * r[3] + 255) // 256) * 256 for r in reqs) + 256
    say(f"case serving give-up mode={mode} requests={len(reqs)}")
    pool, states = make_states(ctx, n_states)
    arena = torch.zeros(total, dtype=torch.uint8, device="cuda")
    srv = vmt.vmt_server_create(ctx, states, arena, total, total, vmt.VMT_OUT_U64, n_streams=2, mode=mode | 2)
    try:
        with pytest.raises(vmt.VmtError) as e:
            vmt.vmt_server_set_watchdog(srv, -1.0)
        assert e.value.code == vmt.VMT_EINVAL
        vmt.vmt_server_set_watchdog(srv, 0.0)
        with pytest.raises(vmt.VmtError) as e:
            vmt.vmt_server_run(srv, reqs, realtime=False)
        assert e.value.code == vmt.VMT_EBUSY
        res1 = e.value.results
        host1 = arena.cpu().numpy()
        assert (res1["status"] == vmt.VMT_EBUSY).all()
        ran = res1["launch"] >= 0
        assert ran.any() and not ran.all()
        # the same server, with the default bound again, serves what did not run
        vmt.vmt_server_set_watchdog(srv, 30.0)
        rest = [i for i in range(len(reqs)) if not ran[i]]
        res2, _ = vmt.vmt_server_run(srv, [reqs[i] for i in rest], realtime=False)
        host2 = arena.cpu().numpy()
        assert (res2["status"] == 0).all()
        tail = [torch.empty(1000, dtype=torch.int64, device="cuda") for _ in range(n_states)]
        for st in range(n_states):
            vmt.vmt_generate_u64(ctx, states[st], 1000, tail[st])
        torch.cuda.synchronize()
    finally:
        vmt.vmt_server_destroy(srv)
    where = {i: (host1, res1[i]) for i in range(len(reqs)) if ran[i]}
    where.update({i: (host2, res2[j]) for j, i in enumerate(rest)})
    gJ = golden_io.lane_poly(MT64, M)
    for st in range(n_states):
        idx = [i for i, r in enumerate(reqs) if r[1] == st]
        # what ran of a state's requests is a prefix of them, in arrival order
        flags = [bool(ran[i]) for i in idx]
        assert flags == sorted(flags, reverse=True), (st, flags)
        ref = O.VStream(MT64, M, O.seed_state(MT64, st + 1), gJ)
        for i in idx:
            host, r = where[i]
            if reqs[i][2] == 1:
                ref.jump(pow2_poly(MT64, reqs[i][4]))
            else:
                off, count = int(r["out_offset"]), reqs[i][3]
                np.testing.assert_array_equal(host[off : off + 8 * count].view(np.uint64), ref.generate(count),
                                              err_msg=f"request {i} state {st}")
        np.testing.assert_array_equal(tail[st].cpu().numpy().view(np.uint64), ref.generate(1000),
                                      err_msg=f"state {st} after both runs")
