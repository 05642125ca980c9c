"""The batched and serving workloads at their full sizes, in the launch
configuration the benchmark times, checked on sampled outputs against the
oracle (tolerance 0).

  batched: 65,536 V-MT19937-32 (M = 16) generators seeded by init_by_array
           with splitmix64(42) keys, log-uniform lengths in [1e3, 1e7) from
           splitmix64(43), the first round of the benchmark's plan (tasks
           longest first over a 96 GiB arena), autotuned shape, launched from
           a captured HIP graph; 24 generators compared in full (the longest,
           the shortest and random ones) and the first 2000 outputs (or all)
           of 40 more; and every output of the round long enough to check
           (more than 19,937 words) passes the linear-complexity check (each
           bit obeys mu), a property that holds at any size.
  batched, every round and both steps: the benchmark's step as it times it
           (same autotuning sample, rounds over the 96 GiB arena, one HIP
           graph holding every round's launch) replayed twice, the second
           replay continuing every stream; the graph also copies the outputs
           of 1,024 sampled generators (the longest and shortest of each round
           and random ones in proportion to the rounds) out of the arena after
           their round, and each is compared in full with the oracle (sha256 of
           all its elements of both steps; a mismatch is then located element
           by element).
  single streams: workloads 1-3 at the launch shape the benchmark's
           autotuning picks (lanes per workgroup, chunk length), two calls in
           a row on one state as the benchmark times them, every element of
           both calls against the oracle.
  serving: 4,096 V-MT19937-64 (M = 8) states, the benchmark's trace (Poisson
           20k/s, 4 KiB - 256 MiB, 10 % jumps by 2^k) for its first 0.25 s,
           long requests split by jump-ahead, outputs retained; every request
           completes, sampled requests equal the oracle replaying their
           state's history, and every output long enough passes the
           linear-complexity check."""
import numpy as np
import pytest

from tests.gpu_helpers import as_u, oracle_key_digests, oracle_stream, pow2_poly, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_16682_amd import vmt  # noqa: E402
from paper_2309_16682_amd.workload import batch_keys, batch_lengths, plan_rounds, serving_trace  # noqa: E402

MT32, MT64 = vmt.VMT_MT32, vmt.VMT_MT64


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = vmt.vmt_ctx_create(0)
    yield c
    torch.cuda.synchronize()
    vmt.vmt_ctx_destroy(c)


def test_batched_workload_first_round(ctx):
    G, M = 65536, 16
    keys = batch_keys(G, seed=42)
    lens = batch_lengths(G, seed=43)
    say("case batched workload: 65536 generators, first round")
    sb = vmt.vmt_state_bytes(MT32, M)
    pool = torch.empty(G * sb, dtype=torch.uint8, device="cuda")
    states = [pool[i * sb : (i + 1) * sb] for i in range(G)]
    vmt.vmt_init_by_array_batch(ctx, keys, M, states)
    sample = np.random.default_rng(1).choice(lens, size=4096, replace=False)
    vmt.vmt_autotune(ctx, vmt.VMT_FAMILY_BATCH, MT32, M, vmt.VMT_OUT_U32, sample, reps=1)
    arena_bytes = 96 << 30
    rounds, offs = plan_rounds(lens, arena_bytes, 4)
    idx = [int(i) for i in rounds[0]]
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    base = arena.data_ptr()
    plan = vmt.vmt_batch_plan_create(ctx, [states[i].data_ptr() for i in idx], [int(lens[i]) for i in idx],
                                     [base + offs[i] for i in idx], vmt.VMT_OUT_U32)
    try:
        side = torch.cuda.Stream()
        g = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                vmt.vmt_batch_plan_launch(plan)
        g.replay()
        torch.cuda.synchronize()
    finally:
        vmt.vmt_batch_plan_destroy(plan)

    def out(i, n):
        return as_u(arena[offs[i] : offs[i] + 4 * n].cpu().view(torch.int32), MT32)

    rng = np.random.default_rng(2)
    by_len = sorted(idx, key=lambda i: int(lens[i]))
    full = [by_len[-1], by_len[-2], by_len[0], by_len[1]] + [int(i) for i in rng.choice(idx, 20, replace=False)]
    for i in full:
        n = int(lens[i])
        np.testing.assert_array_equal(out(i, n), oracle_stream(MT32, M, key=keys[i]).generate(n), err_msg=f"gen {i}")
    for i in rng.choice(idx, 40, replace=False):
        i = int(i)
        n = min(2000, int(lens[i]))
        np.testing.assert_array_equal(out(i, n), oracle_stream(MT32, M, key=keys[i]).generate(n), err_msg=f"gen {i}")
    # every checkable output of the round: the recurrence of its bits
    checked = [i for i in idx if int(lens[i]) > 19937]
    say(f"case batched workload: linear-complexity check of {len(checked)} outputs")
    cnt = torch.full((len(checked),), -1, dtype=torch.int64, device="cuda")
    for j, i in enumerate(checked):
        n = int(lens[i])
        vmt.vmt_check_stream(ctx, MT32, M, vmt.VMT_OUT_U32, arena[offs[i] : offs[i] + 4 * n], n, cnt[j : j + 1])
    torch.cuda.synchronize()
    bad = torch.nonzero(cnt).flatten().cpu().numpy()
    assert len(checked) > 0.5 * len(idx)
    assert bad.size == 0, [(checked[j], int(cnt[j])) for j in bad[:5]]


def test_batched_workload_every_round_both_steps(ctx):
    import hashlib
    import multiprocessing

    G, M, kind = 65536, 16, vmt.VMT_OUT_U32
    keys = batch_keys(G, seed=42)
    lens = batch_lengths(G, seed=43)
    sb = vmt.vmt_state_bytes(MT32, M)
    pool = torch.empty(G * sb, dtype=torch.uint8, device="cuda")
    states = [pool[i * sb : (i + 1) * sb] for i in range(G)]
    vmt.vmt_init_by_array_batch(ctx, keys, M, states)
    tune_lens = np.random.default_rng(17).choice(lens, size=8192, replace=False)  # the benchmark's sample
    vmt.vmt_autotune(ctx, vmt.VMT_FAMILY_BATCH, MT32, M, kind, tune_lens, reps=2)
    shape = vmt.vmt_shape_get(ctx, vmt.VMT_FAMILY_BATCH, MT32, M, kind)
    free, _ = torch.cuda.mem_get_info()
    arena_bytes = max(int(min(96 * 2**30, free - 16 * 2**30)), 1 << 30)
    rounds, offs = plan_rounds(lens, arena_bytes, 4)
    rng = np.random.default_rng(4)
    sample = []
    for idx in rounds:
        idx = np.asarray(idx)
        by = idx[np.argsort(lens[idx], kind="stable")]
        pick = {int(i) for i in list(by[:4]) + list(by[-4:])}
        want = -(-1032 * len(idx) // G)
        rest = [int(i) for i in rng.permutation(idx) if int(i) not in pick][: max(0, want - len(pick))]
        sample.append(sorted(pick | set(rest)))
    flat = [i for r in sample for i in r]
    assert len(flat) >= 1024 and len(set(flat)) == len(flat)
    say(f"case batched every round: {len(rounds)} rounds, shape {shape.threads} threads / {shape.store_bytes} B stores / "
        f"{shape.wg_per_cu} per CU, {len(flat)} sampled generators")
    # the oracle's digests run on CPU workers while the GPU works
    jobs = [(MT32, M, tuple(int(x) for x in keys[i]), (int(lens[i]), int(lens[i]))) for i in flat]
    workers = max(1, min(16, multiprocessing.cpu_count()))
    pool_cpu = multiprocessing.get_context("spawn").Pool(workers)
    try:
        pending = pool_cpu.map_async(oracle_key_digests, jobs, chunksize=4)
        co, tot = {}, 0
        for i in flat:
            co[i] = tot
            tot += (4 * int(lens[i]) + 255) // 256 * 256
        arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
        chk = torch.empty(tot, dtype=torch.uint8, device="cuda")
        base = arena.data_ptr()
        plans = [vmt.vmt_batch_plan_create(ctx, [states[int(i)].data_ptr() for i in idx],
                                           [int(lens[i]) for i in idx], [base + offs[int(i)] for i in idx], kind)
                 for idx in rounds]
        host = []
        try:
            side = torch.cuda.Stream()
            g = torch.cuda.CUDAGraph()
            torch.cuda.synchronize()
            with torch.cuda.stream(side):
                with torch.cuda.graph(g, stream=side):
                    for r, p in enumerate(plans):
                        vmt.vmt_batch_plan_launch(p)
                        for i in sample[r]:
                            n4 = 4 * int(lens[i])
                            chk[co[i] : co[i] + n4].copy_(arena[offs[i] : offs[i] + n4])
            for step in range(2):
                say(f"case batched every round: replay {step + 1}")
                chk.fill_(0)
                torch.cuda.synchronize()
                g.replay()
                torch.cuda.synchronize()
                host.append(chk.cpu().numpy())
        finally:
            torch.cuda.synchronize()
            for p in plans:
                vmt.vmt_batch_plan_destroy(p)
        del arena, chk
        say("case batched every round: waiting for the oracle")
        digests = pending.get(timeout=240)
    finally:
        pool_cpu.terminate()
    for j, i in enumerate(flat):
        n = int(lens[i])
        for step in range(2):
            seg = host[step][co[i] : co[i] + 4 * n]
            if hashlib.sha256(seg.tobytes()).hexdigest() != digests[j][step]:
                ref = oracle_stream(MT32, M, key=keys[i]).generate(2 * n)[step * n : (step + 1) * n]
                np.testing.assert_array_equal(seg.view(np.uint32), ref, err_msg=f"generator {i} step {step + 1}")
                raise AssertionError(f"generator {i} step {step + 1}: digest differs")


# the benchmark's single-stream configurations: name, variant, M, seed, elements, output kind
SINGLE = [
    ("mt32_M16_2^24_u32", MT32, 16, 5489, 1 << 24, "u32"),
    ("mt32_M1_2^24_u32", MT32, 1, 5489, 1 << 24, "u32"),
    ("mt64_M8_2^26_u64", MT64, 8, 5489, 1 << 26, "u64"),
    ("mt64_M8_2^26_f64", MT64, 8, 5489, 1 << 26, "f64"),
    ("sfmt_M4_2^28_u32", vmt.VMT_SFMT, 4, 1234, 1 << 28, "u32"),
    ("sfmt_M64_2^28_u32", vmt.VMT_SFMT, 64, 1234, 1 << 28, "u32"),
    ("sfmt_M64_2^28_f32", vmt.VMT_SFMT, 64, 1234, 1 << 28, "f32"),
    ("sfmt607_M64_2^28_u32", vmt.VMT_SFMT607, 64, 1234, 1 << 28, "u32"),
    ("sfmt11213_M16_2^28_u32", vmt.VMT_SFMT11213, 16, 1234, 1 << 28, "u32"),
]


@pytest.mark.parametrize("name,variant,M,seed,n,kind", SINGLE, ids=[c[0] for c in SINGLE])
def test_single_stream_at_the_autotuned_shape(ctx, name, variant, M, seed, n, kind):
    from oracle import pyoracle as O

    okind = {"u32": vmt.VMT_OUT_U32, "u64": vmt.VMT_OUT_U64, "f64": vmt.VMT_OUT_F64, "f32": vmt.VMT_OUT_F32}[kind]
    best, _ = vmt.vmt_autotune(ctx, vmt.VMT_FAMILY_GENERATE, variant, M, okind, [n], reps=2)
    say(f"case single stream {name}: {best.lanes_per_wg} lanes per workgroup, split 2^{best.split_log2}")
    try:
        st = vmt.new_state(variant, M)
        vmt.vmt_init_genrand(ctx, variant, seed, M, st)
        esz = 8 if kind in ("u64", "f64") else 4
        fn = {"u32": vmt.vmt_generate_u32, "u64": vmt.vmt_generate_u64, "f64": vmt.vmt_uniform_f64,
              "f32": vmt.vmt_uniform_f32}[kind]
        ref = oracle_stream(variant, M, seed=seed)
        for call in range(2):
            out = torch.empty(n * esz, dtype=torch.uint8, device="cuda")
            fn(ctx, st, n, out)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            del out
            r = ref.generate(n)
            if kind == "f64":
                exp = O.map_f64(r)
            elif kind == "f32":
                exp = O.map_f32(r)
            else:
                exp = r
            np.testing.assert_array_equal(got.view(exp.dtype), exp, err_msg=f"{name} call {call + 1}")
    finally:
        vmt.vmt_shape_set(ctx, vmt.VMT_FAMILY_GENERATE, variant, M, okind)


def test_serving_workload_sampled(ctx):
    n_states, M = 4096, 8
    trace = serving_trace(0.25, rate_per_s=20000.0, n_states=n_states, min_bytes=4096, max_bytes=256 << 20,
                          elem_bytes=8, jump_fraction=0.1, kmin=32, kmax=256, seed=11)
    reqs = [(r.t_arrival, r.state, 0 if r.kind == "gen" else 1, r.nelem if r.kind == "gen" else 0, r.k)
            for r in trace]
    total = sum(((8 * r[3] + 255) // 256) * 256 for r in reqs) + 256
    say(f"case serving workload: {len(reqs)} requests, {total / 1e9:.1f} GB retained")
    sb = vmt.vmt_state_bytes(MT64, M)
    pool = torch.empty(n_states * sb, dtype=torch.uint8, device="cuda")
    states = [pool[i * sb : (i + 1) * sb] for i in range(n_states)]
    for i, st in enumerate(states):
        vmt.vmt_init_genrand(ctx, MT64, i + 1, M, st)
    arena = torch.empty(total, dtype=torch.uint8, device="cuda")
    srv = vmt.vmt_server_create(ctx, states, arena, total, 16 << 30, vmt.VMT_OUT_U64, n_streams=4, mode=4 | 2,
                                chunk_elems=1 << 20)
    try:
        res, wall = vmt.vmt_server_run(srv, reqs, realtime=True)
    finally:
        vmt.vmt_server_destroy(srv)
    assert (res["status"] == 0).all()
    assert (res["t_done"] >= res["t_admit"]).all()
    history = {}
    for i, r in enumerate(reqs):
        history.setdefault(r[1], []).append(i)
    gens = [i for i, r in enumerate(reqs) if r[2] == 0]
    rng = np.random.default_rng(3)
    largest = max(gens, key=lambda i: reqs[i][3])
    sample = [largest] + [int(i) for i in rng.choice(gens, 24, replace=False)]
    for i in sample:
        st = reqs[i][1]
        ref = oracle_stream(MT64, M, seed=st + 1)
        for j in sorted(history[st], key=lambda j: (reqs[j][0], j)):
            if j == i:
                break
            if reqs[j][2] == 1:
                ref.jump(pow2_poly(MT64, reqs[j][4]))
            else:
                ref.generate(reqs[j][3])
        n = reqs[i][3]
        off = int(res[i]["out_offset"])
        got = as_u(arena[off : off + 8 * n].cpu().view(torch.int64), MT64)
        np.testing.assert_array_equal(got, ref.generate(n), err_msg=f"request {i} state {st} count {n}")
    # every output long enough (more than 19,937 uint64 halves-pairs): the recurrence of its bits
    checked = [i for i in gens if reqs[i][3] > 19937]
    cnt = torch.full((len(checked),), -1, dtype=torch.int64, device="cuda")
    for j, i in enumerate(checked):
        off, n = int(res[i]["out_offset"]), reqs[i][3]
        vmt.vmt_check_stream(ctx, MT64, M, vmt.VMT_OUT_U64, arena[off : off + 8 * n], n, cnt[j : j + 1])
    torch.cuda.synchronize()
    say(f"case serving workload: linear-complexity check of {len(checked)} outputs")
    bad = torch.nonzero(cnt).flatten().cpu().numpy()
    assert len(checked) > 0.3 * len(gens)
    assert bad.size == 0, [(checked[j], int(cnt[j])) for j in bad[:5]]
