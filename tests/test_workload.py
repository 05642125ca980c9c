"""CPU checks of the seeded workload generators and the round planner (host
logic only: these draw seeds, sizes and arrival times, never the
generators' arithmetic)."""
import numpy as np

from paper_2309_16682_amd.workload import batch_keys, batch_lengths, plan_rounds, serving_trace, splitmix64


def splitmix64_ref(seed, count):
    """splitmix64 (Steele, Lea, Flood 2014) with Python integers."""
    out, s = [], seed
    for _ in range(count):
        s = (s + 0x9E3779B97F4A7C15) & (2**64 - 1)
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & (2**64 - 1)
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & (2**64 - 1)
        out.append(z ^ (z >> 31))
    return out


def test_splitmix64_published_value_and_reference():
    assert int(splitmix64(0, 1)[0]) == 0xE220A8397B1DCDAF  # first output for seed 0
    assert [int(x) for x in splitmix64(42, 100)] == splitmix64_ref(42, 100)


def test_batch_keys_take_two_outputs_per_generator():
    keys = batch_keys(5, seed=42)
    ref = splitmix64_ref(42, 10)
    for g in range(5):
        lo0, hi0, lo1, hi1 = (int(x) for x in keys[g])
        assert lo0 | (hi0 << 32) == ref[2 * g] and lo1 | (hi1 << 32) == ref[2 * g + 1]


def test_batch_lengths_log_uniform_in_range():
    lens = batch_lengths(65536, seed=43)
    assert lens.min() >= 1000 and lens.max() < 10**7
    logs = np.log(lens.astype(np.float64))
    # log-uniform: mean of log between the bounds, about 71.7 G elements in all
    assert abs(logs.mean() - (np.log(1e3) + np.log(1e7)) / 2) < 0.02
    assert 70.5e9 < lens.sum() < 73e9


def test_serving_trace_shape():
    tr = serving_trace(2.0, rate_per_s=20000.0, n_states=4096, min_bytes=4096, max_bytes=256 << 20, elem_bytes=8,
                       jump_fraction=0.1, kmin=32, kmax=256, seed=11)
    t = np.array([r.t_arrival for r in tr])
    assert np.all(np.diff(t) >= 0) and 36000 < len(tr) < 44000
    jumps = [r for r in tr if r.kind == "jump"]
    assert 0.08 < len(jumps) / len(tr) < 0.12 and all(32 <= r.k <= 256 for r in jumps)
    gens = [r for r in tr if r.kind == "gen"]
    assert all(512 <= r.nelem <= (256 << 20) // 8 for r in gens)
    assert all(0 <= r.state < 4096 for r in tr)


def test_plan_rounds_fits_the_arena_and_keeps_tasks_disjoint():
    lens = batch_lengths(4096, seed=43)
    arena = 2 << 30
    rounds, offs = plan_rounds(lens, arena, 4)
    assert sorted(int(i) for r in rounds for i in r) == list(range(4096))
    for idx in rounds:
        spans = sorted((offs[int(i)], offs[int(i)] + 4 * int(lens[i])) for i in idx)
        assert all(a % 256 == 0 for a, _ in spans)
        assert spans[-1][1] <= arena
        assert all(b1 <= a2 for (_, b1), (a2, _) in zip(spans, spans[1:]))
