"""Shared helpers for the GPU parity tests: oracle references and device buffers."""
import functools
import sys

import numpy as np

from oracle import pyoracle as O
from tests import golden_io

VARIANT_NAMES = {0: "mt32", 1: "mt64", 2: "sfmt", 3: "sfmt607", 4: "sfmt1279", 5: "sfmt2281", 6: "sfmt4253",
                 7: "sfmt11213"}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_seed(variant, seed=None, key=None):
    return O.seed_state(variant, seed=seed, key=key)


def oracle_stream(variant, M, seed=None, key=None):
    """Fresh oracle V-stream from init_genrand(seed) or init_by_array(key)."""
    return O.VStream(variant, M, oracle_seed(variant, seed, key), golden_io.lane_poly(variant, M))


@functools.lru_cache(maxsize=None)
def oracle_prefix(variant, M, seed, count):
    """First `count` elements of the V-stream (cached; read-only)."""
    s = oracle_stream(variant, M, seed=seed).generate(count)
    s.setflags(write=False)
    return s


def out_dtype(variant):
    import torch

    return torch.int64 if variant == 1 else torch.int32  # MT19937-64: uint64; the others uint32


def as_u(arr, variant):
    """torch int tensor (cpu) -> numpy unsigned view."""
    a = arr.numpy()
    return a.view(np.uint64) if variant == 1 else a.view(np.uint32)


_POW2 = {}


def pow2_poly(variant, k):
    """t^(2^k) mod mu by the oracle's squaring; every k on the way is kept."""
    chain = _POW2.setdefault(variant, [O.poly_mod(2, golden_io.minpoly(variant))])
    while len(chain) <= k:
        chain.append(O.poly_sqrmod(chain[-1], golden_io.minpoly(variant)))
    return chain[k]


def oracle_key_prefix(args):
    """(variant, M, key, n) -> first n elements of the oracle V-stream from
    init_by_array(key). Top-level so that a spawned worker process can run it:
    it touches neither torch nor the GPU."""
    variant, M, key, n = args
    return oracle_stream(variant, M, key=[int(k) for k in key]).generate(int(n))


def oracle_key_prefixes(variant, M, keys, ns, workers=8):
    """oracle_key_prefix for many keys, on a pool of spawned CPU workers (the
    oracle seeds each generator's M lanes by Horner jumps: a few tenths of a
    second per generator)."""
    import multiprocessing
    import os

    jobs = [(variant, M, tuple(int(x) for x in k), int(n)) for k, n in zip(keys, ns)]
    workers = max(1, min(workers, os.cpu_count() or 1, len(jobs)))
    if workers == 1:
        return [oracle_key_prefix(j) for j in jobs]
    with multiprocessing.get_context("spawn").Pool(workers) as pool:
        return pool.map(oracle_key_prefix, jobs, chunksize=4)


def oracle_jumped_tail(args):
    """(variant, M, seed, pre, k, n) -> the n elements of the oracle V-stream
    from init_genrand(seed) that follow `pre` elements and a jump by 2^k."""
    variant, M, seed, pre, k, n = args
    ref = oracle_stream(variant, M, seed=seed)
    ref.generate(pre)
    ref.jump(pow2_poly(variant, k))
    return ref.generate(n)


def oracle_map(fn, jobs, workers=8):
    """fn over jobs on a pool of spawned CPU workers (fn top-level in this
    module; the workers touch neither torch nor the GPU)."""
    import multiprocessing
    import os

    workers = max(1, min(workers, os.cpu_count() or 1, len(jobs)))
    if workers == 1:
        return [fn(j) for j in jobs]
    with multiprocessing.get_context("spawn").Pool(workers) as pool:
        return pool.map(fn, jobs, chunksize=2)


def oracle_key_digests(args):
    """(variant, M, key, segs) -> sha256 hex digests of consecutive segments
    of the oracle V-stream from init_by_array(key), segs[j] elements each.
    Top-level for spawned workers; touches neither torch nor the GPU."""
    import hashlib

    variant, M, key, segs = args
    ref = oracle_stream(variant, M, key=[int(k) for k in key])
    return [hashlib.sha256(ref.generate(int(n)).tobytes()).hexdigest() for n in segs]
