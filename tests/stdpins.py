"""Black-box pins from the C++ standard library engines.

std::mt19937 and std::mt19937_64 are the MT19937-32/-64 generators with the
published init_genrand seeding; the C++ standard ([rand.predef]) requires the
10000th output of a default-constructed engine (seed 5489) to be 4123659995
and 9981545732273789042 respectively.
"""
import functools
import os
import subprocess
import tempfile

import numpy as np

SRC = r"""
#include <cstdio>
#include <cstdlib>
#include <random>
int main(int argc, char** argv) {
  int bits = atoi(argv[1]);
  unsigned long long seed = strtoull(argv[2], 0, 10);
  long count = atol(argv[3]);
  if (bits == 32) {
    std::mt19937 g((std::mt19937::result_type)seed);
    for (long i = 0; i < count; i++) printf("%u\n", (unsigned)g());
  } else {
    std::mt19937_64 g(seed);
    for (long i = 0; i < count; i++) printf("%llu\n", (unsigned long long)g());
  }
  return 0;
}
"""


@functools.lru_cache(maxsize=None)
def _exe() -> str:
    d = tempfile.mkdtemp(prefix="vmt_stdpin_")
    src = os.path.join(d, "pin.cpp")
    exe = os.path.join(d, "pin")
    with open(src, "w") as f:
        f.write(SRC)
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-o", exe, src])
    return exe


@functools.lru_cache(maxsize=None)
def std_stream(bits: int, seed: int, count: int) -> np.ndarray:
    out = subprocess.check_output([_exe(), str(bits), str(seed), str(count)])
    dt = np.uint32 if bits == 32 else np.uint64
    return np.array([int(v) for v in out.split()], dtype=dt)
