"""Counter-based generator for the substitute ("bench") vectors.

TEST INFRASTRUCTURE: part of the CPU oracle (see ``oracle/__init__.py``).

The paper fills its dynamic substitutes bench with random vectors but does
not state their distribution (Section 5.1; its experiments used Matlab's
mt19937ar).  Both the oracle and the GPU library draw them from SplitMix64
(S. Vigna, public-domain reference ``splitmix64.c``), each side with its own
implementation of that published definition:

    state_c = seed + (c + 1) * 0x9E3779B97F4A7C15           (mod 2^64)
    z = (state_c ^ (state_c >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    out_c = z ^ (z >> 31)

i.e. out_c is the (c+1)-th output of the stream seeded with ``seed``.  Entry i
of bench vector b uses counter c = b*n + i and maps the top 53 bits to
[-1, 1): value = 2 * ((out_c >> 11) * 2^-53) - 1, exact in binary64.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """SplitMix64 outputs for an array of 0-based counters (uint64)."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def bench_vector(n: int, b: int, seed: int) -> np.ndarray:
    """Bench vector ``b`` (0-based), length n, entries in [-1, 1)."""
    c = np.uint64(b) * np.uint64(n) + np.arange(n, dtype=np.uint64)
    bits = splitmix64(seed, c) >> np.uint64(11)
    return 2.0 * (bits.astype(np.float64) * 2.0 ** -53) - 1.0
