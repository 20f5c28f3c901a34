"""SplitMix64 (Steele, Lea and Flood, 2014): the one seeded generator every workload draws from.

It holds no arithmetic of the rational-Arnoldi method: it only turns a 64-bit seed into a
reproducible stream of integers and doubles, so that the oracle and the GPU library receive
bit-identical synthetic inputs.
"""
from __future__ import annotations

import numpy as np

_MASK = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15

# Per-workload base seeds; sub-stream k of workload c is BASE_SEED + c, times 1000, plus k.
BASE_SEED = 2310047340
STREAM_SOURCE = 1
STREAM_RECEIVERS = 2
STREAM_LOAD_PHASE = 3
STREAM_VARIANT = 4
STREAM_ORDERS = 5
STREAM_SPLIT = 6
STREAM_MLP_INIT = 7
STREAM_MINIBATCH = 8


def stream_seed(config: int, stream: int) -> int:
    return ((BASE_SEED + config) * 1000 + stream) & _MASK


class SplitMix64:
    """Counter-based 64-bit generator; state advances by the golden-ratio increment."""

    def __init__(self, seed: int):
        self.state = int(seed) & _MASK

    def next_u64(self) -> int:
        self.state = (self.state + _GOLDEN) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def uniforms(self, n: int) -> np.ndarray:
        return np.array([self.uniform() for _ in range(int(n))], dtype=np.float64)

    def randint(self, n: int) -> int:
        """Integer in [0, n) by floor(u * n)."""
        return min(int(self.uniform() * n), n - 1)

    def sample(self, population, k: int) -> np.ndarray:
        """k distinct items of `population` by a partial Fisher-Yates shuffle."""
        pool = np.array(population, dtype=np.int64).copy()
        n = len(pool)
        if k > n:
            raise ValueError("sample larger than population")
        for i in range(k):
            j = i + self.randint(n - i)
            pool[i], pool[j] = pool[j], pool[i]
        return pool[:k].copy()
