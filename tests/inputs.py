"""Seeded synthetic inputs shared by the GPU tests and the oracle tests.

Nothing here computes any part of the method: it only draws random +1/-1
matrices with the structure the method assumes (column 0 all +1, every
other column balanced) and converts between the two storage layouts:

* unpacked: int8 [n][m][m], entry [k, i, j] = row i, column j of matrix k;
* packed:   uint32 [n][m][W], W = 1 up to order 32, 2 up to 64, 4 up to 128;
  bit (r % 32) of word r // 32 of column j is 1 iff entry (r, j) is -1;
  unused bits and words are 0.
"""
import numpy as np


def words(m: int) -> int:
    return 1 if m <= 32 else (2 if m <= 64 else 4)


def random_population(m: int, n: int, seed: int) -> np.ndarray:
    """n matrices: column 0 all +1, other columns uniformly random balanced."""
    rng = np.random.default_rng(seed)
    base = np.where(np.arange(m) < m // 2, -1, 1).astype(np.int8)
    cols = np.tile(base, (n, m - 1, 1))            # [n][m-1][m]
    idx = rng.random((n, m - 1, m)).argsort(axis=2)
    cols = np.take_along_axis(cols, idx, axis=2)
    pop = np.ones((n, m, m), dtype=np.int8)
    pop[:, :, 1:] = cols.transpose(0, 2, 1)
    return np.ascontiguousarray(pop)


def pack(pop: np.ndarray) -> np.ndarray:
    pop = np.asarray(pop)
    n, m, _ = pop.shape
    W = words(m)
    bits = (pop == -1).astype(np.uint64)          # [n][row][col]
    out = np.zeros((n, m, W), dtype=np.uint32)
    for w in range(W):
        rows = range(32 * w, min(m, 32 * w + 32))
        acc = np.zeros((n, m), dtype=np.uint64)
        for r in rows:
            acc |= bits[:, r, :] << np.uint64(r - 32 * w)
        out[:, :, w] = acc.astype(np.uint32)
    return out


def unpack(packed: np.ndarray, m: int) -> np.ndarray:
    packed = np.asarray(packed, dtype=np.uint32)
    n = packed.shape[0]
    W = words(m)
    packed = packed.reshape(n, m, W)
    pop = np.ones((n, m, m), dtype=np.int8)
    for r in range(m):
        bit = (packed[:, :, r // 32] >> np.uint32(r % 32)) & np.uint32(1)   # [n][col]
        pop[:, r, :] = np.where(bit == 1, -1, 1)
    return pop


def all_m4_normalized() -> np.ndarray:
    """All 6^3 = 216 normalized 4x4 matrices with balanced columns 1..3."""
    import itertools
    balanced = [np.array(v, dtype=np.int8) for v in itertools.product([1, -1], repeat=4)
                if sum(v) == 0]
    out = []
    for c1, c2, c3 in itertools.product(balanced, repeat=3):
        Q = np.ones((4, 4), dtype=np.int8)
        Q[:, 1], Q[:, 2], Q[:, 3] = c1, c2, c3
        out.append(Q)
    return np.stack(out)


# --------------------------------------------------------------------------
# Multi-run workloads: the configurations of the batched and the served
# benchmark, as plain dicts of configuration fields (m, n, seed,
# max_generations, stop_on_found); every other field keeps the plain GA's
# value (binary tournament, crossover 0.5, one pair flip at rate 0.1, SQ).
# --------------------------------------------------------------------------
def batched_workload(meta_seed: int = 4, count: int = 24) -> list:
    """`count` runs: order uniform over {12, 16, 20, 24, 28, 36}, size
    uniform in [2000, 60000], seed meta_seed * 10^6 + i, 300 generations,
    no stop on found."""
    rng = np.random.default_rng(meta_seed)
    out = []
    for i in range(count):
        m = int(rng.choice([12, 16, 20, 24, 28, 36]))
        n = int(rng.integers(2000, 60001))
        out.append(dict(m=m, n=n, seed=meta_seed * 10**6 + i, max_generations=300,
                        stop_on_found=False))
    return out


def served_workload(meta_seed: int = 5, count: int = 2000, rate: float = 50.0):
    """A Poisson stream of `count` search requests at `rate` per second:
    (list of config dicts, arrival times in seconds from the first).  Order
    uniform over the multiples of 4 in [8, 64], size uniform in
    [1000, 50000], seed meta_seed * 10^6 + i, a budget of 2000 generations,
    stop at the first Hadamard matrix."""
    rng = np.random.default_rng(meta_seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(count):
        m = int(4 * rng.integers(2, 17))
        n = int(rng.integers(1000, 50001))
        out.append(dict(m=m, n=n, seed=meta_seed * 10**6 + i, max_generations=2000,
                        stop_on_found=True))
    return out, arrivals
