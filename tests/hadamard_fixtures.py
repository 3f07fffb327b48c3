"""Known Hadamard matrices built from textbook constructions.

These are test fixtures: each construction follows its mathematical
definition and each result is checked with H^T H = m I before use.

* Sylvester: H[i][j] = (-1)^popcount(i & j), order 2^k.
* Paley I: q prime, q = 3 (mod 4): H = I + S with S = [[0, 1^T], [-1, J]],
  J the q x q Jacobsthal matrix J[a][b] = chi(a - b) (chi the quadratic
  character mod q); order q + 1.
* Paley II: q prime, q = 1 (mod 4): C = [[0, 1^T], [1, J]] (symmetric),
  H = C (x) [[1, 1], [1, -1]] + I (x) [[1, -1], [-1, -1]]; order 2(q + 1).
* Kronecker doubling: [[H, H], [H, -H]].

normalize() multiplies each row by its first entry so column 0 is all +1;
a Hadamard matrix normalized this way has every other column balanced.
"""
import numpy as np


def sylvester(m: int) -> np.ndarray:
    assert m & (m - 1) == 0
    i = np.arange(m)
    pc = np.vectorize(lambda x: bin(int(x)).count("1"))(i[:, None] & i[None, :])
    return np.where(pc % 2 == 0, 1, -1).astype(np.int8)


def _is_prime(q: int) -> bool:
    return q > 1 and all(q % d for d in range(2, int(q ** 0.5) + 1))


def _chi(q: int) -> np.ndarray:
    sq = {(x * x) % q for x in range(1, q)}
    return np.array([0] + [1 if a in sq else -1 for a in range(1, q)], dtype=np.int64)


def _jacobsthal(q: int) -> np.ndarray:
    chi = _chi(q)
    a = np.arange(q)
    return chi[(a[:, None] - a[None, :]) % q]


def paley1(q: int) -> np.ndarray:
    assert _is_prime(q) and q % 4 == 3
    J = _jacobsthal(q)
    S = np.zeros((q + 1, q + 1), dtype=np.int64)
    S[0, 1:] = 1
    S[1:, 0] = -1
    S[1:, 1:] = J
    return (np.eye(q + 1, dtype=np.int64) + S).astype(np.int8)


def paley2(q: int) -> np.ndarray:
    assert _is_prime(q) and q % 4 == 1
    J = _jacobsthal(q)
    C = np.zeros((q + 1, q + 1), dtype=np.int64)
    C[0, 1:] = 1
    C[1:, 0] = 1
    C[1:, 1:] = J
    A = np.array([[1, 1], [1, -1]])
    B = np.array([[1, -1], [-1, -1]])
    return (np.kron(C, A) + np.kron(np.eye(q + 1, dtype=np.int64), B)).astype(np.int8)


def double(H: np.ndarray) -> np.ndarray:
    return np.block([[H, H], [H, -H]]).astype(np.int8)


def normalize(H: np.ndarray) -> np.ndarray:
    return (H * H[:, :1]).astype(np.int8)


def is_hadamard(H: np.ndarray) -> bool:
    m = H.shape[0]
    G = H.astype(np.int64).T @ H.astype(np.int64)
    return bool(np.array_equal(G, m * np.eye(m, dtype=np.int64)))


def hadamard(m: int) -> np.ndarray:
    """A normalized Hadamard matrix of order m (m % 4 == 0, 4 <= m <= 128;
    not 52, 92, 100 or 116, which these constructions do not reach)."""
    if m & (m - 1) == 0:
        H = sylvester(m)
    elif _is_prime(m - 1) and (m - 1) % 4 == 3:
        H = paley1(m - 1)
    elif m % 2 == 0 and _is_prime(m // 2 - 1) and (m // 2 - 1) % 4 == 1:
        H = paley2(m // 2 - 1)
    elif m % 2 == 0 and (m // 2) % 4 == 0:
        H = double(hadamard(m // 2))
    else:
        raise ValueError("no construction for order %d" % m)
    H = normalize(H)
    assert is_hadamard(H)
    return H


ORDERS_WITH_FIXTURE = [m for m in range(4, 129, 4) if m not in (52, 92, 100, 116)]
